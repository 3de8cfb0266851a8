// Internal declarations shared by the HIP translation units of libufvc.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <atomic>

namespace ufvc {

// Device-memory accesses through global (address space 1) pointers: the
// loads and stores become global_* instructions, which count only against
// vmcnt.  Generic pointers (e.g. read from a descriptor) would give flat_*
// instructions, which also count against lgkmcnt, so every wait on an LDS
// read would wait for the outstanding global prefetches too.
#define UFVC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T ldg(const T* p) { return *(const UFVC_GLOBAL T*)(p); }
template <class T>
__device__ __forceinline__ void stg(T* p, T v) { *(UFVC_GLOBAL T*)(p) = v; }

// s_waitcnt on the vector-memory counter only (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Copies `bytes` (a multiple of 16) from device memory to LDS, both 16-byte
// aligned, with one wave's direct-to-LDS loads: 1 KB per instruction, no
// registers, all in flight at once.  The data is in LDS once the wave's
// vector-memory counter has drained (wait_vmcnt<0>).
__device__ __forceinline__ void lds_fill16(void* dst, const void* src, int bytes) {
  const int lane = threadIdx.x & 63;
  for (int o = 0; o < bytes; o += 1024)
    if (lane * 16 < bytes - o)
      __builtin_amdgcn_global_load_lds((const UFVC_GLOBAL void*)((const unsigned char*)src + o + lane * 16),
                                       (__attribute__((address_space(3))) void*)((unsigned char*)dst + o),
                                       16, 0, 0);
}
// The same for `n` dwords at 4-byte alignment.
__device__ __forceinline__ void lds_fill4(void* dst, const void* src, int n) {
  const int lane = threadIdx.x & 63;
  for (int o = 0; o < n; o += 64)
    if (lane < n - o)
      __builtin_amdgcn_global_load_lds((const UFVC_GLOBAL void*)((const uint32_t*)src + o + lane),
                                       (__attribute__((address_space(3))) void*)((uint32_t*)dst + o), 4, 0,
                                       0);
}

// Raises a kernel's dynamic-LDS limit to `bytes` once per device.  `done`
// is the caller's per-kernel flag word (bit d: device d done); the fast path
// is one atomic load, the first call on a device sets the attribute under a
// lock, so concurrent host threads (the server's lanes) never race on it.
hipError_t set_lds_limit_once(std::atomic<uint32_t>& done, const void* kern, int bytes);

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- conv ----
enum Prec { P_F32 = 0, P_BF16 = 1, P_FP8 = 2 };
enum Loader {
  LD_NHWC = 0,       // activation tensor, channels innermost, compute type
  LD_UNSHUFFLE = 1,  // float32 frames [T][3][H][W], pixel-unshuffle x8 + replicate pad
  LD_DEQUANT = 2,    // y_hat = (sym - 32) + mu from uint8 symbols and float32 mu
  LD_UP2 = 3,        // nearest x2 upsampling of uint8 z symbols (value sym - 32): the
                     // entropy-parameter conv (params_up2_kernel, its own configurations)
  LD_F32 = 4,        // float32 tensor, channels innermost, feeding a bf16 conv
  LD_REP = 6         // bf16 tensor, channels innermost; input channel c is tensor channel
                     // c mod in_pitch (the split-weight convs over a bf16 input)
};
enum Store {
  ST_BF16 = 0,     // bf16 [pos][pitch], optional ReLU
  ST_F32 = 1,      // float32 [pos][pitch], optional ReLU
  ST_ZSYM = 2,     // z_hat = clamp(rint(z), -32, 32) stored as uint8 z_hat + 32
  ST_SHUFFLE = 3   // pixel-shuffle x8 into frame `group`, crop, clamp to [0, 1]
};

struct ConvArgs {
  int Hin, Win;       // input grid (latent) size used for zero padding
  int Hout, Wout;     // output grid size
  int cin, cout;      // channels per group
  // input
  const void* in;     // activation / frames / symbols
  long in_pitch;      // elements between positions
  long in_goff;       // elements between groups
  const float* mu;    // LD_DEQUANT: mean, [pos][mu_pitch]
  long mu_pitch;
  int T, H, W;        // frames (LD_UNSHUFFLE / ST_SHUFFLE): unpadded size
  // weights: packed [group][slice][tap][cout][32 bytes]
  const void* wpk;
  long w_gstride;     // bytes per group
  // output
  void* out;
  long out_pitch;
  long out_goff;
  int relu;
  // optional float32 term added to every output before the activation
  // (bf16 and float32 stores of single-group layers): add[pos * add_pitch + n].
  // Must not alias out: the autotuner runs a conv more than once.
  const float* add;
  long add_pitch;
  // FP8: per-output-channel weight scales [group][cout]; the amax (float
  // bits) of this layer's input and, for a producer, where its waves record
  // the amax of its own output: AMAX_SPREAD sub-slots AMAX_STRIDE words apart
  // (one 128-byte line each, so the atomics do not queue on one address)
  const float* wscale;
  const unsigned* amax_in;
  unsigned* amax_out;
};
constexpr int AMAX_SPREAD = 64, AMAX_STRIDE = 32;
__device__ __forceinline__ unsigned* amax_sub(unsigned* spread, unsigned who) {
  return spread + (who & (AMAX_SPREAD - 1)) * AMAX_STRIDE;
}

// Launches one conv layer.  `cfg` selects a tile configuration (see
// conv_tile_configs); returns hipErrorInvalidValue for unsupported combos.
hipError_t launch_conv(int prec, int loader, int store, int stride, int cfg,
                       const ConvArgs& a, int groups, hipStream_t s);

// Batched form: one launch over nwork work items (problem index, tile,
// first output channel, group) of the problems in descs (device memory).
hipError_t launch_conv_batch(int prec, int loader, int store, int stride, int cfg,
                             const ConvArgs* descs, const int4* work, int nwork, hipStream_t s);

// Tile configurations: output rows x cols per workgroup and channel tile.
struct TileCfg { int th, tw, bn; };
constexpr int kHyperCfg = 24;   // the stride-2 hyper conv's configuration (its own kernel)
// the entropy-parameter conv's two configurations (its own kernel; 4 x 16 or
// 4 x 24 hyper-latent positions, i.e. 8 x 32 or 8 x 48 outputs, 64 channels)
constexpr int kParamsCfg0 = 37, kParamsCfg1 = 38;
int conv_num_cfgs();
TileCfg conv_cfg(int cfg);
// false for tile configurations a layer cannot use (precision, loader,
// stride and channel counts)
bool conv_cfg_supported(int prec, int loader, int stride, int cin, int cout, int cfg);

// ------------------------------------------------------------ DC block ----
// One fused DC block (ufvc_dcblock.hip): bf16 [h][w][C] in and out, weights
// bf16 (out, in) matrices pw1 (C x C), pw2 (C x C), pw3 (2C x C), pw4
// (C x 2C) and float32 depth-wise taps dw [C][9].
struct DcBlockArgs {
  const __bf16* x;
  __bf16* y;
  int h, w;
  const __bf16* pw1;
  const __bf16* pw2;
  const __bf16* pw3;
  const __bf16* pw4;
  const float* dw;
};
// tile_rows: 4 or 8 (positions per workgroup: tile_rows x 16)
hipError_t launch_dc_block(int C, const DcBlockArgs& a, hipStream_t s, int tile_rows = 8);

// ------------------------------------------------------------- entropy ----
constexpr int NSCALES = 64;
constexpr int NSYM = 65;
constexpr int LANES = 32;
constexpr int LUT_BUCKETS = 256;   // decoder lookup buckets per table row
constexpr int LUT_SLOTS = 65536 / LUT_BUCKETS;
constexpr int SEG_STATE_BYTES = 4 * LANES;

// Device tables built once per context.
struct Tables {
  uint32_t* fc;      // [64][65] freq | cum << 16
  uint32_t* magic;   // [64][65] division multiplier for freq
  uint8_t* shift;    // [64][65] ceil(log2(freq))
  uint16_t* lut;     // [64][256] decoder lookup per 256-slot bucket
  float* thresholds; // [64] (63 used, [63] = +inf)
  uint8_t* tail;     // [64] length of the leading run of frequency-1 symbols
};

hipError_t launch_build_tables(const Tables& t, hipStream_t s);

// Encoder epilogue of the parameter net: idx (and symbols if y != null).
hipError_t launch_params_epilogue(const float* P, const float* y, const float* thr,
                                  uint8_t* idx, uint8_t* sym, long npos, int C,
                                  hipStream_t s);

struct SegInfo { uint32_t start_word; uint32_t nwords; };

// Encodes two symbol streams (z with a fixed row k_z, y with per-symbol rows)
// into per-segment scratch slots.
struct EncStream {
  const uint8_t* sym;
  const uint8_t* idx;   // null: every symbol uses row `fixed_row`
  int fixed_row;
  long n;
  int seg_log2;
  int n_seg;
};
hipError_t launch_rans_encode(const Tables& t, EncStream z, EncStream y, uint8_t* scratch,
                              size_t slot_bytes_z, size_t slot_bytes_y, SegInfo* info,
                              hipStream_t s);

// Writes header + segment table + segments; result[0] = total bytes.  When
// `with_header` is 0 the output is the bare table + segments.
struct HeaderFields {
  uint16_t T, C, H, W;
  uint8_t seg_log2, seg_log2_z, k_z;
  uint32_t model_tag;
  uint8_t flags;   // model structure bits (HDR_FLAG_*), header byte 15
};
constexpr uint8_t HDR_FLAG_QUADTREE = 1;   // four-step progressive means
constexpr uint8_t HDR_FLAG_TEMPORAL = 2;   // coded with the stream's temporal context
// seg_off: n_seg_z + n_seg_y words of scratch for the segments' offsets.
hipError_t launch_compact(const uint8_t* scratch, size_t slot_bytes_z, size_t slot_bytes_y,
                          const SegInfo* info, int n_seg_z, int n_seg_y, int with_header,
                          HeaderFields hf, uint8_t* out, size_t capacity,
                          unsigned long long* result, uint32_t* seg_off, hipStream_t s);

// Validates the stream (header if with_header) and computes segment byte
// offsets into seg_off[n_seg_z + n_seg_y] (0xFFFFFFFF marks unusable).
hipError_t launch_parse(const uint8_t* bs, size_t len, int with_header, HeaderFields expect,
                        int n_seg_z, int n_seg_y, uint32_t* seg_off, uint32_t* seg_len,
                        uint32_t* status, hipStream_t s);

// Symbol / index arrays read by the rANS coders must have CODER_PAD readable
// bytes past their end: the coders fetch whole epochs (1024 symbols of a
// segment) without branching.
constexpr size_t CODER_PAD = 2048;
struct DecStream {
  const uint8_t* idx;   // null: fixed row
  int fixed_row;
  long n;
  int seg_log2;
  int n_seg;
  int seg_base;         // index of the first segment in seg_off/seg_len
  uint8_t* sym_out;
  size_t len;           // bytes of the stream (reads are clamped into it)
};
hipError_t launch_rans_decode(const Tables& t, const uint8_t* bs, const uint32_t* seg_off,
                              const uint32_t* seg_len, DecStream d, uint32_t* status,
                              hipStream_t s);

// ---- Batched (descriptor-driven) forms: one launch for many chunks ----
// Problem descriptors live in device memory; the same kernels run with
// either inline arguments (one chunk) or these arrays (a batch).

// Entropy-parameter epilogue of one chunk (see launch_params_epilogue).
struct EpiDesc {
  const float* P;
  const float* y;    // null in the decoder
  uint8_t* idx;
  uint8_t* sym;
  long npos;
  int C;
  int pad;
};
constexpr int EPI_BLOCK_ELEMS = 4096;  // elements per block of the batched epilogue

// One rANS segment to encode.
struct EncSeg {
  const uint8_t* sym;   // first symbol of the segment (CODER_PAD readable past its stream)
  const uint8_t* idx;   // first table row of the segment, null: fixed_row for all
  uint8_t* slot;        // scratch: 128 state bytes + 2 * cap bytes of words
  SegInfo* info;        // receives the segment's word range
  uint32_t nsym;
  uint32_t cap;         // word capacity of the slot (>= nsym)
  uint32_t fixed_row;
  uint32_t pad;
};

// One rANS segment to decode (offsets come from the parse of its chunk).
struct DecSeg {
  const uint8_t* bs;         // the chunk's stream
  const uint32_t* seg_off;   // this segment's entry of the parse output
  const uint32_t* seg_len;
  const uint8_t* idx;        // first table row of the segment, null: fixed_row
  uint8_t* out;              // first decoded symbol of the segment
  uint32_t* status;
  unsigned long long len;    // bytes of the chunk's stream
  uint32_t nsym;
  uint32_t fixed_row;
};

// Container assembly of one chunk.
struct CompDesc {
  const uint8_t* scratch_z;  // first z slot
  const uint8_t* scratch_y;  // first y slot
  unsigned long long slot_z, slot_y;
  const SegInfo* info;       // z segments then y segments
  int n_seg_z, n_seg_y, with_header, pad;
  HeaderFields hf;
  uint8_t* out;
  unsigned long long capacity;
  unsigned long long* result;
  uint32_t* seg_off;         // scratch: byte offset of each segment in the container
};

// Stream validation of one chunk.
struct ParseDesc {
  const uint8_t* bs;
  unsigned long long len;
  int with_header, n_seg_z, n_seg_y, pad;
  HeaderFields ex;
  uint32_t* seg_off;
  uint32_t* seg_len;
  uint32_t* status;
};

hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s);

// FP8 synthesis: one layer input quantised for the FP8 convs.  dst[pos][c] =
// E4M3(src[pos * src_pitch + c] * 448 / amax) (round to nearest even,
// saturated at 448; scale 1 if amax is 0), for npos positions of C channels
// (a multiple of 16); the FP8 conv rescales by amax / 448.
struct Q8Job {
  const void* src;         // bf16
  long src_pitch;          // elements between positions
  void* dst;               // E4M3, C bytes per position
  long npos;
  int C;
  const unsigned* amax;    // the producer's amax sub-slots (float bits; see ConvArgs::amax_out)
  unsigned* amax_final;    // their maximum, written here for the conv and the caller
};
hipError_t launch_q8(const Q8Job& j, hipStream_t s);
// jobs: device array of n jobs, each of at most max_units 16-channel units
hipError_t launch_q8_batch(const Q8Job* jobs, int n, long max_units, hipStream_t s);
hipError_t launch_params_epilogue_batch(const EpiDesc* d, const int2* work, int nwork,
                                        const float* thr, hipStream_t s);
hipError_t launch_rans_encode_batch(const Tables& t, const EncSeg* segs, int nsegs, hipStream_t s);
hipError_t launch_compact_batch(const CompDesc* d, int nchunks, const int2* map, int nblocks,
                                hipStream_t s);
hipError_t launch_parse_batch(const ParseDesc* d, int nchunks, hipStream_t s);
hipError_t launch_rans_decode_batch(const Tables& t, const DecSeg* segs, int nsegs, bool fixed,
                                    hipStream_t s);

// Device status bits.
constexpr uint32_t ST_BAD_HEADER = 1u;
constexpr uint32_t ST_CORRUPT = 2u;

}  // namespace ufvc
