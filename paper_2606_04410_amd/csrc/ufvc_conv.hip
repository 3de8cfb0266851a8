// 3x3 convolution as implicit GEMM on CDNA4 matrix cores.
//
// GEMM view: M = output positions of a spatial tile (TH x TW), N = output
// channels (BN per workgroup), K = 9 taps x input channels.  Activations are
// channels-innermost, so one input position's channel run is contiguous.
//
// Per workgroup and per K slice of 32 bytes of input channels (16 bf16 or 8
// f32 channels) the kernel stages into LDS
//   * the input halo of the tile, (TH+2) x (TW+2) positions (stride 1) or
//     (2TH+1) x (2TW+1) (stride 2), 32-byte rows with an XOR swizzle of their
//     halves so that 16 consecutive rows hit disjoint banks, and
//   * the packed weights of that slice for all 9 taps and BN channels,
// then every wave runs 9 taps of 32x32 MFMA blocks (bf16 32x32x16 or four
// f32 32x32x2) reading A (positions x channels) from the halo shifted by the
// tap and B (channels x outputs) from the weight rows.  The next slice is
// fetched while the current one is multiplied: straight into a second LDS
// stage for inputs that are copied unchanged, into registers for inputs that
// a loader converts.  Reduction order is fixed: slice, then tap, then the
// MFMA's own order, and does not depend on the tile configuration, so results
// do not depend on how many workgroups cover the output (the patchify
// loader's split-K form sums even and odd slices separately, and is that
// loader's only form).  A second kernel family (conv3x3_ring_kernel, below)
// serves bf16 and FP8 activations at stride 1, and hyper_conv_kernel the
// stride-2 hyper conv (the first family's stride-2 form is not instantiated).
//
// Loaders fuse the producer's layout change into the halo fetch: the x8
// pixel-unshuffle of the patch embedding with edge-replicated padding
// (Sec. 3.1), y_hat = r_hat + mu dequantisation (Sec. 3.4), and nearest x2
// upsampling of the hyper latent (repeated over the three bf16 parts of the
// float32 entropy-parameter weights).  Epilogues fuse ReLU, the float32 or bf16
// store, rounding of z, and the x8 pixel-shuffle store of the frame
// decoders with crop and clamp (Sec. 3.2).
#include <algorithm>
#include <mutex>

#include "ufvc_common.h"

namespace ufvc {

template <int PREC> struct PT;
// E channels per slice; a slice of one position (or weight row) is ROWB bytes
// in LDS, CH chunks of 16 bytes.
template <> struct PT<P_BF16> {
  static constexpr int ESZ = 2, E = 16, ROWB = 32, CH = 2;
};
template <> struct PT<P_F32> {
  static constexpr int ESZ = 4, E = 8, ROWB = 32, CH = 2;
};
typedef int i32x8 __attribute__((ext_vector_type(8)));

// 16 bytes as a native vector (HIP's uint4 is a struct whose copies lower to
// memcpy and can pin staging arrays in scratch memory).
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v4u zero16() { return v4u{0u, 0u, 0u, 0u}; }

__device__ __forceinline__ v4u cvt8(const float* v) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = (__bf16)v[i];
  return __builtin_bit_cast(v4u, r);
}

// 16 bytes of device memory (global load)
__device__ __forceinline__ v4u ld16(const void* p) { return ldg(reinterpret_cast<const v4u*>(p)); }
// 16 bytes of LDS
__device__ __forceinline__ v4u lds16(const unsigned char* p) { return *reinterpret_cast<const v4u*>(p); }

// E4M3 saturates at +-448
__device__ __forceinline__ float sat448(float x) { return fminf(fmaxf(x, -448.f), 448.f); }

// A halo chunk is fetched in two steps so that the loads of the next slice
// stay in flight while the current one is multiplied: fetch_raw issues the
// loads into registers (device-memory words, unconverted), convert_raw turns
// them into 16 bytes of compute-type input when the chunk is written to LDS.
// The chunk covers channels [slice*E + ch*E/2, +E/2) at input position
// (iy, ix); outside the input grid it is
// zero (conv zero padding).  The loads are issued for every lane at clamped
// addresses, and padding and edge replication are applied in convert_raw:
// a lane-divergent branch around a load would make the next write to its
// registers wait for it.
struct Raw {
  v4u a, b;     // up to 32 bytes of activations, frame pixels or means
  v2u c;        // up to 8 bytes of symbols
  unsigned ok;  // inside the input grid
  unsigned rep; // frame loaders: the chunk lies past the right edge
};

template <int PREC, int LD>
__device__ __forceinline__ Raw fetch_raw(const ConvArgs& a, const unsigned char* inb, int slice,
                                         int ch, int iy, int ix) {
  constexpr int E = PT<PREC>::E;
  constexpr int ESZ = PT<PREC>::ESZ;
  Raw r;
  r.a = zero16();
  r.b = zero16();
  r.c = v2u{0u, 0u};
  r.ok = (iy >= 0 && ix >= 0 && iy < a.Hin && ix < a.Win) ? 1u : 0u;
  r.rep = 0u;
  iy = min(max(iy, 0), a.Hin - 1);
  ix = min(max(ix, 0), a.Win - 1);
  const long pos = (long)iy * a.Win + ix;
  if constexpr (LD == LD_NHWC) {
    r.a = ld16(inb + (pos * a.in_pitch + slice * E + ch * (E / 2)) * ESZ);
  } else if constexpr (LD == LD_F32) {
    static_assert(PREC == P_BF16, "use LD_NHWC for float32 compute");
    const float* fp = reinterpret_cast<const float*>(inb) + pos * a.in_pitch + slice * E + ch * (E / 2);
    r.a = __builtin_bit_cast(v4u, ldg(reinterpret_cast<const v4f*>(fp)));
    r.b = __builtin_bit_cast(v4u, ldg(reinterpret_cast<const v4f*>(fp + 4)));
  } else if constexpr (LD == LD_UNSHUFFLE) {
    // channel cb = t*192 + c*64 + i*8 + j  <->  pixel (8 iy + i, 8 ix + j) of plane t*3 + c,
    // rows and columns past the frame replicate its last one.  Frame widths
    // are multiples of 8 (at least 16), so a chunk lies wholly inside the
    // frame or wholly past its right edge (then every value is the last
    // column's, the last of the chunk fetched at the edge).
    constexpr int NPX = PREC == P_BF16 ? 8 : 4;
    const int cb = slice * E + ch * (E / 2);
    const int plane = cb >> 6;             // t*3 + c
    const int i = (cb >> 3) & 7;
    const int j0 = cb & 7;                 // 0 for bf16 (8 pixels), 0 or 4 for f32
    const int py = min(8 * iy + i, a.H - 1);
    const int px = 8 * ix + j0;
    r.rep = px + NPX > a.W ? 1u : 0u;
    const float* row = reinterpret_cast<const float*>(a.in) + ((long)plane * a.H + py) * a.W +
                       min(px, a.W - NPX);
    r.a = __builtin_bit_cast(v4u, ldg(reinterpret_cast<const v4f*>(row)));
    if constexpr (PREC == P_BF16) r.b = __builtin_bit_cast(v4u, ldg(reinterpret_cast<const v4f*>(row + 4)));
  } else if constexpr (LD == LD_DEQUANT) {
    const int c0 = slice * E + ch * (E / 2);
    const unsigned char* sp = reinterpret_cast<const unsigned char*>(a.in) + pos * a.cin + c0;
    const float* mp = a.mu + pos * a.mu_pitch + c0;
    if constexpr (PREC == P_BF16) {
      r.c = ldg(reinterpret_cast<const v2u*>(sp));
      r.a = __builtin_bit_cast(v4u, ldg(reinterpret_cast<const v4f*>(mp)));
      r.b = __builtin_bit_cast(v4u, ldg(reinterpret_cast<const v4f*>(mp + 4)));
    } else {
      r.c.x = ldg(reinterpret_cast<const uint32_t*>(sp));
      r.a = __builtin_bit_cast(v4u, ldg(reinterpret_cast<const v4f*>(mp)));
    }
  } else if constexpr (LD == LD_REP) {
    static_assert(PREC == P_BF16, "the repeating loader feeds bf16 split-weight convs");
    const int c0 = (slice * E + ch * (E / 2)) % (int)a.in_pitch;
    r.a = ld16(inb + (pos * a.in_pitch + c0) * ESZ);
  } else {
    static_assert(LD == LD_NHWC, "loader without a first-family form");
  }
  return r;
}

template <int PREC, int LD>
__device__ __forceinline__ v4u convert_raw(const Raw& r) {
  v4u o;
  if constexpr (LD == LD_NHWC || LD == LD_REP) {
    o = r.a;
  } else if constexpr (LD == LD_F32) {
    const v4f u0 = __builtin_bit_cast(v4f, r.a), u1 = __builtin_bit_cast(v4f, r.b);
    const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
    o = cvt8(v);
  } else if constexpr (LD == LD_UNSHUFFLE) {
    if constexpr (PREC == P_BF16) {
      const v4f u0 = __builtin_bit_cast(v4f, r.a), u1 = __builtin_bit_cast(v4f, r.b);
      float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
      if (r.rep) {
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] = v[7];
      }
      o = cvt8(v);
    } else {
      o = r.a;
      if (r.rep) o = v4u{o.w, o.w, o.w, o.w};
    }
  } else if constexpr (LD == LD_DEQUANT) {
    if constexpr (PREC == P_BF16) {
      const v2u sb = r.c;
      const v4f m0 = __builtin_bit_cast(v4f, r.a), m1 = __builtin_bit_cast(v4f, r.b);
      float v[8];
      v[0] = (float)((int)(sb.x & 255) - 32) + m0.x;
      v[1] = (float)((int)((sb.x >> 8) & 255) - 32) + m0.y;
      v[2] = (float)((int)((sb.x >> 16) & 255) - 32) + m0.z;
      v[3] = (float)((int)(sb.x >> 24) - 32) + m0.w;
      v[4] = (float)((int)(sb.y & 255) - 32) + m1.x;
      v[5] = (float)((int)((sb.y >> 8) & 255) - 32) + m1.y;
      v[6] = (float)((int)((sb.y >> 16) & 255) - 32) + m1.z;
      v[7] = (float)((int)(sb.y >> 24) - 32) + m1.w;
      o = cvt8(v);
    } else {
      const uint32_t sb = r.c.x;
      const v4f m = __builtin_bit_cast(v4f, r.a);
      v4f f;
      f[0] = (float)((int)(sb & 255) - 32) + m.x;
      f[1] = (float)((int)((sb >> 8) & 255) - 32) + m.y;
      f[2] = (float)((int)((sb >> 16) & 255) - 32) + m.z;
      f[3] = (float)((int)(sb >> 24) - 32) + m.w;
      o = __builtin_bit_cast(v4u, f);
    }
  }
  return r.ok ? o : zero16();
}

template <int ST>
__device__ __forceinline__ void store_out(const ConvArgs& a, int grp, int oy, int ox, int n, float v) {
  const long pos = (long)oy * a.Wout + ox;
  if constexpr (ST == ST_BF16 || ST == ST_F32) {
    if (a.add) v += ldg(a.add + pos * a.add_pitch + n);
  }
  if constexpr (ST == ST_BF16) {
    if (a.relu) v = fmaxf(v, 0.f);
    stg(reinterpret_cast<__bf16*>(a.out) + pos * a.out_pitch + grp * a.out_goff + n, (__bf16)v);
  } else if constexpr (ST == ST_F32) {
    if (a.relu) v = fmaxf(v, 0.f);
    stg(reinterpret_cast<float*>(a.out) + pos * a.out_pitch + grp * a.out_goff + n, v);
  } else if constexpr (ST == ST_ZSYM) {
    float z = fminf(fmaxf(rintf(v), -32.f), 32.f);
    stg(reinterpret_cast<unsigned char*>(a.out) + pos * a.out_pitch + n, (unsigned char)((int)z + 32));
  } else {  // ST_SHUFFLE: channel n = c*64 + i*8 + j -> pixel (8 oy + i, 8 ox + j)
    const int c = n >> 6, i = (n >> 3) & 7, j = n & 7;
    const int py = 8 * oy + i, px = 8 * ox + j;
    if (py < a.H && px < a.W)
      stg(reinterpret_cast<float*>(a.out) + (((long)grp * 3 + c) * a.H + py) * a.W + px,
          fminf(fmaxf(v, 0.f), 1.f));
  }
}

// LDS rows hold one position's (or weight row's) slice: 32 bytes (16 bf16,
// 8 f32 or 32 fp8 channels).  Their two 16-byte halves are XOR-swizzled with
// the row index (they swap every 8 rows), so 16 lanes reading the same half
// of 16 consecutive rows hit 64 distinct banks (no padding needed).
template <int ROWB>
__device__ __forceinline__ int lds_off(int row, int chunk) {
  static_assert(ROWB == 32, "32-byte rows");
  return row * 32 + ((chunk ^ ((row >> 3) & 1)) << 4);
}

// Tile position (row-major index into the TH x TW tile) of element j
// (0..31) of 32-position block b.  A block covers two tile rows of 16.  A
// wave-wide 16-byte LDS read runs at full rate only when lanes i and i + 16
// (and i + 32, i + 48) fall on the same banks, so the second row is rotated
// by the halo padding (2): lane i + 16 then reads the halo row 16 or 32
// rows after lane i's, which the swizzle maps to the same banks, for every
// tap.  Stride-2 tiles keep the plain order.
template <int STRIDE, int TW>
__device__ __forceinline__ int blk_pos(int b, int j) {
  if constexpr (STRIDE == 1 && TW == 16) return b * 32 + (j & 16) + ((j & 16) ? ((j - 2) & 15) : j);
  else return b * 32 + j;
}

// Staging pipeline of one tile configuration.  Loaders that copy the input
// unchanged (NHWC, bf16 or f32) stream each slice straight from global memory
// into LDS (global_load_lds_dwordx4: a wave writes 64 consecutive 16-byte
// chunks at a uniform LDS address, each lane fetching the global chunk that
// belongs at its position, XOR swizzle included), through two slice
// buffers: loads run one slice ahead, nothing is staged in registers and the
// block syncs once per slice.  Loaders that convert (unshuffle, dequantise,
// up-sample, quantise) stage through registers into a single buffer, one per
// K group (KS = 2: two wave groups take alternate slices).
template <int PREC, int LD, int STRIDE, int TH, int TW, int WM, int WN, int FN, int KS = 1>
struct Pipe {
  static constexpr int ROWB = PT<PREC>::ROWB, CH = PT<PREC>::CH;
  static constexpr int NWAVES = WM * WN;
  static constexpr int BN = WN * FN * 32;
  static constexpr int HP = STRIDE == 1 ? (TH + 2) * (TW + 2) : (2 * TH + 1) * (2 * TW + 1);
  static constexpr int NCH = (HP + 9 * BN) * CH;                  // 16-byte chunks per slice
  static constexpr int NIW = ((NCH + 63) / 64 + NWAVES - 1) / NWAVES;  // loads per wave and slice
  static constexpr int STAGE = NIW * NWAVES * 64 * 16;            // bytes, padded to whole loads
  static constexpr bool DIRECT =
      KS == 1 && LD == LD_NHWC && (PREC == P_BF16 || PREC == P_F32) && 2 * STAGE <= 160 * 1024;
  static constexpr int GROUP_LDS = (HP + 9 * BN) * ROWB;      // one K group's staging buffer
  static constexpr int LDS = DIRECT ? 2 * STAGE : KS * GROUP_LDS;
};

// Hyper-prior conv (Sec. 3.4): stride 2, pad 1, float32 operands on the
// matrix cores, z_hat = clamp(rint(z), -32, 32) stored as uint8 z_hat + 32.
// One wave per unit of 16 output positions of one row x 16 output channels
// (v_mfma_f32_16x16x4f32): with 32 output channels this gives four times the
// waves of a 32x32-block tiling, each with a quarter of the serial MFMA
// chain, and the layer is too small for anything but that chain to matter.
// Lane l holds position l % 16 of the unit (A row) and channel l % 16 (B
// column); lane group g = l / 16 holds channels 4g..4g+3 of each 16-channel
// chunk, and MFMA j of the chunk takes channel 4g + j.  K order: tap, chunk,
// j, then the MFMA's own sum.  Operands come straight from device memory
// (L2-resident, 16-byte loads, clamped into bounds, zero outside the input),
// nine K steps ahead of the multiplications; the steps are unrolled per
// input-channel count (64 or 128) so that the loads stay where they are.
// Weights are packed [tap][cin / 4][cout][4] floats.
template <int NCH>
__device__ __forceinline__ v4f hyper_mac(const ConvArgs& a, int oy, int ox, int g, const float* y,
                                         const float* wl) {
  constexpr int NS = 9 * NCH, D = 9;
  const long wtap = (long)(16 * NCH) * a.cout;   // floats per tap
  const long wchunk = 16L * a.cout;               // floats per 16 input channels
  v4f va[NS], vb[NS];
  bool ok[NS];
  auto load = [&](int k) {
    const int tap = k / NCH, cc = (k % NCH) * 16;
    const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
    ok[k] = ox < a.Wout && iy >= 0 && ix >= 0 && iy < a.Hin && ix < a.Win;
    va[k] = ldg(reinterpret_cast<const v4f*>(
        y + ((long)min(max(iy, 0), a.Hin - 1) * a.Win + min(max(ix, 0), a.Win - 1)) * a.in_pitch + 4 * g + cc));
    vb[k] = ldg(reinterpret_cast<const v4f*>(wl + tap * wtap + (k % NCH) * wchunk));
  };
#pragma unroll
  for (int k = 0; k < D; ++k) load(k);
  v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (k + D < NS) load(k + D);
    // keep the prefetch ahead of this step's multiplications (the scheduler
    // would otherwise move each load down to its use)
    __builtin_amdgcn_sched_barrier(0);
    const v4f av = ok[k] ? va[k] : v4f{0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, vb[k].x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, vb[k].y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, vb[k].z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, vb[k].w, acc, 0, 0, 0);
  }
  return acc;
}

// (One wave per SIMD is the target: the registers go to loads in flight.)
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2)))
hyper_conv_kernel(ConvArgs a0, const ConvArgs* __restrict__ descs, const int4* __restrict__ work,
                  int nwork) {
  ConvArgs a;
  int tile, n0;
  if (descs) {
    const int wi = blockIdx.x;
    if (wi >= nwork) return;
    const int4 w = work[wi];
    a = descs[w.x];
    tile = w.y;
    n0 = w.z;
  } else {
    a = a0;
    const int nt = a.Hout * ((a.Wout + 15) / 16);
    const int per = (nt + 7) >> 3;
    tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tile >= nt) return;
    n0 = blockIdx.y * 16;
  }
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  const int tiles_x = (a.Wout + 15) / 16;
  const int oy = tile / tiles_x;
  const int ox0 = (tile - oy * tiles_x) * 16;
  const int ox = ox0 + (lane & 15);
  const float* __restrict__ y = static_cast<const float*>(a.in);
  const float* __restrict__ wl =
      static_cast<const float*>(a.wpk) + ((long)g * a.cout + n0 + (lane & 15)) * 4;
  // cin is 64 or 128: the channel counts a context accepts (the single-launch
  // form also checks it before the launch)
  const v4f acc = a.cin == 128 ? hyper_mac<8>(a, oy, ox, g, y, wl) : hyper_mac<4>(a, oy, ox, g, y, wl);
  // acc[r]: position 4g + r of the unit, channel lane % 16
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int px = ox0 + 4 * g + r;
    if (px < a.Wout) store_out<ST_ZSYM>(a, 0, oy, px, n0 + (lane & 15), acc[r]);
  }
}

// ------------------------------------------- entropy-parameter conv ----
// The entropy parameters are a 3x3 conv (zero padding 1) over the nearest x2
// upsampling of z_hat (Sec. 3.4).  Output (2qy + py, 2qx + px) reads z_hat
// rows qy - 1 + py + r, r in {0, 1}: for py = 0, r = 0 collects kernel row 0
// and r = 1 kernel rows 1 and 2; for py = 1, r = 0 collects rows 0 and 1 and
// r = 1 row 2 (columns likewise).  The latent always has even height and
// width, so the upsampling is never cropped and every output parity class
// (py, px) is a 2x2 conv over z_hat with summed weights: 4 taps instead of 9.
// The host sums each class's weights in double and splits them into three
// bf16 parts; products with the symbols (integers -32..32, exact in bf16) are
// exact and the sums float32.
//
// A workgroup takes a 4 x 8FM tile of z_hat positions and 64 output channels;
// wave w computes class (py, px) = (w / 2, w % 2) as FM blocks of 32 positions
// (4 rows x 8 columns) on v_mfma_f32_32x32x16_bf16 with the weights as the
// first operand, so a lane ends with 16 channels of one position.  K order:
// tap, 16-channel half, weight part, then the MFMA's own.  Both operands are
// L2-resident and come straight from device memory, D K steps ahead.
// Weights: [class][tap][part][cout][32 channels] bf16.
template <int FM>
__global__ void __launch_bounds__(256) params_up2_kernel(ConvArgs a0, const ConvArgs* __restrict__ descs,
                                                         const int4* __restrict__ work, int nwork) {
  constexpr int ZTW = 8 * FM;                  // z_hat columns per tile
  constexpr int NS = 8, D = 2;                 // K steps (4 taps x 2 halves), lookahead
  ConvArgs a;
  int tile, n0;
  // Workgroups are dispatched round-robin over the 8 XCDs; each XCD takes a
  // contiguous band of items, numbered tile-major with the channel block
  // fastest, so the four blocks of a tile (a position's 256 channels of P)
  // are written from one L2 at about the same time.
  if (descs) {
    const int per = (nwork + 7) >> 3;
    const int wi = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (wi >= nwork) return;
    const int4 w = work[wi];
    a = descs[w.x];
    tile = w.y;
    n0 = w.z;
  } else {
    a = a0;
    const int nt = ((a.Hout + 7) / 8) * ((a.Wout + 2 * ZTW - 1) / (2 * ZTW));
    const int nb = a.cout / 64;
    const int per = (nt + 7) >> 3;
    const int L = blockIdx.x >> 3;
    tile = (blockIdx.x & 7) * per + L / nb;
    if (tile >= nt) return;
    n0 = (L % nb) * 64;
  }
  const int lane = threadIdx.x & 63;
  const int cls = threadIdx.x >> 6;
  const int py = cls >> 1, px = cls & 1;
  const int kh = lane >> 5;                    // channels 8kh..8kh+7 of a half
  const int j = lane & 31;
  const int hz = a.Hout >> 1, wz = a.Wout >> 1;
  const int tiles_x = (wz + ZTW - 1) / ZTW;
  const int qy = (tile / tiles_x) * 4 + (j >> 3);
  const int qx0 = (tile % tiles_x) * ZTW + (j & 7);
  const unsigned char* __restrict__ zs = static_cast<const unsigned char*>(a.in);
  const __bf16* __restrict__ wl =
      static_cast<const __bf16*>(a.wpk) + ((long)cls * 12 * a.cout + n0 + j) * 32 + kh * 8;

  v4u wa[NS][6];                               // [step][part * 2 + fn]
  v2u zb[NS][FM];
  bool zok[NS][FM];
  auto load = [&](int k) {
    const int t = k >> 1, half = k & 1;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int fn = 0; fn < 2; ++fn)
        wa[k][p * 2 + fn] = ld16(wl + ((long)(t * 3 + p) * a.cout + fn * 32) * 32 + half * 16);
    const int zy = qy - 1 + py + (t >> 1);
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
      const int zx = qx0 + fm * 8 - 1 + px + (t & 1);
      zok[k][fm] = zy >= 0 && zy < hz && zx >= 0 && zx < wz;
      const long zpos = (long)min(max(zy, 0), hz - 1) * wz + min(max(zx, 0), wz - 1);
      zb[k][fm] = ldg(reinterpret_cast<const v2u*>(zs + zpos * a.in_pitch + half * 16 + kh * 8));
    }
  };
  f32x16 acc[FM][2];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < 2; ++fn)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[fm][fn][r] = 0.f;
#pragma unroll
  for (int k = 0; k < D; ++k) load(k);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (k + D < NS) load(k + D);
    // keep the prefetch ahead of this step's multiplications
    __builtin_amdgcn_sched_barrier(0);
    bf16x8 xb[FM];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
      const v2u v = zb[k][fm];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        xb[fm][i] = (__bf16)(float)((int)((v.x >> (8 * i)) & 255u) - 32);
        xb[fm][4 + i] = (__bf16)(float)((int)((v.y >> (8 * i)) & 255u) - 32);
      }
      if (!zok[k][fm]) xb[fm] = bf16x8{};
    }
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int fn = 0; fn < 2; ++fn)
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
          acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, wa[k][p * 2 + fn]),
                                                               xb[fm], acc[fm][fn], 0, 0, 0);
  }
  // Register r of a lane holds channel 8 (r / 4) + 4 kh + r % 4 of position
  // j.  A block's 32 positions x 64 channels pass through LDS (rows of 64
  // floats padded by 4) and leave as 16-byte stores of which 16 consecutive
  // lanes cover one position's 256 contiguous bytes: whole 128-byte lines
  // instead of 32-byte pieces of 32 lines per store.
  constexpr int RS = 68;
  __shared__ __attribute__((aligned(16))) float tbuf[4][32 * RS];
  float* tb = tbuf[cls];
  const int qy0 = (tile / tiles_x) * 4, qxt = (tile % tiles_x) * ZTW;
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) {
#pragma unroll
    for (int fn = 0; fn < 2; ++fn)
#pragma unroll
      for (int g = 0; g < 4; ++g)
        *reinterpret_cast<v4f*>(tb + j * RS + fn * 32 + 8 * g + 4 * kh) =
            v4f{acc[fm][fn][4 * g], acc[fm][fn][4 * g + 1], acc[fm][fn][4 * g + 2], acc[fm][fn][4 * g + 3]};
    // (a wave's LDS accesses complete in order; this only pins the code order)
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int pp = it * 4 + (lane >> 4);
      const v4f v = *reinterpret_cast<const v4f*>(tb + pp * RS + (lane & 15) * 4);
      const int zy = qy0 + (pp >> 3), zx = qxt + fm * 8 + (pp & 7);
      if (zy < hz && zx < wz) {
        const long pos = (long)(2 * zy + py) * a.Wout + 2 * zx + px;
        const int n = n0 + (lane & 15) * 4;
        v4f o = v;
        if (a.add) o += ldg(reinterpret_cast<const v4f*>(a.add + pos * a.add_pitch + n));
        stg(reinterpret_cast<v4f*>(static_cast<float*>(a.out) + pos * a.out_pitch + n), o);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Zero chunk for halo positions outside the input (conv zero padding).
__device__ __attribute__((aligned(64))) unsigned char kZeroChunk[64];


// KS = 2 (split K): the workgroup holds two groups of WM x WN waves; group g
// stages and multiplies slices g, g + 2, g + 4, ... into its own
// accumulators, and group 1 adds its sums into group 0's through LDS at the
// end, so each output is (sum over even slices) + (sum over odd slices).
// Halving the output tile per K group is what lets 64 x 64 wave blocks (one
// LDS fragment read per MFMA instead of 1.5) fill the chip on a layer with
// few output tiles.
template <int PREC, int LD, int ST, int STRIDE, int TH, int TW, int WM, int WN, int FM, int FN, int KS = 1>
__global__ void __launch_bounds__(WM * WN * 64 * KS, KS == 2 ? 2 : 1)   // split K: two waves per SIMD
conv3x3_kernel(ConvArgs a0, const ConvArgs* __restrict__ descs, const int4* __restrict__ work,
               int nwork) {
  constexpr int NT = WM * WN * 64;   // threads of one K group
  constexpr int BM = TH * TW;
  static_assert(BM == WM * FM * 32, "tile rows must match the wave grid");
  constexpr int BN = WN * FN * 32;
  constexpr int HH = STRIDE == 1 ? TH + 2 : 2 * TH + 1;
  constexpr int HW = STRIDE == 1 ? TW + 2 : 2 * TW + 1;
  constexpr int HP = HH * HW;
  constexpr int ROWB = PT<PREC>::ROWB;
  constexpr int CH = PT<PREC>::CH;
  constexpr int HCH = HP * CH;
  constexpr int WCH = 9 * BN * CH;
  constexpr int HIT = (HCH + NT - 1) / NT;
  constexpr int WIT = (WCH + NT - 1) / NT;
  constexpr int E = PT<PREC>::E;
  constexpr int ESZ = PT<PREC>::ESZ;

  using PP = Pipe<PREC, LD, STRIDE, TH, TW, WM, WN, FN, KS>;
  static_assert(KS == 1 || (KS == 2 && !PP::DIRECT), "split K uses the register-staged pipeline");
  static_assert(KS == 1 || WM * WN * FM * FN * 4096 <= PP::LDS, "the K groups' sums pass through LDS");
  extern __shared__ __attribute__((aligned(16))) unsigned char sh[];
  const int kg = KS == 1 ? 0 : (int)(threadIdx.x >= NT);   // K group
  unsigned char* lds_h = sh + kg * PP::GROUP_LDS;
  unsigned char* lds_w = lds_h + HP * ROWB;

  const int tid = threadIdx.x - kg * NT;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN;
  const int wn = wave - wm * WN;
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous band of tiles (or work items) so neighbouring halos and shared
  // weights stay in its L2.  A batched launch reads its problem, tile, channel
  // tile and group from a work list; a single launch derives them from the
  // grid.
  ConvArgs a;
  int tile, n0, grp;
  if (descs) {
    const int per = (nwork + 7) >> 3;
    const int wi = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (wi >= nwork) return;
    const int4 w = work[wi];
    a = descs[w.x];
    tile = w.y;
    n0 = w.z;
    grp = w.w;
  } else {
    a = a0;
    const int nt = ((a.Hout + TH - 1) / TH) * ((a.Wout + TW - 1) / TW);
    const int per = (nt + 7) >> 3;
    tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tile >= nt) return;
    n0 = blockIdx.y * BN;
    grp = blockIdx.z;
  }
  const int tiles_x = (a.Wout + TW - 1) / TW;
  const int oy0 = (tile / tiles_x) * TH;
  const int ox0 = (tile % tiles_x) * TW;
  const int iy0 = STRIDE * oy0 - 1;
  const int ix0 = STRIDE * ox0 - 1;
  const int nslices = a.cin / E;

  const unsigned char* wbase = reinterpret_cast<const unsigned char*>(a.wpk) + grp * a.w_gstride;
  const unsigned char* inb = reinterpret_cast<const unsigned char*>(a.in) +
                            grp * a.in_goff * (LD == LD_F32 ? 4 : ESZ);

  // Staging registers for the next slice.  Written and read only through
  // fully unrolled loops with constant indices so they live in VGPRs.
  Raw hraw[HIT];
  v4u wreg[WIT];
#define UFVC_GLOAD(S_)                                                                   \
  do {                                                                                   \
    _Pragma("unroll") for (int i = 0; i < HIT; ++i) {                                    \
      /* lanes past the halo fetch its last chunk again (not stored) */                  \
      const int q = min(tid + i * NT, HCH - 1);                                          \
      int pos, ch;                                                                       \
      if (LD == LD_UNSHUFFLE) { ch = q / HP; pos = q - ch * HP; }                        \
      else { pos = q / CH; ch = q % CH; }                                                \
      const int hy = pos / HW, hx = pos - (pos / HW) * HW;                               \
      hraw[i] = fetch_raw<PREC, LD>(a, inb, (S_), ch, iy0 + hy, ix0 + hx);               \
    }                                                                                    \
    _Pragma("unroll") for (int i = 0; i < WIT; ++i) {                                    \
      const int q = min(tid + i * NT, WCH - 1);                                          \
      const int row = q / CH, ch = q % CH;                                               \
      const int tap = row / BN, n = row - (row / BN) * BN;                               \
      wreg[i] = ld16(wbase + (((long)((S_) * 9 + tap) * a.cout + n0 + n) * ROWB + ch * 16)); \
    }                                                                                    \
  } while (0)
#define UFVC_LSTORE()                                                                    \
  do {                                                                                   \
    _Pragma("unroll") for (int i = 0; i < HIT; ++i) {                                    \
      const int q = tid + i * NT;                                                        \
      int pos, ch;                                                                       \
      if (LD == LD_UNSHUFFLE) { ch = q / HP; pos = q - ch * HP; }                        \
      else { pos = q / CH; ch = q % CH; }                                                \
      if (HCH % NT == 0 || q < HCH)                                                      \
        *reinterpret_cast<v4u*>(lds_h + lds_off<ROWB>(pos, ch)) =                        \
            convert_raw<PREC, LD>(hraw[i]);                                              \
    }                                                                                    \
    _Pragma("unroll") for (int i = 0; i < WIT; ++i) {                                    \
      const int q = tid + i * NT;                                                        \
      if (WCH % NT == 0 || q < WCH)                                                      \
        *reinterpret_cast<v4u*>(lds_w + lds_off<ROWB>(q / CH, q % CH)) = wreg[i];        \
    }                                                                                    \
  } while (0)

  int arow[FM];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) {
    const int M = blk_pos<STRIDE, TW>(wm * FM + fm, lane & 31);
    const int r = M / TW, c = M - (M / TW) * TW;
    arow[fm] = STRIDE == 1 ? r * HW + c : 2 * r * HW + 2 * c;
  }
  const int khalf = lane >> 5;

  f32x16 acc[FM][FN];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[fm][fn][r] = 0.f;

  auto compute_slice = [&]() {
    // Fragments of tap t + 1 are read from LDS into the second register set
    // before the MFMAs of tap t are issued, so LDS latency overlaps the
    // matrix cores.  A lane's fragment is 16 bytes: half khalf of its row.
    v4u af[2][FM], bf[2][FN];
    auto read_frags = [&](int buf, int tap) {
      const int toff = (tap / 3) * HW + (tap % 3);
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) af[buf][fm] = lds16(lds_h + lds_off<ROWB>(arow[fm] + toff, khalf));
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
        bf[buf][fn] = lds16(lds_w + lds_off<ROWB>(tap * BN + (wn * FN + fn) * 32 + (lane & 31), khalf));
    };
    read_frags(0, 0);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int cur = tap & 1, nxt = cur ^ 1;
      if (tap + 1 < 9) read_frags(nxt, tap + 1);
      // keep the next tap's reads ahead of this tap's MFMAs
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
          if constexpr (PREC == P_BF16) {
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, af[cur][fm]), __builtin_bit_cast(bf16x8, bf[cur][fn]),
                acc[fm][fn], 0, 0, 0);
          } else {
            const v4f fa = __builtin_bit_cast(v4f, af[cur][fm]);
            const v4f fb = __builtin_bit_cast(v4f, bf[cur][fn]);
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa.x, fb.x, acc[fm][fn], 0, 0, 0);
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa.y, fb.y, acc[fm][fn], 0, 0, 0);
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa.z, fb.z, acc[fm][fn], 0, 0, 0);
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa.w, fb.w, acc[fm][fn], 0, 0, 0);
          }
        }
    }
  };
  if constexpr (PP::DIRECT) {
    // slice S_ into ring stage ST_: this wave's NIW loads of 64 chunks
    auto issue = [&](int S_, int ST_) {
      unsigned char* stage = sh + ST_ * PP::STAGE;
#pragma unroll
      for (int j = 0; j < PP::NIW; ++j) {
        const int ins = j * PP::NWAVES + wave;
        const int q = ins * 64 + lane;                 // physical chunk in the stage
        const unsigned char* src = kZeroChunk;
        if (q < HCH) {
          const int row = q / CH;
          const int c = (q % CH) ^ ((row >> 3) & 1);
          const int hy = row / HW, hx = row - (row / HW) * HW;
          const int iy = iy0 + hy, ix = ix0 + hx;
          if (iy >= 0 && ix >= 0 && iy < a.Hin && ix < a.Win)
            src = inb + (((long)iy * a.Win + ix) * a.in_pitch + (long)S_ * E + c * (16 / ESZ)) * ESZ;
        } else if (q < HCH + WCH) {
          const int row = (q - HCH) / CH;
          const int c = ((q - HCH) % CH) ^ ((row >> 3) & 1);
          const int tap = row / BN, n = row - (row / BN) * BN;
          src = wbase + (((long)(S_ * 9 + tap) * a.cout + n0 + n) * ROWB + c * 16);
        }
        __builtin_amdgcn_global_load_lds((const UFVC_GLOBAL void*)src,
                                         (__attribute__((address_space(3))) void*)(stage + ins * 1024),
                                         16, 0, 0);
      }
    };
    issue(0, 0);
    for (int s = 0; s < nslices; ++s) {
      // this wave's loads of slice s have landed; after the barrier every
      // wave's have, and every wave has finished reading the stage the next
      // loads overwrite
      wait_vmcnt<0>();
      asm volatile("s_barrier" ::: "memory");
      if (s + 1 < nslices) issue(s + 1, (s + 1) & 1);
      lds_h = sh + (s & 1) * PP::STAGE;
      lds_w = lds_h + HP * ROWB;
      compute_slice();
    }
    // no load may still be writing LDS when the block ends
    wait_vmcnt<0>();
  } else {
    UFVC_GLOAD(kg);
    for (int s = 0; s < nslices; s += KS) {
      UFVC_LSTORE();
      __syncthreads();
      UFVC_GLOAD(min(s + KS, nslices - KS) + kg);
      compute_slice();
      __syncthreads();
    }
  }
  if constexpr (KS == 2) {
    // group 1's sums to group 0 (the staging buffers are free after the last
    // barrier): 16-byte runs of 4 accumulator registers, lane-contiguous
    v4f* red = reinterpret_cast<v4f*>(sh);
    const int wave_ = tid >> 6;
    if (kg == 1) {
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            red[(((wave_ * FM + fm) * FN + fn) * 4 + q) * 64 + lane] =
                v4f{acc[fm][fn][4 * q], acc[fm][fn][4 * q + 1], acc[fm][fn][4 * q + 2], acc[fm][fn][4 * q + 3]};
    }
    __syncthreads();
    if (kg == 1) return;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const v4f t = red[(((wave_ * FM + fm) * FN + fn) * 4 + q) * 64 + lane];
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[fm][fn][4 * q + i] += t[i];
        }
  }
#undef UFVC_GLOAD
#undef UFVC_LSTORE

  // 32x32 accumulator block: register r of lane l holds row 8(r/4) + 4(l/32) + r%4, column l%32.
  float vmax = 0.f;
#pragma unroll
  for (int fm = 0; fm < FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
      const int n = n0 + (wn * FN + fn) * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int M = blk_pos<STRIDE, TW>(wm * FM + fm, (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3));
        const int oy = oy0 + M / TW, ox = ox0 + M % TW;
        const float v = acc[fm][fn][r];
        if (oy < a.Hout && ox < a.Wout) {
          store_out<ST>(a, grp, oy, ox, n, v);
          if constexpr (ST == ST_BF16) vmax = fmaxf(vmax, fabsf(a.relu ? fmaxf(v, 0.f) : v));
        }
      }
    }
  if constexpr (ST == ST_BF16) {
    // amax of the stored output for the next FP8 layer (non-negative float
    // bits order like unsigned integers, so the maximum is order independent)
    if (a.amax_out) {
      vmax = fmaxf(vmax, 0.f);
      for (int o = 32; o > 0; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o, 64));
      if (lane == 0)
        atomicMax(amax_sub(a.amax_out, (blockIdx.x + gridDim.x * blockIdx.y) * (WM * WN) + wave),
                  __float_as_uint((float)(__bf16)vmax));
    }
  }
}

// ------------------------------------------------ ring-staged bf16 conv ----
// Second kernel family for bf16 NHWC inputs at stride 1 (the synthesis and
// frame-decoder stacks).  Same GEMM view, slice order and tap order as
// conv3x3_kernel, with three changes:
//   * the output block is computed transposed (weights as the MFMA's first
//     operand), so a lane ends with 16 output channels of one position; one
//     lane-half exchange (v_permlane32_swap) gives each lane two runs of 8
//     consecutive channels, stored as 16-byte vectors;
//   * the input halo of a slice is fetched NH - 1 slices ahead through a ring
//     of NH halo stages, the weights one slice ahead through two stages, both
//     straight into LDS, so the activation reads (which miss L2) have several
//     slices of MFMA work to land in;
//   * the global address of every 16-byte chunk a lane fetches is computed
//     once per tile; a slice only adds its offset.
// Stages of one ring configuration.  A stage holds one slice of the halo
// (HCH 16-byte chunks) or of the weights (WCH chunks), written by whole
// 1 KB direct-to-LDS loads: IH (IW) loads per stage, load i issued by wave
// i % NWAVES, so a wave issues at most NIH (NIW) of them; the tail of the
// last load reads the zero chunk into the stage's padding.
template <int TH, int TW, int WM, int WN, int FM, int FN, int NH, int NW>
struct Ring {
  static constexpr int NWAVES = WM * WN;
  static constexpr int BN = WN * FN * 32;
  static constexpr int HW = TW + 2;
  static constexpr int HP = (TH + 2) * HW;
  static constexpr int HCH = HP * 2;           // 16-byte chunks of a halo slice
  static constexpr int WCH = 9 * BN * 2;       // 16-byte chunks of a weight slice
  static constexpr int IH = (HCH + 63) / 64, IW = (WCH + 63) / 64;
  static constexpr int NIH = (IH + NWAVES - 1) / NWAVES;
  static constexpr int NIW = (IW + NWAVES - 1) / NWAVES;
  static constexpr int HSTAGE = IH * 1024;
  static constexpr int WSTAGE = IW * 1024;
  static constexpr int LDS = NH * HSTAGE + NW * WSTAGE;
  static_assert(NH >= 2 && NH <= 3 && NW >= 2 && NW <= 3, "one or two slices of lookahead per stream");
  static_assert(NIH + NIW < 64, "vmcnt range");
};

// s_waitcnt vmcnt(n) for a wave-uniform n <= K (an immediate is needed, so
// count down; waiting for fewer outstanding loads than allowed is safe).
template <int K>
__device__ __forceinline__ void wait_vmcnt_le(int n) {
  if constexpr (K == 0) {
    wait_vmcnt<0>();
  } else {
    if (n >= K) wait_vmcnt<K>();
    else wait_vmcnt_le<K - 1>(n);
  }
}

// Work items of the ring kernel are (tile, channel block, group).  A plain
// launch gives each workgroup one item from its grid position.  The
// persistent form launches as many workgroups as fit on the chip; each walks
// its own list of items and keeps the slice pipeline running across item
// boundaries: the first halo and weight slices of its next item are in
// flight while it finishes (and stores) the current one.  Items are numbered
// group-major, then tile, then channel block; each XCD takes a contiguous
// band of them (workgroups are dispatched round-robin over the 8 XCDs), so
// the workgroups resident on one XCD share input halos and weights in its L2.
//
// F8: E4M3 operands (the input quantised beforehand, per-tensor scale amax /
// 448; weights per output channel).  A slice is then 32 input channels, so
// its halo and weight rows are 32 bytes as in the bf16 form and the stages,
// swizzle and schedule are the same.  One v_mfma_scale_f32_32x32x64_f8f6f4
// takes K = 64 = two taps x 32 channels (lanes 0-31 tap 2p, lanes 32-63 tap
// 2p + 1; the ninth tap's partner is a zero weight row), so a slice is five
// MFMAs per block instead of nine.  The epilogue applies the scales.
template <int ST, int TH, int TW, int WM, int WN, int FM, int FN, int NH, int NW, bool PERSIST, bool F8 = false>
__global__ void __launch_bounds__(WM * WN * 64, PERSIST ? 2 : 1)   // persistent: two waves per SIMD
conv3x3_ring_kernel(ConvArgs a0, const ConvArgs* __restrict__ descs, const int4* __restrict__ work,
                    int nwork) {
  using R = Ring<TH, TW, WM, WN, FM, FN, NH, NW>;
  constexpr int BN = R::BN, HW = R::HW, HCH = R::HCH, WCH = R::WCH;
  constexpr int NIH = R::NIH, NIW = R::NIW, NWAVES = R::NWAVES;
  constexpr int LH = NH - 1, LW = NW - 1;      // slices of lookahead: halo, weights
  static_assert(TH * TW == WM * FM * 32, "tile positions must match the wave grid");
  extern __shared__ __attribute__((aligned(16))) unsigned char sh[];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN;
  const int wn = wave - wm * WN;
  // this wave's loads per stage: load j * NWAVES + wave exists for j < cH (cW)
  const int cH = (R::IH - wave + NWAVES - 1) / NWAVES;
  const int cW = (R::IW - wave + NWAVES - 1) / NWAVES;

  ConvArgs a;
  int first = 0, step = 1, count = 1;          // items first + k * step, k < count
  int tile0 = 0, n00 = 0, grp0 = 0, nt = 1, ncb = 1;
  if (descs) {
    const int per = (nwork + 7) >> 3;
    const int wi = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (wi >= nwork) return;
    const int4 w = work[wi];
    a = descs[w.x];
    tile0 = w.y;
    n00 = w.z;
    grp0 = w.w;
  } else {
    a = a0;
    nt = ((a.Hout + TH - 1) / TH) * ((a.Wout + TW - 1) / TW);
    if constexpr (PERSIST) {
      // nwork carries the group count
      ncb = a.cout / BN;
      const int n = nt * ncb * nwork;
      const int per = (n + 7) >> 3, p8 = gridDim.x >> 3;
      const int lo = (blockIdx.x & 7) * per + (blockIdx.x >> 3), hi = min(n, ((blockIdx.x & 7) + 1) * per);
      if (lo >= hi) return;
      first = lo;
      step = p8;
      count = (hi - lo + p8 - 1) / p8;
    } else {
      const int per = (nt + 7) >> 3;
      tile0 = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
      if (tile0 >= nt) return;
      n00 = blockIdx.y * BN;
      grp0 = blockIdx.z;
    }
  }
  auto item = [&](int k, int& tile, int& n0, int& grp) {
    if (PERSIST && !descs) {
      const int L = first + k * step;
      const int t = L / ncb;
      n0 = (L - t * ncb) * BN;
      tile = t % nt;
      grp = t / nt;
    } else {
      tile = tile0;
      n0 = n00;
      grp = grp0;
    }
  };
  const int tiles_x = (a.Wout + TW - 1) / TW;
  constexpr int ESZ = F8 ? 1 : 2;              // bytes per element
  const int ns = a.cin / (32 / ESZ);
  const int total = count * ns;                // slices over all items
  // FP8: the input's dequantisation scale
  float qscale = 1.f;
  if constexpr (F8) {
    const float amax = __uint_as_float(ldg(a.amax_in));
    if (amax > 0.f) qscale = amax / 448.f;
  }

  // Halo sources of the item the halo loads are on.  LDS chunk q of a stage
  // holds row q / 2, half (q & 1) ^ swizzle(row), the layout the fragment
  // reads expect; rows outside the input read the zero chunk (no slice step).
  const unsigned char* hsrc[NIH];
  int hstep[NIH];
  auto set_halo = [&](int tile, int grp) {
    const int oy0 = (tile / tiles_x) * TH, ox0 = (tile % tiles_x) * TW;
    const unsigned char* inb = reinterpret_cast<const unsigned char*>(a.in) + grp * a.in_goff * ESZ;
#pragma unroll
    for (int j = 0; j < NIH; ++j) {
      const int q = (j * NWAVES + wave) * 64 + lane;
      hsrc[j] = kZeroChunk;
      hstep[j] = 0;
      if (q < HCH) {
        const int row = q >> 1;
        const int c = (q & 1) ^ ((row >> 3) & 1);
        const int iy = oy0 - 1 + row / HW, ix = ox0 - 1 + row % HW;
        if (iy >= 0 && ix >= 0 && iy < a.Hin && ix < a.Win) {
          hsrc[j] = inb + ((long)iy * a.Win + ix) * a.in_pitch * ESZ + c * 16;
          hstep[j] = 32;
        }
      }
    }
  };
  // Weight chunk offsets within a slice for channel block 0 (an item adds
  // n0 * 32); -1 past the slice.
  int woff[NIW];
#pragma unroll
  for (int j = 0; j < NIW; ++j) {
    const int q = (j * NWAVES + wave) * 64 + lane;
    woff[j] = -1;
    if (q < WCH) {
      const int row = q >> 1;
      const int c = (q & 1) ^ ((row >> 3) & 1);
      const int tap = row / BN, n = row - (row / BN) * BN;
      woff[j] = ((tap * a.cout + n) * 32 + c * 16);
    }
  }
  const long wslice = 9L * a.cout * 32;
  auto wbase_of = [&](int n0, int grp) {
    return reinterpret_cast<const unsigned char*>(a.wpk) + grp * a.w_gstride + (long)n0 * 32;
  };
  unsigned char* const hring = sh;
  unsigned char* const wring = sh + NH * R::HSTAGE;

  // the halo and weight load cursors: item, slice
  int hk = 0, hs = 0, wk = 0, ws = 0;
  const unsigned char* wsrc;
  {
    int t, n0, g;
    item(0, t, n0, g);
    set_halo(t, g);
    wsrc = wbase_of(n0, g);
  }
  auto next_h = [&](int stage) {
    if (hs == ns) {
      hs = 0;
      int t, n0, g;
      item(++hk, t, n0, g);
      set_halo(t, g);
    }
#pragma unroll
    for (int j = 0; j < NIH; ++j)
      if (j < cH)
        __builtin_amdgcn_global_load_lds(
            (const UFVC_GLOBAL void*)(hsrc[j] + hs * hstep[j]),
            (__attribute__((address_space(3))) void*)(hring + stage * R::HSTAGE + (j * NWAVES + wave) * 1024),
            16, 0, 0);
    ++hs;
  };
  auto next_w = [&](int stage) {
    if (ws == ns) {
      ws = 0;
      int t, n0, g;
      item(++wk, t, n0, g);
      wsrc = wbase_of(n0, g);
    }
#pragma unroll
    for (int j = 0; j < NIW; ++j)
      if (j < cW) {
        const unsigned char* src = woff[j] >= 0 ? wsrc + ws * wslice + woff[j] : kZeroChunk;
        __builtin_amdgcn_global_load_lds(
            (const UFVC_GLOBAL void*)src,
            (__attribute__((address_space(3))) void*)(wring + stage * R::WSTAGE + (j * NWAVES + wave) * 1024),
            16, 0, 0);
      }
    ++ws;
  };

  // positions (MFMA columns) of this lane in each of the wave's FM blocks
  int xrow[FM];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) {
    const int M = blk_pos<1, TW>(wm * FM + fm, lane & 31);
    xrow[fm] = (M / TW) * HW + (M % TW);
  }
  const int khalf = lane >> 5;
  f32x16 acc[FN][FM];
  auto zero_acc = [&]() {
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[fn][fm][r] = 0.f;
  };
  zero_acc();

  // F8: per lane, the halo offset of its tap in each tap pair
  int toffp[5];
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    const int t = min(2 * p + khalf, 8);
    toffp[p] = (t / 3) * HW + (t % 3);
  }
  auto compute_slice8 = [&](const unsigned char* lh, const unsigned char* lw) {
    i32x8 xf[2][FM], wf[2][FN];
    auto rd32 = [&](const unsigned char* base, int row) {
      const v4u lo = lds16(base + lds_off<32>(row, 0)), hi = lds16(base + lds_off<32>(row, 1));
      return i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    };
    auto read_frags = [&](int buf, int p) {
      const int tap = min(2 * p + khalf, 8);
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) {
        wf[buf][fn] = rd32(lw, tap * BN + (wn * FN + fn) * 32 + (lane & 31));
        // the ninth tap has no partner: zero weights (any halo value then
        // contributes nothing)
        if (p == 4 && khalf) wf[buf][fn] = i32x8{0, 0, 0, 0, 0, 0, 0, 0};
      }
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) xf[buf][fm] = rd32(lh, xrow[fm] + toffp[p]);
    };
    read_frags(0, 0);
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      const int cur = p & 1;
      if (p + 1 < 5) read_frags(cur ^ 1, p + 1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
          // E4M3 x E4M3, block scales 2^0
          acc[fn][fm] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(wf[cur][fn], xf[cur][fm], acc[fn][fm],
                                                                       0, 0, 0, 127, 0, 127);
    }
  };
  auto compute_slice16 = [&](const unsigned char* lh, const unsigned char* lw) {
    v4u xf[2][FM], wf[2][FN];
    auto read_frags = [&](int buf, int tap) {
      const int toff = (tap / 3) * HW + (tap % 3);
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
        wf[buf][fn] = lds16(lw + lds_off<32>(tap * BN + (wn * FN + fn) * 32 + (lane & 31), khalf));
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) xf[buf][fm] = lds16(lh + lds_off<32>(xrow[fm] + toff, khalf));
    };
    read_frags(0, 0);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int cur = tap & 1;
      if (tap + 1 < 9) read_frags(cur ^ 1, tap + 1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
          acc[fn][fm] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, wf[cur][fn]),
                                                               __builtin_bit_cast(bf16x8, xf[cur][fm]),
                                                               acc[fn][fm], 0, 0, 0);
    }
  };
  auto compute_slice = [&](const unsigned char* lh, const unsigned char* lw) {
    if constexpr (F8) compute_slice8(lh, lw);
    else compute_slice16(lh, lw);
  };

  // Lane l holds, per block, position (l & 31) and channels
  // 8 (r / 4) + 4 (l / 32) + r % 4.  Swapping registers r and r + 4 (r % 8
  // < 4) between the lane halves leaves lane l < 32 with channels 0-7 and
  // 16-23 in registers 0-7 and 8-15, lane l + 32 with 8-15 and 24-31.
  float vmax = 0.f;
  auto epilogue = [&](int tile, int n0b, int grp) {
    const int oy0 = (tile / tiles_x) * TH, ox0 = (tile % tiles_x) * TW;
    const int cofs = (lane >> 5) * 8;
#pragma unroll
    for (int fn = 0; fn < FN; ++fn)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) {
        f32x16 v = acc[fn][fm];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[8 * h + r]),
                                                            __float_as_uint(v[8 * h + r + 4]), false, false);
            v[8 * h + r] = __uint_as_float(p[0]);
            v[8 * h + r + 4] = __uint_as_float(p[1]);
          }
        const int M = blk_pos<1, TW>(wm * FM + fm, lane & 31);
        const int oy = oy0 + M / TW, ox = ox0 + M % TW;
        if (oy >= a.Hout || ox >= a.Wout) continue;
        const long pos = (long)oy * a.Wout + ox;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int n = n0b + (wn * FN + fn) * 32 + h * 16 + cofs;   // first of 8 channels
          float o[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) o[k] = v[8 * h + k];
          if constexpr (F8) {
            const float* ws = a.wscale + grp * a.cout + n;
            const v4f s0 = ldg(reinterpret_cast<const v4f*>(ws)), s1 = ldg(reinterpret_cast<const v4f*>(ws + 4));
            const float sc[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
            for (int k = 0; k < 8; ++k) o[k] *= qscale * sc[k];
          }
          if constexpr (ST == ST_BF16 || ST == ST_F32) {
            if (a.add) {
              const float* ad = a.add + pos * a.add_pitch + n;
              const v4f a0 = ldg(reinterpret_cast<const v4f*>(ad)), a1 = ldg(reinterpret_cast<const v4f*>(ad + 4));
              o[0] += a0.x; o[1] += a0.y; o[2] += a0.z; o[3] += a0.w;
              o[4] += a1.x; o[5] += a1.y; o[6] += a1.z; o[7] += a1.w;
            }
            if (a.relu) {
#pragma unroll
              for (int k = 0; k < 8; ++k) o[k] = fmaxf(o[k], 0.f);
            }
          }
          if constexpr (ST == ST_BF16) {
            bf16x8 b;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              b[k] = (__bf16)o[k];
              vmax = fmaxf(vmax, fabsf(o[k]));
            }
            stg(reinterpret_cast<v4u*>(reinterpret_cast<__bf16*>(a.out) + pos * a.out_pitch + grp * a.out_goff + n),
                __builtin_bit_cast(v4u, b));
          } else if constexpr (ST == ST_F32) {
            float* dst = reinterpret_cast<float*>(a.out) + pos * a.out_pitch + grp * a.out_goff + n;
            stg(reinterpret_cast<v4f*>(dst), v4f{o[0], o[1], o[2], o[3]});
            stg(reinterpret_cast<v4f*>(dst + 4), v4f{o[4], o[5], o[6], o[7]});
          } else {
            static_assert(ST == ST_SHUFFLE, "ring kernel stores bf16, float32 or shuffled frames");
            // channels n .. n + 7 = c*64 + i*8 + (0..7): pixels (8 oy + i, 8 ox + 0..7)
            const int c = n >> 6, i = (n >> 3) & 7;
            const int py = 8 * oy + i, px = 8 * ox;
            if (py < a.H) {
#pragma unroll
              for (int k = 0; k < 8; ++k) o[k] = fminf(fmaxf(o[k], 0.f), 1.f);
              float* dst = reinterpret_cast<float*>(a.out) + (((long)grp * 3 + c) * a.H + py) * a.W + px;
              if ((a.W & 3) == 0 && (reinterpret_cast<uintptr_t>(a.out) & 15) == 0 && px + 8 <= a.W) {
                stg(reinterpret_cast<v4f*>(dst), v4f{o[0], o[1], o[2], o[3]});
                stg(reinterpret_cast<v4f*>(dst + 4), v4f{o[4], o[5], o[6], o[7]});
              } else {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                  if (px + k < a.W) stg(dst + k, o[k]);
              }
            }
          }
        }
      }
  };

  // Ring schedule over the slices g = 0 .. total - 1 of all items: halos
  // 0 .. LH - 1 and weights 0 .. LW - 1 before the loop; iteration g issues
  // the stream with the shorter lookahead first, then the other (halo g + LH,
  // weights g + LW).  Loads complete in issue order, so at the top of
  // iteration g halo g and weights g have landed once no more than the loads
  // issued after the later of them are outstanding: those of iteration g - 1
  // that are not needed yet.  (Stores of a finished item, issued after them,
  // only make that wait stricter.)
#pragma unroll
  for (int g = 0; g < LH; ++g)
    if (g < total) next_h(g);
#pragma unroll
  for (int g = 0; g < LW; ++g)
    if (g < total) next_w(g);
  [[maybe_unused]] int ck = 0, cs = 0;
  int c_tile, c_n0, c_grp;
  item(0, c_tile, c_n0, c_grp);
  for (int g = 0; g < total; ++g) {
    if (g == 0) {
      wait_vmcnt<0>();
    } else {
      int after = 0;
      if (g + 1 < total) {
        if constexpr (LH == 2 && LW == 2) after = cH + cW;
        else if constexpr (LH == 1 && LW == 2) after = cW;
        else if constexpr (LH == 2 && LW == 1) after = cH;
      }
      wait_vmcnt_le<NIH + NIW>(after);
    }
    // every wave's chunks of slice g are in LDS, and every wave is done with
    // slice g - 1, whose stages the next loads overwrite
    asm volatile("s_barrier" ::: "memory");
    if constexpr (LH <= LW) {
      if (g + LH < total) next_h((g + LH) % NH);
      if (g + LW < total) next_w((g + LW) % NW);
    } else {
      if (g + LW < total) next_w((g + LW) % NW);
      if (g + LH < total) next_h((g + LH) % NH);
    }
    compute_slice(hring + (g % NH) * R::HSTAGE, wring + (g % NW) * R::WSTAGE);
    if constexpr (PERSIST) {
      if (++cs == ns) {
        epilogue(c_tile, c_n0, c_grp);
        zero_acc();
        cs = 0;
        if (++ck < count) item(ck, c_tile, c_n0, c_grp);
      }
    }
  }
  // no load may still be writing LDS when the block ends
  wait_vmcnt<0>();
  // one item per workgroup: its epilogue after the loop, where the loop's
  // registers are free
  if constexpr (!PERSIST) epilogue(c_tile, c_n0, c_grp);
  if constexpr (ST == ST_BF16) {
    if (a.amax_out) {
      vmax = fmaxf(vmax, 0.f);
      for (int o = 32; o > 0; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o, 64));
      if (lane == 0)
        atomicMax(amax_sub(a.amax_out, (blockIdx.x + gridDim.x * blockIdx.y) * NWAVES + wave),
                  __float_as_uint((float)(__bf16)vmax));
    }
  }
}

// ------------------------------------------------------------ dispatch ----
// cfg: 0 = 8x16 tile, 128 channels, 2x2 waves of 64x64
//      1 = 8x16 tile,  32 channels, 4x1 waves of 32x32 (narrow outputs)
//      2 = 8x16 tile, 192 channels, 2x2 waves of 64x96
//      3 = 4x16 tile, 128 channels, 2x2 waves of 32x64 (more workgroups)
//      4 = 8x16 tile,  64 channels, 2x2 waves of 64x32
//      5 = 16x16 tile, 128 channels, 2x2 waves of 128x64
//      6 = 16x16 tile, 192 channels, 2x2 waves of 128x96
//      7 = 16x16 tile,  64 channels, 2x2 waves of 128x32
//      8 = 16x16 tile, 128 channels, 8 waves (4x2) of 64x64
//      9 = 16x16 tile,  64 channels, 8 waves (4x2) of 64x32
//     ring-staged bf16 NHWC kernel (halo ring of 3 stages):
//     10 = 16x16 tile, 128 channels, 2x2 waves of 128 positions x 64 channels
//     11 = 8x16 tile, 128 channels, 2x2 waves of 64x64
//     12 = 8x16 tile,  64 channels, 2x2 waves of 64x32
//     13 = 16x16 tile,  64 channels, 2x2 waves of 128x32
//     14 = 16x16 tile, 128 channels, 8 waves (4x2) of 64x64
//     15 = 16x16 tile, 192 channels, 2x2 waves of 128x96
//     16 = 8x16 tile, 192 channels, 2x2 waves of 64x96
//     17 = 8x16 tile,  32 channels, 4x1 waves of 32x32
//     18 = 16x16 tile,  64 channels, 4x1 waves of 64x64
//     19 = 8x16 tile,  64 channels, 4x1 waves of 32x64
//     first family again:
//     20 = 8x16 tile,  64 channels, 4x1 waves of 32x64
//     21 = 16x16 tile,  64 channels, 4x1 waves of 64x64
//     22 = 2x16 tile,  32 channels, one wave (small outputs)
//     23 = 4x16 tile,  32 channels, 2x1 waves of 32x32
//   hyper_conv_kernel (the stride-2 hyper conv, float32, and nothing else):
//     24 = 1x16 tile,  16 channels, one wave of 16x16
//   ring kernel with the weights two slices ahead (tile, waves as listed),
//   persistent (P) or one item per workgroup:
//     25 = 16x16 tile, 64 channels, 4x1 waves of 64x64; halo 1 ahead; P
//     26 = 8x16 tile,  64 channels, 4x1 waves of 32x64; halo 2 ahead; P
//     27 = 16x16 tile, 64 channels, 4x1 waves of 64x64; halo 1 ahead
//     28 = 8x16 tile,  64 channels, 4x1 waves of 32x64; halo 2 ahead
//   persistent ring kernel with the weights one slice ahead:
//     29 = 16x16 tile, 64 channels, 4x1 waves of 64x64; halo 2 ahead; P
//     30 = 8x16 tile,  64 channels, 4x1 waves of 32x64; halo 2 ahead; P
//   first family split over K between two wave groups (the patchify loader
//   takes these and only these, so its results never depend on the choice):
//     31 = 8x16 tile,  64 channels, 2 groups of 2x1 waves of 64x64
//     32 = 8x16 tile, 128 channels, 2 groups of 2x2 waves of 64x64
//   ring kernel with one slice of lookahead per stream and small stages, so
//   that three (33, 34) or four (35, 36) workgroups share a CU:
//     33 = 8x16 tile,  64 channels, 4x1 waves of 32x64
//     34 = 8x16 tile,  64 channels, 4x1 waves of 32x64; P
//     35 = 16x16 tile, 32 channels, 4x1 waves of 64x32
//     36 = 16x16 tile, 32 channels, 4x1 waves of 64x32; P
//   params_up2_kernel (the entropy-parameter conv over up2(z_hat), and
//   nothing else; output tile, i.e. twice the hyper-latent tile):
//     37 = 8x32 tile,  64 channels, one wave per output parity class
//     38 = 8x48 tile,  64 channels, one wave per output parity class
static const TileCfg kCfgs[] = {{8, 16, 128}, {8, 16, 32},  {8, 16, 192},  {4, 16, 128},
                                {8, 16, 64},  {16, 16, 128}, {16, 16, 192}, {16, 16, 64},
                                {16, 16, 128}, {16, 16, 64},
                                {16, 16, 128}, {8, 16, 128}, {8, 16, 64},  {16, 16, 64},
                                {16, 16, 128}, {16, 16, 192}, {8, 16, 192}, {8, 16, 32},
                                {16, 16, 64}, {8, 16, 64},
                                {8, 16, 64}, {16, 16, 64}, {2, 16, 32}, {4, 16, 32},
                                {1, 16, 16},
                                {16, 16, 64}, {8, 16, 64}, {16, 16, 64}, {8, 16, 64},
                                {16, 16, 64}, {8, 16, 64},
                                {8, 16, 64}, {8, 16, 128},
                                {8, 16, 64}, {8, 16, 64}, {16, 16, 32}, {16, 16, 32},
                                {8, 32, 64}, {8, 48, 64}};
constexpr int kFirstRing = 10, kLastRing = 19, kFirstRing2 = 25, kLastRing2 = 30;
constexpr int kFirstSplitK = 31, kLastSplitK = 32, kFirstRing3 = 33, kLastRing3 = 36;
int conv_num_cfgs() { return (int)(sizeof(kCfgs) / sizeof(kCfgs[0])); }
bool conv_cfg_supported(int prec, int loader, int stride, int cin, int cout, int cfg) {
  // stride 2 (the hyper conv) has the one configuration, so its results
  // cannot depend on the choice either
  if (stride == 2 || cfg == kHyperCfg)
    return cfg == kHyperCfg && stride == 2 && prec == P_F32 && loader == LD_NHWC &&
           (cin == 64 || cin == 128) && cout % 16 == 0;
  // the entropy-parameter conv over up2(z_hat) has its own kernel, whose two
  // configurations sum in the same order
  const bool params = cfg == kParamsCfg0 || cfg == kParamsCfg1;
  if (loader == LD_UP2 || params)
    return params && loader == LD_UP2 && prec == P_BF16 && stride == 1 && cin == 32 && cout % 64 == 0;
  const bool ring = (cfg >= kFirstRing && cfg <= kLastRing) || (cfg >= kFirstRing2 && cfg <= kLastRing2) ||
                    (cfg >= kFirstRing3 && cfg <= kLastRing3);
  // FP8 synthesis convs: the ring kernel on a quantised copy of the input
  if (prec == P_FP8) return ring && loader == LD_NHWC && stride == 1 && cin % 32 == 0;
  if (cfg >= kFirstSplitK && cfg <= kLastSplitK)
    return loader == LD_UNSHUFFLE && (prec == P_BF16 || prec == P_F32) && stride == 1 &&
           cin % (prec == P_BF16 ? 32 : 16) == 0;
  if (loader == LD_UNSHUFFLE) return false;
  if (ring) return prec == P_BF16 && loader == LD_NHWC && stride == 1 && cin % 16 == 0;
  return cfg >= 0 && cfg < conv_num_cfgs();
}

hipError_t set_lds_limit_once(std::atomic<uint32_t>& done, const void* kern, int bytes) {
  int dev = 0;
  if (const hipError_t e = hipGetDevice(&dev)) return e;
  if (dev < 0 || dev >= 32) return hipErrorInvalidDevice;
  const uint32_t bit = 1u << dev;
  if (done.load(std::memory_order_acquire) & bit) return hipSuccess;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (done.load(std::memory_order_relaxed) & bit) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) done.fetch_or(bit, std::memory_order_release);
  return e;
}

__global__ void zero_u32_kernel(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// One thread per 16 channels of one position: two 16-byte bf16 loads, one
// 16-byte E4M3 store (a plain HBM stream).
// The producer's amax: the maximum of its sub-slots (one wave reads them;
// non-negative float bits order like unsigned integers), written to the
// slot by the first workgroup.
__device__ __forceinline__ float q8_amax(const Q8Job& j) {
  __shared__ unsigned s_amax;
  if (threadIdx.x < 64) {
    unsigned v = threadIdx.x < AMAX_SPREAD ? ldg(j.amax + threadIdx.x * AMAX_STRIDE) : 0u;
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o, 64));
    if (threadIdx.x == 0) {
      s_amax = v;
      if (blockIdx.x == 0) stg(j.amax_final, v);
    }
  }
  __syncthreads();
  return __uint_as_float(s_amax);
}

__device__ __forceinline__ void q8_units(const Q8Job& j, float amax, long u0, long ustep) {
  const int per = j.C >> 4;
  const long units = j.npos * per;
  float qinv = 1.f;
  if (amax > 0.f) qinv = 448.f / amax;
  for (long u = u0; u < units; u += ustep) {
    const long pos = u / per;
    const int c0 = (int)(u - pos * per) * 16;
    const v4u* src = reinterpret_cast<const v4u*>(reinterpret_cast<const __bf16*>(j.src) + pos * j.src_pitch + c0);
    const bf16x8 b0 = __builtin_bit_cast(bf16x8, ldg(src)), b1 = __builtin_bit_cast(bf16x8, ldg(src + 1));
    v4u o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bf16x8& bb = k < 2 ? b0 : b1;
      const int q = (k & 1) * 4;
      int w = __builtin_amdgcn_cvt_pk_fp8_f32(sat448((float)bb[q] * qinv), sat448((float)bb[q + 1] * qinv), 0,
                                              false);
      w = __builtin_amdgcn_cvt_pk_fp8_f32(sat448((float)bb[q + 2] * qinv), sat448((float)bb[q + 3] * qinv), w,
                                          true);
      o[k] = (unsigned)w;
    }
    stg(reinterpret_cast<v4u*>(reinterpret_cast<uint8_t*>(j.dst) + pos * j.C + c0), o);
  }
}

__global__ void __launch_bounds__(256) q8_kernel(Q8Job j) {
  const float amax = q8_amax(j);
  q8_units(j, amax, (long)blockIdx.x * 256 + threadIdx.x, (long)gridDim.x * 256);
}

__global__ void __launch_bounds__(256) q8_batch_kernel(const Q8Job* __restrict__ jobs) {
  const Q8Job j = jobs[blockIdx.y];
  const float amax = q8_amax(j);
  q8_units(j, amax, (long)blockIdx.x * 256 + threadIdx.x, (long)gridDim.x * 256);
}

hipError_t launch_q8(const Q8Job& j, hipStream_t s) {
  if (j.C % 16 || j.npos < 0) return hipErrorInvalidValue;
  const long units = j.npos * (j.C / 16);
  if (units == 0) return hipSuccess;
  const long blocks = std::min<long>((units + 255) / 256, 4096);
  hipLaunchKernelGGL(q8_kernel, dim3((unsigned)blocks), dim3(256), 0, s, j);
  return hipGetLastError();
}

hipError_t launch_q8_batch(const Q8Job* jobs, int n, long max_units, hipStream_t s) {
  if (n <= 0 || max_units <= 0) return hipSuccess;
  const long blocks = std::min<long>((max_units + 255) / 256, 4096);
  hipLaunchKernelGGL(q8_batch_kernel, dim3((unsigned)blocks, (unsigned)n), dim3(256), 0, s, jobs);
  return hipGetLastError();
}
TileCfg conv_cfg(int c) { return kCfgs[c]; }

// descs == nullptr: one problem `a` over a (tiles, cout / BN, groups) grid.
// Otherwise: nwork items of the work list over the problems in descs.
template <int PREC, int LD, int ST, int STRIDE, int TH, int TW, int WM, int WN, int FM, int FN, int KS = 1>
static hipError_t run_conv(const ConvArgs& a, int groups, const ConvArgs* descs, const int4* work,
                           int nwork, hipStream_t s) {
  constexpr int BN = WN * FN * 32;
  constexpr int lds = Pipe<PREC, LD, STRIDE, TH, TW, WM, WN, FN, KS>::LDS;
  auto kern = conv3x3_kernel<PREC, LD, ST, STRIDE, TH, TW, WM, WN, FM, FN, KS>;
  static std::atomic<uint32_t> attr_done{0};
  if (const hipError_t e = set_lds_limit_once(attr_done, reinterpret_cast<const void*>(kern), lds))
    return e;
  dim3 grid;
  if (descs) {
    if (nwork <= 0) return hipSuccess;
    grid = dim3(((nwork + 7) / 8) * 8, 1, 1);
  } else {
    if (a.cout % BN || a.cin % (PT<PREC>::E * KS)) return hipErrorInvalidValue;
    const int tiles = ((a.Hout + TH - 1) / TH) * ((a.Wout + TW - 1) / TW);
    grid = dim3(((tiles + 7) / 8) * 8, a.cout / BN, groups);
  }
  hipLaunchKernelGGL(kern, grid, dim3(WM * WN * 64 * KS), lds, s, a, descs, work, nwork);
  return hipGetLastError();
}

// Workgroups of kern resident on the whole chip at once (per device, cached).
static int chip_slots(std::atomic<int>* cache, const void* kern, int threads, int lds) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 32) return 0;
  int v = cache[dev].load(std::memory_order_acquire);
  if (v > 0) return v;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  v = per_cu * cus;
  if (v > 0) cache[dev].store(v, std::memory_order_release);
  return v;
}

template <int ST, int TH, int TW, int WM, int WN, int FM, int FN, int NH, int NW, bool PERSIST, bool F8>
static hipError_t run_ring(const ConvArgs& a, int groups, const ConvArgs* descs, const int4* work,
                           int nwork, hipStream_t s) {
  using R = Ring<TH, TW, WM, WN, FM, FN, NH, NW>;
  auto kern = conv3x3_ring_kernel<ST, TH, TW, WM, WN, FM, FN, NH, NW, PERSIST, F8>;
  static std::atomic<uint32_t> attr_done{0};
  if (const hipError_t e = set_lds_limit_once(attr_done, reinterpret_cast<const void*>(kern), R::LDS))
    return e;
  dim3 grid;
  int arg = nwork;
  if (descs) {
    if (nwork <= 0) return hipSuccess;
    grid = dim3(((nwork + 7) / 8) * 8, 1, 1);
  } else {
    if (a.cout % R::BN || a.cin % (F8 ? 32 : 16)) return hipErrorInvalidValue;
    const int tiles = ((a.Hout + TH - 1) / TH) * ((a.Wout + TW - 1) / TW);
    if constexpr (PERSIST) {
      static std::atomic<int> slots[32];
      const int sl = chip_slots(slots, reinterpret_cast<const void*>(kern), WM * WN * 64, R::LDS);
      if (sl <= 0) return hipErrorLaunchFailure;
      const long items = (long)tiles * (a.cout / R::BN) * groups;
      const long p = std::min<long>(items, sl);
      grid = dim3((unsigned)(((p + 7) / 8) * 8), 1, 1);
      arg = groups;
    } else {
      grid = dim3(((tiles + 7) / 8) * 8, a.cout / R::BN, groups);
    }
  }
  hipLaunchKernelGGL(kern, grid, dim3(WM * WN * 64), R::LDS, s, a, descs, work, arg);
  return hipGetLastError();
}

static hipError_t run_hyper(const ConvArgs& a, int groups, const ConvArgs* descs, const int4* work,
                            int nwork, hipStream_t s) {
  dim3 grid;
  if (descs) {
    if (nwork <= 0) return hipSuccess;
    grid = dim3(((nwork + 7) / 8) * 8, 1, 1);
  } else {
    if (groups != 1 || a.cout % 16 || (a.cin != 64 && a.cin != 128)) return hipErrorInvalidValue;
    const int tiles = a.Hout * ((a.Wout + 15) / 16);
    grid = dim3(((tiles + 7) / 8) * 8, a.cout / 16, 1);
  }
  hipLaunchKernelGGL(hyper_conv_kernel, grid, dim3(64), 0, s, a, descs, work, nwork);
  return hipGetLastError();
}

template <int FM>
static hipError_t run_params(const ConvArgs& a, const ConvArgs* descs, const int4* work, int nwork,
                             hipStream_t s) {
  dim3 grid;
  if (descs) {
    if (nwork <= 0) return hipSuccess;
    grid = dim3(((nwork + 7) / 8) * 8, 1, 1);
  } else {
    // even latent (never a cropped upsampling), 32 symbol channels, 64-channel
    // output blocks, no activation
    if (((a.Hout | a.Wout) & 1) || a.Hin != a.Hout || a.Win != a.Wout || a.cin != 32 || a.in_pitch != 32 ||
        a.cout <= 0 || a.cout % 64 || a.relu)
      return hipErrorInvalidValue;
    const int tiles = ((a.Hout + 7) / 8) * ((a.Wout + 16 * FM - 1) / (16 * FM));
    if (tiles == 0) return hipSuccess;
    grid = dim3(((tiles + 7) / 8) * 8 * (a.cout / 64), 1, 1);
  }
  hipLaunchKernelGGL(params_up2_kernel<FM>, grid, dim3(256), 0, s, a, descs, work, nwork);
  return hipGetLastError();
}

template <int PREC, int LD, int ST, int STRIDE>
static hipError_t run_cfg(int cfg, const ConvArgs& a, int groups, const ConvArgs* d,
                          const int4* w, int nw, hipStream_t s) {
  if constexpr (STRIDE == 2) {
    // the hyper conv: its one configuration
    if constexpr (PREC == P_F32 && LD == LD_NHWC && ST == ST_ZSYM)
      if (cfg == kHyperCfg) return run_hyper(a, groups, d, w, nw, s);
    return hipErrorInvalidValue;
  }
  if constexpr (PREC != P_FP8) {
  switch (cfg) {
    case 0: return run_conv<PREC, LD, ST, STRIDE, 8, 16, 2, 2, 2, 2>(a, groups, d, w, nw, s);
    case 1: return run_conv<PREC, LD, ST, STRIDE, 8, 16, 4, 1, 1, 1>(a, groups, d, w, nw, s);
    case 2: return run_conv<PREC, LD, ST, STRIDE, 8, 16, 2, 2, 2, 3>(a, groups, d, w, nw, s);
    case 3: return run_conv<PREC, LD, ST, STRIDE, 4, 16, 2, 2, 1, 2>(a, groups, d, w, nw, s);
    case 4: return run_conv<PREC, LD, ST, STRIDE, 8, 16, 2, 2, 2, 1>(a, groups, d, w, nw, s);
    case 5: return run_conv<PREC, LD, ST, STRIDE, 16, 16, 2, 2, 4, 2>(a, groups, d, w, nw, s);
    case 6: return run_conv<PREC, LD, ST, STRIDE, 16, 16, 2, 2, 4, 3>(a, groups, d, w, nw, s);
    case 7: return run_conv<PREC, LD, ST, STRIDE, 16, 16, 2, 2, 4, 1>(a, groups, d, w, nw, s);
    case 8: return run_conv<PREC, LD, ST, STRIDE, 16, 16, 4, 2, 2, 2>(a, groups, d, w, nw, s);
    case 9: return run_conv<PREC, LD, ST, STRIDE, 16, 16, 4, 2, 2, 1>(a, groups, d, w, nw, s);
    case 20: return run_conv<PREC, LD, ST, STRIDE, 8, 16, 4, 1, 1, 2>(a, groups, d, w, nw, s);
    case 21: return run_conv<PREC, LD, ST, STRIDE, 16, 16, 4, 1, 2, 2>(a, groups, d, w, nw, s);
    case 22: return run_conv<PREC, LD, ST, STRIDE, 2, 16, 1, 1, 1, 1>(a, groups, d, w, nw, s);
    case 23: return run_conv<PREC, LD, ST, STRIDE, 4, 16, 2, 1, 1, 1>(a, groups, d, w, nw, s);
    default: break;
  }
  }
  if constexpr (LD == LD_UNSHUFFLE && STRIDE == 1 && (PREC == P_BF16 || PREC == P_F32)) {
    switch (cfg) {
      case 31: return run_conv<PREC, LD, ST, STRIDE, 8, 16, 2, 1, 2, 2, 2>(a, groups, d, w, nw, s);
      case 32: return run_conv<PREC, LD, ST, STRIDE, 8, 16, 2, 2, 2, 2, 2>(a, groups, d, w, nw, s);
      default: break;
    }
  }
  if constexpr ((PREC == P_BF16 || PREC == P_FP8) && LD == LD_NHWC && STRIDE == 1 && ST != ST_ZSYM) {
    constexpr bool F8 = PREC == P_FP8;
    switch (cfg) {
      case 10: return run_ring<ST, 16, 16, 2, 2, 4, 2, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 11: return run_ring<ST, 8, 16, 2, 2, 2, 2, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 12: return run_ring<ST, 8, 16, 2, 2, 2, 1, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 13: return run_ring<ST, 16, 16, 2, 2, 4, 1, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 14: return run_ring<ST, 16, 16, 4, 2, 2, 2, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 15: return run_ring<ST, 16, 16, 2, 2, 4, 3, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 16: return run_ring<ST, 8, 16, 2, 2, 2, 3, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 17: return run_ring<ST, 8, 16, 4, 1, 1, 1, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 18: return run_ring<ST, 16, 16, 4, 1, 2, 2, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 19: return run_ring<ST, 8, 16, 4, 1, 1, 2, 3, 2, false, F8>(a, groups, d, w, nw, s);
      case 25: return run_ring<ST, 16, 16, 4, 1, 2, 2, 2, 3, true, F8>(a, groups, d, w, nw, s);
      case 26: return run_ring<ST, 8, 16, 4, 1, 1, 2, 3, 3, true, F8>(a, groups, d, w, nw, s);
      case 27: return run_ring<ST, 16, 16, 4, 1, 2, 2, 2, 3, false, F8>(a, groups, d, w, nw, s);
      case 28: return run_ring<ST, 8, 16, 4, 1, 1, 2, 3, 3, false, F8>(a, groups, d, w, nw, s);
      case 29: return run_ring<ST, 16, 16, 4, 1, 2, 2, 3, 2, true, F8>(a, groups, d, w, nw, s);
      case 30: return run_ring<ST, 8, 16, 4, 1, 1, 2, 3, 2, true, F8>(a, groups, d, w, nw, s);
      case 33: return run_ring<ST, 8, 16, 4, 1, 1, 2, 2, 2, false, F8>(a, groups, d, w, nw, s);
      case 34: return run_ring<ST, 8, 16, 4, 1, 1, 2, 2, 2, true, F8>(a, groups, d, w, nw, s);
      case 35: return run_ring<ST, 16, 16, 4, 1, 2, 1, 2, 2, false, F8>(a, groups, d, w, nw, s);
      case 36: return run_ring<ST, 16, 16, 4, 1, 2, 1, 2, 2, true, F8>(a, groups, d, w, nw, s);
      default: break;
    }
  }
  switch (cfg) {
    default: return hipErrorInvalidValue;
  }
}

static hipError_t dispatch(int prec, int loader, int store, int stride, int cfg, const ConvArgs& a,
                           int groups, const ConvArgs* d, const int4* w, int nw, hipStream_t s) {
#define UFVC_CONV(P, L, S, STR)                                         \
  if (prec == P && loader == L && store == S && stride == STR)          \
    return run_cfg<P, L, S, STR>(cfg, a, groups, d, w, nw, s);
  // bf16 analysis / synthesis
  UFVC_CONV(P_BF16, LD_UNSHUFFLE, ST_BF16, 1)
  UFVC_CONV(P_BF16, LD_NHWC, ST_BF16, 1)
  UFVC_CONV(P_BF16, LD_NHWC, ST_F32, 1)
  UFVC_CONV(P_BF16, LD_DEQUANT, ST_BF16, 1)
  UFVC_CONV(P_BF16, LD_NHWC, ST_SHUFFLE, 1)
  UFVC_CONV(P_BF16, LD_F32, ST_BF16, 1)
  // entropy parameters: float32 weights as three bf16 parts (exact products)
  UFVC_CONV(P_BF16, LD_REP, ST_F32, 1)
  if (loader == LD_UP2) {
    if (prec != P_BF16 || store != ST_F32 || stride != 1) return hipErrorInvalidValue;
    if (cfg == kParamsCfg0) return run_params<2>(a, d, w, nw, s);
    if (cfg == kParamsCfg1) return run_params<3>(a, d, w, nw, s);
    return hipErrorInvalidValue;
  }
  // fp8 synthesis (input quantised beforehand)
  UFVC_CONV(P_FP8, LD_NHWC, ST_BF16, 1)
  UFVC_CONV(P_FP8, LD_NHWC, ST_SHUFFLE, 1)
  // float32 everything, plus the hyper prior
  UFVC_CONV(P_F32, LD_UNSHUFFLE, ST_F32, 1)
  UFVC_CONV(P_F32, LD_NHWC, ST_F32, 1)
  UFVC_CONV(P_F32, LD_DEQUANT, ST_F32, 1)
  UFVC_CONV(P_F32, LD_NHWC, ST_SHUFFLE, 1)
  UFVC_CONV(P_F32, LD_NHWC, ST_ZSYM, 2)
#undef UFVC_CONV
  return hipErrorInvalidValue;
}

hipError_t launch_conv(int prec, int loader, int store, int stride, int cfg,
                       const ConvArgs& a, int groups, hipStream_t s) {
  return dispatch(prec, loader, store, stride, cfg, a, groups, nullptr, nullptr, 0, s);
}

hipError_t launch_conv_batch(int prec, int loader, int store, int stride, int cfg,
                             const ConvArgs* descs, const int4* work, int nwork, hipStream_t s) {
  ConvArgs none{};
  return dispatch(prec, loader, store, stride, cfg, none, 1, descs, work, nwork, s);
}

}  // namespace ufvc
