// Internal definitions shared by the C ABI sources (context, geometry,
// tiling helpers).
#pragma once
#include <map>
#include <vector>

#include "../../include/ufvc.h"
#include "ufvc_common.h"

namespace ufvc {
constexpr int ZC = 32;   // hyper-latent channels
constexpr int K_Z = 22;  // table row of every z symbol (sigma ~ 1)

struct Layer {
  void* w = nullptr;   // packed [group][slice][tap][cout][32 bytes (64 for fp8)]
  float* wscale = nullptr;  // fp8: per-output-channel dequantisation scale [group][cout]
  long gstride = 0;    // bytes per group
  int cin = 0, cout = 0, groups = 0, prec = 0;
};

struct Workspace {
  int h = 0, w = 0;               // latent size the buffers are sized for
  void* act0 = nullptr;           // [h][w][C], compute type
  void* act1 = nullptr;
  float* y = nullptr;             // [h][w][C]
  uint8_t* zsym = nullptr;        // [hz][wz][32]
  float* P = nullptr;             // [h][w][2C]
  uint8_t* idx = nullptr;         // [h][w][C]
  uint8_t* sym = nullptr;         // [h][w][C]
  void* big0 = nullptr;           // [h][w][T C]
  void* big1 = nullptr;
  float* side = nullptr;          // temporal models: [h][w][2C], a conv of the context
  uint8_t* q8 = nullptr;          // FP8 synthesis: a layer's quantised input, [h][w][T C]
};

struct RansWs {
  size_t scratch_bytes = 0;
  uint8_t* scratch = nullptr;
  int nseg_cap = 0;
  SegInfo* info = nullptr;
  uint32_t* seg_off = nullptr;
  uint32_t* seg_len = nullptr;
  // padded copies of caller-provided symbol / index arrays (the coders read
  // 32-byte windows that may run past the end of an array)
  size_t pad_cap = 0;
  uint8_t* pad_a = nullptr;
  uint8_t* pad_b = nullptr;
};

}  // namespace ufvc

using namespace ufvc;

struct ufvc_ctx {
  ufvc_config cfg{};
  int device = 0;
  Tables tab{};
  Layer a1, a2, a3, h, p, d1, d2, d3, k1, k2, k3;
  // quadtree progressive means: steps 1..3, each [tap][part][C / 8][C][8] bf16
  __bf16* mw = nullptr;
  size_t mw_kstride = 0;
  // temporal context: context network c1, c2 and the context inputs of a1,
  // of the entropy parameters (split into three bf16 parts in the bf16
  // modes) and of d1
  Layer c1, c2, a1c, pc, d1c;
  Workspace ws;
  RansWs rw;
  unsigned long long* result = nullptr;      // device
  unsigned long long* result_host = nullptr; // pinned
  uint32_t* status = nullptr;                // device
  uint32_t* status_host = nullptr;           // pinned
  uint32_t* amax = nullptr;                  // device, N_AMAX float bit patterns (fp8 synthesis)
  hipStream_t last_stream = nullptr;
  int last_h = 0, last_w = 0;
  // per-stage timing (events recorded on the caller's stream around kernels)
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Rec { int stage; hipEvent_t e0, e1; };
  std::vector<Rec> prof_rec;
  // autotuned tile configuration per (conv stage, output height, width)
  std::map<uint64_t, int> tune;
  // test hook: tile configuration used by every conv layer that supports it
  int force_cfg = -1;
};

#define CK(x)                                   \
  do {                                          \
    if ((x) != hipSuccess) return UFVC_E_DEVICE; \
  } while (0)

enum Stage {
  S_A1, S_A2, S_A3, S_HYPER, S_PARAMS_ENC, S_EPI_ENC, S_RANS_ENC, S_COMPACT, S_PARSE,
  S_RANS_DEC_Z, S_PARAMS_DEC, S_EPI_DEC, S_RANS_DEC_Y, S_D1, S_D2, S_D3, S_K1, S_K2, S_K3,
  S_MEANS_ENC, S_MEANS_DEC, S_CTXIN_ENC, S_CTXIN_DEC, S_CHUNKDEC_ENC, S_CTXNET_ENC, S_CTXNET_DEC,
  S_COUNT
};
// autotuner keys of the context layers (distinct from the stage ids above)
enum TuneId { T_A1C = 64, T_PC, T_D1C, T_C1, T_C2 };
static const char* kStageNames[S_COUNT] = {
    "a1_conv", "a2_conv", "a3_conv", "hyper_conv", "params_conv_enc", "params_epilogue_enc",
    "rans_encode", "compact", "parse", "rans_decode_z", "params_conv_dec", "params_epilogue_dec",
    "rans_decode_y", "d1_conv", "d2_conv", "d3_conv", "k1_conv", "k2_conv", "k3_conv",
    "mean_steps_enc", "mean_steps_dec", "context_inputs_enc", "context_inputs_dec",
    "chunk_decoder_enc", "context_net_enc", "context_net_dec"};


namespace ufvc {
inline int default_cfg(int cout, long npos, int stride = 1, int loader = -1, int prec = -1) {
  if (stride == 2) return kHyperCfg;
  if (loader == LD_UP2) return kParamsCfg0;
  // the patchify loader runs split over K (its only configurations)
  if (loader == LD_UNSHUFFLE) return 31;
  // FP8 convs run on the ring kernel only (16x16 or 8x16 tiles, 64 channels)
  if (prec == P_FP8) return npos >= 16384 ? 18 : 19;
  if (cout % 128 == 0) return npos >= 16384 ? 5 : 0;
  if (cout % 192 == 0) return 2;
  if (cout % 64 == 0) return 4;
  return 1;
}

inline uint64_t tune_key(int id, int h, int w) {
  return ((uint64_t)id << 40) | ((uint64_t)h << 20) | (uint64_t)w;
}

inline int act_elem_size(int prec) { return prec == UFVC_FP32 ? 4 : 2; }
inline int conv_prec(int prec) { return prec == UFVC_FP32 ? P_F32 : P_BF16; }
// d2, d3 and the frame heads; d1 (which dequantises the latent) stays at conv_prec
inline int synth_prec(int prec) { return prec == UFVC_BF16_FP8 ? P_FP8 : conv_prec(prec); }
// amax slots of the fp8 synthesis chain: outputs of d1, d2, d3, k1, k2.
// Per context (or batch chunk) AMAX_WORDS words: the N_AMAX slots, then each
// slot's sub-slots, which its producer's waves fill and the quantise pass
// that consumes the slot reduces into it.
constexpr int N_AMAX = 8;
constexpr int AMAX_WORDS = N_AMAX * (1 + AMAX_SPREAD * AMAX_STRIDE);
inline uint32_t* amax_spread(uint32_t* base, int k) {
  return base + N_AMAX + (size_t)k * AMAX_SPREAD * AMAX_STRIDE;
}

inline int nseg_of(long n, int sl) { return n == 0 ? 0 : (int)((n + (1L << sl) - 1) >> sl); }
inline size_t slot_bytes(int sl) { return (size_t)SEG_STATE_BYTES + 2 * ((size_t)1 << sl); }

struct Geom {
  int Hp, Wp, h, w, hz, wz;
  long ny, nz;
  int nseg_y, nseg_z;
};

inline bool geom(const ufvc_ctx* c, int H, int W, Geom& g) {
  if (H < 16 || W < 16 || (H & 7) || (W & 7) || H > 65535 || W > 65535) return false;
  g.Hp = (H + 15) / 16 * 16;
  g.Wp = (W + 15) / 16 * 16;
  g.h = g.Hp / 8;
  g.w = g.Wp / 8;
  g.hz = (g.h + 1) / 2;
  g.wz = (g.w + 1) / 2;
  g.ny = (long)g.h * g.w * c->cfg.C;
  g.nz = (long)g.hz * g.wz * ZC;
  g.nseg_y = nseg_of(g.ny, c->cfg.seg_log2);
  g.nseg_z = nseg_of(g.nz, c->cfg.seg_log2_z);
  return true;
}

// Header flag bits of the model structure a stream needs.
inline uint8_t header_flags(const ufvc_ctx* c) {
  return (uint8_t)((c->cfg.quadtree ? HDR_FLAG_QUADTREE : 0) | (c->cfg.temporal ? HDR_FLAG_TEMPORAL : 0));
}

inline ConvArgs conv_args(int Hin, int Win, int Hout, int Wout, const Layer& L) {
  ConvArgs a{};
  a.Hin = Hin;
  a.Win = Win;
  a.Hout = Hout;
  a.Wout = Wout;
  a.cin = L.cin;
  a.cout = L.cout;
  a.wpk = L.w;
  a.w_gstride = L.gstride;
  a.wscale = L.wscale;
  return a;
}

}  // namespace ufvc

// Batch executor hooks used by the request server (defined in ufvc_batch.hip).
// Shared-arena mode: every plan of `b` lays its chunks out in one arena of at
// most `cap` bytes, grown on demand (call before the first batch).
int batch_set_arena_cap(ufvc_batch* b, size_t cap);
// Arena bytes one chunk of model `c` at H x W takes in a batch (0: invalid size).
size_t batch_chunk_footprint(ufvc_ctx* c, int H, int W);
// Shared-arena mode: allocates the whole capped arena now, so it never grows
// (or drops plans) on a request path.
// Reserves the arena (capped by batch_set_arena_cap), a slab of blob_bytes
// for plans' descriptor blobs with pinned staging of that size, and host
// result arrays for max_batch chunks, so that the batch object's calls
// allocate nothing for compositions whose descriptors fit the slab.
int batch_reserve_arena(ufvc_batch* b, int max_batch, size_t blob_bytes);
// Plans built so far by a batch object.
uint64_t batch_plans_built(const ufvc_batch* b);
