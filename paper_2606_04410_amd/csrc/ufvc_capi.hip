// C ABI of libufvc: context, weight repacking, workspaces, and the encode /
// decode pipelines of one chunk (see include/ufvc.h for the contract).
#include "../../include/ufvc.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "ufvc_common.h"
#include "ufvc_ctx.h"
#include "ufvc_means.h"

using namespace ufvc;

// Fixed device scratch of ufvc_rans_encode_noalloc: one copy per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel or a copy (in host code the name is only a stand-in, not a device
// address); it uses the address hipGetSymbolAddress returned for the device,
// looked up once per device when the first context is created there.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEV = 64;
static void* g_scratch_ptr[NOALLOC_MAX_DEV];
static std::mutex g_scratch_mu;

// Looks up this device's scratch address (the device must be current).
static int noalloc_scratch_init(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return UFVC_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return UFVC_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return UFVC_E_DEVICE;
  g_scratch_ptr[dev] = ptr;
  return UFVC_OK;
}

static void* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

static hipEvent_t prof_event(ufvc_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// Runs one kernel launch; with profiling on, brackets it with events.
template <class F>
static hipError_t stage(ufvc_ctx* c, int id, hipStream_t s, F&& launch) {
  hipEvent_t e0 = nullptr;
  if (c->prof_on && (e0 = prof_event(c)) != nullptr) (void)hipEventRecord(e0, s);
  const hipError_t r = launch();
  if (e0 && r == hipSuccess) {
    hipEvent_t e1 = prof_event(c);
    if (e1) {
      (void)hipEventRecord(e1, s);
      c->prof_rec.push_back({id, e0, e1});
    }
  }
  return r;
}

// Conv tile configurations are chosen per (layer, output size) bucket.  With
// cfg.autotune set, the first call for a bucket times every configuration
// whose channel tile divides the layer's outputs (HIP events: one warm-up
// run, then the fastest of three) and keeps the fastest.  All configurations accumulate
// every output in the same order, so the choice never changes results.
static hipError_t tuned_conv(ufvc_ctx* c, int id, int prec, int ld, int st, const ConvArgs& a,
                             int groups, hipStream_t s, int stride = 1) {
  if (c->force_cfg >= 0 && a.cout % conv_cfg(c->force_cfg).bn == 0 &&
      conv_cfg_supported(prec, ld, stride, a.cin, a.cout, c->force_cfg))
    return launch_conv(prec, ld, st, stride, c->force_cfg, a, groups, s);
  const uint64_t key = tune_key(id, a.Hout, a.Wout);
  auto it = c->tune.find(key);
  if (it != c->tune.end()) return launch_conv(prec, ld, st, stride, it->second, a, groups, s);
  if (!c->cfg.autotune)
    return launch_conv(prec, ld, st, stride, default_cfg(a.cout, (long)a.Hout * a.Wout, stride, ld, prec), a, groups, s);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return hipErrorOutOfMemory;
  int best = -1;
  float best_ms = 1e30f;
  hipError_t err = hipSuccess;
  for (int cfg = 0; cfg < conv_num_cfgs(); ++cfg) {
    const TileCfg t = conv_cfg(cfg);
    if (a.cout % t.bn || !conv_cfg_supported(prec, ld, stride, a.cin, a.cout, cfg)) continue;
    float ms = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      (void)hipEventRecord(e0, s);
      err = launch_conv(prec, ld, st, stride, cfg, a, groups, s);
      if (err != hipSuccess) break;
      (void)hipEventRecord(e1, s);
      if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      if (rep > 0) ms = std::min(ms, t);
    }
    if (err != hipSuccess) break;
    if (ms < best_ms) { best_ms = ms; best = cfg; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess || best < 0) return err != hipSuccess ? err : hipErrorInvalidValue;
  c->tune[key] = best;
  return launch_conv(prec, ld, st, stride, best, a, groups, s);
}

static size_t weight_count_tc(int T, int C) {
  const size_t k9 = 9;
  size_t n = (size_t)C * 192 * T * k9 + 2 * (size_t)C * C * k9 + (size_t)ZC * C * k9 +
             (size_t)2 * C * ZC * k9 + 3 * (size_t)C * C * k9;
  n += (size_t)T * ((size_t)C * C * k9 * 2 + (size_t)192 * C * k9);
  return n;
}

// OCP FP8 E4M3 (bias 7, no infinities, largest finite 448) of x, rounded to
// nearest even and saturated at +-448.
static uint8_t e4m3_rne_sat(double x) {
  const uint8_t sign = std::signbit(x) ? 0x80 : 0;
  double m = std::fabs(x);
  if (!(m < 448.0)) return sign | 0x7E;  // saturate (NaN cannot occur for finite weights)
  if (m < std::ldexp(1.0, -6)) {
    // subnormals: steps of 2^-9; a result of 8 steps is the smallest normal
    return sign | (uint8_t)std::nearbyint(m * 512.0);
  }
  int e = std::ilogb(m);
  long q = std::lrint((m / std::ldexp(1.0, e) - 1.0) * 8.0);  // ties to even
  if (q == 8) { q = 0; ++e; }
  if (e > 8 || (e == 8 && q > 6)) return sign | 0x7E;
  return sign | (uint8_t)(((e + 7) << 3) | q);
}

// Repacks OIHW float32 weights of `groups` groups into the conv kernels'
// layout: [g][slice][tap][cout][row], a slice holding 16 bf16, 8 f32 or 32
// fp8 consecutive input channels (a row of 32 bytes).  FP8 weights carry a
// per-output-channel scale amax / 448 over that channel's taps.
static int upload_layer(Layer& L, const std::vector<const float*>& src, int cout, int cin,
                        int prec_conv) {
  const int E = prec_conv == P_FP8 ? 32 : prec_conv == P_BF16 ? 16 : 8;
  const int esz = prec_conv == P_FP8 ? 1 : prec_conv == P_BF16 ? 2 : 4;
  const int rowb = E * esz;
  if (cin % E) return UFVC_E_UNSUPPORTED;
  const int groups = (int)src.size();
  const int nsl = cin / E;
  const size_t gbytes = (size_t)nsl * 9 * cout * rowb;
  std::vector<uint8_t> buf(gbytes * groups);
  std::vector<float> scales;
  for (int g = 0; g < groups; ++g) {
    const float* W = src[g];
    if (prec_conv == P_FP8) {
      for (int n = 0; n < cout; ++n) {
        float amax = 0.f;
        for (size_t k = 0; k < (size_t)cin * 9; ++k) amax = std::max(amax, std::fabs(W[(size_t)n * cin * 9 + k]));
        scales.push_back(amax > 0.f ? amax / 448.f : 1.f);
      }
    }
    for (int s = 0; s < nsl; ++s)
      for (int tap = 0; tap < 9; ++tap)
        for (int n = 0; n < cout; ++n)
          for (int e = 0; e < E; ++e) {
            const int ci = s * E + e;
            const float v = W[((size_t)n * cin + ci) * 9 + tap];
            uint8_t* d = buf.data() + g * gbytes + ((((size_t)s * 9 + tap) * cout + n) * rowb + e * esz);
            if (esz == 4) {
              std::memcpy(d, &v, 4);
            } else if (esz == 2) {
              const __bf16 b = (__bf16)v;
              std::memcpy(d, &b, 2);
            } else {
              *d = e4m3_rne_sat((double)v / (double)scales[(size_t)g * cout + n]);
            }
          }
  }
  if (hipMalloc(&L.w, buf.size()) != hipSuccess) return UFVC_E_NOMEM;
  CK(hipMemcpy(L.w, buf.data(), buf.size(), hipMemcpyHostToDevice));
  if (!scales.empty()) {
    if (hipMalloc(&L.wscale, 4 * scales.size()) != hipSuccess) return UFVC_E_NOMEM;
    CK(hipMemcpy(L.wscale, scales.data(), 4 * scales.size(), hipMemcpyHostToDevice));
  }
  L.gstride = (long)gbytes;
  L.cin = cin;
  L.cout = cout;
  L.groups = groups;
  L.prec = prec_conv;
  return UFVC_OK;
}

// Entropy-parameter conv weights for the bf16 matrix cores: every float32
// weight w is the exact sum of three bf16 values h + m + l (8 significant
// bits each cover w's 24), stored as three input-channel blocks [h | m | l]
// of the [cout][3 cin][3][3] layer whose loader repeats the cin symbol
// channels three times.  The symbols (-32..32) are exact in bf16 as well, so
// every product is exact and the sums run in float32 as in a float32 conv.
static int upload_split_layer(Layer& L, const float* W, int cout, int cin) {
  std::vector<float> parts((size_t)cout * 3 * cin * 9);
  for (int n = 0; n < cout; ++n)
    for (int ci = 0; ci < cin; ++ci)
      for (int tap = 0; tap < 9; ++tap) {
        const float w = W[((size_t)n * cin + ci) * 9 + tap];
        const float h = (float)(__bf16)w;
        const float r1 = w - h;
        const float m = (float)(__bf16)r1;
        const float r2 = r1 - m;
        const float l = (float)(__bf16)r2;
        if (l != r2 || (double)h + (double)m + (double)l != (double)w) return UFVC_E_UNSUPPORTED;
        const float v[3] = {h, m, l};
        for (int j = 0; j < 3; ++j) parts[((size_t)n * 3 * cin + j * cin + ci) * 9 + tap] = v[j];
      }
  return upload_layer(L, {parts.data()}, cout, 3 * cin, P_BF16);
}

// Entropy-parameter conv weights for params_up2_kernel.  Over up2(z_hat),
// output (2qy + py, 2qx + px) reads z_hat rows qy - 1 + py + r (r = 0, 1),
// row r collecting kernel rows first[py][r] .. last[py][r] (py = 0: r = 0 <-
// dy 0, r = 1 <- dy 1, 2; py = 1: r = 0 <- dy 0, 1, r = 1 <- dy 2), columns
// likewise.  Per class (py, px) and 2x2 tap (r, q) the summed weight (in
// double) is split into three bf16 parts; layout [class][tap][part][cout][cin]
// with cin = 32.
static int upload_params_layer(Layer& L, const float* W, int cout, int cin) {
  if (cin != 32 || cout % 64) return UFVC_E_UNSUPPORTED;
  static const int first[2][2] = {{0, 1}, {0, 2}}, last[2][2] = {{0, 2}, {1, 2}};   // [parity][r]
  std::vector<__bf16> pk((size_t)4 * 4 * 3 * cout * cin);
  for (int cls = 0; cls < 4; ++cls) {
    const int py = cls >> 1, px = cls & 1;
    for (int t = 0; t < 4; ++t) {
      const int r = t >> 1, q = t & 1;
      for (int n = 0; n < cout; ++n)
        for (int ci = 0; ci < cin; ++ci) {
          double w = 0.0;
          for (int dy = first[py][r]; dy <= last[py][r]; ++dy)
            for (int dx = first[px][q]; dx <= last[px][q]; ++dx) w += (double)W[((size_t)n * cin + ci) * 9 + dy * 3 + dx];
          const double h = (double)(float)(__bf16)(float)w;
          const double m = (double)(float)(__bf16)(float)(w - h);
          const double l = (double)(float)(__bf16)(float)(w - h - m);
          const double part[3] = {h, m, l};
          for (int p = 0; p < 3; ++p)
            pk[((((size_t)cls * 4 + t) * 3 + p) * cout + n) * cin + ci] = (__bf16)(float)part[p];
        }
    }
  }
  if (hipMalloc(&L.w, pk.size() * 2) != hipSuccess) return UFVC_E_NOMEM;
  CK(hipMemcpy(L.w, pk.data(), pk.size() * 2, hipMemcpyHostToDevice));
  L.gstride = (long)pk.size() * 2;
  L.cin = cin;
  L.cout = cout;
  L.groups = 1;
  L.prec = P_BF16;
  return UFVC_OK;
}

// Hyper conv weights for hyper_conv_kernel: OIHW float32 [cout][cin][3][3]
// to [tap][cin / 4][cout][4] (four consecutive input channels per 16 bytes).
static int upload_hyper_layer(Layer& L, const float* W, int cout, int cin) {
  if (cin % 16 || cout % 16) return UFVC_E_UNSUPPORTED;
  std::vector<float> pk((size_t)9 * cin * cout);
  for (int tap = 0; tap < 9; ++tap)
    for (int ci = 0; ci < cin; ++ci)
      for (int n = 0; n < cout; ++n)
        pk[(((size_t)tap * (cin / 4) + ci / 4) * cout + n) * 4 + ci % 4] = W[((size_t)n * cin + ci) * 9 + tap];
  if (hipMalloc(&L.w, pk.size() * 4) != hipSuccess) return UFVC_E_NOMEM;
  CK(hipMemcpy(L.w, pk.data(), pk.size() * 4, hipMemcpyHostToDevice));
  L.gstride = (long)pk.size() * 4;
  L.cin = cin;
  L.cout = cout;
  L.groups = 1;
  L.prec = P_F32;
  return UFVC_OK;
}

// Mean-step weights for mean_step_kernel: three OIHW float32 C x C layers,
// each weight split exactly into three bf16 parts h + m + l (as for the
// entropy-parameter conv), to [step][tap][part][C / 8][C][8] bf16 (eight
// consecutive input channels of one output channel per 16 bytes).
static int upload_mean_layers(ufvc_ctx* c, const float* W, int C) {
  const size_t per_in = (size_t)9 * C * C;           // float32 weights per step
  const size_t per = 3 * per_in;                     // bf16 values per step (3 parts)
  std::vector<__bf16> pk(3 * per);
  for (int k = 0; k < 3; ++k)
    for (int n = 0; n < C; ++n)
      for (int ci = 0; ci < C; ++ci)
        for (int tap = 0; tap < 9; ++tap) {
          const float w = W[k * per_in + ((size_t)n * C + ci) * 9 + tap];
          const float h = (float)(__bf16)w;
          const float r1 = w - h;
          const float m = (float)(__bf16)r1;
          const float r2 = r1 - m;
          const float l = (float)(__bf16)r2;
          if (l != r2 || (double)h + (double)m + (double)l != (double)w) return UFVC_E_UNSUPPORTED;
          const float v[3] = {h, m, l};
          for (int p = 0; p < 3; ++p)
            pk[k * per + ((((size_t)tap * 3 + p) * (C / 8) + ci / 8) * C + n) * 8 + ci % 8] = (__bf16)v[p];
        }
  if (hipMalloc(&c->mw, pk.size() * sizeof(__bf16)) != hipSuccess) return UFVC_E_NOMEM;
  CK(hipMemcpy(c->mw, pk.data(), pk.size() * sizeof(__bf16), hipMemcpyHostToDevice));
  c->mw_kstride = per * sizeof(__bf16);
  return UFVC_OK;
}

// Steps 1..3 of the quadtree means on the workspace (encoder: y != null).
static hipError_t run_mean_steps(ufvc_ctx* c, const Geom& g, const float* y, int stage_id,
                                 hipStream_t s) {
  MeanArgs m{};
  m.C = c->cfg.C;
  m.h = g.h;
  m.w = g.w;
  m.sym = c->ws.sym;
  m.P = c->ws.P;
  m.y = y;
  m.sym_out = c->ws.sym;
  m.wpk = c->mw;
  m.w_kstride = c->mw_kstride;
  for (int k = 1; k <= 3; ++k) {
    const hipError_t e = stage(c, stage_id, s, [&] { return launch_mean_step(k, m, s); });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static void free_ws(ufvc_ctx* c) {
  Workspace& w = c->ws;
  void* ptrs[] = {w.act0, w.act1, w.y, w.zsym, w.P, w.idx, w.sym, w.big0, w.big1, w.side, w.q8};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  c->ws = Workspace{};
}

static int ensure_ws(ufvc_ctx* c, int h, int w) {
  if (c->ws.act0 && c->ws.h >= h && c->ws.w >= w) return UFVC_OK;
  (void)hipDeviceSynchronize();
  free_ws(c);
  const int C = c->cfg.C, T = c->cfg.T;
  const size_t npos = (size_t)h * w;
  const size_t hz = (h + 1) / 2, wz = (w + 1) / 2;
  const int es = act_elem_size(c->cfg.precision);
  Workspace& W = c->ws;
  if (hipMalloc(&W.act0, npos * C * es) != hipSuccess) return UFVC_E_NOMEM;
  if (hipMalloc(&W.act1, npos * C * es) != hipSuccess) return UFVC_E_NOMEM;
  if (hipMalloc(&W.y, npos * C * 4) != hipSuccess) return UFVC_E_NOMEM;
  if (hipMalloc(&W.zsym, hz * wz * ZC + CODER_PAD) != hipSuccess) return UFVC_E_NOMEM;
  if (hipMalloc(&W.P, npos * 2 * C * 4) != hipSuccess) return UFVC_E_NOMEM;
  if (hipMalloc(&W.idx, npos * C + CODER_PAD) != hipSuccess) return UFVC_E_NOMEM;
  if (hipMalloc(&W.sym, npos * C + CODER_PAD) != hipSuccess) return UFVC_E_NOMEM;
  if (hipMalloc(&W.big0, npos * C * T * es) != hipSuccess) return UFVC_E_NOMEM;
  if (hipMalloc(&W.big1, npos * C * T * es) != hipSuccess) return UFVC_E_NOMEM;
  if (c->cfg.temporal && hipMalloc(&W.side, npos * 2 * C * 4) != hipSuccess) return UFVC_E_NOMEM;
  if (synth_prec(c->cfg.precision) == P_FP8 && hipMalloc(&W.q8, npos * C * T) != hipSuccess)
    return UFVC_E_NOMEM;
  W.h = h;
  W.w = w;
  return UFVC_OK;
}

static int ensure_rans(ufvc_ctx* c, size_t scratch_bytes, int nseg) {
  RansWs& r = c->rw;
  if (r.scratch_bytes < scratch_bytes) {
    (void)hipDeviceSynchronize();
    if (r.scratch) (void)hipFree(r.scratch);
    r.scratch = nullptr;
    r.scratch_bytes = 0;
    if (hipMalloc(&r.scratch, scratch_bytes) != hipSuccess) return UFVC_E_NOMEM;
    r.scratch_bytes = scratch_bytes;
  }
  if (r.nseg_cap < nseg) {
    (void)hipDeviceSynchronize();
    if (r.info) (void)hipFree(r.info);
    if (r.seg_off) (void)hipFree(r.seg_off);
    if (r.seg_len) (void)hipFree(r.seg_len);
    r.info = nullptr;
    r.seg_off = r.seg_len = nullptr;
    r.nseg_cap = 0;
    if (hipMalloc(&r.info, sizeof(SegInfo) * nseg) != hipSuccess) return UFVC_E_NOMEM;
    if (hipMalloc(&r.seg_off, 4 * (size_t)nseg) != hipSuccess) return UFVC_E_NOMEM;
    if (hipMalloc(&r.seg_len, 4 * (size_t)nseg) != hipSuccess) return UFVC_E_NOMEM;
    r.nseg_cap = nseg;
  }
  return UFVC_OK;
}

static int ensure_pad(ufvc_ctx* c, size_t n) {
  RansWs& r = c->rw;
  if (r.pad_cap >= n + CODER_PAD) return UFVC_OK;
  (void)hipDeviceSynchronize();
  if (r.pad_a) (void)hipFree(r.pad_a);
  if (r.pad_b) (void)hipFree(r.pad_b);
  r.pad_a = r.pad_b = nullptr;
  r.pad_cap = 0;
  if (hipMalloc(&r.pad_a, n + CODER_PAD) != hipSuccess || hipMalloc(&r.pad_b, n + CODER_PAD) != hipSuccess)
    return UFVC_E_NOMEM;
  r.pad_cap = n + CODER_PAD;
  return UFVC_OK;
}


// Options of the synthesis pass for temporal models: d1 adds a conv of the
// context; the context network turns the joint feature F into the next
// context; the encoder runs the chunk decoder only.
struct SynthOpts {
  const float* d1_add = nullptr;   // float32 [pos][C], added to d1 before its ReLU
  void* ctx_out = nullptr;         // next context [pos][C], activation type
  bool heads = true;               // frame-specific decoders (false: F and the context only)
  int prof_stage = -1;             // record the chunk decoder's convs under this stage
  int ctxnet_stage = S_CTXNET_DEC; // ... and the context network's under this one
};

static hipError_t run_synthesis(ufvc_ctx* c, const Geom& g, const uint8_t* sym, const float* mu,
                                long mu_pitch, const float* yhat, int H, int W, float* frames,
                                hipStream_t s, const SynthOpts& o = SynthOpts()) {
  const int C = c->cfg.C, T = c->cfg.T;
  auto sid = [&](int id) { return o.prof_stage >= 0 ? o.prof_stage : id; };
  const int cp = conv_prec(c->cfg.precision);
  const int sp = synth_prec(c->cfg.precision);
  const int act_st = cp == P_BF16 ? ST_BF16 : ST_F32;
  // fp8 layers read a copy of their bf16 input quantised with the amax its
  // producer recorded (one quantise pass per layer, into ws.q8)
  const bool q8 = sp == P_FP8;
  const long npos = (long)g.h * g.w;
  hipError_t e;
  if (q8 && (e = launch_zero_u32(c->amax, AMAX_WORDS, s)) != hipSuccess) return e;
  auto chain = [&](ConvArgs& a, int k) {  // input slot k - 1, output slot k
    if (!q8) return;
    if (k > 0) a.amax_in = c->amax + k - 1;
    if (k < 5) a.amax_out = amax_spread(c->amax, k);
  };
  // FP8 layer k (1..5): its input (channels per position `cpp`) quantised
  // into ws.q8, which the conv then reads; the two launches form one stage
  Q8Job qj{};
  auto quantise = [&](ConvArgs& a, int k, long cpp) {
    if (!q8) return;
    qj = Q8Job{a.in, a.in_pitch, c->ws.q8, npos, (int)cpp, amax_spread(c->amax, k - 1), c->amax + k - 1};
    a.in = c->ws.q8;
    a.in_pitch = cpp;
  };
  auto fp8_first = [&](auto&& conv) -> hipError_t {
    if (q8) {
      const hipError_t r = launch_q8(qj, s);
      if (r != hipSuccess) return r;
    }
    return conv();
  };
  const int sld = LD_NHWC;
  // d1: loads y_hat = r_hat + mu (or a caller-provided float32 y_hat)
  ConvArgs a = conv_args(g.h, g.w, g.h, g.w, c->d1);
  int ld = LD_DEQUANT;
  if (yhat) {
    a.in = yhat;
    a.in_pitch = C;
    ld = cp == P_BF16 ? LD_F32 : LD_NHWC;
  } else {
    a.in = sym;
    a.mu = mu;
    a.mu_pitch = mu_pitch;
  }
  a.out = c->ws.act0;
  a.out_pitch = C;
  a.relu = 1;
  a.add = o.d1_add;
  a.add_pitch = C;
  chain(a, 0);
  e = stage(c, sid(S_D1), s, [&] { return tuned_conv(c, S_D1, cp, ld, act_st, a, 1, s); });
  if (e != hipSuccess) return e;
  a = conv_args(g.h, g.w, g.h, g.w, c->d2);
  a.in = c->ws.act0; a.in_pitch = C; a.out = c->ws.act1; a.out_pitch = C; a.relu = 1;
  chain(a, 1);
  quantise(a, 1, C);
  if ((e = stage(c, sid(S_D2), s, [&] { return fp8_first([&] { return tuned_conv(c, S_D2, sp, sld, act_st, a, 1, s); }); })) != hipSuccess) return e;
  a = conv_args(g.h, g.w, g.h, g.w, c->d3);
  a.in = c->ws.act1; a.in_pitch = C; a.out = c->ws.act0; a.out_pitch = C; a.relu = 1;
  chain(a, 2);
  quantise(a, 2, C);
  if ((e = stage(c, sid(S_D3), s, [&] { return fp8_first([&] { return tuned_conv(c, S_D3, sp, sld, act_st, a, 1, s); }); })) != hipSuccess) return e;
  // temporal models: the next context from F (act0), through act1
  if (o.ctx_out) {
    a = conv_args(g.h, g.w, g.h, g.w, c->c1);
    a.in = c->ws.act0; a.in_pitch = C; a.out = c->ws.act1; a.out_pitch = C; a.relu = 1;
    if ((e = stage(c, o.ctxnet_stage, s, [&] { return tuned_conv(c, T_C1, cp, LD_NHWC, act_st, a, 1, s); })) != hipSuccess)
      return e;
    a = conv_args(g.h, g.w, g.h, g.w, c->c2);
    a.in = c->ws.act1; a.in_pitch = C; a.out = o.ctx_out; a.out_pitch = C; a.relu = 1;
    if ((e = stage(c, o.ctxnet_stage, s, [&] { return tuned_conv(c, T_C2, cp, LD_NHWC, act_st, a, 1, s); })) != hipSuccess)
      return e;
  }
  if (!o.heads) return hipSuccess;
  // k1 of all heads as one GEMM with T*C outputs
  a = conv_args(g.h, g.w, g.h, g.w, c->k1);
  a.in = c->ws.act0; a.in_pitch = C; a.out = c->ws.big0; a.out_pitch = (long)T * C; a.relu = 1;
  chain(a, 3);
  quantise(a, 3, C);
  if ((e = stage(c, S_K1, s, [&] { return fp8_first([&] { return tuned_conv(c, S_K1, sp, sld, act_st, a, 1, s); }); })) != hipSuccess) return e;
  // k2 per head: group t reads channels [tC, tC + C) and writes the same range
  a = conv_args(g.h, g.w, g.h, g.w, c->k2);
  a.in = c->ws.big0; a.in_pitch = (long)T * C; a.in_goff = C;
  a.out = c->ws.big1; a.out_pitch = (long)T * C; a.out_goff = C; a.relu = 1;
  chain(a, 4);
  quantise(a, 4, (long)T * C);
  if ((e = stage(c, S_K2, s, [&] { return fp8_first([&] { return tuned_conv(c, S_K2, sp, sld, act_st, a, T, s); }); })) != hipSuccess) return e;
  // k3 per head with the pixel-shuffle store into frame t
  a = conv_args(g.h, g.w, g.h, g.w, c->k3);
  a.in = c->ws.big1; a.in_pitch = (long)T * C; a.in_goff = C;
  a.out = frames; a.T = T; a.H = H; a.W = W;
  chain(a, 5);
  quantise(a, 5, (long)T * C);
  return stage(c, S_K3, s, [&] { return fp8_first([&] { return tuned_conv(c, S_K3, sp, sld, ST_SHUFFLE, a, T, s); }); });
}

// Temporal models: out (float32 [pos][pitch]) = conv(context, L), the
// context's part of a concatenated input.  The entropy-parameter part keeps
// that conv's float32 arithmetic: in the bf16 modes the context is bf16
// (exact) and the weights are three bf16 parts, so the repeating loader
// feeds each context channel to its three weight blocks.
static hipError_t context_conv(ufvc_ctx* c, const Geom& g, const Layer& L, int tune_id,
                               const void* ctx, float* out, long out_pitch, hipStream_t s) {
  ConvArgs a = conv_args(g.h, g.w, g.h, g.w, L);
  a.in = ctx;
  a.in_pitch = c->cfg.C;
  a.out = out;
  a.out_pitch = out_pitch;
  a.relu = 0;
  const int cp = conv_prec(c->cfg.precision);
  const int ld = (tune_id == T_PC && cp == P_BF16) ? LD_REP : LD_NHWC;
  return tuned_conv(c, tune_id, cp, ld, ST_F32, a, 1, s);
}

extern "C" {

size_t ufvc_weight_count(int T, int C) {
  if (T < 1 || T > 8 || (C != 64 && C != 128)) return 0;
  return weight_count_tc(T, C);
}

int ufvc_create(const ufvc_config* cfg, const float* weights, size_t n_weights, ufvc_ctx** out) {
  if (!cfg || !weights || !out) return UFVC_E_INVAL;
  *out = nullptr;
  if (cfg->T < 1 || cfg->T > 8 || (cfg->C != 64 && cfg->C != 128)) return UFVC_E_INVAL;
  if (cfg->seg_log2 < 5 || cfg->seg_log2 > 24 || cfg->seg_log2_z < 5 || cfg->seg_log2_z > 24)
    return UFVC_E_INVAL;
  if (cfg->precision != UFVC_FP32 && cfg->precision != UFVC_BF16 && cfg->precision != UFVC_BF16_FP8)
    return UFVC_E_UNSUPPORTED;
  if (cfg->quadtree != 0 && cfg->quadtree != 1) return UFVC_E_INVAL;
  if (cfg->temporal != 0 && cfg->temporal != 1) return UFVC_E_INVAL;
  const size_t n_mean = cfg->quadtree ? (size_t)27 * cfg->C * cfg->C : 0;
  const size_t n_temporal = cfg->temporal ? (size_t)54 * cfg->C * cfg->C : 0;
  if (n_weights != weight_count_tc(cfg->T, cfg->C) + n_mean + n_temporal) return UFVC_E_INVAL;
  ufvc_ctx* c = new (std::nothrow) ufvc_ctx();
  if (!c) return UFVC_E_NOMEM;
  c->cfg = *cfg;
  (void)hipGetDevice(&c->device);
  if (const int rc0 = noalloc_scratch_init(c->device)) {
    delete c;
    return rc0;
  }
  const int T = cfg->T, C = cfg->C;
  const int cp = conv_prec(cfg->precision);
  const int sp = synth_prec(cfg->precision);
  // blob offsets in the documented order
  const float* p = weights;
  const float* wa1 = p; p += (size_t)C * 192 * T * 9;
  const float* wa2 = p; p += (size_t)C * C * 9;
  const float* wa3 = p; p += (size_t)C * C * 9;
  const float* wh = p; p += (size_t)ZC * C * 9;
  const float* wp = p; p += (size_t)2 * C * ZC * 9;
  const float* wd1 = p; p += (size_t)C * C * 9;
  const float* wd2 = p; p += (size_t)C * C * 9;
  const float* wd3 = p; p += (size_t)C * C * 9;
  std::vector<const float*> k1s, k2s, k3s;
  for (int t = 0; t < T; ++t) {
    k1s.push_back(p); p += (size_t)C * C * 9;
    k2s.push_back(p); p += (size_t)C * C * 9;
    k3s.push_back(p); p += (size_t)192 * C * 9;
  }
  // k1 of all heads stacked along output channels
  std::vector<float> k1cat((size_t)T * C * C * 9);
  for (int t = 0; t < T; ++t)
    std::memcpy(k1cat.data() + (size_t)t * C * C * 9, k1s[t], sizeof(float) * C * C * 9);
  int rc = UFVC_OK;
  if (!rc) rc = upload_layer(c->a1, {wa1}, C, 192 * T, cp);
  if (!rc) rc = upload_layer(c->a2, {wa2}, C, C, cp);
  if (!rc) rc = upload_layer(c->a3, {wa3}, C, C, cp);
  if (!rc) rc = upload_hyper_layer(c->h, wh, ZC, C);
  if (!rc) rc = upload_params_layer(c->p, wp, 2 * C, ZC);
  if (!rc) rc = upload_layer(c->d1, {wd1}, C, C, cp);
  if (!rc) rc = upload_layer(c->d2, {wd2}, C, C, sp);
  if (!rc) rc = upload_layer(c->d3, {wd3}, C, C, sp);
  if (!rc) rc = upload_layer(c->k1, {k1cat.data()}, T * C, C, sp);
  if (!rc) rc = upload_layer(c->k2, k2s, C, C, sp);
  if (!rc) rc = upload_layer(c->k3, k3s, 192, C, sp);
  if (!rc && cfg->quadtree) rc = upload_mean_layers(c, p, C);
  if (cfg->quadtree) p += (size_t)27 * C * C;
  if (!rc && cfg->temporal) {
    const size_t cc9 = (size_t)C * C * 9;
    const float* wc1 = p;
    const float* wc2 = wc1 + cc9;
    const float* wa1c = wc2 + cc9;
    const float* wpc = wa1c + cc9;
    const float* wd1c = wpc + 2 * cc9;
    if (!rc) rc = upload_layer(c->c1, {wc1}, C, C, cp);
    if (!rc) rc = upload_layer(c->c2, {wc2}, C, C, cp);
    if (!rc) rc = upload_layer(c->a1c, {wa1c}, C, C, cp);
    if (!rc) rc = cp == P_BF16 ? upload_split_layer(c->pc, wpc, 2 * C, C)
                               : upload_layer(c->pc, {wpc}, 2 * C, C, P_F32);
    if (!rc) rc = upload_layer(c->d1c, {wd1c}, C, C, cp);
  }
  if (!rc) {
    Tables& t = c->tab;
    if (hipMalloc(&t.fc, 4 * NSCALES * NSYM) || hipMalloc(&t.magic, 4 * NSCALES * NSYM) ||
        hipMalloc(&t.shift, NSCALES * NSYM) || hipMalloc(&t.lut, NSCALES * LUT_BUCKETS * 2) ||
        hipMalloc(&t.thresholds, 4 * 64) || hipMalloc(&t.tail, 64) || hipMalloc(&c->result, 16) ||
        hipMalloc(&c->status, 16) || hipMalloc(&c->amax, 4 * AMAX_WORDS) || hipHostMalloc(&c->result_host, 16) ||
        hipHostMalloc(&c->status_host, 16))
      rc = UFVC_E_NOMEM;
  }
  if (!rc && (hipMemset(c->status, 0, 16) != hipSuccess || hipMemset(c->amax, 0, 4 * AMAX_WORDS) != hipSuccess))
    rc = UFVC_E_DEVICE;
  if (!rc && launch_build_tables(c->tab, nullptr) != hipSuccess) rc = UFVC_E_DEVICE;
  if (!rc && hipDeviceSynchronize() != hipSuccess) rc = UFVC_E_DEVICE;
  if (rc) {
    ufvc_destroy(c);
    return rc;
  }
  *out = c;
  return UFVC_OK;
}

void ufvc_destroy(ufvc_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  Layer* ls[] = {&c->a1, &c->a2, &c->a3, &c->h,  &c->p,   &c->d1, &c->d2, &c->d3, &c->k1,
                 &c->k2, &c->k3, &c->c1, &c->c2, &c->a1c, &c->pc, &c->d1c};
  for (Layer* l : ls) {
    if (l->w) (void)hipFree(l->w);
    if (l->wscale) (void)hipFree(l->wscale);
  }
  free_ws(c);
  if (c->mw) (void)hipFree(c->mw);
  void* dp[] = {c->tab.fc, c->tab.magic, c->tab.shift, c->tab.lut, c->tab.thresholds, c->tab.tail,
                c->rw.pad_a, c->rw.pad_b, c->result, c->amax,
                c->status, c->rw.scratch, c->rw.info, c->rw.seg_off, c->rw.seg_len};
  for (void* q : dp)
    if (q) (void)hipFree(q);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->result_host) (void)hipHostFree(c->result_host);
  if (c->status_host) (void)hipHostFree(c->status_host);
  delete c;
}

size_t ufvc_max_bitstream_bytes(const ufvc_ctx* c, int H, int W) {
  Geom g;
  if (!c || !geom(c, H, W, g)) return 0;
  return 28 + 4 * (size_t)(g.nseg_y + g.nseg_z) + (size_t)(g.nseg_y + g.nseg_z) * (SEG_STATE_BYTES + 4) +
         2 * (size_t)(g.ny + g.nz);
}

}  // extern "C"

// Encodes one chunk; for a temporal model ctx_in is the stream's context and
// ctx_out receives the next one (formed from the chunk decoder run on this
// chunk's y_hat, as the decoder will).
static int encode_impl(ufvc_ctx* c, const float* frames, int T, int H, int W, uint8_t* bs,
                       size_t capacity, size_t* out_len, hipStream_t s, const void* ctx_in,
                       void* ctx_out) {
  Geom g;
  if (T != c->cfg.T || !geom(c, H, W, g)) return UFVC_E_INVAL;
  int rc = ensure_ws(c, g.h, g.w);
  if (rc) return rc;
  const size_t sbz = slot_bytes(c->cfg.seg_log2_z), sby = slot_bytes(c->cfg.seg_log2);
  rc = ensure_rans(c, sbz * g.nseg_z + sby * g.nseg_y, g.nseg_z + g.nseg_y);
  if (rc) return rc;
  const int C = c->cfg.C;
  const int cp = conv_prec(c->cfg.precision);
  const int act_st = cp == P_BF16 ? ST_BF16 : ST_F32;
  Workspace& ws = c->ws;
  // temporal: a1 sees concat(X, C_i): its context part first
  if (ctx_in)
    CK(stage(c, S_CTXIN_ENC, s, [&] { return context_conv(c, g, c->a1c, T_A1C, ctx_in, ws.side, C, s); }));
  // analysis: patchify fused into a1's loader
  ConvArgs a = conv_args(g.h, g.w, g.h, g.w, c->a1);
  a.in = frames; a.T = T; a.H = H; a.W = W;
  a.out = ws.act0; a.out_pitch = C; a.relu = 1;
  a.add = ctx_in ? ws.side : nullptr; a.add_pitch = C;
  CK(stage(c, S_A1, s, [&] { return tuned_conv(c, S_A1, cp, LD_UNSHUFFLE, act_st, a, 1, s); }));
  a = conv_args(g.h, g.w, g.h, g.w, c->a2);
  a.in = ws.act0; a.in_pitch = C; a.out = ws.act1; a.out_pitch = C; a.relu = 1;
  CK(stage(c, S_A2, s, [&] { return tuned_conv(c, S_A2, cp, LD_NHWC, act_st, a, 1, s); }));
  a = conv_args(g.h, g.w, g.h, g.w, c->a3);
  a.in = ws.act1; a.in_pitch = C; a.out = ws.y; a.out_pitch = C; a.relu = 0;
  CK(stage(c, S_A3, s, [&] { return tuned_conv(c, S_A3, cp, LD_NHWC, ST_F32, a, 1, s); }));
  // hyper prior: stride-2 conv, z_hat = clamp(rint(z)) stored as symbols
  a = conv_args(g.h, g.w, g.hz, g.wz, c->h);
  a.in = ws.y; a.in_pitch = C; a.out = ws.zsym; a.out_pitch = ZC;
  CK(stage(c, S_HYPER, s, [&] { return tuned_conv(c, S_HYPER, P_F32, LD_NHWC, ST_ZSYM, a, 1, s, 2); }));
  // entropy parameters in one pass from up2(z_hat) (temporal: the prior is
  // concat(up2(z_hat), C_i), its context part first)
  if (ctx_in)
    CK(stage(c, S_CTXIN_ENC, s, [&] { return context_conv(c, g, c->pc, T_PC, ctx_in, ws.side, 2 * C, s); }));
  a = conv_args(g.h, g.w, g.h, g.w, c->p);
  a.in = ws.zsym; a.in_pitch = ZC; a.out = ws.P; a.out_pitch = 2 * C;
  a.add = ctx_in ? ws.side : nullptr; a.add_pitch = 2 * C;
  // (tuned under one key for the encoder and the decoder; every configuration
  // gives the same results in any case)
  CK(stage(c, S_PARAMS_ENC, s, [&] { return tuned_conv(c, S_PARAMS_ENC, P_BF16, LD_UP2, ST_F32, a, 1, s); }));
  CK(stage(c, S_EPI_ENC, s, [&] { return launch_params_epilogue(ws.P, ws.y, c->tab.thresholds, ws.idx, ws.sym, (long)g.h * g.w, C, s); }));
  // quadtree: partitions 1..3 re-quantised with their refined means
  if (c->cfg.quadtree) CK(run_mean_steps(c, g, ws.y, S_MEANS_ENC, s));
  // rANS: z with the fixed row, y with per-element rows
  EncStream ez{ws.zsym, nullptr, K_Z, g.nz, c->cfg.seg_log2_z, g.nseg_z};
  EncStream ey{ws.sym, ws.idx, 0, g.ny, c->cfg.seg_log2, g.nseg_y};
  CK(stage(c, S_RANS_ENC, s, [&] { return launch_rans_encode(c->tab, ez, ey, c->rw.scratch, sbz, sby, c->rw.info, s); }));
  HeaderFields hf{(uint16_t)T, (uint16_t)C, (uint16_t)H, (uint16_t)W, (uint8_t)c->cfg.seg_log2,
                  (uint8_t)c->cfg.seg_log2_z, (uint8_t)K_Z, c->cfg.model_tag, header_flags(c)};
  CK(stage(c, S_COMPACT, s, [&] { return launch_compact(c->rw.scratch, sbz, sby, c->rw.info, g.nseg_z, g.nseg_y, 1, hf, bs, capacity,
                    c->result, c->rw.seg_off, s); }));
  CK(hipMemcpyAsync(c->result_host, c->result, 8, hipMemcpyDeviceToHost, s));
  // temporal: the decoder's chunk decoder on this chunk's y_hat, then the
  // context network, so the next context is the decoder's
  if (ctx_in) {
    CK(stage(c, S_CTXIN_ENC, s, [&] { return context_conv(c, g, c->d1c, T_D1C, ctx_in, ws.side, C, s); }));
    SynthOpts o;
    o.d1_add = ws.side;
    o.ctx_out = ctx_out;
    o.heads = false;
    o.prof_stage = S_CHUNKDEC_ENC;
    o.ctxnet_stage = S_CTXNET_ENC;
    CK(run_synthesis(c, g, ws.sym, ws.P, 2 * C, nullptr, H, W, nullptr, s, o));
  }
  CK(hipStreamSynchronize(s));
  c->last_stream = s;
  c->last_h = g.h;
  c->last_w = g.w;
  *out_len = (size_t)c->result_host[0];
  return *out_len > capacity ? UFVC_E_NOSPC : UFVC_OK;
}

// Decodes one chunk; temporal models take the stream's context and write
// the next one.
static int decode_impl(ufvc_ctx* c, const uint8_t* bs, size_t len, int T, int H, int W,
                       float* frames, hipStream_t s, const void* ctx_in, void* ctx_out) {
  Geom g;
  if (T != c->cfg.T || !geom(c, H, W, g)) return UFVC_E_INVAL;
  if (len > 0xFFFFFFF0ull || len < 28) return UFVC_E_INVAL;
  int rc = ensure_ws(c, g.h, g.w);
  if (rc) return rc;
  rc = ensure_rans(c, 0, g.nseg_z + g.nseg_y);
  if (rc) return rc;
  const int C = c->cfg.C;
  Workspace& ws = c->ws;
  HeaderFields ex{(uint16_t)T, (uint16_t)C, (uint16_t)H, (uint16_t)W, (uint8_t)c->cfg.seg_log2,
                  (uint8_t)c->cfg.seg_log2_z, (uint8_t)K_Z, c->cfg.model_tag, header_flags(c)};
  CK(stage(c, S_PARSE, s, [&] { return launch_parse(bs, len, 1, ex, g.nseg_z, g.nseg_y, c->rw.seg_off, c->rw.seg_len, c->status, s); }));
  DecStream dz{nullptr, K_Z, g.nz, c->cfg.seg_log2_z, g.nseg_z, 0, ws.zsym, len};
  CK(stage(c, S_RANS_DEC_Z, s, [&] { return launch_rans_decode(c->tab, bs, c->rw.seg_off, c->rw.seg_len, dz, c->status, s); }));
  if (ctx_in)
    CK(stage(c, S_CTXIN_DEC, s, [&] { return context_conv(c, g, c->pc, T_PC, ctx_in, ws.side, 2 * C, s); }));
  ConvArgs a = conv_args(g.h, g.w, g.h, g.w, c->p);
  a.in = ws.zsym; a.in_pitch = ZC; a.out = ws.P; a.out_pitch = 2 * C;
  a.add = ctx_in ? ws.side : nullptr; a.add_pitch = 2 * C;
  CK(stage(c, S_PARAMS_DEC, s, [&] { return tuned_conv(c, S_PARAMS_ENC, P_BF16, LD_UP2, ST_F32, a, 1, s); }));
  CK(stage(c, S_EPI_DEC, s, [&] { return launch_params_epilogue(ws.P, nullptr, c->tab.thresholds, ws.idx, nullptr, (long)g.h * g.w, C, s); }));
  // all of r_hat in one launch: its tables depend on sigma only
  DecStream dy{ws.idx, 0, g.ny, c->cfg.seg_log2, g.nseg_y, g.nseg_z, ws.sym, len};
  CK(stage(c, S_RANS_DEC_Y, s, [&] { return launch_rans_decode(c->tab, bs, c->rw.seg_off, c->rw.seg_len, dy, c->status, s); }));
  // quadtree: the means of partitions 1..3 from the decoded residuals
  if (c->cfg.quadtree) CK(run_mean_steps(c, g, nullptr, S_MEANS_DEC, s));
  SynthOpts o;
  if (ctx_in) {
    CK(stage(c, S_CTXIN_DEC, s, [&] { return context_conv(c, g, c->d1c, T_D1C, ctx_in, ws.side, C, s); }));
    o.d1_add = ws.side;
    o.ctx_out = ctx_out;
  }
  CK(run_synthesis(c, g, ws.sym, ws.P, 2 * C, nullptr, H, W, frames, s, o));
  c->last_stream = s;
  c->last_h = g.h;
  c->last_w = g.w;
  return UFVC_OK;
}

struct ufvc_stream {
  ufvc_ctx* ctx = nullptr;
  int H = 0, W = 0;
  size_t bytes = 0;          // one context, [h][w][C] activation type
  void* cur = nullptr;       // the next chunk's context
  void* nxt = nullptr;       // written by a call, swapped in on success
  hipStream_t last = nullptr;
};

extern "C" {

int ufvc_encode_chunk(ufvc_ctx* c, const float* frames, int T, int H, int W, uint8_t* bs,
                      size_t capacity, size_t* out_len, void* stream) {
  if (!c || !frames || !bs || !out_len) return UFVC_E_INVAL;
  if (c->cfg.temporal) return UFVC_E_UNSUPPORTED;
  return encode_impl(c, frames, T, H, W, bs, capacity, out_len, (hipStream_t)stream, nullptr, nullptr);
}

int ufvc_decode_chunk(ufvc_ctx* c, const uint8_t* bs, size_t len, int T, int H, int W,
                      float* frames, void* stream) {
  if (!c || !bs || !frames) return UFVC_E_INVAL;
  if (c->cfg.temporal) return UFVC_E_UNSUPPORTED;
  return decode_impl(c, bs, len, T, H, W, frames, (hipStream_t)stream, nullptr, nullptr);
}

int ufvc_stream_create(ufvc_ctx* c, int H, int W, ufvc_stream** out) {
  if (!c || !out) return UFVC_E_INVAL;
  *out = nullptr;
  Geom g;
  if (!c->cfg.temporal || !geom(c, H, W, g)) return UFVC_E_INVAL;
  ufvc_stream* st = new (std::nothrow) ufvc_stream();
  if (!st) return UFVC_E_NOMEM;
  st->ctx = c;
  st->H = H;
  st->W = W;
  st->bytes = (size_t)g.h * g.w * c->cfg.C * act_elem_size(c->cfg.precision);
  if (hipMalloc(&st->cur, st->bytes) != hipSuccess || hipMalloc(&st->nxt, st->bytes) != hipSuccess) {
    ufvc_stream_destroy(st);
    return UFVC_E_NOMEM;
  }
  if (hipMemset(st->cur, 0, st->bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    ufvc_stream_destroy(st);
    return UFVC_E_DEVICE;
  }
  *out = st;
  return UFVC_OK;
}

void ufvc_stream_destroy(ufvc_stream* st) {
  if (!st) return;
  (void)hipDeviceSynchronize();
  if (st->cur) (void)hipFree(st->cur);
  if (st->nxt) (void)hipFree(st->nxt);
  delete st;
}

int ufvc_stream_reset(ufvc_stream* st) {
  if (!st) return UFVC_E_INVAL;
  if (st->last) CK(hipStreamSynchronize(st->last));
  CK(hipMemset(st->cur, 0, st->bytes));
  CK(hipDeviceSynchronize());
  return UFVC_OK;
}

int ufvc_stream_copy_context(ufvc_stream* st, void* dst, size_t bytes) {
  if (!st || !dst || bytes != st->bytes) return UFVC_E_INVAL;
  if (st->last) CK(hipStreamSynchronize(st->last));
  CK(hipMemcpy(dst, st->cur, bytes, hipMemcpyDeviceToHost));
  return UFVC_OK;
}

int ufvc_encode_next(ufvc_stream* st, const float* frames, uint8_t* bs, size_t capacity,
                     size_t* out_len, void* stream) {
  if (!st || !frames || !bs || !out_len) return UFVC_E_INVAL;
  const int rc = encode_impl(st->ctx, frames, st->ctx->cfg.T, st->H, st->W, bs, capacity, out_len,
                             (hipStream_t)stream, st->cur, st->nxt);
  st->last = (hipStream_t)stream;
  if (rc == UFVC_OK) std::swap(st->cur, st->nxt);
  return rc;
}

int ufvc_decode_next(ufvc_stream* st, const uint8_t* bs, size_t len, float* frames, void* stream) {
  if (!st || !bs || !frames) return UFVC_E_INVAL;
  const int rc = decode_impl(st->ctx, bs, len, st->ctx->cfg.T, st->H, st->W, frames,
                             (hipStream_t)stream, st->cur, st->nxt);
  st->last = (hipStream_t)stream;
  if (rc == UFVC_OK) std::swap(st->cur, st->nxt);
  return rc;
}


int ufvc_sync_status(ufvc_ctx* c, void* stream) {
  if (!c) return UFVC_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  CK(hipMemcpyAsync(c->status_host, c->status, 4, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  const uint32_t st = c->status_host[0];
  CK(hipMemsetAsync(c->status, 0, 4, s));
  CK(hipStreamSynchronize(s));
  if (st & ST_BAD_HEADER) return UFVC_E_INVAL;
  if (st & ST_CORRUPT) return UFVC_E_CORRUPT;
  return UFVC_OK;
}

int ufvc_get_tables(ufvc_ctx* c, uint16_t* freq, uint16_t* cum, float* thr) {
  if (!c || !freq || !cum || !thr) return UFVC_E_INVAL;
  std::vector<uint32_t> fc(NSCALES * NSYM);
  CK(hipDeviceSynchronize());
  CK(hipMemcpy(fc.data(), c->tab.fc, 4 * fc.size(), hipMemcpyDeviceToHost));
  CK(hipMemcpy(thr, c->tab.thresholds, 4 * 63, hipMemcpyDeviceToHost));
  for (int i = 0; i < NSCALES * NSYM; ++i) {
    freq[i] = (uint16_t)(fc[i] & 0xFFFF);
    cum[i] = (uint16_t)(fc[i] >> 16);
  }
  return UFVC_OK;
}

int ufvc_rans_encode(ufvc_ctx* c, const uint8_t* sym, const uint8_t* idx, size_t n, int sl,
                     uint8_t* out, size_t capacity, size_t* out_len, void* stream) {
  if (!c || !sym || !idx || !out || !out_len || sl < 5 || sl > 24) return UFVC_E_INVAL;
  if (n > ((size_t)1 << 32)) return UFVC_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const int nseg = nseg_of((long)n, sl);
  int rc = ensure_rans(c, slot_bytes(sl) * (nseg > 0 ? nseg : 1), nseg > 0 ? nseg : 1);
  if (!rc) rc = ensure_pad(c, n);
  if (rc) return rc;
  if (n) {
    CK(hipMemcpyAsync(c->rw.pad_a, sym, n, hipMemcpyDeviceToDevice, s));
    CK(hipMemcpyAsync(c->rw.pad_b, idx, n, hipMemcpyDeviceToDevice, s));
  }
  EncStream ez{nullptr, nullptr, 0, 0, 5, 0};
  EncStream ey{c->rw.pad_a, c->rw.pad_b, 0, (long)n, sl, nseg};
  CK(launch_rans_encode(c->tab, ez, ey, c->rw.scratch, 0, slot_bytes(sl), c->rw.info, s));
  HeaderFields hf{};
  CK(launch_compact(c->rw.scratch, 0, slot_bytes(sl), c->rw.info, 0, nseg, 0, hf, out, capacity,
                    c->result, c->rw.seg_off, s));
  CK(hipMemcpyAsync(c->result_host, c->result, 8, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  *out_len = (size_t)c->result_host[0];
  return *out_len > capacity ? UFVC_E_NOSPC : UFVC_OK;
}

int ufvc_rans_encode_noalloc(ufvc_ctx* c, const uint8_t* sym, const uint8_t* idx, size_t n, int sl,
                             uint8_t* out, size_t capacity, size_t* out_len, void* stream) {
  if (!c || !sym || !idx || !out || !out_len || sl < 5 || sl > 24) return UFVC_E_INVAL;
  if (n > ((size_t)1 << 32)) return UFVC_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const int nseg = nseg_of((long)n, sl);
  // scratch layout: padded symbol copy, padded index copy, segment slots,
  // segment word ranges, segment byte offsets (each part 256-byte aligned)
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t pad_bytes = up(n + CODER_PAD);
  const size_t o_idx = pad_bytes;
  const size_t o_slot = 2 * pad_bytes;
  const size_t o_info = o_slot + up(slot_bytes(sl) * (size_t)nseg);
  const size_t o_off = o_info + up(sizeof(SegInfo) * (size_t)nseg);
  const size_t need = o_off + up(4 * (size_t)nseg);
  if (need > NOALLOC_SCRATCH_BYTES) return UFVC_E_SCRATCH;
  uint8_t* base = static_cast<uint8_t*>(noalloc_scratch(c->device));
  if (!base) return UFVC_E_DEVICE;
  if (n) {
    CK(hipMemcpyAsync(base, sym, n, hipMemcpyDeviceToDevice, s));
    CK(hipMemcpyAsync(base + o_idx, idx, n, hipMemcpyDeviceToDevice, s));
  }
  SegInfo* info = reinterpret_cast<SegInfo*>(base + o_info);
  EncStream ez{nullptr, nullptr, 0, 0, 5, 0};
  EncStream ey{base, base + o_idx, 0, (long)n, sl, nseg};
  CK(launch_rans_encode(c->tab, ez, ey, base + o_slot, 0, slot_bytes(sl), info, s));
  HeaderFields hf{};
  CK(launch_compact(base + o_slot, 0, slot_bytes(sl), info, 0, nseg, 0, hf, out, capacity, c->result,
                    reinterpret_cast<uint32_t*>(base + o_off), s));
  CK(hipMemcpyAsync(c->result_host, c->result, 8, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  *out_len = (size_t)c->result_host[0];
  return *out_len > capacity ? UFVC_E_NOSPC : UFVC_OK;
}

int ufvc_rans_decode(ufvc_ctx* c, const uint8_t* in, size_t len, const uint8_t* idx, size_t n,
                     int sl, uint8_t* sym, void* stream) {
  if (!c || !in || !idx || !sym || sl < 5 || sl > 24 || len > 0xFFFFFFF0ull) return UFVC_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const int nseg = nseg_of((long)n, sl);
  if (len < 4 * (size_t)nseg + 4) return UFVC_E_INVAL;
  int rc = ensure_rans(c, 0, nseg > 0 ? nseg : 1);
  if (!rc) rc = ensure_pad(c, n);
  if (rc) return rc;
  if (n) CK(hipMemcpyAsync(c->rw.pad_b, idx, n, hipMemcpyDeviceToDevice, s));
  HeaderFields ex{};
  CK(launch_parse(in, len, 0, ex, 0, nseg, c->rw.seg_off, c->rw.seg_len, c->status, s));
  DecStream d{c->rw.pad_b, 0, (long)n, sl, nseg, 0, sym, len};
  CK(launch_rans_decode(c->tab, in, c->rw.seg_off, c->rw.seg_len, d, c->status, s));
  c->last_stream = s;
  return UFVC_OK;
}

int ufvc_synthesize(ufvc_ctx* c, const float* y_hat, int T, int H, int W, float* frames, void* stream) {
  if (!c || !y_hat || !frames) return UFVC_E_INVAL;
  Geom g;
  if (T != c->cfg.T || !geom(c, H, W, g)) return UFVC_E_INVAL;
  int rc = ensure_ws(c, g.h, g.w);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  CK(run_synthesis(c, g, nullptr, nullptr, 0, y_hat, H, W, frames, s));
  c->last_stream = s;
  c->last_h = g.h;
  c->last_w = g.w;
  return UFVC_OK;
}

int ufvc_profile_enable(ufvc_ctx* c, int on) {
  if (!c) return UFVC_E_INVAL;
  CK(hipDeviceSynchronize());
  c->prof_rec.clear();
  c->ev_used = 0;
  c->prof_on = on != 0;
  return UFVC_OK;
}

int ufvc_profile_stage_count(void) { return S_COUNT; }

const char* ufvc_profile_stage_name(int i) { return (i >= 0 && i < S_COUNT) ? kStageNames[i] : nullptr; }

int ufvc_profile_read(ufvc_ctx* c, double* total_ms, int* count, int n) {
  if (!c || !total_ms || !count || n < S_COUNT) return UFVC_E_INVAL;
  CK(hipDeviceSynchronize());
  for (int i = 0; i < n; ++i) { total_ms[i] = 0.0; count[i] = 0; }
  for (const auto& r : c->prof_rec) {
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, r.e0, r.e1));
    total_ms[r.stage] += ms;
    count[r.stage] += 1;
  }
  c->prof_rec.clear();
  c->ev_used = 0;
  return UFVC_OK;
}

int ufvc_get_tuning(ufvc_ctx* c, int H, int W, int* cfg, int n) {
  Geom g;
  if (!c || !cfg || n < 9 || !geom(c, H, W, g)) return UFVC_E_INVAL;
  const int ids[9] = {S_A1, S_A2, S_A3, S_D1, S_D2, S_D3, S_K1, S_K2, S_K3};
  for (int i = 0; i < 9; ++i) {
    auto it = c->tune.find(tune_key(ids[i], g.h, g.w));
    cfg[i] = it == c->tune.end() ? -1 : it->second;
  }
  return UFVC_OK;
}

int ufvc_num_tile_configs(void) { return conv_num_cfgs(); }

int ufvc_force_tile_config(ufvc_ctx* c, int cfg) {
  if (!c || cfg < -1 || cfg >= conv_num_cfgs()) return UFVC_E_INVAL;
  c->force_cfg = cfg;
  return UFVC_OK;
}

int ufvc_tile_config(int cfg, int* th, int* tw, int* bn) {
  if (cfg < 0 || cfg >= conv_num_cfgs() || !th || !tw || !bn) return UFVC_E_INVAL;
  const TileCfg t = conv_cfg(cfg);
  *th = t.th;
  *tw = t.tw;
  *bn = t.bn;
  return UFVC_OK;
}

int ufvc_copy_buffer(ufvc_ctx* c, int which, void* dst, size_t bytes) {
  if (!c || !dst || !c->ws.act0) return UFVC_E_INVAL;
  const size_t npos = (size_t)c->last_h * c->last_w;
  const size_t nz = (size_t)((c->last_h + 1) / 2) * ((c->last_w + 1) / 2) * ZC;
  const int C = c->cfg.C;
  const size_t es = act_elem_size(c->cfg.precision);
  const void* src = nullptr;
  size_t need = 0;
  switch (which) {
    case UFVC_BUF_Y: src = c->ws.y; need = npos * C * 4; break;
    case UFVC_BUF_ZSYM: src = c->ws.zsym; need = nz; break;
    case UFVC_BUF_PARAMS: src = c->ws.P; need = npos * 2 * C * 4; break;
    case UFVC_BUF_IDX: src = c->ws.idx; need = npos * C; break;
    case UFVC_BUF_SYM: src = c->ws.sym; need = npos * C; break;
    case UFVC_BUF_D2: src = c->ws.act1; need = npos * C * es; break;
    case UFVC_BUF_F: src = c->ws.act0; need = npos * C * es; break;
    case UFVC_BUF_K1: src = c->ws.big0; need = npos * C * c->cfg.T * es; break;
    case UFVC_BUF_K2: src = c->ws.big1; need = npos * C * c->cfg.T * es; break;
    case UFVC_BUF_AMAX: src = c->amax; need = 4 * N_AMAX; break;
    default: return UFVC_E_INVAL;
  }
  if (bytes != need) return UFVC_E_INVAL;
  CK(hipStreamSynchronize(c->last_stream));
  CK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  return UFVC_OK;
}

}  // extern "C"
