// Batched encode / decode of many chunks of uneven size: every pipeline
// stage is one launch (per tile configuration) over the chunks of the batch.
//
// A plan is built per batch composition (the list of (model, H, W)): a device
// arena with each chunk's activations, latents, symbols, rANS slots and
// parse outputs; the per-stage conv problem descriptors and work lists; the
// rANS segment descriptors; the epilogue, parse and container descriptors.
// All of them live at fixed device addresses for the life of the plan, so a
// decode captured into a hipGraph stays valid: before every call the host
// rewrites only the descriptor entries that depend on the caller's buffers
// (frames, bit-streams, lengths) with one copy, outside the graph.
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "ufvc_ctx.h"

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t kMaxPlans = 32;   // cached batch compositions per batch object
inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

struct ChunkPlan {
  int model, T, H, W;
  Geom g;
  // arena offsets
  size_t act0, act1, y, zsym, P, idx, sym, big0, big1, scratch, info, seg_off, seg_len;
  size_t q8;                      // FP8 synthesis: quantised layer input (0 otherwise)
  size_t slot_z, slot_y;
};

// One launch of a conv stage: problems [desc0, desc0 + ndesc) of the stage's
// descriptor table and work items [work0, work0 + nwork) of its work list.
struct ConvLaunch {
  int cfg;
  int work0, nwork;
};

struct ConvStage {
  int prec, loader, store, stride;
  int desc0;                       // first descriptor of this stage in conv_descs
  std::vector<ConvLaunch> launches;
};

}  // namespace

struct ufvc_batch {
  std::vector<ufvc_ctx*> models;
  struct Plan {
    std::vector<int> key;          // (model, H, W) per chunk
    std::vector<ChunkPlan> chunks;
    uint8_t* arena = nullptr;
    size_t arena_bytes = 0;
    bool owns_arena = true;        // false: the batch object's shared arena
    // descriptor blob (device) and its host mirror
    uint8_t* dblob = nullptr;
    size_t blob_bytes = 0;         // dblob's size
    bool blob_pooled = false;      // dblob lies in the batch object's slab
    std::vector<uint8_t> hblob;
    size_t off_conv = 0, off_work = 0, off_epi_e = 0, off_epi_d = 0, off_epi_work = 0,
           off_encseg = 0, off_comp = 0, off_compmap = 0, off_parse = 0, off_decz = 0, off_decy = 0,
           off_status = 0, off_result = 0, off_amax = 0, off_q8 = 0;
    long q8_units[5] = {0, 0, 0, 0, 0};   // FP8: largest quantise job of d2 d3 k1 k2 k3
    size_t dyn_bytes = 0;          // leading part of the blob rewritten per call
    bool uploaded = false;         // static part already on the device
    int n_conv = 0, n_work = 0, n_epi_work = 0, n_encseg = 0, n_compblk = 0, n_decz = 0, n_decy = 0;
    // conv stages
    ConvStage enc_stage[5];        // a1 a2 a3 hyper params
    ConvStage dec_stage[7];        // params d1 d2 d3 k1 k2 k3
    // call-varying descriptor indices (in units of the descriptor tables)
    std::vector<int> a1_desc, k3_desc;
    // decode graph
    uint64_t decodes = 0;          // decode calls so far (the graph is captured from the second)
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    uint64_t last_use = 0;         // LRU stamp
    int n_launches = 0, n_stages = 0;
  };
  std::map<std::vector<int>, std::unique_ptr<Plan>> plans;
  // launch policy: 0 = one launch per tile configuration in a stage,
  // 1 = one configuration (hence one launch) per stage for the whole batch:
  // the default, measured faster on the 48-chunk mix (12.8 k against
  // 12.4 k frames/s)
  int policy = 1;
  uint64_t use_clock = 0, plans_built = 0, plans_evicted = 0;
  const Plan* last_plan = nullptr;
  uint8_t* staging = nullptr;      // pinned host copy of a descriptor blob
  size_t staging_bytes = 0;
  hipEvent_t staged = nullptr;     // last upload from staging
  hipStream_t capture = nullptr;   // capture stream (the null stream cannot be captured)
  unsigned long long* results_host = nullptr;
  uint32_t* status_host = nullptr;
  int host_cap = 0;
  // shared-arena mode (arena_cap > 0): every plan lays its chunks out from the
  // start of one arena, grown on demand up to arena_cap; calls on a batch
  // object are stream-ordered, so plans never use it at the same time
  size_t arena_cap = 0;
  uint8_t* shared = nullptr;
  size_t shared_bytes = 0;
  // descriptor-blob slab (reserved with the arena): plans' descriptor blobs
  // are carved from it first-fit (offset -> bytes of each free range), so a
  // new batch composition allocates nothing on the request path; a blob
  // that does not fit even after evicting every other plan gets its own
  // allocation
  uint8_t* blob_slab = nullptr;
  size_t blob_cap = 0;
  std::map<size_t, size_t> blob_free;
};

namespace {

template <class T>
T* at(uint8_t* base, size_t off) { return reinterpret_cast<T*>(base + off); }

void free_plan(ufvc_batch* b, ufvc_batch::Plan* p) {
  if (!p) return;
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->arena && p->owns_arena) (void)hipFree(p->arena);
  if (p->dblob && !p->blob_pooled) (void)hipFree(p->dblob);
  if (p->dblob && p->blob_pooled) {
    // back to the slab's free ranges, merged with its neighbours
    size_t off = (size_t)(p->dblob - b->blob_slab), len = p->blob_bytes;
    auto nx = b->blob_free.lower_bound(off);
    if (nx != b->blob_free.end() && off + len == nx->first) {
      len += nx->second;
      nx = b->blob_free.erase(nx);
    }
    if (nx != b->blob_free.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += len;
        return;
      }
    }
    b->blob_free[off] = len;
  }
}

// Drops the least recently used plan, after its last call on stream s has
// finished with its descriptors and graph.
hipError_t evict_lru(ufvc_batch* b, hipStream_t s) {
  auto lru = b->plans.begin();
  for (auto j = b->plans.begin(); j != b->plans.end(); ++j)
    if (j->second->last_use < lru->second->last_use) lru = j;
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (b->last_plan == lru->second.get()) b->last_plan = nullptr;
  free_plan(b, lru->second.get());
  b->plans.erase(lru);
  b->plans_evicted += 1;
  return hipSuccess;
}

// Device memory for a plan's descriptor blob: first fit in the slab,
// evicting least recently used plans while none fits; otherwise (no slab,
// or a blob larger than what the slab can free) an allocation of its own.
int alloc_blob(ufvc_batch* b, ufvc_batch::Plan& P, size_t bytes, hipStream_t s) {
  bytes = align_up(bytes);
  P.blob_bytes = bytes;
  if (b->blob_slab && bytes <= b->blob_cap) {
    for (;;) {
      for (auto it = b->blob_free.begin(); it != b->blob_free.end(); ++it) {
        if (it->second < bytes) continue;
        const size_t off = it->first, rest = it->second - bytes;
        b->blob_free.erase(it);
        if (rest) b->blob_free[off + bytes] = rest;
        P.dblob = b->blob_slab + off;
        P.blob_pooled = true;
        return UFVC_OK;
      }
      if (b->plans.empty()) break;
      CK(evict_lru(b, s));
    }
  }
  if (hipMalloc(&P.dblob, bytes) != hipSuccess) return UFVC_E_NOMEM;
  return UFVC_OK;
}

ConvArgs conv_of(int Hin, int Win, int Hout, int Wout, const Layer& L) {
  return conv_args(Hin, Win, Hout, Wout, L);
}

int pick_cfg(ufvc_ctx* c, int stage_id, int prec, int ld, int stride, const ConvArgs& a, int fixed) {
  if (fixed >= 0) return fixed;
  if (c->force_cfg >= 0 && a.cout % conv_cfg(c->force_cfg).bn == 0 &&
      conv_cfg_supported(prec, ld, stride, a.cin, a.cout, c->force_cfg))
    return c->force_cfg;
  auto it = c->tune.find(tune_key(stage_id, a.Hout, a.Wout));
  if (it != c->tune.end()) return it->second;
  return default_cfg(a.cout, (long)a.Hout * a.Wout, stride, ld, prec);
}

// Builds the work list entries of one conv stage: per chunk one problem
// descriptor, per (group, channel tile, spatial tile) one work item; problems
// with the same tile configuration share a launch.
void add_stage(ufvc_batch::Plan& P, ConvStage& st, std::vector<ConvArgs>& descs,
               std::vector<int4>& work, const std::vector<ConvArgs>& per_chunk,
               const std::vector<int>& groups, const std::vector<int>& cfgs) {
  st.desc0 = (int)descs.size();
  for (const ConvArgs& a : per_chunk) descs.push_back(a);
  std::map<int, std::vector<int>> by_cfg;
  for (size_t i = 0; i < per_chunk.size(); ++i) by_cfg[cfgs[i]].push_back((int)i);
  for (auto& kv : by_cfg) {
    const TileCfg t = conv_cfg(kv.first);
    ConvLaunch L{kv.first, (int)work.size(), 0};
    for (int i : kv.second) {
      const ConvArgs& a = per_chunk[i];
      const int tiles = ((a.Hout + t.th - 1) / t.th) * ((a.Wout + t.tw - 1) / t.tw);
      if (kv.first == kParamsCfg0 || kv.first == kParamsCfg1) {
        // the entropy-parameter kernel: channel blocks of a tile adjacent
        for (int tile = 0; tile < tiles; ++tile)
          for (int n0 = 0; n0 < a.cout; n0 += t.bn) work.push_back(make_int4(st.desc0 + i, tile, n0, 0));
        continue;
      }
      for (int g = 0; g < groups[i]; ++g)
        for (int n0 = 0; n0 < a.cout; n0 += t.bn)
          for (int tile = 0; tile < tiles; ++tile) work.push_back(make_int4(st.desc0 + i, tile, n0, g));
    }
    L.nwork = (int)work.size() - L.work0;
    st.launches.push_back(L);
  }
  (void)P;
}

// Places one chunk's buffers in an arena at `off` (advanced past them).
int layout_chunk(ufvc_ctx* c, int model, int H, int W, ChunkPlan& cp, size_t& off) {
  const int C = c->cfg.C;
  const int es = act_elem_size(c->cfg.precision);
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
  cp = ChunkPlan{};
  cp.model = model;
  cp.T = c->cfg.T;
  cp.H = H;
  cp.W = W;
  if (!geom(c, cp.H, cp.W, cp.g)) return UFVC_E_INVAL;
  const size_t npos = (size_t)cp.g.h * cp.g.w;
  cp.slot_z = slot_bytes(c->cfg.seg_log2_z);
  cp.slot_y = slot_bytes(c->cfg.seg_log2);
  cp.act0 = take(npos * C * es);
  cp.act1 = take(npos * C * es);
  cp.y = take(npos * C * 4);
  cp.zsym = take((size_t)cp.g.nz + CODER_PAD);
  cp.P = take(npos * 2 * C * 4);
  cp.idx = take(npos * C + CODER_PAD);
  cp.sym = take(npos * C + CODER_PAD);
  cp.big0 = take(npos * C * cp.T * es);
  cp.big1 = take(npos * C * cp.T * es);
  cp.q8 = synth_prec(c->cfg.precision) == P_FP8 ? take(npos * C * cp.T) : 0;
  cp.scratch = take(cp.slot_z * cp.g.nseg_z + cp.slot_y * cp.g.nseg_y);
  const int nseg = cp.g.nseg_z + cp.g.nseg_y;
  cp.info = take(sizeof(SegInfo) * nseg);
  cp.seg_off = take(4 * (size_t)nseg);
  cp.seg_len = take(4 * (size_t)nseg);
  return UFVC_OK;
}

// Arena for the plan: its own allocation, or the shared arena (grown, which
// drops the plans laid out in the old one).
int plan_arena(ufvc_batch* b, ufvc_batch::Plan& P) {
  if (!b->arena_cap) {
    if (hipMalloc(&P.arena, P.arena_bytes) != hipSuccess) return UFVC_E_NOMEM;
    return UFVC_OK;
  }
  if (P.arena_bytes > b->arena_cap) return UFVC_E_NOSPC;
  if (P.arena_bytes > b->shared_bytes) {
    (void)hipDeviceSynchronize();
    for (auto& kv : b->plans) free_plan(b, kv.second.get());
    b->plans.clear();
    if (b->shared) (void)hipFree(b->shared);
    b->shared = nullptr;
    b->shared_bytes = 0;
    const size_t want = std::min(b->arena_cap, align_up(P.arena_bytes + P.arena_bytes / 4));
    if (hipMalloc(&b->shared, want) != hipSuccess) return UFVC_E_NOMEM;
    b->shared_bytes = want;
  }
  P.arena = b->shared;
  P.owns_arena = false;
  return UFVC_OK;
}

int build_plan(ufvc_batch* b, const ufvc_chunk* chunks, int n, ufvc_batch::Plan& P, hipStream_t s) {
  ufvc_ctx* m0 = b->models[0];
  const int C = m0->cfg.C;
  const int sl = m0->cfg.seg_log2, slz = m0->cfg.seg_log2_z;
  // arena layout
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    ChunkPlan cp;
    const int rc = layout_chunk(b->models[chunks[i].model], chunks[i].model, chunks[i].H,
                                chunks[i].W, cp, off);
    if (rc) return rc;
    P.chunks.push_back(cp);
  }
  // fp8 amax slots of all chunks, cleared together before every decode
  P.off_amax = off;
  off = align_up(off + 4 * (size_t)AMAX_WORDS * n);
  P.arena_bytes = off;
  if (const int rc = plan_arena(b, P)) return rc;
  uint8_t* A = P.arena;
  const int cp_prec = conv_prec(m0->cfg.precision);
  const int sp = synth_prec(m0->cfg.precision);
  const bool q8 = sp == P_FP8;
  const int sld = LD_NHWC;   // FP8 layers read a quantised copy (see quant below)
  const int act_st = cp_prec == P_BF16 ? ST_BF16 : ST_F32;
  // input slot k - 1, output slot k of chunk i's synthesis chain
  auto chain = [&](ConvArgs& a, int i, int k) {
    if (!q8) return;
    uint32_t* slots = at<uint32_t>(A, P.off_amax) + (size_t)AMAX_WORDS * i;
    if (k > 0) a.amax_in = slots + k - 1;
    if (k < 5) a.amax_out = amax_spread(slots, k);
  };
  // FP8 layer k (1..5) of chunk i reads a quantised copy of its input
  // (`cpp` channels per position); the batch quantises all chunks' inputs in
  // one launch before the layer's stage
  std::vector<Q8Job> q8jobs[5];
  auto quant = [&](ConvArgs& a, int i, int k, long cpp) {
    if (!q8) return;
    const ChunkPlan& q = P.chunks[i];
    const long npos = (long)q.g.h * q.g.w;
    uint32_t* slots = at<uint32_t>(A, P.off_amax) + (size_t)AMAX_WORDS * i;
    q8jobs[k - 1].push_back(Q8Job{a.in, a.in_pitch, A + q.q8, npos, (int)cpp, amax_spread(slots, k - 1),
                                  slots + k - 1});
    P.q8_units[k - 1] = std::max(P.q8_units[k - 1], npos * (cpp / 16));
    a.in = A + q.q8;
    a.in_pitch = cpp;
  };

  // ---- conv stages
  std::vector<ConvArgs> descs;
  std::vector<int4> work;
  auto stage = [&](ConvStage& st, int id, int prec, int ld, int sto, int stride, int fixed_cfg,
                   auto make) {
    st.prec = prec; st.loader = ld; st.store = sto; st.stride = stride;
    std::vector<ConvArgs> per;
    std::vector<int> groups, cfgs;
    for (int i = 0; i < n; ++i) {
      int g = 1;
      ConvArgs a = make(i, g);
      per.push_back(a);
      groups.push_back(g);
      cfgs.push_back(pick_cfg(b->models[P.chunks[i].model], id, prec, ld, stride, a, fixed_cfg));
    }
    if (b->policy == 1 && n > 1) {
      // one launch: the configuration of the chunk with the most work, if
      // every chunk of the batch can use it
      int big = 0;
      double most = -1.0;
      for (int i = 0; i < n; ++i) {
        const double wk = (double)per[i].Hout * per[i].Wout * per[i].cout * groups[i];
        if (wk > most) { most = wk; big = i; }
      }
      const int c0 = cfgs[big];
      bool ok = true;
      for (int i = 0; i < n && ok; ++i)
        ok = per[i].cout % conv_cfg(c0).bn == 0 &&
             conv_cfg_supported(prec, ld, stride, per[i].cin, per[i].cout, c0);
      if (ok) std::fill(cfgs.begin(), cfgs.end(), c0);
    }
    add_stage(P, st, descs, work, per, groups, cfgs);
    P.n_launches += (int)st.launches.size();
    P.n_stages += 1;
  };
  // encoder
  stage(P.enc_stage[0], S_A1, cp_prec, LD_UNSHUFFLE, act_st, 1, -1, [&](int i, int&) {
    const ChunkPlan& q = P.chunks[i];
    ufvc_ctx* c = b->models[q.model];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, c->a1);
    a.in = nullptr;  // the caller's frames, set per call
    a.T = q.T; a.H = q.H; a.W = q.W;
    a.out = A + q.act0; a.out_pitch = C; a.relu = 1;
    return a;
  });
  for (int i = 0; i < n; ++i) P.a1_desc.push_back(P.enc_stage[0].desc0 + i);
  stage(P.enc_stage[1], S_A2, cp_prec, LD_NHWC, act_st, 1, -1, [&](int i, int&) {
    const ChunkPlan& q = P.chunks[i];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, b->models[q.model]->a2);
    a.in = A + q.act0; a.in_pitch = C; a.out = A + q.act1; a.out_pitch = C; a.relu = 1;
    return a;
  });
  stage(P.enc_stage[2], S_A3, cp_prec, LD_NHWC, ST_F32, 1, -1, [&](int i, int&) {
    const ChunkPlan& q = P.chunks[i];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, b->models[q.model]->a3);
    a.in = A + q.act1; a.in_pitch = C; a.out = A + q.y; a.out_pitch = C; a.relu = 0;
    return a;
  });
  stage(P.enc_stage[3], S_HYPER, P_F32, LD_NHWC, ST_ZSYM, 2, -1, [&](int i, int&) {
    const ChunkPlan& q = P.chunks[i];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.hz, q.g.wz, b->models[q.model]->h);
    a.in = A + q.y; a.in_pitch = C; a.out = A + q.zsym; a.out_pitch = ZC;
    return a;
  });
  // both params stages use the encoder's tuning key (one choice for both)
  auto params_stage = [&](ConvStage& st, int id) {
    stage(st, id, P_BF16, LD_UP2, ST_F32, 1, -1, [&](int i, int&) {
      const ChunkPlan& q = P.chunks[i];
      ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, b->models[q.model]->p);
      a.in = A + q.zsym; a.in_pitch = ZC; a.out = A + q.P; a.out_pitch = 2 * C;
      return a;
    });
  };
  params_stage(P.enc_stage[4], S_PARAMS_ENC);
  // decoder
  params_stage(P.dec_stage[0], S_PARAMS_ENC);
  stage(P.dec_stage[1], S_D1, cp_prec, LD_DEQUANT, act_st, 1, -1, [&](int i, int&) {
    const ChunkPlan& q = P.chunks[i];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, b->models[q.model]->d1);
    a.in = A + q.sym; a.mu = reinterpret_cast<const float*>(A + q.P); a.mu_pitch = 2 * C;
    a.out = A + q.act0; a.out_pitch = C; a.relu = 1;
    chain(a, i, 0);
    return a;
  });
  stage(P.dec_stage[2], S_D2, sp, sld, act_st, 1, -1, [&](int i, int&) {
    const ChunkPlan& q = P.chunks[i];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, b->models[q.model]->d2);
    a.in = A + q.act0; a.in_pitch = C; a.out = A + q.act1; a.out_pitch = C; a.relu = 1;
    chain(a, i, 1);
    quant(a, i, 1, C);
    return a;
  });
  stage(P.dec_stage[3], S_D3, sp, sld, act_st, 1, -1, [&](int i, int&) {
    const ChunkPlan& q = P.chunks[i];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, b->models[q.model]->d3);
    a.in = A + q.act1; a.in_pitch = C; a.out = A + q.act0; a.out_pitch = C; a.relu = 1;
    chain(a, i, 2);
    quant(a, i, 2, C);
    return a;
  });
  stage(P.dec_stage[4], S_K1, sp, sld, act_st, 1, -1, [&](int i, int&) {
    const ChunkPlan& q = P.chunks[i];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, b->models[q.model]->k1);
    a.in = A + q.act0; a.in_pitch = C; a.out = A + q.big0; a.out_pitch = (long)q.T * C; a.relu = 1;
    chain(a, i, 3);
    quant(a, i, 3, C);
    return a;
  });
  stage(P.dec_stage[5], S_K2, sp, sld, act_st, 1, -1, [&](int i, int& g) {
    const ChunkPlan& q = P.chunks[i];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, b->models[q.model]->k2);
    a.in = A + q.big0; a.in_pitch = (long)q.T * C; a.in_goff = C;
    a.out = A + q.big1; a.out_pitch = (long)q.T * C; a.out_goff = C; a.relu = 1;
    chain(a, i, 4);
    quant(a, i, 4, (long)q.T * C);
    g = q.T;
    return a;
  });
  stage(P.dec_stage[6], S_K3, sp, sld, ST_SHUFFLE, 1, -1, [&](int i, int& g) {
    const ChunkPlan& q = P.chunks[i];
    ConvArgs a = conv_of(q.g.h, q.g.w, q.g.h, q.g.w, b->models[q.model]->k3);
    a.in = A + q.big1; a.in_pitch = (long)q.T * C; a.in_goff = C;
    a.out = nullptr;  // the caller's frames, set per call
    a.T = q.T; a.H = q.H; a.W = q.W;
    chain(a, i, 5);
    quant(a, i, 5, (long)q.T * C);
    g = q.T;
    return a;
  });
  for (int i = 0; i < n; ++i) P.k3_desc.push_back(P.dec_stage[6].desc0 + i);

  // ---- entropy descriptors
  std::vector<EpiDesc> epi_e, epi_d;
  std::vector<int2> epi_work;
  std::vector<EncSeg> encseg;
  std::vector<CompDesc> comp;
  std::vector<int2> compmap;
  std::vector<ParseDesc> parse;
  std::vector<DecSeg> decz, decy;
  for (int i = 0; i < n; ++i) {
    const ChunkPlan& q = P.chunks[i];
    ufvc_ctx* c = b->models[q.model];
    const long npos = (long)q.g.h * q.g.w;
    EpiDesc e{reinterpret_cast<const float*>(A + q.P), reinterpret_cast<const float*>(A + q.y),
              A + q.idx, A + q.sym, npos, C, 0};
    epi_e.push_back(e);
    e.y = nullptr;
    e.sym = nullptr;
    epi_d.push_back(e);
    const long total = npos * C;
    for (long blk = 0; blk * EPI_BLOCK_ELEMS < total; ++blk) epi_work.push_back(make_int2(i, (int)blk));
    SegInfo* info = at<SegInfo>(A, q.info);
    for (int sgi = 0; sgi < q.g.nseg_z + q.g.nseg_y; ++sgi) {
      const bool isz = sgi < q.g.nseg_z;
      const int si = isz ? sgi : sgi - q.g.nseg_z;
      const int l2 = isz ? slz : sl;
      const long base = (long)si << l2;
      const long ns = isz ? q.g.nz : q.g.ny;
      EncSeg es_{};
      es_.sym = (isz ? A + q.zsym : A + q.sym) + base;
      es_.idx = isz ? nullptr : A + q.idx + base;
      es_.slot = isz ? A + q.scratch + (size_t)si * q.slot_z
                     : A + q.scratch + (size_t)q.g.nseg_z * q.slot_z + (size_t)si * q.slot_y;
      es_.info = info + sgi;
      es_.nsym = (uint32_t)std::min((long)1 << l2, ns - base);
      es_.cap = 1u << l2;
      es_.fixed_row = isz ? K_Z : 0;
      encseg.push_back(es_);
      compmap.push_back(make_int2(i, sgi));
      DecSeg ds{};
      ds.bs = nullptr;  // the caller's stream, set per call
      ds.seg_off = at<uint32_t>(A, q.seg_off) + sgi;
      ds.seg_len = at<uint32_t>(A, q.seg_len) + sgi;
      ds.idx = isz ? nullptr : A + q.idx + base;
      ds.out = (isz ? A + q.zsym : A + q.sym) + base;
      ds.status = nullptr;  // set below (device status array)
      ds.len = 0;
      ds.nsym = es_.nsym;
      ds.fixed_row = isz ? K_Z : 0;
      (isz ? decz : decy).push_back(ds);
    }
    CompDesc cd{};
    cd.scratch_z = A + q.scratch;
    cd.scratch_y = A + q.scratch + (size_t)q.g.nseg_z * q.slot_z;
    cd.slot_z = q.slot_z;
    cd.slot_y = q.slot_y;
    cd.info = info;
    cd.seg_off = at<uint32_t>(A, q.seg_off);
    cd.n_seg_z = q.g.nseg_z;
    cd.n_seg_y = q.g.nseg_y;
    cd.with_header = 1;
    cd.hf = HeaderFields{(uint16_t)q.T, (uint16_t)C, (uint16_t)q.H, (uint16_t)q.W, (uint8_t)sl,
                         (uint8_t)slz, (uint8_t)K_Z, c->cfg.model_tag};
    comp.push_back(cd);
    ParseDesc pd{};
    pd.with_header = 1;
    pd.n_seg_z = q.g.nseg_z;
    pd.n_seg_y = q.g.nseg_y;
    pd.ex = cd.hf;
    pd.seg_off = at<uint32_t>(A, q.seg_off);
    pd.seg_len = at<uint32_t>(A, q.seg_len);
    parse.push_back(pd);
  }

  // ---- blob layout
  size_t bo = 0;
  auto place = [&](size_t bytes) { const size_t o = bo; bo = align_up(bo + bytes); return o; };
  P.n_conv = (int)descs.size();
  P.n_work = (int)work.size();
  P.n_epi_work = (int)epi_work.size();
  P.n_encseg = (int)encseg.size();
  P.n_compblk = (int)compmap.size();
  P.n_decz = (int)decz.size();
  P.n_decy = (int)decy.size();
  // tables that depend on the caller's buffers first (re-uploaded every
  // call), then the static ones (uploaded once per plan)
  P.off_conv = place(sizeof(ConvArgs) * descs.size());
  P.off_comp = place(sizeof(CompDesc) * n);
  P.off_parse = place(sizeof(ParseDesc) * n);
  P.off_decz = place(sizeof(DecSeg) * decz.size());
  P.off_decy = place(sizeof(DecSeg) * decy.size());
  P.dyn_bytes = bo;
  P.off_work = place(sizeof(int4) * work.size());
  P.off_epi_e = place(sizeof(EpiDesc) * n);
  P.off_epi_d = place(sizeof(EpiDesc) * n);
  P.off_epi_work = place(sizeof(int2) * epi_work.size());
  P.off_encseg = place(sizeof(EncSeg) * encseg.size());
  P.off_compmap = place(sizeof(int2) * compmap.size());
  P.off_status = place(4 * (size_t)n);
  P.off_result = place(8 * (size_t)n);
  if (q8) P.off_q8 = place(sizeof(Q8Job) * 5 * (size_t)n);
  P.hblob.assign(bo, 0);
  if (const int rc = alloc_blob(b, P, bo, s)) return rc;
  uint8_t* H = P.hblob.data();
  uint8_t* D = P.dblob;
  uint32_t* dstatus = at<uint32_t>(D, P.off_status);
  unsigned long long* dresult = at<unsigned long long>(D, P.off_result);
  for (int i = 0; i < n; ++i) {
    comp[i].result = dresult + i;
    parse[i].status = dstatus + i;
  }
  // per-segment status pointers: chunk of each segment
  {
    size_t zi = 0, yi = 0;
    for (int i = 0; i < n; ++i) {
      const ChunkPlan& q = P.chunks[i];
      for (int k = 0; k < q.g.nseg_z; ++k) decz[zi++].status = dstatus + i;
      for (int k = 0; k < q.g.nseg_y; ++k) decy[yi++].status = dstatus + i;
    }
  }
  std::memcpy(H + P.off_conv, descs.data(), sizeof(ConvArgs) * descs.size());
  std::memcpy(H + P.off_work, work.data(), sizeof(int4) * work.size());
  std::memcpy(H + P.off_epi_e, epi_e.data(), sizeof(EpiDesc) * n);
  std::memcpy(H + P.off_epi_d, epi_d.data(), sizeof(EpiDesc) * n);
  std::memcpy(H + P.off_epi_work, epi_work.data(), sizeof(int2) * epi_work.size());
  std::memcpy(H + P.off_encseg, encseg.data(), sizeof(EncSeg) * encseg.size());
  std::memcpy(H + P.off_comp, comp.data(), sizeof(CompDesc) * n);
  std::memcpy(H + P.off_compmap, compmap.data(), sizeof(int2) * compmap.size());
  std::memcpy(H + P.off_parse, parse.data(), sizeof(ParseDesc) * n);
  std::memcpy(H + P.off_decz, decz.data(), sizeof(DecSeg) * decz.size());
  std::memcpy(H + P.off_decy, decy.data(), sizeof(DecSeg) * decy.size());
  if (q8)
    for (int k = 0; k < 5; ++k) {
      if ((int)q8jobs[k].size() != n) return UFVC_E_INVAL;
      std::memcpy(H + P.off_q8 + sizeof(Q8Job) * (size_t)k * n, q8jobs[k].data(), sizeof(Q8Job) * n);
    }
  return UFVC_OK;
}

// Writes the call-varying descriptor fields into the host mirror and uploads
// the blob through pinned staging on `s`.
int upload(ufvc_batch* b, ufvc_batch::Plan& P, const ufvc_chunk* chunks, int n, bool encode,
           hipStream_t s) {
  uint8_t* H = P.hblob.data();
  ConvArgs* cd = at<ConvArgs>(H, P.off_conv);
  CompDesc* comp = at<CompDesc>(H, P.off_comp);
  ParseDesc* parse = at<ParseDesc>(H, P.off_parse);
  DecSeg* decz = at<DecSeg>(H, P.off_decz);
  DecSeg* decy = at<DecSeg>(H, P.off_decy);
  size_t zi = 0, yi = 0;
  for (int i = 0; i < n; ++i) {
    const ChunkPlan& q = P.chunks[i];
    if (encode) {
      cd[P.a1_desc[i]].in = chunks[i].frames;
      comp[i].out = chunks[i].bitstream;
      comp[i].capacity = chunks[i].capacity;
    } else {
      cd[P.k3_desc[i]].out = chunks[i].frames_out;
      parse[i].bs = chunks[i].bitstream;
      parse[i].len = chunks[i].len;
      for (int k = 0; k < q.g.nseg_z; ++k, ++zi) { decz[zi].bs = chunks[i].bitstream; decz[zi].len = chunks[i].len; }
      for (int k = 0; k < q.g.nseg_y; ++k, ++yi) { decy[yi].bs = chunks[i].bitstream; decy[yi].len = chunks[i].len; }
    }
  }
  if (b->staging_bytes < P.hblob.size()) {
    if (b->staged) (void)hipEventSynchronize(b->staged);
    if (b->staging) (void)hipHostFree(b->staging);
    b->staging = nullptr;
    b->staging_bytes = 0;
    if (hipHostMalloc(&b->staging, P.hblob.size()) != hipSuccess) return UFVC_E_NOMEM;
    b->staging_bytes = P.hblob.size();
  }
  if (b->staged) CK(hipEventSynchronize(b->staged));
  const size_t bytes = P.uploaded ? P.dyn_bytes : P.hblob.size();
  std::memcpy(b->staging, H, bytes);
  CK(hipMemcpyAsync(P.dblob, b->staging, bytes, hipMemcpyHostToDevice, s));
  CK(hipEventRecord(b->staged, s));
  P.uploaded = true;
  return UFVC_OK;
}

hipError_t run_stage(ufvc_batch::Plan& P, const ConvStage& st, hipStream_t s) {
  const ConvArgs* d = at<ConvArgs>(P.dblob, P.off_conv);
  const int4* w = at<int4>(P.dblob, P.off_work);
  for (const ConvLaunch& L : st.launches) {
    const hipError_t e = launch_conv_batch(st.prec, st.loader, st.store, st.stride, L.cfg, d,
                                           w + L.work0, L.nwork, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_decode(ufvc_batch* b, ufvc_batch::Plan& P, hipStream_t s) {
  ufvc_ctx* m0 = b->models[0];
  uint8_t* D = P.dblob;
  const int n = (int)P.chunks.size();
  hipError_t e = launch_zero_u32(at<uint32_t>(D, P.off_status), n, s);
  if (e != hipSuccess) return e;
  if (synth_prec(m0->cfg.precision) == P_FP8 &&
      (e = launch_zero_u32(at<uint32_t>(P.arena, P.off_amax), AMAX_WORDS * n, s)) != hipSuccess)
    return e;
  if ((e = launch_parse_batch(at<ParseDesc>(D, P.off_parse), n, s)) != hipSuccess) return e;
  if ((e = launch_rans_decode_batch(m0->tab, at<DecSeg>(D, P.off_decz), P.n_decz, true, s)) != hipSuccess) return e;
  if ((e = run_stage(P, P.dec_stage[0], s)) != hipSuccess) return e;
  if ((e = launch_params_epilogue_batch(at<EpiDesc>(D, P.off_epi_d), at<int2>(D, P.off_epi_work),
                                        P.n_epi_work, m0->tab.thresholds, s)) != hipSuccess)
    return e;
  if ((e = launch_rans_decode_batch(m0->tab, at<DecSeg>(D, P.off_decy), P.n_decy, false, s)) != hipSuccess) return e;
  const bool q8 = synth_prec(m0->cfg.precision) == P_FP8;
  for (int k = 1; k < 7; ++k) {
    // FP8 layers d2 .. k3: their inputs quantised first
    if (q8 && k >= 2 &&
        (e = launch_q8_batch(at<Q8Job>(D, P.off_q8) + (size_t)(k - 2) * n, n, P.q8_units[k - 2], s)) != hipSuccess)
      return e;
    if ((e = run_stage(P, P.dec_stage[k], s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Runs single-chunk encode and decode once for every (model, H, W) bucket that
// the model's autotuner has not seen, so batch launches use tuned tiles.
int tune_buckets(ufvc_batch* b, const ufvc_chunk* chunks, int n, hipStream_t s) {
  std::map<std::vector<int>, int> seen;
  for (int i = 0; i < n; ++i) {
    ufvc_ctx* c = b->models[chunks[i].model];
    if (!c->cfg.autotune) continue;
    std::vector<int> k{chunks[i].model, chunks[i].H, chunks[i].W};
    if (seen.count(k)) continue;
    seen[k] = 1;
    Geom g;
    if (!geom(c, chunks[i].H, chunks[i].W, g)) return UFVC_E_INVAL;
    if (c->tune.count(tune_key(S_K3, g.h, g.w))) continue;
    const size_t nfr = (size_t)c->cfg.T * 3 * chunks[i].H * chunks[i].W;
    float* fr = nullptr;
    float* fo = nullptr;
    uint8_t* bs = nullptr;
    const size_t cap = ufvc_max_bitstream_bytes(c, chunks[i].H, chunks[i].W);
    if (hipMalloc(&fr, 4 * nfr) || hipMalloc(&fo, 4 * nfr) || hipMalloc(&bs, cap)) return UFVC_E_NOMEM;
    CK(hipMemsetAsync(fr, 0, 4 * nfr, s));
    size_t len = 0;
    int rc = ufvc_encode_chunk(c, fr, c->cfg.T, chunks[i].H, chunks[i].W, bs, cap, &len, s);
    if (!rc) rc = ufvc_decode_chunk(c, bs, len, c->cfg.T, chunks[i].H, chunks[i].W, fo, s);
    if (!rc) rc = ufvc_sync_status(c, s);
    (void)hipFree(fr);
    (void)hipFree(fo);
    (void)hipFree(bs);
    if (rc) return rc;
  }
  return UFVC_OK;
}

int get_plan(ufvc_batch* b, const ufvc_chunk* chunks, int n, hipStream_t s, ufvc_batch::Plan** out) {
  std::vector<int> key;
  for (int i = 0; i < n; ++i) {
    if (chunks[i].model < 0 || chunks[i].model >= (int)b->models.size()) return UFVC_E_INVAL;
    key.push_back(chunks[i].model);
    key.push_back(chunks[i].H);
    key.push_back(chunks[i].W);
  }
  auto it = b->plans.find(key);
  if (it != b->plans.end()) {
    it->second->last_use = ++b->use_clock;
    b->last_plan = it->second.get();
    *out = it->second.get();
    return UFVC_OK;
  }
  // bounded cache: the least recently used plan goes (after its last call on
  // this stream has finished with its descriptors and graph)
  if (b->plans.size() >= kMaxPlans) CK(evict_lru(b, s));
  // tuning runs single-chunk calls on the shared model contexts, and plans
  // read their tuning maps: one plan build at a time across batch objects
  static std::mutex build_mu;
  std::lock_guard<std::mutex> lock(build_mu);
  int rc = tune_buckets(b, chunks, n, s);
  if (rc) return rc;
  std::unique_ptr<ufvc_batch::Plan> P(new (std::nothrow) ufvc_batch::Plan());
  if (!P) return UFVC_E_NOMEM;
  P->key = key;
  rc = build_plan(b, chunks, n, *P, s);
  if (rc) {
    free_plan(b, P.get());
    return rc;
  }
  if (b->host_cap < n) {
    if (b->results_host) (void)hipHostFree(b->results_host);
    if (b->status_host) (void)hipHostFree(b->status_host);
    b->results_host = nullptr;
    b->status_host = nullptr;
    b->host_cap = 0;
    if (hipHostMalloc(&b->results_host, 8 * (size_t)n) || hipHostMalloc(&b->status_host, 4 * (size_t)n))
      return UFVC_E_NOMEM;
    b->host_cap = n;
  }
  P->last_use = ++b->use_clock;
  b->plans_built += 1;
  b->last_plan = P.get();
  *out = P.get();
  b->plans[key] = std::move(P);
  return UFVC_OK;
}

}  // namespace

int batch_set_arena_cap(ufvc_batch* b, size_t cap) {
  if (!b || !b->plans.empty() || b->arena_cap) return UFVC_E_INVAL;
  b->arena_cap = cap;
  return UFVC_OK;
}

int batch_reserve_arena(ufvc_batch* b, int max_batch, size_t blob_bytes) {
  if (!b || !b->arena_cap || b->shared || b->blob_slab || max_batch < 1) return UFVC_E_INVAL;
  if (hipMalloc(&b->shared, b->arena_cap) != hipSuccess) return UFVC_E_NOMEM;
  b->shared_bytes = b->arena_cap;
  blob_bytes = blob_bytes / ALIGN * ALIGN;
  if (blob_bytes) {
    if (hipMalloc(&b->blob_slab, blob_bytes) != hipSuccess) return UFVC_E_NOMEM;
    b->blob_cap = blob_bytes;
    b->blob_free[0] = blob_bytes;
    // pinned staging for any blob the slab can hold
    if (hipHostMalloc(&b->staging, blob_bytes) != hipSuccess) return UFVC_E_NOMEM;
    b->staging_bytes = blob_bytes;
  }
  if (hipHostMalloc(&b->results_host, 8 * (size_t)max_batch) != hipSuccess ||
      hipHostMalloc(&b->status_host, 4 * (size_t)max_batch) != hipSuccess)
    return UFVC_E_NOMEM;
  b->host_cap = max_batch;
  return UFVC_OK;
}

uint64_t batch_plans_built(const ufvc_batch* b) { return b ? b->plans_built : 0; }

size_t batch_chunk_footprint(ufvc_ctx* c, int H, int W) {
  ChunkPlan cp;
  size_t off = 0;
  if (layout_chunk(c, 0, H, W, cp, off)) return 0;
  return off + align_up(4 * (size_t)AMAX_WORDS);  // + its share of the per-batch amax block
}

extern "C" {

int ufvc_batch_create(ufvc_ctx* const* models, int n_models, ufvc_batch** out) {
  if (!models || n_models < 1 || !out) return UFVC_E_INVAL;
  *out = nullptr;
  const ufvc_config& c0 = models[0]->cfg;
  for (int i = 0; i < n_models; ++i) {
    if (!models[i]) return UFVC_E_INVAL;
    const ufvc_config& ci = models[i]->cfg;
    if (ci.C != c0.C || ci.precision != c0.precision || ci.seg_log2 != c0.seg_log2 ||
        ci.seg_log2_z != c0.seg_log2_z)
      return UFVC_E_INVAL;
    // the batched pipeline has no quadtree mean steps and no stream contexts
    if (ci.quadtree || ci.temporal) return UFVC_E_UNSUPPORTED;
  }
  ufvc_batch* b = new (std::nothrow) ufvc_batch();
  if (!b) return UFVC_E_NOMEM;
  b->models.assign(models, models + n_models);
  if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) {
    if (b->staged) (void)hipEventDestroy(b->staged);
    delete b;
    return UFVC_E_DEVICE;
  }
  *out = b;
  return UFVC_OK;
}

int ufvc_batch_set_policy(ufvc_batch* b, int policy) {
  if (!b || (policy != 0 && policy != 1)) return UFVC_E_INVAL;
  if (policy == b->policy) return UFVC_OK;
  CK(hipDeviceSynchronize());
  for (auto& kv : b->plans) free_plan(b, kv.second.get());
  b->plans.clear();
  b->last_plan = nullptr;
  b->policy = policy;
  return UFVC_OK;
}

int ufvc_batch_stats(ufvc_batch* b, uint64_t* stats, int n) {
  if (!b || !stats || n < 6) return UFVC_E_INVAL;
  stats[0] = b->plans_built;
  stats[1] = b->plans_evicted;
  stats[2] = b->plans.size();
  stats[3] = b->last_plan ? (uint64_t)b->last_plan->n_stages : 0;
  stats[4] = b->last_plan ? (uint64_t)b->last_plan->n_launches : 0;
  stats[5] = (uint64_t)b->policy;
  return UFVC_OK;
}

void ufvc_batch_destroy(ufvc_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : b->plans) free_plan(b, kv.second.get());
  if (b->shared) (void)hipFree(b->shared);
  if (b->blob_slab) (void)hipFree(b->blob_slab);
  if (b->staging) (void)hipHostFree(b->staging);
  if (b->results_host) (void)hipHostFree(b->results_host);
  if (b->status_host) (void)hipHostFree(b->status_host);
  if (b->staged) (void)hipEventDestroy(b->staged);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

int ufvc_encode_batch(ufvc_batch* b, ufvc_chunk* chunks, int n, void* stream) {
  if (!b || !chunks || n < 1) return UFVC_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < n; ++i) {
    if (!chunks[i].frames || !chunks[i].bitstream) return UFVC_E_INVAL;
  }
  ufvc_batch::Plan* P = nullptr;
  int rc = get_plan(b, chunks, n, s, &P);
  if (rc) return rc;
  rc = upload(b, *P, chunks, n, true, s);
  if (rc) return rc;
  ufvc_ctx* m0 = b->models[0];
  uint8_t* D = P->dblob;
  for (int k = 0; k < 5; ++k) CK(run_stage(*P, P->enc_stage[k], s));
  CK(launch_params_epilogue_batch(at<EpiDesc>(D, P->off_epi_e), at<int2>(D, P->off_epi_work),
                                  P->n_epi_work, m0->tab.thresholds, s));
  CK(launch_rans_encode_batch(m0->tab, at<EncSeg>(D, P->off_encseg), P->n_encseg, s));
  CK(launch_compact_batch(at<CompDesc>(D, P->off_comp), n, at<int2>(D, P->off_compmap), P->n_compblk, s));
  CK(hipMemcpyAsync(b->results_host, D + P->off_result, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  int worst = UFVC_OK;
  for (int i = 0; i < n; ++i) {
    chunks[i].len = (size_t)b->results_host[i];
    chunks[i].status = chunks[i].len > chunks[i].capacity ? UFVC_E_NOSPC : UFVC_OK;
    if (chunks[i].status) worst = chunks[i].status;
  }
  return worst;
}

int ufvc_decode_batch(ufvc_batch* b, ufvc_chunk* chunks, int n, int use_graph, void* stream) {
  if (!b || !chunks || n < 1) return UFVC_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < n; ++i) {
    if (!chunks[i].frames_out || !chunks[i].bitstream || chunks[i].len < 28 ||
        chunks[i].len > 0xFFFFFFF0ull)
      return UFVC_E_INVAL;
  }
  ufvc_batch::Plan* P = nullptr;
  int rc = get_plan(b, chunks, n, s, &P);
  if (rc) return rc;
  rc = upload(b, *P, chunks, n, false, s);
  if (rc) return rc;
  // a composition's first decode runs eagerly; the graph is captured when it
  // recurs, so one-off compositions (common in serving) never pay the
  // capture and instantiation on the request path
  const bool first = P->decodes++ == 0;
  if (!use_graph || (first && !P->gexec)) {
    CK(run_decode(b, *P, s));
    return UFVC_OK;
  }
  if (!P->gexec) {
    // capture on the batch's own stream; the graph is then launched on `s`
    CK(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    const hipError_t e = run_decode(b, *P, b->capture);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->capture, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return UFVC_E_DEVICE;
    }
    P->graph = g;
    CK(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0));
  }
  CK(hipGraphLaunch(P->gexec, s));
  return UFVC_OK;
}

int ufvc_batch_sync_status(ufvc_batch* b, ufvc_chunk* chunks, int n, void* stream) {
  if (!b || !chunks || n < 1) return UFVC_E_INVAL;
  std::vector<int> key;
  for (int i = 0; i < n; ++i) {
    key.push_back(chunks[i].model);
    key.push_back(chunks[i].H);
    key.push_back(chunks[i].W);
  }
  auto it = b->plans.find(key);
  if (it == b->plans.end()) return UFVC_E_INVAL;
  ufvc_batch::Plan& P = *it->second;
  hipStream_t s = (hipStream_t)stream;
  CK(hipMemcpyAsync(b->status_host, P.dblob + P.off_status, 4 * (size_t)n, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  int worst = UFVC_OK;
  for (int i = 0; i < n; ++i) {
    const uint32_t st = b->status_host[i];
    chunks[i].status = (st & ST_BAD_HEADER) ? UFVC_E_INVAL : (st & ST_CORRUPT) ? UFVC_E_CORRUPT : UFVC_OK;
    if (chunks[i].status && !worst) worst = chunks[i].status;
  }
  return worst;
}

}  // extern "C"
