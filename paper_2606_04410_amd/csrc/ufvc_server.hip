// Request server: continuous batching of chunk encode / decode requests over
// the batch executor, with admission by HBM footprint.
//
// Each lane is one host thread with its own HIP stream and batch object (in
// shared-arena mode, capped at the lane's share of the budget).  A free lane
// forms its next batch from the queue: the oldest request, then further
// queued requests of the same kind in arrival order, while the batch's arena
// fits the lane and the footprint of everything admitted and unfinished fits
// the budget.  It runs the batch on its stream, waits for that stream only,
// and publishes the completions.  Lanes run concurrently, so one batch's
// latency-bound entropy coding overlaps another batch's convolutions, and
// requests that arrive meanwhile are picked up by whichever lane frees first.
#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "ufvc_ctx.h"

struct ufvc_server {
  struct Req {
    ufvc_request r;
    uint64_t ticket;
    size_t arena;       // working arena bytes in a batch
    size_t footprint;   // arena + the request's own device buffers
    double t_submit;
  };
  struct Lane {
    hipStream_t stream = nullptr;
    ufvc_batch* batch = nullptr;
    std::thread th;
  };
  std::vector<ufvc_ctx*> models;
  ufvc_server_config cfg{};
  size_t lane_cap = 0;      // a lane's arena
  size_t blob_cap = 0;      // a lane's descriptor-blob slab
  size_t req_budget = 0;    // the budget less the lanes' slabs: admitted request footprints
  int device = 0;
  std::vector<Lane> lanes;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req> queue;
  std::deque<ufvc_completion> done;
  size_t in_flight_bytes = 0, peak_bytes = 0;
  uint64_t next_ticket = 1, n_in_flight = 0, n_completed = 0, n_batches = 0;
  bool stopping = false;
  std::chrono::steady_clock::time_point t0;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

constexpr size_t kDefaultBudget = 64ull << 30;

// Forms the next batch for lane `li` (called with the lock held); empty when
// nothing can be admitted now.  With small_pixels set (and two or more
// lanes), lane 0 prefers small requests: it starts from the oldest request
// of at most small_pixels per frame and batches only such requests, so a
// large request at the head of the queue cannot hold every lane; when no
// small request is queued it takes the oldest as the other lanes do.
std::vector<ufvc_server::Req> take_batch(ufvc_server* S, int li) {
  std::vector<ufvc_server::Req> out;
  if (S->queue.empty()) return out;
  const long small = S->cfg.small_pixels;
  auto is_small = [&](const ufvc_server::Req& q) { return (long)q.r.H * q.r.W <= small; };
  bool small_only = false;
  auto head = S->queue.begin();
  if (small > 0 && li == 0 && S->lanes.size() >= 2) {
    auto f = std::find_if(S->queue.begin(), S->queue.end(), is_small);
    if (f != S->queue.end()) {
      head = f;
      small_only = true;
    }
  }
  const int kind = head->r.kind;
  size_t arena = 0, foot = 0;
  for (auto it = head; it != S->queue.end() && (int)out.size() < S->cfg.max_batch;) {
    if (it->r.kind != kind || (small_only && !is_small(*it))) {
      ++it;
      continue;
    }
    if (arena + it->arena > S->lane_cap || S->in_flight_bytes + foot + it->footprint > S->req_budget) {
      if (out.empty()) return out;   // the oldest request waits for memory
      break;
    }
    arena += it->arena;
    foot += it->footprint;
    out.push_back(*it);
    it = S->queue.erase(it);
  }
  S->in_flight_bytes += foot;
  S->peak_bytes = std::max(S->peak_bytes, S->in_flight_bytes);
  S->n_in_flight += out.size();
  return out;
}

void run_batch(ufvc_server* S, ufvc_server::Lane& L, std::vector<ufvc_server::Req>& reqs,
               std::vector<ufvc_completion>& comp) {
  const double t_admit = S->now_us();
  // one plan per (model, H, W) multiset: order the chunks canonically
  std::vector<int> order(reqs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    const ufvc_request& x = reqs[a].r;
    const ufvc_request& y = reqs[b].r;
    if (x.model != y.model) return x.model < y.model;
    if (x.H != y.H) return x.H < y.H;
    if (x.W != y.W) return x.W < y.W;
    return a < b;
  });
  std::vector<ufvc_chunk> chunks(reqs.size());
  for (size_t k = 0; k < order.size(); ++k) {
    const ufvc_request& r = reqs[order[k]].r;
    ufvc_chunk& c = chunks[k];
    c.model = r.model;
    c.H = r.H;
    c.W = r.W;
    c.frames = r.frames;
    c.frames_out = r.frames_out;
    c.bitstream = r.bitstream;
    c.capacity = r.capacity;
    c.len = r.kind == UFVC_REQ_DECODE ? r.len : 0;
    c.status = INT_MIN;
  }
  const int n = (int)chunks.size();
  int rc;
  if (reqs[0].r.kind == UFVC_REQ_ENCODE) {
    rc = ufvc_encode_batch(L.batch, chunks.data(), n, L.stream);
  } else {
    rc = ufvc_decode_batch(L.batch, chunks.data(), n, S->cfg.use_graph, L.stream);
    if (rc == UFVC_OK) rc = ufvc_batch_sync_status(L.batch, chunks.data(), n, L.stream);
  }
  if (rc != UFVC_OK) (void)hipStreamSynchronize(L.stream);
  const double t_done = S->now_us();
  comp.clear();
  for (size_t k = 0; k < order.size(); ++k) {
    const ufvc_server::Req& q = reqs[order[k]];
    ufvc_completion c{};
    c.ticket = q.ticket;
    c.tag = q.r.tag;
    c.status = chunks[k].status == INT_MIN ? (rc != UFVC_OK ? rc : UFVC_E_DEVICE) : chunks[k].status;
    c.batch_size = n;
    c.len = q.r.kind == UFVC_REQ_ENCODE ? chunks[k].len : q.r.len;
    c.t_submit_us = q.t_submit;
    c.t_admit_us = t_admit;
    c.t_done_us = t_done;
    comp.push_back(c);
  }
}

void lane_main(ufvc_server* S, int li) {
  (void)hipSetDevice(S->device);
  ufvc_server::Lane& L = S->lanes[li];
  std::vector<ufvc_completion> comp;
  for (;;) {
    std::vector<ufvc_server::Req> reqs;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        reqs = take_batch(S, li);
        if (!reqs.empty()) break;
        if (S->stopping && S->queue.empty()) return;
        S->cv_work.wait(lk);
      }
    }
    run_batch(S, L, reqs, comp);
    size_t foot = 0;
    for (const auto& q : reqs) foot += q.footprint;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->in_flight_bytes -= foot;
      S->n_in_flight -= reqs.size();
      S->n_completed += reqs.size();
      S->n_batches += 1;
      for (const auto& c : comp) S->done.push_back(c);
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

int ufvc_server_create(ufvc_ctx* const* models, int n_models, const ufvc_server_config* cfg,
                       ufvc_server** out) {
  if (!models || n_models < 1 || !cfg || !out) return UFVC_E_INVAL;
  *out = nullptr;
  if (cfg->lanes < 1 || cfg->lanes > 8 || cfg->max_batch < 1 || cfg->max_batch > 64 ||
      cfg->small_pixels < 0)
    return UFVC_E_INVAL;
  ufvc_server* S = new (std::nothrow) ufvc_server();
  if (!S) return UFVC_E_NOMEM;
  S->models.assign(models, models + n_models);
  S->cfg = *cfg;
  if (!S->cfg.hbm_budget) S->cfg.hbm_budget = kDefaultBudget;
  // each lane's share of the budget: a descriptor-blob slab (1/16 of the
  // share, at most 64 MiB), the rest its arena
  const size_t share = S->cfg.hbm_budget / (size_t)S->cfg.lanes;
  S->blob_cap = std::min<size_t>(share / 16, 64ull << 20) & ~(size_t)4095;
  S->lane_cap = share - S->blob_cap;
  S->req_budget = S->cfg.hbm_budget - S->blob_cap * (size_t)S->cfg.lanes;
  S->device = models[0]->device;
  S->t0 = std::chrono::steady_clock::now();
  S->lanes.resize(cfg->lanes);
  int rc = UFVC_OK;
  for (auto& L : S->lanes) {
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess) {
      rc = UFVC_E_DEVICE;
      break;
    }
    if ((rc = ufvc_batch_create(models, n_models, &L.batch)) != UFVC_OK) break;
    if ((rc = batch_set_arena_cap(L.batch, S->lane_cap)) != UFVC_OK) break;
    // the lane's whole share now (arena, descriptor slab, staging, host
    // result arrays): no allocation, arena growth or plan loss on the
    // request path
    if ((rc = batch_reserve_arena(L.batch, S->cfg.max_batch, S->blob_cap)) != UFVC_OK) break;
  }
  if (rc != UFVC_OK) {
    for (auto& L : S->lanes) {
      if (L.batch) ufvc_batch_destroy(L.batch);
      if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    delete S;
    return rc;
  }
  for (int i = 0; i < cfg->lanes; ++i) S->lanes[i].th = std::thread(lane_main, S, i);
  *out = S;
  return UFVC_OK;
}

int ufvc_server_submit(ufvc_server* S, const ufvc_request* req, uint64_t* ticket) {
  if (!S || !req) return UFVC_E_INVAL;
  const ufvc_request& r = *req;
  if (r.model < 0 || r.model >= (int)S->models.size()) return UFVC_E_INVAL;
  if (r.kind != UFVC_REQ_ENCODE && r.kind != UFVC_REQ_DECODE) return UFVC_E_INVAL;
  ufvc_ctx* c = S->models[r.model];
  const size_t arena = batch_chunk_footprint(c, r.H, r.W);
  if (!arena) return UFVC_E_INVAL;
  const size_t frame_bytes = (size_t)c->cfg.T * 3 * r.H * r.W * sizeof(float);
  size_t io;
  if (r.kind == UFVC_REQ_ENCODE) {
    if (!r.frames || !r.bitstream) return UFVC_E_INVAL;
    io = frame_bytes + r.capacity;
  } else {
    if (!r.frames_out || !r.bitstream || r.len < 28 || r.len > 0xFFFFFFF0ull) return UFVC_E_INVAL;
    io = frame_bytes + r.len;
  }
  if (arena > S->lane_cap || arena + io > S->req_budget) return UFVC_E_NOSPC;
  ufvc_server::Req q;
  q.r = r;
  q.arena = arena;
  q.footprint = arena + io;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return UFVC_E_INVAL;
    q.ticket = S->next_ticket++;
    q.t_submit = S->now_us();
    S->queue.push_back(q);
  }
  if (ticket) *ticket = q.ticket;
  S->cv_work.notify_one();
  return UFVC_OK;
}

int ufvc_server_poll(ufvc_server* S, ufvc_completion* out, int max, int timeout_ms) {
  if (!S || !out || max < 1) return UFVC_E_INVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->done.empty() && timeout_ms > 0)
    S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !S->done.empty(); });
  int k = 0;
  while (k < max && !S->done.empty()) {
    out[k++] = S->done.front();
    S->done.pop_front();
  }
  return k;
}

int ufvc_server_stats(ufvc_server* S, uint64_t* stats, int n) {
  if (!S || !stats || n < 1) return UFVC_E_INVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  uint64_t built = 0;
  for (const auto& L : S->lanes) built += batch_plans_built(L.batch);
  const uint64_t v[8] = {S->queue.size(), S->n_in_flight, S->n_completed, S->n_batches,
                         S->peak_bytes, S->cfg.hbm_budget, built,
                         (S->lane_cap + S->blob_cap) * S->lanes.size()};
  for (int i = 0; i < n && i < 8; ++i) stats[i] = v[i];
  return UFVC_OK;
}

void ufvc_server_destroy(ufvc_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  for (auto& L : S->lanes)
    if (L.th.joinable()) L.th.join();
  for (auto& L : S->lanes) {
    if (L.batch) ufvc_batch_destroy(L.batch);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  delete S;
}

}  // extern "C"
