// Single-step entropy coding of the chunk latent (Sec. 3.4).
//
// * build_tables: Gaussian CDF tables in FP64 (64 log-spaced scales in
//   [0.11, 64], 65 residual values in [-32, 32], 16-bit total), the float32
//   scale-index thresholds, the multiplier/shift pairs that turn the
//   encoder's division by a frequency into a multiply-high (Granlund and
//   Montgomery 1994, "Division by invariant integers using multiplication"),
//   and a 256-bucket slot -> symbol lookup for the decoder.
// * params_epilogue: sigma = clamp(softplus(.), 0.11, 64) in float32 and its
//   table index for every latent element; in the encoder also the residual
//   symbol r_hat = round(y - mu).  The mean is never needed for coding.
// * rans_encode / rans_decode: 32-lane interleaved rANS (Duda 2013; Giesen
//   2014), state in [2^16, 2^32), 16-bit renormalisation.  One half-wave
//   (32 lanes of a wave64) owns one segment, so a wave codes two segments.
//   The lanes of a step find their word slots with a ballot + popcount
//   prefix count; all per-step traffic goes through LDS (see below).
// * compact / parse: container assembly with coalesced copies, and the
//   decoder's header validation and segment offset scan.
#include "ufvc_common.h"

namespace ufvc {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr uint32_t RANS_L = 1u << 16;

// ------------------------------------------------------------- tables ----
__global__ void build_tables_kernel(Tables t) {
  const int k = threadIdx.x;
  if (k >= NSCALES) return;
  const double lo = log(0.11), hi = log(64.0);
  const double s = exp(lo + k * (hi - lo) / 63.0);
  if (k < NSCALES - 1) {
    const double s1 = exp(lo + (k + 1) * (hi - lo) / 63.0);
    t.thresholds[k] = (float)sqrt(s * s1);
  } else {
    t.thresholds[k] = __builtin_inff();
  }
  // Mass of residual r under N(0, s^2) on [r - 1/2, r + 1/2); r = -32 takes
  // the left tail; r > 0 mirrors r < 0 so the table is exactly symmetric.
  uint32_t f[NSYM];
  const double sq2 = sqrt(2.0);
  for (int r = -32; r <= 0; ++r) {
    double p;
    if (r == 0) {
      p = erf(0.5 / (s * sq2));
    } else if (r == -32) {
      p = 0.5 * erfc(-((r + 0.5) / s) / sq2);
    } else {
      p = 0.5 * erfc(-((r + 0.5) / s) / sq2) - 0.5 * erfc(-((r - 0.5) / s) / sq2);
    }
    const uint32_t q = 1u + (uint32_t)floor(p * (double)(65536 - NSYM));
    f[r + 32] = q;
    f[32 - r] = q;
  }
  uint32_t sum = 0;
  for (int i = 0; i < NSYM; ++i) sum += f[i];
  f[32] += 65536u - sum;
  uint32_t cum = 0;
  for (int i = 0; i < NSYM; ++i) {
    const uint32_t fi = f[i];
    t.fc[k * NSYM + i] = fi | (cum << 16);
    const uint32_t l = 32u - __clz(fi - 1u);  // ceil(log2(fi)), 0 for fi = 1
    const unsigned long long num = (((1ull << l) - fi) << 32);
    t.magic[k * NSYM + i] = (uint32_t)(num / fi + 1ull);
    t.shift[k * NSYM + i] = (uint8_t)l;
    cum += fi;
  }
  // Decoder lookup, 256 buckets of 256 slots per row.  lut[b] (16 bits):
  // bits 0..6 hold base + 1 and bits 7..14 an offset o: a middle slot s of
  // the bucket decodes to base + (s % 256 >= o).  A bucket whose first middle
  // slot belongs to s0 and that holds s0 + 1 from offset o > 0 on stores
  // (s0, o); a bucket wholly inside s0 stores (s0 - 1, 0).  Bit 15 marks a
  // slow bucket: it holds three or more symbols, or frequency-1 tail slots;
  // its base is s0, where a scan starts.  The tails (leading run of
  // frequency-1 symbols and its mirror, fewer than 33 slots) sit in the first
  // and last bucket and map slot -> symbol in closed form.
  uint32_t tail = 0;
  while (tail < 32 && f[tail] == 1u) ++tail;
  t.tail[k] = (uint8_t)tail;
  const uint32_t mid_end = 65536u - tail;
  int sidx = 0;
  uint32_t c = 0;
  for (int b = 0; b < LUT_BUCKETS; ++b) {
    const uint32_t b0 = (uint32_t)b * LUT_SLOTS;
    const uint32_t first = max(b0, tail);
    const uint32_t last = min(b0 + LUT_SLOTS, mid_end);
    uint32_t entry = 0x8000u | 1u;
    if (first < last) {
      while (sidx + 1 < NSYM && c + f[sidx] <= first) { c += f[sidx]; ++sidx; }
      const uint32_t end0 = c + f[sidx];
      bool slow = tail > 0 && (first > b0 || last < b0 + LUT_SLOTS);
      if (end0 < last && (sidx + 1 >= NSYM || end0 + f[sidx + 1] < last)) slow = true;
      uint32_t base1 = (uint32_t)sidx + 1u, off = 0;
      if (!slow) {
        if (end0 < last) off = end0 - b0;   // 1 .. 255
        else base1 = (uint32_t)sidx;        // base s0 - 1, offset 0
      }
      entry = base1 | (off << 7) | (slow ? 0x8000u : 0u);
    }
    t.lut[k * LUT_BUCKETS + b] = (uint16_t)entry;
  }
}

hipError_t launch_build_tables(const Tables& t, hipStream_t s) {
  hipLaunchKernelGGL(build_tables_kernel, dim3(1), dim3(64), 0, s, t);
  return hipGetLastError();
}

// ------------------------------------------------------ params epilogue ----
typedef float v4f __attribute__((ext_vector_type(4)));

// Threshold table of the scale index, in LDS, with its log spacing.  The
// thresholds are geometric midpoints of log-spaced scales, so the count of
// thresholds <= sigma is within one of 1 + floor((log sigma - log t0) / step)
// (step = log(t62 / t0) / 62); one exact float32 comparison each way fixes it.
struct ThrTable {
  const float* t;   // 64 floats, t[63] = +inf
  float lt0, inv_step;
};
__device__ __forceinline__ ThrTable thr_table(const float* s_thr) {
  const float lt0 = __logf(s_thr[0]);
  return ThrTable{s_thr, lt0, 62.f / (__logf(s_thr[62]) - lt0)};
}

// CDF table index of one scale logit: sigma = clamp(softplus(x), 0.11, 64)
// in float32 (softplus as max(x, 0) + log1p(exp(-|x|)), with the hardware
// exp and log), then the number of thresholds <= sigma.
__device__ __forceinline__ uint32_t scale_index(float xs, const ThrTable& tt) {
  const float sp = fmaxf(xs, 0.f) + __logf(1.f + __expf(-fabsf(xs)));
  const float sigma = fminf(fmaxf(sp, 0.11f), 64.f);
  const int g = (int)floorf((__logf(sigma) - tt.lt0) * tt.inv_step) + 1;
  const int k0 = min(max(g, 0), 63);
  const float lo = tt.t[max(k0 - 1, 0)];
  const float hi = tt.t[k0];
  return (uint32_t)(k0 - ((k0 > 0 && lo > sigma) ? 1 : 0) + (hi <= sigma ? 1 : 0));
}

// Four consecutive latent elements e .. e + 3 (e % 4 == 0, C % 4 == 0: one
// position, four channels): 16-byte loads of the scale logits (and, in the
// encoder, of the means and y), one 4-byte store of indices (and symbols).
__device__ __forceinline__ void params_quad(const float* __restrict__ P, const float* __restrict__ y,
                                            const ThrTable& tt, uint8_t* __restrict__ idx,
                                            uint8_t* __restrict__ sym, int C, long e) {
  const long pos = e / C;
  const int c = (int)(e - pos * C);
  const v4f xs = ldg(reinterpret_cast<const v4f*>(P + pos * 2 * C + C + c));
  uint32_t iq = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) iq |= scale_index(xs[k], tt) << (8 * k);
  stg(reinterpret_cast<uint32_t*>(idx + e), iq);
  if (y) {
    const v4f mu = ldg(reinterpret_cast<const v4f*>(P + pos * 2 * C + c));
    const v4f yy = ldg(reinterpret_cast<const v4f*>(y + e));
    uint32_t sq = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float r = fminf(fmaxf(rintf(yy[k] - mu[k]), -32.f), 32.f);
      sq |= (uint32_t)((int)r + 32) << (8 * k);
    }
    stg(reinterpret_cast<uint32_t*>(sym + e), sq);
  }
}

__global__ void __launch_bounds__(256)
params_epilogue_kernel(const float* __restrict__ P, const float* __restrict__ y,
                       const float* __restrict__ thr, uint8_t* __restrict__ idx,
                       uint8_t* __restrict__ sym, long npos, int C) {
  __shared__ float s_thr[64];
  if (threadIdx.x < 64) s_thr[threadIdx.x] = thr[threadIdx.x];
  __syncthreads();
  const ThrTable tt = thr_table(s_thr);
  const long quads = npos * C / 4;
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < quads;
       q += (long)gridDim.x * blockDim.x)
    params_quad(P, y, tt, idx, sym, C, 4 * q);
}

__global__ void __launch_bounds__(256)
params_epilogue_batch_kernel(const EpiDesc* __restrict__ descs, const int2* __restrict__ work,
                             const float* __restrict__ thr) {
  __shared__ float s_thr[64];
  if (threadIdx.x < 64) s_thr[threadIdx.x] = thr[threadIdx.x];
  __syncthreads();
  const ThrTable tt = thr_table(s_thr);
  const int2 w = work[blockIdx.x];
  const EpiDesc d = descs[w.x];
  const long total = d.npos * d.C;
  const long e0 = (long)w.y * EPI_BLOCK_ELEMS;
  const long e1 = min(e0 + EPI_BLOCK_ELEMS, total);
  for (long e = e0 + 4 * threadIdx.x; e < e1; e += 4 * blockDim.x)
    params_quad(d.P, d.y, tt, d.idx, d.sym, d.C, e);
}

hipError_t launch_params_epilogue(const float* P, const float* y, const float* thr,
                                  uint8_t* idx, uint8_t* sym, long npos, int C,
                                  hipStream_t s) {
  if (C % 4) return hipErrorInvalidValue;
  const long quads = npos * C / 4;
  long blocks = (quads + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(params_epilogue_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     P, y, thr, idx, sym, npos, C);
  return hipGetLastError();
}

hipError_t launch_params_epilogue_batch(const EpiDesc* d, const int2* work, int nwork,
                                        const float* thr, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL(params_epilogue_batch_kernel, dim3(nwork), dim3(256), 0, s, d, work, thr);
  return hipGetLastError();
}

// --------------------------------------------------------- rANS encode ----
// One wave per block, one segment per half-wave.  A segment is processed in
// epochs of EP steps, last epoch first.  Each lane fetches its own symbols and
// table rows of the next epoch (one coalesced byte load per step across the
// half-wave) into registers while the current epoch is coded, so a step's
// table reads depend only on registers and run ahead of the state chain; the
// words a step pushes are placed with a ballot + popcount prefix into an LDS
// staging buffer and written to the segment slot with coalesced stores once
// per epoch.
constexpr int EP = 32;                 // steps per epoch
constexpr int EPB = EP * LANES;        // symbols per epoch and segment

struct EncSegLds {
  // at most one word per symbol, then (index EPB) the store target of lanes
  // that push no word
  uint16_t words[EPB + 2];
};
constexpr size_t ENC_TAB_BYTES = NSCALES * NSYM * 9;  // fc + magic (u32) + shift (u8)
constexpr size_t ENC_LDS_BYTES = ((ENC_TAB_BYTES + 15) & ~(size_t)15) + 2 * sizeof(EncSegLds);

// Symbol and index arrays handed to the coders carry CODER_PAD readable bytes
// past their end (more than one epoch), so the per-epoch prefetches never
// branch; positions past a segment's end are masked by the callers.

// Segment `seg` of the (z, y) stream pair of one chunk as a descriptor.
__device__ __forceinline__ EncSeg enc_seg_of(const EncStream& z, const EncStream& y,
                                             uint8_t* scratch, size_t slot_z, size_t slot_y,
                                             SegInfo* info, int seg) {
  const bool isz = seg < z.n_seg;
  const int si = isz ? seg : seg - z.n_seg;
  const EncStream& st = isz ? z : y;
  const long base = (long)si << st.seg_log2;
  EncSeg e;
  e.sym = st.sym + base;
  e.idx = st.idx ? st.idx + base : nullptr;
  e.slot = isz ? scratch + (size_t)si * slot_z
               : scratch + (size_t)z.n_seg * slot_z + (size_t)si * slot_y;
  e.info = info + seg;
  e.nsym = (uint32_t)min((long)1 << st.seg_log2, st.n - base);
  e.cap = 1u << st.seg_log2;
  e.fixed_row = (uint32_t)st.fixed_row;
  e.pad = 0;
  return e;
}

__global__ void __launch_bounds__(64)
rans_encode_kernel(Tables t, EncStream z, EncStream y, uint8_t* __restrict__ scratch,
                   size_t slot_z, size_t slot_y, SegInfo* __restrict__ info,
                   const EncSeg* __restrict__ segd, int nsegd) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint32_t* s_fc = reinterpret_cast<uint32_t*>(lds);
  uint32_t* s_mg = s_fc + NSCALES * NSYM;
  uint8_t* s_sh = reinterpret_cast<uint8_t*>(s_mg + NSCALES * NSYM);
  EncSegLds* segs = reinterpret_cast<EncSegLds*>(lds + ((ENC_TAB_BYTES + 15) & ~(size_t)15));
  // tables straight into LDS (in flight while the segment set-up runs)
  static_assert((NSCALES * NSYM * 4) % 16 == 0 && NSCALES * NSYM % 16 == 0, "table sizes");
  lds_fill16(s_fc, t.fc, NSCALES * NSYM * 4);
  lds_fill16(s_mg, t.magic, NSCALES * NSYM * 4);
  lds_fill16(s_sh, t.shift, NSCALES * NSYM);

  const int half = threadIdx.x >> 5;
  const int lane = threadIdx.x & 31;
  const int shsel = threadIdx.x & 32;
  const int nseg = segd ? nsegd : z.n_seg + y.n_seg;
  const int seg0 = blockIdx.x * 2;
  const int seg = seg0 + half;
  const bool active = seg < nseg;
  // an inactive half mirrors the pair's first segment with no symbols, so its
  // unconditional prefetches stay in bounds
  EncSeg me = segd ? segd[active ? seg : seg0]
                   : enc_seg_of(z, y, scratch, slot_z, slot_y, info, active ? seg : seg0);
  const uint32_t n_other = segd ? segd[seg0 + 1 < nseg ? seg0 + 1 : seg0].nsym
                                : enc_seg_of(z, y, scratch, slot_z, slot_y, info,
                                             seg0 + 1 < nseg ? seg0 + 1 : seg0).nsym;
  const uint32_t n_first = segd ? segd[seg0].nsym
                                : enc_seg_of(z, y, scratch, slot_z, slot_y, info, seg0).nsym;
  // both halves run the larger epoch count of the pair, so barriers stay uniform
  const int nep = (int)((max(n_first, n_other) + EPB - 1) / EPB);
  const uint8_t* __restrict__ sym = me.sym;
  const uint8_t* __restrict__ idxp = me.idx;
  const uint32_t fixed = min(me.fixed_row, 63u);
  const int nsym = active ? (int)me.nsym : 0;
  uint8_t* slot = me.slot;
  uint16_t* __restrict__ words = reinterpret_cast<uint16_t*>(slot + SEG_STATE_BYTES);
  EncSegLds& L = segs[half];
  const uint32_t cap = me.cap;
  uint32_t cursor = cap;
  uint32_t x = RANS_L;

  // raw symbols and rows of each step of the next epoch (used only in the
  // epoch after the one that issued the loads, so they have a whole epoch to
  // arrive)
  uint32_t sn[EP], kn[EP];
  const int nep_own = (nsym + EPB - 1) / EPB;
  auto prefetch = [&](int ep) {
    // epochs outside this segment's own [0, nep_own) and inactive halves
    // re-read epoch 0, which is in bounds
    const long pos = (ep >= 0 && ep < nep_own ? (long)ep * EPB : 0) + lane;
#pragma unroll
    for (int u = 0; u < EP; ++u) {
      sn[u] = ldg(sym + pos + u * LANES);
      kn[u] = ldg((idxp ? idxp : sym) + pos + u * LANES);
    }
  };

  prefetch(nep - 1);
  wait_vmcnt<0>();   // tables in LDS
  for (int ep = nep - 1; ep >= 0; --ep) {
    // table entry (row * NSYM + symbol) of each step of this epoch
    uint32_t ec[EP];
#pragma unroll
    for (int u = 0; u < EP; ++u) ec[u] = (idxp ? min(kn[u], 63u) : fixed) * NSYM + min(sn[u], 64u);
    prefetch(ep - 1);
    const uint32_t cstart = cursor;
#pragma unroll
    for (int u = EP - 1; u >= 0; --u) {
      const int j = ep * EPB + u * LANES + lane;
      const bool valid = active && j < nsym;
      const uint32_t e = ec[u];
      const uint32_t fc = s_fc[e];
      const uint32_t mg = s_mg[e];
      const uint32_t l = s_sh[e];
      const uint32_t f = fc & 0xFFFFu, c = fc >> 16;
      const bool emit = valid && x >= (f << 16);
      const unsigned long long bal = __ballot(emit);
      const uint32_t m = (uint32_t)(bal >> shsel);
      const uint32_t cnt = __popc(m);
      const uint32_t rank = __popc(m & ((1u << lane) - 1u));
      // word goes to slot position cursor - cnt + rank, staged in reverse;
      // lanes that push none store into the sink, so no branch is needed
      const uint32_t wi = emit ? cstart - 1u - (cursor - cnt + rank) : (uint32_t)EPB;
      L.words[wi] = (uint16_t)(x & 0xFFFFu);
      x = emit ? x >> 16 : x;
      cursor -= cnt;
      const uint32_t t1 = __umulhi(mg, x);
      const uint32_t q = (t1 + ((x - t1) >> (l > 0 ? 1u : 0u))) >> (l > 0 ? l - 1u : 0u);
      const uint32_t xu = (q << 16) + (x - q * f) + c;
      x = valid ? xu : x;
    }
    __syncthreads();
    // flush this epoch's words [cursor, cstart) with coalesced stores
    if (active) {
      const uint32_t nep_words = cstart - cursor;
      for (uint32_t i = lane; i < nep_words; i += LANES)
        stg(words + cursor + i, L.words[cstart - 1u - (cursor + i)]);
    }
    __syncthreads();
  }
  if (active) {
    stg(reinterpret_cast<uint32_t*>(slot) + lane, x);
    if (lane == 0) {
      SegInfo si;
      si.start_word = cursor;
      si.nwords = cap - cursor;
      *me.info = si;
    }
  }
}

static hipError_t set_enc_lds() {
  static std::atomic<uint32_t> done{0};
  return set_lds_limit_once(done, reinterpret_cast<const void*>(rans_encode_kernel), (int)ENC_LDS_BYTES);
}

hipError_t launch_rans_encode(const Tables& t, EncStream z, EncStream y, uint8_t* scratch,
                              size_t slot_bytes_z, size_t slot_bytes_y, SegInfo* info,
                              hipStream_t s) {
  const int nseg = z.n_seg + y.n_seg;
  if (nseg == 0) return hipSuccess;
  if (const hipError_t e = set_enc_lds()) return e;
  hipLaunchKernelGGL(rans_encode_kernel, dim3((nseg + 1) / 2), dim3(64), ENC_LDS_BYTES, s, t, z, y,
                     scratch, slot_bytes_z, slot_bytes_y, info, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_rans_encode_batch(const Tables& t, const EncSeg* segs, int nsegs, hipStream_t s) {
  if (nsegs <= 0) return hipSuccess;
  EncStream none{nullptr, nullptr, 0, 0, 5, 0};
  if (const hipError_t e = set_enc_lds()) return e;
  hipLaunchKernelGGL(rans_encode_kernel, dim3((nsegs + 1) / 2), dim3(64), ENC_LDS_BYTES, s, t, none,
                     none, nullptr, 0, 0, nullptr, segs, nsegs);
  return hipGetLastError();
}

// ------------------------------------------------------------- compact ----
__device__ __forceinline__ uint32_t seg_bytes_of(const SegInfo& si) {
  return (SEG_STATE_BYTES + 2u * si.nwords + 3u) & ~3u;
}

// Exclusive scan of per-thread run sums over a block (at most 1024 threads):
// returns the sum of the runs of all lower threads; *total gets the block's
// sum.  s_wave holds one entry per wave.
__device__ unsigned long long block_exclusive_scan(unsigned long long run, unsigned long long* s_wave,
                                                   unsigned long long* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long inc = run;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long v = __shfl_up(inc, o, 64);
    if (lane >= o) inc += v;
  }
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  unsigned long long before = 0, tot = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wave) before += s_wave[w];
    tot += s_wave[w];
  }
  __syncthreads();
  *total = tot;
  return before + inc - run;
}

// Container assembly, one block per segment.  Every block sums the byte
// counts of all segments and of those before its own (thread t owns the
// contiguous run [t K, t K + K), K = ceil(n_seg / blockDim); one block scan
// of the run sums, read back at the block's own segment), which gives the
// total size, checked against the capacity, and its segment's byte offset;
// block 0 also writes the header, the segment table and the size.  When the
// container does not fit the capacity nothing is written to the output.
// Then the block copies its segment: the 32 final states, then the words.
__global__ void __launch_bounds__(256)
compact_kernel(CompDesc d0, const CompDesc* __restrict__ descs, const int2* __restrict__ map) {
  __shared__ unsigned long long s_wave[4];
  __shared__ unsigned long long s_run_before[256];
  int b = blockIdx.x;
  CompDesc d;
  if (descs) {
    const int2 m = map[blockIdx.x];
    d = descs[m.x];
    b = m.y;
  } else {
    d = d0;
  }
  const SegInfo* __restrict__ info = d.info;
  const int n_seg_z = d.n_seg_z;
  const int nseg = n_seg_z + d.n_seg_y;
  if (b >= max(nseg, 1)) return;   // (an empty stream still gets block 0: the header)
  const size_t h0 = (d.with_header ? 28u : 0u) + 4u * (size_t)nseg;
  const int K = (nseg + (int)blockDim.x - 1) / (int)blockDim.x;
  const int r0 = min((int)threadIdx.x * K, nseg), r1 = min(r0 + K, nseg);
  unsigned long long run = 0;
  for (int i = r0; i < r1; ++i) run += seg_bytes_of(info[i]);
  unsigned long long all = 0;
  const unsigned long long before = block_exclusive_scan(run, s_wave, &all);
  s_run_before[threadIdx.x] = before;
  __syncthreads();
  const unsigned long long total = h0 + all;
  if (total > d.capacity) {
    if (b == 0 && threadIdx.x == 0) d.result[0] = total;
    return;
  }
  uint8_t* __restrict__ out = d.out;
  if (b == 0) {
    // the size, the segment table and the header
    if (threadIdx.x == 0) d.result[0] = total;
    uint32_t* tab = reinterpret_cast<uint32_t*>(out + (d.with_header ? 28 : 0));
    for (int i = r0; i < r1; ++i) tab[i] = seg_bytes_of(info[i]);
    if (d.with_header && threadIdx.x == 0) {
      const HeaderFields hf = d.hf;
      uint32_t* h = reinterpret_cast<uint32_t*>(out);
      h[0] = 0x31564655u;  // "UFV1"
      h[1] = (uint32_t)hf.T | ((uint32_t)hf.C << 16);
      h[2] = (uint32_t)hf.H | ((uint32_t)hf.W << 16);
      h[3] = (uint32_t)hf.seg_log2 | ((uint32_t)hf.seg_log2_z << 8) | ((uint32_t)hf.k_z << 16) |
             ((uint32_t)hf.flags << 24);
      h[4] = hf.model_tag;
      h[5] = (uint32_t)d.n_seg_z;
      h[6] = (uint32_t)d.n_seg_y;
    }
  }
  if (b >= nseg) return;
  // this segment's offset: the runs before its owner's, then the owner's
  // own segments before it (a handful of cache hits)
  const int owner = b / K;
  unsigned long long off = h0 + s_run_before[owner];
  for (int i = owner * K; i < b; ++i) off += seg_bytes_of(info[i]);
  if (threadIdx.x == 0) d.seg_off[b] = (uint32_t)off;
  const SegInfo si = info[b];
  const uint8_t* src = b < n_seg_z ? d.scratch_z + (size_t)b * d.slot_z
                                   : d.scratch_y + (size_t)(b - n_seg_z) * d.slot_y;
  uint8_t* dst = out + off;
  if (threadIdx.x < LANES)
    reinterpret_cast<uint32_t*>(dst)[threadIdx.x] = reinterpret_cast<const uint32_t*>(src)[threadIdx.x];
  // words in pairs: 4-byte stores (dst is 4-byte aligned: every segment's
  // byte count is a multiple of 4); an odd count ends with the zero pad word
  const uint16_t* ws = reinterpret_cast<const uint16_t*>(src + SEG_STATE_BYTES) + si.start_word;
  uint32_t* wd = reinterpret_cast<uint32_t*>(dst + SEG_STATE_BYTES);
  const uint32_t npairs = (si.nwords + 1u) >> 1;
  for (uint32_t k = threadIdx.x; k < npairs; k += blockDim.x) {
    const uint32_t lo = ws[2 * k];
    const uint32_t hi = 2 * k + 1 < si.nwords ? ws[2 * k + 1] : 0u;
    wd[k] = lo | (hi << 16);
  }
}

hipError_t launch_compact(const uint8_t* scratch, size_t slot_bytes_z, size_t slot_bytes_y,
                          const SegInfo* info, int n_seg_z, int n_seg_y, int with_header,
                          HeaderFields hf, uint8_t* out, size_t capacity,
                          unsigned long long* result, uint32_t* seg_off, hipStream_t s) {
  const int nseg = n_seg_z + n_seg_y;
  CompDesc d{};
  d.scratch_z = scratch;
  d.scratch_y = scratch + (size_t)n_seg_z * slot_bytes_z;
  d.slot_z = slot_bytes_z;
  d.slot_y = slot_bytes_y;
  d.info = info;
  d.n_seg_z = n_seg_z;
  d.n_seg_y = n_seg_y;
  d.with_header = with_header;
  d.hf = hf;
  d.out = out;
  d.capacity = capacity;
  d.result = result;
  d.seg_off = seg_off;
  hipLaunchKernelGGL(compact_kernel, dim3(nseg > 0 ? nseg : 1), dim3(256), 0, s, d, (const CompDesc*)nullptr,
                     (const int2*)nullptr);
  return hipGetLastError();
}

hipError_t launch_compact_batch(const CompDesc* d, int nchunks, const int2* map, int nblocks,
                                hipStream_t s) {
  if (nchunks <= 0 || nblocks <= 0) return hipSuccess;
  CompDesc none{};
  hipLaunchKernelGGL(compact_kernel, dim3(nblocks), dim3(256), 0, s, none, d, map);
  return hipGetLastError();
}

// --------------------------------------------------------------- parse ----
// One block per stream.  Thread t owns the contiguous run of segment-table
// entries [t K, t K + K), K = ceil(n_seg / blockDim): it sums its run (the
// only round of device-memory reads on the path; thread 0 also reads the
// header meanwhile), one block scan of the run sums gives every run's start
// offset, and a second pass over the run (cache hits) writes the offsets.
// A stream is rejected, with every offset 0xFFFFFFFF, for a header that does
// not match (ST_BAD_HEADER), or sizes below the 128 state bytes, not a
// multiple of 4, or not tiling the rest of the stream exactly (ST_CORRUPT).
__global__ void __launch_bounds__(256)
parse_kernel(ParseDesc d0, const ParseDesc* __restrict__ descs) {
  __shared__ unsigned long long s_wave[4];
  __shared__ int s_hdr_bad;
  const ParseDesc d = descs ? descs[blockIdx.x] : d0;
  const uint8_t* __restrict__ bs = d.bs;
  const size_t len = (size_t)d.len;
  const int with_header = d.with_header;
  const HeaderFields ex = d.ex;
  const int n_seg_z = d.n_seg_z, n_seg_y = d.n_seg_y;
  uint32_t* __restrict__ seg_off = d.seg_off;
  uint32_t* __restrict__ seg_len = d.seg_len;
  uint32_t* __restrict__ status = d.status;
  const int nseg = n_seg_z + n_seg_y;
  const size_t h0 = (with_header ? 28u : 0u) + 4u * (size_t)nseg;
  const bool short_stream = len < h0;   // the table itself is not there: nothing is read
  if (threadIdx.x == 0) {
    int bad = short_stream ? 1 : 0;
    if (!bad && with_header) {
      const uint32_t* h = reinterpret_cast<const uint32_t*>(bs);
      if (h[0] != 0x31564655u) bad = 1;
      if (h[1] != ((uint32_t)ex.T | ((uint32_t)ex.C << 16))) bad = 1;
      if (h[2] != ((uint32_t)ex.H | ((uint32_t)ex.W << 16))) bad = 1;
      if (h[3] != ((uint32_t)ex.seg_log2 | ((uint32_t)ex.seg_log2_z << 8) | ((uint32_t)ex.k_z << 16) |
                   ((uint32_t)ex.flags << 24)))
        bad = 1;
      if (h[4] != ex.model_tag || h[5] != (uint32_t)n_seg_z || h[6] != (uint32_t)n_seg_y) bad = 1;
    }
    s_hdr_bad = bad;
  }
  const uint32_t* tab = reinterpret_cast<const uint32_t*>(bs + (with_header ? 28 : 0));
  const int K = (nseg + (int)blockDim.x - 1) / (int)blockDim.x;
  const int r0 = min((int)threadIdx.x * K, nseg), r1 = min(r0 + K, nseg);
  unsigned long long run = 0;
  int badsz = 0;
  if (!short_stream)
    for (int i = r0; i < r1; ++i) {
      const uint32_t sb = tab[i];
      if (sb < (uint32_t)SEG_STATE_BYTES || (sb & 3u)) badsz = 1;
      run += sb;
    }
  const int anybad = __syncthreads_or(badsz);   // also publishes s_hdr_bad
  unsigned long long total = 0;
  unsigned long long off = h0 + block_exclusive_scan(run, s_wave, &total);   // this run's first offset
  const bool hdr_bad = s_hdr_bad != 0;
  const bool ok = !hdr_bad && !anybad && h0 + total == len;
  for (int i = r0; i < r1; ++i) {
    const uint32_t sb = ok ? tab[i] : 0u;
    seg_off[i] = ok ? (uint32_t)off : 0xFFFFFFFFu;
    seg_len[i] = sb;
    off += sb;
  }
  if (threadIdx.x == 0) {
    if (hdr_bad) atomicOr(status, ST_BAD_HEADER);
    else if (!ok) atomicOr(status, ST_CORRUPT);
  }
}

hipError_t launch_parse(const uint8_t* bs, size_t len, int with_header, HeaderFields expect,
                        int n_seg_z, int n_seg_y, uint32_t* seg_off, uint32_t* seg_len,
                        uint32_t* status, hipStream_t s) {
  ParseDesc d{};
  d.bs = bs;
  d.len = len;
  d.with_header = with_header;
  d.n_seg_z = n_seg_z;
  d.n_seg_y = n_seg_y;
  d.ex = expect;
  d.seg_off = seg_off;
  d.seg_len = seg_len;
  d.status = status;
  hipLaunchKernelGGL(parse_kernel, dim3(1), dim3(256), 0, s, d, (const ParseDesc*)nullptr);
  return hipGetLastError();
}

hipError_t launch_parse_batch(const ParseDesc* d, int nchunks, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  ParseDesc none{};
  hipLaunchKernelGGL(parse_kernel, dim3(nchunks), dim3(256), 0, s, none, d);
  return hipGetLastError();
}

// --------------------------------------------------------- rANS decode ----
// One wave per block, one segment per half-wave, epochs of EP steps.  Per
// segment the LDS holds a ring of RING words of the stream and the decoded
// symbols of one epoch; each lane holds the table rows of its steps of the
// current and the next epoch in registers.  Refill rule: at each epoch start
// the ring must hold the worst case of the epoch (EPB words past the cursor);
// 1024 more words are fetched in the background whenever fewer than two
// epochs' worth are buffered.  With at most EPB words consumed per epoch this
// keeps the invariant and never overwrites unread words (buffered - consumed
// < 3 EPB <= RING).  A step's dependent chain is three LDS reads: the bucket
// lookup, the symbol's frequency / cumulative pair and, on renormalisation,
// the next stream word.
constexpr int RING = 4096;   // words

struct DecSegLds {
  uint16_t ring[RING];
  uint8_t out[EPB];
};
constexpr size_t DEC_TAB_BYTES = NSCALES * NSYM * 4 + NSCALES * LUT_BUCKETS * 2 + NSCALES;
constexpr size_t DEC_LDS_BYTES = DEC_TAB_BYTES + 2 * sizeof(DecSegLds);

// Segment `si` of one decoded stream as a descriptor.
__device__ __forceinline__ DecSeg dec_seg_of(const uint8_t* bs, const uint32_t* seg_off,
                                             const uint32_t* seg_len, const DecStream& d,
                                             uint32_t* status, int si) {
  const long base = (long)si << d.seg_log2;
  DecSeg e;
  e.bs = bs;
  e.seg_off = seg_off + d.seg_base + si;
  e.seg_len = seg_len + d.seg_base + si;
  e.idx = d.idx ? d.idx + base : nullptr;
  e.out = d.sym_out + base;
  e.status = status;
  e.len = d.len;
  e.nsym = (uint32_t)min((long)1 << d.seg_log2, d.n - base);
  e.fixed_row = (uint32_t)d.fixed_row;
  return e;
}

// FIXED: every symbol of the stream uses the row fixed_row (no index array).
template <bool FIXED>
__global__ void __launch_bounds__(64)
rans_decode_kernel(Tables t, const uint8_t* __restrict__ bs0, const uint32_t* __restrict__ seg_off0,
                   const uint32_t* __restrict__ seg_len0, DecStream d, uint32_t* __restrict__ status0,
                   const DecSeg* __restrict__ segd, int nsegd) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint32_t* s_fc = reinterpret_cast<uint32_t*>(lds);
  uint16_t* s_lut = reinterpret_cast<uint16_t*>(lds + NSCALES * NSYM * 4);
  uint8_t* s_tail = reinterpret_cast<uint8_t*>(s_lut + NSCALES * LUT_BUCKETS);
  DecSegLds* segs = reinterpret_cast<DecSegLds*>(lds + DEC_TAB_BYTES);
  s_tail[threadIdx.x] = t.tail[threadIdx.x];
  if constexpr (!FIXED) {
    // all rows, straight into LDS (in flight while the segment set-up runs)
    lds_fill16(s_fc, t.fc, NSCALES * NSYM * 4);
    lds_fill16(s_lut, t.lut, NSCALES * LUT_BUCKETS * 2);
  }

  const int half = threadIdx.x >> 5;
  const int lane = threadIdx.x & 31;
  const int shsel = threadIdx.x & 32;
  const int nseg = segd ? nsegd : d.n_seg;
  const int seg0 = blockIdx.x * 2;
  const int sidx = seg0 + half;
  const bool active = sidx < nseg;
  // an inactive half mirrors the pair's first segment with no symbols
  const DecSeg me = segd ? segd[active ? sidx : seg0]
                         : dec_seg_of(bs0, seg_off0, seg_len0, d, status0, active ? sidx : seg0);
  const uint32_t n_first = segd ? segd[seg0].nsym
                                : dec_seg_of(bs0, seg_off0, seg_len0, d, status0, seg0).nsym;
  const int o1 = seg0 + 1 < nseg ? seg0 + 1 : seg0;
  const uint32_t n_other = segd ? segd[o1].nsym
                                : dec_seg_of(bs0, seg_off0, seg_len0, d, status0, o1).nsym;
  // both halves run the larger epoch count of the pair, so barriers stay uniform
  const int nep = (int)((max(n_first, n_other) + EPB - 1) / EPB);
  const uint8_t* __restrict__ bs = me.bs;
  uint32_t* __restrict__ status = me.status;
  const uint32_t off = active ? ldg(me.seg_off) : 0xFFFFFFFFu;
  const bool usable = off != 0xFFFFFFFFu;
  const int nsym = active ? (int)me.nsym : 0;
  const uint32_t slen = usable ? ldg(me.seg_len) : (uint32_t)SEG_STATE_BYTES;
  const uint32_t nw = (slen - SEG_STATE_BYTES) >> 1;    // words including a pad word
  const uint32_t* __restrict__ wdw =
      reinterpret_cast<const uint32_t*>(bs + (usable ? off : 0) + SEG_STATE_BYTES);
  // last readable dword of the stream, for clamped background fetches
  const long last_dw = ((long)(me.len & ~3ull) - 4) / 4;
  const long wdw0 = ((usable ? (long)off : 0) + SEG_STATE_BYTES) / 4;
  uint8_t* __restrict__ out = me.out;
  DecSegLds& L = segs[half];

  uint32_t x = usable ? ldg(reinterpret_cast<const uint32_t*>(bs + off) + lane) : RANS_L;
  uint32_t cursor = 0, loaded = 0;

  // background word fetch: 512 dwords (1024 words) starting at `loaded`
  uint32_t wreg[16];
  bool wpend = false;
  const uint32_t* __restrict__ bsdw = reinterpret_cast<const uint32_t*>(bs);
  auto fetch_words = [&]() {
    // unconditional loads clamped into the stream; dwords past the segment's
    // end are never consumed by a valid stream
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const long dw = wdw0 + (long)((loaded >> 1) + lane + 32u * i);
      wreg[i] = ldg(bsdw + min(dw, last_dw));
    }
    wpend = true;
  };
  auto commit_words = [&]() {
    if (wpend) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const uint32_t w = loaded + 2u * (lane + 32u * i);
        *reinterpret_cast<uint32_t*>(&L.ring[w & (RING - 1)]) = wreg[i];
      }
      loaded += 2u * 512u;
      wpend = false;
    }
  };
  // table row offset (row * NSYM) of each step of the next epoch; epochs past
  // this segment's own count re-read epoch 0 (in bounds)
  const uint32_t frow = min(me.fixed_row, 63u);
  if constexpr (FIXED) {
    // only the fixed rows of the pair's segments (the same row, normally)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t r = __shfl(frow, h * 32, 64);
      lds_fill4(s_fc + r * NSYM, t.fc + r * NSYM, NSYM);
      lds_fill16(s_lut + r * LUT_BUCKETS, t.lut + r * LUT_BUCKETS, LUT_BUCKETS * 2);
    }
  }
  uint32_t rn[EP];
  const int nep_own = (nsym + EPB - 1) / EPB;
  auto fetch_rows = [&](int ep) {
    // raw bytes; clamped only when the next epoch copies them, so the loads
    // have a whole epoch to arrive
    if constexpr (!FIXED) {
      const long pos = (long)(ep < nep_own ? ep : 0) * EPB + lane;
#pragma unroll
      for (int u = 0; u < EP; ++u) rn[u] = ldg(me.idx + pos + u * LANES);
    }
  };

  fetch_words();
  commit_words();
  fetch_rows(0);
  wait_vmcnt<0>();   // tables in LDS
  for (int ep = 0; ep < nep; ++ep) {
    uint32_t rc[EP];
#pragma unroll
    for (int u = 0; u < EP; ++u) rc[u] = FIXED ? frow : min(rn[u], 63u);
    commit_words();
    __syncthreads();
    fetch_rows(ep + 1);
    if (loaded - cursor < 2u * EPB) fetch_words();
#pragma unroll
    for (int u = 0; u < EP; ++u) {
      const int j = ep * EPB + u * LANES + lane;
      const bool valid = active && j < nsym;
      const uint32_t row = rc[u];
      const uint32_t slot = x & 0xFFFFu;
      const uint32_t e = s_lut[row * LUT_BUCKETS + (slot >> 8)];
      uint32_t sy = (e & 127u) - 1u + ((slot & 255u) >= ((e >> 7) & 255u) ? 1u : 0u);
      if (e & 0x8000u) {
        // slow bucket: frequency-1 tails in closed form (slot s is symbol s
        // on the left, 64 - (65535 - s) on the right), else a scan from s0
        const uint32_t tl = s_tail[row];
        const bool left = slot < tl, right = slot >= 65536u - tl;
        uint32_t sc = (e & 127u) - 1u;
        if (!left && !right)
          while (sc < NSYM - 1 && (s_fc[row * NSYM + sc + 1] >> 16) <= slot) ++sc;
        sy = left ? slot : (right ? slot - (65536u - NSYM) : sc);
      }
      const uint32_t fc = s_fc[row * NSYM + sy];
      const uint32_t f = fc & 0xFFFFu, c = fc >> 16;
      uint32_t xn = f * (x >> 16) + slot - c;
      const bool need = valid && xn < RANS_L;
      const unsigned long long bal = __ballot(need);
      const uint32_t m = (uint32_t)(bal >> shsel);
      const uint32_t cnt = __popc(m);
      const uint32_t rank = __popc(m & ((1u << lane) - 1u));
      // every lane reads (an in-bounds ring word; some lane of the wave
      // renormalises at nearly every step anyway), so no branch is needed
      const uint32_t wnext = L.ring[(cursor + rank) & (RING - 1)];
      xn = need ? ((xn << 16) | wnext) : xn;
      if (valid) x = xn;
      L.out[u * LANES + lane] = (uint8_t)sy;
      cursor += cnt;
    }
    __syncthreads();
    // decoded symbols of the epoch, 32 contiguous bytes per lane
    const long pos = (long)ep * EPB + lane * 32;
    if (active) {
      if (pos + 32 <= nsym) {
        stg(reinterpret_cast<v4u*>(out + pos), *reinterpret_cast<const v4u*>(&L.out[lane * 32]));
        stg(reinterpret_cast<v4u*>(out + pos + 16), *reinterpret_cast<const v4u*>(&L.out[lane * 32 + 16]));
      } else {
        for (int i = 0; i < 32; ++i)
          if (pos + i < nsym) stg(out + pos + i, (uint8_t)(usable ? L.out[lane * 32 + i] : 32));
      }
    }
  }
  if (!active) return;
  if (!usable) {
    if (lane == 0) atomicOr(status, ST_CORRUPT);
    return;
  }
  // integrity: every lane back at L, every word consumed (one zero pad word
  // may follow an odd count)
  bool bad = x != RANS_L;
  if (cursor > nw) {
    bad = true;
  } else if (cursor < nw) {
    const bool pad_ok = (cursor + 1u == nw) && (cursor & 1u) &&
                        reinterpret_cast<const uint16_t*>(wdw)[cursor] == 0;
    if (!pad_ok) bad = true;
  }
  const unsigned long long anybad = __ballot(bad);
  if (((uint32_t)(anybad >> shsel)) != 0u && lane == 0) atomicOr(status, ST_CORRUPT);
}

template <bool FIXED>
static hipError_t set_dec_lds() {
  static std::atomic<uint32_t> done{0};
  return set_lds_limit_once(done, reinterpret_cast<const void*>(rans_decode_kernel<FIXED>),
                            (int)DEC_LDS_BYTES);
}

hipError_t launch_rans_decode(const Tables& t, const uint8_t* bs, const uint32_t* seg_off,
                              const uint32_t* seg_len, DecStream d, uint32_t* status,
                              hipStream_t s) {
  if (d.n_seg == 0) return hipSuccess;
  const dim3 grid((d.n_seg + 1) / 2);
  hipError_t e;
  if (d.idx) {
    if ((e = set_dec_lds<false>()) != hipSuccess) return e;
    hipLaunchKernelGGL(rans_decode_kernel<false>, grid, dim3(64), DEC_LDS_BYTES, s, t, bs, seg_off,
                       seg_len, d, status, nullptr, 0);
  } else {
    if ((e = set_dec_lds<true>()) != hipSuccess) return e;
    hipLaunchKernelGGL(rans_decode_kernel<true>, grid, dim3(64), DEC_LDS_BYTES, s, t, bs, seg_off,
                       seg_len, d, status, nullptr, 0);
  }
  return hipGetLastError();
}

hipError_t launch_rans_decode_batch(const Tables& t, const DecSeg* segs, int nsegs, bool fixed,
                                    hipStream_t s) {
  if (nsegs <= 0) return hipSuccess;
  const dim3 grid((nsegs + 1) / 2);
  DecStream none{};
  hipError_t e;
  if (!fixed) {
    if ((e = set_dec_lds<false>()) != hipSuccess) return e;
    hipLaunchKernelGGL(rans_decode_kernel<false>, grid, dim3(64), DEC_LDS_BYTES, s, t, nullptr,
                       nullptr, nullptr, none, nullptr, segs, nsegs);
  } else {
    if ((e = set_dec_lds<true>()) != hipSuccess) return e;
    hipLaunchKernelGGL(rans_decode_kernel<true>, grid, dim3(64), DEC_LDS_BYTES, s, t, nullptr,
                       nullptr, nullptr, none, nullptr, segs, nsegs);
  }
  return hipGetLastError();
}

}  // namespace ufvc
