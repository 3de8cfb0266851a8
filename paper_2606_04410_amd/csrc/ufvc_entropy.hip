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
//   prefix count; the encoder writes words backwards from the end of a
//   per-segment slot, the decoder reads them forwards through a two-chunk
//   register window with lane permutes.
// * compact / parse: container assembly with coalesced copies, and the
//   decoder's header validation and segment offset scan.
#include "ufvc_common.h"

namespace ufvc {

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
  // lut[b] = last symbol whose cumulative count is <= 256 b
  int sidx = 0;
  uint32_t c = 0;
  for (int b = 0; b < 256; ++b) {
    const uint32_t slot = (uint32_t)b << 8;
    while (sidx + 1 < NSYM && c + f[sidx] <= slot) { c += f[sidx]; ++sidx; }
    t.lut[k * 256 + b] = (uint8_t)sidx;
  }
}

hipError_t launch_build_tables(const Tables& t, hipStream_t s) {
  hipLaunchKernelGGL(build_tables_kernel, dim3(1), dim3(64), 0, s, t);
  return hipGetLastError();
}

// ------------------------------------------------------ params epilogue ----
__global__ void __launch_bounds__(256)
params_epilogue_kernel(const float* __restrict__ P, const float* __restrict__ y,
                       const float* __restrict__ thr, uint8_t* __restrict__ idx,
                       uint8_t* __restrict__ sym, long npos, int C) {
  __shared__ float s_thr[64];
  if (threadIdx.x < 64) s_thr[threadIdx.x] = thr[threadIdx.x];
  __syncthreads();
  const long total = npos * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const long pos = e / C;
    const int c = (int)(e - pos * C);
    const float xs = P[pos * 2 * C + C + c];
    const float sp = fmaxf(xs, 0.f) + log1pf(expf(-fabsf(xs)));
    const float sigma = fminf(fmaxf(sp, 0.11f), 64.f);
    // number of thresholds <= sigma (thr[63] = +inf)
    int k = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
      if (s_thr[k + step - 1] <= sigma) k += step;
    idx[e] = (uint8_t)k;
    if (y) {
      const float mu = P[pos * 2 * C + c];
      const float r = fminf(fmaxf(rintf(y[e] - mu), -32.f), 32.f);
      sym[e] = (uint8_t)((int)r + 32);
    }
  }
}

hipError_t launch_params_epilogue(const float* P, const float* y, const float* thr,
                                  uint8_t* idx, uint8_t* sym, long npos, int C,
                                  hipStream_t s) {
  const long total = npos * C;
  long blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(params_epilogue_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     P, y, thr, idx, sym, npos, C);
  return hipGetLastError();
}

// --------------------------------------------------------- rANS encode ----
constexpr int PF = 16;  // steps of symbols/indices fetched ahead

__global__ void __launch_bounds__(256)
rans_encode_kernel(Tables t, EncStream z, EncStream y, uint8_t* __restrict__ scratch,
                   size_t slot_z, size_t slot_y, SegInfo* __restrict__ info) {
  __shared__ uint32_t s_fc[NSCALES * NSYM];
  __shared__ uint32_t s_mg[NSCALES * NSYM];
  __shared__ uint8_t s_sh[NSCALES * NSYM];
  for (int i = threadIdx.x; i < NSCALES * NSYM; i += blockDim.x) {
    s_fc[i] = t.fc[i];
    s_mg[i] = t.magic[i];
    s_sh[i] = t.shift[i];
  }
  __syncthreads();

  const int half = threadIdx.x >> 5;
  const int lane = threadIdx.x & 31;
  const int seg = blockIdx.x * 8 + half;
  if (seg >= z.n_seg + y.n_seg) return;
  const bool isz = seg < z.n_seg;
  const int sidx = isz ? seg : seg - z.n_seg;
  const uint8_t* __restrict__ sym = isz ? z.sym : y.sym;
  const uint8_t* __restrict__ idxp = isz ? z.idx : y.idx;
  const int fixed = isz ? z.fixed_row : y.fixed_row;
  const int sl = isz ? z.seg_log2 : y.seg_log2;
  const long n = isz ? z.n : y.n;
  const long base = (long)sidx << sl;
  const int nsym = (int)min((long)1 << sl, n - base);
  const int steps = (nsym + LANES - 1) / LANES;
  uint8_t* slot = isz ? scratch + (size_t)sidx * slot_z
                      : scratch + (size_t)z.n_seg * slot_z + (size_t)sidx * slot_y;
  uint16_t* words = reinterpret_cast<uint16_t*>(slot + SEG_STATE_BYTES);
  const uint32_t cap = 1u << sl;
  uint32_t cursor = cap;
  uint32_t x = RANS_L;
  const int shsel = threadIdx.x & 32;

  uint8_t cs[PF], ci[PF], ns[PF], ni[PF];
  auto fetch = [&](int blk, uint8_t* ds, uint8_t* di) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int j = (blk * PF + u) * LANES + lane;
      const bool v = blk >= 0 && j < nsym;
      ds[u] = v ? sym[base + j] : 0;
      di[u] = v ? (idxp ? idxp[base + j] : (uint8_t)fixed) : 0;
    }
  };
  const int nblk = (steps + PF - 1) / PF;
  fetch(nblk - 1, cs, ci);
  for (int blk = nblk - 1; blk >= 0; --blk) {
    fetch(blk - 1, ns, ni);
#pragma unroll
    for (int u = PF - 1; u >= 0; --u) {
      const int step = blk * PF + u;
      if (step < steps) {
        const int j = step * LANES + lane;
        const bool valid = j < nsym;
        const int e = (int)min((uint32_t)ci[u], 63u) * NSYM + (int)min((uint32_t)cs[u], 64u);
        const uint32_t fc = s_fc[e];
        const uint32_t f = fc & 0xFFFFu, c = fc >> 16;
        const bool emit = valid && x >= (f << 16);
        const unsigned long long bal = __ballot(emit);
        const uint32_t m = (uint32_t)(bal >> shsel);
        const uint32_t cnt = __popc(m);
        const uint32_t rank = __popc(m & ((1u << lane) - 1u));
        if (emit) {
          words[cursor - cnt + rank] = (uint16_t)(x & 0xFFFFu);
          x >>= 16;
        }
        cursor -= cnt;
        if (valid) {
          const uint32_t mg = s_mg[e];
          const uint32_t l = s_sh[e];
          const uint32_t t1 = __umulhi(mg, x);
          const uint32_t q = (t1 + ((x - t1) >> (l > 0 ? 1u : 0u))) >> (l > 0 ? l - 1u : 0u);
          x = (q << 16) + (x - q * f) + c;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) { cs[u] = ns[u]; ci[u] = ni[u]; }
  }
  reinterpret_cast<uint32_t*>(slot)[lane] = x;
  if (lane == 0) {
    SegInfo si;
    si.start_word = cursor;
    si.nwords = cap - cursor;
    info[seg] = si;
  }
}

hipError_t launch_rans_encode(const Tables& t, EncStream z, EncStream y, uint8_t* scratch,
                              size_t slot_bytes_z, size_t slot_bytes_y, SegInfo* info,
                              hipStream_t s) {
  const int nseg = z.n_seg + y.n_seg;
  if (nseg == 0) return hipSuccess;
  hipLaunchKernelGGL(rans_encode_kernel, dim3((nseg + 7) / 8), dim3(256), 0, s, t, z, y,
                     scratch, slot_bytes_z, slot_bytes_y, info);
  return hipGetLastError();
}

// ------------------------------------------------------------- compact ----
__device__ __forceinline__ uint32_t seg_bytes_of(const SegInfo& si) {
  return (SEG_STATE_BYTES + 2u * si.nwords + 3u) & ~3u;
}

__device__ unsigned long long block_sum(unsigned long long v, unsigned long long* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  unsigned long long tot = 0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) tot += red[i];
  __syncthreads();
  return tot;
}

__global__ void __launch_bounds__(256)
compact_kernel(const uint8_t* __restrict__ scratch, size_t slot_z, size_t slot_y,
               const SegInfo* __restrict__ info, int n_seg_z, int n_seg_y, int with_header,
               HeaderFields hf, uint8_t* __restrict__ out, size_t capacity,
               unsigned long long* __restrict__ result) {
  __shared__ unsigned long long red[8];
  const int nseg = n_seg_z + n_seg_y;
  const int b = blockIdx.x;
  const size_t h0 = (with_header ? 28u : 0u) + 4u * (size_t)nseg;
  unsigned long long before = 0, all = 0;
  for (int i = threadIdx.x; i < nseg; i += blockDim.x) {
    const unsigned long long sb = seg_bytes_of(info[i]);
    all += sb;
    if (i < b) before += sb;
  }
  before = block_sum(before, red);
  all = block_sum(all, red);
  const unsigned long long total = h0 + all;
  if (b == 0 && threadIdx.x == 0) result[0] = total;
  if (total > capacity) return;
  if (b == 0) {
    if (with_header && threadIdx.x == 0) {
      uint32_t* h = reinterpret_cast<uint32_t*>(out);
      h[0] = 0x31564655u;  // "UFV1"
      h[1] = (uint32_t)hf.T | ((uint32_t)hf.C << 16);
      h[2] = (uint32_t)hf.H | ((uint32_t)hf.W << 16);
      h[3] = (uint32_t)hf.seg_log2 | ((uint32_t)hf.seg_log2_z << 8) | ((uint32_t)hf.k_z << 16);
      h[4] = hf.model_tag;
      h[5] = (uint32_t)n_seg_z;
      h[6] = (uint32_t)n_seg_y;
    }
    uint32_t* tab = reinterpret_cast<uint32_t*>(out + (with_header ? 28 : 0));
    for (int i = threadIdx.x; i < nseg; i += blockDim.x) tab[i] = seg_bytes_of(info[i]);
  }
  if (b >= nseg) return;
  const SegInfo si = info[b];
  const uint8_t* src = b < n_seg_z ? scratch + (size_t)b * slot_z
                                   : scratch + (size_t)n_seg_z * slot_z + (size_t)(b - n_seg_z) * slot_y;
  uint8_t* dst = out + h0 + before;
  if (threadIdx.x < LANES)
    reinterpret_cast<uint32_t*>(dst)[threadIdx.x] = reinterpret_cast<const uint32_t*>(src)[threadIdx.x];
  const uint16_t* ws = reinterpret_cast<const uint16_t*>(src + SEG_STATE_BYTES) + si.start_word;
  uint16_t* wd = reinterpret_cast<uint16_t*>(dst + SEG_STATE_BYTES);
  for (uint32_t i = threadIdx.x; i < si.nwords; i += blockDim.x) wd[i] = ws[i];
  if ((si.nwords & 1u) && threadIdx.x == 0) wd[si.nwords] = 0;
}

hipError_t launch_compact(const uint8_t* scratch, size_t slot_bytes_z, size_t slot_bytes_y,
                          const SegInfo* info, int n_seg_z, int n_seg_y, int with_header,
                          HeaderFields hf, uint8_t* out, size_t capacity,
                          unsigned long long* result, hipStream_t s) {
  const int nseg = n_seg_z + n_seg_y;
  hipLaunchKernelGGL(compact_kernel, dim3(nseg > 0 ? nseg : 1), dim3(256), 0, s, scratch,
                     slot_bytes_z, slot_bytes_y, info, n_seg_z, n_seg_y, with_header, hf, out,
                     capacity, result);
  return hipGetLastError();
}

// --------------------------------------------------------------- parse ----
__global__ void __launch_bounds__(256)
parse_kernel(const uint8_t* __restrict__ bs, size_t len, int with_header, HeaderFields ex,
             int n_seg_z, int n_seg_y, uint32_t* __restrict__ seg_off,
             uint32_t* __restrict__ seg_len, uint32_t* __restrict__ status) {
  __shared__ unsigned long long red[8];
  __shared__ int s_bad;
  const int nseg = n_seg_z + n_seg_y;
  const size_t h0 = (with_header ? 28u : 0u) + 4u * (size_t)nseg;
  if (threadIdx.x == 0) {
    int bad = 0;
    if (len < h0) bad = 1;
    if (!bad && with_header) {
      const uint32_t* h = reinterpret_cast<const uint32_t*>(bs);
      if (h[0] != 0x31564655u) bad = 1;
      if (h[1] != ((uint32_t)ex.T | ((uint32_t)ex.C << 16))) bad = 1;
      if (h[2] != ((uint32_t)ex.H | ((uint32_t)ex.W << 16))) bad = 1;
      if (h[3] != ((uint32_t)ex.seg_log2 | ((uint32_t)ex.seg_log2_z << 8) | ((uint32_t)ex.k_z << 16)))
        bad = 1;
      if (h[4] != ex.model_tag || h[5] != (uint32_t)n_seg_z || h[6] != (uint32_t)n_seg_y) bad = 1;
    }
    s_bad = bad;
  }
  __syncthreads();
  if (s_bad) {
    for (int i = threadIdx.x; i < nseg; i += blockDim.x) { seg_off[i] = 0xFFFFFFFFu; seg_len[i] = 0; }
    if (threadIdx.x == 0) atomicOr(status, ST_BAD_HEADER);
    return;
  }
  const uint32_t* tab = reinterpret_cast<const uint32_t*>(bs + (with_header ? 28 : 0));
  // sizes must be >= 128 and multiples of 4, and must tile the rest exactly
  unsigned long long tot = 0;
  int badsz = 0;
  for (int i = threadIdx.x; i < nseg; i += blockDim.x) {
    const uint32_t sb = tab[i];
    if (sb < (uint32_t)SEG_STATE_BYTES || (sb & 3u)) badsz = 1;
    tot += sb;
  }
  tot = block_sum(tot, red);
  const unsigned long long nbad = block_sum((unsigned long long)badsz, red);
  const bool ok = nbad == 0 && h0 + tot == len;
  // exclusive scan, 256 entries at a time
  unsigned long long carry = h0;
  __shared__ unsigned long long sc[256];
  for (int c0 = 0; c0 < nseg; c0 += 256) {
    const int i = c0 + threadIdx.x;
    const unsigned long long v = (i < nseg) ? tab[i] : 0ull;
    sc[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const unsigned long long add = threadIdx.x >= o ? sc[threadIdx.x - o] : 0ull;
      __syncthreads();
      sc[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nseg) {
      seg_off[i] = ok ? (uint32_t)(carry + sc[threadIdx.x] - v) : 0xFFFFFFFFu;
      seg_len[i] = ok ? (uint32_t)v : 0u;
    }
    const unsigned long long last = sc[255];
    __syncthreads();
    carry += last;
  }
  if (!ok && threadIdx.x == 0) atomicOr(status, ST_CORRUPT);
}

hipError_t launch_parse(const uint8_t* bs, size_t len, int with_header, HeaderFields expect,
                        int n_seg_z, int n_seg_y, uint32_t* seg_off, uint32_t* seg_len,
                        uint32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(parse_kernel, dim3(1), dim3(256), 0, s, bs, len, with_header, expect,
                     n_seg_z, n_seg_y, seg_off, seg_len, status);
  return hipGetLastError();
}

// --------------------------------------------------------- rANS decode ----
__global__ void __launch_bounds__(256)
rans_decode_kernel(Tables t, const uint8_t* __restrict__ bs, const uint32_t* __restrict__ seg_off,
                   const uint32_t* __restrict__ seg_len, DecStream d, uint32_t* __restrict__ status) {
  __shared__ uint32_t s_fc[NSCALES * NSYM];
  __shared__ uint8_t s_lut[NSCALES * 256];
  for (int i = threadIdx.x; i < NSCALES * NSYM; i += blockDim.x) s_fc[i] = t.fc[i];
  for (int i = threadIdx.x; i < NSCALES * 256; i += blockDim.x) s_lut[i] = t.lut[i];
  __syncthreads();

  const int half = threadIdx.x >> 5;
  const int lane = threadIdx.x & 31;
  const int sidx = blockIdx.x * 8 + half;
  if (sidx >= d.n_seg) return;
  const long base = (long)sidx << d.seg_log2;
  const int nsym = (int)min((long)1 << d.seg_log2, d.n - base);
  const int steps = (nsym + LANES - 1) / LANES;
  const uint32_t off = seg_off[d.seg_base + sidx];
  const uint32_t slen = seg_len[d.seg_base + sidx];
  uint8_t* __restrict__ out = d.sym_out + base;
  if (off == 0xFFFFFFFFu) {
    for (int j = lane; j < nsym; j += LANES) out[j] = 32;
    return;
  }
  uint32_t x = reinterpret_cast<const uint32_t*>(bs + off)[lane];
  const uint16_t* __restrict__ words = reinterpret_cast<const uint16_t*>(bs + off + SEG_STATE_BYTES);
  const uint32_t nw = (slen - SEG_STATE_BYTES) >> 1;
  uint32_t wbase = 0, cursor = 0;
  uint32_t w0 = lane < nw ? words[lane] : 0u;
  uint32_t w1 = (uint32_t)(LANES + lane) < nw ? words[LANES + lane] : 0u;
  const int shsel = threadIdx.x & 32;

  uint8_t ci[PF], ni[PF];
  auto fetch = [&](int blk, uint8_t* di) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int j = (blk * PF + u) * LANES + lane;
      const bool v = j < nsym;
      di[u] = v ? (d.idx ? d.idx[base + j] : (uint8_t)d.fixed_row) : 0;
    }
  };
  const int nblk = (steps + PF - 1) / PF;
  fetch(0, ci);
  for (int blk = 0; blk < nblk; ++blk) {
    fetch(blk + 1, ni);
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int step = blk * PF + u;
      if (step < steps) {
        const int j = step * LANES + lane;
        const bool valid = j < nsym;
        const int row = (int)min((uint32_t)ci[u], 63u);
        const int rowb = row * NSYM;
        const uint32_t slot = x & 0xFFFFu;
        uint32_t sy = s_lut[row * 256 + (slot >> 8)];
        uint32_t fc = s_fc[rowb + sy];
        while (sy < NSYM - 1) {
          const uint32_t nfc = s_fc[rowb + sy + 1];
          if ((nfc >> 16) > slot) break;
          ++sy;
          fc = nfc;
        }
        const uint32_t f = fc & 0xFFFFu, c = fc >> 16;
        uint32_t xn = f * (x >> 16) + slot - c;
        const bool need = valid && xn < RANS_L;
        const unsigned long long bal = __ballot(need);
        const uint32_t m = (uint32_t)(bal >> shsel);
        const uint32_t cnt = __popc(m);
        const uint32_t rank = __popc(m & ((1u << lane) - 1u));
        const uint32_t widx = cursor + rank - wbase;  // < 64 by the window invariant
        const int src = shsel + (int)(widx & 31u);
        const uint32_t v0 = __shfl(w0, src, 64);
        const uint32_t v1 = __shfl(w1, src, 64);
        if (need) xn = (xn << 16) | (widx < 32u ? v0 : v1);
        if (valid) {
          x = xn;
          out[j] = (uint8_t)sy;
        }
        cursor += cnt;
        if (cursor - wbase >= 32u) {
          wbase += 32u;
          w0 = w1;
          const uint32_t wi = wbase + LANES + lane;
          w1 = wi < nw ? words[wi] : 0u;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) ci[u] = ni[u];
  }
  // integrity: every lane back at L, every word consumed (one zero pad word
  // may follow an odd count)
  bool bad = x != RANS_L;
  if (cursor > nw) bad = true;
  else if (cursor < nw) {
    const bool pad_ok = (cursor + 1u == nw) && (cursor & 1u) && words[cursor] == 0;
    if (!pad_ok) bad = true;
  }
  const unsigned long long anybad = __ballot(bad);
  if (((uint32_t)(anybad >> shsel)) != 0u && lane == 0) atomicOr(status, ST_CORRUPT);
}

hipError_t launch_rans_decode(const Tables& t, const uint8_t* bs, const uint32_t* seg_off,
                              const uint32_t* seg_len, DecStream d, uint32_t* status,
                              hipStream_t s) {
  if (d.n_seg == 0) return hipSuccess;
  hipLaunchKernelGGL(rans_decode_kernel, dim3((d.n_seg + 7) / 8), dim3(256), 0, s, t, bs,
                     seg_off, seg_len, d, status);
  return hipGetLastError();
}

}  // namespace ufvc
