// Quadtree progressive means (Sec. 3.4 with Fig. 3 (a)): after the single
// pass has given every element's scale and base mean, partitions 1, 2 and 3
// of the latent get refined means one step at a time, each from the decoded
// residuals of the partitions before it.  No bit-stream interaction: the
// decoder runs these steps after its one-step rANS decode of all of r_hat,
// the encoder runs them before coding, quantising each partition with its
// refined mean.
//
// Partition of element (c, v, u): channel group g = 4c / C, spatial phase
// q = 2 (v & 1) + (u & 1), rank(q) = {0, 2, 3, 1}[q], part = (rank + g) & 3.
// Step k:  mu = mu_base + sum_{taps, c'} W_k[c][c'][tap] r_hat[c'][neighbour]
// over the neighbours' elements with part < k, written only on part k.
//
// Kernel shape.  Every output of step k at phase q belongs to the one channel
// group g = (k - rank(q)) & 3, so per phase the step is a stride-2 conv with
// C / 4 outputs; and because all outputs of a wave share the phase, the phase
// of every tap's input, hence which input channel groups are in partitions
// < k, is the same for the whole wave: the other groups' K steps are skipped
// (they would add exact zeros).  Step k has 9 k C / 64 K steps of 16
// channels, against 9 C / 16 for the full conv.
//
// One wave per unit of 16 output positions of one phase row x 16 output
// channels on v_mfma_f32_16x16x32_bf16: lane l holds position l % 16 (A row)
// and output channel l % 16 (B column); lane group gq = l / 16 holds input
// channels 8gq..8gq+7 of each 32-channel chunk.  The residuals (-32..32) are
// exact in bf16, and every float32 weight is the exact sum of three bf16
// parts (h + m + l, checked when the model is created), so each chunk runs
// three MFMAs on the same residuals, one per part: every product is exact
// and the sums are float32, as in a float32 conv.  K order: tap, chunk
// (ascending partition at C = 128), part, then the MFMA's own sum: fixed,
// so the encoder and the decoder compute the same means bit for bit.  Chunks
// of later partitions only are not visited; in a chunk that straddles two
// groups (C = 64) the lanes of a later group feed zeros.  Operands are read
// straight from device memory (the symbols are 4 MB at 1080p, L2-resident),
// six K steps ahead of the multiplications.
#include "ufvc_common.h"
#include "ufvc_means.h"

namespace ufvc {

typedef float mv4f __attribute__((ext_vector_type(4)));

__constant__ int kPhaseRank[4] = {0, 2, 3, 1};

typedef __bf16 mbf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int mv4u __attribute__((ext_vector_type(4)));
typedef unsigned int mv2u __attribute__((ext_vector_type(2)));

// NC: 32-channel chunks of C.  Returns the 16 x 16 block: acc[r] is position
// 4 gq + r of the unit, output channel n.  At C = 128 a chunk is one channel
// group, so only the K groups of earlier partitions are visited (9 K steps);
// at C = 64 a chunk holds two groups, every chunk is visited and lanes of a
// later group feed zeros.
template <int K, int NC>
__device__ __forceinline__ mv4f mean_mac(const MeanArgs& a, int qy, int qx, int vo, int uo, int gq,
                                         const __bf16* __restrict__ wl) {
  constexpr bool ONE_GROUP = NC == 4;                    // C = 128: 32 channels per group
  constexpr int NS = ONE_GROUP ? 9 * K : 9 * NC, D = 6;
  const int C = a.C;
  const int cg = C / 4;
  mv2u va[NS];
  mv4u vb[NS][3];
  bool ok[NS], act[NS];
  auto load = [&](int s) {
    const int tap = ONE_GROUP ? s / K : s / NC;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int iy = 2 * vo + qy + dy, ix = 2 * uo + qx + dx;
    const int rank = kPhaseRank[2 * ((qy + dy) & 1) + ((qx + dx) & 1)];
    // ONE_GROUP: the (s % K)-th earlier partition's group is chunk (m - rank) & 3
    const int ch = ONE_GROUP ? (((s % K) - rank) & 3) : s % NC;
    const int c0 = ch * 32 + 8 * gq;                    // this lane's 8 input channels
    const int part = (rank + c0 / cg) & 3;              // their partition at this tap
    ok[s] = uo < a.wo && iy >= 0 && ix >= 0 && iy < a.h && ix < a.w && part < K;
    const int p_first = (rank + (ch * 32) / cg) & 3, p_last = (rank + (ch * 32 + 31) / cg) & 3;
    act[s] = ONE_GROUP || p_first < K || p_last < K;
    const int cy = min(max(iy, 0), a.h - 1), cx = min(max(ix, 0), a.w - 1);
    va[s] = ldg(reinterpret_cast<const mv2u*>(a.sym + ((long)cy * a.w + cx) * C + c0));
#pragma unroll
    for (int p = 0; p < 3; ++p)
      vb[s][p] = ldg(reinterpret_cast<const mv4u*>(wl + (((long)(tap * 3 + p) * (C / 8) + c0 / 8) * C) * 8));
  };
#pragma unroll
  for (int s = 0; s < D && s < NS; ++s) load(s);
  mv4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (s + D < NS) load(s + D);
    // keep the prefetch ahead of this step's multiplications
    __builtin_amdgcn_sched_barrier(0);
    if (!act[s]) continue;
    mbf16x8 r;
    const mv2u v = ok[s] ? va[s] : mv2u{0x20202020u, 0x20202020u};   // symbol 32 = residual 0
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      r[j] = (__bf16)((float)(int)((v.x >> (8 * j)) & 0xFFu) - 32.f);
      r[4 + j] = (__bf16)((float)(int)((v.y >> (8 * j)) & 0xFFu) - 32.f);
    }
#pragma unroll
    for (int p = 0; p < 3; ++p)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(r, __builtin_bit_cast(mbf16x8, vb[s][p]), acc, 0, 0, 0);
  }
  return acc;
}

template <int K, int NC>
__global__ void __launch_bounds__(64) mean_step_kernel(MeanArgs a) {
  // grid: x = XCD-banded unit of (phase, phase row, 16 columns), y = 16-channel tile
  const int units_x = (a.wo + 15) / 16;
  const int nunits = 4 * a.ho * units_x;
  const int per = (nunits + 7) >> 3;
  const int unit = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (unit >= nunits) return;
  const int q = unit / (a.ho * units_x);
  const int rem = unit - q * a.ho * units_x;
  const int vo = rem / units_x;
  const int uo0 = (rem - vo * units_x) * 16;
  const int qy = q >> 1, qx = q & 1;
  const int lane = threadIdx.x & 63;
  const int gq = lane >> 4;
  const int cg = a.C / 4;
  const int gout = (K - kPhaseRank[q]) & 3;
  const int n = gout * cg + blockIdx.y * 16 + (lane & 15);
  const __bf16* __restrict__ wl = a.wk + (long)n * 8;
  const mv4f acc = mean_mac<K, NC>(a, qy, qx, vo, uo0 + (lane & 15), gq, wl);
  // acc[r]: position 4 gq + r of the unit, output channel n
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int uo = uo0 + 4 * gq + r;
    if (uo >= a.wo) continue;
    const long pos = (long)(2 * vo + qy) * a.w + 2 * uo + qx;
    float* pm = a.P + pos * 2 * a.C + n;
    const float mu = ldg(pm) + acc[r];
    stg(pm, mu);
    if (a.y) {
      const float d = ldg(a.y + pos * a.C + n) - mu;
      const float rq = fminf(fmaxf(rintf(d), -32.f), 32.f);
      stg(a.sym_out + pos * a.C + n, (uint8_t)((int)rq + 32));
    }
  }
}

template <int K>
static hipError_t launch_step(const MeanArgs& a, hipStream_t s) {
  const int units = 4 * a.ho * ((a.wo + 15) / 16);
  const dim3 grid(((units + 7) / 8) * 8, a.C / 64, 1);
  if (a.C == 128)
    hipLaunchKernelGGL((mean_step_kernel<K, 4>), grid, dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((mean_step_kernel<K, 2>), grid, dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mean_step(int k, const MeanArgs& a0, hipStream_t s) {
  if ((a0.C != 64 && a0.C != 128) || (a0.h & 1) || (a0.w & 1) || a0.h <= 0 || a0.w <= 0)
    return hipErrorInvalidValue;
  MeanArgs a = a0;
  a.ho = a.h / 2;
  a.wo = a.w / 2;
  a.wk = reinterpret_cast<const __bf16*>(reinterpret_cast<const unsigned char*>(a0.wpk) +
                                        (size_t)(k - 1) * a0.w_kstride);
  switch (k) {
    case 1: return launch_step<1>(a, s);
    case 2: return launch_step<2>(a, s);
    case 3: return launch_step<3>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ufvc
