// The DC block (supplementary material: the depth-wise convolution block of
// DCVC-RT, the one primitive the paper's modules are built from), fused into
// one kernel:
//
//   t  = relu(pw1 x)          d  = dw3x3 t          x1 = x + pw2 d
//   u  = relu(pw3 x1)         y  = x1 + pw4 u
//
// pw1, pw2: C -> C; pw3: C -> 2C; pw4: 2C -> C (1 x 1); dw: one 3 x 3 filter
// per channel, zero padding.  No biases.  bf16 operands on the matrix cores
// with float32 accumulation; t, d, x1 (as pw3's input) and u are rounded to
// bf16 where they are staged, the residual sums stay float32 until the
// output is rounded to bf16.
//
// A workgroup (8 waves) owns an 8 x 16 tile of positions.  It reads the tile
// and its one-position halo (10 x 18) once from HBM into LDS, runs all five
// steps out of LDS, and writes the 8 x 16 outputs once: HBM traffic is the
// input and output tensors only (plus the L2-resident weights), where the
// five steps as separate kernels would move the C- and 2C-channel
// intermediates through HBM.  pw1 runs on the halo positions as well (the
// depth-wise step needs them), 180 of 128 positions.
//
// The point-wise steps are GEMMs with weights as the MFMA's first operand
// (32 output channels per block, straight from L2: rows of the (out, in)
// matrix are 16-byte K chunks) and 32 positions as its second, read from
// LDS.  LDS tensors are chunk-major, [C / 8][rows][8 bf16], so the 32 lanes
// reading one 16-byte chunk of 32 consecutive positions hit distinct banks,
// and lanes l and l + 32 (the next chunk, same rows) hit the same ones.
// Lane l ends with position l % 32 and channels 8 (r / 4) + 4 (l / 32) + r % 4
// of its block; one v_permlane32_swap per register pair turns that into two
// runs of 8 consecutive channels per lane, written as 16-byte chunks.
#include "../../include/ufvc.h"

#include <atomic>
#include <new>
#include <vector>

#include "ufvc_common.h"

namespace ufvc {

namespace dcb {
constexpr int TW = 16, HW = TW + 2;
constexpr int NT = 512;         // 8 waves
// Tile of TH x 16 positions: halo rows padded to whole 32-position blocks.
template <int TH>
struct Tile {
  static constexpr int HH = TH + 2;
  static constexpr int HROWS = (HH * HW + 31) / 32 * 32;
  static constexpr int IROWS = TH * TW;
};
}  // namespace dcb

typedef unsigned int dv4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dv4u lds_ld16(const unsigned char* p) {
  return *reinterpret_cast<const dv4u*>(p);
}
__device__ __forceinline__ void lds_st16(unsigned char* p, dv4u v) {
  *reinterpret_cast<dv4u*>(p) = v;
}

// Offset of chunk `ch` of row `row` in a chunk-major LDS tensor of `rows` rows.
__device__ __forceinline__ int cm_off(int ch, int row, int rows) { return (ch * rows + row) * 16; }

// Swaps registers r and r + 4 (r % 8 < 4) between lane halves: lane l < 32
// then holds channels 0-7 (v[0..7]) and 16-23 (v[8..15]) of the block, lane
// l + 32 channels 8-15 and 24-31.
__device__ __forceinline__ void halves_to_runs(f32x16& v) {
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[8 * h + r]),
                                                      __float_as_uint(v[8 * h + r + 4]), false, false);
      v[8 * h + r] = __uint_as_float(p[0]);
      v[8 * h + r + 4] = __uint_as_float(p[1]);
    }
}

__device__ __forceinline__ dv4u pack8(const float* o) {
  bf16x8 b;
#pragma unroll
  for (int k = 0; k < 8; ++k) b[k] = (__bf16)o[k];
  return __builtin_bit_cast(dv4u, b);
}

__device__ __forceinline__ void unpack8(dv4u v, float* o) {
  const bf16x8 b = __builtin_bit_cast(bf16x8, v);
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = (float)b[k];
}

// Weight fragments of one 32-output-channel block of a point-wise step:
// lane l holds row cb*32 + l%32 of the (out, in) bf16 matrix W (row pitch
// K), K chunks 2 ks + l/32.  Loaded once per step and reused for every
// position block of the wave.
template <int K>
struct WFrag {
  dv4u f[K / 16];
};
template <int K>
__device__ __forceinline__ WFrag<K> load_wfrag(const __bf16* __restrict__ W, int cb, int lane) {
  WFrag<K> w;
  const __bf16* wrow = W + (long)(cb * 32 + (lane & 31)) * K + 8 * (lane >> 5);
#pragma unroll
  for (int ks = 0; ks < K / 16; ++ks) w.f[ks] = ldg(reinterpret_cast<const dv4u*>(wrow + ks * 16));
  return w;
}

// One 32 x 32 block: W block x Act[pb*32 .. +32][0..K), Act chunk-major with
// `rows` rows.
template <int K>
__device__ __forceinline__ f32x16 pw_block(const WFrag<K>& w, const unsigned char* act, int rows,
                                           int pb, int lane) {
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  const int kh = lane >> 5;
  const int row = pb * 32 + (lane & 31);
#pragma unroll
  for (int ks = 0; ks < K / 16; ++ks) {
    const dv4u xf = lds_ld16(act + cm_off(2 * ks + kh, row, rows));
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, w.f[ks]),
                                                  __builtin_bit_cast(bf16x8, xf), acc, 0, 0, 0);
  }
  return acc;
}

template <int C, int TH>
__global__ void __launch_bounds__(dcb::NT) dc_block_kernel(DcBlockArgs a) {
  const float* __restrict__ dwt = a.dw;
  using namespace dcb;
  constexpr int HH = Tile<TH>::HH, HROWS = Tile<TH>::HROWS, IROWS = Tile<TH>::IROWS;
  constexpr int NCH = C / 8;          // 16-byte chunks per position
  constexpr int NCB = C / 32;         // 32-channel blocks of C
  constexpr int X_BYTES = NCH * HROWS * 16;
  constexpr int D_BYTES = NCH * IROWS * 16;
  static_assert(2 * NCH * IROWS * 16 <= X_BYTES + D_BYTES, "u must fit the x and d regions");
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  unsigned char* sx = lds;                      // x, halo rows      (later u, 2C channels)
  unsigned char* sd = lds + X_BYTES;            // d, inner rows
  unsigned char* st = lds + X_BYTES + D_BYTES;  // t, halo rows      (later x1 as bf16)
  unsigned char* su = lds;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_x = (a.w + TW - 1) / TW;
  const int ntiles = tiles_x * ((a.h + TH - 1) / TH);
  // XCD-aware order: each of the 8 XCDs takes a contiguous band of tiles
  const int per = (ntiles + 7) >> 3;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntiles) return;
  const int ty0 = (tile / tiles_x) * TH, tx0 = (tile % tiles_x) * TW;
  const __bf16* __restrict__ x = a.x;

  // Every wave keeps one 32-channel block per step (8 waves, NCB | 8), so
  // its weight fragments are loaded once per step, the next step's while
  // the current one runs (pw1's and pw2's with the tile).
  const int cbw = wave % NCB;          // C-output steps (pw1, pw2, pw4)
  const int cb3 = wave % (2 * NCB);    // pw3 (2C outputs)
  WFrag<C> w1 = load_wfrag<C>(a.pw1, cbw, lane);
  WFrag<C> w2 = load_wfrag<C>(a.pw2, cbw, lane);

  // 1. x tile and halo -> LDS (zero outside the image and in the padding
  //    rows).  Sixteen consecutive threads take one chunk of sixteen
  //    consecutive halo rows (distinct LDS banks).  Every load of the tile is
  //    issued before the first LDS store, so their latencies overlap.
  {
    constexpr int NLD = NCH * HROWS / NT;
    static_assert(NCH * HROWS % NT == 0, "whole load rounds");
    dv4u v[NLD];
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = tid + k * NT;
      const int grp = i / (16 * NCH), rem = i - grp * 16 * NCH;
      const int ch = rem >> 4, row = grp * 16 + (rem & 15);
      const int gy = ty0 + row / HW - 1, gx = tx0 + row % HW - 1;
      const bool in = row < HH * HW && gy >= 0 && gy < a.h && gx >= 0 && gx < a.w;
      const int cy = min(max(gy, 0), a.h - 1), cx = min(max(gx, 0), a.w - 1);
      v[k] = ldg(reinterpret_cast<const dv4u*>(x + ((long)cy * a.w + cx) * C + ch * 8));
      if (!in) v[k] = dv4u{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = tid + k * NT;
      const int grp = i / (16 * NCH), rem = i - grp * 16 * NCH;
      lds_st16(sx + cm_off(rem >> 4, grp * 16 + (rem & 15), HROWS), v[k]);
    }
  }
  __syncthreads();

  const int cofs = (lane >> 5) * 8;   // first channel of this lane's runs within 16
  const int prow = lane & 31;

  // 2. t = relu(pw1 x) on all halo rows (zero rows stay zero: no bias).
  for (int b = wave; b < NCB * (HROWS / 32); b += NT / 64) {
    const int cb = cbw, pb = b / NCB;
    f32x16 v = pw_block<C>(w1, sx, HROWS, pb, lane);
    halves_to_runs(v);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float o[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) o[k] = fmaxf(v[8 * h + k], 0.f);
      const int ch = (cb * 32 + h * 16 + cofs) / 8;
      lds_st16(st + cm_off(ch, pb * 32 + prow, HROWS), pack8(o));
    }
  }
  __syncthreads();

  // 3. d = dw3x3 t on the inner rows: thread -> one inner position, chunks
  //    (tid / 128) + 4 j (wave-uniform, so the taps' weights are scalar loads).
  {
    const int p = tid & (IROWS - 1);
    const int pr = p / TW, pc = p % TW;
    // the chunk is the same for the whole wave: its taps are scalar loads
    for (int ch = __builtin_amdgcn_readfirstlane(tid / IROWS); ch < NCH; ch += NT / IROWS) {
      float acc[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] = 0.f;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int hrow = (pr + tap / 3) * HW + pc + tap % 3;
        float tv[8];
        unpack8(lds_ld16(st + cm_off(ch, hrow, HROWS)), tv);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = fmaf(dwt[(ch * 8 + k) * 9 + tap], tv[k], acc[k]);
      }
      lds_st16(sd + cm_off(ch, p, IROWS), pack8(acc));
    }
  }
  __syncthreads();

  // 4. x1 = x + pw2 d (float32, kept in registers for the final residual;
  //    each wave's blocks in pw4 are the same), and bf16(x1) -> LDS (t's
  //    region) as pw3's input.
  WFrag<C> w3 = load_wfrag<C>(a.pw3, cb3, lane);
  constexpr int NB2 = NCB * (IROWS / 32);           // 32 x 32 blocks of a C-output step
  constexpr int BPW = (NB2 + 7) / 8;                // per wave
  f32x16 x1[BPW];
#pragma unroll
  for (int j = 0; j < BPW; ++j) {
    const int b = wave + 8 * j;
    if (b >= NB2) break;
    const int cb = cbw, pb = b / NCB;
    f32x16 v = pw_block<C>(w2, sd, IROWS, pb, lane);
    halves_to_runs(v);
    const int p = pb * 32 + prow;
    const int hrow = (p / TW + 1) * HW + p % TW + 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int ch = (cb * 32 + h * 16 + cofs) / 8;
      float xv[8];
      unpack8(lds_ld16(sx + cm_off(ch, hrow, HROWS)), xv);
#pragma unroll
      for (int k = 0; k < 8; ++k) v[8 * h + k] += xv[k];
    }
    x1[j] = v;
  }
  __syncthreads();   // x and t are no longer read
#pragma unroll
  for (int j = 0; j < BPW; ++j) {
    const int b = wave + 8 * j;
    if (b >= NB2) break;
    const int cb = b % NCB, pb = b / NCB;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float o[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) o[k] = x1[j][8 * h + k];
      const int ch = (cb * 32 + h * 16 + cofs) / 8;
      lds_st16(st + cm_off(ch, pb * 32 + prow, IROWS), pack8(o));
    }
  }
  __syncthreads();

  // 5. u = relu(pw3 x1) -> LDS (x and d regions), 2C channels.
  WFrag<2 * C> w4 = load_wfrag<2 * C>(a.pw4, cbw, lane);
  for (int b = wave; b < 2 * NCB * (IROWS / 32); b += NT / 64) {
    const int cb = cb3, pb = b / (2 * NCB);
    f32x16 v = pw_block<C>(w3, st, IROWS, pb, lane);
    halves_to_runs(v);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float o[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) o[k] = fmaxf(v[8 * h + k], 0.f);
      const int ch = (cb * 32 + h * 16 + cofs) / 8;
      lds_st16(su + cm_off(ch, pb * 32 + prow, IROWS), pack8(o));
    }
  }
  __syncthreads();

  // 6. y = x1 + pw4 u -> bf16 output.
#pragma unroll
  for (int j = 0; j < BPW; ++j) {
    const int b = wave + 8 * j;
    if (b >= NB2) break;
    const int cb = cbw, pb = b / NCB;
    f32x16 v = pw_block<2 * C>(w4, su, IROWS, pb, lane);
    halves_to_runs(v);
    const int p = pb * 32 + prow;
    const int gy = ty0 + p / TW, gx = tx0 + p % TW;
    if (gy >= a.h || gx >= a.w) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float o[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) o[k] = v[8 * h + k] + x1[j][8 * h + k];
      const int c0 = cb * 32 + h * 16 + cofs;
      stg(reinterpret_cast<dv4u*>(a.y + ((long)gy * a.w + gx) * C + c0), pack8(o));
    }
  }
}

template <int C, int TH>
static hipError_t launch_dcb(const DcBlockArgs& a, hipStream_t s) {
  using namespace dcb;
  constexpr int LDS = (C / 8) * (2 * Tile<TH>::HROWS + Tile<TH>::IROWS) * 16;
  static std::atomic<uint32_t> attr{0};
  if (const hipError_t e =
          set_lds_limit_once(attr, reinterpret_cast<const void*>(dc_block_kernel<C, TH>), LDS))
    return e;
  const int tiles = ((a.w + TW - 1) / TW) * ((a.h + TH - 1) / TH);
  hipLaunchKernelGGL((dc_block_kernel<C, TH>), dim3(((tiles + 7) / 8) * 8), dim3(NT), LDS, s, a);
  return hipGetLastError();
}

// Tile rows: 8 (the default: 128 KB of LDS at C = 128, one workgroup per CU)
// or 4 (80 KB, but its register count still allows only one workgroup of
// eight waves per CU, and pw1 then runs on 2x the inner positions: 29 us
// against 20 us for one 1080p latent).
hipError_t launch_dc_block(int C, const DcBlockArgs& a, hipStream_t s, int tile_rows) {
  if (a.h <= 0 || a.w <= 0) return hipSuccess;
  if (tile_rows == 8) {
    if (C == 128) return launch_dcb<128, 8>(a, s);
    if (C == 64) return launch_dcb<64, 8>(a, s);
  } else if (tile_rows == 4) {
    if (C == 128) return launch_dcb<128, 4>(a, s);
    if (C == 64) return launch_dcb<64, 4>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ufvc

using namespace ufvc;

struct ufvc_dcblock {
  int C = 0;
  __bf16* w = nullptr;   // pw1 | pw2 | pw3 | pw4, bf16
  float* dw = nullptr;   // [C][9]
};

extern "C" {

int ufvc_dcblock_create(int C, const float* weights, size_t n_weights, ufvc_dcblock** out) {
  if (!weights || !out || (C != 64 && C != 128)) return UFVC_E_INVAL;
  *out = nullptr;
  const size_t cc = (size_t)C * C;
  if (n_weights != 6 * cc + 9 * (size_t)C) return UFVC_E_INVAL;
  // blob order: pw1, dw, pw2, pw3, pw4
  const float* pw1 = weights;
  const float* dw = pw1 + cc;
  const float* pw2 = dw + 9 * (size_t)C;
  const float* pw3 = pw2 + cc;
  const float* pw4 = pw3 + 2 * cc;
  std::vector<__bf16> wb(6 * cc);
  for (size_t i = 0; i < cc; ++i) wb[i] = (__bf16)pw1[i];
  for (size_t i = 0; i < cc; ++i) wb[cc + i] = (__bf16)pw2[i];
  for (size_t i = 0; i < 2 * cc; ++i) wb[2 * cc + i] = (__bf16)pw3[i];
  for (size_t i = 0; i < 2 * cc; ++i) wb[4 * cc + i] = (__bf16)pw4[i];
  ufvc_dcblock* b = new (std::nothrow) ufvc_dcblock();
  if (!b) return UFVC_E_NOMEM;
  b->C = C;
  if (hipMalloc(&b->w, wb.size() * sizeof(__bf16)) != hipSuccess ||
      hipMalloc(&b->dw, 9 * (size_t)C * sizeof(float)) != hipSuccess) {
    ufvc_dcblock_destroy(b);
    return UFVC_E_NOMEM;
  }
  if (hipMemcpy(b->w, wb.data(), wb.size() * sizeof(__bf16), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->dw, dw, 9 * (size_t)C * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    ufvc_dcblock_destroy(b);
    return UFVC_E_DEVICE;
  }
  *out = b;
  return UFVC_OK;
}

void ufvc_dcblock_destroy(ufvc_dcblock* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  if (b->w) (void)hipFree(b->w);
  if (b->dw) (void)hipFree(b->dw);
  delete b;
}

int ufvc_dcblock_run(ufvc_dcblock* b, const uint16_t* x, uint16_t* y, int h, int w, void* stream) {
  if (!b || !x || !y || h < 1 || w < 1 || (const void*)x == (const void*)y) return UFVC_E_INVAL;
  const size_t cc = (size_t)b->C * b->C;
  DcBlockArgs a{};
  a.x = reinterpret_cast<const __bf16*>(x);
  a.y = reinterpret_cast<__bf16*>(y);
  a.h = h;
  a.w = w;
  a.pw1 = b->w;
  a.pw2 = b->w + cc;
  a.pw3 = b->w + 2 * cc;
  a.pw4 = b->w + 4 * cc;
  a.dw = b->dw;
  return launch_dc_block(b->C, a, (hipStream_t)stream) == hipSuccess ? UFVC_OK : UFVC_E_DEVICE;
}

}  // extern "C"
