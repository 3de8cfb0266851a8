// Frame format conversions around the codec's YUV444 interface (supplementary
// material, RGB section: RGB and YUV420 video are converted to YUV444 for
// inference and back afterwards; RGB with BT.709).
//
// Full range, values in [0, 1], chroma centred at 1/2; BT.709 luma weights
// Kr = 0.2126, Kb = 0.0722.  4:2:0 -> 4:4:4 repeats each chroma sample over
// its 2 x 2 block; 4:4:4 -> 4:2:0 takes the block mean.  RGB output is
// clamped to [0, 1].
//
// Layouts (float32): YUV444 and RGB are [T][3][H][W] planes; YUV420 is T
// planar frames, each Y [H][W], then Cb and Cr [H/2][W/2].
//
// All four kernels are pure streaming (HBM-bound): every thread moves whole
// 16-byte vectors, rows are contiguous, and no value is read twice.
#include "../../include/ufvc.h"
#include "ufvc_common.h"

namespace ufvc {

typedef float cv4f __attribute__((ext_vector_type(4)));
typedef float cv2f __attribute__((ext_vector_type(2)));

constexpr float KR = 0.2126f, KB = 0.0722f, KG = 1.0f - 0.2126f - 0.0722f;
constexpr float CB_S = 1.0f / (2.0f * (1.0f - 0.0722f));   // (B - Y) -> Cb - 1/2
constexpr float CR_S = 1.0f / (2.0f * (1.0f - 0.2126f));   // (R - Y) -> Cr - 1/2
constexpr float CB_I = 2.0f * (1.0f - 0.0722f);
constexpr float CR_I = 2.0f * (1.0f - 0.2126f);

// One thread per 4 consecutive pixels of one frame (H W divisible by 4).
__global__ void __launch_bounds__(256) rgb_to_yuv444_kernel(const float* __restrict__ src,
                                                            float* __restrict__ dst, long plane,
                                                            long nvec) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nvec; i += (long)gridDim.x * blockDim.x) {
    const long t = i / (plane / 4), p = (i - t * (plane / 4)) * 4;
    const long base = t * 3 * plane + p;
    const cv4f r = ldg(reinterpret_cast<const cv4f*>(src + base));
    const cv4f g = ldg(reinterpret_cast<const cv4f*>(src + base + plane));
    const cv4f b = ldg(reinterpret_cast<const cv4f*>(src + base + 2 * plane));
    const cv4f y = KR * r + KG * g + KB * b;
    stg(reinterpret_cast<cv4f*>(dst + base), y);
    stg(reinterpret_cast<cv4f*>(dst + base + plane), (b - y) * CB_S + 0.5f);
    stg(reinterpret_cast<cv4f*>(dst + base + 2 * plane), (r - y) * CR_S + 0.5f);
  }
}

__device__ __forceinline__ cv4f clamp01(cv4f v) {
  return cv4f{fminf(fmaxf(v.x, 0.f), 1.f), fminf(fmaxf(v.y, 0.f), 1.f), fminf(fmaxf(v.z, 0.f), 1.f),
              fminf(fmaxf(v.w, 0.f), 1.f)};
}

__global__ void __launch_bounds__(256) yuv444_to_rgb_kernel(const float* __restrict__ src,
                                                            float* __restrict__ dst, long plane,
                                                            long nvec) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nvec; i += (long)gridDim.x * blockDim.x) {
    const long t = i / (plane / 4), p = (i - t * (plane / 4)) * 4;
    const long base = t * 3 * plane + p;
    const cv4f y = ldg(reinterpret_cast<const cv4f*>(src + base));
    const cv4f cb = ldg(reinterpret_cast<const cv4f*>(src + base + plane)) - 0.5f;
    const cv4f cr = ldg(reinterpret_cast<const cv4f*>(src + base + 2 * plane)) - 0.5f;
    const cv4f r = y + CR_I * cr;
    const cv4f b = y + CB_I * cb;
    const cv4f g = (y - KR * r - KB * b) * (1.0f / KG);
    stg(reinterpret_cast<cv4f*>(dst + base), clamp01(r));
    stg(reinterpret_cast<cv4f*>(dst + base + plane), clamp01(g));
    stg(reinterpret_cast<cv4f*>(dst + base + 2 * plane), clamp01(b));
  }
}

// One thread per 4 consecutive pixels of one row: Y copied, each of the two
// chroma samples under them written twice (W divisible by 4).
__global__ void __launch_bounds__(256) yuv420_to_444_kernel(const float* __restrict__ src,
                                                            float* __restrict__ dst, int H, int W,
                                                            long nvec) {
  const long plane = (long)H * W, qplane = plane / 4, frame420 = plane + 2 * qplane;
  const int vw = W / 4;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nvec; i += (long)gridDim.x * blockDim.x) {
    const long t = i / ((long)H * vw);
    const long r = i - t * H * vw;
    const int row = (int)(r / vw), x = (int)(r - (long)row * vw) * 4;
    const float* f = src + t * frame420;
    float* o = dst + t * 3 * plane + (long)row * W + x;
    stg(reinterpret_cast<cv4f*>(o), ldg(reinterpret_cast<const cv4f*>(f + (long)row * W + x)));
    const long cidx = (long)(row / 2) * (W / 2) + x / 2;
    const cv2f cb = ldg(reinterpret_cast<const cv2f*>(f + plane + cidx));
    const cv2f cr = ldg(reinterpret_cast<const cv2f*>(f + plane + qplane + cidx));
    stg(reinterpret_cast<cv4f*>(o + plane), cv4f{cb.x, cb.x, cb.y, cb.y});
    stg(reinterpret_cast<cv4f*>(o + 2 * plane), cv4f{cr.x, cr.x, cr.y, cr.y});
  }
}

// One thread per 2 rows x 4 columns: the two Y vectors copied, two chroma
// samples of each plane from their 2 x 2 blocks.
__global__ void __launch_bounds__(256) yuv444_to_420_kernel(const float* __restrict__ src,
                                                            float* __restrict__ dst, int H, int W,
                                                            long nvec) {
  const long plane = (long)H * W, qplane = plane / 4, frame420 = plane + 2 * qplane;
  const int vw = W / 4, hh = H / 2;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nvec; i += (long)gridDim.x * blockDim.x) {
    const long t = i / ((long)hh * vw);
    const long r = i - t * hh * vw;
    const int row2 = (int)(r / vw), x = (int)(r - (long)row2 * vw) * 4;
    const float* f = src + t * 3 * plane + (long)(2 * row2) * W + x;
    float* o = dst + t * frame420;
    stg(reinterpret_cast<cv4f*>(o + (long)(2 * row2) * W + x), ldg(reinterpret_cast<const cv4f*>(f)));
    stg(reinterpret_cast<cv4f*>(o + (long)(2 * row2 + 1) * W + x), ldg(reinterpret_cast<const cv4f*>(f + W)));
    const long cidx = (long)row2 * (W / 2) + x / 2;
#pragma unroll
    for (int c = 1; c <= 2; ++c) {
      const cv4f a = ldg(reinterpret_cast<const cv4f*>(f + c * plane));
      const cv4f b = ldg(reinterpret_cast<const cv4f*>(f + c * plane + W));
      // (a0 + a1 + b0 + b1) / 4 in a fixed order
      const cv2f m = cv2f{((a.x + a.y) + (b.x + b.y)) * 0.25f, ((a.z + a.w) + (b.z + b.w)) * 0.25f};
      stg(reinterpret_cast<cv2f*>(o + plane + (c - 1) * qplane + cidx), m);
    }
  }
}

static dim3 stream_grid(long nvec) {
  long blocks = (nvec + 255) / 256;
  if (blocks > 65536) blocks = 65536;   // grid-stride beyond that
  return dim3((unsigned)(blocks > 0 ? blocks : 1));
}

}  // namespace ufvc

using namespace ufvc;

extern "C" int ufvc_convert_frames(const float* src, int src_fmt, float* dst, int dst_fmt, int T,
                                   int H, int W, void* stream) {
  if (!src || !dst || T < 1 || H < 2 || W < 4 || (W & 3) || (H & 1)) return UFVC_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const long plane = (long)H * W;
  if (src_fmt == UFVC_FMT_RGB709 && dst_fmt == UFVC_FMT_YUV444) {
    const long nvec = T * plane / 4;
    hipLaunchKernelGGL(rgb_to_yuv444_kernel, stream_grid(nvec), dim3(256), 0, s, src, dst, plane, nvec);
  } else if (src_fmt == UFVC_FMT_YUV444 && dst_fmt == UFVC_FMT_RGB709) {
    const long nvec = T * plane / 4;
    hipLaunchKernelGGL(yuv444_to_rgb_kernel, stream_grid(nvec), dim3(256), 0, s, src, dst, plane, nvec);
  } else if (src_fmt == UFVC_FMT_YUV420 && dst_fmt == UFVC_FMT_YUV444) {
    if (src == dst) return UFVC_E_INVAL;
    const long nvec = T * plane / 4;
    hipLaunchKernelGGL(yuv420_to_444_kernel, stream_grid(nvec), dim3(256), 0, s, src, dst, H, W, nvec);
  } else if (src_fmt == UFVC_FMT_YUV444 && dst_fmt == UFVC_FMT_YUV420) {
    if (src == dst) return UFVC_E_INVAL;
    const long nvec = T * plane / 8;
    hipLaunchKernelGGL(yuv444_to_420_kernel, stream_grid(nvec), dim3(256), 0, s, src, dst, H, W, nvec);
  } else {
    return UFVC_E_UNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? UFVC_OK : UFVC_E_DEVICE;
}
