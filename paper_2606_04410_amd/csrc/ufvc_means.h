// Quadtree progressive means (see ufvc_means.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ufvc {

struct MeanArgs {
  int C, h, w;          // latent channels (64 or 128) and size (h, w even)
  int ho, wo;           // h / 2, w / 2 (set by the launcher)
  const uint8_t* sym;   // [h][w][C] symbols r_hat + 32 (partitions < k are read)
  float* P;             // [h][w][2C]: mu in the first C channels, refined in place on partition k
  const float* y;       // encoder: y [h][w][C] (partition k is quantised); decoder: null
  uint8_t* sym_out;     // encoder: symbol output (may alias sym: different partitions)
  const __bf16* wpk;    // step weights [step 1..3][tap][part h, m, l][C / 8][C][8] bf16
  size_t w_kstride;     // bytes per step
  const __bf16* wk;     // this step's weights (set by the launcher)
};

// Step k (1..3) of the progressive means: reads the symbols of partitions
// < k and the base means of partition k, writes partition k's means (and,
// in the encoder, its symbols).
hipError_t launch_mean_step(int k, const MeanArgs& a, hipStream_t s);

}  // namespace ufvc
