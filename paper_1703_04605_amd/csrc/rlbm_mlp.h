// Layout of the learned Landau-frame guess network (9 -> 64 -> 64 -> 64 -> 3,
// SiLU) and of its device state.  Parameters are one float vector:
// W1 [64 x 9], b1 [64], W2 [64 x 64], b2 [64], W3 [64 x 64], b3 [64],
// W4 [3 x 64], b4 [3]  (row-major, z = W a + b), 9155 values.
#pragma once
#include <hip/hip_runtime.h>

#define RLBM_MLP_NPARAM 9155

constexpr int RLBM_MLP_IN[4] = {9, 64, 64, 64};
constexpr int RLBM_MLP_OUT[4] = {64, 64, 64, 3};
constexpr int RLBM_MLP_WOFF[4] = {0, 640, 4800, 8960};
constexpr int RLBM_MLP_BOFF[4] = {576, 4736, 8896, 9152};
// matrix-core fragments (32x32x16 bf16): output tiles of 32 units and k-steps of 16
constexpr int RLBM_MLP_TILES[4] = {2, 2, 2, 1};
constexpr int RLBM_MLP_KSTEPS[4] = {1, 4, 4, 4};
constexpr int RLBM_MLP_FOFF[4] = {0, 2, 10, 18};   // in (tile, kstep) items of 64 lanes x 8 bf16
constexpr int RLBM_MLP_BFOFF[4] = {0, 2, 4, 6};    // in tiles of 64 lanes x 16 floats
#define RLBM_MLP_NFRAG 22
#define RLBM_MLP_NBFRAG 7

struct rlbm_mlp {
  int max_batch = 0;
  int t = 0;                       // Adam step count
  float* base = nullptr;           // one allocation for the float buffers below
  float *master = nullptr, *bf = nullptr, *grad = nullptr, *mom1 = nullptr, *mom2 = nullptr;
  float* norm = nullptr;           // mx[9], sx[9], my[3], sy[3]
  float h_norm[24];
  float *X = nullptr, *Xraw = nullptr, *Y = nullptr, *D4 = nullptr, *Z4 = nullptr, *loss = nullptr;
  float* Z[3] = {nullptr, nullptr, nullptr};
  float* A[3] = {nullptr, nullptr, nullptr};
  float* D[3] = {nullptr, nullptr, nullptr};
  unsigned short* frag = nullptr;  // bf16 weight fragments for the in-step inference
  float* biasfrag = nullptr;       // bias fragments (accumulator layout)
  float* part = nullptr;           // per-chunk partial weight gradients [chunks][64][65]
};

// Re-rounds the bf16 copies and re-packs the fragments after a weight change.
int rlbm_mlp_refresh(rlbm_mlp* m, hipStream_t s);
