// Shapes, argument structs and launchers of the learned-seeder kernels (seednet.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vapr {

constexpr int SEED_GRID = 8;
constexpr int SEED_VOXELS = SEED_GRID * SEED_GRID * SEED_GRID;  // 512
constexpr float SEED_CUBE_LO = -0.75f, SEED_CUBE_HI = 0.75f;
constexpr int SEED_J = 7;
constexpr int SEED_IN = 2 * SEED_J + SEED_VOXELS;               // 526 features
constexpr int SEED_IN_PAD = 544;                                 // padded to a multiple of 32
constexpr int SEED_HID = 256;
constexpr int SEED_SLOTS = 8;
constexpr int SEED_T = 32;
constexpr int SEED_TRAJ = SEED_T * SEED_J;                       // 224 values per seed
constexpr int SEED_OUT = SEED_SLOTS * SEED_TRAJ;                 // 1792

enum GemmEpilogue { GEMM_PLAIN = 0, GEMM_GELU = 1, GEMM_GELU_GRAD = 2, GEMM_SEED_TRAJ = 3 };

struct GemmArgs {
  int M, N, K;
  const uint16_t* A;  // BF16; A(m, k) at A[m * sam + k * sak]
  int64_t sam, sak;
  const uint16_t* B;  // BF16; B(k, n) at B[k * sbk + n * sbn]
  int64_t sbk, sbn;
  const float* bias;  // [N] or null
  int epilogue;
  float* aux;         // [M][ldc] pre-activation (written by GELU, read by GELU_GRAD)
  float* C;           // [M][ldc] FP32 result or null
  uint16_t* C16;      // [M][ldc] BF16 result or null
  int64_t ldc;
  const float* start;  // [M][7] (GEMM_SEED_TRAJ only)
  const float* goal;   // [M][7] (GEMM_SEED_TRAJ only)
};

struct AdamArgs {
  float lr, b1, b2, eps;
  float inv_bc1, inv_bc2;  // 1 / (1 - b1^t), 1 / (1 - b2^t)
};

hipError_t launch_occupancy(hipStream_t s, int W, int K, const float* pose, const float* half, float* occ);
hipError_t launch_features(hipStream_t s, int n, const float* start, const float* goal, const float* occ,
                           uint16_t* x);
hipError_t launch_gemm_bf16(hipStream_t s, const GemmArgs& g, bool a_k, bool b_n);
hipError_t launch_seed_traj(hipStream_t s, int n, const float* y, const float* start, const float* goal, float* out);
hipError_t launch_seed_dev(hipStream_t s, int n, int m, const float* traj, const float* start, const float* goal,
                           float* dev);
hipError_t launch_seed_loss(hipStream_t s, int n, const float* y, const float* tgt, const float* valid, float coef,
                            double* per_problem, int32_t* assign, float* dy, double inv_valid, double* loss);
hipError_t launch_column_sum(hipStream_t s, int M, int N, const float* X, int64_t ldx, float* out);
hipError_t launch_adam(hipStream_t s, int64_t n, float* w, uint16_t* w16, const float* g, float* m, float* v,
                       const AdamArgs& a);

}  // namespace vapr
