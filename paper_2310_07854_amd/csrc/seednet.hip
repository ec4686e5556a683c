// HIP kernels of the learned trajectory seeder (a network in place of the geometric planner that
// seeds trajectory optimisation, Sec. II-A, III-B, VI-B):
//   k_occupancy   8x8x8 occupancy of the cube [-0.75, 0.75]^3 m per world
//   k_features    [start, goal, occupancy] as BF16 rows of 544 (526 values + zero padding)
//   k_gemm_bf16   C = A B (+ bias) on MFMA (BF16 operands, FP32 accumulation) with fused epilogues:
//                 plain, GELU (keeping the pre-activation), or times GELU'(pre-activation)
//   k_seed_loss   min-over-slot matching loss and its gradient per problem
//   k_column_sum  bias gradients
//   k_adam        Adam update of FP32 master weights plus their BF16 copies
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "seednet.hpp"

namespace vapr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float from_bf16(uint16_t c) { return __uint_as_float((uint32_t)c << 16); }

// GELU(z) = z Phi(z) and its derivative Phi(z) + z phi(z), with the device library's erff / expf
__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---- occupancy ------------------------------------------------------------------------------------

// one block per world, one thread per voxel pair; voxel (x, y, z), index (z * 8 + y) * 8 + x, is
// occupied when min_k sd_k(centre) <= e / 2 with e = 0.1875 m
__global__ __launch_bounds__(256) void k_occupancy(const float* __restrict__ pose, const float* __restrict__ half,
                                                   int K, float* __restrict__ occ) {
  const int w = blockIdx.x;
  const float e = (SEED_CUBE_HI - SEED_CUBE_LO) / SEED_GRID;
  for (int v = threadIdx.x; v < SEED_VOXELS; v += blockDim.x) {
    const int x = v % SEED_GRID, y = (v / SEED_GRID) % SEED_GRID, z = v / (SEED_GRID * SEED_GRID);
    const float p[3] = {SEED_CUBE_LO + (x + 0.5f) * e, SEED_CUBE_LO + (y + 0.5f) * e, SEED_CUBE_LO + (z + 0.5f) * e};
    float best = INFINITY;
    for (int k = 0; k < K; ++k) {
      const float* P = pose + ((int64_t)w * K + k) * 12;
      const float* h = half + ((int64_t)w * K + k) * 3;
      const float d[3] = {p[0] - P[3], p[1] - P[7], p[2] - P[11]};
      float o2 = 0.f, amax = -INFINITY;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        // u_c = (R^T (p - centre))_c = sum_r R[r][c] d_r
        const float u = fmaf(P[c], d[0], fmaf(P[4 + c], d[1], P[8 + c] * d[2]));
        const float a = fabsf(u) - h[c];
        const float m = fmaxf(a, 0.f);
        o2 = fmaf(m, m, o2);
        amax = fmaxf(amax, a);
      }
      best = fminf(best, sqrtf(o2) + fminf(amax, 0.f));
    }
    occ[(int64_t)w * SEED_VOXELS + v] = best <= 0.5f * e ? 1.f : 0.f;
  }
}

// ---- features ---------------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_features(int n, const float* __restrict__ start, const float* __restrict__ goal,
                                                  const float* __restrict__ occ, uint16_t* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)n * SEED_IN_PAD) return;
  const int64_t r = i / SEED_IN_PAD;
  const int c = (int)(i - r * SEED_IN_PAD);
  float v = 0.f;
  if (c < SEED_J) v = start[r * SEED_J + c];
  else if (c < 2 * SEED_J) v = goal[r * SEED_J + c - SEED_J];
  else if (c < SEED_IN) v = occ[r * SEED_VOXELS + c - 2 * SEED_J];
  x[i] = to_bf16(v);
}

// ---- GEMM on MFMA -------------------------------------------------------------------------------------
//
// Block tile 64 x 64, four wavefronts of 32 x 32 (2 x 2 MFMA 16x16x32 tiles), K in steps of 32.  A
// and B tiles are staged in LDS with k contiguous ([m][k] and [n][k], rows padded to 40 elements), so
// a lane's MFMA operand (row lane % 16, k = 8 (lane / 16) .. + 7) is one 16-byte read.  The
// accumulator of lane l holds rows 4 (l / 16) + e, column l % 16 of its 16x16 tile.
// A_K: A(m, k) contiguous in k (else in m); B_N: B(k, n) contiguous in n (else in k).

constexpr int GT = 64, GK = 32, GPAD = 40;

template <bool A_K, bool B_N>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[GT * GPAD];
  __shared__ __attribute__((aligned(16))) uint16_t sB[GT * GPAD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += GK) {
    // A tile -> sA[r][kc .. kc + 7]
    {
      uint16_t v[8];
      int r, kc;
      if constexpr (A_K) {
        r = tid >> 2;
        kc = (tid & 3) * 8;
        const int m = m0 + r;
        if (m < g.M) {
          const uint4 q = *reinterpret_cast<const uint4*>(g.A + (int64_t)m * g.sam + k0 + kc);
          v[0] = q.x & 0xffff; v[1] = q.x >> 16; v[2] = q.y & 0xffff; v[3] = q.y >> 16;
          v[4] = q.z & 0xffff; v[5] = q.z >> 16; v[6] = q.w & 0xffff; v[7] = q.w >> 16;
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = 0;
        }
      } else {
        r = tid & 63;
        kc = (tid >> 6) * 8;
        const int m = m0 + r;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = m < g.M ? g.A[(int64_t)m + (int64_t)(k0 + kc + e) * g.sak] : (uint16_t)0;
      }
      uint4 q;
      q.x = v[0] | ((uint32_t)v[1] << 16); q.y = v[2] | ((uint32_t)v[3] << 16);
      q.z = v[4] | ((uint32_t)v[5] << 16); q.w = v[6] | ((uint32_t)v[7] << 16);
      *reinterpret_cast<uint4*>(sA + r * GPAD + kc) = q;
    }
    // B tile -> sB[c][kc .. kc + 7]
    {
      uint16_t v[8];
      int c, kc;
      if constexpr (B_N) {
        c = tid & 63;
        kc = (tid >> 6) * 8;
        const int n = n0 + c;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = n < g.N ? g.B[(int64_t)(k0 + kc + e) * g.sbk + n] : (uint16_t)0;
      } else {
        c = tid >> 2;
        kc = (tid & 3) * 8;
        const int n = n0 + c;
        if (n < g.N) {
          const uint4 q = *reinterpret_cast<const uint4*>(g.B + (int64_t)n * g.sbn + k0 + kc);
          v[0] = q.x & 0xffff; v[1] = q.x >> 16; v[2] = q.y & 0xffff; v[3] = q.y >> 16;
          v[4] = q.z & 0xffff; v[5] = q.z >> 16; v[6] = q.w & 0xffff; v[7] = q.w >> 16;
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = 0;
        }
      }
      uint4 q;
      q.x = v[0] | ((uint32_t)v[1] << 16); q.y = v[2] | ((uint32_t)v[3] << 16);
      q.z = v[4] | ((uint32_t)v[5] << 16); q.w = v[6] | ((uint32_t)v[7] << 16);
      *reinterpret_cast<uint4*>(sB + c * GPAD + kc) = q;
    }
    __syncthreads();
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *reinterpret_cast<const bf16x8*>(sA + (wm + i * 16 + (lane & 15)) * GPAD + 8 * (lane >> 4));
      b[i] = *reinterpret_cast<const bf16x8*>(sB + (wn + i * 16 + (lane & 15)) * GPAD + 8 * (lane >> 4));
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + j * 16 + (lane & 15);
      if (n >= g.N) continue;
      const float bias = g.bias ? g.bias[n] : 0.f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + e;
        if (m >= g.M) continue;
        const int64_t o = (int64_t)m * g.ldc + n;
        float v = acc[i][j][e] + bias;
        if (g.epilogue == GEMM_GELU) {
          g.aux[o] = v;
          v = gelu_f(v);
        } else if (g.epilogue == GEMM_GELU_GRAD) {
          v *= gelu_grad_f(g.aux[o]);
        }
        if (g.C) g.C[o] = v;
        if (g.C16) g.C16[o] = to_bf16(v);
      }
    }
}

// ---- seed trajectories ------------------------------------------------------------------------------

// out[r][s][t][j] = start + (goal - start) t / 31 + (t in 1..30 ? y[r][(s * 32 + t) * 7 + j] : 0)
__global__ __launch_bounds__(256) void k_seed_traj(int n, const float* __restrict__ y, const float* __restrict__ start,
                                                   const float* __restrict__ goal, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)n * SEED_OUT) return;
  const int64_t r = i / SEED_OUT;
  const int k = (int)(i - r * SEED_OUT);
  const int j = k % SEED_J, t = (k / SEED_J) % SEED_T;
  const float s0 = start[r * SEED_J + j], g0 = goal[r * SEED_J + j];
  const float line = fmaf(g0 - s0, (float)t / (float)(SEED_T - 1), s0);
  out[i] = (t == 0 || t == SEED_T - 1) ? (t == 0 ? s0 : g0) : line + y[i];
}

// ---- loss -------------------------------------------------------------------------------------------

// one wavefront per problem; lane = slot * 8 + target
__global__ __launch_bounds__(64) void k_seed_loss(const float* __restrict__ y, const float* __restrict__ tgt,
                                                  const float* __restrict__ valid, float coef,
                                                  double* __restrict__ per_problem, int32_t* __restrict__ assign,
                                                  float* __restrict__ dy) {
  __shared__ float e[SEED_SLOTS * SEED_SLOTS];
  __shared__ int as[SEED_SLOTS];
  const int n = blockIdx.x, lane = threadIdx.x;
  const float* yn = y + (int64_t)n * SEED_OUT;
  const float* tn = tgt + (int64_t)n * SEED_OUT;
  {
    const int s = lane >> 3, j = lane & 7;
    float acc = 0.f;
    for (int i = 0; i < SEED_TRAJ; ++i) {
      const float d = yn[s * SEED_TRAJ + i] - tn[j * SEED_TRAJ + i];
      acc = fmaf(d, d, acc);
    }
    e[s * SEED_SLOTS + j] = acc * (1.0f / SEED_TRAJ);
  }
  __syncthreads();
  if (lane < SEED_SLOTS) {
    const int j = lane;
    int bs = 0;
    float be = e[j];
    for (int s = 1; s < SEED_SLOTS; ++s)
      if (e[s * SEED_SLOTS + j] < be) {
        be = e[s * SEED_SLOTS + j];
        bs = s;
      }
    as[j] = bs;
    assign[(int64_t)n * SEED_SLOTS + j] = bs;
  }
  __syncthreads();
  if (lane == 0) {
    double L = 0.0;
    for (int j = 0; j < SEED_SLOTS; ++j)
      if (valid[(int64_t)n * SEED_SLOTS + j] != 0.f) L += (double)e[as[j] * SEED_SLOTS + j];
    per_problem[n] = L;
  }
  for (int i = lane; i < SEED_OUT; i += 64) {
    const int s = i / SEED_TRAJ, t = i - s * SEED_TRAJ;
    float g = 0.f;
    for (int j = 0; j < SEED_SLOTS; ++j)
      if (as[j] == s && valid[(int64_t)n * SEED_SLOTS + j] != 0.f) g += yn[i] - tn[j * SEED_TRAJ + t];
    dy[(int64_t)n * SEED_OUT + i] = coef * g;
  }
}

// total loss = sum over problems (fixed order, one wavefront) / number of valid targets
__global__ __launch_bounds__(64) void k_seed_loss_total(const double* __restrict__ per_problem, int n, double inv,
                                                        double* __restrict__ out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += per_problem[i];
  __shared__ double part[64];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 64; ++i) t += part[i];
    *out = t * inv;
  }
}

// ---- bias gradients, Adam ------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_column_sum(int M, int N, const float* __restrict__ X, int64_t ldx,
                                                    float* __restrict__ out) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += X[(int64_t)m * ldx + n];
  out[n] = s;
}

__global__ __launch_bounds__(256) void k_adam(int64_t n, float* __restrict__ w, uint16_t* __restrict__ w16,
                                              const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = fmaf(a.b1, m[i], (1.f - a.b1) * gi);
  const float vi = fmaf(a.b2, v[i], (1.f - a.b2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - a.lr * (mi * a.inv_bc1) / (sqrtf(vi * a.inv_bc2) + a.eps);
  w[i] = wi;
  if (w16) w16[i] = to_bf16(wi);
}

// ---- launchers ----------------------------------------------------------------------------------------

static inline unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_occupancy(hipStream_t s, int W, int K, const float* pose, const float* half, float* occ) {
  hipLaunchKernelGGL(k_occupancy, dim3(W), dim3(256), 0, s, pose, half, K, occ);
  return hipGetLastError();
}

hipError_t launch_features(hipStream_t s, int n, const float* start, const float* goal, const float* occ,
                           uint16_t* x) {
  hipLaunchKernelGGL(k_features, dim3(nblocks((int64_t)n * SEED_IN_PAD, 256)), dim3(256), 0, s, n, start, goal,
                     occ, x);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(hipStream_t s, const GemmArgs& g, bool a_k, bool b_n) {
  const dim3 grid(nblocks(g.M, GT), nblocks(g.N, GT)), block(256);
  if (a_k && b_n) hipLaunchKernelGGL((k_gemm_bf16<true, true>), grid, block, 0, s, g);
  else if (a_k) hipLaunchKernelGGL((k_gemm_bf16<true, false>), grid, block, 0, s, g);
  else if (b_n) hipLaunchKernelGGL((k_gemm_bf16<false, true>), grid, block, 0, s, g);
  else hipLaunchKernelGGL((k_gemm_bf16<false, false>), grid, block, 0, s, g);
  return hipGetLastError();
}

hipError_t launch_seed_traj(hipStream_t s, int n, const float* y, const float* start, const float* goal, float* out) {
  hipLaunchKernelGGL(k_seed_traj, dim3(nblocks((int64_t)n * SEED_OUT, 256)), dim3(256), 0, s, n, y, start, goal, out);
  return hipGetLastError();
}

hipError_t launch_seed_loss(hipStream_t s, int n, const float* y, const float* tgt, const float* valid, float coef,
                            double* per_problem, int32_t* assign, float* dy, double inv_valid, double* loss) {
  hipLaunchKernelGGL(k_seed_loss, dim3(n), dim3(64), 0, s, y, tgt, valid, coef, per_problem, assign, dy);
  hipLaunchKernelGGL(k_seed_loss_total, dim3(1), dim3(64), 0, s, per_problem, n, inv_valid, loss);
  return hipGetLastError();
}

hipError_t launch_column_sum(hipStream_t s, int M, int N, const float* X, int64_t ldx, float* out) {
  hipLaunchKernelGGL(k_column_sum, dim3(nblocks(N, 256)), dim3(256), 0, s, M, N, X, ldx, out);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, int64_t n, float* w, uint16_t* w16, const float* g, float* m, float* v,
                       const AdamArgs& a) {
  hipLaunchKernelGGL(k_adam, dim3(nblocks(n, 256)), dim3(256), 0, s, n, w, w16, g, m, v, a);
  return hipGetLastError();
}

}  // namespace vapr
