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

// one thread per 8 consecutive columns of a row (one 16-byte store); 68 chunks per 544-wide row
__global__ __launch_bounds__(256) void k_features(int n, const float* __restrict__ start, const float* __restrict__ goal,
                                                  const float* __restrict__ occ, uint16_t* __restrict__ x) {
  constexpr int CH = SEED_IN_PAD / 8;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n * CH) return;
  const int r = i / CH, c0 = (i - r * CH) * 8;
  uint16_t v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int c = c0 + e;
    float f = 0.f;
    if (c < SEED_J) f = start[r * SEED_J + c];
    else if (c < 2 * SEED_J) f = goal[r * SEED_J + c - SEED_J];
    else if (c < SEED_IN) f = occ[(int64_t)r * SEED_VOXELS + c - 2 * SEED_J];
    v[e] = to_bf16(f);
  }
  uint4 q;
  q.x = v[0] | ((uint32_t)v[1] << 16); q.y = v[2] | ((uint32_t)v[3] << 16);
  q.z = v[4] | ((uint32_t)v[5] << 16); q.w = v[6] | ((uint32_t)v[7] << 16);
  *reinterpret_cast<uint4*>(x + (int64_t)r * SEED_IN_PAD + c0) = q;
}

// ---- GEMM on MFMA -------------------------------------------------------------------------------------
//
// Block tile 64 x 64, four wavefronts of 32 x 32 (2 x 2 MFMA 16x16x32 tiles), K in steps of 32.  A
// and B tiles are staged in LDS with k contiguous ([m][k] and [n][k], rows padded to 40 elements), so
// a lane's MFMA operand (row lane % 16, k = 8 (lane / 16) .. + 7) is one 16-byte read.  The
// accumulator of lane l holds rows 4 (l / 16) + e, column l % 16 of its 16x16 tile.
// A_K: A(m, k) contiguous in k (else in m); B_N: B(k, n) contiguous in n (else in k).

constexpr int GK = 32, GPAD = 40;
constexpr int64_t GEMM_BIG_TILES_MIN = 1024;  // 128 x 128 tiles from this many on

// Seed-trajectory epilogue for output column n: the straight line from start to goal plus the
// network's deviation v at interior timesteps, start / goal exactly at the ends.  The column's joint,
// line fraction t / (T - 1) and kind depend on n only, so a thread works them out once for the four
// columns it writes; se holds the block's TM start rows, then its TM goal rows ([2][TM][7]).
struct TrajCol {
  int j;       // joint
  float frac;  // t / (T - 1)
  int kind;    // 0 start, 1 goal, 2 interior
};
__device__ __forceinline__ TrajCol traj_col(int n) {
  const int k = n % SEED_TRAJ, t = k / SEED_J, j = k - t * SEED_J;
  return TrajCol{j, (float)t / (float)(SEED_T - 1), t == 0 ? 0 : (t == SEED_T - 1 ? 1 : 2)};
}
template <int TM>
__device__ __forceinline__ float seed_traj_value(const float* se, int r, const TrajCol& c, float v) {
  const float s0 = se[r * SEED_J + c.j], g0 = se[(TM + r) * SEED_J + c.j];
  const float line = fmaf(g0 - s0, c.frac, s0);
  return c.kind == 0 ? s0 : (c.kind == 1 ? g0 : line + v);
}


// One operand tile (64 rows x 32 k) is stored in LDS as [row][k] (row stride GPAD halfwords), with
// the four 8-element k chunks of a row permuted by an XOR with bits 4..5 of the row: the transposing
// writes below (rows 4 apart in one instruction) then fall in distinct banks, and an MFMA operand
// read (16 rows of one 16-row group, one chunk per lane group) stays a permutation of the unswizzled
// one.  Rows past `rows` read as zero; K is a multiple of 32, so k is always in range.
//   load_kc / store_kc: element (row, k) at p[row * rs + k] (k contiguous): one 16-byte load per
//            thread, one 16-byte LDS write
//   load_rc / store_rc: element (row, k) at p[row + k * ks] (rows contiguous): with `vec` (ks a
//            multiple of 8, p 16-byte aligned) two 8-byte loads per thread, 4 rows at k and k + 1,
//            written as 4 32-bit (k, k + 1) pairs; otherwise 8 scalar loads per thread
__device__ __forceinline__ int lds_off(int row, int chunk) { return row * GPAD + ((chunk ^ ((row >> 4) & 3)) << 3); }

__device__ __forceinline__ uint4 pack8(const uint16_t v[8]) {
  uint4 q;
  q.x = v[0] | ((uint32_t)v[1] << 16); q.y = v[2] | ((uint32_t)v[3] << 16);
  q.z = v[4] | ((uint32_t)v[5] << 16); q.w = v[6] | ((uint32_t)v[7] << 16);
  return q;
}

struct Frag {
  uint4 q;
};

__device__ __forceinline__ Frag load_kc(const uint16_t* __restrict__ p, int64_t rs, int row0, int rows, int k0, int tid) {
  const int r = tid >> 2, kc = (tid & 3) * 8;
  Frag f{make_uint4(0u, 0u, 0u, 0u)};
  if (row0 + r < rows) f.q = *reinterpret_cast<const uint4*>(p + (int64_t)(row0 + r) * rs + k0 + kc);
  return f;
}

__device__ __forceinline__ void store_kc(const Frag& f, uint16_t* __restrict__ s, int tid) {
  *reinterpret_cast<uint4*>(s + lds_off(tid >> 2, tid & 3)) = f.q;
}

__device__ __forceinline__ Frag load_rc(const uint16_t* __restrict__ p, int64_t ks, int row0, int rows, int k0,
                                        bool vec, int tid) {
  uint16_t v[8];
  if (vec) {
    // q.x, q.y: rows 4 nc .. + 3 at k = 2 kp; q.z, q.w: the same rows at k + 1
    const int nc = tid & 15, kp = tid >> 4;
    const int r = row0 + nc * 4;
    const uint16_t* q0 = p + (int64_t)r + (int64_t)(k0 + 2 * kp) * ks;
    const uint16_t* q1 = q0 + ks;
    if (r + 3 < rows) {
      const uint2 a = *reinterpret_cast<const uint2*>(q0), b = *reinterpret_cast<const uint2*>(q1);
      return Frag{make_uint4(a.x, a.y, b.x, b.y)};
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] = r + e < rows ? q0[e] : (uint16_t)0;
      v[4 + e] = r + e < rows ? q1[e] : (uint16_t)0;
    }
  } else {
    const int r = tid & 63, kc = (tid >> 6) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      v[e] = row0 + r < rows ? p[(int64_t)(row0 + r) + (int64_t)(k0 + kc + e) * ks] : (uint16_t)0;
  }
  return Frag{pack8(v)};
}

__device__ __forceinline__ void store_rc(const Frag& f, bool vec, uint16_t* __restrict__ s, int tid) {
  if (vec) {
    const int nc = tid & 15, kp = tid >> 4;
    const uint32_t lo[2] = {f.q.x, f.q.y}, hi[2] = {f.q.z, f.q.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t a = (lo[e >> 1] >> (16 * (e & 1))) & 0xffff, b = (hi[e >> 1] >> (16 * (e & 1))) & 0xffff;
      *reinterpret_cast<uint32_t*>(s + lds_off(nc * 4 + e, kp >> 2) + 2 * (kp & 3)) = a | (b << 16);
    }
  } else {
    *reinterpret_cast<uint4*>(s + lds_off(tid & 63, tid >> 6)) = f.q;
  }
}

// Block -> output tile.  Workgroups go to the 8 XCDs round-robin by linear id; give XCD x a
// contiguous run of tiles in row-major (row tile, column tile) order, so that the column tiles of
// one row tile, which share its A rows, run on one XCD and meet them in its L2.
__device__ __forceinline__ int xcd_tile(int L, int T) {
  const int q = T >> 3, r = T & 7, x = L & 7, j = L >> 3;
  return x * q + min(x, r) + j;
}

// Workgroup barrier for LDS traffic only: this wave's LDS operations are complete (lgkmcnt 0), then
// s_barrier.  Unlike __syncthreads() it does not wait for the wave's outstanding global stores, so
// the output stores of one half of a tile stay in flight while the next half is staged.  The memory
// clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// One workgroup (4 wavefronts in 2 x 2) per TM x TN output tile; each wavefront computes a
// (TM / 2) x (TN / 2) block as (TM / 32) x (TN / 32) MFMA tiles of 16 x 16.  Operand tiles are staged
// 64 rows at a time with the helpers above.  64 x 64 tiles serve small problems (training batches);
// 128 x 128 tiles, with 16 MFMAs per wavefront and K step, amortise the staging and addressing of
// each step over four times the matrix work on large ones.
template <bool A_K, bool B_N, int TM, int TN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM * TN > 64 * 64 ? 3 : 1))) void k_gemm_bf16(
    GemmArgs g) {
  static_assert(TM % 64 == 0 && TN % 64 == 0, "tiles are staged 64 rows at a time");
  constexpr int FM = TM / 32, FN = TN / 32;  // MFMA tiles per wavefront along m and n
  constexpr int CPAD = TN + 4;               // staged output row stride (floats)
  constexpr int STAGE = (TM + TN) * GPAD;    // halfwords of one operand stage
  static_assert((TM / 2) * CPAD * 4 <= 2 * STAGE * 2, "half an output tile must fit in the operand stages");
  // two stages of operand tiles (the next K step is loaded into registers while the MFMAs run on
  // the current one); after the K loop the same memory stages half of the output tile at a time
  __shared__ __attribute__((aligned(16))) uint16_t smem[2][STAGE];
  __shared__ float se[2 * TM * SEED_J];  // start / goal rows of the block (GEMM_SEED_TRAJ)
  float* sC = reinterpret_cast<float*>(&smem[0][0]);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n_tiles_n = (g.N + TN - 1) / TN;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int m0 = (tile / n_tiles_n) * TM, n0 = (tile % n_tiles_n) * TN;
  if (g.epilogue == GEMM_SEED_TRAJ) {
    // read before the K loop, whose barriers publish them
    for (int i = tid; i < 2 * TM * SEED_J; i += 256) {
      const int h = i / (TM * SEED_J), q = i - h * TM * SEED_J;
      const int64_t o = (int64_t)m0 * SEED_J + q;
      se[i] = o < (int64_t)g.M * SEED_J ? (h ? g.goal : g.start)[o] : 0.f;
    }
  }
  const int wm = (wave & 1) * (TM / 2), wn = (wave >> 1) * (TN / 2);
  const bool a_vec = (g.sak & 7) == 0 && (reinterpret_cast<uintptr_t>(g.A) & 15) == 0;
  const bool b_vec = (g.sbk & 7) == 0 && (reinterpret_cast<uintptr_t>(g.B) & 15) == 0;
  // operand rows c * 64 .. c * 64 + 63 of the tile at k step k0
  auto load_a = [&](int c, int k0) {
    if constexpr (A_K) return load_kc(g.A, g.sam, m0 + 64 * c, g.M, k0, tid);
    else return load_rc(g.A, g.sak, m0 + 64 * c, g.M, k0, a_vec, tid);
  };
  auto load_b = [&](int c, int k0) {
    if constexpr (B_N) return load_rc(g.B, g.sbk, n0 + 64 * c, g.N, k0, b_vec, tid);
    else return load_kc(g.B, g.sbn, n0 + 64 * c, g.N, k0, tid);
  };
  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // the output columns of this thread in the write-back (the same for every row it writes): their
  // bias, loaded before the K loop so that its latency is hidden there
  constexpr int CG = TN / 4;                 // 4-column groups per row
  const int cc = (tid % CG) * 4;
  float bias4[4] = {0.f, 0.f, 0.f, 0.f};
  if (g.bias) {
    const int nb = n0 + cc;
    if (nb + 3 < g.N && ((reinterpret_cast<uintptr_t>(g.bias + nb)) & 15) == 0) {
      const float4 b4 = *reinterpret_cast<const float4*>(g.bias + nb);
      bias4[0] = b4.x; bias4[1] = b4.y; bias4[2] = b4.z; bias4[3] = b4.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) bias4[e] = nb + e < g.N ? g.bias[nb + e] : 0.f;
    }
  }

  Frag fa[TM / 64], fb[TN / 64];
#pragma unroll
  for (int c = 0; c < TM / 64; ++c) fa[c] = load_a(c, 0);
#pragma unroll
  for (int c = 0; c < TN / 64; ++c) fb[c] = load_b(c, 0);
  for (int k0 = 0, st = 0; k0 < g.K; k0 += GK, st ^= 1) {
    uint16_t* sA = smem[st];
    uint16_t* sB = smem[st] + TM * GPAD;
#pragma unroll
    for (int c = 0; c < TM / 64; ++c) {
      if constexpr (A_K) store_kc(fa[c], sA + 64 * c * GPAD, tid);
      else store_rc(fa[c], a_vec, sA + 64 * c * GPAD, tid);
    }
#pragma unroll
    for (int c = 0; c < TN / 64; ++c) {
      if constexpr (B_N) store_rc(fb[c], b_vec, sB + 64 * c * GPAD, tid);
      else store_kc(fb[c], sB + 64 * c * GPAD, tid);
    }
    // one barrier per step: the stage written here was last read two steps ago, before the
    // previous barrier
    __syncthreads();
    if (k0 + GK < g.K) {
#pragma unroll
      for (int c = 0; c < TM / 64; ++c) fa[c] = load_a(c, k0 + GK);
#pragma unroll
      for (int c = 0; c < TN / 64; ++c) fb[c] = load_b(c, k0 + GK);
    }
    bf16x8 a[FM], b[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(sA + lds_off(wm + i * 16 + (lane & 15), lane >> 4));
#pragma unroll
    for (int j = 0; j < FN; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(sB + lds_off(wn + j * 16 + (lane & 15), lane >> 4));
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  __syncthreads();

  // write back through LDS, TM / 2 rows at a time (the waves with wm = (TM / 2) h stage half h):
  // thread t takes 4 consecutive columns (t % CG) * 4 of rows t / CG + (256 / CG) rr, so a
  // wavefront stores full row segments of 4 TN bytes per instruction
  const bool vec = (g.ldc & 3) == 0 && (((uintptr_t)g.C | (uintptr_t)g.aux) & 15) == 0 && ((uintptr_t)g.C16 & 7) == 0;
  TrajCol tc[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) tc[e] = traj_col(n0 + cc + e);
  constexpr int RS = 256 / CG;               // rows per sweep of the workgroup
  for (int h = 0; h < 2; ++h) {
    if ((wave & 1) == h) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            sC[(i * 16 + 4 * (lane >> 4) + e) * CPAD + wn + j * 16 + (lane & 15)] = acc[i][j][e];
    }
    lds_barrier();
#pragma unroll
    for (int rr = 0; rr < (TM / 2) / RS; ++rr) {
      const int r = tid / CG + RS * rr, m = m0 + (TM / 2) * h + r;
      const int nb = n0 + cc;
      if (m >= g.M || nb >= g.N) continue;
      const int64_t o = (int64_t)m * g.ldc + nb;
      const float4 t4 = *reinterpret_cast<const float4*>(sC + r * CPAD + cc);
      float v[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] += bias4[e];
      if (vec && nb + 3 < g.N) {
        if (g.epilogue == GEMM_GELU) {
          if (g.aux) *reinterpret_cast<float4*>(g.aux + o) = make_float4(v[0], v[1], v[2], v[3]);
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = gelu_f(v[e]);
        } else if (g.epilogue == GEMM_GELU_GRAD) {
          const float4 z = *reinterpret_cast<const float4*>(g.aux + o);
          v[0] *= gelu_grad_f(z.x); v[1] *= gelu_grad_f(z.y); v[2] *= gelu_grad_f(z.z); v[3] *= gelu_grad_f(z.w);
        } else if (g.epilogue == GEMM_SEED_TRAJ) {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = seed_traj_value<TM>(se, (TM / 2) * h + r, tc[e], v[e]);
        }
        if (g.C) *reinterpret_cast<float4*>(g.C + o) = make_float4(v[0], v[1], v[2], v[3]);
        if (g.C16) {
          uint2 q;
          q.x = to_bf16(v[0]) | ((uint32_t)to_bf16(v[1]) << 16);
          q.y = to_bf16(v[2]) | ((uint32_t)to_bf16(v[3]) << 16);
          *reinterpret_cast<uint2*>(g.C16 + o) = q;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (nb + e >= g.N) break;
          float w = v[e];
          if (g.epilogue == GEMM_GELU) {
            if (g.aux) g.aux[o + e] = w;
            w = gelu_f(w);
          } else if (g.epilogue == GEMM_GELU_GRAD) {
            w *= gelu_grad_f(g.aux[o + e]);
          } else if (g.epilogue == GEMM_SEED_TRAJ) {
            w = seed_traj_value<TM>(se, (TM / 2) * h + r, tc[e], w);
          }
          if (g.C) g.C[o + e] = w;
          if (g.C16) g.C16[o + e] = to_bf16(w);
        }
      }
    }
    lds_barrier();  // the staged half has been read before the next one overwrites it
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

// inverse of k_seed_traj over m trajectories per problem: dev = traj - line, with the same line
// (start and goal exactly at the ends)
__global__ __launch_bounds__(256) void k_seed_dev(int64_t total, int m, const float* __restrict__ traj,
                                                  const float* __restrict__ start, const float* __restrict__ goal,
                                                  float* __restrict__ dev) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t r = i / ((int64_t)m * SEED_TRAJ);
  const int k = (int)(i % SEED_TRAJ);
  const int j = k % SEED_J, t = k / SEED_J;
  const float s0 = start[r * SEED_J + j], g0 = goal[r * SEED_J + j];
  const float line = fmaf(g0 - s0, (float)t / (float)(SEED_T - 1), s0);
  dev[i] = traj[i] - (t == 0 ? s0 : (t == SEED_T - 1 ? g0 : line));
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

// one block per 64 columns: each of the 16 wavefronts sums every 16th row over the block's columns
// (one coalesced 256-byte row segment per load, four independent partial sums in flight), then the
// 16 partial sums are added in LDS
__global__ __launch_bounds__(1024) void k_column_sum(int M, int N, const float* __restrict__ X, int64_t ldx,
                                                     float* __restrict__ out) {
  __shared__ float part[16][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  if (n < N) {
    int m = wv;
    for (; m + 48 < M; m += 64) {
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] += X[(int64_t)(m + 16 * u) * ldx + n];
    }
    for (; m < M; m += 16) s[0] += X[(int64_t)m * ldx + n];
  }
  part[wv][lane] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  if (wv == 0 && n < N) {
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += part[w][lane];
    out[n] = t;
  }
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
  hipLaunchKernelGGL(k_features, dim3(nblocks((int64_t)n * (SEED_IN_PAD / 8), 256)), dim3(256), 0, s, n, start, goal,
                     occ, x);
  return hipGetLastError();
}

template <int TM, int TN>
static hipError_t launch_gemm_tiles(hipStream_t s, const GemmArgs& g, bool a_k, bool b_n) {
  const int64_t tiles = (int64_t)nblocks(g.M, TM) * nblocks(g.N, TN);
  if (tiles > INT32_MAX) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tiles), block(256);
  if (a_k && b_n) hipLaunchKernelGGL((k_gemm_bf16<true, true, TM, TN>), grid, block, 0, s, g);
  else if (a_k) hipLaunchKernelGGL((k_gemm_bf16<true, false, TM, TN>), grid, block, 0, s, g);
  else if (b_n) hipLaunchKernelGGL((k_gemm_bf16<false, true, TM, TN>), grid, block, 0, s, g);
  else hipLaunchKernelGGL((k_gemm_bf16<false, false, TM, TN>), grid, block, 0, s, g);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(hipStream_t s, const GemmArgs& g, bool a_k, bool b_n) {
  // 128 x 128 tiles once they still give every CU several workgroups (large batches: inference);
  // 64 x 64 tiles otherwise (training batches)
  // (A with k contiguous: the forward layers; the transposed-A instantiation would not fit three
  // wavefronts per SIMD)
  const int64_t big_tiles = (int64_t)nblocks(g.M, 128) * nblocks(g.N, 128);
  if (a_k && big_tiles >= GEMM_BIG_TILES_MIN) return launch_gemm_tiles<128, 128>(s, g, a_k, b_n);
  return launch_gemm_tiles<64, 64>(s, g, a_k, b_n);
}

hipError_t launch_seed_traj(hipStream_t s, int n, const float* y, const float* start, const float* goal, float* out) {
  hipLaunchKernelGGL(k_seed_traj, dim3(nblocks((int64_t)n * SEED_OUT, 256)), dim3(256), 0, s, n, y, start, goal, out);
  return hipGetLastError();
}

hipError_t launch_seed_dev(hipStream_t s, int n, int m, const float* traj, const float* start, const float* goal,
                           float* dev) {
  const int64_t total = (int64_t)n * m * SEED_TRAJ;
  hipLaunchKernelGGL(k_seed_dev, dim3(nblocks(total, 256)), dim3(256), 0, s, total, m, traj, start, goal, dev);
  return hipGetLastError();
}

hipError_t launch_seed_loss(hipStream_t s, int n, const float* y, const float* tgt, const float* valid, float coef,
                            double* per_problem, int32_t* assign, float* dy, double inv_valid, double* loss) {
  hipLaunchKernelGGL(k_seed_loss, dim3(n), dim3(64), 0, s, y, tgt, valid, coef, per_problem, assign, dy);
  hipLaunchKernelGGL(k_seed_loss_total, dim3(1), dim3(64), 0, s, per_problem, n, inv_valid, loss);
  return hipGetLastError();
}

hipError_t launch_column_sum(hipStream_t s, int M, int N, const float* X, int64_t ldx, float* out) {
  hipLaunchKernelGGL(k_column_sum, dim3(nblocks(N, 64)), dim3(1024), 0, s, M, N, X, ldx, out);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, int64_t n, float* w, uint16_t* w16, const float* g, float* m, float* v,
                       const AdamArgs& a) {
  hipLaunchKernelGGL(k_adam, dim3(nblocks(n, 256)), dim3(256), 0, s, n, w, w16, g, m, v, a);
  return hipGetLastError();
}

}  // namespace vapr
