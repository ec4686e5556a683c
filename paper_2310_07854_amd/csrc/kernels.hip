// HIP kernels for gfx950 of one trajectory-optimisation iteration (Sec. III-B):
//   k_fk          step (2) forward kinematics -> link poses L, sphere centres S, bound cost
//   k_sphere_cost step (3) world (oriented cuboids) and self-pair costs -> distances D, gradients G
//   k_swept       step (3), trajectory optimisation: swept world term between consecutive
//                 timesteps -> swept gradients X, swept cost
//   k_reduce      step (4) aggregation into FP64 trajectory-candidate costs
//   k_adjoint     step (5) reverse accumulation down the chain -> joint gradients J
//   k_optimizer   steps (6), (7), (1): line-search selection, L-BFGS update, next candidates
// plus the element-wise codec and the workspace repacking used for inspection.
//
// Mapping: one configuration per lane, 64 configurations per wavefront; the stored tensors are
// tiled per wavefront (layout.hpp) so every tensor access of a wavefront is 256 contiguous bytes.
// Robot tables and cuboids are read with wave-uniform addresses, which the compiler turns into
// scalar loads: the inner cuboid loop runs on SGPR operands with no LDS traffic.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <stdint.h>

#include "codec.hpp"
#include "kernels.hpp"
#include "layout.hpp"

namespace vapr {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workspace header: the forward pass's last kernel writes it (first thread of block 0, plain vector
// stores); the consumers compare context id and pass number before reading the workspace.
__device__ __forceinline__ void ws_stamp(const WsStamp& st) {
  if (st.hdr && blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < WH_WORDS; ++i) st.hdr[i] = st.w[i];
  }
}
// true when the workspace holds the forward pass the host expects; otherwise the first thread of
// block 0 raises the context's stale-workspace flag
__device__ __forceinline__ bool ws_current(const WsCheck& ck) {
  if (!ck.hdr) return true;
  const bool ok = ck.hdr[WH_CTX] == ck.ctx && ck.hdr[WH_GEN] == ck.gen;
  if (!ok && blockIdx.x == 0 && threadIdx.x == 0) *ck.status = 1u;
  return ok;
}

// Read-only tables (robot, cuboids) are read through the constant address space: they are never
// written while a kernel runs, so wave-uniform reads become scalar (SMEM) loads into SGPRs.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)p;
}
// sphere s of the robot table: (cx, cy, cz, r)
__device__ __forceinline__ float4 sphere_of(const float4* sph, int s) {
  const cptr<float> p = as_const(reinterpret_cast<const float*>(sph)) + 4 * s;
  return make_float4(p[0], p[1], p[2], p[3]);
}

// ---- stored-tensor group access (format dispatched once per group, wave-uniform) -------------

// A lane's view of a stored tensor: plane p of the lane's configuration is base[p * 64].  The same
// formula serves the tensor in HBM (base = block start + lane) and a block staged in LDS.
__device__ __forceinline__ uint32_t* lane_base(const TV& t, int64_t b) {
  return t.p + ((b >> 6) * t.P) * 64 + (b & 63);
}

// values of a group after a round trip through an emulated ExMy type (codes then values)
template <int N>
__device__ __forceinline__ void exmy_group(const TV& t, float (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = exmy_round(v[i] * t.inv, t.xe, t.xm) * t.scale;
}

// ---- packed ExMy groups: group `slot` of N values occupies ceil(N / q) words, q = floor(32 / b) ------

template <int N>
__device__ __forceinline__ void pxm_store(const TV& t, uint32_t* lane, int slot, const float (&v)[N]) {
  const int dw = (N + t.pq - 1) / t.pq;
  pxm_store_words<N>(v, t.xe, t.xm, t.pq, t.inv, lane + slot * dw * 64, 64);
}

template <int N>
__device__ __forceinline__ void pxm_load(const TV& t, const uint32_t* lane, int slot, float (&v)[N]) {
  const int dw = (N + t.pq - 1) / t.pq;
  pxm_load_words<N>(lane + slot * dw * 64, 64, t.xe, t.xm, t.pq, t.scale, v);
}

template <int N>
__device__ __forceinline__ float pxm_load_elem(const TV& t, const uint32_t* lane, int slot, int pos) {
  const int q = t.pq, b = 1 + t.xe + t.xm;
  const int dw = (N + q - 1) / q;
  const uint32_t w = lane[(slot * dw + pos / q) * 64];
  const uint32_t mask = b >= 32 ? 0xffffffffu : (1u << b) - 1u;
  return exmy_decode((w >> ((pos % q) * b)) & mask, t.xe, t.xm) * t.scale;
}

// ---- format-dispatched group access ---------------------------------------------------------------

template <int F, int N>
__device__ __forceinline__ void store_group_t(const TV& t, int64_t b, int slot, const float (&v_in)[N]) {
  if constexpr (F == PXM) {
    pxm_store<N>(t, lane_base(t, b), slot, v_in);
  } else {
    constexpr int DW = group_dwords(F, N);
    uint32_t w[DW];
    encode_group<F, N>(v_in, t.inv, w);
    uint32_t* base = lane_base(t, b) + slot * DW * 64;
#pragma unroll
    for (int k = 0; k < DW; ++k) base[k * 64] = w[k];
  }
}

template <int N>
__device__ __forceinline__ void store_group(const TV& t, int64_t b, int slot, const float (&v)[N]) {
  switch (t.fmt) {
    case F32: store_group_t<F32, N>(t, b, slot, v); break;
    case F16: store_group_t<F16, N>(t, b, slot, v); break;
    case BF16: store_group_t<BF16, N>(t, b, slot, v); break;
    case E4M3: store_group_t<E4M3, N>(t, b, slot, v); break;
    case E5M2: store_group_t<E5M2, N>(t, b, slot, v); break;
    case E3M2: store_group_t<E3M2, N>(t, b, slot, v); break;
    case E2M1: store_group_t<E2M1, N>(t, b, slot, v); break;
    default: store_group_t<PXM, N>(t, b, slot, v); break;
  }
}

// A group of N values produced one at a time by get(i), for groups too large to hold at once: the
// fixed formats pack every 16 values into whole dwords, so the group is encoded and stored 16 values
// at a time (the same words as the whole group's); packed ExMy codes go word by word.
template <int F, int N, typename Get>
__device__ __forceinline__ void store_group_from_t(const TV& t, int64_t b, int slot, Get get) {
  static_assert(N % 16 == 0, "16-value chunks");
  uint32_t* lane = lane_base(t, b);
  if constexpr (F == PXM) {
    const int q = t.pq, bits = 1 + t.xe + t.xm;
    uint32_t* base = lane + slot * ((N + q - 1) / q) * 64;
    uint32_t acc = 0u;
    int c = 0, k = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      acc |= exmy_encode(get(i) * t.inv, t.xe, t.xm) << (c * bits);
      if (++c == q) {
        base[k * 64] = acc;
        ++k;
        acc = 0u;
        c = 0;
      }
    }
    if (c) base[k * 64] = acc;
  } else {
    constexpr int DW = group_dwords(F, N), DW16 = group_dwords(F, 16);
    static_assert(DW == DW16 * (N / 16), "whole dwords per 16 values");
    uint32_t* base = lane + slot * DW * 64;
#pragma unroll
    for (int k = 0; k < N / 16; ++k) {
      float v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = get(16 * k + i);
      uint32_t w[DW16];
      encode_group<F, 16>(v, t.inv, w);
#pragma unroll
      for (int d = 0; d < DW16; ++d) base[(k * DW16 + d) * 64] = w[d];
    }
  }
}

template <int N, typename Get>
__device__ __forceinline__ void store_group_from(const TV& t, int64_t b, int slot, Get get) {
  switch (t.fmt) {
    case F32: store_group_from_t<F32, N>(t, b, slot, get); break;
    case F16: store_group_from_t<F16, N>(t, b, slot, get); break;
    case BF16: store_group_from_t<BF16, N>(t, b, slot, get); break;
    case E4M3: store_group_from_t<E4M3, N>(t, b, slot, get); break;
    case E5M2: store_group_from_t<E5M2, N>(t, b, slot, get); break;
    case E3M2: store_group_from_t<E3M2, N>(t, b, slot, get); break;
    case E2M1: store_group_from_t<E2M1, N>(t, b, slot, get); break;
    default: store_group_from_t<PXM, N>(t, b, slot, get); break;
  }
}

// group `slot` of N values of tensor t, from a lane base (HBM or an LDS image of the same layout)
template <int F, int N>
__device__ __forceinline__ void load_group_at(const TV& t, const uint32_t* base, int slot, float (&v)[N]) {
  if constexpr (F == PXM) {
    pxm_load<N>(t, base, slot, v);
  } else {
    constexpr int DW = group_dwords(F, N);
    uint32_t w[DW];
#pragma unroll
    for (int k = 0; k < DW; ++k) w[k] = base[(slot * DW + k) * 64];
    decode_group<F, N>(w, t.scale, v);
  }
}

template <int N>
__device__ __forceinline__ void load_group_fmt(const TV& t, const uint32_t* base, int slot, float (&v)[N]) {
  switch (t.fmt) {
    case F32: load_group_at<F32, N>(t, base, slot, v); break;
    case F16: load_group_at<F16, N>(t, base, slot, v); break;
    case BF16: load_group_at<BF16, N>(t, base, slot, v); break;
    case E4M3: load_group_at<E4M3, N>(t, base, slot, v); break;
    case E5M2: load_group_at<E5M2, N>(t, base, slot, v); break;
    case E3M2: load_group_at<E3M2, N>(t, base, slot, v); break;
    case E2M1: load_group_at<E2M1, N>(t, base, slot, v); break;
    default: load_group_at<PXM, N>(t, base, slot, v); break;
  }
}

template <int N>
__device__ __forceinline__ void load_group(const TV& t, int64_t b, int slot, float (&v)[N]) {
  load_group_fmt<N>(t, lane_base(t, b), slot, v);
}

// stored value of element `pos` of the group of N values in slot `slot`
template <int F, int N>
__device__ __forceinline__ float load_elem_at(const TV& t, const uint32_t* base, int slot, int pos) {
  if constexpr (F == PXM) {
    return pxm_load_elem<N>(t, base, slot, pos);
  } else {
    constexpr int DW = group_dwords(F, N);
    constexpr int BITS = Fmt<F>::BITS;
    const int bit = pos * BITS, wi = bit >> 5, sh = bit & 31;
    uint64_t v = base[(slot * DW + wi) * 64];
    if (sh + BITS > 32) v |= (uint64_t)base[(slot * DW + wi + 1) * 64] << 32;
    const uint32_t code = (uint32_t)(v >> sh) & (BITS == 32 ? 0xffffffffu : ((1u << BITS) - 1u));
    return decode_one<F>(code, t.scale);
  }
}

template <int N>
__device__ __forceinline__ float load_elem_fmt(const TV& t, const uint32_t* base, int slot, int pos) {
  switch (t.fmt) {
    case F32: return load_elem_at<F32, N>(t, base, slot, pos);
    case F16: return load_elem_at<F16, N>(t, base, slot, pos);
    case BF16: return load_elem_at<BF16, N>(t, base, slot, pos);
    case E4M3: return load_elem_at<E4M3, N>(t, base, slot, pos);
    case E5M2: return load_elem_at<E5M2, N>(t, base, slot, pos);
    case E3M2: return load_elem_at<E3M2, N>(t, base, slot, pos);
    case E2M1: return load_elem_at<E2M1, N>(t, base, slot, pos);
    default: return load_elem_at<PXM, N>(t, base, slot, pos);
  }
}

template <int N>
__device__ __forceinline__ float load_elem(const TV& t, int64_t b, int slot, int pos) {
  return load_elem_fmt<N>(t, lane_base(t, b), slot, pos);
}

// stored values of a group after a round trip through the format (what a reader will see)
template <int F, int N>
__device__ __forceinline__ void roundtrip_t(const TV& t, float (&v)[N]) {
  if constexpr (F == PXM) {
    exmy_group<N>(t, v);
  } else {
    constexpr int DW = group_dwords(F, N);
    uint32_t w[DW];
    encode_group<F, N>(v, t.inv, w);
    decode_group<F, N>(w, t.scale, v);
  }
}

template <int N>
__device__ __forceinline__ void roundtrip(const TV& t, float (&v)[N]) {
  switch (t.fmt) {
    case F32: roundtrip_t<F32, N>(t, v); break;
    case F16: roundtrip_t<F16, N>(t, v); break;
    case BF16: roundtrip_t<BF16, N>(t, v); break;
    case E4M3: roundtrip_t<E4M3, N>(t, v); break;
    case E5M2: roundtrip_t<E5M2, N>(t, v); break;
    case E3M2: roundtrip_t<E3M2, N>(t, v); break;
    case E2M1: roundtrip_t<E2M1, N>(t, v); break;
    default: roundtrip_t<PXM, N>(t, v); break;
  }
}

// ---- serial chain, link poses of a tile in LDS ---------------------------------------------------

// LDS image of the poses of links 1..8 of a 64-configuration tile: value k of link l ([R | t]
// row-major) for lane j is word ((l - 1) * 12 + k) * 64 + j, so a wavefront-wide access touches 64
// consecutive words, one per bank.  The base, link 0, is the identity and is not stored.
constexpr int TILE_POSE_WORDS = N_FIXED * LINK_VALUES * 64;

// T_0 = I, T_j = T_{j-1} F_j Rz(q_j) (j = 1..7), T_8 = T_7 F_8, each link written to the tile as
// it is formed.
__device__ __forceinline__ void chain_to_tile(const float* __restrict__ fixed, const float (&qv)[N_JOINTS],
                                              float* tile, int lane) {
  float R[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
  float t[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int l = 0; l < N_FIXED; ++l) {
    const cptr<float> F = as_const(fixed) + l * LINK_VALUES;
    float nR[9], nt[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j < 3; ++j)
        nR[i * 3 + j] = fmaf(R[i * 3 + 0], F[0 * 4 + j], fmaf(R[i * 3 + 1], F[1 * 4 + j], R[i * 3 + 2] * F[2 * 4 + j]));
      nt[i] = fmaf(R[i * 3 + 0], F[3], fmaf(R[i * 3 + 1], F[7], fmaf(R[i * 3 + 2], F[11], t[i])));
    }
    if (l < N_JOINTS) {
      float s, c;
      sincosf(qv[l], &s, &c);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float c0 = nR[i * 3 + 0], c1 = nR[i * 3 + 1];
        nR[i * 3 + 0] = fmaf(c, c0, s * c1);
        nR[i * 3 + 1] = fmaf(c, c1, -s * c0);
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = nR[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) t[i] = nt[i];
    float* out = tile + l * LINK_VALUES * 64 + lane;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      out[(i * 4 + 0) * 64] = R[i * 3 + 0];
      out[(i * 4 + 1) * 64] = R[i * 3 + 1];
      out[(i * 4 + 2) * 64] = R[i * 3 + 2];
      out[(i * 4 + 3) * 64] = t[i];
    }
  }
}

// pose of link l (1..8) of this lane
__device__ __forceinline__ void pose_from_tile(const float* tile, int l, int lane, float (&T)[LINK_VALUES]) {
  const float* p = tile + (l - 1) * LINK_VALUES * 64 + lane;
#pragma unroll
  for (int k = 0; k < LINK_VALUES; ++k) T[k] = p[k * 64];
}

typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bound_cost(const RobotArgs& R, const float (&qv)[N_JOINTS]) {
  float bc = 0.f;
#pragma unroll
  for (int j = 0; j < N_JOINTS; ++j) {
    const float over = fmaxf(qv[j] - R.q_hi[j], 0.f), under = fmaxf(R.q_lo[j] - qv[j], 0.f);
    bc = fmaf(over, over, fmaf(under, under, bc));
  }
  return bc;
}

// ---- K1: forward kinematics ---------------------------------------------------------------------

// Row c (R_c0, R_c1, R_c2, t_c) of the pose of link l (1..8), read as explicit LDS instructions so
// that it stays inside its wave-uniform branch (the compiler would otherwise hoist the guarded reads
// of every sphere out of their branches and keep all of them live): two ds_read2st64_b32 (two words
// 64 words apart each), then a wait.  Link 0 is the identity.
__device__ __forceinline__ void pose_row_guarded(const float* tile, int l, int c, int lane, float (&r)[4]) {
  if (l == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = k == c ? 1.f : 0.f;
    return;
  }
  const uint32_t addr = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float*)(
      tile + ((l - 1) * LINK_VALUES + c * 4) * 64 + lane);
  f32x2 a, b;
  asm volatile(
      "ds_read2st64_b32 %0, %2 offset0:0 offset1:1\n"
      "ds_read2st64_b32 %1, %2 offset0:2 offset1:3\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a), "=&v"(b)
      : "v"(addr)
      : "memory");
  r[0] = a.x; r[1] = a.y; r[2] = b.x; r[3] = b.y;
}

// World centres of sphere group g (p_s = R_l c_s + t_l), one coordinate plane at a time: a plane
// needs only its row of each pose, so its 16 values are the only ones held, and it is stored as
// soon as it is formed.  The row is re-read from the tile only when the link changes from one
// sphere to the next; robots list their spheres link by link, so a group reads two or three poses.
// The zero padding sits on link 0.
template <int FS>
__device__ __forceinline__ void place_group(const RobotArgs& R, const TV& S, int64_t b, int g, const float* tile,
                                            int lane) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float v[SPH_GROUP];
    float r[4];
    int cur = as_const(R.link)[g * SPH_GROUP];
    pose_row_guarded(tile, cur, c, lane, r);
#pragma unroll
    for (int i = 0; i < SPH_GROUP; ++i) {
      const int s = g * SPH_GROUP + i;
      const float4 cs = sphere_of(R.sph, s);
      const int l = as_const(R.link)[s];
      if (l != cur) {
        cur = l;
        pose_row_guarded(tile, l, c, lane, r);
      }
      v[i] = fmaf(r[0], cs.x, fmaf(r[1], cs.y, fmaf(r[2], cs.z, r[3])));
      // computed here, not sunk past the next pose change (which would keep every row version live)
      asm volatile("" : "+v"(v[i]));
    }
    store_group_t<FS, SPH_GROUP>(S, b, g * 3 + c, v);
  }
}

// One block of four wavefronts per 64-configuration tile: wavefront 0 runs the chain into LDS, then
// the sphere groups and the two link-pose groups are shared out over the wavefronts.
template <int FS>
__global__ __launch_bounds__(256) void k_fk(const float* __restrict__ q, RobotArgs R, TV L, TV S,
                                            float* __restrict__ bound, int64_t B, int store_L,
                                            const float* __restrict__ goal, float* __restrict__ posec,
                                            int64_t cfg_per_world, CostArgs cp) {
  __shared__ float tile[TILE_POSE_WORDS];
  const int wave = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 64 + lane;
  const bool live = b < B;
  if (wave == 0) {
    float qv[N_JOINTS];
#pragma unroll
    for (int j = 0; j < N_JOINTS; ++j) qv[j] = live ? q[b * N_JOINTS + j] : 0.f;
    if (live) bound[b] = bound_cost(R, qv);
    chain_to_tile(R.fixed, qv, tile, lane);
    if (goal && live) {
      // pose cost of link 8 against the goal of the configuration's world (read back from this
      // lane's own tile entries)
      const float* g = goal + (b / cfg_per_world) * LINK_VALUES;
      float sp = 0.f, sr = 0.f;
#pragma unroll
      for (int k = 0; k < LINK_VALUES; ++k) {
        const float e = tile[((N_FIXED - 1) * LINK_VALUES + k) * 64 + lane] - g[k];
        if ((k & 3) == 3) sp = fmaf(e, e, sp);
        else sr = fmaf(e, e, sr);
      }
      posec[b] = fmaf(cp.w_gp, sp, cp.w_gr * sr);
    }
  }
  __syncthreads();
  if (!live) return;
  const int ng = uniform(R.n_groups);
  const int n_items = ng + (store_L ? L_GROUPS : 0);
  // items: sphere groups, then link-pose groups; wavefront 0 (which ran the chain) starts at item 3
  for (int it = (wave + 3) & 3; it < n_items; it += 4) {
    if (it < ng) {
      place_group<FS>(R, S, b, it, tile, lane);
    } else {
      const int gr = it - ng;
      const float* src = tile + gr * L_GROUP * 64 + lane;
      store_group_from<L_GROUP>(L, b, gr, [&](int i) { return src[i * 64]; });
    }
  }
}

// ---- K2: sphere costs ---------------------------------------------------------------------------

// Signed distance to one cuboid and its gradient (per-lane cuboid).
__device__ __forceinline__ void cuboid_sd_grad(const float* __restrict__ bx, float px, float py, float pz, float& sd,
                                               float& gx, float& gy, float& gz) {
  const float4 b0 = *reinterpret_cast<const float4*>(bx);
  const float4 b1 = *reinterpret_cast<const float4*>(bx + 4);
  const float4 b2 = *reinterpret_cast<const float4*>(bx + 8);
  const float4 b3 = *reinterpret_cast<const float4*>(bx + 12);
  const float A[9] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w, b2.x};
  const float o[3] = {b2.y, b2.z, b2.w};
  const float h[3] = {b3.x, b3.y, b3.z};
  float u[3], a[3], m[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u[i] = fmaf(A[i * 3 + 0], px, fmaf(A[i * 3 + 1], py, A[i * 3 + 2] * pz)) - o[i];
    a[i] = fabsf(u[i]) - h[i];
    m[i] = fmaxf(a[i], 0.f);
  }
  const float n2 = fmaf(m[0], m[0], fmaf(m[1], m[1], m[2] * m[2]));
  float n[3];
  if (n2 > 1e-24f) {
    // hardware reciprocal square root (about 1 ulp): distance and unit direction in one step, in
    // place of a correctly rounded square root and division (about 15 instructions more)
    const float inv = __builtin_amdgcn_rsqf(n2);
    sd = n2 * inv;
#pragma unroll
    for (int i = 0; i < 3; ++i) n[i] = (u[i] >= 0.f ? m[i] : -m[i]) * inv;
  } else if (n2 > 0.f) {
    // within 1e-12 of the surface (n2 may be subnormal, which the hardware rsq flushes)
    sd = sqrtf(n2);
    const float inv = 1.0f / sd;
#pragma unroll
    for (int i = 0; i < 3; ++i) n[i] = (u[i] >= 0.f ? m[i] : -m[i]) * inv;
  } else {
    const int ax = (a[0] >= a[1] && a[0] >= a[2]) ? 0 : (a[1] >= a[2] ? 1 : 2);
    sd = ax == 0 ? a[0] : (ax == 1 ? a[1] : a[2]);
    const float uu = ax == 0 ? u[0] : (ax == 1 ? u[1] : u[2]);
    const float sg = uu >= 0.f ? 1.f : -1.f;
    n[0] = ax == 0 ? sg : 0.f;
    n[1] = ax == 1 ? sg : 0.f;
    n[2] = ax == 2 ? sg : 0.f;
  }
  // gradient R n = A^T n
  gx = fmaf(A[0], n[0], fmaf(A[3], n[1], A[6] * n[2]));
  gy = fmaf(A[1], n[0], fmaf(A[4], n[1], A[7] * n[2]));
  gz = fmaf(A[2], n[0], fmaf(A[5], n[1], A[8] * n[2]));
}

// A sphere whose closest-cuboid key exceeds (eta + r)^2 by a margin far above the rounding of the
// key and of the exact distance is out of reach: its activation depth is exactly 0 and its gradient
// +0, whatever the exact distance computation would give, so that computation is skipped.
__device__ __forceinline__ bool out_of_reach(float key, float eta, float r) {
  const float e = eta + r;
  return key > e * e * 1.0001f;
}

// Closest cuboid of NA spheres against the K cuboids of one world.  The comparison key is
// |max(a,0)|^2 outside (> 0) and max_i a_i inside (<= 0), a monotone function of the signed
// distance, so no square root is taken per pair; the first index wins ties.
template <int NA, int N = SPH_GROUP>
__device__ __forceinline__ void closest_cuboids(cptr<float> wbox, int K, const float (&px)[N], const float (&py)[N],
                                                const float (&pz)[N], float (&best)[N], int (&bk)[N]) {
  for (int k = 0; k < K; ++k) {
    const cptr<float> bx = wbox + k * 16;
    const float A0 = bx[0], A1 = bx[1], A2 = bx[2], A3 = bx[3], A4 = bx[4], A5 = bx[5], A6 = bx[6], A7 = bx[7],
                A8 = bx[8];
    const float o0 = bx[9], o1 = bx[10], o2 = bx[11], h0 = bx[12], h1 = bx[13], h2 = bx[14];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      // the same rounding as the per-lane key of the culled path
      const float u0 = fmaf(A0, px[i], fmaf(A1, py[i], fmaf(A2, pz[i], -o0)));
      const float u1 = fmaf(A3, px[i], fmaf(A4, py[i], fmaf(A5, pz[i], -o1)));
      const float u2 = fmaf(A6, px[i], fmaf(A7, py[i], fmaf(A8, pz[i], -o2)));
      const float a0 = fabsf(u0) - h0, a1 = fabsf(u1) - h1, a2 = fabsf(u2) - h2;
      const float m0 = fmaxf(a0, 0.f), m1 = fmaxf(a1, 0.f), m2 = fmaxf(a2, 0.f);
      const float key = fmaf(m0, m0, fmaf(m1, m1, fmaf(m2, m2, fminf(fmaxf(fmaxf(a0, a1), a2), 0.f))));
      if (key < best[i]) {
        best[i] = key;
        bk[i] = k;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_sphere_cost(RobotArgs R, WorldArgs W, TV S, TV D, TV G,
                                                     float* __restrict__ selfc, ShapeArgs sh, CostArgs cp) {
  const int64_t wave_first = (int64_t)blockIdx.x * 256 + uniform(threadIdx.x & ~63);
  if (wave_first >= sh.B) return;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= sh.B) return;
  const int64_t wave_last = (wave_first + 63 < sh.B ? wave_first + 63 : sh.B - 1);
  const int w_lo = uniform((int)(wave_first / sh.cfg_per_world));
  const int w_hi = uniform((int)(wave_last / sh.cfg_per_world));
  const int my_w = (int)(b / sh.cfg_per_world);
  const int K = uniform(W.K);
  const int ng = uniform(R.n_groups);
  const int n_s = uniform(R.n_s);
  float self_acc = 0.f;

  for (int g = 0; g < ng; ++g) {
    float px[SPH_GROUP], py[SPH_GROUP], pz[SPH_GROUP];
    load_group<SPH_GROUP>(S, b, g * 3 + 0, px);
    load_group<SPH_GROUP>(S, b, g * 3 + 1, py);
    load_group<SPH_GROUP>(S, b, g * 3 + 2, pz);
    float best[SPH_GROUP];
    int bk[SPH_GROUP];
#pragma unroll
    for (int i = 0; i < SPH_GROUP; ++i) {
      best[i] = INFINITY;
      bk[i] = 0;
    }
    const int active = uniform(min(SPH_GROUP, n_s - g * SPH_GROUP));
    for (int w = w_lo; w <= w_hi; ++w) {
      if (my_w != w) continue;
      // readfirstlane keeps the address uniform (inside this branch w equals the per-lane my_w)
      const cptr<float> wbox = as_const(W.box) + (int64_t)uniform(w) * K * 16;
      if (active > 12) closest_cuboids<16>(wbox, K, px, py, pz, best, bk);
      else if (active > 8) closest_cuboids<12>(wbox, K, px, py, pz, best, bk);
      else if (active > 4) closest_cuboids<8>(wbox, K, px, py, pz, best, bk);
      else closest_cuboids<4>(wbox, K, px, py, pz, best, bk);
    }

    float dv[SPH_GROUP], gx[SPH_GROUP], gy[SPH_GROUP], gz[SPH_GROUP];
    const float* mybox = W.box + (int64_t)my_w * K * 16;
#pragma unroll
    for (int i = 0; i < SPH_GROUP; ++i) {
      dv[i] = 0.f;
      gx[i] = gy[i] = gz[i] = 0.f;
      const float r = sphere_of(R.sph, g * SPH_GROUP + i).w;
      if (i < active && K > 0 && !out_of_reach(best[i], cp.eta, r)) {
        float sd, nx, ny, nz;
        cuboid_sd_grad(mybox + bk[i] * 16, px[i], py[i], pz[i], sd, nx, ny, nz);
        const float d = fmaxf(cp.eta - (sd - r), 0.f);
        dv[i] = d;
        if (d > 0.f) {
          const float coef = -2.f * cp.w_c * d;
          gx[i] = coef * nx;
          gy[i] = coef * ny;
          gz[i] = coef * nz;
        }
      }
    }
    // self pairs: every pair is visited from both spheres; each visit adds its own sphere's
    // gradient and the lower index adds the cost, so no cross-lane or atomic accumulation is needed
#pragma unroll
    for (int i = 0; i < SPH_GROUP; ++i) {
      if (i >= active) continue;
      const int s = g * SPH_GROUP + i;
      const float rs = sphere_of(R.sph, s).w;
      const int j0 = as_const(R.csr_off)[s], j1 = as_const(R.csr_off)[s + 1];
      for (int j = j0; j < j1; ++j) {
        const int t = as_const(R.csr_nbr)[j];
        const int tg = t / SPH_GROUP, tp = t % SPH_GROUP;
        const float tx = load_elem<SPH_GROUP>(S, b, tg * 3 + 0, tp);
        const float ty = load_elem<SPH_GROUP>(S, b, tg * 3 + 1, tp);
        const float tz = load_elem<SPH_GROUP>(S, b, tg * 3 + 2, tp);
        const float dx = px[i] - tx, dy = py[i] - ty, dz = pz[i] - tz;
        const float dist = sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        const float e = dist - rs - sphere_of(R.sph, t).w;
        const float act = fmaxf(cp.eta - e, 0.f);
        if (act > 0.f) {
          if (dist > 0.f) {
            const float coef = -2.f * cp.w_s * act / dist;
            gx[i] = fmaf(coef, dx, gx[i]);
            gy[i] = fmaf(coef, dy, gy[i]);
            gz[i] = fmaf(coef, dz, gz[i]);
          }
          if (s < t) self_acc = fmaf(act, act, self_acc);
        }
      }
    }
    store_group<SPH_GROUP>(D, b, g, dv);
    store_group<SPH_GROUP>(G, b, g * 3 + 0, gx);
    store_group<SPH_GROUP>(G, b, g * 3 + 1, gy);
    store_group<SPH_GROUP>(G, b, g * 3 + 2, gz);
  }
  selfc[b] = cp.w_s * self_acc;
}

// ---- K2 on a block staged in LDS, with exact cuboid culling -------------------------------------
//
// One workgroup per block of 64 configurations and one wavefront per group of 16 spheres.  Each
// wavefront decodes its own group's stored positions once and leaves them, as FP32, in the block's
// LDS image, where the self-pair partners of any group are read.
//
// Culling: a voxel grid over the region where any cuboid can be within reach holds, per world and
// voxel, a bit per cuboid that may lie within eta + r_max (+ margin) of some point of the voxel.  A
// cuboid without the bit has clearance >= eta for every sphere in the voxel, so it can change
// neither the activation depth (clamped at zero) nor the closest cuboid of an active sphere: the
// result is identical to testing every cuboid.

#ifndef VAPR_CULL_SPHERES
#define VAPR_CULL_SPHERES 8
#endif
// spheres sharing one candidate list (divides 16).  Eight: each gathered cuboid (64 bytes per lane)
// serves eight tests; the longer unions cost fewer instructions than the extra gathers of lists of
// four (measured on trajectory and inverse-kinematics batches; sixteen is slower on trajectories)
constexpr int CQ = VAPR_CULL_SPHERES;


__device__ __forceinline__ int voxel_of(const GridArgs& g, float x, float y, float z) {
  const float fx = (x - g.ox) * g.inv_cell, fy = (y - g.oy) * g.inv_cell, fz = (z - g.oz) * g.inv_cell;
  const float n = (float)g.n;
  // also false for NaN coordinates
  if (!(fx >= 0.f && fx < n && fy >= 0.f && fy < n && fz >= 0.f && fz < n)) return -1;
  return ((int)fz * g.n + (int)fy) * g.n + (int)fx;
}

// one sphere against one cuboid held in registers (A = R^T rows in c0, c1, c2.x; o = c2.yzw;
// h = c3.xyz), running closest-cuboid key; the first index wins ties
__device__ __forceinline__ void cuboid_key_v(const float4& c0, const float4& c1, const float4& c2, const float4& c3,
                                             float px, float py, float pz, int k, float& best, int& bk) {
  const float u0 = fmaf(c0.x, px, fmaf(c0.y, py, fmaf(c0.z, pz, -c2.y)));
  const float u1 = fmaf(c0.w, px, fmaf(c1.x, py, fmaf(c1.y, pz, -c2.z)));
  const float u2 = fmaf(c1.z, px, fmaf(c1.w, py, fmaf(c2.x, pz, -c2.w)));
  const float a0 = fabsf(u0) - c3.x, a1 = fabsf(u1) - c3.y, a2 = fabsf(u2) - c3.z;
  const float m0 = fmaxf(a0, 0.f), m1 = fmaxf(a1, 0.f), m2 = fmaxf(a2, 0.f);
  // |m|^2 outside (max a > 0, the min term is 0) and max a inside (m = 0): the min term goes in as
  // the innermost addend, which gives the same value to the bit as adding it last, one instruction
  // fewer
  const float key = fmaf(m0, m0, fmaf(m1, m1, fmaf(m2, m2, fminf(fmaxf(fmaxf(a0, a1), a2), 0.f))));
  if (key < best) {
    best = key;
    bk = k;
  }
}

// lowest candidate of a lane's list (removed from it) with its cuboid loaded; -1 when empty
__device__ __forceinline__ int pop_cuboid(uint64_t& m, const float* wbox, float4& c0, float4& c1, float4& c2,
                                          float4& c3) {
  if (!m) return -1;
  const int k = __builtin_ctzll(m);
  m &= m - 1;
  const float4* c4 = reinterpret_cast<const float4*>(wbox + k * 16);
  c0 = c4[0];
  c1 = c4[1];
  c2 = c4[2];
  c3 = c4[3];
  return k;
}

// The candidate list m against spheres i0 .. i0 + CQ - 1, cuboid k at base + 16 k (the world's table
// in memory, or the block's LDS copy), two cuboid buffers used in turn so that the next candidate's
// load is in flight while the current one is tested.
template <int N = SPH_GROUP, int Q = CQ>
__device__ __forceinline__ void walk_list(uint64_t m, const float* base, int i0, const float (&px)[N],
                                          const float (&py)[N], const float (&pz)[N], float (&best)[N],
                                          int (&bk)[N]) {
  float4 a0, a1, a2, a3, b0, b1, b2, b3;
  int ka = pop_cuboid(m, base, a0, a1, a2, a3);
  while (ka >= 0) {
    const int kb = pop_cuboid(m, base, b0, b1, b2, b3);
#pragma unroll
    for (int i = i0; i < i0 + Q; ++i) cuboid_key_v(a0, a1, a2, a3, px[i], py[i], pz[i], ka, best[i], bk[i]);
    if (kb < 0) break;
    ka = pop_cuboid(m, base, a0, a1, a2, a3);
#pragma unroll
    for (int i = i0; i < i0 + Q; ++i) cuboid_key_v(b0, b1, b2, b3, px[i], py[i], pz[i], kb, best[i], bk[i]);
  }
}

// NB self-pair visits of sphere s (centre q, radius rs) from its visit list at e: partner centres
// from the block's LDS image (all NB loads issued before the first test), the sphere's gradient
// into g, and the cost of the pairs whose partner has the higher index into acc.  A pair whose
// squared centre distance exceeds the entry's lim2 has an activation of exactly zero.
template <int NB>
__device__ __forceinline__ void pair_visits(cptr<float> e, const float* pos, int lane, int s, float qx, float qy,
                                            float qz, float rs, const CostArgs& cp, float& gx, float& gy,
                                            float& gz, float& acc) {
  float tx[NB], ty[NB], tz[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const float* pp = pos + (unsigned)__float_as_int(e[4 * u]) * 3u * 64u + lane;
    tx[u] = pp[0];
    ty[u] = pp[64];
    tz[u] = pp[128];
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const float dx = qx - tx[u], dy = qy - ty[u], dz = qz - tz[u];
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    if (!(d2 <= e[4 * u + 2])) continue;
    // hardware reciprocal square root (about 1 ulp): distance and unit direction in one step;
    // coincident centres give distance 0 and no gradient
    const float inv = __builtin_amdgcn_rsqf(d2);
    const bool apart = d2 > 0.f;
    const float dist = apart ? d2 * inv : 0.f;
    const float ev = dist - rs - e[4 * u + 1];
    const float act = fmaxf(cp.eta - ev, 0.f);
    if (act > 0.f) {
      const float coef = (-2.f * cp.w_s) * act * inv;
      if (apart) {
        gx = fmaf(coef, dx, gx);
        gy = fmaf(coef, dy, gy);
        gz = fmaf(coef, dz, gz);
      }
      if (s < __float_as_int(e[4 * u])) acc = fmaf(act, act, acc);
    }
  }
}

// Sphere s's whole visit list [j0, j1): four visits at a time, then a pair and a single for the
// remainder (the counts are the same in every lane).
__device__ __forceinline__ void sphere_pair_visits(const RobotArgs& R, const float* pos, int lane, int s, float qx,
                                                   float qy, float qz, float rs, const CostArgs& cp, float& gx,
                                                   float& gy, float& gz, float& acc) {
  const int j0 = as_const(R.pair_off)[s], j1 = as_const(R.pair_off)[s + 1];
  const cptr<float> tab = as_const(reinterpret_cast<const float*>(R.pair_tab));
  const int j4 = j0 + ((j1 - j0) & ~3);
  for (int j = j0; j < j4; j += 4) pair_visits<4>(tab + 4 * j, pos, lane, s, qx, qy, qz, rs, cp, gx, gy, gz, acc);
  int j = j4;
  if ((j1 - j) & 2) {
    pair_visits<2>(tab + 4 * j, pos, lane, s, qx, qy, qz, rs, cp, gx, gy, gz, acc);
    j += 2;
  }
  if (j < j1) pair_visits<1>(tab + 4 * j, pos, lane, s, qx, qy, qz, rs, cp, gx, gy, gz, acc);
}

template <int FS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3))) void k_sphere_cost_blk(RobotArgs R, WorldArgs W, GridArgs Gd, TV S, TV D, TV G,
                                                          float* __restrict__ selfc, ShapeArgs sh, CostArgs cp) {
  extern __shared__ float lds_f[];
  const int lane = threadIdx.x & 63;
  const int g = uniform(threadIdx.x >> 6);
  const int ng = uniform(R.n_groups);
  const int n_s = uniform(R.n_s);
  const int K = uniform(W.K);
  const int64_t blk = blockIdx.x;
  const int64_t b = blk * 64 + lane;
  const bool valid = b < sh.B;
  float* pos = lds_f;                                // sphere s, component c: pos[(s * 3 + c) * 64 + lane]
  float* part = lds_f + n_s * 3 * 64;                // [ng][64] self-cost partials
  float* cub = part + ng * 64;                       // the block's world's cuboids (culled path)
  const int64_t first = blk * 64;
  const int64_t last = (first + 63 < sh.B ? first + 63 : sh.B - 1);
  const int w_lo = uniform((int)(first / sh.cfg_per_world));
  const int w_hi = uniform((int)(last / sh.cfg_per_world));
  // one world for the whole block and at most 64 cuboids: its cuboids go to LDS, read there by the
  // candidate walks and the closest cuboid's distance instead of gathered from memory per lane
  const bool staged = Gd.MW > 0 && Gd.MW <= 2 && w_lo == w_hi;
  if (staged) {
    const float* src = W.box + (int64_t)w_lo * K * 16;
    for (int i = threadIdx.x; i < K * 16; i += blockDim.x) cub[i] = src[i];
  }

  float px[SPH_GROUP], py[SPH_GROUP], pz[SPH_GROUP];
  if (valid) {
    const uint32_t* sb = lane_base(S, b);
    load_group_at<FS, SPH_GROUP>(S, sb, g * 3 + 0, px);
    load_group_at<FS, SPH_GROUP>(S, sb, g * 3 + 1, py);
    load_group_at<FS, SPH_GROUP>(S, sb, g * 3 + 2, pz);
  } else {
#pragma unroll
    for (int i = 0; i < SPH_GROUP; ++i) px[i] = py[i] = pz[i] = 0.f;
  }
  const int active = uniform(min(SPH_GROUP, n_s - g * SPH_GROUP));
  {
    float* mine = pos + g * SPH_GROUP * 3 * 64 + lane;
#pragma unroll
    for (int i = 0; i < SPH_GROUP; ++i) {
      if (i >= active) continue;  // the image holds the n_s real spheres only
      mine[(i * 3 + 0) * 64] = px[i];
      mine[(i * 3 + 1) * 64] = py[i];
      mine[(i * 3 + 2) * 64] = pz[i];
    }
  }
  __syncthreads();

  const int my_w = valid ? (int)(b / sh.cfg_per_world) : -1;

  float best[SPH_GROUP];
  int bk[SPH_GROUP];
#pragma unroll
  for (int i = 0; i < SPH_GROUP; ++i) {
    best[i] = INFINITY;
    bk[i] = 0;
  }

  if (Gd.MW > 0) {
    // Each lane walks its own candidate list (the union over CQ spheres of its voxels' masks),
    // reading the cuboid from its world's table: the wavefront iterates as often as its busiest
    // lane needs, not over the union of all lanes' candidates.
    if (valid) {
      const float* wbox = W.box + (int64_t)my_w * K * 16;
      const uint32_t* wmask = Gd.mask + (int64_t)my_w * ((int64_t)Gd.n * Gd.n * Gd.n) * Gd.MW;
      if (Gd.MW <= 2) {
        // up to 64 cuboids: every sphere's mask gathered at once into one 64-bit list per CQ
        // spheres, then each list walked with the next cuboid's load in flight during the current
        // tests
        uint64_t mq[SPH_GROUP / CQ];
#pragma unroll
        for (int q = 0; q < SPH_GROUP / CQ; ++q) mq[q] = 0;
#pragma unroll
        for (int i = 0; i < SPH_GROUP; ++i) {
          const int v = i < active ? voxel_of(Gd, px[i], py[i], pz[i]) : -1;
          if (v >= 0) {
            const uint32_t* mp = wmask + (int64_t)v * Gd.MW;
            mq[i / CQ] |= (uint64_t)mp[0] | (Gd.MW > 1 ? (uint64_t)mp[1] << 32 : 0);
          }
        }
#pragma unroll
        for (int q = 0; q < SPH_GROUP / CQ; ++q) {
          const int i0 = q * CQ;
          if (i0 >= active) continue;
          if (staged) walk_list(mq[q], cub, i0, px, py, pz, best, bk);
          else walk_list(mq[q], wbox, i0, px, py, pz, best, bk);
        }
      } else {
#pragma unroll
        for (int i0 = 0; i0 < SPH_GROUP; i0 += CQ) {
          if (i0 >= active) continue;
          int vox[CQ];
#pragma unroll
          for (int i = 0; i < CQ; ++i)
            vox[i] = (i0 + i < active) ? voxel_of(Gd, px[i0 + i], py[i0 + i], pz[i0 + i]) : -1;
          for (int mw = 0; mw < Gd.MW; ++mw) {
            uint32_t m = 0;
#pragma unroll
            for (int i = 0; i < CQ; ++i)
              if (vox[i] >= 0) m |= wmask[(int64_t)vox[i] * Gd.MW + mw];
            while (m) {
              const int k = mw * 32 + __builtin_ctz(m);
              m &= m - 1;
              const float4* c4 = reinterpret_cast<const float4*>(wbox + k * 16);
              const float4 c0 = c4[0], c1 = c4[1], c2 = c4[2], c3 = c4[3];
#pragma unroll
              for (int i = i0; i < i0 + CQ; ++i) cuboid_key_v(c0, c1, c2, c3, px[i], py[i], pz[i], k, best[i], bk[i]);
            }
          }
        }
      }
    }
  } else {
    for (int w = w_lo; w <= w_hi; ++w) {
      if (my_w != w) continue;
      const cptr<float> wbox = as_const(W.box) + (int64_t)uniform(w) * K * 16;
      if (active > 12) closest_cuboids<16>(wbox, K, px, py, pz, best, bk);
      else if (active > 8) closest_cuboids<12>(wbox, K, px, py, pz, best, bk);
      else if (active > 4) closest_cuboids<8>(wbox, K, px, py, pz, best, bk);
      else closest_cuboids<4>(wbox, K, px, py, pz, best, bk);
    }
  }

  float dv[SPH_GROUP], gx[SPH_GROUP], gy[SPH_GROUP], gz[SPH_GROUP];
  const float* mybox = W.box + (int64_t)(valid ? my_w : 0) * K * 16;
#pragma unroll
  for (int i = 0; i < SPH_GROUP; ++i) {
    dv[i] = 0.f;
    gx[i] = gy[i] = gz[i] = 0.f;
    const float r = i < active ? sphere_of(R.sph, g * SPH_GROUP + i).w : 0.f;
    if (i < active && K > 0 && valid && !out_of_reach(best[i], cp.eta, r)) {
      float sd, nx, ny, nz;
      if (staged) cuboid_sd_grad(cub + bk[i] * 16, px[i], py[i], pz[i], sd, nx, ny, nz);
      else cuboid_sd_grad(mybox + bk[i] * 16, px[i], py[i], pz[i], sd, nx, ny, nz);
      const float d = fmaxf(cp.eta - (sd - r), 0.f);
      dv[i] = d;
      if (d > 0.f) {
        const float coef = -2.f * cp.w_c * d;
        gx[i] = coef * nx;
        gy[i] = coef * ny;
        gz[i] = coef * nz;
      }
    }
  }
  // Self pairs: partners of any group are read from the LDS image four at a time (one scalar load
  // of four table entries), then two and one for the rest of the list.  A visit whose squared centre distance exceeds the pair's bound is
  // inactive and ends there; the others take the exact path.  Each pair is visited from both of its
  // spheres: each visit adds its own sphere's gradient and the lower index adds the cost, so no
  // cross-lane or atomic accumulation is needed.
  float self_acc = 0.f;
#pragma unroll
  for (int i = 0; i < SPH_GROUP; ++i) {
    if (i >= active) continue;
    const int s = g * SPH_GROUP + i;
    sphere_pair_visits(R, pos, lane, s, px[i], py[i], pz[i], sphere_of(R.sph, s).w, cp, gx[i], gy[i], gz[i], self_acc);
  }
  if (valid) {
    store_group<SPH_GROUP>(D, b, g, dv);
    store_group<SPH_GROUP>(G, b, g * 3 + 0, gx);
    store_group<SPH_GROUP>(G, b, g * 3 + 1, gy);
    store_group<SPH_GROUP>(G, b, g * 3 + 2, gz);
  }
  part[g * 64 + lane] = self_acc;
  __syncthreads();
  if (g == 0 && valid) {
    float sum = 0.f;
    for (int gg = 0; gg < ng; ++gg) sum += part[gg * 64 + lane];
    selfc[b] = cp.w_s * sum;
  }
}

// ---- K2 with two wavefronts per sphere group ---------------------------------------------------
//
// The work of k_sphere_cost_blk, split finer: wavefront w of the block owns half h = w & 1 (8
// spheres) of sphere group g = w >> 1.  A wavefront then needs half the registers, and the CU holds
// twice the wavefronts for the same LDS per block, which is what covers the latency of the
// candidate walks and of the partner reads.  Per sphere the arithmetic is unchanged: the same
// candidate lists of 8 spheres, the same closest-cuboid keys, the same pair visits in the same order.
// At the end the second half of each group leaves its 8 results in LDS (over the position image,
// no longer needed) and the first half encodes and stores the group's 16 values.
//
// Occupancy: the candidate walks hold one cuboid at a time (16 registers fewer than a double
// buffer), and the kernel is held to 80 VGPRs, six wavefronts per SIMD: three 512-thread blocks per
// CU, which the 52 KB of LDS per block (60 spheres) allow.  The few values that no longer fit are
// spilled in the set-up before the walks and around the final stores, not in the walks or the pair
// visits; the extra block per CU covers the candidate loads and partner reads that one cuboid in
// flight no longer does (at 94 VGPRs with two cuboids in flight, two blocks per CU, the kernel took
// 10 % longer).  Packed ExMy positions, whose decode needs more registers, keep two blocks per CU.
constexpr int HS = SPH_GROUP / 2;

size_t sphere_cost_half_lds_bytes(int n_s, int n_groups) {
  const size_t img = std::max((size_t)n_s * 3 * 64, (size_t)n_groups * 4 * HS * 64);
  return (img + (size_t)2 * n_groups * 64 + 64 * 16) * sizeof(float);
}

// The candidate list m against the half's spheres, one cuboid at a time (the other wavefronts of the
// CU cover the load's latency).
template <int N>
__device__ __forceinline__ void walk_list_single(uint64_t m, const float* base, const float (&px)[N],
                                                 const float (&py)[N], const float (&pz)[N], float (&best)[N],
                                                 int (&bk)[N]) {
  float4 c0, c1, c2, c3;
  for (int k = pop_cuboid(m, base, c0, c1, c2, c3); k >= 0; k = pop_cuboid(m, base, c0, c1, c2, c3)) {
#pragma unroll
    for (int i = 0; i < N; ++i) cuboid_key_v(c0, c1, c2, c3, px[i], py[i], pz[i], k, best[i], bk[i]);
  }
}

// Values h * 8 .. h * 8 + 7 of a stored group of 16.  Every storage format but FP6 packs 8 values into
// half the group's dwords, which are read alone; FP6 groups (3 dwords) and packed ExMy groups are
// decoded whole.
template <int FS>
__device__ __forceinline__ void load_half_at(const TV& t, const uint32_t* base, int slot, int h, float (&v)[HS]) {
  if constexpr (FS == E3M2 || FS == PXM) {
    float f[SPH_GROUP];
    load_group_at<FS, SPH_GROUP>(t, base, slot, f);
#pragma unroll
    for (int i = 0; i < HS; ++i) v[i] = h ? f[HS + i] : f[i];
  } else {
    constexpr int DW = group_dwords(FS, SPH_GROUP), DWH = DW / 2;
    static_assert(group_dwords(FS, HS) == DWH, "8 values fill half a group's dwords");
    uint32_t w[DWH];
#pragma unroll
    for (int k = 0; k < DWH; ++k) w[k] = base[(slot * DW + h * DWH + k) * 64];
    decode_group<FS, HS>(w, t.scale, v);
  }
}

template <int FS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(FS == PXM ? 4 : 6))) void k_sphere_cost_half(
    RobotArgs R, WorldArgs W, GridArgs Gd, TV S, TV D, TV G, float* __restrict__ selfc, ShapeArgs sh, CostArgs cp) {
  extern __shared__ float lds_f[];
  const int lane = threadIdx.x & 63;
  const int wv = uniform(threadIdx.x >> 6);
  const int g = wv >> 1, h = wv & 1;
  const int ng = uniform(R.n_groups);
  const int n_s = uniform(R.n_s);
  const int K = uniform(W.K);
  // Workgroups go to the eight XCDs in turn (workgroup i to XCD i mod 8); the first 8 floor(nb / 8)
  // are remapped so that each XCD takes one contiguous run of tiles, i.e. of worlds, and its L2 holds
  // the voxel masks and cuboids of the few worlds it is working on.
  const int64_t nb = gridDim.x, full = nb / 8 * 8, bid = blockIdx.x;
  const int64_t blk = bid < full ? (bid % 8) * (nb / 8) + bid / 8 : bid;
  const int64_t b = blk * 64 + lane;
  const bool valid = b < sh.B;
  const int img_words = max(n_s * 3 * 64, ng * 4 * HS * 64);
  float* pos = lds_f;                      // sphere s, component c: pos[(s * 3 + c) * 64 + lane]
  float* part = lds_f + img_words;         // [2 ng][64] self-cost partials
  float* cub = part + 2 * ng * 64;         // the block's world's cuboids (culled path)
  const int64_t first = blk * 64;
  const int64_t last = (first + 63 < sh.B ? first + 63 : sh.B - 1);
  const int w_lo = uniform((int)(first / sh.cfg_per_world));
  const int w_hi = uniform((int)(last / sh.cfg_per_world));
  const bool staged = Gd.MW > 0 && Gd.MW <= 2 && w_lo == w_hi;
  if (staged) {
    const float* src = W.box + (int64_t)w_lo * K * 16;
    for (int i = threadIdx.x; i < K * 16; i += blockDim.x) cub[i] = src[i];
  }

  const int s0 = g * SPH_GROUP + h * HS;                 // first sphere of this half
  const int active = uniform(max(0, min(HS, n_s - s0)));
  float px[HS], py[HS], pz[HS];
  if (valid) {
    const uint32_t* sb = lane_base(S, b);
    load_half_at<FS>(S, sb, g * 3 + 0, h, px);
    load_half_at<FS>(S, sb, g * 3 + 1, h, py);
    load_half_at<FS>(S, sb, g * 3 + 2, h, pz);
  } else {
#pragma unroll
    for (int i = 0; i < HS; ++i) px[i] = py[i] = pz[i] = 0.f;
  }
  {
    float* mine = pos + s0 * 3 * 64 + lane;
#pragma unroll
    for (int i = 0; i < HS; ++i) {
      if (i >= active) continue;  // the image holds the n_s real spheres only
      mine[(i * 3 + 0) * 64] = px[i];
      mine[(i * 3 + 1) * 64] = py[i];
      mine[(i * 3 + 2) * 64] = pz[i];
    }
  }
  __syncthreads();

  const int my_w = valid ? (int)(b / sh.cfg_per_world) : -1;
  float best[HS];
  int bk[HS];
#pragma unroll
  for (int i = 0; i < HS; ++i) {
    best[i] = INFINITY;
    bk[i] = 0;
  }
  if (active > 0) {
    if (Gd.MW > 0) {
      if (valid) {
        const float* wbox = W.box + (int64_t)my_w * K * 16;
        const uint32_t* wmask = Gd.mask + (int64_t)my_w * ((int64_t)Gd.n * Gd.n * Gd.n) * Gd.MW;
        if (Gd.MW <= 2) {
          // one candidate list for the half's 8 spheres: the union of their voxels' masks
          uint64_t mq = 0;
#pragma unroll
          for (int i = 0; i < HS; ++i) {
            const int v = i < active ? voxel_of(Gd, px[i], py[i], pz[i]) : -1;
            if (v >= 0) {
              const uint32_t* mp = wmask + (int64_t)v * Gd.MW;
              mq |= (uint64_t)mp[0] | (Gd.MW > 1 ? (uint64_t)mp[1] << 32 : 0);
            }
          }
          if (staged) walk_list_single<HS>(mq, cub, px, py, pz, best, bk);
          else walk_list_single<HS>(mq, wbox, px, py, pz, best, bk);
        } else {
          int vox[HS];
#pragma unroll
          for (int i = 0; i < HS; ++i) vox[i] = i < active ? voxel_of(Gd, px[i], py[i], pz[i]) : -1;
          for (int mw = 0; mw < Gd.MW; ++mw) {
            uint32_t m = 0;
#pragma unroll
            for (int i = 0; i < HS; ++i)
              if (vox[i] >= 0) m |= wmask[(int64_t)vox[i] * Gd.MW + mw];
            while (m) {
              const int k = mw * 32 + __builtin_ctz(m);
              m &= m - 1;
              const float4* c4 = reinterpret_cast<const float4*>(wbox + k * 16);
              const float4 c0 = c4[0], c1 = c4[1], c2 = c4[2], c3 = c4[3];
#pragma unroll
              for (int i = 0; i < HS; ++i) cuboid_key_v(c0, c1, c2, c3, px[i], py[i], pz[i], k, best[i], bk[i]);
            }
          }
        }
      }
    } else {
      for (int w = w_lo; w <= w_hi; ++w) {
        if (my_w != w) continue;
        const cptr<float> wbox = as_const(W.box) + (int64_t)uniform(w) * K * 16;
        if (active > 4) closest_cuboids<HS, HS>(wbox, K, px, py, pz, best, bk);
        else closest_cuboids<4, HS>(wbox, K, px, py, pz, best, bk);
      }
    }
  }

  // From here on a sphere's own centre is read back from the image when needed rather than kept in
  // registers through the rest of the kernel (that keeps the wavefront within 80 registers).
  const float* own = pos + s0 * 3 * 64 + lane;
  float dv[HS], gx[HS], gy[HS], gz[HS];
  const float* mybox = W.box + (int64_t)(valid ? my_w : 0) * K * 16;
#pragma unroll
  for (int i = 0; i < HS; ++i) {
    dv[i] = 0.f;
    gx[i] = gy[i] = gz[i] = 0.f;
    const float r = i < active ? sphere_of(R.sph, s0 + i).w : 0.f;
    if (i < active && K > 0 && valid && !out_of_reach(best[i], cp.eta, r)) {
      float sd, nx, ny, nz;
      const float qx = own[(i * 3 + 0) * 64], qy = own[(i * 3 + 1) * 64], qz = own[(i * 3 + 2) * 64];
      if (staged) cuboid_sd_grad(cub + bk[i] * 16, qx, qy, qz, sd, nx, ny, nz);
      else cuboid_sd_grad(mybox + bk[i] * 16, qx, qy, qz, sd, nx, ny, nz);
      const float d = fmaxf(cp.eta - (sd - r), 0.f);
      dv[i] = d;
      if (d > 0.f) {
        const float coef = -2.f * cp.w_c * d;
        gx[i] = coef * nx;
        gy[i] = coef * ny;
        gz[i] = coef * nz;
      }
    }
    // one sphere's cuboid at a time: the compiler would otherwise hoist the LDS reads of later
    // spheres' cuboids (they cannot fault) and hold them in registers
    asm volatile("" ::: "memory");
  }
  // Self pairs, as in k_sphere_cost_blk: partners from the LDS image four at a time (then two and
  // one), every pair visited from both spheres, the lower index adding the cost.
  float self_acc = 0.f;
#pragma unroll
  for (int i = 0; i < HS; ++i) {
    if (i >= active) continue;
    const int s = s0 + i;
    const float qx = own[(i * 3 + 0) * 64], qy = own[(i * 3 + 1) * 64], qz = own[(i * 3 + 2) * 64];
    sphere_pair_visits(R, pos, lane, s, qx, qy, qz, sphere_of(R.sph, s).w, cp, gx[i], gy[i], gz[i], self_acc);
  }
  __syncthreads();  // the position image is read for the last time above
  float* xg = pos + g * (4 * HS * 64) + lane;
  if (h == 1) {
#pragma unroll
    for (int i = 0; i < HS; ++i) {
      xg[(0 * HS + i) * 64] = dv[i];
      xg[(1 * HS + i) * 64] = gx[i];
      xg[(2 * HS + i) * 64] = gy[i];
      xg[(3 * HS + i) * 64] = gz[i];
    }
  }
  part[wv * 64 + lane] = self_acc;
  __syncthreads();
  if (h == 0 && valid) {
    float v[SPH_GROUP];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int i = 0; i < HS; ++i) {
        v[i] = c == 0 ? dv[i] : (c == 1 ? gx[i] : (c == 2 ? gy[i] : gz[i]));
        v[HS + i] = xg[(c * HS + i) * 64];
      }
      if (c == 0) store_group<SPH_GROUP>(D, b, g, v);
      else store_group<SPH_GROUP>(G, b, g * 3 + (c - 1), v);
    }
  }
  if (wv == 0 && valid) {
    float sum = 0.f;
    for (int k = 0; k < 2 * ng; ++k) sum += part[k * 64 + lane];
    selfc[b] = cp.w_s * sum;
  }
}

// ---- swept sphere collision (the swept world term of trajectory optimisation) --------------------
//
// Between consecutive timesteps of one trajectory-candidate each sphere centre moves on the straight
// segment between its two stored positions, sampled at u_j = j / (k + 1), j = 1..k.  The segment
// (t, t+1) adds (w_sw / k) sum_s sum_j d_j^2 to configuration t, and its gradient goes to both ends
// with weights (1 - u_j) and u_j.
//
// A wavefront owns 63 consecutive configurations c = 63 W + lane (lanes 0..62); each of those lanes
// evaluates the segment (c, c + 1), and lane 63 evaluates (63 W - 1, 63 W), the segment that ends at
// lane 0.  Every segment is thus evaluated once (64 lanes for 63 configurations), and the gradient
// at the far end moves one lane up with a cross-lane permute: configuration c receives its own
// segment's near-end gradient plus the far-end gradient of the segment (c - 1, c), with no atomics
// and in a fixed order.
//
// Spheres go four at a time, and two samples of each at once: the 8 sample points share one
// candidate list (the union of their voxels' masks, walked in increasing cuboid index), so each
// candidate cuboid is gathered once for 8 tests instead of 4.  Sample points of one segment lie close
// together, so the union is barely longer than each sample's own list.  Closest
// cuboid by the same comparison key as the discrete term, exact distance and gradient for the
// winner.  The grid is conservative for any point a robot sphere can occupy, so the result is the one
// every cuboid would give; without the grid (or beyond 64 cuboids) every cuboid is tested.
#ifndef VAPR_SWEPT_SAMPLES
#define VAPR_SWEPT_SAMPLES 2
#endif
#ifndef VAPR_SWEPT_SPHERES
#define VAPR_SWEPT_SPHERES 4
#endif
constexpr int SW_Q = VAPR_SWEPT_SPHERES;   // spheres per candidate list (divides 16)
constexpr int SW_KS = VAPR_SWEPT_SAMPLES;  // samples per sphere sharing the list (SW_Q * SW_KS <= 16)
static_assert(SW_Q * SW_KS <= SPH_GROUP && SPH_GROUP % SW_Q == 0, "a chunk holds at most 16 sample points");

// the candidate list m against the first NA points, two cuboid buffers used in turn so that the next
// candidate's load is in flight while the current one is tested
template <int NA>
__device__ __forceinline__ void walk_candidates(uint64_t m, const float* wbox, const float (&px)[SPH_GROUP],
                                                const float (&py)[SPH_GROUP], const float (&pz)[SPH_GROUP],
                                                float (&best)[SPH_GROUP], int (&bk)[SPH_GROUP]) {
  float4 a0, a1, a2, a3, b0, b1, b2, b3;
  int ka = pop_cuboid(m, wbox, a0, a1, a2, a3);
  while (ka >= 0) {
    const int kb = pop_cuboid(m, wbox, b0, b1, b2, b3);
#pragma unroll
    for (int n = 0; n < NA; ++n) cuboid_key_v(a0, a1, a2, a3, px[n], py[n], pz[n], ka, best[n], bk[n]);
    if (kb < 0) break;
    ka = pop_cuboid(m, wbox, a0, a1, a2, a3);
#pragma unroll
    for (int n = 0; n < NA; ++n) cuboid_key_v(b0, b1, b2, b3, px[n], py[n], pz[n], kb, best[n], bk[n]);
  }
}

// the live points of a chunk of nj samples (1 <= nj <= NJ) against the candidate list (cuboid k at
// wbox + 16 k), or against every cuboid
template <int NJ>
__device__ __forceinline__ void swept_chunk_walk(int nj, uint64_t m, const float* wbox, const float (&px)[SPH_GROUP],
                                                 const float (&py)[SPH_GROUP], const float (&pz)[SPH_GROUP],
                                                 float (&best)[SPH_GROUP], int (&bk)[SPH_GROUP]) {
  if constexpr (NJ > 1) {
    if (nj < NJ) return swept_chunk_walk<NJ - 1>(nj, m, wbox, px, py, pz, best, bk);
  }
  walk_candidates<NJ * SW_Q>(m, wbox, px, py, pz, best, bk);
}
template <int NJ>
__device__ __forceinline__ void swept_chunk_dense(int nj, cptr<float> wbox, int K, const float (&px)[SPH_GROUP],
                                                  const float (&py)[SPH_GROUP], const float (&pz)[SPH_GROUP],
                                                  float (&best)[SPH_GROUP], int (&bk)[SPH_GROUP]) {
  if constexpr (NJ > 1) {
    if (nj < NJ) return swept_chunk_dense<NJ - 1>(nj, wbox, K, px, py, pz, best, bk);
  }
  closest_cuboids<NJ * SW_Q>(wbox, K, px, py, pz, best, bk);
}

// X of one sphere group of each wavefront, [wave][sphere * 3 + component][lane], until it is stored,
// then one world's cuboids (culled path, at most 64 of 16 floats): 53,248 bytes, three workgroups
// per CU. (An 80-byte cuboid stride, 54,272 bytes, leaves room for only two, and the kernel measured
// 12% slower than without the copy.)
constexpr int SWEPT_XS_FLOATS = 4 * SPH_GROUP * 3 * 64;
constexpr int SWEPT_LDS_BYTES = (SWEPT_XS_FLOATS + 64 * 16) * (int)sizeof(float);

// 3 wavefronts per SIMD: the register budget (168) that four spheres by two samples fit without
// spilling, and what the LDS staging allows (three 53 KB workgroups per CU)
template <int FS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_swept(RobotArgs R, WorldArgs W, GridArgs Gd, TV S, TV X,
                                               float* __restrict__ sweptc, ShapeArgs sh, CostArgs cp) {
  extern __shared__ float lds_sw[];
  const int lane = threadIdx.x & 63;
  float* xs = lds_sw + (threadIdx.x >> 6) * (SPH_GROUP * 3 * 64) + lane;
  const int64_t wv = (int64_t)blockIdx.x * 4 + uniform(threadIdx.x >> 6);
  const int64_t first = wv * 63;
  const bool culled = Gd.MW > 0 && Gd.MW <= 2;
  // culled path: the world of the workgroup's middle configuration has its cuboids copied to LDS;
  // wavefronts whose segments all lie in that world read them there, the others from memory
  float* cub = lds_sw + SWEPT_XS_FLOATS;
  const int64_t mid = min((int64_t)blockIdx.x * 4 * 63 + 2 * 63, sh.B - 1);
  const int w_st = uniform((int)(mid / sh.cfg_per_world));
  if (culled) {
    const int kf = uniform(W.K) * 16;
    const float* srcb = W.box + (int64_t)w_st * kf;
    for (int i = threadIdx.x; i < kf; i += blockDim.x) cub[i] = srcb[i];
  }
  __syncthreads();
  if (first >= sh.B) return;  // whole wavefront: its own configurations and lane 63's segment lie past B
  const int64_t c = first + lane;                       // own configuration (lanes 0..62)
  const int64_t a = lane < 63 ? c : first - 1;          // segment start
  const bool seg = a >= 0 && a + 1 < sh.B && (a % sh.T) != sh.T - 1;
  const bool own = lane < 63 && c < sh.B;
  const int64_t a_lo = first > 0 ? first - 1 : 0;
  const int64_t a_hi = (first + 62 < sh.B ? first + 62 : sh.B - 1);
  const int w_lo = uniform((int)(a_lo / sh.cfg_per_world));
  const int w_hi = uniform((int)(a_hi / sh.cfg_per_world));
  const int my_w = (int)((a >= 0 ? a : 0) / sh.cfg_per_world);
  const int K = uniform(W.K);
  const int ng = uniform(R.n_groups);
  const int n_s = uniform(R.n_s);
  const int k_sw = uniform(cp.k_sw);
  const float coef_base = -2.f * cp.w_sw / (float)k_sw;
  const int src = ((lane + 63) & 63) << 2;              // ds_bpermute address of lane - 1
  const bool staged = culled && w_lo == w_hi && w_lo == w_st;
  const int64_t n3 = (int64_t)Gd.n * Gd.n * Gd.n;
  const uint32_t* b0 = lane_base(S, seg ? a : 0);
  const uint32_t* b1 = lane_base(S, seg ? a + 1 : 0);
  const float* wbox = W.box + (int64_t)my_w * K * 16;
  float cost = 0.f;

  for (int g = 0; g < ng; ++g) {
    const int active = uniform(min(SPH_GROUP, n_s - g * SPH_GROUP));
    for (int q4 = 0; q4 < SPH_GROUP; q4 += SW_Q) {
      float p0[3][SW_Q], dp[3][SW_Q], lo[3][SW_Q], hi[3][SW_Q];
#pragma unroll
      for (int i = 0; i < SW_Q; ++i) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          float v0 = 0.f, v1 = 0.f;
          if (seg && q4 + i < active) {
            v0 = load_elem_at<FS, SPH_GROUP>(S, b0, g * 3 + q, q4 + i);
            v1 = load_elem_at<FS, SPH_GROUP>(S, b1, g * 3 + q, q4 + i);
          }
          p0[q][i] = v0;
          dp[q][i] = v1 - v0;
          lo[q][i] = hi[q][i] = 0.f;
        }
      }
      if (q4 < active) {
        for (int j0 = 1; j0 <= k_sw; j0 += SW_KS) {
          const int nj = uniform(min(SW_KS, k_sw - j0 + 1));  // samples of this chunk
          // point n = jj * SW_Q + i: sphere q4 + i at sample j0 + jj (the first SW_Q nj are live)
          float uu[SW_KS], px[SPH_GROUP], py[SPH_GROUP], pz[SPH_GROUP], best[SPH_GROUP];
          int bk[SPH_GROUP];
#pragma unroll
          for (int jj = 0; jj < SW_KS; ++jj) uu[jj] = (float)(j0 + jj) / (float)(k_sw + 1);
#pragma unroll
          for (int n = 0; n < SW_Q * SW_KS; ++n) {
            const int jj = n / SW_Q, i = n % SW_Q;
            px[n] = fmaf(uu[jj], dp[0][i], p0[0][i]);
            py[n] = fmaf(uu[jj], dp[1][i], p0[1][i]);
            pz[n] = fmaf(uu[jj], dp[2][i], p0[2][i]);
            best[n] = INFINITY;
            bk[n] = 0;
          }
          if (culled) {
            if (seg) {
              const uint32_t* gm = Gd.mask + (int64_t)my_w * n3 * Gd.MW;
              uint64_t m = 0;
#pragma unroll
              for (int n = 0; n < SW_Q * SW_KS; ++n) {
                if (n / SW_Q >= nj || q4 + n % SW_Q >= active) continue;
                const int vox = voxel_of(Gd, px[n], py[n], pz[n]);
                if (vox < 0) continue;
                const uint32_t* mv = gm + (int64_t)vox * Gd.MW;
                m |= (uint64_t)mv[0] | (Gd.MW > 1 ? (uint64_t)mv[1] << 32 : 0ull);
              }
              if (staged) swept_chunk_walk<SW_KS>(nj, m, cub, px, py, pz, best, bk);
              else swept_chunk_walk<SW_KS>(nj, m, wbox, px, py, pz, best, bk);
            }
          } else {
            for (int w = w_lo; w <= w_hi; ++w) {
              if (my_w != w || !seg) continue;
              const cptr<float> ubox = as_const(W.box) + (int64_t)uniform(w) * K * 16;
              swept_chunk_dense<SW_KS>(nj, ubox, K, px, py, pz, best, bk);
            }
          }
          if (seg && K > 0) {
#pragma unroll
            for (int n = 0; n < SW_Q * SW_KS; ++n) {
              const int jj = n / SW_Q, i = n % SW_Q;
              // no candidate (key INFINITY) or none within reach: the depth is zero
              if (jj >= nj || q4 + i >= active) continue;
              const float r = sphere_of(R.sph, g * SPH_GROUP + q4 + i).w;
              if (out_of_reach(best[n], cp.eta, r)) continue;
              float sd, nx, ny, nz;
              if (staged) cuboid_sd_grad(cub + bk[n] * 16, px[n], py[n], pz[n], sd, nx, ny, nz);
              else cuboid_sd_grad(wbox + bk[n] * 16, px[n], py[n], pz[n], sd, nx, ny, nz);
              const float d = fmaxf(cp.eta - (sd - r), 0.f);
              if (d > 0.f) {
                cost = fmaf(d, d, cost);
                const float cf = coef_base * d;
                const float gx = cf * nx, gy = cf * ny, gz = cf * nz;
                lo[0][i] = fmaf(1.f - uu[jj], gx, lo[0][i]);
                lo[1][i] = fmaf(1.f - uu[jj], gy, lo[1][i]);
                lo[2][i] = fmaf(1.f - uu[jj], gz, lo[2][i]);
                hi[0][i] = fmaf(uu[jj], gx, hi[0][i]);
                hi[1][i] = fmaf(uu[jj], gy, hi[1][i]);
                hi[2][i] = fmaf(uu[jj], gz, hi[2][i]);
              }
            }
          }
        }
      }
      // far-end gradient of the segment (c - 1, c) from lane - 1 (lane 63 for lane 0)
#pragma unroll
      for (int i = 0; i < SW_Q; ++i) {
        const float fx = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(hi[0][i])));
        const float fy = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(hi[1][i])));
        const float fz = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(hi[2][i])));
        xs[((q4 + i) * 3 + 0) * 64] = lo[0][i] + fx;
        xs[((q4 + i) * 3 + 1) * 64] = lo[1][i] + fy;
        xs[((q4 + i) * 3 + 2) * 64] = lo[2][i] + fz;
      }
    }
    if (own) {
      float xg[SPH_GROUP], yg[SPH_GROUP], zg[SPH_GROUP];
#pragma unroll
      for (int i = 0; i < SPH_GROUP; ++i) {
        xg[i] = xs[(i * 3 + 0) * 64];
        yg[i] = xs[(i * 3 + 1) * 64];
        zg[i] = xs[(i * 3 + 2) * 64];
      }
      store_group<SPH_GROUP>(X, c, g * 3 + 0, xg);
      store_group<SPH_GROUP>(X, c, g * 3 + 1, yg);
      store_group<SPH_GROUP>(X, c, g * 3 + 2, zg);
    }
  }
  if (own) sweptc[c] = (cp.w_sw / (float)k_sw) * cost;
}

// ---- K3: aggregation -----------------------------------------------------------------------------

// ---- wavefront reductions: DPP steps inside each 16-lane row, then the four row results added in
// a fixed order (the same value in every lane; the wavefront must be fully active) ----------------

constexpr int DPP_SWAP1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int DPP_SWAP2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <- lane 7 - i of its half-row
constexpr int DPP_MIRROR = 0x140;       // lane i <- lane 15 - i of its row

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = dpp_u32<CTRL>((uint32_t)u), hi = dpp_u32<CTRL>((uint32_t)(u >> 32));
  return __longlong_as_double((long long)((hi << 32) | lo));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __longlong_as_double((long long)((hi << 32) | lo));
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<DPP_SWAP1>(v);
  v += dpp_f64<DPP_SWAP2>(v);
  v += dpp_f64<DPP_HALF_MIRROR>(v);
  v += dpp_f64<DPP_MIRROR>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// configuration cost of b: w_c sum_s d_s^2 (FP64) + self + w_b bound (+ swept, + pose).  D's groups
// are loaded four at a time, all four in flight together (the index clamped to the last group, so
// no branch separates the loads), then added in sphere order.
template <int FD>
__device__ __forceinline__ double cfg_cost(const TV& D, const float* __restrict__ selfc,
                                          const float* __restrict__ boundc, const float* __restrict__ sweptc,
                                          const float* __restrict__ posec, int64_t b, const CostArgs& cp, int n_s) {
  const int ng = (n_s + SPH_GROUP - 1) / SPH_GROUP;
  const uint32_t* base = lane_base(D, b);
  double sq = 0.0;
  for (int g0 = 0; g0 < ng; g0 += 4) {
    float dv[4][SPH_GROUP];
#pragma unroll
    for (int j = 0; j < 4; ++j) load_group_at<FD, SPH_GROUP>(D, base, min(g0 + j, ng - 1), dv[j]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int active = g0 + j < ng ? min(SPH_GROUP, n_s - (g0 + j) * SPH_GROUP) : 0;
#pragma unroll
      for (int i = 0; i < SPH_GROUP; ++i)
        if (i < active) sq = fma((double)dv[j][i], (double)dv[j][i], sq);
    }
  }
  double c = (double)cp.w_c * sq + (double)selfc[b] + (double)cp.w_b * (double)boundc[b];
  if (sweptc) c += (double)sweptc[b];
  if (posec) c += (double)posec[b];
  return c;
}

// one-timestep trajectories (inverse kinematics): one configuration per lane; the trajectory cost is
// the configuration cost, as the general kernel's sum over one timestep gives
template <int FD>
__global__ __launch_bounds__(256) void k_reduce_t1(TV D, const float* __restrict__ selfc,
                                                   const float* __restrict__ boundc, const float* __restrict__ sweptc,
                                                   const float* __restrict__ posec, double* __restrict__ cost_traj,
                                                   float* __restrict__ cost_cfg, ShapeArgs sh, CostArgs cp, int n_s,
                                                   WsStamp st) {
  ws_stamp(st);
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= sh.B) return;
  const double c = cfg_cost<FD>(D, selfc, boundc, sweptc, posec, b, cp, n_s);
  if (cost_cfg) cost_cfg[b] = (float)c;
  cost_traj[b] = c;
}

template <int FD>
__global__ __launch_bounds__(256) void k_reduce(TV D, const float* __restrict__ selfc,
                                                const float* __restrict__ boundc, const float* __restrict__ sweptc,
                                                const float* __restrict__ posec, const float* __restrict__ q,
                                                double* __restrict__ cost_traj, float* __restrict__ cost_cfg,
                                                ShapeArgs sh, CostArgs cp, int n_s, WsStamp st) {
  ws_stamp(st);
  const int64_t tc = (int64_t)blockIdx.x * 4 + uniform(threadIdx.x >> 6);
  if (tc >= sh.n_tc) return;
  const int lane = threadIdx.x & 63;
  const int T = sh.T;
  double acc = 0.0;
  for (int t0 = 0; t0 < T; t0 += 64) {
    const int t = t0 + lane;
    if (t < T) {
      const int64_t b = tc * T + t;
      const double c = cfg_cost<FD>(D, selfc, boundc, sweptc, posec, b, cp, n_s);
      if (cost_cfg) cost_cfg[b] = (float)c;
      double sm = 0.0;
      if (t + 1 < T) {
#pragma unroll
        for (int j = 0; j < N_JOINTS; ++j) {
          const double dq = (double)q[(b + 1) * N_JOINTS + j] - (double)q[b * N_JOINTS + j];
          sm = fma(dq, dq, sm);
        }
      }
      acc += c + (double)cp.w_v * sm;
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) cost_traj[tc] = acc;
}

// ---- K4: reverse accumulation -------------------------------------------------------------------

// Sphere gradients of group g for this lane (the swept gradient, stored in a tensor of its own,
// added when present).
template <int FG, bool HAS_X>
__device__ __forceinline__ void load_sphere_grads(const TV& G, const uint32_t* gbase, const TV& X,
                                                  const uint32_t* xbase, int g, float (&gx)[SPH_GROUP],
                                                  float (&gy)[SPH_GROUP], float (&gz)[SPH_GROUP]) {
  load_group_at<FG, SPH_GROUP>(G, gbase, g * 3 + 0, gx);
  load_group_at<FG, SPH_GROUP>(G, gbase, g * 3 + 1, gy);
  load_group_at<FG, SPH_GROUP>(G, gbase, g * 3 + 2, gz);
  if constexpr (HAS_X) {
    float vx[SPH_GROUP], vy[SPH_GROUP], vz[SPH_GROUP];
    load_group_fmt<SPH_GROUP>(X, xbase, g * 3 + 0, vx);
    load_group_fmt<SPH_GROUP>(X, xbase, g * 3 + 1, vy);
    load_group_fmt<SPH_GROUP>(X, xbase, g * 3 + 2, vz);
#pragma unroll
    for (int i = 0; i < SPH_GROUP; ++i) {
      gx[i] += vx[i];
      gy[i] += vy[i];
      gz[i] += vz[i];
    }
  }
}

// Adds the spheres of group g that sit on link l to f = sum g_s and C = sum c_s g_s^T (C[3 m + k]
// = sum c_m g_k, c_s the sphere centre in the link frame), in increasing sphere index.  Neither sum
// needs the link's pose: with x_s = R c_s + o, the moment about the world origin is
// sum x_s x g_s = vee(R C) + o x f (link_moment).
__device__ __forceinline__ void group_link_sums(const RobotArgs& R, int g, int l, const float (&gx)[SPH_GROUP],
                                                const float (&gy)[SPH_GROUP], const float (&gz)[SPH_GROUP],
                                                float (&f)[3], float (&C)[9]) {
#pragma unroll
  for (int i = 0; i < SPH_GROUP; ++i) {
    const int s = g * SPH_GROUP + i;
    if (as_const(R.link)[s] != l) continue;
    const float4 c = sphere_of(R.sph, s);
    const float cv[3] = {c.x, c.y, c.z}, gv[3] = {gx[i], gy[i], gz[i]};
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] += gv[k];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
#pragma unroll
      for (int k = 0; k < 3; ++k) C[m * 3 + k] = fmaf(cv[m], gv[k], C[m * 3 + k]);
    }
  }
}

// m = vee(R C) + o x f for the pose T = [R | o]: with P = R C, vee(P) = (P_yz - P_zy, P_zx - P_xz,
// P_xy - P_yx); then both scaled by s (a power of two, so the scaling is exact)
__device__ __forceinline__ void link_moment(const float (&T)[LINK_VALUES], const float (&C)[9], float s,
                                            float (&f)[3], float (&m)[3]) {
  auto P = [&](int j, int k) {
    return fmaf(T[j * 4 + 0], C[0 * 3 + k], fmaf(T[j * 4 + 1], C[1 * 3 + k], T[j * 4 + 2] * C[2 * 3 + k]));
  };
  const float ox = T[3], oy = T[7], oz = T[11];
  m[0] = (P(1, 2) - P(2, 1)) + fmaf(oy, f[2], -oz * f[1]);
  m[1] = (P(2, 0) - P(0, 2)) + fmaf(oz, f[0], -ox * f[2]);
  m[2] = (P(0, 1) - P(1, 0)) + fmaf(ox, f[1], -oy * f[0]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f[k] *= s;
    m[k] *= s;
  }
}

// The sphere gradients are decoded without their power-of-two scale when it can be applied to the
// sums instead (no swept gradient to add first): f, C and the moment are linear in them, so the
// result is the same to the bit and each group saves a multiply per value.
template <bool HAS_X>
__device__ __forceinline__ float fold_scale(TV& G) {
  if constexpr (HAS_X) {
    return 1.f;
  } else {
    const float s = G.scale;
    G.scale = 1.f;
    return s;
  }
}

constexpr int ADJ_Q_ROWS = 64 + 2;                          // joint rows b0 - 1 .. b0 + 64
// After the link's owner has read its pose, the first two rotation columns of the link's tile slot
// hold the link's force (f) and moment (m); the last phase reads only z = the third column and o.
constexpr int ADJ_F[3] = {0, 4, 8}, ADJ_M[3] = {1, 5, 9}, ADJ_Z[3] = {2, 6, 10}, ADJ_O[3] = {3, 7, 11};

// Pose cost at the end effector (pose T8 = [R | p], goal [R_g | p_g]): force 2 w_gp (p - p_g) at p
// and couple -2 w_gr m(R R_g^T), added to the force and moment about the world origin.
__device__ __forceinline__ void pose_cost_wrench(const float (&T8)[LINK_VALUES], const float* __restrict__ g,
                                                 const CostArgs& cp, float (&f)[3], float (&m)[3]) {
  float Fp[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) Fp[r] = 2.f * cp.w_gp * (T8[r * 4 + 3] - g[r * 4 + 3]);
  // (R R_g^T)_{ik} = sum_c R_ic Rg_kc
  auto RRg = [&](int i, int k) {
    return fmaf(T8[i * 4 + 0], g[k * 4 + 0], fmaf(T8[i * 4 + 1], g[k * 4 + 1], T8[i * 4 + 2] * g[k * 4 + 2]));
  };
  const float mx = RRg(1, 2) - RRg(2, 1), my = RRg(2, 0) - RRg(0, 2), mz = RRg(0, 1) - RRg(1, 0);
  const float c2 = -2.f * cp.w_gr;
  const float px = T8[3], py = T8[7], pz = T8[11];
  const float Mp[3] = {fmaf(py, Fp[2], fmaf(-pz, Fp[1], c2 * mx)), fmaf(pz, Fp[0], fmaf(-px, Fp[2], c2 * my)),
                       fmaf(px, Fp[1], fmaf(-py, Fp[0], c2 * mz))};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    f[k] = Fp[k] + f[k];
    m[k] = Mp[k] + m[k];
  }
}

// One block of four wavefronts per 64-configuration tile; wavefront w owns links w + 1 and w + 5.
// Phase 1: each wavefront forms the pose-free sums of its links from the sphere groups that hold
// their spheres (one group at a time); then the poses of links 1..8 go into the tile (decoded from L
// by wavefronts 0-1, or recomputed by wavefront 0) and the joint rows the last phase reads (the
// tile's and one on each side) into qs (wavefronts 2-3).  Phase 2: each owner turns its links' sums
// into a force and a moment with the link's pose (adding the pose cost at link 8) and leaves them in
// the link's tile slot.  Phase 3 (wavefront 0): the joint gradients from the tip to the base.  The
// block's LDS (26 KB) allows six blocks per CU; the wavefronts are held to 128 VGPRs, four per SIMD
// (not with a swept gradient, whose groups are decoded beside the sphere gradients').
template <int FG, bool HAS_X>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HAS_X ? 1 : 4))) void k_adjoint(
    const float* __restrict__ q, RobotArgs R, TV L, TV G, TV X, TV J, const double* __restrict__ up,
    float* __restrict__ grad_q, ShapeArgs sh, CostArgs cp, int recompute, const float* __restrict__ goal,
    WsCheck ck) {
  __shared__ float tile[TILE_POSE_WORDS];
  __shared__ float qs[ADJ_Q_ROWS * N_JOINTS];  // row b0 - 1 + r at r * 7
  const int wave = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t b0 = (int64_t)blockIdx.x * 64;
  const int64_t b = b0 + lane;
  const bool live = b < sh.B;
  if (!ws_current(ck)) {
    // not the forward pass this call was issued for: NaN gradients, nothing read from the workspace
    if (wave == 0 && live && grad_q) {
#pragma unroll
      for (int j = 0; j < N_JOINTS; ++j) grad_q[b * N_JOINTS + j] = __builtin_nanf("");
    }
    return;
  }

  // the sums need no pose: they come first, so that their loads are in flight before the staging's
  const uint32_t* gbase = lane_base(G, b);
  const uint32_t* xbase = HAS_X ? lane_base(X, b) : nullptr;
  TV Gd = G;
  const float gs = fold_scale<HAS_X>(Gd);
  float f[2][3], C[2][9];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int k = 0; k < 3; ++k) f[h][k] = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) C[h][k] = 0.f;
    const int l = wave + 1 + 4 * h;
    if (live) {
      const cptr<int> lg = as_const(R.link_groups) + 2 * l;
      const int g_lo = lg[0], g_hi = lg[1];
      for (int g = g_lo; g < g_hi; ++g) {
        float gx[SPH_GROUP], gy[SPH_GROUP], gz[SPH_GROUP];
        load_sphere_grads<FG, HAS_X>(Gd, gbase, X, xbase, g, gx, gy, gz);
        group_link_sums(R, g, l, gx, gy, gz, f[h], C[h]);
      }
    }
  }
  if (wave >= 2) {
    const int64_t base = (b0 - 1) * N_JOINTS, end = sh.B * N_JOINTS;
    for (int i = (int)threadIdx.x - 128; i < ADJ_Q_ROWS * N_JOINTS; i += 128) {
      const int64_t o = base + i;
      qs[i] = (o >= 0 && o < end) ? q[o] : 0.f;
    }
  }
  if (recompute) {
    if (wave == 0) {
      float qv[N_JOINTS];
#pragma unroll
      for (int j = 0; j < N_JOINTS; ++j) qv[j] = live ? q[b * N_JOINTS + j] : 0.f;
      chain_to_tile(R.fixed, qv, tile, lane);
    }
  } else if (wave < L_GROUPS) {
    float v[L_GROUP];
    if (live) {
      load_group<L_GROUP>(L, b, wave, v);
    } else {
#pragma unroll
      for (int i = 0; i < L_GROUP; ++i) v[i] = 0.f;
    }
#pragma unroll
    for (int i = 0; i < L_GROUP; ++i) tile[(wave * L_GROUP + i) * 64 + lane] = v[i];
  }
  __syncthreads();

#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int l = wave + 1 + 4 * h;
    float T[LINK_VALUES], m[3];
    pose_from_tile(tile, l, lane, T);
    link_moment(T, C[h], gs, f[h], m);
    if (l == N_FIXED && goal && live) pose_cost_wrench(T, goal + (b / sh.cfg_per_world) * LINK_VALUES, cp, f[h], m);
    float* w = tile + (l - 1) * LINK_VALUES * 64 + lane;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      w[ADJ_F[c] * 64] = f[h][c];
      w[ADJ_M[c] * 64] = m[c];
    }
  }
  __syncthreads();
  if (wave != 0 || !live) return;

  // tip to base: F_j, M_j over links >= j; J_j = z_j . (M_j - o_j x F_j)
  float Jv[J_GROUP];
  float F[3] = {0.f, 0.f, 0.f}, M[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int l = N_FIXED; l >= 1; --l) {
    const float* T = tile + (l - 1) * LINK_VALUES * 64 + lane;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      F[c] += T[ADJ_F[c] * 64];
      M[c] += T[ADJ_M[c] * 64];
    }
    if (l <= N_JOINTS) {
      const float zx = T[ADJ_Z[0] * 64], zy = T[ADJ_Z[1] * 64], zz = T[ADJ_Z[2] * 64];
      const float ox = T[ADJ_O[0] * 64], oy = T[ADJ_O[1] * 64], oz = T[ADJ_O[2] * 64];
      const float tx = M[0] - (oy * F[2] - oz * F[1]);
      const float ty = M[1] - (oz * F[0] - ox * F[2]);
      const float tz = M[2] - (ox * F[1] - oy * F[0]);
      Jv[l - 1] = fmaf(zx, tx, fmaf(zy, ty, zz * tz));
    }
  }
  const float* qr = qs + (lane + 1) * N_JOINTS;  // row b; rows b - 1 and b + 1 beside it
  float qv[N_JOINTS];
#pragma unroll
  for (int j = 0; j < N_JOINTS; ++j) qv[j] = qr[j];
  const int T = sh.T;
  const int64_t tc = b / T;
  const int t = (int)(b - tc * T);
  const float scale = up ? (float)up[tc] : 1.f;
#pragma unroll
  for (int j = 0; j < N_JOINTS; ++j) {
    const float over = fmaxf(qv[j] - R.q_hi[j], 0.f), under = fmaxf(R.q_lo[j] - qv[j], 0.f);
    float gj = fmaf(cp.w_b, 2.f * over - 2.f * under, Jv[j]);
    float sm = 0.f;
    if (t >= 1) sm += 2.f * (qv[j] - qr[j - N_JOINTS]);
    if (t + 1 < T) sm -= 2.f * (qr[j + N_JOINTS] - qv[j]);
    gj = fmaf(cp.w_v, sm, gj);
    Jv[j] = gj * scale;
  }
  Jv[N_JOINTS] = 0.f;
  store_group<J_GROUP>(J, b, 0, Jv);
  if (grad_q) {
    roundtrip<J_GROUP>(J, Jv);
#pragma unroll
    for (int j = 0; j < N_JOINTS; ++j) grad_q[b * N_JOINTS + j] = Jv[j];
  }
}

// ---- K5: line search + L-BFGS ----------------------------------------------------------------

// variables per lane: NE = ceil(7 T / 64), a template parameter (1..7 for T <= 64)
constexpr int OPT_NE_MAX = (MAX_OPT_T * N_JOINTS + 63) / 64;

__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, __uint_as_float(dpp_u32<DPP_SWAP1>(__float_as_uint(v))));
  v = fmaxf(v, __uint_as_float(dpp_u32<DPP_SWAP2>(__float_as_uint(v))));
  v = fmaxf(v, __uint_as_float(dpp_u32<DPP_HALF_MIRROR>(__float_as_uint(v))));
  v = fmaxf(v, __uint_as_float(dpp_u32<DPP_MIRROR>(__float_as_uint(v))));
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}

// -g capped so that its largest component is at most max_step (scale computed in FP64)
// Reductions over the GL lanes that hold one trajectory: the whole wavefront (GL = 64), or one of
// its eight 8-lane groups (GL = 8: the DPP steps inside each half-row, every lane of the group ends
// with the group's value; the other groups are never read).
template <int GL>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (GL == 64) {
    return wave_sum(v);
  } else {
    static_assert(GL == 8, "8-lane or whole-wavefront groups");
    v += dpp_f64<DPP_SWAP1>(v);
    v += dpp_f64<DPP_SWAP2>(v);
    v += dpp_f64<DPP_HALF_MIRROR>(v);
    return v;
  }
}

template <int GL>
__device__ __forceinline__ float group_max(float v) {
  if constexpr (GL == 64) {
    return wave_max(v);
  } else {
    static_assert(GL == 8, "8-lane or whole-wavefront groups");
    v = fmaxf(v, __uint_as_float(dpp_u32<DPP_SWAP1>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dpp_u32<DPP_SWAP2>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dpp_u32<DPP_HALF_MIRROR>(__float_as_uint(v))));
    return v;
  }
}

template <int OPT_NE, int GL>
__device__ __forceinline__ void steepest(const float (&g)[OPT_NE], float max_step, float (&d)[OPT_NE]) {
  float gm = 0.f;
#pragma unroll
  for (int k = 0; k < OPT_NE; ++k) gm = fmaxf(gm, fabsf(g[k]));
  gm = group_max<GL>(gm);
  double scale = 1.0;
  if (gm > 0.f) scale = fmin(1.0, (double)max_step / (double)gm);
#pragma unroll
  for (int k = 0; k < OPT_NE; ++k) d[k] = (float)(-(double)g[k] * scale);
}
__constant__ float c_alpha[MAX_LS] = {1.0f, 0.5f, 0.25f, 0.125f};

// GL lanes per trajectory: 64 (one trajectory per wavefront, n <= 64 OPT_NE variables), or 8 for
// one-configuration trajectories (n = 7: eight trajectories per wavefront, one variable per lane).
template <int OPT_NE, int GL>
__global__ __launch_bounds__(256) void k_optimizer(OptArgs o, TV J, const double* __restrict__ cost_in,
                                                   float* __restrict__ q_cand, int mode, WsCheck ck) {
  // a workspace that does not hold the expected forward pass leaves the optimiser state untouched
  if (!ws_current(ck)) return;
  const int lane = GL == 64 ? (threadIdx.x & 63) : (threadIdx.x & (GL - 1));
  const int tr = GL == 64 ? blockIdx.x * 4 + uniform(threadIdx.x >> 6) : (blockIdx.x * 256 + threadIdx.x) / GL;
  if (tr >= o.n_traj) return;  // a whole group
  const int T = o.T, n = T * N_JOINTS, m = o.m, n_ls = o.n_ls;
  const int64_t vb = (int64_t)tr * n;
  float x[OPT_NE], g[OPT_NE], d[OPT_NE];
#pragma unroll
  for (int k = 0; k < OPT_NE; ++k) {
    const int e = lane + GL * k;
    x[k] = e < n ? o.x[vb + e] : 0.f;
    g[k] = e < n ? o.g[vb + e] : 0.f;
    d[k] = e < n ? o.d[vb + e] : 0.f;
  }
  auto cand_grad = [&](int cand, int e) -> float {
    const int t = e / N_JOINTS, j = e - t * N_JOINTS;
    if (o.pin && (t == 0 || t == T - 1)) return 0.f;  // start and goal are pinned
    const int64_t b = ((int64_t)tr * (mode == 0 ? 1 : n_ls) + cand) * T + t;
    return load_elem<J_GROUP>(J, b, 0, j);
  };
  int len = o.hist_len[tr], head = o.hist_head[tr], flags = 0, acc = 0;

  if (mode == 0) {
#pragma unroll
    for (int k = 0; k < OPT_NE; ++k) {
      const int e = lane + GL * k;
      g[k] = e < n ? cand_grad(0, e) : 0.f;
    }
    steepest<OPT_NE, GL>(g, o.max_step, d);
    len = 0;
    head = 0;
    if (lane == 0) o.cost[tr] = cost_in[tr];
  } else {
    double gd = 0.0;
#pragma unroll
    for (int k = 0; k < OPT_NE; ++k) gd = fma((double)g[k], (double)d[k], gd);
    gd = group_sum<GL>(gd);
    const double c0 = o.cost[tr];
    int sel = -1;
    for (int i = 0; i < n_ls; ++i) {
      if (cost_in[(int64_t)tr * n_ls + i] <= c0 + 1e-4 * (double)c_alpha[i] * gd) {
        sel = i;
        break;
      }
    }
    if (sel < 0) {
      int bi = 0;
      for (int i = 1; i < n_ls; ++i)
        if (cost_in[(int64_t)tr * n_ls + i] < cost_in[(int64_t)tr * n_ls + bi]) bi = i;
      if (cost_in[(int64_t)tr * n_ls + bi] < c0) sel = bi;
    }
    acc = sel;
    if (sel < 0) {
      // keep x, drop the history, keep backtracking along the same direction
      len = 0;
      head = 0;
      flags = 2;
      const float shrink = 0.5f * c_alpha[n_ls - 1];
#pragma unroll
      for (int k = 0; k < OPT_NE; ++k) d[k] *= shrink;
    } else {
      const float alpha = c_alpha[sel];
      float s[OPT_NE], y[OPT_NE];
      double sy = 0.0, ss = 0.0, yy = 0.0;
#pragma unroll
      for (int k = 0; k < OPT_NE; ++k) {
        const int e = lane + GL * k;
        const float xn = fmaf(alpha, d[k], x[k]);
        const float gn = e < n ? cand_grad(sel, e) : 0.f;
        s[k] = e < n ? xn - x[k] : 0.f;
        y[k] = gn - g[k];
        x[k] = e < n ? xn : 0.f;
        g[k] = gn;
        sy = fma((double)s[k], (double)y[k], sy);
        ss = fma((double)s[k], (double)s[k], ss);
        yy = fma((double)y[k], (double)y[k], yy);
      }
      sy = group_sum<GL>(sy);
      ss = group_sum<GL>(ss);
      yy = group_sum<GL>(yy);
      if (lane == 0) o.cost[tr] = cost_in[(int64_t)tr * n_ls + sel];
      if (sy > 1e-10 * sqrt(ss) * sqrt(yy)) {
        const int64_t hb = ((int64_t)tr * m + head) * n;
#pragma unroll
        for (int k = 0; k < OPT_NE; ++k) {
          const int e = lane + GL * k;
          if (e < n) {
            o.s_hist[hb + e] = s[k];
            o.y_hist[hb + e] = y[k];
          }
        }
        if (lane == 0) o.rho[(int64_t)tr * m + head] = 1.0 / sy;
        head = (head + 1) % m;
        len = min(len + 1, m);
        flags |= 1;
      }
      // two-loop recursion, newest pair first, on the history loaded into registers up front (every
      // load in flight together; the recursion itself then waits only on its reductions)
      float hs[MAX_HIST][OPT_NE], hy[MAX_HIST][OPT_NE];
      double rho_h[MAX_HIST], a_it[MAX_HIST];
#pragma unroll
      for (int it = 0; it < MAX_HIST; ++it) {
        rho_h[it] = 0.0;
        if (it < len) {
          const int slot = (head - 1 - it + 2 * m) % m;
          const int64_t hb = ((int64_t)tr * m + slot) * n;
          rho_h[it] = o.rho[(int64_t)tr * m + slot];
#pragma unroll
          for (int k = 0; k < OPT_NE; ++k) {
            const int e = lane + GL * k;
            hs[it][k] = e < n ? o.s_hist[hb + e] : 0.f;
            hy[it][k] = e < n ? o.y_hist[hb + e] : 0.f;
          }
        }
      }
      double qv[OPT_NE];
#pragma unroll
      for (int k = 0; k < OPT_NE; ++k) qv[k] = (double)g[k];
      double gamma = 1.0;
#pragma unroll
      for (int it = 0; it < MAX_HIST; ++it) {
        a_it[it] = 0.0;
        if (it < len) {
          double sq = 0.0, sy0 = 0.0, yy0 = 0.0;
#pragma unroll
          for (int k = 0; k < OPT_NE; ++k) {
            sq = fma((double)hs[it][k], qv[k], sq);
            if (it == 0) {
              sy0 = fma((double)hs[it][k], (double)hy[it][k], sy0);
              yy0 = fma((double)hy[it][k], (double)hy[it][k], yy0);
            }
          }
          a_it[it] = rho_h[it] * group_sum<GL>(sq);
          if (it == 0) gamma = group_sum<GL>(sy0) / group_sum<GL>(yy0);
#pragma unroll
          for (int k = 0; k < OPT_NE; ++k) qv[k] = fma(-a_it[it], (double)hy[it][k], qv[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < OPT_NE; ++k) qv[k] *= gamma;
#pragma unroll
      for (int it = MAX_HIST - 1; it >= 0; --it) {
        if (it < len) {
          double yr = 0.0;
#pragma unroll
          for (int k = 0; k < OPT_NE; ++k) {
            // converted again here: keeping FP64 copies from the first pass would double the
            // registers the history needs
            asm volatile("" : "+v"(hs[it][k]), "+v"(hy[it][k]));
            yr = fma((double)hy[it][k], qv[k], yr);
          }
          const double beta = rho_h[it] * group_sum<GL>(yr);
#pragma unroll
          for (int k = 0; k < OPT_NE; ++k) qv[k] = fma(a_it[it] - beta, (double)hs[it][k], qv[k]);
        }
      }
      double gdn = 0.0;
#pragma unroll
      for (int k = 0; k < OPT_NE; ++k) {
        d[k] = (float)(-qv[k]);
        gdn = fma((double)g[k], (double)d[k], gdn);
      }
      gdn = group_sum<GL>(gdn);
      if (len == 0) {
        steepest<OPT_NE, GL>(g, o.max_step, d);
      } else if (gdn >= 0.0) {
        len = 0;
        head = 0;
        flags |= 2;
        steepest<OPT_NE, GL>(g, o.max_step, d);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < OPT_NE; ++k) {
    const int e = lane + GL * k;
    if (e < n) {
      o.x[vb + e] = x[k];
      o.g[vb + e] = g[k];
      o.d[vb + e] = d[k];
      for (int i = 0; i < n_ls; ++i) q_cand[((int64_t)tr * n_ls + i) * n + e] = fmaf(c_alpha[i], d[k], x[k]);
    }
  }
  if (lane == 0) {
    o.hist_len[tr] = len;
    o.hist_head[tr] = head;
    o.accepted[tr] = acc;
    o.flags[tr] = flags;
  }
}

// ---- element-wise codec -------------------------------------------------------------------------

template <int F>
__global__ __launch_bounds__(256) void k_quantize(float inv, const float* __restrict__ in, uint8_t* __restrict__ out,
                                                  int64_t n) {
  constexpr int DW = group_dwords(F, 16);
  const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = gi * 16;
  if (i0 >= n) return;
  float v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = (i0 + i < n) ? in[i0 + i] : 0.f;
  uint32_t w[DW];
  encode_group<F, 16>(v, inv, w);
  if (i0 + 16 <= n) {
    uint32_t* o32 = reinterpret_cast<uint32_t*>(out) + gi * DW;
#pragma unroll
    for (int k = 0; k < DW; ++k) o32[k] = w[k];
  } else {
    const int64_t total = (n * Fmt<F>::BITS + 7) / 8;
    const int64_t start = gi * DW * 4;
    for (int64_t by = start; by < total; ++by) {
      const int k = (int)(by - start);
      out[by] = (uint8_t)(w[k >> 2] >> ((k & 3) * 8));
    }
  }
}

template <int F>
__global__ __launch_bounds__(256) void k_dequantize(float scale, const uint8_t* __restrict__ in,
                                                    float* __restrict__ out, int64_t n) {
  constexpr int DW = group_dwords(F, 16);
  const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = gi * 16;
  if (i0 >= n) return;
  uint32_t w[DW];
  if (i0 + 16 <= n) {
    const uint32_t* i32 = reinterpret_cast<const uint32_t*>(in) + gi * DW;
#pragma unroll
    for (int k = 0; k < DW; ++k) w[k] = i32[k];
  } else {
#pragma unroll
    for (int k = 0; k < DW; ++k) w[k] = 0;
    const int64_t total = (n * Fmt<F>::BITS + 7) / 8;
    const int64_t start = gi * DW * 4;
    for (int64_t by = start; by < total; ++by) {
      const int k = (int)(by - start);
      w[k >> 2] |= (uint32_t)in[by] << ((k & 3) * 8);
    }
  }
  float v[16];
  decode_group<F, 16>(w, scale, v);
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (i0 + i < n) out[i0 + i] = v[i];
}

// ---- workspace <-> canonical order repacking (no arithmetic on values) --------------------------

// slot and position inside the slot's group of element `loc` of one configuration
__device__ __forceinline__ void elem_slot(int tensor, int loc, int& slot, int& pos) {
  switch (tensor) {
    case T_L: {
      const int l = loc / LINK_VALUES, k = loc % LINK_VALUES;
      slot = l / 4;
      pos = (l % 4) * LINK_VALUES + k;
    } break;
    case T_S:
    case T_G: {
      const int s = loc / 3, c = loc % 3;
      slot = (s / SPH_GROUP) * 3 + c;
      pos = s % SPH_GROUP;
    } break;
    case T_D:
      slot = loc / SPH_GROUP;
      pos = loc % SPH_GROUP;
      break;
    default:
      slot = 0;
      pos = loc;
      break;
  }
}

__device__ __forceinline__ int group_size(int tensor) {
  return tensor == T_L ? L_GROUP : (tensor == T_J ? J_GROUP : SPH_GROUP);
}

__device__ __forceinline__ uint32_t get_code(const TV& t, int tensor, int64_t b, int slot, int pos) {
  const int bits = format_bits(t.fmt);
  const int DW = group_dwords(t.fmt, group_size(tensor));
  const int bit = pos * bits, wi = bit >> 5, sh = bit & 31;
  uint64_t v = t.p[plane_index(b, t.P, slot * DW + wi)];
  if (sh + bits > 32) v |= (uint64_t)t.p[plane_index(b, t.P, slot * DW + wi + 1)] << 32;
  return (uint32_t)(v >> sh) & (bits == 32 ? 0xffffffffu : ((1u << bits) - 1u));
}

__device__ __forceinline__ uint32_t read_flat(const uint8_t* flat, int64_t e, int bits) {
  const int64_t bit = e * bits;
  const int64_t by = bit >> 3;
  const int sh = (int)(bit & 7);
  uint64_t v = 0;
  const int nbytes = (sh + bits + 7) / 8;
  for (int k = 0; k < nbytes; ++k) v |= (uint64_t)flat[by + k] << (8 * k);
  return (uint32_t)(v >> sh) & (bits == 32 ? 0xffffffffu : ((1u << bits) - 1u));
}

// export: one thread per 16 consecutive canonical elements
__global__ __launch_bounds__(256) void k_export(TV t, int tensor, int64_t B, int ecfg, uint8_t* __restrict__ flat) {
  const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total_e = B * ecfg;
  const int64_t e0 = gi * 16;
  if (e0 >= total_e) return;
  const int bits = format_bits(t.fmt);
  uint64_t acc = 0;
  int nb = 0;
  int64_t byte_out = e0 * bits / 8;  // 16 * bits is a whole number of bytes
  const int64_t total_bytes = (total_e * bits + 7) / 8;
  for (int i = 0; i < 16; ++i) {
    const int64_t e = e0 + i;
    uint32_t c = 0;
    if (e < total_e) {
      const int64_t b = e / ecfg;
      int slot, pos;
      elem_slot(tensor, (int)(e - b * ecfg), slot, pos);
      c = get_code(t, tensor, b, slot, pos);
    }
    acc |= (uint64_t)c << nb;
    nb += bits;
    while (nb >= 8) {
      if (byte_out < total_bytes) flat[byte_out] = (uint8_t)acc;
      ++byte_out;
      acc >>= 8;
      nb -= 8;
    }
  }
}

// import: one thread per (configuration, slot) group
__global__ __launch_bounds__(256) void k_import(TV t, int tensor, int64_t B, int ecfg, int n_slots, int n_s,
                                                const uint8_t* __restrict__ flat) {
  const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gi >= B * n_slots) return;
  const int64_t b = gi / n_slots;
  const int slot = (int)(gi - b * n_slots);
  const int gs = group_size(tensor);
  const int bits = format_bits(t.fmt);
  const int DW = group_dwords(t.fmt, gs);
  uint32_t w[L_GROUP];  // largest group: 48 FP32 values
  for (int k = 0; k < DW; ++k) w[k] = 0;
  for (int pos = 0; pos < gs; ++pos) {
    // canonical element of (slot, pos), if any
    int loc = -1;
    switch (tensor) {
      case T_L: loc = (slot * 4 + pos / LINK_VALUES) * LINK_VALUES + pos % LINK_VALUES; break;
      case T_S:
      case T_G: {
        const int s = (slot / 3) * SPH_GROUP + pos;
        loc = s < n_s ? s * 3 + slot % 3 : -1;
      } break;
      case T_D: {
        const int s = slot * SPH_GROUP + pos;
        loc = s < n_s ? s : -1;
      } break;
      default: loc = pos < N_JOINTS ? pos : -1; break;
    }
    if (loc < 0 || loc >= ecfg) continue;
    const uint32_t c = read_flat(flat, b * ecfg + loc, bits);
    const int bit = pos * bits, wi = bit >> 5, sh = bit & 31;
    const uint64_t v = (uint64_t)c << sh;
    w[wi] |= (uint32_t)v;
    if (sh + bits > 32) w[wi + 1] |= (uint32_t)(v >> 32);
  }
  for (int k = 0; k < DW; ++k) t.p[plane_index(b, t.P, slot * DW + k)] = w[k];
}

// Packed ExMy tensors: the flat buffer holds the codes in canonical element order, floor(32 / b) to a
// word (the same packing as the workspace groups).  Export: one thread per flat word; import: one
// thread per (configuration, slot) group.
__device__ __forceinline__ uint32_t pxm_code_at(const TV& t, int tensor, int64_t b, int slot, int pos) {
  const int q = t.pq, bits = 1 + t.xe + t.xm;
  const int DW = pxm_group_dwords(t.xe, t.xm, group_size(tensor));
  const uint32_t w = t.p[plane_index(b, t.P, slot * DW + pos / q)];
  return (w >> ((pos % q) * bits)) & (bits >= 32 ? 0xffffffffu : (1u << bits) - 1u);
}

__global__ __launch_bounds__(256) void k_export_pxm(TV t, int tensor, int64_t B, int ecfg, uint32_t* __restrict__ flat) {
  const int64_t wi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int q = t.pq, bits = 1 + t.xe + t.xm;
  const int64_t total_e = B * ecfg;
  if (wi * q >= total_e) return;
  uint32_t w = 0;
  for (int j = 0; j < q; ++j) {
    const int64_t e = wi * q + j;
    if (e >= total_e) break;
    const int64_t b = e / ecfg;
    int slot, pos;
    elem_slot(tensor, (int)(e - b * ecfg), slot, pos);
    w |= pxm_code_at(t, tensor, b, slot, pos) << (j * bits);
  }
  flat[wi] = w;
}

__global__ __launch_bounds__(256) void k_import_pxm(TV t, int tensor, int64_t B, int ecfg, int n_slots, int n_s,
                                                    const uint32_t* __restrict__ flat) {
  const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gi >= B * n_slots) return;
  const int64_t b = gi / n_slots;
  const int slot = (int)(gi - b * n_slots);
  const int gs = group_size(tensor);
  const int q = t.pq, bits = 1 + t.xe + t.xm;
  const uint32_t mask = bits >= 32 ? 0xffffffffu : (1u << bits) - 1u;
  const int DW = pxm_group_dwords(t.xe, t.xm, gs);
  uint32_t w[L_GROUP];  // at most 48 words (one code a word)
  for (int k = 0; k < DW; ++k) w[k] = 0;
  for (int pos = 0; pos < gs; ++pos) {
    int loc = -1;
    switch (tensor) {
      case T_L: loc = (slot * 4 + pos / LINK_VALUES) * LINK_VALUES + pos % LINK_VALUES; break;
      case T_S:
      case T_G: {
        const int s = (slot / 3) * SPH_GROUP + pos;
        loc = s < n_s ? s * 3 + slot % 3 : -1;
      } break;
      case T_D: {
        const int s = slot * SPH_GROUP + pos;
        loc = s < n_s ? s : -1;
      } break;
      default: loc = pos < N_JOINTS ? pos : -1; break;
    }
    if (loc < 0 || loc >= ecfg) continue;
    const int64_t e = b * ecfg + loc;
    const uint32_t c = (flat[e / q] >> ((e % q) * bits)) & mask;
    w[pos / q] |= c << ((pos % q) * bits);
  }
  for (int k = 0; k < DW; ++k) t.p[plane_index(b, t.P, slot * DW + k)] = w[k];
}

// packed ExMy element-wise codec: one thread per output word (q = floor(32 / b) values)
__global__ __launch_bounds__(256) void k_quantize_pxm(int E, int M, float inv, const float* __restrict__ in,
                                                      uint32_t* __restrict__ out, int64_t n) {
  const int q = pxm_per_word(E, M), b = 1 + E + M;
  const int64_t wi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (wi * q >= n) return;
  uint32_t w = 0;
  for (int j = 0; j < q; ++j) {
    const int64_t i = wi * q + j;
    if (i >= n) break;
    w |= exmy_encode(in[i] * inv, E, M) << (j * b);
  }
  out[wi] = w;
}

__global__ __launch_bounds__(256) void k_dequantize_pxm(int E, int M, float scale, const uint32_t* __restrict__ in,
                                                        float* __restrict__ out, int64_t n) {
  const int q = pxm_per_word(E, M), b = 1 + E + M;
  const uint32_t mask = b >= 32 ? 0xffffffffu : (1u << b) - 1u;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  out[i] = exmy_decode((in[i / q] >> ((i % q) * b)) & mask, E, M) * scale;
}

// ---- launch wrappers ----------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

hipError_t launch_fk(hipStream_t s, const float* q, const RobotArgs& R, const TV& L, const TV& S, float* bound,
                     int64_t B, int store_L, const float* goal, float* posec, int64_t cfg_per_world,
                     const CostArgs& cp) {
  const dim3 grid(blocks_for(B, 64)), block(256);
  switch (S.fmt) {
#define VAPR_FK_CASE(F) \
  case F: hipLaunchKernelGGL(k_fk<F>, grid, block, 0, s, q, R, L, S, bound, B, store_L, goal, posec, cfg_per_world, cp); \
    break;
    VAPR_FK_CASE(F32) VAPR_FK_CASE(F16) VAPR_FK_CASE(BF16) VAPR_FK_CASE(E4M3) VAPR_FK_CASE(E5M2)
    VAPR_FK_CASE(E3M2) VAPR_FK_CASE(E2M1) VAPR_FK_CASE(PXM)
#undef VAPR_FK_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sphere_cost(hipStream_t s, const RobotArgs& R, const WorldArgs& W, const TV& S, const TV& D,
                              const TV& G, float* selfc, const ShapeArgs& sh, const CostArgs& cp) {
  hipLaunchKernelGGL(k_sphere_cost, dim3(blocks_for(sh.B, 256)), dim3(256), 0, s, R, W, S, D, G, selfc, sh, cp);
  return hipGetLastError();
}

size_t sphere_cost_lds_bytes(int n_s, int n_groups) {
  return ((size_t)n_s * 3 * 64 + (size_t)n_groups * 64 + 64 * 16) * sizeof(float);
}

hipError_t launch_sphere_cost_half(hipStream_t s, const RobotArgs& R, const WorldArgs& W, const GridArgs& Gd,
                                   const TV& S, const TV& D, const TV& G, float* selfc, const ShapeArgs& sh,
                                   const CostArgs& cp) {
  const size_t lds = sphere_cost_half_lds_bytes(R.n_s, R.n_groups);
  const dim3 grid(blocks_for(sh.B, 64)), block(128 * R.n_groups);
  switch (S.fmt) {
#define VAPR_K2H(F) \
  case F: hipLaunchKernelGGL(k_sphere_cost_half<F>, grid, block, lds, s, R, W, Gd, S, D, G, selfc, sh, cp); break;
    VAPR_K2H(F32) VAPR_K2H(F16) VAPR_K2H(BF16) VAPR_K2H(E4M3) VAPR_K2H(E5M2) VAPR_K2H(E3M2) VAPR_K2H(E2M1) VAPR_K2H(PXM)
#undef VAPR_K2H
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_sphere_cost_blk(hipStream_t s, const RobotArgs& R, const WorldArgs& W, const GridArgs& Gd,
                                  const TV& S, const TV& D, const TV& G, float* selfc, const ShapeArgs& sh,
                                  const CostArgs& cp) {
  const size_t lds = sphere_cost_lds_bytes(R.n_s, R.n_groups);
  const dim3 grid(blocks_for(sh.B, 64)), block(64 * R.n_groups);
  switch (S.fmt) {
#define VAPR_K2(F) \
  case F: hipLaunchKernelGGL(k_sphere_cost_blk<F>, grid, block, lds, s, R, W, Gd, S, D, G, selfc, sh, cp); break;
    VAPR_K2(F32) VAPR_K2(F16) VAPR_K2(BF16) VAPR_K2(E4M3) VAPR_K2(E5M2) VAPR_K2(E3M2) VAPR_K2(E2M1) VAPR_K2(PXM)
#undef VAPR_K2
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t s, const TV& D, const float* selfc, const float* boundc, const float* sweptc,
                         const float* posec, const float* q, double* cost_traj, float* cost_cfg, const ShapeArgs& sh,
                         const CostArgs& cp, int n_s, const WsStamp& st) {
  switch (D.fmt) {
#define VAPR_REDUCE_CASE(F)                                                                                   \
  case F:                                                                                                     \
    if (sh.T == 1)                                                                                            \
      hipLaunchKernelGGL(k_reduce_t1<F>, dim3(blocks_for(sh.B, 256)), dim3(256), 0, s, D, selfc, boundc, sweptc, \
                         posec, cost_traj, cost_cfg, sh, cp, n_s, st);                                        \
    else                                                                                                      \
      hipLaunchKernelGGL(k_reduce<F>, dim3(blocks_for(sh.n_tc, 4)), dim3(256), 0, s, D, selfc, boundc, sweptc, \
                         posec, q, cost_traj, cost_cfg, sh, cp, n_s, st);                                     \
    break;
    VAPR_REDUCE_CASE(F32) VAPR_REDUCE_CASE(F16) VAPR_REDUCE_CASE(BF16) VAPR_REDUCE_CASE(E4M3)
    VAPR_REDUCE_CASE(E5M2) VAPR_REDUCE_CASE(E3M2) VAPR_REDUCE_CASE(E2M1) VAPR_REDUCE_CASE(PXM)
#undef VAPR_REDUCE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_swept(hipStream_t s, const RobotArgs& R, const WorldArgs& W, const GridArgs& Gd, const TV& S,
                        const TV& X, float* sweptc, const ShapeArgs& sh, const CostArgs& cp) {
  const int64_t waves = (sh.B + 62) / 63;
  const dim3 grid(blocks_for(waves, 4)), block(256);
  switch (S.fmt) {
#define VAPR_SWEPT_CASE(F) \
  case F: hipLaunchKernelGGL(k_swept<F>, grid, block, SWEPT_LDS_BYTES, s, R, W, Gd, S, X, sweptc, sh, cp); break;
    VAPR_SWEPT_CASE(F32) VAPR_SWEPT_CASE(F16) VAPR_SWEPT_CASE(BF16) VAPR_SWEPT_CASE(E4M3) VAPR_SWEPT_CASE(E5M2)
    VAPR_SWEPT_CASE(E3M2) VAPR_SWEPT_CASE(E2M1) VAPR_SWEPT_CASE(PXM)
#undef VAPR_SWEPT_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(hipStream_t s, const float* q, const RobotArgs& R, const TV& L, const TV& G, const TV& X,
                          const TV& J, const double* up, float* grad_q, const ShapeArgs& sh, const CostArgs& cp,
                          int recompute, const float* goal, const WsCheck& ck) {
  const dim3 grid(blocks_for(sh.B, 64)), block(256);
  switch (G.fmt) {
#define VAPR_ADJ_CASE(F) \
  case F:                                                                                                     \
    if (X.P) hipLaunchKernelGGL((k_adjoint<F, true>), grid, block, 0, s, q, R, L, G, X, J, up, grad_q, sh, cp, recompute, goal, ck); \
    else hipLaunchKernelGGL((k_adjoint<F, false>), grid, block, 0, s, q, R, L, G, X, J, up, grad_q, sh, cp, recompute, goal, ck); \
    break;
    VAPR_ADJ_CASE(F32) VAPR_ADJ_CASE(F16) VAPR_ADJ_CASE(BF16) VAPR_ADJ_CASE(E4M3) VAPR_ADJ_CASE(E5M2)
    VAPR_ADJ_CASE(E3M2) VAPR_ADJ_CASE(E2M1) VAPR_ADJ_CASE(PXM)
#undef VAPR_ADJ_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_optimizer(hipStream_t s, const OptArgs& o, const TV& J, const double* cost_in, float* q_cand,
                            int mode, const WsCheck& ck) {
  if (o.T == 1) {
    hipLaunchKernelGGL((k_optimizer<1, 8>), dim3(blocks_for(o.n_traj, 32)), dim3(256), 0, s, o, J, cost_in, q_cand,
                       mode, ck);
    return hipGetLastError();
  }
  const dim3 grid(blocks_for(o.n_traj, 4)), block(256);
  switch ((o.T * N_JOINTS + 63) / 64) {
#define VAPR_OPT_CASE(NE) \
  case NE: hipLaunchKernelGGL((k_optimizer<NE, 64>), grid, block, 0, s, o, J, cost_in, q_cand, mode, ck); break;
    VAPR_OPT_CASE(1) VAPR_OPT_CASE(2) VAPR_OPT_CASE(3) VAPR_OPT_CASE(4) VAPR_OPT_CASE(5) VAPR_OPT_CASE(6)
    VAPR_OPT_CASE(7)
#undef VAPR_OPT_CASE
    default: return hipErrorInvalidValue;
  }
  static_assert(OPT_NE_MAX == 7, "optimizer instantiations cover T <= 64");
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_round_exmy(int E, int M, float inv, float scale, const float* __restrict__ in,
                                                    float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = exmy_round(in[i] * inv, E, M) * scale;
}

hipError_t launch_round_exmy(hipStream_t s, int E, int M, float inv, float scale, const float* in, float* out,
                             int64_t n) {
  hipLaunchKernelGGL(k_round_exmy, dim3(blocks_for(n, 256)), dim3(256), 0, s, E, M, inv, scale, in, out, n);
  return hipGetLastError();
}

hipError_t launch_quantize_exmy(hipStream_t s, int E, int M, float inv, const float* in, uint32_t* out, int64_t n) {
  const int64_t words = (n + pxm_per_word(E, M) - 1) / pxm_per_word(E, M);
  hipLaunchKernelGGL(k_quantize_pxm, dim3(blocks_for(words, 256)), dim3(256), 0, s, E, M, inv, in, out, n);
  return hipGetLastError();
}

hipError_t launch_dequantize_exmy(hipStream_t s, int E, int M, float scale, const uint32_t* in, float* out,
                                  int64_t n) {
  hipLaunchKernelGGL(k_dequantize_pxm, dim3(blocks_for(n, 256)), dim3(256), 0, s, E, M, scale, in, out, n);
  return hipGetLastError();
}

hipError_t launch_quantize(hipStream_t s, int fmt, float inv, const float* in, uint8_t* out, int64_t n) {
  const dim3 grid(blocks_for((n + 15) / 16, 256)), block(256);
  switch (fmt) {
    case F32: hipLaunchKernelGGL(k_quantize<F32>, grid, block, 0, s, inv, in, out, n); break;
    case F16: hipLaunchKernelGGL(k_quantize<F16>, grid, block, 0, s, inv, in, out, n); break;
    case BF16: hipLaunchKernelGGL(k_quantize<BF16>, grid, block, 0, s, inv, in, out, n); break;
    case E4M3: hipLaunchKernelGGL(k_quantize<E4M3>, grid, block, 0, s, inv, in, out, n); break;
    case E5M2: hipLaunchKernelGGL(k_quantize<E5M2>, grid, block, 0, s, inv, in, out, n); break;
    case E3M2: hipLaunchKernelGGL(k_quantize<E3M2>, grid, block, 0, s, inv, in, out, n); break;
    default: hipLaunchKernelGGL(k_quantize<E2M1>, grid, block, 0, s, inv, in, out, n); break;
  }
  return hipGetLastError();
}

hipError_t launch_dequantize(hipStream_t s, int fmt, float scale, const uint8_t* in, float* out, int64_t n) {
  const dim3 grid(blocks_for((n + 15) / 16, 256)), block(256);
  switch (fmt) {
    case F32: hipLaunchKernelGGL(k_dequantize<F32>, grid, block, 0, s, scale, in, out, n); break;
    case F16: hipLaunchKernelGGL(k_dequantize<F16>, grid, block, 0, s, scale, in, out, n); break;
    case BF16: hipLaunchKernelGGL(k_dequantize<BF16>, grid, block, 0, s, scale, in, out, n); break;
    case E4M3: hipLaunchKernelGGL(k_dequantize<E4M3>, grid, block, 0, s, scale, in, out, n); break;
    case E5M2: hipLaunchKernelGGL(k_dequantize<E5M2>, grid, block, 0, s, scale, in, out, n); break;
    case E3M2: hipLaunchKernelGGL(k_dequantize<E3M2>, grid, block, 0, s, scale, in, out, n); break;
    default: hipLaunchKernelGGL(k_dequantize<E2M1>, grid, block, 0, s, scale, in, out, n); break;
  }
  return hipGetLastError();
}

hipError_t launch_repack(hipStream_t s, int tensor, const TV& t, int64_t B, int ecfg, int n_s, uint8_t* flat,
                         int direction) {
  if (direction == 0 && t.fmt == PXM) {
    const int64_t words = (B * ecfg + t.pq - 1) / t.pq;
    hipLaunchKernelGGL(k_export_pxm, dim3(blocks_for(words, 256)), dim3(256), 0, s, t, tensor, B, ecfg,
                       reinterpret_cast<uint32_t*>(flat));
  } else if (direction == 0) {
    hipLaunchKernelGGL(k_export, dim3(blocks_for((B * ecfg + 15) / 16, 256)), dim3(256), 0, s, t, tensor, B, ecfg,
                       flat);
  } else {
    int n_slots;
    const int ng = (n_s + SPH_GROUP - 1) / SPH_GROUP;
    switch (tensor) {
      case T_L: n_slots = L_GROUPS; break;
      case T_S:
      case T_G: n_slots = ng * 3; break;
      case T_D: n_slots = ng; break;
      default: n_slots = 1; break;
    }
    if (t.fmt == PXM)
      hipLaunchKernelGGL(k_import_pxm, dim3(blocks_for(B * n_slots, 256)), dim3(256), 0, s, t, tensor, B, ecfg,
                         n_slots, n_s, reinterpret_cast<const uint32_t*>(flat));
    else
      hipLaunchKernelGGL(k_import, dim3(blocks_for(B * n_slots, 256)), dim3(256), 0, s, t, tensor, B, ecfg, n_slots,
                         n_s, (const uint8_t*)flat);
  }
  return hipGetLastError();
}

}  // namespace vapr

namespace vapr {

__global__ void k_ws_stamp(WsStamp st) { ws_stamp(st); }

// Collision-free test of each configuration of a forward pass, from its stored tensors: every
// sphere's activation depth below eta (clearance > 0), no joint beyond its limits (bound cost 0) and
// every self pair apart (|p_a - p_b| - r_a - r_b > 0).  One configuration per thread.
__global__ __launch_bounds__(256) void k_collision_free(RobotArgs R, TV S, TV D, const float* __restrict__ boundc,
                                                        float eta, int64_t B, int32_t* __restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const int n_s = R.n_s;
  bool ok = boundc[b] == 0.f;
  for (int g = 0; g < R.n_groups && ok; ++g) {
    float dv[SPH_GROUP];
    load_group<SPH_GROUP>(D, b, g, dv);
#pragma unroll
    for (int i = 0; i < SPH_GROUP; ++i)
      if (g * SPH_GROUP + i < n_s && !(dv[i] < eta)) ok = false;
  }
  for (int a = 0; a < n_s && ok; ++a) {
    const int j0 = R.csr_off[a], j1 = R.csr_off[a + 1];
    if (j0 == j1) continue;
    const int ga = a / SPH_GROUP, ia = a % SPH_GROUP;
    const float ax = load_elem<SPH_GROUP>(S, b, ga * 3 + 0, ia), ay = load_elem<SPH_GROUP>(S, b, ga * 3 + 1, ia),
                az = load_elem<SPH_GROUP>(S, b, ga * 3 + 2, ia);
    const float ra = R.sph[a].w;
    for (int j = j0; j < j1 && ok; ++j) {
      const int t = R.csr_nbr[j];
      if (t < a) continue;  // each pair once
      const int gt = t / SPH_GROUP, it = t % SPH_GROUP;
      const float dx = ax - load_elem<SPH_GROUP>(S, b, gt * 3 + 0, it);
      const float dy = ay - load_elem<SPH_GROUP>(S, b, gt * 3 + 1, it);
      const float dz = az - load_elem<SPH_GROUP>(S, b, gt * 3 + 2, it);
      const float dist = sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
      if (!(dist - ra - R.sph[t].w > 0.f)) ok = false;
    }
  }
  out[b] = ok ? 1 : 0;
}

// Workspace of the allocation-free entry point: one array per device, held until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device memory: the device
// address comes from hipGetSymbolAddress below, once per device with that device current, and only
// that address is passed to kernels.
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

hipError_t scratch_address(void** ptr, size_t* bytes) {
  *bytes = SCRATCH_BYTES;
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

hipError_t launch_collision_free(hipStream_t s, const RobotArgs& R, const TV& S, const TV& D, const float* boundc,
                                 float eta, int64_t B, int32_t* out) {
  hipLaunchKernelGGL(k_collision_free, dim3(blocks_for(B, 256)), dim3(256), 0, s, R, S, D, boundc, eta, B, out);
  return hipGetLastError();
}

// ---- diagnostics: workspace poisoning and code census --------------------------------------------

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// 0: an ordinary value, 1: the format's largest finite magnitude, 2: Inf or NaN
__device__ __forceinline__ int code_class(const TV& t, uint32_t c) {
  int bits;
  uint32_t maxmag;
  if (t.fmt == PXM) {
    const int E = t.xe, M = t.xm;
    bits = 1 + E + M;
    const bool ieee = E == 8 || (E == 5 && M == 10);
    const uint32_t mall = M ? (1u << M) - 1u : 0u;
    maxmag = ieee ? ((((1u << E) - 2u) << M) | mall) : ((1u << (E + M)) - 1u);
  } else {
    switch (t.fmt) {
      case F32: bits = 32, maxmag = Fmt<F32>::MAXMAG; break;
      case F16: bits = 16, maxmag = Fmt<F16>::MAXMAG; break;
      case BF16: bits = 16, maxmag = Fmt<BF16>::MAXMAG; break;
      case E4M3: bits = 8, maxmag = Fmt<E4M3>::MAXMAG; break;
      case E5M2: bits = 8, maxmag = Fmt<E5M2>::MAXMAG; break;
      case E3M2: bits = 6, maxmag = Fmt<E3M2>::MAXMAG; break;
      default: bits = 4, maxmag = Fmt<E2M1>::MAXMAG; break;
    }
  }
  const uint32_t mag = c & (bits >= 32 ? 0x7fffffffu : ((1u << (bits - 1)) - 1u));
  return mag > maxmag ? 2 : (mag == maxmag ? 1 : 0);
}

// One thread per element of the B configurations (canonical order, padding spheres excluded); a
// wavefront adds its counts with one atomic per class.
__global__ __launch_bounds__(256) void k_code_census(TV t, int tensor, int64_t B, int ecfg,
                                                     unsigned long long* __restrict__ counts) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int cls = 0;
  if (e < B * ecfg) {
    const int64_t b = e / ecfg;
    int slot, pos;
    elem_slot(tensor, (int)(e - b * ecfg), slot, pos);
    const uint32_t c = t.fmt == PXM ? pxm_code_at(t, tensor, b, slot, pos) : get_code(t, tensor, b, slot, pos);
    cls = code_class(t, c);
  }
  const unsigned long long n1 = __popcll(__ballot(cls == 1)), n2 = __popcll(__ballot(cls == 2));
  if ((threadIdx.x & 63) == 0) {
    if (n1) atomicAdd(counts, n1);
    if (n2) atomicAdd(counts + 1, n2);
  }
}

hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, int64_t n, uint32_t v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_code_census(hipStream_t s, int tensor, const TV& t, int64_t B, int ecfg,
                              unsigned long long* counts) {
  if (B * ecfg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_code_census, dim3(blocks_for(B * ecfg, 256)), dim3(256), 0, s, t, tensor, B, ecfg, counts);
  return hipGetLastError();
}

hipError_t launch_ws_stamp(hipStream_t s, const WsStamp& st) {
  hipLaunchKernelGGL(k_ws_stamp, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

}  // namespace vapr
