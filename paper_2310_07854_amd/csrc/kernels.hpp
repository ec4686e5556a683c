// Kernel argument structs and launch wrappers shared by kernels.hip and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"

namespace vapr {

struct RobotArgs {
  const float* fixed;    // [8][12] F_1..F_8, row-major [R | t]
  const float4* sph;     // [n_groups*16] (cx, cy, cz, r); padding spheres are zero
  const int* link;       // [n_groups*16] link of each sphere; padding -> 0
  const int* csr_off;    // [n_s + 1] self-pair partners of each sphere
  const int* csr_nbr;    // [2 * n_pairs]
  const int* link_groups;  // [N_LINKS][2]: first and one-past-last sphere group holding a sphere of the link
  // Self-pair visits of sphere s: pair_tab[pair_off[s] .. pair_off[s + 1]), entries (partner index
  // as int bits, partner radius, lim2, 0), where lim2 bounds the squared centre distance beyond
  // which the pair is certainly inactive.
  const int* pair_off;
  const float4* pair_tab;
  int n_s, n_groups;
  float q_lo[N_JOINTS], q_hi[N_JOINTS];
};

struct WorldArgs {
  const float* box;  // [W][K][16]: A = R^T row-major (9), o = A c (3), h (3), pad
  int K;
};

struct GridArgs {  // cuboid candidate masks per world and voxel (MW == 0: test every cuboid)
  const uint32_t* mask;  // [W][n^3][MW]
  float ox, oy, oz, inv_cell;
  int n, MW;
};

struct TV {  // one stored tensor inside a workspace
  uint32_t* p;
  int fmt;
  int P;
  float scale;  // 2^k
  float inv;    // 2^-k
  int xe, xm;   // fmt PXM: an emulated ExMy type (exponent, mantissa bits) stored as packed codes,
  int pq;       // pq = floor(32 / (1 + xe + xm)) codes per word
};

struct ShapeArgs {
  int64_t B;
  int T, n_ls, tpw;
  int64_t cfg_per_world;
  int64_t n_tc;
};

struct CostArgs {
  float eta, w_c, w_s, w_b, w_v;
  int k_sw;    // swept samples per segment (0: off)
  float w_sw;
  float w_gp, w_gr;  // pose cost weights (position, rotation)
};

struct OptArgs {
  int n_traj, T, n_ls, m;
  int pin;  // 1: rows t = 0 and T - 1 keep zero gradient (trajectory optimisation)
  float max_step;
  float* x;
  float* g;
  float* d;
  double* cost;
  float* s_hist;
  float* y_hist;
  double* rho;
  int* hist_len;
  int* hist_head;
  int* accepted;
  int* flags;
};

enum KernelId {
  K_FK = 0, K_SPHERE = 1, K_REDUCE = 2, K_ADJOINT = 3, K_OPT = 4, K_CODEC = 5, K_REPACK = 6, K_SWEPT = 7,
  N_KERNEL_IDS = 8
};

// launch wrappers (return hipError_t of the launch)
// goal [W][12] (row-major [R | p] of link 8 per world) or null; posec [B] receives the pose cost
hipError_t launch_fk(hipStream_t s, const float* q, const RobotArgs& R, const TV& L, const TV& S, float* bound,
                     int64_t B, int store_L, const float* goal, float* posec, int64_t cfg_per_world,
                     const CostArgs& cp);
hipError_t launch_sphere_cost(hipStream_t s, const RobotArgs& R, const WorldArgs& W, const TV& S, const TV& D,
                              const TV& G, float* selfc, const ShapeArgs& sh, const CostArgs& cp);
// LDS bytes of the block-staged sphere-cost kernel (used while they fit in 64 KiB)
size_t sphere_cost_lds_bytes(int n_s, int n_groups);
// two wavefronts per sphere group (up to 8 groups, LDS sphere_cost_half_lds_bytes <= 64 KiB)
size_t sphere_cost_half_lds_bytes(int n_s, int n_groups);
hipError_t launch_sphere_cost_half(hipStream_t s, const RobotArgs& R, const WorldArgs& W, const GridArgs& Gd,
                                   const TV& S, const TV& D, const TV& G, float* selfc, const ShapeArgs& sh,
                                   const CostArgs& cp);
hipError_t launch_sphere_cost_blk(hipStream_t s, const RobotArgs& R, const WorldArgs& W, const GridArgs& Gd,
                                  const TV& S, const TV& D, const TV& G, float* selfc, const ShapeArgs& sh,
                                  const CostArgs& cp);
// swept term (cp.k_sw > 0): X and the swept cost per configuration from S
hipError_t launch_swept(hipStream_t s, const RobotArgs& R, const WorldArgs& W, const GridArgs& Gd, const TV& S,
                        const TV& X, float* sweptc, const ShapeArgs& sh, const CostArgs& cp);
// sweptc, posec: per-configuration swept and pose costs added to the configuration cost, or null
hipError_t launch_reduce(hipStream_t s, const TV& D, const float* selfc, const float* boundc, const float* sweptc,
                         const float* posec, const float* q, double* cost_traj, float* cost_cfg, const ShapeArgs& sh,
                         const CostArgs& cp, int n_s, const WsStamp& st);
// X.P == 0: no swept gradient; goal null: no pose cost
hipError_t launch_adjoint(hipStream_t s, const float* q, const RobotArgs& R, const TV& L, const TV& G, const TV& X,
                          const TV& J, const double* up, float* grad_q, const ShapeArgs& sh, const CostArgs& cp,
                          int recompute, const float* goal, const WsCheck& ck);
hipError_t launch_optimizer(hipStream_t s, const OptArgs& o, const TV& J, const double* cost_in, float* q_cand,
                            int mode, const WsCheck& ck);
// header write of a workspace outside a forward pass (stage-wise imports, resets)
hipError_t launch_ws_stamp(hipStream_t s, const WsStamp& st);
hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, int64_t n, uint32_t v);
hipError_t launch_code_census(hipStream_t s, int tensor, const TV& t, int64_t B, int ecfg,
                              unsigned long long* counts);
// device address of the current device's static scratch (the allocation-free entry point's
// workspace) and its size; call once per device with that device current
hipError_t scratch_address(void** ptr, size_t* bytes);
// per configuration 1 if collision-free (every clearance and self-pair clearance > 0, no joint beyond
// its limits) from a forward pass's stored S, D and bound cost, else 0
hipError_t launch_collision_free(hipStream_t s, const RobotArgs& R, const TV& S, const TV& D, const float* boundc,
                                 float eta, int64_t B, int32_t* out);
hipError_t launch_quantize(hipStream_t s, int fmt, float inv, const float* in, uint8_t* out, int64_t n);
hipError_t launch_round_exmy(hipStream_t s, int E, int M, float inv, float scale, const float* in, float* out,
                             int64_t n);
hipError_t launch_dequantize(hipStream_t s, int fmt, float scale, const uint8_t* in, float* out, int64_t n);
// packed codes of an emulated ExMy type, floor(32 / b) per word
hipError_t launch_quantize_exmy(hipStream_t s, int E, int M, float inv, const float* in, uint32_t* out, int64_t n);
hipError_t launch_dequantize_exmy(hipStream_t s, int E, int M, float scale, const uint32_t* in, float* out,
                                  int64_t n);
// tensor: T_L .. T_J; per-configuration element count ecfg; direction 0 export (ws -> flat), 1 import
hipError_t launch_repack(hipStream_t s, int tensor, const TV& t, int64_t B, int ecfg, int n_s, uint8_t* flat,
                         int direction);

}  // namespace vapr
