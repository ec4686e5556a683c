// Host side of the C ABI declared in include/vapr.h: argument validation, robot/world tables,
// workspace layout and bookkeeping, kernel launches on the caller's stream, per-kernel event timing.
#include "../../include/vapr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "layout.hpp"
#include "seednet.hpp"

using namespace vapr;

namespace {

thread_local std::string g_thread_err;

// What the host knows of a workspace: the forward pass that last completed into it.  The same
// context id and pass number are in the workspace's header, written by that pass's last kernel;
// the backward and optimiser kernels compare the two before reading anything else.
struct WsRecord {
  int n_worlds, tpw, T, n_ls;
  int64_t B;
  PrecisionCfg prec;
  uint64_t robot_gen, params_gen, gen;
};

std::atomic<uint64_t> g_next_ctx_uid{1};

// Device address of each device's static scratch, looked up once per device (by the first
// vapr_create on it, with the device current).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
size_t g_scratch_bytes = 0;

hipError_t device_scratch(int device, void** ptr, size_t* bytes) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    size_t n = 0;
    const hipError_t e = scratch_address(&p, &n);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    g_scratch_bytes = n;
  }
  *ptr = g_scratch_ptr[device];
  *bytes = g_scratch_bytes;
  return hipSuccess;
}

struct ProfEvent {
  int id;
  hipEvent_t start, stop;
};

}  // namespace

struct vapr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t uid = 0;        // process-unique context id (workspace headers)
  uint64_t fwd_gen = 0;    // forward passes issued (workspace headers)
  uint64_t params_gen = 0; // cost-parameter changes
  uint32_t* d_status = nullptr;  // device flag: a consumer kernel met a workspace it was not issued for
  void* scratch = nullptr;       // this device's static workspace (allocation-free entry point)
  size_t scratch_bytes = 0;
  // robot
  bool has_robot = false;
  uint64_t robot_gen = 0;
  int n_s = 0, n_groups = 0, n_pairs = 0;
  float* d_fixed = nullptr;
  float4* d_sph = nullptr;
  int* d_link = nullptr;
  int* d_csr_off = nullptr;
  int* d_csr_nbr = nullptr;
  int* d_link_groups = nullptr;
  float q_lo[N_JOINTS], q_hi[N_JOINTS];
  std::vector<float> h_radius;             // host copies for the self-pair table
  std::vector<int> h_csr_off, h_csr_nbr;
  float4* d_pair_tab = nullptr;            // rebuilt lazily when the robot or eta change
  int* d_pair_off = nullptr;
  bool pairs_valid = false;
  // worlds
  bool has_worlds = false;
  int n_worlds = 0, n_cuboids = 0;
  float* d_box = nullptr;
  // goal poses of inverse kinematics (one per world), or none
  int n_goals = 0;
  float* d_goal = nullptr;
  std::vector<float> h_pose, h_half;  // host copies for the culling grid
  // culling grid (built lazily when robot, worlds or eta change)
  bool cull = true;
  bool grid_valid = false;
  uint32_t* d_grid = nullptr;
  GridArgs grid{};
  float r_max = 0.f;
  // largest |value| any configuration can give the stored poses and sphere centres (the chain's
  // translation lengths add up along it, rotations keep lengths): overflow guard of the scales
  double reach_L = 0.0, reach_S = 0.0;
  // settings
  PrecisionCfg prec{};
  CostArgs params{0.02f, 100.f, 100.f, 10.f, 1.f, 0, 100.f, 100.f, 10.f};
  std::unordered_map<const void*, WsRecord> ws;
  std::string err;
  unsigned long long* d_census = nullptr;  // two counters of vapr_ws_census (allocated at first use)
  // profiling
  bool prof = false;
  std::vector<ProfEvent> prof_live;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms[N_KERNEL_IDS] = {};
  int64_t prof_n[N_KERNEL_IDS] = {};
};

namespace {

int fail(vapr_ctx* ctx, int status, const std::string& msg) {
  g_thread_err = msg;
  if (ctx) ctx->err = msg;
  return status;
}

int hip_fail(vapr_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, VAPR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define VAPR_HIP(ctx, call)                                 \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);  \
  } while (0)

bool valid_format(const vapr_tensor_format& f) {
  if (f.fmt == VAPR_EXMY)
    return f.exp_bits >= 1 && f.exp_bits <= 8 && f.man_bits >= 0 && f.man_bits <= 23 && f.scale_exp >= -16 &&
           f.scale_exp <= 16;
  if (f.fmt < VAPR_F32 || f.fmt > VAPR_E2M1) return false;
  if (f.scale_exp < -16 || f.scale_exp > 16) return false;
  if (f.fmt == VAPR_F32 && f.scale_exp != 0) return false;
  return true;
}

bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

bool rotation_ok(const float* tf34) {
  // rows of R are tf34[0..2], tf34[4..6], tf34[8..10]
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += (double)tf34[k * 4 + i] * (double)tf34[k * 4 + j];
      if (std::fabs(s - (i == j ? 1.0 : 0.0)) >= 1e-5) return false;
    }
  return true;
}

template <typename T>
int upload(vapr_ctx* ctx, T** dst, const T* src, size_t n) {
  T* p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)&p, n * sizeof(T));
  if (e != hipSuccess) return fail(ctx, VAPR_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (src) {
    e = hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p);
      return hip_fail(ctx, e, "hipMemcpy");
    }
  }
  *dst = p;
  return VAPR_OK;
}

void free_robot(vapr_ctx* ctx) {
  (void)hipFree(ctx->d_fixed);
  (void)hipFree(ctx->d_sph);
  (void)hipFree(ctx->d_link);
  (void)hipFree(ctx->d_csr_off);
  (void)hipFree(ctx->d_csr_nbr);
  (void)hipFree(ctx->d_link_groups);
  (void)hipFree(ctx->d_pair_tab);
  (void)hipFree(ctx->d_pair_off);
  ctx->d_pair_tab = nullptr;
  ctx->d_pair_off = nullptr;
  ctx->pairs_valid = false;
  ctx->d_fixed = nullptr;
  ctx->d_sph = nullptr;
  ctx->d_link = nullptr;
  ctx->d_csr_off = ctx->d_csr_nbr = nullptr;
  ctx->d_link_groups = nullptr;
  ctx->has_robot = false;
}

// an emulated ExMy type is stored as its own packed codes
TensorFormat tensor_format(const vapr_tensor_format& f) {
  if (f.fmt == VAPR_EXMY) return TensorFormat{PXM, f.scale_exp, f.exp_bits, f.man_bits};
  return TensorFormat{f.fmt, f.scale_exp, 0, 0};
}

vapr_tensor_format api_format(const TensorFormat& t) {
  if (t.xe) return vapr_tensor_format{VAPR_EXMY, t.scale_exp, t.xe, t.xm};
  return vapr_tensor_format{t.fmt, t.scale_exp, 0, 0};
}

PrecisionCfg to_cfg(const vapr_precision& p) {
  PrecisionCfg c{};
  c.t[T_L] = tensor_format(p.link_poses);
  c.t[T_S] = tensor_format(p.sphere_pos);
  c.t[T_D] = tensor_format(p.sphere_dist);
  c.t[T_G] = tensor_format(p.sphere_grad);
  c.t[T_J] = tensor_format(p.joint_grad);
  c.t[T_X] = tensor_format(p.swept_grad);
  c.recompute = p.recompute_poses ? 1 : 0;
  return c;
}

// same formats, pose mode and swept sampling (which decides whether X and the swept cost exist)
bool same_prec(const PrecisionCfg& a, const PrecisionCfg& b) {
  for (int i = 0; i < 6; ++i)
    if (a.t[i].fmt != b.t[i].fmt || a.t[i].scale_exp != b.t[i].scale_exp || a.t[i].xe != b.t[i].xe ||
        a.t[i].xm != b.t[i].xm)
      return false;
  return a.recompute == b.recompute && a.sweep == b.sweep && a.pose == b.pose;
}

// Largest finite value of a stored format at its scale when it overflows to Inf (FP16, BF16 and the
// IEEE-like emulated types E5M10 and E8My); +inf for the saturating formats, whose overflow stays
// finite.
double overflow_limit(const TensorFormat& f) {
  double mf;
  if (f.xe) {
    if (!((f.xe == 5 && f.xm == 10) || f.xe == 8)) return INFINITY;
    const int bias = (1 << (f.xe - 1)) - 1;
    mf = (2.0 - std::ldexp(1.0, -f.xm)) * std::ldexp(1.0, (1 << f.xe) - 2 - bias);
  } else if (f.fmt == F16) {
    mf = 65504.0;
  } else if (f.fmt == BF16) {
    mf = (2.0 - std::ldexp(1.0, -7)) * std::ldexp(1.0, 127);
  } else {
    return INFINITY;
  }
  return mf * std::ldexp(1.0, f.scale_exp);
}

// VAPR_OK, or the reason why some configuration's poses or sphere centres would overflow to Inf
int check_reach(vapr_ctx* ctx) {
  char msg[256];
  const double lim_s = overflow_limit(ctx->prec.t[T_S]);
  if (ctx->reach_S > lim_s) {
    std::snprintf(msg, sizeof msg,
                  "sphere centres reach %.4g m, beyond the largest value %.4g of the sphere_pos format at its scale "
                  "(they would overflow to Inf): raise its scale_exp", ctx->reach_S, lim_s);
    return fail(ctx, VAPR_E_INVALID, msg);
  }
  const double lim_l = overflow_limit(ctx->prec.t[T_L]);
  if (!ctx->prec.recompute && ctx->reach_L > lim_l) {
    std::snprintf(msg, sizeof msg,
                  "link poses reach %.4g, beyond the largest value %.4g of the link_poses format at its scale "
                  "(they would overflow to Inf): raise its scale_exp", ctx->reach_L, lim_l);
    return fail(ctx, VAPR_E_INVALID, msg);
  }
  return VAPR_OK;
}

// 64-bit FNV-1a over the fields same_prec compares (the workspace header's precision tag)
uint64_t prec_tag(const PrecisionCfg& p) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for (int i = 0; i < 6; ++i) {
    mix(p.t[i].fmt);
    mix(p.t[i].scale_exp);
    mix(p.t[i].xe);
    mix(p.t[i].xm);
  }
  mix(p.recompute);
  mix(p.sweep);
  mix(p.pose);
  return h;
}

// The record of a forward pass about to be written into ws, and the header words that go with it.
WsRecord new_record(vapr_ctx* ctx, int n_worlds, int tpw, int T, int n_ls, int64_t B) {
  return WsRecord{n_worlds, tpw, T, n_ls, B, ctx->prec, ctx->robot_gen, ctx->params_gen, ++ctx->fwd_gen};
}

WsStamp stamp_of(const vapr_ctx* ctx, void* ws, const WsRecord& r) {
  WsStamp st{};
  st.hdr = static_cast<uint64_t*>(ws);
  st.w[WH_MAGIC] = WS_MAGIC;
  st.w[WH_CTX] = ctx->uid;
  st.w[WH_GEN] = r.gen;
  st.w[WH_B] = (uint64_t)r.B;
  st.w[WH_SHAPE] = (uint64_t)r.T | (uint64_t)r.n_ls << 16 | (uint64_t)ctx->n_s << 24;
  st.w[WH_PREC] = prec_tag(r.prec);
  st.w[WH_ROBOT] = r.robot_gen;
  st.w[WH_PARAMS] = r.params_gen;
  return st;
}

WsCheck check_of(const vapr_ctx* ctx, const void* ws, const WsRecord& r) {
  return WsCheck{static_cast<const uint64_t*>(ws), ctx->uid, r.gen, ctx->d_status};
}

// the record of ws if it holds a forward pass under the context's current robot, precision and cost
// parameters; otherwise a failure message
const WsRecord* current_record(const vapr_ctx* ctx, const void* ws, const char** why) {
  auto it = ctx->ws.find(ws);
  if (it == ctx->ws.end()) {
    *why = "workspace holds no forward pass of this context";
    return nullptr;
  }
  const WsRecord& r = it->second;
  if (!same_prec(r.prec, ctx->prec)) *why = "precision changed since the forward pass";
  else if (r.robot_gen != ctx->robot_gen) *why = "robot changed since the forward pass";
  else if (r.params_gen != ctx->params_gen) *why = "cost parameters changed since the forward pass";
  else return &r;
  return nullptr;
}

TV tensor_view(void* ws, const Layout& L, const PrecisionCfg& pc, int t) {
  TV v;
  v.p = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + L.off[t == T_X ? OFF_X : t]);
  v.fmt = pc.t[t].fmt;
  v.P = L.P[t];
  v.scale = std::ldexp(1.0f, pc.t[t].scale_exp);
  v.inv = std::ldexp(1.0f, -pc.t[t].scale_exp);
  v.xe = pc.t[t].xe;
  v.xm = pc.t[t].xm;
  v.pq = pc.t[t].fmt == PXM ? pxm_per_word(v.xe, v.xm) : 0;
  return v;
}

RobotArgs robot_args(const vapr_ctx* ctx) {
  RobotArgs R{};
  R.fixed = ctx->d_fixed;
  R.sph = ctx->d_sph;
  R.link = ctx->d_link;
  R.csr_off = ctx->d_csr_off;
  R.csr_nbr = ctx->d_csr_nbr;
  R.link_groups = ctx->d_link_groups;
  R.pair_tab = ctx->d_pair_tab;
  R.pair_off = ctx->d_pair_off;
  R.n_s = ctx->n_s;
  R.n_groups = ctx->n_groups;
  for (int j = 0; j < N_JOINTS; ++j) {
    R.q_lo[j] = ctx->q_lo[j];
    R.q_hi[j] = ctx->q_hi[j];
  }
  return R;
}

int check_shape(vapr_ctx* ctx, int n_worlds, int tpw, int T, int n_ls, int64_t* B) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!ctx->has_robot) return fail(ctx, VAPR_E_STATE, "no robot uploaded");
  if (n_worlds < 1 || tpw < 1 || T < 1 || T > MAX_T || n_ls < 1 || n_ls > MAX_LS)
    return fail(ctx, VAPR_E_INVALID, "batch shape out of range");
  const int64_t b = (int64_t)n_worlds * tpw * n_ls * T;
  if (b > ((int64_t)1 << 31)) return fail(ctx, VAPR_E_INVALID, "batch too large");
  *B = b;
  return VAPR_OK;
}

ShapeArgs shape_args(int n_worlds, int tpw, int T, int n_ls) {
  ShapeArgs sh;
  sh.T = T;
  sh.n_ls = n_ls;
  sh.tpw = tpw;
  sh.cfg_per_world = (int64_t)tpw * n_ls * T;
  sh.n_tc = (int64_t)n_worlds * tpw * n_ls;
  sh.B = sh.n_tc * T;
  return sh;
}

// timed launch helper
template <typename F>
int timed(vapr_ctx* ctx, int id, F&& launch, const char* what) {
  hipEvent_t a = nullptr, b = nullptr;
  if (ctx && ctx->prof) {
    for (hipEvent_t* ev : {&a, &b}) {
      if (!ctx->prof_pool.empty()) {
        *ev = ctx->prof_pool.back();
        ctx->prof_pool.pop_back();
      } else {
        VAPR_HIP(ctx, hipEventCreate(ev));
      }
    }
    VAPR_HIP(ctx, hipEventRecord(a, ctx->stream));
  }
  hipError_t e = launch();
  if (e != hipSuccess) return hip_fail(ctx, e, what);
  if (ctx && ctx->prof) {
    VAPR_HIP(ctx, hipEventRecord(b, ctx->stream));
    ctx->prof_live.push_back({id, a, b});
  }
  return VAPR_OK;
}

// Self-pair visit lists, one per sphere in CSR order: (partner, partner radius, lim2, 0).
// lim2 >= ((r_s + r_t + eta) * (1 + 2^-8))^2, rounded up: a pair whose FP32 squared centre distance
// exceeds it has clearance above eta by far more than the rounding of the clearance, so its
// activation is exactly zero.
int build_pair_table(vapr_ctx* ctx) {
  if (ctx->d_pair_tab || ctx->d_pair_off) {
    VAPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->d_pair_tab);
    (void)hipFree(ctx->d_pair_off);
    ctx->d_pair_tab = nullptr;
    ctx->d_pair_off = nullptr;
  }
  const double eta = ctx->params.eta;
  auto as_float = [](int v) {
    float f;
    std::memcpy(&f, &v, sizeof f);
    return f;
  };
  std::vector<int> off(ctx->n_s + 1, 0);
  std::vector<float4> tab;
  for (int s = 0; s < ctx->n_s; ++s) {
    for (int j = ctx->h_csr_off[s]; j < ctx->h_csr_off[s + 1]; ++j) {
      const int t = ctx->h_csr_nbr[j];
      const double lim = ((double)ctx->h_radius[s] + (double)ctx->h_radius[t] + eta) * (1.0 + 1.0 / 256.0);
      float lim2 = (float)(lim * lim);
      if ((double)lim2 < lim * lim) lim2 = std::nextafter(lim2, INFINITY);
      tab.push_back(make_float4(as_float(t), ctx->h_radius[t], lim2, 0.f));
    }
    off[s + 1] = (int)tab.size();
  }
  int st;
  if ((st = upload(ctx, &ctx->d_pair_tab, tab.empty() ? nullptr : tab.data(), tab.size())) ||
      (st = upload(ctx, &ctx->d_pair_off, off.data(), off.size())))
    return st;
  ctx->pairs_valid = true;
  return VAPR_OK;
}

// Candidate masks for exact cuboid culling.  The signed distance to a box is 1-Lipschitz, so for
// any point x of a voxel with centre c and half-diagonal hv, sd(x) >= sd(c) - hv.  A cuboid whose
// sd at the centre is >= hv + eta + r_max + margin is at clearance >= eta from every sphere in the
// voxel; its bit stays clear.  The margin (1 mm) covers float32 rounding of the voxel assignment
// and of the clearance on the GPU.  Points outside the grid are out of reach of every cuboid.
// Voxel edge 5 cm, at most 64 voxels a side (grids wider than 3.2 m take coarser voxels).  Finer
// voxels give shorter candidate lists (about 15% fewer issued tests than 8 cm on the 64-cuboid
// worlds) at 8 B a voxel per world of 64 cuboids.
constexpr double GRID_CELL = 0.05;
constexpr int GRID_NMAX = 64;
int build_grid(vapr_ctx* ctx) {
  ctx->grid = GridArgs{};
  if (ctx->d_grid) {
    VAPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->d_grid);
    ctx->d_grid = nullptr;
  }
  const int W = ctx->n_worlds, K = ctx->n_cuboids;
  ctx->grid_valid = true;
  if (!ctx->cull || K == 0) return VAPR_OK;
  const double margin = 1e-3;
  const double reach = (double)ctx->params.eta + (double)ctx->r_max + margin;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  std::vector<double> ext((size_t)W * K * 3);
  for (size_t i = 0; i < (size_t)W * K; ++i) {
    const float* P = ctx->h_pose.data() + i * 12;
    const float* h = ctx->h_half.data() + i * 3;
    for (int r = 0; r < 3; ++r) {
      double e = 0;
      for (int c = 0; c < 3; ++c) e += std::fabs((double)P[r * 4 + c]) * h[c];
      ext[i * 3 + r] = e;
      lo[r] = std::min(lo[r], (double)P[r * 4 + 3] - e - reach);
      hi[r] = std::max(hi[r], (double)P[r * 4 + 3] + e + reach);
    }
  }
  const double span = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
  const int n = std::max(1, std::min(GRID_NMAX, (int)std::ceil(span / GRID_CELL)));
  const double cell = span / n;
  const double hv = cell * std::sqrt(3.0) * 0.5;
  const int MW = (K + 31) / 32;
  const size_t n3 = (size_t)n * n * n;
  std::vector<uint32_t> mask((size_t)W * n3 * MW, 0u);
  for (int w = 0; w < W; ++w)
    for (int k = 0; k < K; ++k) {
      const size_t i = (size_t)w * K + k;
      const float* P = ctx->h_pose.data() + i * 12;
      const float* h = ctx->h_half.data() + i * 3;
      int i0[3], i1[3];
      for (int r = 0; r < 3; ++r) {
        const double c = P[r * 4 + 3], e = ext[i * 3 + r] + reach + hv;
        i0[r] = std::max(0, (int)std::floor((c - e - lo[r]) / cell));
        i1[r] = std::min(n - 1, (int)std::floor((c + e - lo[r]) / cell));
      }
      for (int z = i0[2]; z <= i1[2]; ++z)
        for (int y = i0[1]; y <= i1[1]; ++y)
          for (int x = i0[0]; x <= i1[0]; ++x) {
            const double pc[3] = {lo[0] + (x + 0.5) * cell, lo[1] + (y + 0.5) * cell, lo[2] + (z + 0.5) * cell};
            double d[3], a[3], o2 = 0, amax = -1e300;
            for (int r = 0; r < 3; ++r) d[r] = pc[r] - P[r * 4 + 3];
            for (int c = 0; c < 3; ++c) {
              const double u = P[0 * 4 + c] * d[0] + P[1 * 4 + c] * d[1] + P[2 * 4 + c] * d[2];
              a[c] = std::fabs(u) - h[c];
              const double m = std::max(a[c], 0.0);
              o2 += m * m;
              amax = std::max(amax, a[c]);
            }
            const double sd = std::sqrt(o2) + std::min(amax, 0.0);
            if (sd < hv + reach) {
              const size_t v = ((size_t)z * n + y) * n + x;
              mask[((size_t)w * n3 + v) * MW + k / 32] |= 1u << (k % 32);
            }
          }
    }
  int st = upload(ctx, &ctx->d_grid, mask.data(), mask.size());
  if (st) return st;
  ctx->grid.mask = ctx->d_grid;
  ctx->grid.ox = (float)lo[0];
  ctx->grid.oy = (float)lo[1];
  ctx->grid.oz = (float)lo[2];
  ctx->grid.inv_cell = (float)(1.0 / cell);
  ctx->grid.n = n;
  ctx->grid.MW = MW;
  return VAPR_OK;
}

// Forward pass into ws.  static_ws: ws is the library's static scratch (the allocation-free entry
// point): the lookup tables must already be built (building them allocates), no host record is
// kept and the forward pass's record goes to *out_rec instead.
int run_fwd(vapr_ctx* ctx, int first, int n_worlds, int tpw, int T, int n_ls, const float* q, void* ws,
            size_t ws_bytes, double* cost_traj, float* cost_cfg, bool static_ws = false, WsRecord* out_rec = nullptr) {
  int64_t B;
  int st = check_shape(ctx, n_worlds, tpw, T, n_ls, &B);
  if (st) return st;
  if (first < 1 || first > 3) return fail(ctx, VAPR_E_INVALID, "first stage must be 1, 2 or 3");
  if (!ctx->has_worlds) return fail(ctx, VAPR_E_STATE, "no worlds uploaded");
  if ((st = check_reach(ctx))) return st;
  if (n_worlds > ctx->n_worlds) return fail(ctx, VAPR_E_INVALID, "n_worlds exceeds the uploaded worlds");
  if (!q || !ws || !cost_traj) return fail(ctx, VAPR_E_INVALID, "null pointer");
  const Layout L = make_layout(B, ctx->n_s, ctx->prec);
  if (ws_bytes < L.bytes) {
    if (static_ws)
      return fail(ctx, VAPR_E_INVALID,
                  "batch needs a " + std::to_string(L.bytes) + "-byte workspace; the static workspace holds " +
                      std::to_string(ws_bytes) + " bytes");
    return fail(ctx, VAPR_E_INVALID, "workspace too small");
  }
  if (static_ws && (!ctx->pairs_valid || !ctx->grid_valid))
    return fail(ctx, VAPR_E_STATE,
                "lookup tables not built: run one vapr_cost_fwd after changing the robot, worlds, culling or cost "
                "parameters (building them allocates device memory)");
  if (first >= 2) {
    const char* why = nullptr;
    const WsRecord* r = current_record(ctx, ws, &why);
    if (!r) return fail(ctx, VAPR_E_STATE, why);
    if (r->B != B || r->T != T || r->n_ls != n_ls)
      return fail(ctx, VAPR_E_STATE, "workspace holds a forward pass of another shape");
  }
  const ShapeArgs sh = shape_args(n_worlds, tpw, T, n_ls);
  if (!ctx->pairs_valid && (st = build_pair_table(ctx))) return st;
  const RobotArgs R = robot_args(ctx);
  const TV tL = tensor_view(ws, L, ctx->prec, T_L), tS = tensor_view(ws, L, ctx->prec, T_S),
           tD = tensor_view(ws, L, ctx->prec, T_D), tG = tensor_view(ws, L, ctx->prec, T_G);
  float* selfc = reinterpret_cast<float*>(static_cast<char*>(ws) + L.off[OFF_SELF]);
  float* boundc = reinterpret_cast<float*>(static_cast<char*>(ws) + L.off[OFF_BOUND]);
  float* sweptc = ctx->prec.sweep ? reinterpret_cast<float*>(static_cast<char*>(ws) + L.off[OFF_SWEPT]) : nullptr;
  float* posec = ctx->prec.pose ? reinterpret_cast<float*>(static_cast<char*>(ws) + L.off[OFF_POSE]) : nullptr;
  if (ctx->prec.pose && n_worlds > ctx->n_goals)
    return fail(ctx, VAPR_E_INVALID, "n_worlds exceeds the uploaded goal poses");
  hipStream_t s = ctx->stream;
  // from here on the workspace's old contents are being replaced: it holds no usable forward pass
  // until this one has been queued completely
  if (!static_ws) ctx->ws.erase(ws);
  const WsRecord rec = new_record(ctx, n_worlds, tpw, T, n_ls, B);
  const WsStamp stamp = stamp_of(ctx, ws, rec);
  if (first <= 1) {
    const CostArgs cpk = ctx->params;
    const float* goal = ctx->prec.pose ? ctx->d_goal : nullptr;
    st = timed(ctx, K_FK,
               [&] {
                 return launch_fk(s, q, R, tL, tS, boundc, B, ctx->prec.recompute ? 0 : 1, goal, posec,
                                  sh.cfg_per_world, cpk);
               },
               "k_fk launch");
    if (st) return st;
  }
  if (first <= 2) {
    WorldArgs W{ctx->d_box, ctx->n_cuboids};
    const CostArgs cp = ctx->params;
    if (!ctx->grid_valid && (st = build_grid(ctx))) return st;
    const GridArgs Gd = ctx->grid;
    if (ctx->n_groups <= 8 && sphere_cost_half_lds_bytes(ctx->n_s, ctx->n_groups) <= 65536) {
      st = timed(ctx, K_SPHERE, [&] { return launch_sphere_cost_half(s, R, W, Gd, tS, tD, tG, selfc, sh, cp); },
                 "k_sphere_cost_half launch");
    } else if (sphere_cost_lds_bytes(ctx->n_s, ctx->n_groups) <= 65536) {
      st = timed(ctx, K_SPHERE, [&] { return launch_sphere_cost_blk(s, R, W, Gd, tS, tD, tG, selfc, sh, cp); },
                 "k_sphere_cost_blk launch");
    } else {
      st = timed(ctx, K_SPHERE, [&] { return launch_sphere_cost(s, R, W, tS, tD, tG, selfc, sh, cp); },
                 "k_sphere_cost launch");
    }
    if (st) return st;
    if (ctx->prec.sweep) {
      const TV tX = tensor_view(ws, L, ctx->prec, T_X);
      st = timed(ctx, K_SWEPT, [&] { return launch_swept(s, R, W, Gd, tS, tX, sweptc, sh, cp); }, "k_swept launch");
      if (st) return st;
    }
  }
  const CostArgs cp = ctx->params;
  const int n_s = ctx->n_s;
  st = timed(ctx, K_REDUCE,
             [&] {
               return launch_reduce(s, tD, selfc, boundc, sweptc, posec, q, cost_traj, cost_cfg, sh, cp, n_s, stamp);
             },
             "k_reduce launch");
  if (st) return st;
  if (static_ws) *out_rec = rec;
  else ctx->ws[ws] = rec;
  return VAPR_OK;
}

int tensor_count(const vapr_ctx* ctx, int tensor) {
  switch (tensor) {
    case VAPR_T_LINK_POSES: return N_FIXED * LINK_VALUES;
    case VAPR_T_SPHERE_POS:
    case VAPR_T_SPHERE_GRAD:
    case VAPR_T_SWEPT_GRAD: return ctx->n_s * 3;
    case VAPR_T_SPHERE_DIST: return ctx->n_s;
    case VAPR_T_JOINT_GRAD: return N_JOINTS;
    default: return 1;
  }
}

int check_opt(vapr_ctx* ctx, const vapr_lbfgs_state* st, const void* ws, int init, WsRecord* rec) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!st || !ws) return fail(ctx, VAPR_E_INVALID, "null pointer");
  if (!st->x || !st->g || !st->d || !st->cost || !st->s_hist || !st->y_hist || !st->rho || !st->hist_len ||
      !st->hist_head || !st->accepted || !st->flags)
    return fail(ctx, VAPR_E_INVALID, "null optimiser buffer");
  if (st->T < 1 || st->T > MAX_OPT_T || st->n_ls < 1 || st->n_ls > MAX_LS || st->m < 1 || st->m > MAX_HIST ||
      st->n_traj < 1 || !(st->max_step > 0.f) || !std::isfinite(st->max_step))
    return fail(ctx, VAPR_E_INVALID, "optimiser shape out of range");
  const char* why = nullptr;
  const WsRecord* rp = current_record(ctx, ws, &why);
  if (!rp) return fail(ctx, VAPR_E_STATE, why);
  const WsRecord& r = *rp;
  if ((int64_t)r.n_worlds * r.tpw != st->n_traj || r.T != st->T || r.n_ls != (init ? 1 : st->n_ls))
    return fail(ctx, VAPR_E_STATE, "workspace shape does not match the optimiser state");
  *rec = r;
  return VAPR_OK;
}

OptArgs opt_args(const vapr_lbfgs_state* st) {
  OptArgs o;
  o.n_traj = st->n_traj;
  o.T = st->T;
  o.n_ls = st->n_ls;
  o.m = st->m;
  o.max_step = st->max_step;
  o.x = st->x;
  o.g = st->g;
  o.d = st->d;
  o.cost = st->cost;
  o.s_hist = st->s_hist;
  o.y_hist = st->y_hist;
  o.rho = st->rho;
  o.hist_len = st->hist_len;
  o.hist_head = st->hist_head;
  o.accepted = st->accepted;
  o.flags = st->flags;
  o.pin = st->free_ends ? 0 : 1;
  return o;
}

int run_opt(vapr_ctx* ctx, const vapr_lbfgs_state* st, const void* ws, size_t ws_bytes, const double* cost,
            float* q_cand, int mode) {
  WsRecord rec;
  int s = check_opt(ctx, st, ws, mode == 0, &rec);
  if (s) return s;
  if (!cost || !q_cand) return fail(ctx, VAPR_E_INVALID, "null pointer");
  const Layout L = make_layout(rec.B, ctx->n_s, ctx->prec);
  if (ws_bytes < L.bytes) return fail(ctx, VAPR_E_INVALID, "workspace too small");
  const TV tJ = tensor_view(const_cast<void*>(ws), L, ctx->prec, T_J);
  const OptArgs o = opt_args(st);
  const WsCheck ck = check_of(ctx, ws, rec);
  return timed(ctx, K_OPT, [&] { return launch_optimizer(ctx->stream, o, tJ, cost, q_cand, mode, ck); },
               "k_optimizer launch");
}

// Backward pass over the forward pass `r` held in ws (checked by the caller).
int run_bwd(vapr_ctx* ctx, const float* q, void* ws, size_t ws_bytes, const WsRecord& r, const double* grad_cost_traj,
            float* grad_q) {
  const Layout L = make_layout(r.B, ctx->n_s, ctx->prec);
  if (ws_bytes < L.bytes) return fail(ctx, VAPR_E_INVALID, "workspace too small");
  const ShapeArgs sh = shape_args(r.n_worlds, r.tpw, r.T, r.n_ls);
  const RobotArgs R = robot_args(ctx);
  const TV tL = tensor_view(ws, L, ctx->prec, T_L), tG = tensor_view(ws, L, ctx->prec, T_G),
           tJ = tensor_view(ws, L, ctx->prec, T_J), tX = tensor_view(ws, L, ctx->prec, T_X);
  const CostArgs cp = ctx->params;
  const int rec = ctx->prec.recompute;
  const float* goal = ctx->prec.pose ? ctx->d_goal : nullptr;
  if (goal && r.n_worlds > ctx->n_goals) return fail(ctx, VAPR_E_STATE, "goal poses changed since the forward pass");
  const WsCheck ck = check_of(ctx, ws, r);
  return timed(ctx, K_ADJOINT,
               [&] {
                 return launch_adjoint(ctx->stream, q, R, tL, tG, tX, tJ, grad_cost_traj, grad_q, sh, cp, rec, goal,
                                       ck);
               },
               "k_adjoint launch");
}

}  // namespace

extern "C" {

int vapr_abi_version(void) { return VAPR_ABI_VERSION; }

const char* vapr_status_string(int status) {
  switch (status) {
    case VAPR_OK: return "ok";
    case VAPR_E_INVALID: return "invalid argument";
    case VAPR_E_OOM: return "out of device memory";
    case VAPR_E_HIP: return "HIP error";
    case VAPR_E_UNSUPPORTED: return "unsupported";
    case VAPR_E_STATE: return "invalid state";
    default: return "unknown status";
  }
}

const char* vapr_last_error(const vapr_ctx* ctx) { return ctx ? ctx->err.c_str() : g_thread_err.c_str(); }

int vapr_create(vapr_ctx** out, int device, void* hip_stream) {
  if (!out) return fail(nullptr, VAPR_E_INVALID, "null output pointer");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (device < 0 || device >= n || device >= MAX_DEVICES)
    return fail(nullptr, VAPR_E_INVALID, "device index out of range");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  e = device_scratch(device, &scratch, &scratch_bytes);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
  uint32_t* status = nullptr;
  e = hipMalloc((void**)&status, sizeof(uint32_t));
  if (e != hipSuccess) return fail(nullptr, VAPR_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  e = hipMemset(status, 0, sizeof(uint32_t));
  if (e != hipSuccess) {
    (void)hipFree(status);
    return hip_fail(nullptr, e, "hipMemset");
  }
  vapr_ctx* c = new vapr_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->uid = g_next_ctx_uid.fetch_add(1);
  c->d_status = status;
  c->scratch = scratch;
  c->scratch_bytes = scratch_bytes;
  vapr_precision p{};
  p.link_poses = p.sphere_pos = p.sphere_dist = p.sphere_grad = p.joint_grad = {VAPR_F32, 0};
  c->prec = to_cfg(p);
  *out = c;
  return VAPR_OK;
}

int vapr_destroy(vapr_ctx* ctx) {
  if (!ctx) return VAPR_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_robot(ctx);
  (void)hipFree(ctx->d_box);
  (void)hipFree(ctx->d_goal);
  (void)hipFree(ctx->d_grid);
  (void)hipFree(ctx->d_status);
  (void)hipFree(ctx->d_census);
  for (auto& pe : ctx->prof_live) {
    (void)hipEventDestroy(pe.start);
    (void)hipEventDestroy(pe.stop);
  }
  for (auto ev : ctx->prof_pool) (void)hipEventDestroy(ev);
  delete ctx;
  return VAPR_OK;
}

int vapr_set_stream(vapr_ctx* ctx, void* hip_stream) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return VAPR_OK;
}

int vapr_set_robot(vapr_ctx* ctx, int n_joints, const float* fixed_tf, int n_spheres, const float* sphere_center,
                   const float* sphere_radius, const int32_t* sphere_link, int n_pairs, const int32_t* pairs,
                   const float* q_lo, const float* q_hi) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (n_joints != N_JOINTS) return fail(ctx, VAPR_E_UNSUPPORTED, "only 7-joint arms are supported");
  if (!fixed_tf || !sphere_center || !sphere_radius || !sphere_link || !q_lo || !q_hi || (n_pairs > 0 && !pairs))
    return fail(ctx, VAPR_E_INVALID, "null pointer");
  if (n_spheres < 1 || n_spheres > MAX_SPHERES) return fail(ctx, VAPR_E_INVALID, "n_spheres out of range");
  if (n_pairs < 0 || n_pairs > MAX_PAIRS) return fail(ctx, VAPR_E_INVALID, "n_pairs out of range");
  if (!finite_all(fixed_tf, N_FIXED * 12) || !finite_all(sphere_center, (size_t)n_spheres * 3) ||
      !finite_all(sphere_radius, n_spheres) || !finite_all(q_lo, N_JOINTS) || !finite_all(q_hi, N_JOINTS))
    return fail(ctx, VAPR_E_INVALID, "non-finite robot data");
  for (int j = 0; j < N_FIXED; ++j)
    if (!rotation_ok(fixed_tf + j * 12)) return fail(ctx, VAPR_E_INVALID, "fixed transform is not a rotation");
  for (int s = 0; s < n_spheres; ++s) {
    if (!(sphere_radius[s] > 0.f)) return fail(ctx, VAPR_E_INVALID, "sphere radius must be > 0");
    if (sphere_link[s] < 0 || sphere_link[s] >= N_LINKS) return fail(ctx, VAPR_E_INVALID, "sphere link out of range");
  }
  for (int j = 0; j < N_JOINTS; ++j)
    if (q_lo[j] > q_hi[j]) return fail(ctx, VAPR_E_INVALID, "q_lo > q_hi");
  std::vector<std::vector<int>> nbr(n_spheres);
  for (int p = 0; p < n_pairs; ++p) {
    const int a = pairs[2 * p], b = pairs[2 * p + 1];
    if (a < 0 || b < 0 || a >= n_spheres || b >= n_spheres || a == b)
      return fail(ctx, VAPR_E_INVALID, "self-collision pair out of range");
    nbr[a].push_back(b);
    nbr[b].push_back(a);
  }
  const int ng = (n_spheres + SPH_GROUP - 1) / SPH_GROUP;
  std::vector<float4> sph((size_t)ng * SPH_GROUP, make_float4(0.f, 0.f, 0.f, 0.f));
  std::vector<int> link((size_t)ng * SPH_GROUP, 0);
  for (int s = 0; s < n_spheres; ++s) {
    sph[s] = make_float4(sphere_center[3 * s], sphere_center[3 * s + 1], sphere_center[3 * s + 2], sphere_radius[s]);
    link[s] = sphere_link[s];
  }
  // per link: the range of sphere groups that hold its spheres (empty range: none)
  std::vector<int> lgr(2 * N_LINKS, 0);
  for (int l = 0; l < N_LINKS; ++l) {
    int lo = -1, hi = -1;
    for (int s = 0; s < n_spheres; ++s)
      if (sphere_link[s] == l) {
        if (lo < 0) lo = s / SPH_GROUP;
        hi = s / SPH_GROUP + 1;
      }
    if (lo >= 0) {
      lgr[2 * l] = lo;
      lgr[2 * l + 1] = hi;
    }
  }
  std::vector<int> off(n_spheres + 1, 0), flat;
  for (int s = 0; s < n_spheres; ++s) {
    off[s + 1] = off[s] + (int)nbr[s].size();
    for (int t : nbr[s]) flat.push_back(t);
  }
  if (ctx->has_robot || ctx->d_fixed) {
    VAPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    free_robot(ctx);
  }
  int st;
  if ((st = upload(ctx, &ctx->d_fixed, fixed_tf, N_FIXED * 12)) ||
      (st = upload(ctx, &ctx->d_sph, sph.data(), sph.size())) ||
      (st = upload(ctx, &ctx->d_link, link.data(), link.size())) ||
      (st = upload(ctx, &ctx->d_csr_off, off.data(), off.size())) ||
      (st = upload(ctx, &ctx->d_csr_nbr, flat.empty() ? nullptr : flat.data(), flat.size())) ||
      (st = upload(ctx, &ctx->d_link_groups, lgr.data(), lgr.size()))) {
    free_robot(ctx);
    return st;
  }
  ctx->n_s = n_spheres;
  ctx->n_groups = ng;
  ctx->n_pairs = n_pairs;
  for (int j = 0; j < N_JOINTS; ++j) {
    ctx->q_lo[j] = q_lo[j];
    ctx->q_hi[j] = q_hi[j];
  }
  ctx->h_radius.assign(sphere_radius, sphere_radius + n_spheres);
  ctx->h_csr_off = off;
  ctx->h_csr_nbr = flat;
  ctx->pairs_valid = false;
  ctx->has_robot = true;
  ctx->robot_gen++;
  ctx->r_max = 0.f;
  for (int i = 0; i < n_spheres; ++i) ctx->r_max = std::max(ctx->r_max, sphere_radius[i]);
  // |t_l| <= sum of the translation lengths of F_1..F_l; |p_s| <= |t_l(s)| + |c_s|; rotation
  // entries are at most 1
  double reach_link[N_LINKS] = {0.0};
  for (int l = 1; l < N_LINKS; ++l) {
    const float* F = fixed_tf + (l - 1) * 12;
    reach_link[l] = reach_link[l - 1] + std::sqrt((double)F[3] * F[3] + (double)F[7] * F[7] + (double)F[11] * F[11]);
  }
  ctx->reach_L = std::max(1.0, reach_link[N_LINKS - 1]);
  ctx->reach_S = 0.0;
  for (int i = 0; i < n_spheres; ++i) {
    const float* c = sphere_center + 3 * i;
    ctx->reach_S = std::max(ctx->reach_S, reach_link[sphere_link[i]] +
                                              std::sqrt((double)c[0] * c[0] + (double)c[1] * c[1] + (double)c[2] * c[2]));
  }
  ctx->grid_valid = false;
  return VAPR_OK;
}

int vapr_robot_reach(const vapr_ctx* cctx, double* link_poses, double* sphere_pos) {
  vapr_ctx* ctx = const_cast<vapr_ctx*>(cctx);
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!link_poses || !sphere_pos) return fail(ctx, VAPR_E_INVALID, "null pointer");
  if (!ctx->has_robot) return fail(ctx, VAPR_E_STATE, "no robot uploaded");
  *link_poses = ctx->reach_L;
  *sphere_pos = ctx->reach_S;
  return VAPR_OK;
}

int vapr_set_worlds(vapr_ctx* ctx, int n_worlds, int n_cuboids, const float* pose, const float* half_ext) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (n_worlds < 1 || n_worlds > 65536 || n_cuboids < 0 || n_cuboids > MAX_CUBOIDS)
    return fail(ctx, VAPR_E_INVALID, "world shape out of range");
  const size_t nb = (size_t)n_worlds * n_cuboids;
  if (nb > 0 && (!pose || !half_ext)) return fail(ctx, VAPR_E_INVALID, "null pointer");
  if (nb > 0 && (!finite_all(pose, nb * 12) || !finite_all(half_ext, nb * 3)))
    return fail(ctx, VAPR_E_INVALID, "non-finite world data");
  // per cuboid: A = R^T row-major, o = A c, h, pad
  std::vector<float> box(nb * 16 + 16, 0.f);
  for (size_t i = 0; i < nb; ++i) {
    const float* P = pose + i * 12;
    if (!rotation_ok(P)) return fail(ctx, VAPR_E_INVALID, "cuboid pose is not a rotation");
    float* B = box.data() + i * 16;
    for (int r = 0; r < 3; ++r) {
      double o = 0;
      for (int c = 0; c < 3; ++c) {
        B[r * 3 + c] = P[c * 4 + r];
        o += (double)P[c * 4 + r] * (double)P[c * 4 + 3];
      }
      B[9 + r] = (float)o;
      const float h = half_ext[i * 3 + r];
      if (!(h > 0.f)) return fail(ctx, VAPR_E_INVALID, "half extents must be > 0");
      B[12 + r] = h;
    }
  }
  if (ctx->d_box) {
    VAPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->d_box);
    ctx->d_box = nullptr;
    ctx->has_worlds = false;
  }
  int st = upload(ctx, &ctx->d_box, box.data(), box.size());
  if (st) return st;
  ctx->n_worlds = n_worlds;
  ctx->n_cuboids = n_cuboids;
  ctx->has_worlds = true;
  ctx->h_pose.assign(pose, pose + nb * 12);
  ctx->h_half.assign(half_ext, half_ext + nb * 3);
  ctx->grid_valid = false;
  return VAPR_OK;
}

int vapr_set_goals(vapr_ctx* ctx, int n, const float* goal) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (n < 0 || n > 65536) return fail(ctx, VAPR_E_INVALID, "goal count out of range");
  if (n > 0 && !goal) return fail(ctx, VAPR_E_INVALID, "null pointer");
  if (n > 0 && !finite_all(goal, (size_t)n * 12)) return fail(ctx, VAPR_E_INVALID, "non-finite goal pose");
  if (n > 0)
    for (int i = 0; i < n; ++i)
      if (!rotation_ok(goal + (size_t)i * 12)) return fail(ctx, VAPR_E_INVALID, "goal pose is not a rotation");
  if (ctx->d_goal) {
    VAPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(ctx->d_goal);
    ctx->d_goal = nullptr;
  }
  ctx->n_goals = 0;
  ctx->prec.pose = 0;
  if (n == 0) return VAPR_OK;
  int st = upload(ctx, &ctx->d_goal, goal, (size_t)n * 12);
  if (st) return st;
  ctx->n_goals = n;
  ctx->prec.pose = 1;
  return VAPR_OK;
}

int vapr_set_precision(vapr_ctx* ctx, const vapr_precision* p) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!p) return fail(ctx, VAPR_E_INVALID, "null precision");
  const vapr_tensor_format* f[6] = {&p->link_poses, &p->sphere_pos, &p->sphere_dist,
                                    &p->sphere_grad, &p->joint_grad, &p->swept_grad};
  for (int i = 0; i < 6; ++i)
    if (!valid_format(*f[i])) return fail(ctx, VAPR_E_INVALID, "unknown format or scale out of range");
  const int sweep = ctx->prec.sweep, pose = ctx->prec.pose;
  ctx->prec = to_cfg(*p);
  ctx->prec.sweep = sweep;
  ctx->prec.pose = pose;
  return VAPR_OK;
}

int vapr_get_precision(const vapr_ctx* ctx, vapr_precision* p) {
  if (!ctx || !p) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  vapr_tensor_format* f[6] = {&p->link_poses, &p->sphere_pos, &p->sphere_dist,
                              &p->sphere_grad, &p->joint_grad, &p->swept_grad};
  for (int i = 0; i < 6; ++i) *f[i] = api_format(ctx->prec.t[i]);
  p->recompute_poses = ctx->prec.recompute;
  return VAPR_OK;
}

int vapr_set_cost_params(vapr_ctx* ctx, const vapr_cost_params* p) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!p) return fail(ctx, VAPR_E_INVALID, "null params");
  const float v[8] = {p->eta, p->w_coll, p->w_self, p->w_bound, p->w_smooth, p->w_swept, p->w_goal_pos, p->w_goal_rot};
  if (!finite_all(v, 8) || !(p->eta > 0.f) || p->w_coll < 0.f || p->w_self < 0.f || p->w_bound < 0.f ||
      p->w_smooth < 0.f || p->w_swept < 0.f || p->swept_steps < 0 || p->swept_steps > MAX_SWEEP ||
      p->w_goal_pos < 0.f || p->w_goal_rot < 0.f)
    return fail(ctx, VAPR_E_INVALID, "cost parameters out of range");
  ctx->params = CostArgs{p->eta,       p->w_coll,   p->w_self,     p->w_bound,    p->w_smooth,
                         p->swept_steps, p->w_swept, p->w_goal_pos, p->w_goal_rot};
  ctx->prec.sweep = p->swept_steps;
  ctx->params_gen++;
  ctx->grid_valid = false;
  ctx->pairs_valid = false;
  return VAPR_OK;
}

int vapr_set_culling(vapr_ctx* ctx, int enable) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  ctx->cull = enable != 0;
  ctx->grid_valid = false;
  return VAPR_OK;
}

int vapr_get_culling_grid(vapr_ctx* ctx, int world, vapr_grid_info* info, uint32_t* mask_out,
                          size_t capacity_words) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!info) return fail(ctx, VAPR_E_INVALID, "null info");
  if (!ctx->has_robot) return fail(ctx, VAPR_E_STATE, "no robot uploaded");
  if (!ctx->has_worlds) return fail(ctx, VAPR_E_STATE, "no worlds uploaded");
  if (world < 0 || world >= ctx->n_worlds) return fail(ctx, VAPR_E_INVALID, "world out of range");
  int st;
  if (!ctx->grid_valid && (st = build_grid(ctx))) return st;
  const GridArgs& g = ctx->grid;
  *info = vapr_grid_info{};
  if (g.MW == 0) return VAPR_OK;
  info->n = g.n;
  info->mask_words = g.MW;
  info->origin[0] = g.ox;
  info->origin[1] = g.oy;
  info->origin[2] = g.oz;
  info->inv_cell = g.inv_cell;
  if (!mask_out) return VAPR_OK;
  const size_t words = (size_t)g.n * g.n * g.n * g.MW;
  if (capacity_words < words) return fail(ctx, VAPR_E_INVALID, "mask buffer too small");
  VAPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  VAPR_HIP(ctx, hipMemcpy(mask_out, g.mask + (size_t)world * words, words * 4, hipMemcpyDeviceToHost));
  return VAPR_OK;
}

int vapr_workspace_size(const vapr_ctx* cctx, int n_worlds, int tpw, int T, int n_ls, size_t* bytes) {
  vapr_ctx* ctx = const_cast<vapr_ctx*>(cctx);
  if (!bytes) return fail(ctx, VAPR_E_INVALID, "null output pointer");
  int64_t B;
  int st = check_shape(ctx, n_worlds, tpw, T, n_ls, &B);
  if (st) return st;
  *bytes = make_layout(B, ctx->n_s, ctx->prec).bytes;
  return VAPR_OK;
}

int vapr_cost_fwd(vapr_ctx* ctx, int n_worlds, int tpw, int T, int n_ls, const float* q, void* ws, size_t ws_bytes,
                  double* cost_traj, float* cost_cfg) {
  return run_fwd(ctx, 1, n_worlds, tpw, T, n_ls, q, ws, ws_bytes, cost_traj, cost_cfg);
}

int vapr_cost_fwd_from(vapr_ctx* ctx, int first, int n_worlds, int tpw, int T, int n_ls, const float* q, void* ws,
                       size_t ws_bytes, double* cost_traj, float* cost_cfg) {
  return run_fwd(ctx, first, n_worlds, tpw, T, n_ls, q, ws, ws_bytes, cost_traj, cost_cfg);
}

int vapr_cost_bwd(vapr_ctx* ctx, const float* q, void* ws, size_t ws_bytes, const double* grad_cost_traj,
                  float* grad_q) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!q || !ws) return fail(ctx, VAPR_E_INVALID, "null pointer");
  const char* why = nullptr;
  const WsRecord* rp = current_record(ctx, ws, &why);
  if (!rp) return fail(ctx, VAPR_E_STATE, why);
  return run_bwd(ctx, q, ws, ws_bytes, *rp, grad_cost_traj, grad_q);
}

int vapr_cost_fwd_bwd_noalloc(vapr_ctx* ctx, int n_worlds, int tpw, int T, int n_ls, const float* q,
                              const double* grad_cost_traj, double* cost_traj, float* cost_cfg, float* grad_q) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!grad_q) return fail(ctx, VAPR_E_INVALID, "null grad_q");
  if (!ctx->scratch) return fail(ctx, VAPR_E_STATE, "no static workspace on this device");
  // per-kernel event timing is left out: creating events allocates
  const bool prof = ctx->prof;
  ctx->prof = false;
  WsRecord rec{};
  int st = run_fwd(ctx, 1, n_worlds, tpw, T, n_ls, q, ctx->scratch, ctx->scratch_bytes, cost_traj, cost_cfg, true,
                   &rec);
  if (!st) st = run_bwd(ctx, q, ctx->scratch, ctx->scratch_bytes, rec, grad_cost_traj, grad_q);
  ctx->prof = prof;
  return st;
}

int vapr_optimizer_init(vapr_ctx* ctx, const vapr_lbfgs_state* st, const void* ws, size_t ws_bytes,
                        const double* cost0, float* q_cand) {
  return run_opt(ctx, st, ws, ws_bytes, cost0, q_cand, 0);
}

int vapr_optimizer_step(vapr_ctx* ctx, const vapr_lbfgs_state* st, const void* ws, size_t ws_bytes,
                        const double* cost_cand, float* q_cand) {
  return run_opt(ctx, st, ws, ws_bytes, cost_cand, q_cand, 1);
}

size_t vapr_packed_bytes(int fmt, int64_t n) {
  if (fmt < VAPR_F32 || fmt > VAPR_E2M1 || n < 0) return 0;  // VAPR_EXMY: vapr_exmy_packed_bytes
  return (size_t)((n * format_bits(fmt) + 7) / 8);
}

size_t vapr_exmy_packed_bytes(int exp_bits, int man_bits, int64_t n) {
  if (exp_bits < 1 || exp_bits > 8 || man_bits < 0 || man_bits > 23 || n < 0) return 0;
  const int64_t q = pxm_per_word(exp_bits, man_bits);
  return (size_t)((n + q - 1) / q) * 4;
}

static int codec_check(int fmt, int scale_exp, const void* in, const void* out, int64_t n) {
  vapr_tensor_format f{fmt, scale_exp, 0, 0};
  if (fmt == VAPR_EXMY)
    return fail(nullptr, VAPR_E_INVALID, "emulated ExMy types: use vapr_quantize_exmy / vapr_dequantize_exmy");
  if (!valid_format(f)) return fail(nullptr, VAPR_E_INVALID, "unknown format or scale out of range");
  if (n < 0 || n > ((int64_t)1 << 32)) return fail(nullptr, VAPR_E_INVALID, "element count out of range");
  if (n > 0 && (!in || !out)) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 3)
    return fail(nullptr, VAPR_E_INVALID, "buffers must be 4-byte aligned");
  return VAPR_OK;
}

int vapr_quantize(int fmt, int scale_exp, const float* in, void* out, int64_t n, void* hip_stream) {
  int st = codec_check(fmt, scale_exp, in, out, n);
  if (st || n == 0) return st;
  hipError_t e = launch_quantize(static_cast<hipStream_t>(hip_stream), fmt, std::ldexp(1.0f, -scale_exp), in,
                                 static_cast<uint8_t*>(out), n);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_quantize launch");
}

int vapr_dequantize(int fmt, int scale_exp, const void* in, float* out, int64_t n, void* hip_stream) {
  int st = codec_check(fmt, scale_exp, in, out, n);
  if (st || n == 0) return st;
  hipError_t e = launch_dequantize(static_cast<hipStream_t>(hip_stream), fmt, std::ldexp(1.0f, scale_exp),
                                   static_cast<const uint8_t*>(in), out, n);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_dequantize launch");
}

static int exmy_codec_check(int exp_bits, int man_bits, int scale_exp, const void* in, const void* out, int64_t n) {
  const vapr_tensor_format f{VAPR_EXMY, scale_exp, exp_bits, man_bits};
  if (!valid_format(f)) return fail(nullptr, VAPR_E_INVALID, "ExMy bits or scale out of range");
  if (n < 0 || n > ((int64_t)1 << 32)) return fail(nullptr, VAPR_E_INVALID, "element count out of range");
  if (n > 0 && (!in || !out)) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 3)
    return fail(nullptr, VAPR_E_INVALID, "buffers must be 4-byte aligned");
  return VAPR_OK;
}

int vapr_quantize_exmy(int exp_bits, int man_bits, int scale_exp, const float* in, void* out, int64_t n,
                       void* hip_stream) {
  int st = exmy_codec_check(exp_bits, man_bits, scale_exp, in, out, n);
  if (st || n == 0) return st;
  hipError_t e = launch_quantize_exmy(static_cast<hipStream_t>(hip_stream), exp_bits, man_bits,
                                      std::ldexp(1.0f, -scale_exp), in, static_cast<uint32_t*>(out), n);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_quantize_pxm launch");
}

int vapr_dequantize_exmy(int exp_bits, int man_bits, int scale_exp, const void* in, float* out, int64_t n,
                         void* hip_stream) {
  int st = exmy_codec_check(exp_bits, man_bits, scale_exp, in, out, n);
  if (st || n == 0) return st;
  hipError_t e = launch_dequantize_exmy(static_cast<hipStream_t>(hip_stream), exp_bits, man_bits,
                                        std::ldexp(1.0f, scale_exp), static_cast<const uint32_t*>(in), out, n);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_dequantize_pxm launch");
}

int vapr_round_exmy(int exp_bits, int man_bits, int scale_exp, const float* in, float* out, int64_t n,
                    void* hip_stream) {
  vapr_tensor_format f{VAPR_EXMY, scale_exp, exp_bits, man_bits};
  if (!valid_format(f)) return fail(nullptr, VAPR_E_INVALID, "ExMy bits or scale out of range");
  if (n < 0 || n > ((int64_t)1 << 32)) return fail(nullptr, VAPR_E_INVALID, "element count out of range");
  if (n == 0) return VAPR_OK;
  if (!in || !out) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  hipError_t e = launch_round_exmy(static_cast<hipStream_t>(hip_stream), exp_bits, man_bits,
                                   std::ldexp(1.0f, -scale_exp), std::ldexp(1.0f, scale_exp), in, out, n);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_round_exmy launch");
}

// ---- learned seeder ---------------------------------------------------------------------------

int vapr_seed_occupancy(int n_worlds, int n_cuboids, const float* pose, const float* half_ext, float* occ,
                        void* hip_stream) {
  if (n_worlds < 1 || n_worlds > (1 << 20) || n_cuboids < 0 || n_cuboids > MAX_CUBOIDS)
    return fail(nullptr, VAPR_E_INVALID, "world shape out of range");
  if (!occ || (n_cuboids > 0 && (!pose || !half_ext))) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  hipError_t e = launch_occupancy(static_cast<hipStream_t>(hip_stream), n_worlds, n_cuboids, pose, half_ext, occ);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_occupancy launch");
}

int vapr_seed_features(int n, const float* start, const float* goal, const float* occ, uint16_t* x,
                       void* hip_stream) {
  if (n < 0) return fail(nullptr, VAPR_E_INVALID, "n < 0");
  if (n == 0) return VAPR_OK;
  if (n > INT32_MAX / (SEED_IN_PAD / 8)) return fail(nullptr, VAPR_E_INVALID, "n too large");
  if (!start || !goal || !occ || !x) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  if (reinterpret_cast<uintptr_t>(x) % 16) return fail(nullptr, VAPR_E_INVALID, "x must be 16-byte aligned");
  hipError_t e = launch_features(static_cast<hipStream_t>(hip_stream), n, start, goal, occ, x);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_features launch");
}

int vapr_seed_trajectories(int n, const float* y, const float* start, const float* goal, float* out,
                           void* hip_stream) {
  if (n < 0) return fail(nullptr, VAPR_E_INVALID, "n < 0");
  if (n == 0) return VAPR_OK;
  if (!y || !start || !goal || !out) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  hipError_t e = launch_seed_traj(static_cast<hipStream_t>(hip_stream), n, y, start, goal, out);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_seed_traj launch");
}

int vapr_gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t a_ms, int64_t a_ks, const uint16_t* B,
                   int64_t b_ks, int64_t b_ns, const float* bias, int epilogue, float* aux, float* C,
                   uint16_t* C_bf16, int64_t ldc, void* hip_stream) {
  if (M < 1 || N < 1 || K < 32 || K % 32) return fail(nullptr, VAPR_E_INVALID, "GEMM shape (K a multiple of 32)");
  if (!A || !B || (!C && !C_bf16)) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  if (epilogue < VAPR_GEMM_PLAIN || epilogue > VAPR_GEMM_GELU_GRAD) return fail(nullptr, VAPR_E_INVALID, "epilogue");
  if (epilogue == VAPR_GEMM_GELU_GRAD && !aux) return fail(nullptr, VAPR_E_INVALID, "GELU_GRAD needs aux");
  if (ldc < N) return fail(nullptr, VAPR_E_INVALID, "ldc < N");
  const bool a_k = a_ks == 1, b_n = b_ns == 1;
  if (!(a_k || a_ms == 1) || !(b_n || b_ks == 1)) return fail(nullptr, VAPR_E_INVALID, "one stride of A and B must be 1");
  if (a_k && (a_ms % 8 || reinterpret_cast<uintptr_t>(A) % 16))
    return fail(nullptr, VAPR_E_INVALID, "k-contiguous A needs a row stride multiple of 8 and 16-byte alignment");
  if (!b_n && (b_ns % 8 || reinterpret_cast<uintptr_t>(B) % 16))
    return fail(nullptr, VAPR_E_INVALID, "k-contiguous B needs a column stride multiple of 8 and 16-byte alignment");
  GemmArgs g{M, N, K, A, a_ms, a_ks, B, b_ks, b_ns, bias, epilogue, aux, C, C_bf16, ldc, nullptr, nullptr};
  hipError_t e = launch_gemm_bf16(static_cast<hipStream_t>(hip_stream), g, a_k, b_n);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_gemm_bf16 launch");
}

int vapr_seed_head(int n, const uint16_t* a3, int64_t lda, const uint16_t* W4, const float* b4, const float* start,
                   const float* goal, float* traj, void* hip_stream) {
  if (n < 0) return fail(nullptr, VAPR_E_INVALID, "n < 0");
  if (n == 0) return VAPR_OK;
  if (!a3 || !W4 || !b4 || !start || !goal || !traj) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  if (lda < SEED_HID || lda % 8 || reinterpret_cast<uintptr_t>(a3) % 16)
    return fail(nullptr, VAPR_E_INVALID, "a3 needs a row stride >= 256, a multiple of 8, and 16-byte alignment");
  GemmArgs g{n, SEED_OUT, SEED_HID, a3, lda, 1, W4, SEED_OUT, 1, b4, GEMM_SEED_TRAJ, nullptr, traj, nullptr,
             SEED_OUT, start, goal};
  hipError_t e = launch_gemm_bf16(static_cast<hipStream_t>(hip_stream), g, true, true);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_gemm_bf16 (seed head) launch");
}

int vapr_seed_loss(int n, const float* y, const float* targets, const float* valid, int n_valid, double* loss,
                   int32_t* assign, float* dy, double* partial, void* hip_stream) {
  if (n < 1 || n_valid < 1 || n_valid > 8 * n) return fail(nullptr, VAPR_E_INVALID, "n or n_valid out of range");
  if (!y || !targets || !valid || !loss || !assign || !dy || !partial) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  const float coef = (float)(2.0 / ((double)SEED_TRAJ * n_valid));
  hipError_t e = launch_seed_loss(static_cast<hipStream_t>(hip_stream), n, y, targets, valid, coef, partial, assign,
                                  dy, 1.0 / n_valid, loss);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_seed_loss launch");
}

int vapr_seed_deviations(int n, int m, const float* traj, const float* start, const float* goal, float* dev,
                         void* hip_stream) {
  if (n < 0 || m < 1) return fail(nullptr, VAPR_E_INVALID, "n < 0 or m < 1");
  if (n == 0) return VAPR_OK;
  if (!traj || !start || !goal || !dev) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  hipError_t e = launch_seed_dev(static_cast<hipStream_t>(hip_stream), n, m, traj, start, goal, dev);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_seed_dev launch");
}

int vapr_column_sum(int M, int N, const float* X, int64_t ldx, float* out, void* hip_stream) {
  if (M < 1 || N < 1 || ldx < N) return fail(nullptr, VAPR_E_INVALID, "shape");
  if (!X || !out) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  hipError_t e = launch_column_sum(static_cast<hipStream_t>(hip_stream), M, N, X, ldx, out);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_column_sum launch");
}

int vapr_adam(int64_t n, float* w, uint16_t* w_bf16, const float* g, float* m, float* v, float lr, float b1,
              float b2, float eps, int step, void* hip_stream) {
  if (n < 0 || step < 1) return fail(nullptr, VAPR_E_INVALID, "n < 0 or step < 1");
  if (!(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f && eps >= 0.f && std::isfinite(lr)))
    return fail(nullptr, VAPR_E_INVALID, "Adam hyper-parameters");
  if (n == 0) return VAPR_OK;
  if (!w || !g || !m || !v) return fail(nullptr, VAPR_E_INVALID, "null pointer");
  AdamArgs a{lr, b1, b2, eps, (float)(1.0 / (1.0 - std::pow((double)b1, step))),
             (float)(1.0 / (1.0 - std::pow((double)b2, step)))};
  hipError_t e = launch_adam(static_cast<hipStream_t>(hip_stream), n, w, w_bf16, g, m, v, a);
  return e == hipSuccess ? VAPR_OK : hip_fail(nullptr, e, "k_adam launch");
}

static int ws_io(vapr_ctx* ctx, int n_worlds, int tpw, int T, int n_ls, void* ws, size_t ws_bytes, int tensor,
                 void* buf, size_t buf_bytes, int direction) {
  int64_t B;
  int st = check_shape(ctx, n_worlds, tpw, T, n_ls, &B);
  if (st) return st;
  if (!ws || !buf) return fail(ctx, VAPR_E_INVALID, "null pointer");
  if (tensor < VAPR_T_LINK_POSES || tensor > VAPR_T_POSE_COST) return fail(ctx, VAPR_E_INVALID, "unknown tensor");
  if (tensor == VAPR_T_POSE_COST && !ctx->prec.pose)
    return fail(ctx, VAPR_E_INVALID, "no pose cost: no goal poses are set");
  if ((tensor == VAPR_T_SWEPT_GRAD || tensor == VAPR_T_SWEPT_COST) && !ctx->prec.sweep)
    return fail(ctx, VAPR_E_INVALID, "no swept tensors: the swept term is off (swept_steps = 0)");
  const Layout L = make_layout(B, ctx->n_s, ctx->prec);
  if (ws_bytes < L.bytes) return fail(ctx, VAPR_E_INVALID, "workspace too small");
  if (direction == 0) {
    const char* why = nullptr;
    const WsRecord* r = current_record(ctx, ws, &why);
    if (!r) return fail(ctx, VAPR_E_STATE, why);
    if (r->B != B || r->T != T || r->n_ls != n_ls)
      return fail(ctx, VAPR_E_STATE, "workspace holds a forward pass of another shape");
  }
  if (tensor == VAPR_T_SELF_COST || tensor == VAPR_T_BOUND_COST || tensor == VAPR_T_SWEPT_COST ||
      tensor == VAPR_T_POSE_COST) {
    if (buf_bytes < (size_t)B * 4) return fail(ctx, VAPR_E_INVALID, "buffer too small");
    const int slot = tensor == VAPR_T_SELF_COST    ? OFF_SELF
                     : tensor == VAPR_T_BOUND_COST ? OFF_BOUND
                     : tensor == VAPR_T_SWEPT_COST ? OFF_SWEPT
                                                   : OFF_POSE;
    char* arr = static_cast<char*>(ws) + L.off[slot];
    st = timed(ctx, K_REPACK,
               [&] {
                 return direction == 0 ? hipMemcpyAsync(buf, arr, (size_t)B * 4, hipMemcpyDeviceToDevice, ctx->stream)
                                       : hipMemcpyAsync(arr, buf, (size_t)B * 4, hipMemcpyDeviceToDevice, ctx->stream);
               },
               "scalar copy");
  } else {
    if (tensor == VAPR_T_LINK_POSES && ctx->prec.recompute)
      return fail(ctx, VAPR_E_INVALID, "no link-pose tensor in recompute mode");
    const int ecfg = tensor_count(ctx, tensor);
    const int t = tensor == VAPR_T_SWEPT_GRAD ? T_X : tensor;  // X is laid out like G
    const TensorFormat& tf = ctx->prec.t[t];
    const size_t need = tf.fmt == PXM ? vapr_exmy_packed_bytes(tf.xe, tf.xm, B * ecfg) : vapr_packed_bytes(tf.fmt, B * ecfg);
    if (buf_bytes < need) return fail(ctx, VAPR_E_INVALID, "buffer too small");
    if (tf.fmt == PXM && (reinterpret_cast<uintptr_t>(buf) & 3))
      return fail(ctx, VAPR_E_INVALID, "packed ExMy buffers must be 4-byte aligned");
    const TV tv = tensor_view(ws, L, ctx->prec, t);
    const int n_s = ctx->n_s;
    const int shape_of = t == T_X ? T_G : t;
    st = timed(ctx, K_REPACK,
               [&] {
                 return launch_repack(ctx->stream, shape_of, tv, B, ecfg, n_s, static_cast<uint8_t*>(buf), direction);
               },
               "repack launch");
  }
  if (st) return st;
  if (direction == 1) {
    // an imported tensor stands for a forward pass: a new pass number in the header and the record
    ctx->ws.erase(ws);
    const WsRecord rec = new_record(ctx, n_worlds, tpw, T, n_ls, B);
    const hipError_t e = launch_ws_stamp(ctx->stream, stamp_of(ctx, ws, rec));
    if (e != hipSuccess) return hip_fail(ctx, e, "k_ws_stamp launch");
    ctx->ws[ws] = rec;
  }
  return VAPR_OK;
}

int vapr_ws_export(vapr_ctx* ctx, int n_worlds, int tpw, int T, int n_ls, const void* ws, size_t ws_bytes, int tensor,
                   void* out, size_t out_bytes) {
  return ws_io(ctx, n_worlds, tpw, T, n_ls, const_cast<void*>(ws), ws_bytes, tensor, out, out_bytes, 0);
}

int vapr_ws_import(vapr_ctx* ctx, int n_worlds, int tpw, int T, int n_ls, void* ws, size_t ws_bytes, int tensor,
                   const void* in, size_t in_bytes) {
  return ws_io(ctx, n_worlds, tpw, T, n_ls, ws, ws_bytes, tensor, const_cast<void*>(in), in_bytes, 1);
}

int vapr_ws_reset(vapr_ctx* ctx, void* ws, size_t ws_bytes) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!ws) return fail(ctx, VAPR_E_INVALID, "null pointer");
  if (ws_bytes < WS_HEADER_BYTES) return fail(ctx, VAPR_E_INVALID, "workspace smaller than its header");
  // forget every record inside the buffer: their memory has been handed out again
  const char* lo = static_cast<const char*>(ws);
  const char* hi = lo + ws_bytes;
  for (auto it = ctx->ws.begin(); it != ctx->ws.end();) {
    const char* p = static_cast<const char*>(it->first);
    if (p >= lo && p < hi) it = ctx->ws.erase(it);
    else ++it;
  }
  WsStamp st{};
  st.hdr = static_cast<uint64_t*>(ws);
  const hipError_t e = launch_ws_stamp(ctx->stream, st);
  return e == hipSuccess ? VAPR_OK : hip_fail(ctx, e, "k_ws_stamp launch");
}

int vapr_ws_poison(vapr_ctx* ctx, void* ws, size_t ws_bytes) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (!ws) return fail(ctx, VAPR_E_INVALID, "null pointer");
  if (ws_bytes < WS_HEADER_BYTES || ws_bytes % 4) return fail(ctx, VAPR_E_INVALID, "workspace size");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(ctx, VAPR_E_INVALID, "workspace not 256-byte aligned");
  int st = vapr_ws_reset(ctx, ws, ws_bytes);
  if (st) return st;
  uint32_t* body = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + WS_HEADER_BYTES);
  const hipError_t e = launch_fill_u32(ctx->stream, body, (int64_t)((ws_bytes - WS_HEADER_BYTES) / 4), 0xFFFFFFFFu);
  return e == hipSuccess ? VAPR_OK : hip_fail(ctx, e, "k_fill_u32 launch");
}

int vapr_ws_census(vapr_ctx* ctx, int n_worlds, int tpw, int T, int n_ls, const void* ws, size_t ws_bytes,
                   int tensor, int64_t* counts) {
  int64_t B;
  int st = check_shape(ctx, n_worlds, tpw, T, n_ls, &B);
  if (st) return st;
  if (!ws || !counts) return fail(ctx, VAPR_E_INVALID, "null pointer");
  if (tensor < VAPR_T_LINK_POSES || tensor > VAPR_T_SWEPT_GRAD || tensor == VAPR_T_SELF_COST ||
      tensor == VAPR_T_BOUND_COST)
    return fail(ctx, VAPR_E_INVALID, "census covers the stored code tensors only");
  if (tensor == VAPR_T_LINK_POSES && ctx->prec.recompute)
    return fail(ctx, VAPR_E_INVALID, "no link-pose tensor in recompute mode");
  if (tensor == VAPR_T_SWEPT_GRAD && !ctx->prec.sweep)
    return fail(ctx, VAPR_E_INVALID, "no swept tensors: the swept term is off (swept_steps = 0)");
  const Layout L = make_layout(B, ctx->n_s, ctx->prec);
  if (ws_bytes < L.bytes) return fail(ctx, VAPR_E_INVALID, "workspace too small");
  const char* why = nullptr;
  const WsRecord* r = current_record(ctx, ws, &why);
  if (!r) return fail(ctx, VAPR_E_STATE, why);
  if (r->B != B || r->T != T || r->n_ls != n_ls)
    return fail(ctx, VAPR_E_STATE, "workspace holds a forward pass of another shape");
  if (!ctx->d_census && (st = upload(ctx, &ctx->d_census, static_cast<const unsigned long long*>(nullptr), 2)))
    return st;
  const unsigned long long zero[2] = {0ull, 0ull};
  VAPR_HIP(ctx, hipMemcpyAsync(ctx->d_census, zero, sizeof zero, hipMemcpyHostToDevice, ctx->stream));
  const int t = tensor == VAPR_T_SWEPT_GRAD ? T_X : tensor;
  const TV tv = tensor_view(const_cast<void*>(ws), L, ctx->prec, t);
  const hipError_t e = launch_code_census(ctx->stream, t == T_X ? T_G : t, tv, B, tensor_count(ctx, tensor),
                                          ctx->d_census);
  if (e != hipSuccess) return hip_fail(ctx, e, "k_code_census launch");
  unsigned long long got[2];
  VAPR_HIP(ctx, hipMemcpyAsync(got, ctx->d_census, sizeof got, hipMemcpyDeviceToHost, ctx->stream));
  VAPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  counts[0] = (int64_t)got[0];
  counts[1] = (int64_t)got[1];
  return VAPR_OK;
}

int vapr_collision_free(vapr_ctx* ctx, int n_worlds, int tpw, int T, int n_ls, const void* ws, size_t ws_bytes,
                        int32_t* free_cfg) {
  int64_t B;
  int st = check_shape(ctx, n_worlds, tpw, T, n_ls, &B);
  if (st) return st;
  if (!ws || !free_cfg) return fail(ctx, VAPR_E_INVALID, "null pointer");
  const Layout L = make_layout(B, ctx->n_s, ctx->prec);
  if (ws_bytes < L.bytes) return fail(ctx, VAPR_E_INVALID, "workspace too small");
  const char* why = nullptr;
  const WsRecord* r = current_record(ctx, ws, &why);
  if (!r) return fail(ctx, VAPR_E_STATE, why);
  if (r->B != B || r->T != T || r->n_ls != n_ls)
    return fail(ctx, VAPR_E_STATE, "workspace holds a forward pass of another shape");
  void* w = const_cast<void*>(ws);
  const TV tS = tensor_view(w, L, ctx->prec, T_S), tD = tensor_view(w, L, ctx->prec, T_D);
  const float* boundc = reinterpret_cast<const float*>(static_cast<const char*>(ws) + L.off[OFF_BOUND]);
  const RobotArgs R = robot_args(ctx);
  const float eta = ctx->params.eta;
  const hipError_t e = launch_collision_free(ctx->stream, R, tS, tD, boundc, eta, B, free_cfg);
  return e == hipSuccess ? VAPR_OK : hip_fail(ctx, e, "k_collision_free launch");
}

int vapr_sync(vapr_ctx* ctx) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  VAPR_HIP(ctx, hipSetDevice(ctx->device));
  VAPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  uint32_t flag = 0;
  VAPR_HIP(ctx, hipMemcpy(&flag, ctx->d_status, sizeof flag, hipMemcpyDeviceToHost));
  if (!flag) return VAPR_OK;
  const uint32_t zero = 0;
  VAPR_HIP(ctx, hipMemcpy(ctx->d_status, &zero, sizeof zero, hipMemcpyHostToDevice));
  return fail(ctx, VAPR_E_STATE,
              "a backward or optimiser call met a workspace that no longer held the forward pass it was issued "
              "for (its gradients were written as NaN, optimiser state was left unchanged)");
}

int vapr_profile_enable(vapr_ctx* ctx, int enable) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  for (auto& pe : ctx->prof_live) {
    ctx->prof_pool.push_back(pe.start);
    ctx->prof_pool.push_back(pe.stop);
  }
  ctx->prof_live.clear();
  for (int i = 0; i < N_KERNEL_IDS; ++i) {
    ctx->prof_ms[i] = 0;
    ctx->prof_n[i] = 0;
  }
  ctx->prof = enable != 0;
  return VAPR_OK;
}

int vapr_profile_read(vapr_ctx* ctx, double* total_ms, int64_t* launches, int n_ids) {
  if (!ctx) return fail(nullptr, VAPR_E_INVALID, "null context");
  if (n_ids < 0 || (n_ids > 0 && (!total_ms || !launches))) return fail(ctx, VAPR_E_INVALID, "bad output arrays");
  VAPR_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& pe : ctx->prof_live) {
    float ms = 0.f;
    VAPR_HIP(ctx, hipEventElapsedTime(&ms, pe.start, pe.stop));
    ctx->prof_ms[pe.id] += ms;
    ctx->prof_n[pe.id] += 1;
    ctx->prof_pool.push_back(pe.start);
    ctx->prof_pool.push_back(pe.stop);
  }
  ctx->prof_live.clear();
  for (int i = 0; i < n_ids; ++i) {
    total_ms[i] = i < N_KERNEL_IDS ? ctx->prof_ms[i] : 0.0;
    launches[i] = i < N_KERNEL_IDS ? ctx->prof_n[i] : 0;
  }
  return VAPR_OK;
}

}  // extern "C"
