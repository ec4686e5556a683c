/*
 * vapr.h -- C ABI of the variable-precision trajectory-optimisation cost library for MI355X.
 *
 * The library evaluates, for a batch of joint configurations of a 7-joint serial arm in worlds of
 * oriented cuboids, the trajectory-optimisation cost and its joint-space gradient, and runs the
 * line-search + L-BFGS step that consumes them (the optimisation iteration of Sec. III-B of
 * "VaPr: Variable-Precision Tensors to Accelerate Robot Motion Planning").  The five large
 * intermediate tensors of that iteration -- link poses L, sphere positions S, per-sphere distances
 * D, sphere-position gradients G and joint gradients J (Sec. III-C) -- are stored in per-tensor
 * formats chosen from FP32, FP16, BF16, FP8 E4M3/E5M2, FP6 E3M2 and FP4 E2M1 (Sec. IV-A, V-B);
 * all arithmetic is FP32, reductions feeding the line search are FP64.
 *
 * Conventions shared by every call
 *  - Every function returns a vapr_status.  Argument errors are detected on the host before any
 *    work is queued and leave all state unchanged.  VAPR_E_HIP reports a failed HIP call or kernel
 *    launch; faults inside kernels surface at the caller's next synchronisation.
 *  - "dev" pointers are device memory on the context's device, "host" pointers host memory.
 *    Device buffers must be 4-byte aligned (torch allocations are).  The caller owns every buffer it
 *    passes; the library owns only its copies of the robot and world tables.
 *  - All device work is queued on the context's HIP stream, asynchronously; host pointers are
 *    consumed before the call returns.
 *  - A context is used by one host thread at a time.
 *  - Configuration layout: a batch of B = n_worlds * traj_per_world * n_ls * T configurations is
 *    ordered b = ((traj * n_ls + cand) * T + t) with traj = world * traj_per_world + seed, so the
 *    T timesteps of one trajectory candidate are contiguous and all candidates of a world are
 *    contiguous.  q is row-major [B][7] FP32.
 */
#ifndef VAPR_H
#define VAPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VAPR_ABI_VERSION 4

typedef enum {
  VAPR_OK = 0,
  VAPR_E_INVALID = 1,      /* bad argument: null pointer, size out of range, unknown enum, ...   */
  VAPR_E_OOM = 2,          /* the library could not allocate its robot/world tables             */
  VAPR_E_HIP = 3,          /* a HIP runtime call or kernel launch failed                        */
  VAPR_E_UNSUPPORTED = 4,  /* valid request this build does not implement (e.g. n_joints != 7)  */
  VAPR_E_STATE = 5         /* call order violated: no robot/world, workspace not from a forward
                              pass of this shape and precision, optimiser shape mismatch        */
} vapr_status;

/* Storage formats (Sec. IV-A).  Encoding rounds to nearest, ties to even; subnormals are kept.
 * FP16/BF16 overflow to Inf (IEEE); E4M3/E5M2/E3M2/E2M1 saturate to their largest finite value,
 * Inf inputs included.  NaN gives a NaN code where the format has one and is outside the contract
 * for E3M2/E2M1.  Packed layout: element i occupies bits [b*i, b*i+b) of a little-endian bit
 * stream (b = 32, 16, 16, 8, 8, 6, 4). */
typedef enum {
  VAPR_F32 = 0,
  VAPR_F16 = 1,   /* E5M10, bias 15, max 65504            */
  VAPR_BF16 = 2,  /* E8M7,  bias 127                      */
  VAPR_E4M3 = 3,  /* bias 7, max 448, NaN = S.1111.111    */
  VAPR_E5M2 = 4,  /* bias 15, max 57344                   */
  VAPR_E3M2 = 5,  /* FP6, bias 3, max 28, no Inf/NaN      */
  VAPR_E2M1 = 6,  /* FP4, bias 1, max 6, no Inf/NaN       */
  VAPR_EXMY = 7   /* any type of the paper's search space (Sec. IV-A, IV-B), 1 <= exp_bits <= 8,
                     0 <= man_bits <= 23, b = 1 + exp_bits + man_bits bits, encoded in software:
                     bias 2^(exp_bits-1) - 1, subnormals kept, ties to even; E5M10 and the
                     8-exponent-bit types (E8M7, E8M23, ...) follow IEEE (overflow to Inf, Inf and
                     NaN codes in the top exponent field), every other type has no Inf/NaN and
                     saturates (a NaN input stores the largest magnitude: outside the contract).
                     Code: sign at bit b-1, biased exponent, mantissa.  Stored packed
                     floor(32 / b) codes to a 32-bit word from the low bits up (the paper's
                     register packing: 3 FP10, 5 FP6, 6 FP5 ...), the unused top bits zero; so
                     the tensor moves b-bit codes, not FP32 values.  Takes a scale like the
                     others. */
} vapr_format;

/* One stored tensor's format with a power-of-two scale: a value x is stored as
 * enc(fp32(x) * 2^-scale_exp) and read back as the FP32 value dec(code) * 2^scale_exp (exact; only
 * scaled-up BF16 codes can leave FP32 range and read back as Inf).  -16 <= scale_exp <= 16, and
 * scale_exp must be 0 for VAPR_F32. */
typedef struct {
  int32_t fmt;
  int32_t scale_exp;
  int32_t exp_bits;  /* VAPR_EXMY only (ignored otherwise) */
  int32_t man_bits;
} vapr_tensor_format;

/* Precision assignment, one format per large tensor (Sec. IV-B).  recompute_poses != 0 drops the
 * link-pose tensor: the backward pass recomputes the poses from q instead of reading L. */
typedef struct {
  vapr_tensor_format link_poses;   /* L: links 1..8 as row-major 3x4 [R | t], 96 values/config  */
  vapr_tensor_format sphere_pos;   /* S: sphere centres in the world frame, n_s x 3 per config  */
  vapr_tensor_format sphere_dist;  /* D: activation depth max(0, eta - clearance), n_s          */
  vapr_tensor_format sphere_grad;  /* G: d(config cost)/d(sphere centre), n_s x 3               */
  vapr_tensor_format joint_grad;   /* J: d(loss)/dq, 7 per config                               */
  int32_t recompute_poses;
  vapr_tensor_format swept_grad;   /* X: swept-term gradient w.r.t. the sphere centres, n_s x 3
                                      (stored only while swept_steps > 0)                       */
} vapr_precision;

/* Cost weights (Sec. III-B step (3); the paper gives no values).
 * configuration cost c = w_coll * sum_s d_s^2 + w_self * sum_pairs max(0, eta - e)^2
 *                        + w_bound * sum_j (max(0, q_j - hi_j)^2 + max(0, lo_j - q_j)^2)
 *                        + swept cost of the segment (t, t+1)
 * trajectory cost      = sum_t c_t + w_smooth * sum_t |q_{t+1} - q_t|^2
 * with d_s = max(0, eta - min_k(sd_k(p_s) - r_s)) and e = |p_a - p_b| - r_a - r_b.
 * Swept term (the swept collision of trajectory optimisation, whose output is the paper's fifth
 * large tensor, Sec. III-C; the paper does not define the sweep): with k = swept_steps > 0, each
 * sphere centre is sampled at p_j = (1 - u_j) p_s(t) + u_j p_s(t+1), u_j = j / (k + 1), j = 1..k,
 * between the stored positions of consecutive timesteps of one trajectory-candidate, and the
 * segment adds (w_swept / k) sum_s sum_j d(p_j)^2 to configuration t (nothing for the last
 * timestep).  Its gradient w.r.t. the sphere centres, summed over the two segments at each
 * timestep, is the stored tensor X; the backward pass adds it to G.
 * Pose cost (inverse kinematics, Sec. II-A, III-B; no formula in the paper): with goal poses set,
 * each configuration also pays w_goal_pos |p - p_g|^2 + w_goal_rot ||R - R_g||_F^2 for its link-8
 * pose [R | p] against the goal [R_g | p_g] of its world.
 * Defaults: eta 0.02 m, w_coll 100, w_self 100, w_bound 10, w_smooth 1, swept_steps 0 (off),
 * w_swept 100, w_goal_pos 100, w_goal_rot 10.  0 <= swept_steps <= 16.  Changing swept_steps
 * changes the workspace size, as does setting or clearing goal poses. */
typedef struct {
  float eta;
  float w_coll;
  float w_self;
  float w_bound;
  float w_smooth;
  int32_t swept_steps;
  float w_swept;
  float w_goal_pos;  /* pose cost weights (used while goal poses are set, vapr_set_goals) */
  float w_goal_rot;
} vapr_cost_params;

typedef struct vapr_ctx vapr_ctx;

/* Library ABI version (VAPR_ABI_VERSION). */
int vapr_abi_version(void);

/* Create a context on HIP device `device` queuing work on `hip_stream` (a hipStream_t; NULL is the
 * null stream).  Defaults: all tensors FP32 stored mode, default cost weights.  *out is set on
 * success only. */
int vapr_create(vapr_ctx** out, int device, void* hip_stream);
/* Free the context and the library-owned tables.  NULL is accepted. */
int vapr_destroy(vapr_ctx* ctx);
/* Replace the stream used by later calls. */
int vapr_set_stream(vapr_ctx* ctx, void* hip_stream);

/* Upload the arm and its sphere model (Sec. II-B: kinematics and self-distance queries).  Host
 * arrays, copied:
 *   fixed_tf      [n_joints+1][3][4]  F_1..F_8; T_j = T_{j-1} F_j Rz(q_j) (j <= 7), T_8 = T_7 F_8,
 *                                      T_0 = I.  Each rotation block must satisfy |R^T R - I| < 1e-5.
 *   sphere_center [n_spheres][3]       in the frame of the sphere's link
 *   sphere_radius [n_spheres]          > 0
 *   sphere_link   [n_spheres]          link index 0..8 (0 = fixed base)
 *   pairs         [n_pairs][2]         self-collision sphere pairs, a != b
 *   q_lo, q_hi    [n_joints]           joint limits, q_lo <= q_hi
 * Limits: n_joints == 7 (else VAPR_E_UNSUPPORTED), 1 <= n_spheres <= 256, 0 <= n_pairs <= 4096.
 * Replaces a previous robot; workspaces sized for another sphere count become invalid. */
int vapr_set_robot(vapr_ctx* ctx, int n_joints, const float* fixed_tf, int n_spheres,
                   const float* sphere_center, const float* sphere_radius, const int32_t* sphere_link,
                   int n_pairs, const int32_t* pairs, const float* q_lo, const float* q_hi);

/* The robot's reach: bounds on |value| of every stored link-pose entry (at least 1, the rotation
 * entries) and every sphere-centre coordinate over all configurations (metres), the quantities
 * the overflow guard of vapr_set_precision compares with the formats' ranges.  For choosing scales. */
int vapr_robot_reach(const vapr_ctx* ctx, double* link_poses, double* sphere_pos);

/* Upload the worlds (Sec. II-B: robot-environment distance queries).  Host arrays, copied:
 *   pose     [n_worlds][n_cuboids][3][4]  world <- box transform [R | c]; |R^T R - I| < 1e-5
 *   half_ext [n_worlds][n_cuboids][3]     > 0
 * Limits: 1 <= n_worlds <= 65536, 0 <= n_cuboids <= 256. */
int vapr_set_worlds(vapr_ctx* ctx, int n_worlds, int n_cuboids, const float* pose, const float* half_ext);

/* Goal poses of inverse kinematics, one per world: goal host [n][3][4], row-major [R_g | p_g] of
 * link 8 (R_g a rotation to 1e-5).  n = 0 clears them (no pose cost).  Copied; a forward pass with
 * goals needs n >= its n_worlds.  Inverse kinematics runs as trajectories of one timestep
 * (T = 1), whose rows the optimiser leaves free (vapr_lbfgs_state.free_ends = 1). */
int vapr_set_goals(vapr_ctx* ctx, int n, const float* goal);

/* Select the storage format of each large tensor (Sec. IV-B, V-B).  Unknown format or scale out
 * of range -> VAPR_E_INVALID.  Workspaces filled under another precision become invalid.
 * Overflow guard: FP16, BF16 and the IEEE-like emulated types (E5M10, E8My) overflow to Inf.  A
 * forward pass fails with VAPR_E_INVALID, before any launch, when the robot's reach -- the sum of
 * its fixed translation lengths up to a link, plus the sphere offset, at most 1 for rotation
 * entries -- exceeds the largest value of the link-pose or sphere-position format at its scale, so
 * no configuration can store Inf there.  The saturating formats clamp instead. */
int vapr_set_precision(vapr_ctx* ctx, const vapr_precision* p);
int vapr_get_precision(const vapr_ctx* ctx, vapr_precision* p);

/* Set the cost weights (all finite, eta > 0, weights >= 0). */
int vapr_set_cost_params(vapr_ctx* ctx, const vapr_cost_params* p);

/* Exact cuboid culling in the sphere-cost stage (default on).  A voxel grid records, per world,
 * which cuboids can come within eta + max sphere radius of each voxel; a sphere tests only the
 * cuboids marked in its voxel (spheres outside the grid test none).  Results are identical with
 * and without culling (it skips only cuboids whose clearance is >= eta); enable = 0 tests every
 * cuboid.  The grid is rebuilt on the next forward pass after the robot, the worlds or eta change. */
int vapr_set_culling(vapr_ctx* ctx, int enable);

/* Layout of the culling grid of every world: n^3 voxels of edge `cell` from `origin`; voxel
 * (x, y, z) = (floor((p - origin) / cell) per axis, in FP32: (p - origin) * (1 / cell)) has index
 * (z * n + y) * n + x and holds mask_words 32-bit words, bit k of word k / 32 set when cuboid k may
 * lie within reach.  n = 0 when culling is off or the worlds hold no cuboid. */
typedef struct {
  int n;
  int mask_words;
  float origin[3];
  float inv_cell; /* 1 / cell, as the kernels use it */
} vapr_grid_info;

/* Inspect the culling grid (built on demand; needs a robot and worlds): fills *info and, when
 * mask_out is not NULL, copies world `world`'s n^3 * mask_words words to the host buffer mask_out
 * of capacity_words words (VAPR_E_INVALID if too small or world out of range).  Synchronous; for
 * tests and measurement, not for the hot path. */
int vapr_get_culling_grid(vapr_ctx* ctx, int world, vapr_grid_info* info, uint32_t* mask_out,
                          size_t capacity_words);

/* Workspace state.  A workspace holds the forward pass that last completed into it.  Its first 256
 * bytes are a header written by that pass's last kernel: magic, context id, the context's pass
 * number, B, shape, a tag of the precision assignment, robot and cost-parameter generations.  The
 * host keeps a record per workspace address; vapr_cost_bwd, vapr_optimizer_init/step,
 * vapr_cost_fwd_from (first > 1) and vapr_ws_export check it synchronously (VAPR_E_STATE when the
 * workspace holds no forward pass of this context, or one of another shape, or the precision,
 * robot or cost parameters changed since).  The backward and optimiser kernels then compare the
 * header's context id and pass number with the record's before reading anything else: a workspace
 * whose memory was overwritten in the meantime gives NaN gradients (backward) or leaves the
 * optimiser state untouched, and raises a flag that vapr_sync reports.
 *
 * vapr_ws_reset: announce a newly allocated buffer (or one being reused) as a workspace before its
 * first use.  It forgets every record of an address inside [ws, ws + ws_bytes) -- memory that was
 * freed and handed out again must not pass for the forward pass it once held -- and clears the
 * header on the stream.  ws_bytes >= 256. */
int vapr_ws_reset(vapr_ctx* ctx, void* ws, size_t ws_bytes);

/* Debugging aid: vapr_ws_reset, then every byte after the header set to 0xFF on the stream (NaN in
 * FP32, FP16, BF16, FP8; the largest negative magnitude in FP6/FP4 and the saturating ExMy types).
 * A forward and backward pass from a poisoned workspace must give results bit-identical to a clean
 * one: every location a stage reads was written by an earlier stage of the same pass.  ws dev,
 * 256-byte aligned, ws_bytes a multiple of 4. */
int vapr_ws_poison(vapr_ctx* ctx, void* ws, size_t ws_bytes);

/* Census of one stored code tensor (VAPR_T_LINK_POSES, _SPHERE_POS, _SPHERE_DIST, _SPHERE_GRAD,
 * _JOINT_GRAD, _SWEPT_GRAD) of the forward pass ws holds, over its B configurations in canonical
 * order (padding spheres excluded): counts[0] = codes at the format's largest finite magnitude,
 * where a saturating format (FP8, FP6, FP4, the non-IEEE ExMy types) puts every value beyond its
 * range; counts[1] = Inf or NaN codes, where FP32/FP16/BF16 and the IEEE-like ExMy types put them.
 * It watches the static power-of-two scales of Sec. IV-B: counts that appear or grow during an
 * optimisation show values outgrowing the scale.  counts host int64[2]; synchronises the stream
 * (not for graph capture).  VAPR_E_STATE as for vapr_ws_export. */
int vapr_ws_census(vapr_ctx* ctx, int n_worlds, int traj_per_world, int T, int n_ls, const void* ws,
                   size_t ws_bytes, int tensor, int64_t* counts);

/* Collision check of a forward pass (the success test of planning, Sec. VI-A: a trajectory is
 * usable when it is collision-free): free_cfg dev [B] int32 receives 1 for a configuration whose
 * every sphere clears every cuboid (stored activation depth d < eta, i.e. clearance > 0), whose
 * every self pair is apart (|p_a - p_b| - r_a - r_b > 0, from the stored sphere centres) and whose
 * joints are within their limits (bound cost 0), else 0.  ws must hold a forward pass of this shape
 * under the current settings (VAPR_E_STATE otherwise); with reduced formats the test reads the
 * stored (quantised) S and D. */
int vapr_collision_free(vapr_ctx* ctx, int n_worlds, int traj_per_world, int T, int n_ls, const void* ws,
                        size_t ws_bytes, int32_t* free_cfg);

/* Synchronise the context's stream and report what its kernels found: VAPR_E_STATE (once, the flag
 * is cleared) when a backward or optimiser kernel met a workspace whose header did not match. */
int vapr_sync(vapr_ctx* ctx);

/* Bytes of device workspace a forward/backward pass of this batch shape needs at the current
 * precision and swept setting (the 256-byte header, then L, S, D, G, J and two FP32 scalars per
 * configuration, plus X and a third scalar while swept_steps > 0).  Requires a robot. */
int vapr_workspace_size(const vapr_ctx* ctx, int n_worlds, int traj_per_world, int T, int n_ls,
                        size_t* bytes);

/* Forward pass: kinematics -> sphere costs -> aggregation (Sec. III-B steps (2)-(4)).
 *   q         dev [B][7]               configurations in the layout above
 *   ws        dev, ws_bytes >= vapr_workspace_size(...)
 *   cost_traj dev [n_worlds*traj_per_world*n_ls] FP64, trajectory-candidate costs
 *   cost_cfg  dev [B] FP32 per-configuration cost, or NULL
 * 1 <= T <= 4096, 1 <= n_ls <= 4, n_worlds <= the uploaded world count.  Requires robot and
 * worlds (VAPR_E_STATE otherwise).  Records ws as holding a forward pass of this shape. */
int vapr_cost_fwd(vapr_ctx* ctx, int n_worlds, int traj_per_world, int T, int n_ls, const float* q,
                  void* ws, size_t ws_bytes, double* cost_traj, float* cost_cfg);

/* Backward pass (Sec. III-B step (5)): joint gradient of sum_tc grad_cost_traj[tc] * cost_traj[tc].
 *   q              dev [B][7], the same configurations as the forward pass
 *   ws             a workspace filled by vapr_cost_fwd (or vapr_ws_import) of the same shape under
 *                  the current precision, else VAPR_E_STATE
 *   grad_cost_traj dev [n_traj*n_ls] FP64 upstream gradient, or NULL for all ones
 *   grad_q         dev [B][7] FP32 receives dec(enc(J)), the stored joint gradient, or NULL
 * J is always written to ws in its storage format (what vapr_optimizer_step reads). */
int vapr_cost_bwd(vapr_ctx* ctx, const float* q, void* ws, size_t ws_bytes, const double* grad_cost_traj,
                  float* grad_q);

/* Forward and backward pass without a caller workspace and without allocating, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as vapr_cost_fwd followed by vapr_cost_bwd (q,
 * grad_cost_traj, cost_traj, cost_cfg and grad_q as there; grad_cost_traj and cost_cfg may be NULL,
 * grad_q must not be), with the stored tensors kept in a static workspace of 64 MiB on each device
 * the library runs on, held until the process ends.  A batch whose workspace (vapr_workspace_size)
 * exceeds 64 MiB fails with VAPR_E_INVALID before any launch.  The lookup tables must already be
 * built: after changing the robot, worlds, culling or cost parameters run one vapr_cost_fwd first
 * (VAPR_E_STATE otherwise).  Every call on a device shares that device's static workspace, which
 * keeps the last call's contents: calls that overlap on one device (other streams, other contexts,
 * other host threads) race and must be serialised by the caller.  Per-kernel event timing does not
 * cover these launches. */
int vapr_cost_fwd_bwd_noalloc(vapr_ctx* ctx, int n_worlds, int traj_per_world, int T, int n_ls, const float* q,
                              const double* grad_cost_traj, double* cost_traj, float* cost_cfg, float* grad_q);

/* Optimiser state for n_traj trajectories of T timesteps (n = T*7 variables each), all dev,
 * caller-owned (checkpointing is a copy of these buffers).  Unless free_ends, rows t = 0 and
 * t = T-1 keep their values (start and goal of a trajectory). */
typedef struct {
  int32_t n_traj, T, n_ls, m;  /* 1 <= T <= 64, 1 <= n_ls <= 4, 1 <= m <= 8                      */
  float max_step;              /* > 0: cap on a joint's move at alpha = 1 along steepest descent  */
  float* x;                    /* [n_traj][n] current point                                       */
  float* g;                    /* [n_traj][n] gradient at x (pinned rows zero)                    */
  float* d;                    /* [n_traj][n] search direction                                    */
  double* cost;                /* [n_traj]    cost at x                                           */
  float* s_hist;               /* [n_traj][m][n] ring of position differences                     */
  float* y_hist;               /* [n_traj][m][n] ring of gradient differences                     */
  double* rho;                 /* [n_traj][m] 1 / (s.y)                                           */
  int32_t* hist_len;           /* [n_traj]    pairs held (0..m)                                   */
  int32_t* hist_head;          /* [n_traj]    ring slot the next pair goes to                     */
  int32_t* accepted;           /* [n_traj]    last accepted candidate index, -1 = none            */
  int32_t* flags;              /* [n_traj]    bit 0 pair stored, bit 1 direction reset            */
  int32_t free_ends;           /* 0: rows t = 0 and t = T-1 stay fixed (trajectory optimisation); */
                               /* 1: every row moves (inverse kinematics, T = 1)                 */
} vapr_lbfgs_state;

/* Start the optimiser (Sec. III-B step (1)).  x must hold the start point; ws holds a forward +
 * backward pass at x with n_ls = 1 and upstream all ones (its J is the gradient) and cost0 dev
 * [n_traj] FP64 its costs.  Sets g (pinned rows zeroed), cost, the capped steepest-descent direction
 * d = -g * min(1, max_step / |g|_inf), empty history, and writes the first candidates q_cand dev
 * [n_traj][st.n_ls][T][7]: q = fp32(x + alpha_i d), alpha = 1, 1/2, 1/4, 1/8. */
int vapr_optimizer_init(vapr_ctx* ctx, const vapr_lbfgs_state* st, const void* ws, size_t ws_bytes,
                        const double* cost0, float* q_cand);

/* One iteration's line-search selection and L-BFGS update (Sec. III-B steps (6), (7)) followed by
 * the next candidates (step (1)).  ws holds the forward + backward pass of the current candidates
 * (n_ls = st.n_ls, upstream all ones) and cost_cand dev [n_traj*n_ls] FP64 their costs.  Accepts the
 * first candidate meeting Armijo (c1 = 1e-4), else the cheapest if below the current cost, else
 * none (x kept, history cleared, d scaled by alpha_min / 2 to keep backtracking); stores (s, y) when
 * s.y > 1e-10|s||y|; two-loop direction with FP64 dots, or the capped steepest-descent direction
 * when the history is empty or the two-loop result is not a descent direction (history cleared).
 * Writes the next candidates to q_cand, which may alias the buffer the current candidates were
 * read from. */
int vapr_optimizer_step(vapr_ctx* ctx, const vapr_lbfgs_state* st, const void* ws, size_t ws_bytes,
                        const double* cost_cand, float* q_cand);

/* Element-wise codec on the context-free current device (Sec. V-B conversion of a tensor on
 * write and read), storage formats (VAPR_F32 .. VAPR_E2M1).  in/out dev; out holds
 * vapr_packed_bytes(fmt, n) bytes in the packed layout.
 * stream: hipStream_t or NULL.  0 <= n <= 2^32. */
int vapr_quantize(int fmt, int scale_exp, const float* in, void* out, int64_t n, void* hip_stream);
/* Emulated ExMy rounding (VAPR_EXMY rules): out[i] = round(in[i] 2^-scale_exp) 2^scale_exp, FP32
 * device arrays of n elements (in == out allowed). */
int vapr_round_exmy(int exp_bits, int man_bits, int scale_exp, const float* in, float* out, int64_t n,
                    void* hip_stream);
int vapr_dequantize(int fmt, int scale_exp, const void* in, float* out, int64_t n, void* hip_stream);
/* The same for an emulated ExMy type (VAPR_EXMY): out holds vapr_exmy_packed_bytes(exp_bits,
 * man_bits, n) bytes, code i at bits (i % q) b of 32-bit word i / q, q = floor(32 / b). */
int vapr_quantize_exmy(int exp_bits, int man_bits, int scale_exp, const float* in, void* out, int64_t n,
                       void* hip_stream);
int vapr_dequantize_exmy(int exp_bits, int man_bits, int scale_exp, const void* in, float* out, int64_t n,
                         void* hip_stream);
/* Bytes of n packed codes: vapr_packed_bytes for the storage formats (0 for VAPR_EXMY), and
 * 4 ceil(n / floor(32 / b)) for an ExMy type (0 when its bits are out of range). */
size_t vapr_exmy_packed_bytes(int exp_bits, int man_bits, int64_t n);

/* ---- Learned trajectory seeder ----------------------------------------------------------------
 * A network proposes initial trajectories for the optimiser in place of the geometric planner
 * (Sec. II-A: a network trained for an environment can seed trajectory optimisation; Sec. VI-B:
 * better seeding cuts planning attempts).  The paper defines no network.  The one built here maps
 * x = [start (7), goal (7), occupancy (512)] through three GELU layers of 256 units to 8 seeds x 32
 * timesteps x 7 joints (deviations from the straight line, endpoints pinned by the optimiser).
 * Weights enter the matrix cores as BF16 with FP32 accumulation; master weights and Adam moments
 * are FP32.  Every pointer below is device memory on the current device, every call queues its
 * work on `hip_stream` (hipStream_t or NULL) and checks its arguments before any launch. */

/* Occupancy of the cube [-0.75, 0.75]^3 m cut into 8^3 voxels of edge 0.1875 m, per world:
 * occ[w][v] = 1 when the smallest signed distance from voxel v's centre to world w's cuboids is
 * <= 0.09375 m, else 0, with v = (z * 8 + y) * 8 + x.  pose [W][K][3][4] (world <- box [R | c]),
 * half_ext [W][K][3], occ [W][512] FP32.  K = 0 gives an empty grid.  1 <= W <= 2^20, 0 <= K <= 256. */
int vapr_seed_occupancy(int n_worlds, int n_cuboids, const float* pose, const float* half_ext, float* occ,
                        void* hip_stream);

/* Network input rows x[r] = BF16([start[r] (7), goal[r] (7), occ[r] (512), 18 zeros]), x [n][544]
 * (the width padded to a multiple of 32 for the matrix cores).  start, goal [n][7], occ [n][512]. */
int vapr_seed_features(int n, const float* start, const float* goal, const float* occ, uint16_t* x,
                       void* hip_stream);

/* Seed trajectories from the network output: out[r][s][t][j] = start[r][j] + (goal[r][j] -
 * start[r][j]) t / 31 + y[r][(s * 32 + t) * 7 + j] for t = 1..30, and exactly start / goal at
 * t = 0 / 31.  y [n][1792], start, goal [n][7], out [n][8][32][7]. */
int vapr_seed_trajectories(int n, const float* y, const float* start, const float* goal, float* out,
                           void* hip_stream);

enum { VAPR_GEMM_PLAIN = 0, VAPR_GEMM_GELU = 1, VAPR_GEMM_GELU_GRAD = 2 };

/* Z = A B (+ bias[n]) on the matrix cores: A (M x K) and B (K x N) BF16 (uint16 codes), FP32
 * accumulation, for the seeder's dense layers and their backward products.  A(m, k) is
 * A[m * a_ms + k * a_ks], B(k, n) is B[k * b_ks + n * b_ns]; one stride of each operand must be 1,
 * and when it is the k stride the other stride must be a multiple of 8 with the pointer 16-byte
 * aligned.  K must be a positive multiple of 32; M, N >= 1.  Epilogue:
 *   VAPR_GEMM_PLAIN      out = Z
 *   VAPR_GEMM_GELU       aux = Z (when aux is not null: training keeps it for the backward
 *                        pass, inference passes null), out = GELU(Z) = Z Phi(Z)
 *   VAPR_GEMM_GELU_GRAD  out = Z * GELU'(aux)                             (aux read)
 * out goes to C (FP32) and/or C_bf16 (round to nearest even), [M][ldc], ldc >= N; at least one. */
int vapr_gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t a_ms, int64_t a_ks, const uint16_t* B,
                   int64_t b_ks, int64_t b_ns, const float* bias, int epilogue, float* aux, float* C,
                   uint16_t* C_bf16, int64_t ldc, void* hip_stream);

/* The network's output layer fused with the trajectory construction (inference): traj = the
 * trajectories vapr_seed_trajectories builds from y = a3 W4 + b4, bit-identical to that pair of
 * calls, without y ever reaching memory.  a3 [n][lda] BF16 codes (lda >= 256, a multiple of 8,
 * 16-byte aligned) = the last hidden layer, W4 [256][1792] BF16 codes, b4 [1792] FP32, start, goal
 * [n][7] FP32, traj [n][8][32][7] FP32; all device memory owned by the caller. */
int vapr_seed_head(int n, const uint16_t* a3, int64_t lda, const uint16_t* W4, const float* b4, const float* start,
                   const float* goal, float* traj, void* hip_stream);

/* Deviations of m trajectories per problem from the straight line (the inverse of
 * vapr_seed_trajectories, for training targets): dev[r][i][t][j] = traj[r][i][t][j] - line, with
 * line = start[r][j] + (goal[r][j] - start[r][j]) t / 31 for t = 1..30, start at t = 0 and goal at
 * t = 31.  traj, dev [n][m][32][7], start, goal [n][7]; dev may alias traj. */
int vapr_seed_deviations(int n, int m, const float* traj, const float* start, const float* goal, float* dev,
                         void* hip_stream);

/* Min-over-slot matching loss of n problems: y [n][1792] predicted deviations (8 slots x 224),
 * targets [n][1792] (8 target trajectories), valid [n][8] (0 / nonzero).  e_sj = mean over 224 of
 * (y_s - t_j)^2; each valid target takes its smallest e (ties to the lowest slot, assign [n][8]);
 * *loss = sum of those / n_valid (FP64, dev).  dy [n][1792] = dL/dy.  partial [n] doubles is
 * caller-owned scratch.  n_valid must be the number of nonzero valid entries (>= 1). */
int vapr_seed_loss(int n, const float* y, const float* targets, const float* valid, int n_valid, double* loss,
                   int32_t* assign, float* dy, double* partial, void* hip_stream);

/* out[j] = sum_i X[i * ldx + j] for j < N (bias gradients), FP32, rows summed in 16 interleaved
 * groups and then across groups (within M * 2^-24 * sum_i |X[i][j]| of the exact sum).  M, N >= 1,
 * ldx >= N. */
int vapr_column_sum(int M, int N, const float* X, int64_t ldx, float* out, void* hip_stream);

/* Adam step `step` (>= 1) on n FP32 weights w with gradient g and moments m, v (FP32, updated in
 * place): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * w -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps); w_bf16 (may be NULL) receives
 * BF16(w). */
int vapr_adam(int64_t n, float* w, uint16_t* w_bf16, const float* g, float* m, float* v, float lr, float b1,
              float b2, float eps, int step, void* hip_stream);
size_t vapr_packed_bytes(int fmt, int64_t n);

/* Tensor identifiers for workspace export/import. */
typedef enum {
  VAPR_T_LINK_POSES = 0,   /* codes, canonical order [B][8][12]  (stored mode only)          */
  VAPR_T_SPHERE_POS = 1,   /* codes, [B][n_s][3]                                           */
  VAPR_T_SPHERE_DIST = 2,  /* codes, [B][n_s]                                              */
  VAPR_T_SPHERE_GRAD = 3,  /* codes, [B][n_s][3]                                           */
  VAPR_T_JOINT_GRAD = 4,   /* codes, [B][7]                                                */
  VAPR_T_SELF_COST = 5,    /* FP32 [B]: w_self * sum over pairs of max(0, eta - e)^2       */
  VAPR_T_BOUND_COST = 6,   /* FP32 [B]: unweighted joint-limit cost                        */
  VAPR_T_SWEPT_GRAD = 7,   /* codes, [B][n_s][3]            (swept_steps > 0 only)          */
  VAPR_T_SWEPT_COST = 8,   /* FP32 [B]: swept cost of the segment (t, t+1)  (idem)         */
  VAPR_T_POSE_COST = 9     /* FP32 [B]: weighted pose cost      (goal poses set only)      */
} vapr_tensor;

/* Copy one stored tensor between a workspace and a dense buffer in canonical element order, in the
 * packed layout of the tensor's current format (vapr_packed_bytes(fmt, count) bytes; for an ExMy
 * type vapr_exmy_packed_bytes(exp_bits, man_bits, count) bytes, 4-byte aligned).  Used to inspect
 * and to seed individual stages.  Import records ws as holding a forward pass of this shape (so a
 * backward pass may follow).  out/in dev; sizes checked against the shape. */
int vapr_ws_export(vapr_ctx* ctx, int n_worlds, int traj_per_world, int T, int n_ls, const void* ws,
                   size_t ws_bytes, int tensor, void* out, size_t out_bytes);
int vapr_ws_import(vapr_ctx* ctx, int n_worlds, int traj_per_world, int T, int n_ls, void* ws,
                   size_t ws_bytes, int tensor, const void* in, size_t in_bytes);

/* Run the forward pass from stage `first` on: 1 = kinematics (same as vapr_cost_fwd), 2 = sphere
 * costs then aggregation (reads S from ws), 3 = aggregation only (reads D and the two scalars). */
int vapr_cost_fwd_from(vapr_ctx* ctx, int first, int n_worlds, int traj_per_world, int T, int n_ls,
                       const float* q, void* ws, size_t ws_bytes, double* cost_traj, float* cost_cfg);

/* Per-kernel timing with HIP events recorded around each launch on the context's stream.
 * enable != 0 starts recording (and clears totals); vapr_profile_read synchronises the stream and
 * returns, per kernel id (0 fk, 1 sphere_cost, 2 reduce, 3 adjoint, 4 optimizer, 5 codec, 6 repack,
 * 7 swept),
 * the summed milliseconds and launch counts for up to n_ids ids. */
int vapr_profile_enable(vapr_ctx* ctx, int enable);
int vapr_profile_read(vapr_ctx* ctx, double* total_ms, int64_t* launches, int n_ids);

/* Static description of a status code; the last error message of a context (or of the calling
 * thread when ctx is NULL).  Never NULL. */
const char* vapr_status_string(int status);
const char* vapr_last_error(const vapr_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* VAPR_H */
