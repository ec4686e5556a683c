// Workspace layout of the stored tensors (Sec. III-C) in HBM.
//
// Every tensor is a set of dword "planes" per configuration, tiled by blocks of 64 configurations
// (one wavefront, one configuration per lane): dword (b, p) of a tensor with P planes lives at
//     base + ((b >> 6) * P + p) * 64 + (b & 63).
// A wavefront therefore reads or writes 256 contiguous bytes per instruction and a block's whole
// tensor is one contiguous run of P * 256 bytes.
//
// Plane contents (values packed as in codec.hpp, dw(n) = dwords of a packed group of n values; a
// packed ExMy type holds floor(32 / b) codes a dword, so dw(n) = ceil(n / floor(32 / b))):
//   L  links 1..8, [R | t] row-major: 2 groups of 48 values (links 1-4, 5-8)   2 * dw(48) planes
//   S  ceil(n_s/16) groups of 16 spheres x 3 components, plane = (g*3 + c)*dw(16) + w
//   D  ceil(n_s/16) groups of 16 spheres,                plane = g*dw(16) + w
//   G  like S
//   J  one group of 8 values (7 joints + a zero)          dw(8) planes
//   X  swept sphere gradient, like S (only with the swept term on)
// followed by FP32 arrays [Bp]: self cost, bound cost (then X), with the swept term the swept cost,
// and with goal poses the pose cost.  Regions are 256-byte aligned and follow a 256-byte header
// (WsHeader) that the last kernel of every forward pass writes: which context and which of its
// forward passes filled the workspace, under what shape, precision, robot and cost parameters.  The
// consumers of a forward pass (adjoint, optimiser) compare the context id and pass number with the
// ones the host expects before they read anything else.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "codec.hpp"

namespace vapr {

constexpr int N_JOINTS = 7;
constexpr int N_FIXED = 8;          // F_1..F_8
constexpr int N_LINKS = 9;          // link 0 (base) .. link 8
constexpr int LINK_VALUES = 12;
constexpr int L_GROUP = 48;         // 4 links per packed group
constexpr int L_GROUPS = 2;
constexpr int SPH_GROUP = 16;
constexpr int J_GROUP = 8;
constexpr int MAX_SPHERES = 256;
constexpr int MAX_PAIRS = 4096;
constexpr int MAX_CUBOIDS = 256;
constexpr int MAX_T = 4096;
constexpr int MAX_LS = 4;
constexpr int MAX_OPT_T = 64;
constexpr int MAX_HIST = 8;
constexpr int MAX_SWEEP = 16;       // swept samples per segment

struct TensorFormat {
  int fmt;        // storage format (PXM for an emulated ExMy type)
  int scale_exp;
  int xe, xm;     // emulated ExMy type (xe > 0), else 0
};

// dwords of a packed group of n values
__host__ __device__ inline int tf_group_dwords(const TensorFormat& f, int n) {
  return f.fmt == PXM ? pxm_group_dwords(f.xe, f.xm, n) : group_dwords(f.fmt, n);
}

struct PrecisionCfg {
  TensorFormat t[6];  // L, S, D, G, J, X
  int recompute;
  int sweep;          // swept samples per segment (0: no X tensor and no swept cost)
  int pose;           // 1: goal poses are set, the workspace holds the pose cost
};

enum { T_L = 0, T_S = 1, T_D = 2, T_G = 3, T_J = 4, T_X = 5 };
// byte-offset slots of the FP32 arrays and of X
enum { OFF_SELF = 5, OFF_BOUND = 6, OFF_X = 7, OFF_SWEPT = 8, OFF_POSE = 9 };

// Header words (uint64 each) at the start of a workspace.
enum {
  WH_MAGIC = 0,     // WS_MAGIC
  WH_CTX = 1,       // id of the context that ran the forward pass (never 0)
  WH_GEN = 2,       // that context's forward-pass number (never 0)
  WH_B = 3,         // configurations
  WH_SHAPE = 4,     // T | n_ls << 16 | n_s << 24
  WH_PREC = 5,      // hash of the precision assignment (formats, scales, pose mode, swept samples)
  WH_ROBOT = 6,     // robot generation of the context
  WH_PARAMS = 7,    // cost-parameter generation of the context
  WH_WORDS = 8
};
constexpr uint64_t WS_MAGIC = 0x3130535752504156ull;  // "VAPRWS01" little-endian
constexpr size_t WS_HEADER_BYTES = 256;

struct WsStamp {  // written by the forward pass: hdr[i] = w[i]
  uint64_t* hdr;
  uint64_t w[WH_WORDS];
};

struct WsCheck {  // read by the consumers of a forward pass
  const uint64_t* hdr;
  uint64_t ctx, gen;    // expected WH_CTX / WH_GEN
  uint32_t* status;     // bit 0 set when the header does not match (stale workspace)
};

struct Layout {
  int64_t B, Bp, nblk;
  int n_s, n_groups;
  int P[6];             // planes per tensor (X: 0 without the swept term)
  size_t off[10];       // byte offsets: L S D G J self bound X swept pose
  size_t bytes;
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline Layout make_layout(int64_t B, int n_s, const PrecisionCfg& pc) {
  Layout L{};
  L.B = B;
  L.Bp = (B + 63) / 64 * 64;
  L.nblk = L.Bp / 64;
  L.n_s = n_s;
  L.n_groups = (n_s + SPH_GROUP - 1) / SPH_GROUP;
  L.P[T_L] = pc.recompute ? 0 : L_GROUPS * tf_group_dwords(pc.t[T_L], L_GROUP);
  L.P[T_S] = L.n_groups * 3 * tf_group_dwords(pc.t[T_S], SPH_GROUP);
  L.P[T_D] = L.n_groups * tf_group_dwords(pc.t[T_D], SPH_GROUP);
  L.P[T_G] = L.n_groups * 3 * tf_group_dwords(pc.t[T_G], SPH_GROUP);
  L.P[T_J] = tf_group_dwords(pc.t[T_J], J_GROUP);
  L.P[T_X] = pc.sweep ? L.n_groups * 3 * tf_group_dwords(pc.t[T_X], SPH_GROUP) : 0;
  size_t o = WS_HEADER_BYTES;
  for (int i = 0; i < 5; ++i) {
    L.off[i] = o;
    o += align256((size_t)L.P[i] * (size_t)L.Bp * 4);
  }
  L.off[OFF_SELF] = o;
  o += align256((size_t)L.Bp * 4);
  L.off[OFF_BOUND] = o;
  o += align256((size_t)L.Bp * 4);
  L.off[OFF_X] = o;
  o += align256((size_t)L.P[T_X] * (size_t)L.Bp * 4);
  L.off[OFF_SWEPT] = o;
  if (pc.sweep) o += align256((size_t)L.Bp * 4);
  L.off[OFF_POSE] = o;
  if (pc.pose) o += align256((size_t)L.Bp * 4);
  L.bytes = o;
  return L;
}

__host__ __device__ inline int64_t plane_index(int64_t b, int P, int p) {
  return ((b >> 6) * P + p) * 64 + (b & 63);
}

}  // namespace vapr
