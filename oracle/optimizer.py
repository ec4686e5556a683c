"""Parallel line search and L-BFGS step in FP64.  TEST INFRASTRUCTURE.

Each iteration (Sec. III-B) evaluates N step scales of the current direction in one batch (1),
picks one of them by line search (6), and computes the next L-BFGS direction and updates the
history buffers (7).  The paper's own equation reference for the step scales is dangling, so the
rule below is a reading (per trajectory, n = T * 7 variables, the start and goal rows pinned):

  candidates  x_i = fp32(x + alpha_i d),  alpha = (1, 1/2, 1/4, 1/8)[:N]
  accept      the first i with c_i <= c + 1e-4 alpha_i g.d  (Armijo, FP64); otherwise the
              lowest-cost candidate if it is below c (first index on ties); otherwise none:
              stay at x, clear the history and keep backtracking along the same direction,
              d = fp32(d * alpha_min / 2)
  update      s = fp32(x_i - x), y = fp32(g_i - g); keep (s, y, rho = 1/(s.y)) in a ring of m pairs
              when s.y > 1e-10 |s| |y|
  direction   two-loop recursion over the history, initial scaling gamma = s.y / y.y of the newest
              pair, vectors and dots in FP64, d = fp32(-r); with no history, or if g.d >= 0 (the
              history is then cleared), the steepest-descent direction capped so that no joint
              moves more than max_step at alpha = 1: d = fp32(-g * min(1, max_step / |g|_inf))
Gradients are zero on the pinned rows t = 0 and t = T - 1 of trajectory optimisation; inverse
kinematics (one configuration per "trajectory", T = 1) pins nothing.

Parity pins (tests/test_oracle_optimizer.py): the two-loop direction equals the dense inverse-Hessian
product of the BFGS updates built from the same pairs; secant condition H y = s for the newest
pair; Armijo selection worked by hand on 1-D cases; on a convex quadratic the iteration converges.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

ALPHAS = (1.0, 0.5, 0.25, 0.125)
ARMIJO_C1 = 1e-4
CURVATURE_EPS = 1e-10
MAX_STEP = float(np.float32(0.2))  # radians per joint at alpha = 1 (a float32 value, as the GPU holds it)
N_JOINTS = 7


def fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def pin_rows(g: np.ndarray, T: int, pin: bool = True) -> np.ndarray:
    """Zero the start and goal rows of a [T*7] (or [..., T*7]) gradient (pin=False: a copy)."""
    g = np.array(g, dtype=np.float64, copy=True)
    if not pin:
        return g
    v = g.reshape(g.shape[:-1] + (T, N_JOINTS))
    v[..., 0, :] = 0.0
    v[..., T - 1, :] = 0.0
    return g


@dataclass
class TrajState:
    x: np.ndarray                # [n] float32 values
    g: np.ndarray                # [n]
    d: np.ndarray                # [n]
    cost: float
    hist: List[Tuple[np.ndarray, np.ndarray, float]] = field(default_factory=list)  # oldest first


def two_loop(g: np.ndarray, hist) -> np.ndarray:
    """r = H g by the L-BFGS two-loop recursion (FP64)."""
    q = np.array(g, dtype=np.float64)
    alphas = []
    for s, y, rho in reversed(hist):
        a = rho * float(s @ q)
        q = q - a * y
        alphas.append(a)
    if hist:
        s, y, _ = hist[-1]
        gamma = float(s @ y) / float(y @ y)
    else:
        gamma = 1.0
    r = gamma * q
    for (s, y, rho), a in zip(hist, reversed(alphas)):
        beta = rho * float(y @ r)
        r = r + (a - beta) * s
    return r


def dense_inverse_hessian(hist, n: int) -> np.ndarray:
    """H from H0 = gamma I and the BFGS inverse updates applied oldest to newest."""
    if hist:
        s, y, _ = hist[-1]
        gamma = float(s @ y) / float(y @ y)
    else:
        gamma = 1.0
    H = gamma * np.eye(n)
    I = np.eye(n)
    for s, y, rho in hist:
        V = I - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


def steepest(g: np.ndarray, max_step: float = MAX_STEP) -> np.ndarray:
    """-g capped so that its largest component is at most max_step."""
    gmax = float(np.max(np.abs(g))) if g.size else 0.0
    scale = min(1.0, max_step / gmax) if gmax > 0.0 else 1.0
    return fp32(-g * scale)


def direction(st: TrajState, m: int, max_step: float = MAX_STEP) -> Tuple[np.ndarray, bool]:
    """(d, reset): the next search direction from the state's gradient and history."""
    if not st.hist:
        return steepest(st.g, max_step), False
    r = two_loop(st.g, st.hist)
    d = fp32(-r)
    if float(st.g @ d) >= 0.0:
        st.hist.clear()
        return steepest(st.g, max_step), True
    return d, False


def candidates(x: np.ndarray, d: np.ndarray, n_ls: int) -> np.ndarray:
    """[..., n_ls, n] candidate points fp32(x + alpha_i d)."""
    a = np.asarray(ALPHAS[:n_ls]).reshape((n_ls,) + (1,) * (x.ndim - 1) + (1,))
    return fp32(x[None] + a * d[None]).swapaxes(0, -2) if x.ndim > 1 else fp32(x[None] + a * d[None])


def init_state(x0: np.ndarray, cost0: float, g0: np.ndarray, T: int, max_step: float = MAX_STEP,
               pin: bool = True) -> TrajState:
    g = pin_rows(fp32(g0), T, pin)
    return TrajState(x=fp32(x0), g=g, d=steepest(g, max_step), cost=float(cost0))


def select(cost: float, gd: float, cand_cost: np.ndarray) -> int:
    """Index of the accepted candidate, or -1."""
    for i, ci in enumerate(cand_cost):
        if ci <= cost + ARMIJO_C1 * ALPHAS[i] * gd:
            return i
    i = int(np.argmin(cand_cost))
    return i if cand_cost[i] < cost else -1


def step(st: TrajState, cand_cost: np.ndarray, cand_grad: np.ndarray, T: int, m: int = 8,
         max_step: float = MAX_STEP, pin: bool = True) -> dict:
    """One iteration for one trajectory.  cand_grad [n_ls, n] are the joint gradients of the
    candidates (pinned rows are zeroed here).  Mutates st; returns what was decided."""
    n_ls = cand_cost.shape[0]
    gd = float(st.g @ st.d)
    i = select(st.cost, gd, cand_cost)
    info = {"accepted": i, "gd": gd, "curvature_ok": False, "reset": False}
    if i < 0:
        st.hist.clear()
        st.d = fp32(st.d * (ALPHAS[n_ls - 1] * 0.5))
        info["reset"] = True
        return info
    x_new = fp32(st.x + ALPHAS[i] * st.d)
    g_new = pin_rows(fp32(cand_grad[i]), T, pin)
    s = fp32(x_new - st.x)
    y = fp32(g_new - st.g)
    sy = float(s @ y)
    if sy > CURVATURE_EPS * np.sqrt(float(s @ s)) * np.sqrt(float(y @ y)):
        st.hist.append((s, y, 1.0 / sy))
        if len(st.hist) > m:
            st.hist.pop(0)
        info["curvature_ok"] = True
    st.x, st.g, st.cost = x_new, g_new, float(cand_cost[i])
    st.d, info["reset"] = direction(st, m, max_step)
    return info
