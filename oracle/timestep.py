"""IRK time stepping of the Stokes/Oseen DAE and reference solutions (Sec. 3.1, 5.1).

TEST INFRASTRUCTURE ONLY (oracle).

One step: build F from (u^n, p^n) and the forcing interpolated at t^n + c_i dt, solve
J k = F (initial guess: the previous step's stages, zero at the first step, as for the
Newton iteration of Sec. 3.2), then u^{n+1} = u^n + dt sum_j b_j k_j^u and likewise
for p.  Errors as in Sec. 5.1: relative L2 error of the velocity, absolute L2 error of
the pressure after shifting it to zero mean.

semidiscrete_exact() gives the exact solution of the spatially discrete DAE for a
forcing g(x) e^{alpha t}, by reduction to the discretely divergence-free subspace
Z = null(B^T) and a generalised eigendecomposition: a closed form that the RK stepper
must approach at the order of its tableau.  Pinned by tests/test_oracle_timestep.py.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .stage import StageSystem


def step(S: StageSystem, b: np.ndarray, c: np.ndarray, forcing, t: float, u: np.ndarray, p: np.ndarray,
         solve, k0: np.ndarray):
    """Advance (u, p) by one step of size S.dt; solve(F, k0) -> k."""
    fn = [S.th.interpolate(forcing, t + ci * S.dt) for ci in c]
    F = S.rhs(fn, u, p)
    k = solve(F, k0)
    u_new, p_new = u.copy(), p.copy()
    for j in range(S.r):
        ku, kp = S.split(k, j)
        u_new += S.dt * b[j] * ku
        p_new += S.dt * b[j] * kp
    return u_new, p_new, k


def dense_solver(S: StageSystem, transpose: bool = False):
    """Direct solve of J k = F (or J^T k = F) with one pinned pressure per stage,
    pressure means removed."""
    J = S.J.toarray()
    if transpose:
        J = J.T.copy()
    pins = [i * S.ns + S.th.nvel for i in range(S.r)]
    for q in pins:
        J[q, :] = 0.0
        J[:, q] = 0.0
        J[q, q] = 1.0
    lu = sla.lu_factor(J)

    def solve(F, k0=None):
        F = np.array(F, dtype=np.float64)
        F[pins] = 0.0
        return S.project_pressure_mean(sla.lu_solve(lu, F))

    return solve


def semidiscrete_exact(S: StageSystem, u0: np.ndarray, g_nodal: np.ndarray, alpha: float, T: float) -> np.ndarray:
    """Exact u(T) of M u' + L u + B p = e^{alpha t} M_fa g, B^T u = 0, u(0) = u0
    (u0 must satisfy B^T u0 = 0; L symmetric, i.e. no wind)."""
    th = S.th
    Z = sla.null_space(S.B.T.toarray())
    Mz = Z.T @ (S.Mv @ Z)
    Lz = Z.T @ (S.Lv @ Z)
    G = np.concatenate([S.Ms_free_all @ g_nodal[:, c] for c in range(th.dim)])
    lam, V = sla.eigh(Lz, Mz)  # V^T Mz V = I
    y0 = np.linalg.solve(Mz, Z.T @ (S.Mv @ u0))
    eta0 = V.T @ (Mz @ y0)
    gz = V.T @ (Z.T @ G)
    eta = np.exp(-lam * T) * eta0 + gz * (np.exp(alpha * T) - np.exp(-lam * T)) / (alpha + lam)
    return Z @ (V @ eta)


def velocity_error(S: StageSystem, u: np.ndarray, exact, t: float) -> float:
    """Relative L2 error of the free-velocity vector u against a callable."""
    th = S.th
    nodal = np.zeros((th.nnodes, th.dim))
    for c in range(th.dim):
        nodal[th.free, c] = u[c * th.nfree:(c + 1) * th.nfree]
    err = th.l2_norm_p2(nodal, exact, t)
    ref = th.l2_norm_p2(np.zeros_like(nodal), lambda x, tt: -exact(x, tt), t)
    return err / ref


def pressure_error(S: StageSystem, p: np.ndarray) -> float:
    """Absolute L2 norm of p (exact pressure zero) after the zero-mean shift."""
    th = S.th
    shift = th.p1_integral(p) / th.volume()
    return th.l2_norm_p1(p - shift)
