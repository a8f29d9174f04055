"""Discrete adjoint of a sequence of IRK steps (gradient of a tracking loss).

TEST INFRASTRUCTURE ONLY (oracle).

Not in the paper: the gradient of L = 1/2 (u^N - u_hat)^T M (u^N - u_hat) with respect
to the nodal forcing of every stage of every step, the viscosity nu and the initial
state, through N steps of the IRK scheme of Sec. 3.1 (stage solve J k^n = F(s^n, f^n),
update s^{n+1} = s^n + dt sum_j b_j k_j^n).  Reverse sweep, for n = N-1 .. 0:
    lam^n   = J^{-T} (dt b (x) gbar_{n+1})
    grad f^n_i = M_fa^T lam_i^u
    gbar_n  = gbar_{n+1} + (dF/ds)^T lam^n
            = gbar_{n+1} + [ -L^T sum_i lam_i^u - B sum_i lam_i^p ; -B^T sum_i lam_i^u ]
    dL/dnu += lam^nT (dF/dnu - dJ/dnu k^n),  K = nu K_1:
            = -sum_i lam_i^u . K_1 u^n - dt sum_ij a_ij lam_i^u . K_1 k_j^u.
The loss is a reading (the workload only says "L2 misfit").

Pinned by tests/test_oracle_adjoint.py: central finite differences of the forward map
(exact up to rounding for the forcing and the initial state, since u^N is affine in
them and L quadratic), second-order-accurate differences in nu.
"""
from __future__ import annotations

import numpy as np

from .stage import StageSystem


def forward(S: StageSystem, b, f_all, state0, solve):
    """f_all[n][i]: (nnodes, dim) nodal forcing of stage i of step n.  Returns the
    states s^0..s^N and stages k^0..k^{N-1}."""
    nvel = S.th.nvel
    states, ks = [np.array(state0, dtype=np.float64)], []
    k = np.zeros(S.n)
    for fn in f_all:
        s = states[-1]
        F = S.rhs(list(fn), s[:nvel], s[nvel:])
        k = solve(F, k)
        new = s.copy()
        for j in range(S.r):
            new += S.dt * b[j] * k[j * S.ns:(j + 1) * S.ns]
        states.append(new)
        ks.append(k)
    return states, ks


def loss(S: StageSystem, state, target_u):
    e = state[: S.th.nvel] - target_u
    return 0.5 * float(e @ (S.Mv @ e))


def gradient(S: StageSystem, b, f_all, state0, target_u, solve, solve_T):
    th = S.th
    nvel, nf, d = th.nvel, th.nfree, th.dim
    states, ks = forward(S, b, f_all, state0, solve)
    L = loss(S, states[-1], target_u)
    gbar = np.zeros(S.ns)
    gbar[:nvel] = S.Mv @ (states[-1][:nvel] - target_u)
    K1v = S.Kv / S.nu
    Lv = S.Lv
    gf = [[None] * S.r for _ in f_all]
    gnu = 0.0
    for n in range(len(f_all) - 1, -1, -1):
        G = np.concatenate([S.dt * b[i] * gbar for i in range(S.r)])
        lam = solve_T(G)
        lu = [lam[i * S.ns:i * S.ns + nvel] for i in range(S.r)]
        lp = [lam[i * S.ns + nvel:(i + 1) * S.ns] for i in range(S.r)]
        for i in range(S.r):
            gf[n][i] = np.stack([S.Ms_free_all.T @ lu[i][c * nf:(c + 1) * nf] for c in range(d)], axis=1)
        su, spr = sum(lu), sum(lp)
        gs = np.concatenate([-(Lv.T @ su) - S.B @ spr, -(S.B.T @ su)])
        u_n = states[n][:nvel]
        kk = ks[n]
        for i in range(S.r):
            gnu -= lu[i] @ (K1v @ u_n)
            for j in range(S.r):
                gnu -= S.dt * S.A[i, j] * (lu[i] @ (K1v @ kk[j * S.ns:j * S.ns + nvel]))
        gbar = gbar + gs
    return L, gf, gnu, gbar
