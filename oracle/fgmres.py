"""Flexible GMRES with right preconditioning (Sec. 4).

TEST INFRASTRUCTURE ONLY (oracle).

The paper uses FGMRES as the outer Krylov method because its preconditioner (a
multigrid cycle, possibly with inner Krylov relaxation) is costly and may vary.
Readings where the paper is silent: restart length m (default 30), modified
Gram--Schmidt, Givens rotations on the Hessenberg matrix, stop when the
unpreconditioned 2-norm residual estimate falls to rtol times the initial residual
norm ||F - J k0||, and the final solution has each stage's pressure mean removed.

Pinned by tests/test_oracle_multigrid.py: the converged solution equals a dense
direct solve; the residual recomputed from scratch equals the Arnoldi estimate.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SolveInfo:
    iterations: int = 0
    converged: bool = False
    rel_residual: float = np.inf
    history: list = field(default_factory=list)


def fgmres(apply_J, apply_prec, F, x0, rtol=1e-8, maxit=1000, restart=30, project=None):
    x = np.array(x0, dtype=np.float64, copy=True)
    info = SolveInfo()
    r = F - apply_J(x)
    beta0 = np.linalg.norm(r)
    info.history.append(beta0)
    if beta0 == 0.0:
        info.converged, info.rel_residual = True, 0.0
        return (project(x) if project else x), info
    its = 0
    while its < maxit:
        r = F - apply_J(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * beta0:
            info.converged = True
            break
        m = restart
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        j_end = 0
        for j in range(m):
            z = apply_prec(V[j])
            Z.append(z)
            w = apply_J(z)
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_end = j + 1
            info.history.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= rtol * beta0 or its >= maxit:
                break
        y = np.zeros(j_end)
        for i in range(j_end - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_end] @ y[i + 1:j_end]) / H[i, i]
        for i in range(j_end):
            x = x + y[i] * Z[i]
        if abs(g[j_end]) <= rtol * beta0:
            info.converged = True
            break
    info.iterations = its
    if project is not None:
        x = project(x)
    info.rel_residual = float(np.linalg.norm(F - apply_J(x)) / beta0)
    return x, info
