"""Temporal-order pin: the IRK stepper against the exact semi-discrete solution."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.fem import TaylorHood
from oracle.stage import StageSystem
from oracle.tableau import tableau
from oracle.timestep import dense_solver, semidiscrete_exact, step
from paper_2202_07381_amd import workloads as wl

# classical order of each family (Sec. 5): 2r-1, 2r, 2r-2
ORDERS = {("radauIIA", 2): 3, ("radauIIA", 3): 5, ("gauss", 2): 4, ("lobattoIIIC", 2): 2, ("lobattoIIIC", 3): 4}


def g(x, t):
    return np.stack([np.sin(np.pi * x[:, 0]) * x[:, 1], np.cos(x[:, 1]) * x[:, 0]], 1) * np.exp(t)


@pytest.mark.parametrize("key", sorted(ORDERS))
def test_temporal_order(key):
    xyz, cells = wl.square_mesh(4)
    th = TaylorHood(xyz, cells)
    A, b, c = tableau(*key)
    errs = []
    for N in (8, 16, 32):
        S = StageSystem(th, A, 1.0 / N, 0.02)
        Z = sla.null_space(S.B.T.toarray())
        u0 = Z @ np.random.default_rng(0).standard_normal(Z.shape[1])
        solve = dense_solver(S)
        u, p, k = u0.copy(), np.zeros(th.nverts), np.zeros(S.n)
        for n in range(N):
            u, p, k = step(S, b, c, g, n / N, u, p, solve, k)
        errs.append(np.linalg.norm(u - semidiscrete_exact(S, u0, th.interpolate(g, 0.0), 1.0, 1.0)))
    rate = np.log2(errs[-2] / errs[-1])
    assert abs(rate - ORDERS[key]) < 0.2, (errs, rate)
