"""Pins for oracle/adjoint.py: the adjoint gradient against finite differences of the
oracle's own forward map (dense solves)."""
import numpy as np
import pytest

from oracle.adjoint import forward, gradient, loss
from oracle.fem import TaylorHood
from oracle.stage import StageSystem
from oracle.tableau import tableau
from oracle.timestep import dense_solver
from paper_2202_07381_amd import workloads as wl


def _problem(dim, nu, wind=False):
    xyz, cells = wl.square_mesh(4) if dim == 2 else wl.cube_mesh(2)
    th = TaylorHood(xyz, cells)
    A, b, c = tableau("radauIIA", 2)
    wn = th.interpolate(wl.wind_2d(3, 4)) if wind else None
    S = StageSystem(th, A, 0.05, nu, wn)
    rng = np.random.default_rng(21)
    f_all = [[rng.standard_normal((th.nnodes, dim)) for _ in range(2)] for _ in range(3)]
    s0 = np.zeros(S.ns)
    target = rng.standard_normal(th.nvel)
    return S, b, f_all, s0, target


def _L(S, b, f_all, s0, target):
    states, _ = forward(S, b, f_all, s0, dense_solver(S))
    return loss(S, states[-1], target)


@pytest.mark.parametrize("dim,wind", [(2, False), (2, True), (3, False)])
def test_forcing_and_state_gradient_matches_fd(dim, wind):
    S, b, f_all, s0, target = _problem(dim, 0.7, wind)
    L, gf, gnu, g0 = gradient(S, b, f_all, s0, target, dense_solver(S), dense_solver(S, transpose=True))
    rng = np.random.default_rng(22)
    dirs = [[rng.standard_normal(f.shape) for f in fn] for fn in f_all]
    h = 1e-3  # central differences are exact for a quadratic up to rounding
    fp = [[f + h * v for f, v in zip(fn, dn)] for fn, dn in zip(f_all, dirs)]
    fm = [[f - h * v for f, v in zip(fn, dn)] for fn, dn in zip(f_all, dirs)]
    fd = (_L(S, b, fp, s0, target) - _L(S, b, fm, s0, target)) / (2 * h)
    ad = sum(float(np.sum(g * v)) for gn, dn in zip(gf, dirs) for g, v in zip(gn, dn))
    assert abs(fd - ad) <= 1e-8 * abs(ad)
    v0 = rng.standard_normal(S.ns)
    v0[S.th.nvel:] = 0.0
    fd0 = (_L(S, b, f_all, s0 + h * v0, target) - _L(S, b, f_all, s0 - h * v0, target)) / (2 * h)
    assert abs(fd0 - g0 @ v0) <= 1e-8 * abs(fd0)


def test_viscosity_gradient_matches_fd():
    S, b, f_all, s0, target = _problem(2, 0.7)
    _, _, gnu, _ = gradient(S, b, f_all, s0, target, dense_solver(S), dense_solver(S, transpose=True))
    h = 1e-4
    A = S.A
    Sp = StageSystem(S.th, A, S.dt, 0.7 + h)
    Sm = StageSystem(S.th, A, S.dt, 0.7 - h)
    fd = (_L(Sp, b, f_all, s0, target) - _L(Sm, b, f_all, s0, target)) / (2 * h)
    assert abs(fd - gnu) <= 1e-6 * abs(gnu)
