"""Pins for oracle/multigrid.py and oracle/fgmres.py."""
import numpy as np
import pytest

from oracle.fgmres import fgmres
from oracle.multigrid import Hierarchy
from oracle.tableau import tableau
from oracle.timestep import dense_solver
from paper_2202_07381_amd import workloads as wl


def _setup(n_coarse=4, nlev=3, fam="radauIIA", r=2, dt=1 / 16, nu=1.0, wind=None, dtype=np.float64, weighted=True):
    A, b, c = tableau(fam, r)
    H = Hierarchy(wl.square_hierarchy(n_coarse, nlev), A, dt, nu, wind=wind, dtype=dtype, weighted=weighted)
    S = H.finest
    f = wl.forcing_2d(1)
    F = S.rhs([S.th.interpolate(f)] * r, np.zeros(S.th.nvel), np.zeros(S.th.nverts))
    return H, S, F


def test_coarse_solve_exact():
    H, S, F = _setup(nlev=1)
    x = H.coarse_solve(F)
    assert np.linalg.norm(F - S.J @ x) < 1e-13 * np.linalg.norm(F)


def test_fgmres_mg_matches_direct_solve():
    H, S, F = _setup(n_coarse=4, nlev=2)
    x, info = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-13, 200, 30, project=S.project_pressure_mean)
    xd = dense_solver(S)(F)
    assert info.converged
    assert np.linalg.norm(x - xd) < 1e-10 * np.linalg.norm(xd)


def test_arnoldi_estimate_equals_true_residual():
    H, S, F = _setup()
    for maxit in (3, 7):
        x, info = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-14, maxit, 30)
        true = np.linalg.norm(F - S.J @ x)
        assert abs(true - info.history[-1]) < 1e-12 * info.history[0]


def test_weighting_reading():
    # the literal (unweighted) omega=0.5 sweep is not a useful preconditioner here;
    # the partition-of-unity weighted one converges fast (reading of the damping).
    Hw, S, F = _setup()
    _, iw = fgmres(S.apply, Hw.vcycle, F, np.zeros_like(F), 1e-8, 60, 30)
    Hu, S2, F2 = _setup(weighted=False)
    _, iu = fgmres(S2.apply, Hu.vcycle, F2, np.zeros_like(F2), 1e-8, 60, 30)
    assert iw.converged and iw.iterations <= 15
    assert not iu.converged


@pytest.mark.slow
def test_mesh_independent_iterations():
    its = []
    for nlev in (3, 4, 5):  # 16^2, 32^2, 64^2 with a 4x4 coarsest mesh
        H, S, F = _setup(nlev=nlev)
        _, info = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 100, 30)
        assert info.converged
        its.append(info.iterations)
    assert max(its) / min(its) <= 1.5, its


def test_vcycle_transpose_dot_product():
    H, S, F = _setup(fam="gauss", r=2, wind=wl.wind_2d(3, 16), nu=0.05)
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(S.n), rng.standard_normal(S.n)
    lhs = H.vcycle(x) @ y
    rhs = x @ H.vcycle_transpose(y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_oseen_converges():
    H, S, F = _setup(fam="gauss", r=2, nu=0.01, dt=5e-3, wind=wl.wind_2d(3, 16))
    assert S.Cs is not None
    _, info = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 100, 30)
    assert info.converged


def test_mixed_precision_reaches_fp64_tolerance():
    H, S, F = _setup(dtype=np.float32)
    x, info = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 100, 30, project=S.project_pressure_mean)
    assert info.converged and info.rel_residual <= 1e-8
    H64, _, _ = _setup()
    x64, _ = fgmres(S.apply, H64.vcycle, F, np.zeros_like(F), 1e-8, 100, 30, project=S.project_pressure_mean)
    assert np.linalg.norm(x - x64) / np.linalg.norm(x64) < 1e-6


# ------------------------------------------------------------ Chebyshev relaxation
def test_chebyshev_interval_reading():
    """The paper's interval [2, 8] follows its own [lambda/4, lambda] rule with lambda the
    largest eigenvalue of S J, S the undamped additive operator (Sec. 5.1): on the 8x8
    mesh the spectrum's largest real part is just below 8 and the smallest is the
    pressure null space's 0."""
    A, b, c = tableau("radauIIA", 2)
    H = Hierarchy(wl.square_hierarchy(4, 2), A, 1.0 / 32, 1.0, weighted=False, smoother="chebyshev")
    J = H.systems[1].J.toarray()
    SJ = np.column_stack([H.smoothers[1].apply_S(J[:, i]) for i in range(J.shape[0])])
    ev = np.linalg.eigvals(SJ)
    assert 7.0 < ev.real.max() < 8.0
    assert abs(ev.real.min()) < 1e-10


@pytest.mark.slow
def test_chebyshev_mg_mesh_independent():
    """FGMRES with the Chebyshev-relaxed V-cycle ([2, 8], 2/2 steps, unweighted operator)
    converges in a mesh-independent number of iterations (Sec. 5.1)."""
    its = []
    for nl in (3, 4):
        A, b, c = tableau("radauIIA", 3)
        lv = wl.square_hierarchy(4, nl)
        H = Hierarchy(lv, A, 0.5 / (4 * 2 ** (nl - 1)), 1.0, weighted=False, smoother="chebyshev")
        S = H.finest
        f = wl.forcing_2d(1)
        F = S.rhs([S.th.interpolate(f, 0.0)] * S.r, np.zeros(S.th.nvel), np.zeros(S.th.nverts))
        x, info = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 100, 30, project=S.project_pressure_mean)
        assert info.converged
        assert np.linalg.norm(F - S.apply(x)) <= 1e-8 * np.linalg.norm(F) * 1.0001
        its.append(info.iterations)
    assert max(its) <= 14 and abs(its[0] - its[1]) <= 2


def test_chebyshev_vcycle_transpose_dot_product():
    """The transposed Chebyshev-relaxed V-cycle is the transpose of the V-cycle as a
    linear map (the adjoint's relaxation is Chebyshev with J^T and S^T)."""
    A, b, c = tableau("gauss", 2)
    H = Hierarchy(wl.square_hierarchy(4, 3), A, 5e-3, 0.05, wind=wl.wind_2d(3, 16), weighted=False,
                  smoother="chebyshev")
    S = H.finest
    rng = np.random.default_rng(6)
    x, y = rng.standard_normal(S.n), rng.standard_normal(S.n)
    lhs = H.vcycle(x) @ y
    rhs = x @ H.vcycle_transpose(y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("wind", [False, True])
def test_gmres_relaxed_fgmres_matches_direct_solve(wind):
    """FGMRES with the GMRES-relaxed V-cycle (a nonlinear preconditioner, so the outer
    iteration must be flexible; Sec. 4.1, 4.2) reaches the dense direct solution for
    Stokes and for an Oseen operator within 15 iterations."""
    A, b, c = tableau("gauss", 2)
    kw = dict(wind=wl.wind_2d(3, 16)) if wind else {}
    H = Hierarchy(wl.square_hierarchy(4, 3), A, 5e-3, 0.05 if wind else 1.0, smoother="gmres", **kw)
    S = H.finest
    f = wl.forcing_2d(1)
    F = S.rhs([S.th.interpolate(f, 0.0)] * S.r, np.zeros(S.th.nvel), np.zeros(S.th.nverts))
    x, info = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-10, 100, 30, project=S.project_pressure_mean)
    assert info.converged and info.iterations <= 15
    xd = S.project_pressure_mean(np.linalg.lstsq(S.J.toarray(), F, rcond=None)[0])
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
