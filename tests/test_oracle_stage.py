"""Pins for oracle/stage.py: the stage equations of Sec. 3.1 written stage by stage."""
import numpy as np
import pytest

from oracle.fem import TaylorHood
from oracle.stage import StageSystem
from oracle.tableau import tableau
from paper_2202_07381_amd import workloads as wl


def _system(fam="radauIIA", r=3, wind=None, n=4, dt=0.1, nu=0.7):
    xyz, cells = wl.square_mesh(n)
    th = TaylorHood(xyz, cells)
    A, b, c = tableau(fam, r)
    wn = th.interpolate(wind) if wind is not None else None
    return StageSystem(th, A, dt, nu, wn), th


@pytest.mark.parametrize("fam,r", [("radauIIA", 3), ("gauss", 2)])
@pytest.mark.parametrize("windy", [False, True])
def test_kronecker_equals_stage_equations(fam, r, windy):
    S, th = _system(fam, r, wl.StreamWind(np.array([1.0]), np.array([2.0]), np.array([0.3]), 1.0) if windy else None)
    rng = np.random.default_rng(1)
    k = rng.standard_normal(S.n)
    # M k_i^u + dt sum_j a_ij (L k_j^u + B k_j^p)  and  dt sum_j a_ij B^T k_j^u, stage by stage
    L = S.Ks + (S.Cs if S.Cs is not None else 0)
    out = []
    for i in range(r):
        ku_i, _ = S.split(k, i)
        vel = np.concatenate([S.Ms @ ku_i[c * th.nfree:(c + 1) * th.nfree] for c in range(2)])
        pre = np.zeros(th.nverts)
        for j in range(r):
            ku, kp = S.split(k, j)
            Lk = np.concatenate([L @ ku[c * th.nfree:(c + 1) * th.nfree] for c in range(2)])
            vel += S.dt * S.A[i, j] * (Lk + S.B @ kp)
            pre += S.dt * S.A[i, j] * (S.B.T @ ku)
        out.append(np.concatenate([vel, pre]))
    ref = np.concatenate(out)
    assert np.abs(S.apply(k) - ref).max() <= 1e-14 * np.abs(ref).max()


def test_rhs_equals_stage_equations():
    S, th = _system()
    rng = np.random.default_rng(2)
    u, p = rng.standard_normal(th.nvel), rng.standard_normal(th.nverts)
    f = [rng.standard_normal((th.nnodes, 2)) for _ in range(S.r)]
    F = S.rhs(f, u, p)
    Mfull = th.scalar_mass_full()
    for i in range(S.r):
        Fu, Fp = S.split(F, i)
        Mf = np.concatenate([(Mfull @ f[i][:, c])[th.free] for c in range(2)])
        Ku = np.concatenate([S.Ks @ u[c * th.nfree:(c + 1) * th.nfree] for c in range(2)])
        assert np.allclose(Fu, Mf - Ku - S.B @ p, atol=1e-14)
        assert np.allclose(Fp, -S.B.T @ u, atol=1e-14)
        assert abs(Fp.sum()) < 1e-13  # consistent with the pressure null vectors


def test_nullspace():
    S, _ = _system()
    Z = S.nullspace()
    assert np.abs(S.J @ Z).max() < 1e-14
    assert np.abs(S.J.T @ Z).max() < 1e-14
    # and nothing else: rank deficiency is exactly r
    sv = np.linalg.svd(S.J.toarray(), compute_uv=False)
    assert (sv < 1e-12 * sv[0]).sum() == S.r


# ------------------------------------------------------------- boundary data
def _steady_fields():
    # divergence-free P2 velocity and P1 pressure: discretisation exact
    u0 = lambda x, t=0.0: np.stack([x[:, 1] ** 2, x[:, 0] ** 2], axis=1)
    p0 = lambda x: x[:, 0] + x[:, 1]
    return u0, p0


@pytest.mark.parametrize("mesh", ["square", "crossed"])
def test_dirichlet_steady_solution_gives_zero_rhs(mesh):
    """u = (y^2, x^2), p = x + y solve steady Stokes with f = -nu Lap u + grad p =
    (1 - 2 nu, 1 - 2 nu); both lie in P2 x P1, so with the boundary terms F vanishes."""
    from oracle.fem import TaylorHood
    from oracle.stage import StageSystem
    from oracle.tableau import tableau

    xyz, cells = wl.square_mesh(6) if mesh == "square" else wl.crossed_mesh(3)
    th = TaylorHood(xyz, cells)
    nu = 0.7
    A, b, c = tableau("radauIIA", 2)
    S = StageSystem(th, A, 0.1, nu)
    u0, p0 = _steady_fields()
    g = u0(th.node_xyz)
    f = np.full((th.nnodes, 2), 1.0 - 2.0 * nu)
    F = S.rhs([f, f], th.free_velocity(g), p0(th.xyz)) + S.rhs_dirichlet(g, [g, g])
    scale = np.abs(S.rhs([f, f], th.free_velocity(g), p0(th.xyz))).max()
    assert np.abs(F).max() < 1e-13 * max(scale, 1.0)
    # without the boundary terms the residual is O(1)
    assert np.abs(S.rhs([f, f], th.free_velocity(g), p0(th.xyz))).max() > 1e-3


@pytest.mark.parametrize("family,r", [("radauIIA", 2), ("radauIIA", 3), ("gauss", 2), ("lobattoIIIC", 3)])
def test_dirichlet_linear_in_time_stage_derivatives(family, r):
    """u = t u0, p = t p0 with f = u0 + t(-nu Lap u0 + grad p0): the exact stage
    derivatives (u0, p0) at every stage (A 1 = c) solve J k = F including the boundary
    terms, for every tableau."""
    from oracle.fem import TaylorHood
    from oracle.stage import StageSystem
    from oracle.tableau import tableau

    th = TaylorHood(*wl.square_mesh(5))
    nu, dt, tn = 0.4, 0.05, 0.3
    A, b, c = tableau(family, r)
    S = StageSystem(th, A, dt, nu)
    u0, p0 = _steady_fields()
    U0 = u0(th.node_xyz)
    fstage = [U0 + (tn + ci * dt) * (1.0 - 2.0 * nu) for ci in c]
    F = S.rhs(fstage, th.free_velocity(tn * U0), tn * p0(th.xyz))
    F = F + S.rhs_dirichlet(tn * U0, [(tn + ci * dt) * U0 for ci in c])
    k = np.concatenate([np.concatenate([th.free_velocity(U0), p0(th.xyz)])] * r)
    assert np.abs(S.J @ k - F).max() < 1e-12 * np.abs(F).max()
