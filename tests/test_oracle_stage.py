"""Pins for oracle/stage.py: the stage equations of Sec. 3.1 written stage by stage."""
import numpy as np
import pytest
import scipy.sparse as sp

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
