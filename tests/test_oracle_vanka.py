"""Pins for oracle/vanka.py: Fig. 1 patch shape, patch-size statistics, exactness."""
import numpy as np
import pytest

from oracle.fem import TaylorHood
from oracle.stage import StageSystem
from oracle.tableau import tableau
from oracle.vanka import VankaSmoother, multiplicity, patch_dofs
from paper_2202_07381_amd import workloads as wl


def test_interior_patch_is_fig1():
    # Fig. 1: 19 velocity nodes (x2 components) and one pressure node per stage
    xyz, cells = wl.square_mesh(8)
    th = TaylorHood(xyz, cells)
    v = 4 * 9 + 4
    pat = patch_dofs(th, 1)[v]
    assert pat.size == 39
    assert (pat >= th.nvel).sum() == 1 and pat[-1] == th.nvel + v
    # the 19 nodes: a 3x3 block of the doubled lattice around v plus 10 more (Fig. 1)
    nodes = th.free[pat[pat < th.nfree]]
    lat = np.rint(th.node_xyz[nodes] * 16).astype(int) - 8
    expect = {(x, y) for x in (-1, 0, 1) for y in (-1, 0, 1)}
    expect |= {(0, -2), (0, 2), (-2, 0), (2, 0), (2, -2), (1, -2), (2, -1), (-2, 1), (-2, 2), (-1, 2)}
    assert set(map(tuple, lat)) == expect


@pytest.mark.parametrize("n,sum_n,sum_n2", [(16, 9327, 330081), (32, 38607, 1436289)])
def test_patch_statistics(n, sum_n, sum_n2):
    # sums of per-stage patch sizes by independent topology counting
    xyz, cells = wl.square_mesh(n)
    th = TaylorHood(xyz, cells)
    sizes = np.array([p.size for p in patch_dofs(th, 1)])
    assert sizes.sum() == sum_n and (sizes**2).sum() == sum_n2
    assert set(sizes) == {3, 9, 11, 15, 27, 29, 33, 39}


def test_interior_patch_3d():
    xyz, cells = wl.cube_mesh(4)
    th = TaylorHood(xyz, cells)
    v = (2 * 5 + 2) * 5 + 2
    assert patch_dofs(th, 1)[v].size == 196  # 65 nodes x 3 + 1


@pytest.mark.parametrize("r", [1, 2, 3])
def test_cover_and_multiplicity(r):
    xyz, cells = wl.square_mesh(6)
    th = TaylorHood(xyz, cells)
    pats = patch_dofs(th, r)
    D = multiplicity(pats, r * th.nstage)
    assert D.min() >= 1
    assert D.max() == 7
    for i in range(r):
        assert np.all(D[i * th.nstage + th.nvel:(i + 1) * th.nstage] == 1)
    assert all(p.size == r * (pats[0].size // r) for p in pats[:1])


def test_single_patch_exactness():
    xyz, cells = wl.square_mesh(6)
    th = TaylorHood(xyz, cells)
    A, b, c = tableau("radauIIA", 3)
    S = StageSystem(th, A, 0.05, 1.0)
    pats = patch_dofs(th, 3)
    sm = VankaSmoother(S.J, pats, 1.0, weighted=False)
    rng = np.random.default_rng(3)
    for v in (0, 17, 24):
        e = np.zeros(S.n)
        e[pats[v]] = rng.standard_normal(pats[v].size)
        Je = S.J @ e
        inv = [g for g in sm.groups if g[0].shape[1] == pats[v].size][0]
        row = [i for i in range(inv[0].shape[0]) if np.array_equal(inv[0][i], pats[v])][0]
        back = np.zeros(S.n)
        back[pats[v]] = inv[1][row] @ Je[pats[v]]
        # a computed inverse applied to A e returns e to within a small multiple of
        # cond(A_v) * eps (forward error of an inverse-based solve)
        cond = np.linalg.cond(S.J[pats[v]][:, pats[v]].toarray())
        assert np.abs(back - e).max() < 16 * cond * np.finfo(float).eps * np.abs(e).max()


# ------------------------------------------------------------ Chebyshev relaxation
def _cheb_T(m, x):
    """Chebyshev polynomial of the first kind in closed form."""
    x = np.asarray(x, dtype=float)
    inside = np.abs(x) <= 1
    out = np.empty_like(x)
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** m * np.cosh(m * np.arccosh(np.abs(xo)))
    return out


@pytest.mark.parametrize("steps", [1, 2, 3, 5])
def test_chebyshev_error_polynomial(steps):
    """On a diagonal S J the error after m steps is T_m((theta - s l)/delta) / T_m(theta/delta)
    times the initial error, for eigenvalues inside and outside [lo, hi] (Sec. 5.1's
    relaxation, Chebyshev polynomials of the first kind)."""
    from oracle.vanka import chebyshev_iteration

    lo, hi = 2.0, 8.0
    lam = np.array([0.3, 1.0, 2.0, 3.7, 5.0, 6.5, 8.0, 9.5, 12.0])
    s = np.array([1.0, 0.5, 2.0, 1.0, 0.25, 1.5, 1.0, 0.5, 2.0])
    sl = s * lam
    e0 = np.random.default_rng(7).standard_normal(lam.size)
    xstar = np.random.default_rng(8).standard_normal(lam.size)
    F = lam * xstar
    k = chebyshev_iteration(lambda x: lam * x, lambda r: s * r, F, xstar - e0, steps, lo, hi)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    expect = _cheb_T(steps, (theta - sl) / delta) / _cheb_T(steps, np.array([theta / delta]))[0]
    assert np.allclose((xstar - k) / e0, expect, rtol=1e-12, atol=1e-13)


# ------------------------------------------------------------ GMRES relaxation
def _vanka_case():
    xyz, cells = wl.square_mesh(4)
    th = TaylorHood(xyz, cells)
    A, b, c = tableau("radauIIA", 2)
    S = StageSystem(th, A, 0.05, 1.0)
    sm = VankaSmoother(S.J, patch_dofs(th, 2), 1.0, weighted=True)
    rng = np.random.default_rng(41)
    return S, sm, rng.standard_normal(S.n), rng.standard_normal(S.n)


def test_gmres_relaxation_one_step_is_minimal_residual():
    """m = 1: with z = S r_0 and q = S J z, the step minimising ||S (F - J (k + a z))|| has
    a = <q, z> / <q, q> (the one-dimensional least-squares problem in closed form)."""
    S, sm, F, k0 = _vanka_case()
    for tr in (False, True):
        J = S.J.T if tr else S.J
        z = sm.apply_S(F - J @ k0, tr)
        q = sm.apply_S(J @ z, tr)
        expect = k0 + (q @ z) / (q @ q) * z
        got = sm.gmres(F, k0, J, 1, tr)
        assert np.linalg.norm(got - expect) <= 1e-12 * np.linalg.norm(expect)


def test_gmres_relaxation_matches_krylov_least_squares():
    """m = 3 against a least-squares solve over the power basis z, Mz, M^2 z (M = S J) of
    the Krylov space: the GMRES iterate is k + K c with c minimising ||z - M K c||; and
    the preconditioned residual norm does not grow with m."""
    S, sm, F, k0 = _vanka_case()
    J = S.J
    M = lambda x: sm.apply_S(J @ x)
    z = sm.apply_S(F - J @ k0)
    K = np.stack([z, M(z), M(M(z))], axis=1)
    MK = np.stack([M(K[:, i]) for i in range(3)], axis=1)
    c = np.linalg.lstsq(MK, z, rcond=None)[0]
    expect = k0 + K @ c
    got = sm.gmres(F, k0, J, 3)
    assert np.linalg.norm(got - expect) <= 1e-9 * np.linalg.norm(expect)
    norms = [np.linalg.norm(sm.apply_S(F - J @ sm.gmres(F, k0, J, m))) for m in range(0, 5)]
    assert all(norms[i + 1] <= norms[i] * (1 + 1e-12) for i in range(4))


def test_gmres_relaxation_full_dimension_is_exact():
    """With as many steps as unknowns GMRES solves S J k = S F exactly (nonsingular S), and
    an invariant Krylov space (S J = I) ends the cycle early with the exact solution."""
    from oracle.vanka import gmres_relaxation

    rng = np.random.default_rng(43)
    n = 7
    J = rng.standard_normal((n, n)) + 4 * np.eye(n)
    Sm = rng.standard_normal((n, n)) + 3 * np.eye(n)
    F, k0 = rng.standard_normal(n), rng.standard_normal(n)
    got = gmres_relaxation(lambda x: J @ x, lambda r: Sm @ r, F, k0, n)
    assert np.allclose(got, np.linalg.solve(J, F), rtol=1e-9, atol=1e-10)
    Jinv = np.linalg.inv(J)
    got = gmres_relaxation(lambda x: J @ x, lambda r: Jinv @ r, F, k0, 3)
    assert np.allclose(got, np.linalg.solve(J, F), rtol=1e-12, atol=1e-12)
    assert np.array_equal(gmres_relaxation(lambda x: J @ x, lambda r: Sm @ r, J @ k0, k0, 3), k0)


# ------------------------------------------------- spectrum estimate (Chebyshev interval)
def test_ritz_values_match_projected_operator():
    """Ritz values from m Arnoldi steps on M = S J equal the eigenvalues of Q^T M Q for an
    orthonormal basis Q of span{v0, M v0, ..., M^{m-1} v0} (QR of the power basis, an
    independent construction); with m = dimension they are M's eigenvalues."""
    from oracle.vanka import arnoldi_ritz

    S, sm, _, v0 = _vanka_case()
    J = S.J
    M = lambda x: sm.apply_S(J @ x)
    m = 6
    K = [v0 / np.linalg.norm(v0)]
    for _ in range(m - 1):
        w = M(K[-1])
        K.append(w / np.linalg.norm(w))
    Q, _ = np.linalg.qr(np.stack(K, axis=1))
    proj = np.linalg.eigvals(Q.T @ np.stack([M(Q[:, i]) for i in range(m)], axis=1))
    H, ritz = arnoldi_ritz(lambda x: J @ x, sm.apply_S, v0, m)
    assert H.shape == (m + 1, m)
    proj = proj[np.argsort(-proj.real, kind="stable")]
    assert np.allclose(ritz, proj, rtol=1e-8, atol=1e-8)
    rng = np.random.default_rng(44)
    n = 8
    A = rng.standard_normal((n, n))
    _, ritz = arnoldi_ritz(lambda x: A @ x, lambda r: r, rng.standard_normal(n), n)
    ev = np.linalg.eigvals(A)
    assert np.allclose(np.sort_complex(ritz), np.sort_complex(ev), atol=1e-9)


def test_ritz_estimate_of_the_chebyshev_interval():
    """On the 8x8 Stokes mesh (the setting of Sec. 5.1's [2, 8]) 20 Arnoldi steps put the
    largest Ritz value of S J within 2% of the largest real eigenvalue part of the dense
    S J, which lies in (7, 8)."""
    from oracle.multigrid import Hierarchy
    from oracle.vanka import arnoldi_ritz

    A, b, c = tableau("radauIIA", 2)
    H = Hierarchy(wl.square_hierarchy(4, 2), A, 1.0 / 32, 1.0, weighted=False, smoother="chebyshev")
    J = H.systems[1].J
    sm = H.smoothers[1]
    dense = np.linalg.eigvals(np.column_stack([sm.apply_S(J.toarray()[:, i]) for i in range(J.shape[0])]))
    _, ritz = arnoldi_ritz(lambda x: J @ x, sm.apply_S, np.random.default_rng(45).standard_normal(J.shape[0]), 20)
    lam = dense.real.max()
    assert 7.0 < lam < 8.0
    assert abs(ritz[0].real - lam) < 0.02 * lam
