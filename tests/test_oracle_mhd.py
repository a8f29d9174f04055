"""Pins of the linearised MHD stage system and its multigrid (oracle/mhd.py; Sec. 3.3,
4.1, 4.2, Fig. 1 right)."""
import numpy as np
import pytest

from oracle.fem import TaylorHood
from oracle.fgmres import fgmres
from oracle.mhd import MHDHierarchy, MHDSpace, coarsen_b0, island_state, nedelec_prolongation
from oracle.tableau import tableau
from oracle.transfer import interpolation_matrices
from paper_2202_07381_amd import workloads as wl


def _spaces(nc=2, nl=2):
    lv = wl.square_hierarchy(nc, nl)
    return lv, [MHDSpace(TaylorHood(m.xyz, m.cells)) for m in lv]


def _field(x):
    return np.stack([np.sin(2 * x[:, 1]) + x[:, 0] ** 2, np.cos(x[:, 0] + 0.3 * x[:, 1])], axis=1)


def test_nedelec_tangential_moments():
    """The edge functional (line integral along the edge from its lower to its higher
    vertex) of every basis function on every cell is the identity."""
    _, (s,) = _spaces(2, 1)
    th = s.th
    g, wg = np.polynomial.legendre.leggauss(3)
    lo, hi = s._edge_ends()
    mom = np.zeros((th.ncells, 3, 3))  # [cell, edge functional, basis]
    for t, wt in zip(0.5 * (g + 1), 0.5 * wg):
        for e in range(3):
            lam = np.zeros((th.ncells, 3))
            c = np.arange(th.ncells)
            lam[c, lo[:, e]] = 1 - t
            lam[c, hi[:, e]] = t
            for cc in range(th.ncells):
                val, _ = s.nedelec_at(lam[cc][None, :])
                tang = th.xyz[th.cells[cc, hi[cc, e]]] - th.xyz[th.cells[cc, lo[cc, e]]]
                mom[cc, e] += wt * val[cc, 0] @ tang
    assert np.abs(mom - np.eye(3)[None]).max() < 1e-13


def test_curl_of_gradient_and_multiplier_coupling():
    """grad P1 lies in the Nedelec space with degrees of freedom G s (s_hi - s_lo): its
    curl vanishes on every cell, and the multiplier block -(grad s, c) equals -M_B G."""
    _, (s,) = _spaces(4, 1)
    G = s.discrete_gradient()
    sv = np.random.default_rng(1).standard_normal(s.th.nverts)
    _, curl = s.nedelec_at(np.array([[1 / 3, 1 / 3, 1 / 3]]))
    gdofs = (G @ sv)[s.cell_edges]
    assert np.abs(np.einsum("ce,ce->c", curl, gdofs)).max() < 1e-12 * np.abs(gdofs).max() * s.th.ncells
    w0, b0 = island_state(s)
    M, S = s.operators(100.0, 100.0, w0, b0)
    blk = S[s.off_B:s.off_p, s.off_g:]
    ref = -(s.edge_mass_all() @ G)[s.efree][:, s.vint]
    assert abs(blk - ref).max() < 1e-13 * abs(ref).max()
    assert abs(S[s.off_g:, s.off_B:s.off_p] - ref.T).max() < 1e-13 * abs(ref).max()


def test_nedelec_prolongation_commutes_and_reproduces_constants():
    """P_B G_c = G_f P_1 on continuous P1 fields vanishing on the boundary, and the
    full Nedelec interpolation maps the degrees of freedom of a constant field to its
    fine ones."""
    lv, (c, f) = _spaces(2, 2)
    Pu, Pp = interpolation_matrices(c.th, f.th)
    PB = nedelec_prolongation(c, f)
    Gc = c.discrete_gradient()[c.efree][:, c.vint]
    Gf = f.discrete_gradient()[f.efree][:, f.vint]
    Pg = Pp[f.vint][:, c.vint]
    assert abs(PB @ Gc - Gf @ Pg).max() < 1e-13
    const = np.array([0.7, -1.3])
    dofs = lambda s_: (s_.th.xyz[s_.th.edges[:, 1]] - s_.th.xyz[s_.th.edges[:, 0]]) @ const  # noqa: E731
    Pall = nedelec_prolongation(c, f, free_only=False)
    assert np.abs(Pall @ dofs(c) - dofs(f)).max() < 1e-14


def test_coarse_state_is_the_coarse_interpolant():
    lv, (c, f) = _spaces(2, 2)
    got = coarsen_b0(f, c, f.edge_dofs(_field))
    assert np.abs(got - c.edge_dofs(_field)).max() < 1e-12


def test_lorentz_induction_coupling_is_skew_for_constant_field():
    """With a constant B0 (so curl B0 = 0) and w = 0 the velocity-field couplings are
    adjoint up to sign: S_uB = -S_Bu^T."""
    _, (s,) = _spaces(4, 1)
    b0 = (s.th.xyz[s.th.edges[:, 1]] - s.th.xyz[s.th.edges[:, 0]]) @ np.array([0.4, 1.1])
    M, S = s.operators(10.0, 10.0, np.zeros((s.th.nnodes, 2)), b0)
    uB = S[: s.off_B, s.off_B:s.off_p]
    Bu = S[s.off_B:s.off_p, : s.off_B]
    assert abs(uB).max() > 1e-3
    assert abs(uB + Bu.T).max() < 1e-14 * abs(uB).max() * 100


def test_interior_patch_is_figure_one_right():
    """Interior vertex of the diagonal-split mesh: 6 cells, 7 vertices, 12 edges, so 19
    P2 velocity nodes (2 components), 12 Nedelec edges, one pressure and one multiplier:
    52 unknowns per stage."""
    _, (s,) = _spaces(4, 1)
    pats = s.patches(2)
    n = 4
    v = 2 * (n + 1) + 2
    assert pats[v].size == 2 * 52
    assert max(p.size for p in pats) == 2 * 52


@pytest.mark.parametrize("Re", [1.0, 100.0])
def test_fgmres_vcycle_reaches_direct_solve(Re):
    A, _, _ = tableau("lobattoIIIC", 2)
    lv = wl.square_hierarchy(2, 3)
    sf = MHDSpace(TaylorHood(lv[-1].xyz, lv[-1].cells))
    w0, b0 = island_state(sf)
    H = MHDHierarchy(lv, A, 0.025, Re, Re, w0, b0)
    S = H.systems[-1]
    F = S.J @ np.random.default_rng(2).standard_normal(S.n)
    x, info = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-12, 200, 30, project=S.project_pressure_mean)
    assert info.converged and info.iterations <= 30
    J = S.J.toarray()
    pins = [i * sf.ns + sf.off_p for i in range(2)]
    for q in pins:
        J[q, :] = 0.0
        J[:, q] = 0.0
        J[q, q] = 1.0
    rhs = F.copy()
    rhs[pins] = 0.0
    xd = S.project_pressure_mean(np.linalg.solve(J, rhs))
    # FGMRES stops on the residual (1e-12): the solutions agree to that times cond(J)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.cond(J) * np.linalg.norm(xd)


def test_mhd_vcycle_equals_textbook_propagator():
    from test_oracle_vcycle_propagator import TOL, _check, _Propagator

    A, _, _ = tableau("lobattoIIIC", 2)
    lv = wl.square_hierarchy(2, 2)
    sf = MHDSpace(TaylorHood(lv[-1].xyz, lv[-1].cells))
    w0, b0 = island_state(sf)
    H = MHDHierarchy(lv, A, 0.025, 50.0, 50.0, w0 + 0.3, b0)
    _check(H, _Propagator(H, 0.5, True), 16, 21, TOL)


def test_single_patch_exactness():
    """One patch solve of the stage-coupled system recovers any vector supported on the
    patch (Sec. 4.2): R_v^T A_v^{-1} R_v J e = e, for an interior, an edge and a corner
    vertex of the linearised MHD operator."""
    A, _, _ = tableau("lobattoIIIC", 2)
    lv = wl.square_hierarchy(2, 2)
    sf = MHDSpace(TaylorHood(lv[-1].xyz, lv[-1].cells))
    w0, b0 = island_state(sf)
    H = MHDHierarchy(lv, A, 0.025, 50.0, 20.0, w0 + 0.3, b0)
    J = H.ops[-1]
    pats = sf.patches(2)
    rng = np.random.default_rng(4)
    n = 4
    for v in (2 * (n + 1) + 2, 2, 0):
        idx = pats[v]
        e = np.zeros(J.shape[0])
        e[idx] = rng.standard_normal(idx.size)
        Av = J[idx][:, idx].toarray()
        got = np.zeros_like(e)
        got[idx] = np.linalg.solve(Av, (J @ e)[idx])
        assert np.abs(got - e).max() <= 16 * np.linalg.cond(Av) * np.finfo(float).eps * np.abs(e).max()
