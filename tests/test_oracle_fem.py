"""Pins for oracle/fem.py: textbook element matrices, closed-form integrals, counts."""
import numpy as np
import pytest

from oracle.fem import TaylorHood
from paper_2202_07381_amd import workloads as wl


def test_p2_triangle_mass_matches_textbook():
    # |T|/180 * [[6,-1,-1,0,-4,0],...] in the order v0,v1,v2,e01,e02,e12:
    # a vertex couples -4 to the opposite edge and 0 to its adjacent edges.
    xyz = np.array([[0.1, 0.2], [1.3, 0.4], [0.5, 1.7]])
    th = TaylorHood(xyz, np.array([[0, 1, 2]]))
    area = 0.5 * abs(np.linalg.det(np.array([xyz[1] - xyz[0], xyz[2] - xyz[0]])))
    ref = np.array([
        [6, -1, -1, 0, 0, -4],
        [-1, 6, -1, 0, -4, 0],
        [-1, -1, 6, -4, 0, 0],
        [0, 0, -4, 32, 16, 16],
        [0, -4, 0, 16, 32, 16],
        [-4, 0, 0, 16, 16, 32],
    ]) * area / 180.0
    assert np.allclose(th.element_mass()[0], ref, rtol=0, atol=1e-15)


def test_p2_triangle_stiffness_reference_element():
    # reference-triangle P2 stiffness, vertex diagonal entries: 1 (right angle), 1/2, 1/2
    th = TaylorHood(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 1, 2]]))
    K = th.element_stiffness()[0]
    assert np.allclose(np.diag(K)[:3], [1.0, 0.5, 0.5], atol=1e-14)
    assert np.allclose(np.diag(K)[3:], [8 / 3, 8 / 3, 8 / 3], atol=1e-14)
    assert np.allclose(K.sum(axis=1), 0, atol=1e-14)


@pytest.mark.parametrize("n,counts", [(4, (25, 81, 187, 123)), (16, (289, 1089, 2467, 2211))])
def test_counts_2d(n, counts):
    xyz, cells = wl.square_mesh(n)
    th = TaylorHood(xyz, cells)
    assert (th.nverts, th.nnodes, 2 * th.nnodes + th.nverts, th.nstage) == counts


def test_counts_3d():
    xyz, cells = wl.cube_mesh(4)
    th = TaylorHood(xyz, cells)
    assert (th.nverts, th.nnodes, 3 * th.nnodes + th.nverts, th.nstage) == (125, 729, 2312, 1154)


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_sum_and_stiffness_kernel(dim):
    xyz, cells = wl.square_mesh(4) if dim == 2 else wl.cube_mesh(2)
    th = TaylorHood(xyz, cells)
    M = th.scalar_mass_full()
    assert abs(M.sum() - 1.0) < 1e-13
    K = th._assemble_nodes(th.element_stiffness())
    assert np.abs(K @ np.ones(th.nnodes)).max() < 1e-12
    # int x*y over the unit square/cube via the mass matrix: 1^T M I(xy)
    xy = th.node_xyz[:, 0] * th.node_xyz[:, 1]
    assert abs(np.ones(th.nnodes) @ (M @ xy) - 0.25) < 1e-13


def test_divergence_closed_form_2d():
    # u = (x^2, x y), q = 1 + x + 2y: -int q div u = -int (1+x+2y) 3x = -4
    xyz, cells = wl.square_mesh(3)
    th = TaylorHood(xyz, cells)
    Bc = th.divergence_full()
    X = th.node_xyz
    u = [X[:, 0] ** 2, X[:, 0] * X[:, 1]]
    q = 1 + th.xyz[:, 0] + 2 * th.xyz[:, 1]
    val = sum(u[c] @ (Bc[c] @ q) for c in range(2))
    assert abs(val + 4.0) < 1e-13


def test_divergence_closed_form_3d():
    # u = (x^2, x y, y z), q = 1 + z: div u = 3x + y, -int (1+z)(3x+y) = -3
    xyz, cells = wl.cube_mesh(2)
    th = TaylorHood(xyz, cells)
    Bc = th.divergence_full()
    X = th.node_xyz
    u = [X[:, 0] ** 2, X[:, 0] * X[:, 1], X[:, 1] * X[:, 2]]
    q = 1 + th.xyz[:, 2]
    val = sum(u[c] @ (Bc[c] @ q) for c in range(3))
    assert abs(val + 3.0) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_divergence_kills_constants_after_elimination(dim):
    xyz, cells = wl.square_mesh(6) if dim == 2 else wl.cube_mesh(2)
    th = TaylorHood(xyz, cells)
    B = th.divergence()
    assert np.abs(B @ np.ones(th.nverts)).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_convection_skew_for_constant_wind(dim):
    xyz, cells = wl.square_mesh(5) if dim == 2 else wl.cube_mesh(2)
    th = TaylorHood(xyz, cells)
    w = th.interpolate(wl.ConstantField(np.array([0.7, -1.3, 0.4][:dim])))
    _, _, C, _ = th.scalar_matrices(1.0, w)
    x = np.random.default_rng(0).standard_normal(th.nfree)
    assert abs(x @ (C @ x)) < 1e-12 * np.abs(C).sum()
    assert abs(x @ (C @ x)) < 1e-13
    # C is not symmetric (it is skew on the free space)
    assert abs((C - C.T).sum()) >= 0 and np.abs((C + C.T).toarray()).max() < 1e-13


def test_nested_parent_maps():
    for lv in (wl.square_hierarchy(2, 3), wl.cube_hierarchy(1, 3)):
        for c, f in zip(lv[:-1], lv[1:]):
            # every fine vertex of a fine cell lies in the closed parent cell
            d = f.dim
            x0 = c.xyz[c.cells[f.parent, 0]]
            Jm = np.stack([c.xyz[c.cells[f.parent, k + 1]] - x0 for k in range(d)], axis=2)
            for v in range(d + 1):
                xi = np.linalg.solve(Jm, (f.xyz[f.cells[:, v]] - x0)[..., None])[..., 0]
                lam = np.hstack([1 - xi.sum(1, keepdims=True), xi])
                assert lam.min() > -1e-12


# ------------------------------------------------------------------ crossed mesh
def _crossed_counts(n):
    V = (n + 1) ** 2 + n * n            # corners + quad centres
    E = 2 * n * (n + 1) + 4 * n * n     # quad sides + four spokes per quad
    return V, E


@pytest.mark.parametrize("n", [2, 3, 5])
def test_crossed_mesh_counts(n):
    """Crossed quads (Sec. 5.1): vertex, P2 node and per-stage DOF counts equal the
    closed forms; every cell positively oriented; the cells tile the unit square."""
    xyz, cells = wl.crossed_mesh(n)
    th = TaylorHood(xyz, cells)
    V, E = _crossed_counts(n)
    assert th.nverts == V and th.nnodes == V + E and cells.shape[0] == 4 * n * n
    assert 2 * th.nnodes + th.nverts == 3 * V + 2 * E
    p = xyz[cells]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                  - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    assert area.min() > 0 and abs(area.sum() - 1.0) < 1e-14


def test_crossed_hierarchy_nesting_and_paper_size():
    """Red refinement of the crossed 8x8 mesh: children inside their parents, counts of
    the crossed mesh at 8 * 2^l, and 1,182,211 DOFs per stage (Dirichlet included) at
    l = 5, the paper's "about 1.1 million" (Sec. 5.1)."""
    lv = wl.crossed_hierarchy(8, 3)
    for l in range(1, 3):
        f, c = lv[l], lv[l - 1]
        cen = f.xyz[f.cells].mean(axis=1)
        P = c.xyz[c.cells[f.parent]]  # (nc, 3, 2)
        T = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)
        lam = np.linalg.solve(T, (cen - P[:, 0])[..., None])[..., 0]
        assert lam.min() > 0 and (lam.sum(axis=1)).max() < 1
        V, E = _crossed_counts(8 * 2 ** l)
        th = TaylorHood(f.xyz, f.cells)
        assert th.nverts == V and th.nnodes == V + E
    V, E = _crossed_counts(8 * 2 ** 5)
    assert 3 * V + 2 * E == 1182211
