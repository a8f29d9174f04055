"""Pins for oracle/transfer.py: polynomial reproduction and the Galerkin identity."""
import numpy as np
import pytest

from oracle.fem import TaylorHood
from oracle.stage import StageSystem
from oracle.tableau import tableau
from oracle.transfer import _locate, interpolation_matrices, p2_values, stage_prolongation
from paper_2202_07381_amd import workloads as wl


def _pair(dim):
    lv = wl.square_hierarchy(2, 2) if dim == 2 else wl.cube_hierarchy(1, 2)
    return TaylorHood(lv[0].xyz, lv[0].cells), TaylorHood(lv[1].xyz, lv[1].cells)


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_reproduces_quadratics(dim):
    c, f = _pair(dim)
    # full-space interpolation built from point location, checked on x_i x_j
    cell, lam = _locate(c, f.node_xyz)
    w = p2_values(lam, dim)
    for a in range(dim):
        for b in range(a, dim):
            q = lambda X: X[:, a] * X[:, b] + 0.3 * X[:, a] - 0.2
            vals = (w * q(c.node_xyz)[c.cell_nodes[cell]]).sum(axis=1)
            assert np.abs(vals - q(f.node_xyz)).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_reproduces_linears(dim):
    c, f = _pair(dim)
    _, Pp = interpolation_matrices(c, f)
    lin = lambda X: 1.0 + X @ np.arange(1, dim + 1)
    assert np.abs(Pp @ lin(c.xyz) - lin(f.xyz)).max() < 1e-14


def test_p2_weights_are_the_canonical_set():
    c, f = _pair(2)
    Pu, _ = interpolation_matrices(c, f)
    allowed = np.array([1.0, 0.75, 0.375, -0.125, 0.5, 0.25])
    assert np.all(np.min(np.abs(Pu.data[:, None] - allowed[None, :]), axis=1) < 1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_galerkin_identity(dim):
    lv = wl.square_hierarchy(2, 2) if dim == 2 else wl.cube_hierarchy(1, 2)
    A, b, cc = tableau("radauIIA", 2)
    sys = [StageSystem(TaylorHood(m.xyz, m.cells), A, 0.05, 0.8) for m in lv]
    Pu, Pp = interpolation_matrices(sys[0].th, sys[1].th)
    P = stage_prolongation(Pu, Pp, dim, 2)
    G = (P.T @ sys[1].J @ P).toarray()
    Jc = sys[0].J.toarray()
    assert np.abs(G - Jc).max() < 1e-13 * np.abs(Jc).max()
