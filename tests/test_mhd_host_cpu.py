"""The library's host assembly of the linearised MHD stage system (irk_mhd_host_operators,
no device work) against the oracle (oracle/mhd.py; Sec. 3.3, 4.1): the spatial mass M
and operator S of every level of a hierarchy, with the state rediscretised on the coarse
levels, and the prolongations diag(P_u, P_B, P_p, P_gamma).  Both sides integrate
exactly (the library by moments of barycentric monomials, the oracle by quadrature), so
the entries agree to rounding: 1e-13 relative to the largest entry."""
import numpy as np
import pytest

from oracle.fem import TaylorHood
from oracle.mhd import MHDHierarchy, MHDSpace, island_state
from oracle.tableau import tableau
from paper_2202_07381_amd import irkmg
from paper_2202_07381_amd import workloads as wl


def _state(lv, seed):
    w0, b0 = wl.island_coalescence(lv[-1].xyz, lv[-1].cells)
    if seed is not None:
        w0 = 0.3 * np.random.default_rng(seed).standard_normal(w0.shape)
    return w0, b0


@pytest.mark.parametrize("nc,nl,Re,Rem,seed", [(2, 3, 50.0, 20.0, 3), (3, 2, 5000.0, 5000.0, None)])
def test_host_operators_match_oracle(nc, nl, Re, Rem, seed):
    lv = wl.square_hierarchy(nc, nl)
    w0, b0 = _state(lv, seed)
    A, _, _ = tableau("lobattoIIIC", 2)
    H = MHDHierarchy(lv, A, 0.025, Re, Rem, w0, b0)
    for level in range(nl):
        M, S, P = irkmg.irk_mhd_host_operators(lv, level, Re, Rem, w0, b0)
        assert M.shape == H.M[level].shape
        assert abs(M - H.M[level]).max() <= 1e-13 * abs(H.M[level]).max()
        assert abs(S - H.S[level]).max() <= 1e-13 * abs(H.S[level]).max()
        if level == 0:
            assert P is None
            continue
        ns, nsc = H.spaces[level].ns, H.spaces[level - 1].ns
        Po = H.P[level][:ns, :nsc]
        assert P.shape == Po.shape and P.nnz == Po.nnz
        assert abs(P - Po).max() <= 1e-14


@pytest.mark.parametrize("hier", ["square", "crossed"])
def test_island_input_is_the_oracle_island_state(hier):
    """The shared input generator gives the oracle's island-coalescence state."""
    lv = (wl.square_hierarchy(3, 2) if hier == "square" else wl.crossed_hierarchy(2, 2))[-1]
    w_o, b_o = island_state(MHDSpace(TaylorHood(lv.xyz, lv.cells)))
    w, b = wl.island_coalescence(lv.xyz, lv.cells)
    assert w.shape == w_o.shape and not w.any()
    assert np.abs(b - b_o).max() <= 1e-15 * np.abs(b_o).max()


def test_host_operators_reject_invalid_meshes():
    lv = wl.square_hierarchy(2, 2)
    w0, b0 = _state(lv, None)
    with pytest.raises(irkmg.IrkError) as e:
        irkmg.irk_mhd_host_operators(lv, 5, 1.0, 1.0, w0, b0)
    assert e.value.status == irkmg.IRK_EINVAL
    with pytest.raises(irkmg.IrkError) as e:
        irkmg.irk_mhd_host_operators(lv, 0, -1.0, 1.0, w0, b0)
    assert e.value.status == irkmg.IRK_EINVAL
    bad = [lv[0], wl.MeshLevel(2, lv[1].xyz, lv[1].cells[:-1], lv[1].parent[:-1])]
    with pytest.raises(irkmg.IrkError) as e:
        irkmg.irk_mhd_host_operators(bad, 1, 1.0, 1.0, w0, b0)
    assert e.value.status == irkmg.IRK_EINVAL
    cube = wl.cube_hierarchy(1, 1) if hasattr(wl, "cube_hierarchy") else None
    if cube is not None:
        with pytest.raises(irkmg.IrkError):
            irkmg.irk_mhd_host_operators(cube, 0, 1.0, 1.0, w0, b0)


def test_host_operators_threaded_assembly():
    """On a 64 x 64 level the host assembly runs on threads (pattern rows, vertex-disjoint
    cell groups, patch lists): the result matches the oracle to rounding and is bitwise
    the same on a second call."""
    lv = wl.square_hierarchy(4, 5)
    w0, b0 = _state(lv, 5)
    M, S, P = irkmg.irk_mhd_host_operators(lv, 4, 300.0, 200.0, w0, b0)
    Mo, So = MHDSpace(TaylorHood(lv[-1].xyz, lv[-1].cells)).operators(300.0, 200.0, w0, b0)
    assert abs(M - Mo).max() <= 1e-13 * abs(Mo).max()
    assert abs(S - So).max() <= 1e-13 * abs(So).max()
    M2, S2, P2 = irkmg.irk_mhd_host_operators(lv, 4, 300.0, 200.0, w0, b0)
    for x, y in ((M, M2), (S, S2), (P, P2)):
        assert (x.indptr == y.indptr).all() and (x.indices == y.indices).all() and (x.data == y.data).all()


def test_host_operators_vertex_of_high_valence():
    """A fan of 70 triangles around one vertex (more cells around a vertex than the
    assembly's 64 cell groups can separate): the cells are assembled in order on one
    thread and the operators still match the oracle."""
    m = 70
    t = 2 * np.pi * np.arange(m) / m
    xyz = np.concatenate([[[0.0, 0.0]], np.stack([np.cos(t), np.sin(t)], 1)])
    cells = np.array([[0, 1 + i, 1 + (i + 1) % m] for i in range(m)], dtype=np.int64)
    lv = [wl.MeshLevel(2, xyz, cells, None)]
    th = TaylorHood(xyz, cells)
    rng = np.random.default_rng(8)
    w0 = 0.2 * rng.standard_normal((xyz.shape[0] + th.nedges, 2))
    b0 = rng.standard_normal(th.nedges)
    M, S, _ = irkmg.irk_mhd_host_operators(lv, 0, 40.0, 30.0, w0, b0)
    Mo, So = MHDSpace(th).operators(40.0, 30.0, w0, b0)
    assert abs(M - Mo).max() <= 1e-13 * abs(Mo).max()
    assert abs(S - So).max() <= 1e-13 * abs(So).max()
