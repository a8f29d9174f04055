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
