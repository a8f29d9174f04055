"""Set-up is deterministic where the host assembly runs on threads.

The level operators, patches and Dirichlet couplings are assembled on host threads once a
level is large enough (rows by ranges, element matrices in groups of cells that share no
vertex, patch lists in two passes).  Two handles built from the same input must apply
bitwise the same V-cycle: on a 64 x 64 Oseen hierarchy (convection assembled, 8 cell
groups) and on a 16^3 Kuhn-cube Stokes hierarchy (31 cell groups), each with enough
cells per group for several threads.  The assembled values themselves are checked
against the oracle by the parity suite; this checks that threads leave no trace.
"""
import numpy as np
import pytest

from tests.gpu_cases import say, to_dev, to_host
from paper_2202_07381_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim", [2, 3])
def test_two_setups_give_bitwise_equal_vcycles(dim):
    import torch

    from paper_2202_07381_amd import irkmg

    if dim == 2:
        lv = wl.square_hierarchy(4, 5)
        A, b, c = irkmg.irk_tableau_builtin("radauIIA", 3)
        wind = wl.wind_2d(3, 64)(irkmg.irk_mesh_p2_nodes(lv[-1]))
        nu, dt = 0.01, 5e-3
    else:
        lv = wl.cube_hierarchy(2, 4)
        A, b, c = irkmg.irk_tableau_builtin("radauIIA", 2)
        wind, nu, dt = None, 1.0, 1e-2
    outs = []
    for k in range(2):
        say(f"[repeatable] dim={dim} set-up {k}")
        g = irkmg.IrkMG(lv, A, b, c, dt, nu, wind_nodal=wind)
        N = g.irk_mg_ndofs()
        r = to_dev(wl.random_vector(N, 11))
        z = torch.empty_like(r)
        g.irk_mg_vcycle(r, z)
        torch.cuda.synchronize()
        outs.append(to_host(z))
        del g
    say(f"[repeatable] dim={dim} N={outs[0].size} max |z| {np.abs(outs[0]).max():.3e}")
    assert np.isfinite(outs[0]).all()
    assert np.array_equal(outs[0], outs[1])
