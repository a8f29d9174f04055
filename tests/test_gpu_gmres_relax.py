"""GPU parity of the GMRES relaxation (Sec. 4.2: a Vanka-preconditioned GMRES iteration
as the relaxation; Sec. 5.4 uses it for its convective problem) against the oracle,
through the C ABI: one cycle of m left-preconditioned GMRES steps with the weighted
additive operator, classical Gram--Schmidt, from the current iterate.  Tolerances: one
relaxation step 1e-10 (the patch inverses are factored differently on the two sides and
the step normalises and solves a small least-squares problem); V-cycles
1e-11 as for the other relaxations; FGMRES solutions after equal
iteration counts 1e-10."""
import numpy as np
import pytest

from gpu_cases import forcing_rhs, gpu_of, levels_of, oracle_of, relerr, say, to_dev, to_host
from test_gpu_parity import VCYCLE_TOL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GR_CASES = ["c1", "r3", "oseen", "3d2", "cross"]


@pytest.mark.parametrize("form", [0, 2])
@pytest.mark.parametrize("case", GR_CASES)
def test_gmres_step_each_level(case, form):
    g, H = gpu_of(case, patch_form=form, smoother=2), oracle_of(case, smoother="gmres")
    rng = np.random.default_rng(51)
    for lev in range(1, g.nlevels):
        J = H.systems[lev].J
        F, k0 = rng.standard_normal(J.shape[0]), rng.standard_normal(J.shape[0])
        for tr in (False, True):
            say(f"[gmres step] case={case} form={form} level={lev} transpose={tr}")
            k = to_dev(k0)
            g.irk_level_sweep(lev, to_dev(F), k, transpose=tr)
            ref = H.smoothers[lev].gmres(F, k0, J.T if tr else J, 1, tr)
            assert relerr(to_host(k), ref) < 1e-10


@pytest.mark.parametrize("form", [0, 2])
@pytest.mark.parametrize("case", GR_CASES)
def test_gmres_vcycle(case, form):
    g, H = gpu_of(case, patch_form=form, smoother=2), oracle_of(case, smoother="gmres")
    r = np.random.default_rng(52).standard_normal(g.irk_mg_ndofs())
    z = torch.zeros(r.size, dtype=torch.float64, device="cuda")
    tol = VCYCLE_TOL
    say(f"[gmres vcycle] case={case} form={form}")
    g.irk_mg_vcycle(to_dev(r), z)
    err = relerr(to_host(z), H.vcycle(r))
    g.irk_mg_vcycle_transpose(to_dev(r), z)
    err_t = relerr(to_host(z), H.vcycle_transpose(r))
    say(f"[gmres vcycle] case={case} form={form} err={err:.2e} err^T={err_t:.2e} tol={tol:.2e}")
    assert err < tol and err_t < tol


@pytest.mark.parametrize("case", GR_CASES)
def test_gmres_fgmres_matches_oracle(case):
    from oracle.fgmres import fgmres

    g, H = gpu_of(case, smoother=2), oracle_of(case, smoother="gmres")
    S = H.finest
    F = forcing_rhs(case)
    for rtol, maxit in ((1e-8, 200), (1e-30, 4)):
        say(f"[gmres fgmres] case={case} rtol={rtol}")
        k = torch.zeros(F.size, dtype=torch.float64, device="cuda")
        info = g.irk_fgmres_solve(to_dev(F), k, rtol=rtol, maxit=maxit, restart=30)
        xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), rtol, maxit, 30, project=S.project_pressure_mean)
        assert info["iterations"] == io.iterations
        assert relerr(to_host(k), xo) < 1e-10


def test_gmres_three_steps_and_adjoint():
    """3 pre- and post-steps (the count of Sec. 5.4) on the Oseen case: V-cycle, FGMRES and
    the adjoint solve against the oracle."""
    from oracle.fgmres import fgmres
    from oracle.multigrid import Hierarchy
    from oracle.tableau import tableau
    from gpu_cases import CASES, wind_of
    from paper_2202_07381_amd import irkmg

    dim, nc, nl, fam, r, dt, nu, ws = CASES["oseen"]
    lv = levels_of("oseen")
    A, b, c = irkmg.irk_tableau_builtin(fam, r)
    nodes = irkmg.irk_mesh_p2_nodes(lv[-1])
    g = irkmg.IrkMG(lv, A, b, c, dt, nu, wind_nodal=wind_of("oseen")(nodes), pre=3, post=3, smoother=2)
    H = Hierarchy(lv, tableau(fam, r)[0], dt, nu, wind=wind_of("oseen"), pre=3, post=3, smoother="gmres")
    S = H.finest
    rv = np.random.default_rng(53).standard_normal(S.n)
    z = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    say("[gmres 3/3] vcycle")
    g.irk_mg_vcycle(to_dev(rv), z)
    err = relerr(to_host(z), H.vcycle(rv))
    say(f"[gmres 3/3] vcycle err={err:.2e}")
    assert err < VCYCLE_TOL
    F = forcing_rhs("oseen")
    say("[gmres 3/3] fgmres")
    k = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    info = g.irk_fgmres_solve(to_dev(F), k, rtol=1e-8, maxit=100)
    xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 100, 30, project=S.project_pressure_mean)
    assert info["converged"] and info["iterations"] == io.iterations
    assert relerr(to_host(k), xo) < 1e-10
    G = S.J.T @ np.random.default_rng(54).standard_normal(S.n)
    say("[gmres 3/3] adjoint")
    lam = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    info = g.irk_adjoint_solve(to_dev(G), lam, rtol=1e-8, maxit=100)
    xo, io = fgmres(S.apply_transpose, H.vcycle_transpose, G, np.zeros_like(G), 1e-8, 100, 30,
                    project=S.project_pressure_mean)
    assert info["converged"] and info["iterations"] == io.iterations
    assert relerr(to_host(lam), xo) < 1e-10
    g.close()


def test_gmres_options_rejected():
    from paper_2202_07381_amd import irkmg

    A, b, c = irkmg.irk_tableau_builtin("radauIIA", 2)
    for pre, post in ((9, 2), (2, 9)):
        with pytest.raises(irkmg.IrkError) as e:
            irkmg.IrkMG(levels_of("c1"), A, b, c, 1 / 16, 1.0, smoother=2, pre=pre, post=post)
        assert e.value.status == irkmg.IRK_EINVAL
    with pytest.raises(irkmg.IrkError) as e:
        irkmg.IrkMG(levels_of("c1"), A, b, c, 1 / 16, 1.0, smoother=3)
    assert e.value.status == irkmg.IRK_EINVAL
