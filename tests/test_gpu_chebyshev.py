"""GPU parity of the Chebyshev-accelerated relaxation (Sec. 5.1: the unweighted additive
Vanka operator accelerated by Chebyshev polynomials of the first kind on [2, 8], 2 pre-
and 2 post-steps) against the oracle, through the C ABI.  Tolerances as in
test_gpu_parity.py: one relaxation step 1e-11 (patch inverses factored differently on
the two sides), V-cycles 1e-11 (as in test_gpu_parity.py), FGMRES solutions after equal
iteration counts 1e-10."""
import numpy as np
import pytest

from gpu_cases import forcing_rhs, gpu_of, oracle_of, relerr, say, to_dev, to_host
from test_gpu_parity import VCYCLE_TOL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CHEB_CASES = ["c1", "r3", "oseen", "lob3", "3d2", "cross"]


@pytest.mark.parametrize("form", [0, 2])
@pytest.mark.parametrize("case", CHEB_CASES)
def test_chebyshev_step_each_level(case, form):
    g, H = gpu_of(case, patch_form=form, smoother=1), oracle_of(case, smoother="chebyshev")
    rng = np.random.default_rng(31)
    for lev in range(1, g.nlevels):
        J = H.systems[lev].J
        F, k0 = rng.standard_normal(J.shape[0]), rng.standard_normal(J.shape[0])
        for tr in (False, True):
            say(f"[cheb step] case={case} form={form} level={lev} transpose={tr}")
            k = to_dev(k0)
            g.irk_level_sweep(lev, to_dev(F), k, transpose=tr)
            ref = H.smoothers[lev].chebyshev(F, k0, J.T if tr else J, 1, 2.0, 8.0, tr)
            assert relerr(to_host(k), ref) < 1e-11


@pytest.mark.parametrize("form", [0, 2])
@pytest.mark.parametrize("case", CHEB_CASES)
def test_chebyshev_vcycle(case, form):
    g, H = gpu_of(case, patch_form=form, smoother=1), oracle_of(case, smoother="chebyshev")
    r = np.random.default_rng(32).standard_normal(g.irk_mg_ndofs())
    z = torch.zeros(r.size, dtype=torch.float64, device="cuda")
    say(f"[cheb vcycle] case={case} form={form}")
    g.irk_mg_vcycle(to_dev(r), z)
    err = relerr(to_host(z), H.vcycle(r))
    g.irk_mg_vcycle_transpose(to_dev(r), z)
    err_t = relerr(to_host(z), H.vcycle_transpose(r))
    say(f"[cheb vcycle] case={case} form={form} err={err:.2e} err^T={err_t:.2e} tol={VCYCLE_TOL:.0e}")
    assert err < VCYCLE_TOL and err_t < VCYCLE_TOL


@pytest.mark.parametrize("case", CHEB_CASES)
def test_chebyshev_fgmres_matches_oracle(case):
    from oracle.fgmres import fgmres

    g, H = gpu_of(case, smoother=1), oracle_of(case, smoother="chebyshev")
    S = H.finest
    F = forcing_rhs(case)
    say(f"[cheb fgmres] case={case}")
    k = torch.zeros(F.size, dtype=torch.float64, device="cuda")
    info = g.irk_fgmres_solve(to_dev(F), k, rtol=1e-8, maxit=200, restart=30)
    xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 200, 30, project=S.project_pressure_mean)
    assert info["converged"] and info["iterations"] == io.iterations
    assert relerr(to_host(k), xo) < 1e-10


def test_chebyshev_options_rejected():
    from paper_2202_07381_amd import irkmg
    from gpu_cases import levels_of

    A, b, c = irkmg.irk_tableau_builtin("radauIIA", 2)
    for lo, hi in ((0.0, 8.0), (8.0, 2.0), (2.0, float("inf"))):
        with pytest.raises(irkmg.IrkError) as e:
            irkmg.IrkMG(levels_of("c1"), A, b, c, 1 / 16, 1.0, smoother=1, interval=(lo, hi))
        assert e.value.status == irkmg.IRK_EINVAL
    g = gpu_of("c1", smoother=1)
    with pytest.raises(irkmg.IrkError) as e:
        irkmg.IrkBatch([g], autotune=False)
    assert e.value.status == irkmg.IRK_EINVAL


@pytest.mark.parametrize("case", ["c1", "oseen", "cross"])
def test_chebyshev_adjoint_solve_matches_oracle(case):
    """The transposed system J^T lam = G (the adjoint solve) preconditioned by the
    transposed Chebyshev V-cycle: equal iteration counts and solutions to 1e-10."""
    from oracle.fgmres import fgmres

    g, H = gpu_of(case, smoother=1), oracle_of(case, smoother="chebyshev")
    S = H.finest
    G = S.J.T @ np.random.default_rng(34).standard_normal(S.n)  # consistent right-hand side
    for rtol, maxit in ((1e-8, 200), (1e-30, 5)):
        say(f"[cheb adjoint] case={case} rtol={rtol}")
        lam = torch.zeros(S.n, dtype=torch.float64, device="cuda")
        info = g.irk_adjoint_solve(to_dev(G), lam, rtol=rtol, maxit=maxit)
        xo, io = fgmres(S.apply_transpose, H.vcycle_transpose, G, np.zeros_like(G), rtol, maxit, 30,
                        project=S.project_pressure_mean)
        assert info["iterations"] == io.iterations
        assert relerr(to_host(lam), xo) < 1e-10


@pytest.mark.parametrize("case", ["c1", "cross", "3d2"])
def test_ritz_estimate_matches_oracle(case):
    """Arnoldi on the relaxation operator S J of each level (Sec. 5.1's interval rule):
    the Hessenberg matrix to 1e-11 of its largest entry and the Ritz values, as a set, to
    1e-8 against the oracle's, from the same start vector."""
    from oracle.vanka import arnoldi_ritz

    g, H = gpu_of(case, smoother=1), oracle_of(case, smoother="chebyshev")
    rng = np.random.default_rng(55)
    for lev in range(1, g.nlevels):
        J = H.systems[lev].J
        steps = min(12, J.shape[0] - 1)
        v0 = rng.standard_normal(J.shape[0])
        say(f"[ritz] case={case} level={lev} steps={steps}")
        Hg, rg = g.irk_mg_ritz(lev, steps, to_dev(v0))
        Ho, ro = arnoldi_ritz(lambda x: J @ x, H.smoothers[lev].apply_S, v0, steps)
        assert rg.size == ro.size == steps
        assert np.abs(Hg - Ho).max() <= 1e-11 * np.abs(Ho).max()
        # the same values (a conjugate pair's order within equal real parts may differ)
        tol = 1e-8 * np.abs(ro).max()
        assert all(np.min(np.abs(rg - z)) <= tol for z in ro)
        assert all(np.min(np.abs(ro - z)) <= tol for z in rg)
        assert abs(rg[0].real - ro[0].real) <= tol


def test_interval_from_ritz_estimate():
    """[lambda/4, lambda] from the finest level's largest Ritz value (the paper's rule)
    set on the handle; the V-cycle then matches the oracle's with that interval."""
    from oracle.multigrid import Hierarchy
    from oracle.tableau import tableau
    from gpu_cases import CASES, levels_of

    case = "cross"
    g = gpu_of(case, smoother=1)
    dim, nc, nl, fam, r, dt, nu, ws = CASES[case]
    lev = g.nlevels - 1
    v0 = np.random.default_rng(56).standard_normal(g.irk_mg_ndofs(lev))
    say("[ritz interval] estimate")
    _, ritz = g.irk_mg_ritz(lev, 20, to_dev(v0))
    lam = float(ritz[0].real)
    say(f"[ritz interval] lambda_max estimate {lam:.4f}")
    assert lam > 1.0
    g.irk_mg_set_interval(lam / 4, lam)
    try:
        Ho = Hierarchy(levels_of(case), tableau(fam, r)[0], dt, nu, weighted=False, smoother="chebyshev",
                       interval=(lam / 4, lam))
        rv = np.random.default_rng(57).standard_normal(g.irk_mg_ndofs())
        z = torch.zeros(rv.size, dtype=torch.float64, device="cuda")
        say("[ritz interval] vcycle")
        g.irk_mg_vcycle(to_dev(rv), z)
        err = relerr(to_host(z), Ho.vcycle(rv))
        say(f"[ritz interval] vcycle err={err:.2e}")
        assert err < VCYCLE_TOL
    finally:
        g.irk_mg_set_interval(2.0, 8.0)  # the cached handle keeps the paper's interval
    from paper_2202_07381_amd import irkmg
    with pytest.raises(irkmg.IrkError):
        g.irk_mg_set_interval(3.0, 2.0)
