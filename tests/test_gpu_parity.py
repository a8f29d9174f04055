"""GPU parity of every step of the hot path against the CPU oracle, through the C ABI.

Tolerances: single operator applications (residual, transfers) 1e-13 relative to the
largest entry; patch sweeps 1e-11 (the patch inverses come from different elimination
orders on the two sides, so they agree to the conditioning of the patch matrices
times the unit roundoff); coarse solve and V-cycle max(1e-12, 4 cond_S(J_0) eps) with
Skeel's componentwise condition number cond_S(J_0) = || |J_0^{-1}| |J_0| ||_inf of the
pinned coarse operator (1e3 to 6e5 on these cases, against normwise condition numbers
up to 1.3e8, which come from the scaling of the stage blocks): the oracle solves by LU
with partial pivoting, the library by its stored inverse followed by one step of FP64
iterative refinement, two solves whose forward errors are bounded by a small multiple
of cond_S eps (Skeel's bound for a solve that is componentwise backward stable, which
one refinement step in working precision provides); whole V-cycles (every relaxation)
1e-11, about 20 times the largest difference measured (4.8e-13 on the 128 x 128 case;
1e-14 to 7e-14 on the small cases, while the coarse solve alone differs by up to 7e-11
on them); the measured errors are printed; FGMRES solutions after equal iteration
counts 1e-10 relative (the target stated for the method).  Sweeps, V-cycles and solves run with the patch forms 0 (dense patch
inverses), 1 (inverses factored through the stage eigenbasis) and 2 (automatic: for
r >= 2 the symmetric factored form, wrapped diagonals of each block inverse, on the
Stokes cases, else form 1), which apply the same operator up to rounding."""
import numpy as np
import pytest

from gpu_cases import CASES, SMALL, forcing_rhs, gpu_of, levels_of, oracle_of, relerr, say, to_dev, to_host, wind_of

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ALL = list(SMALL)
FORMS = [0, 1, 2]


@pytest.mark.parametrize("case", ALL)
def test_apply_all_levels(case):
    g, H = gpu_of(case), oracle_of(case)
    rng = np.random.default_rng(11)
    for lev in range(g.nlevels):
        J = H.systems[lev].J
        x = rng.standard_normal(J.shape[0])
        for tr in (False, True):
            say(f"[apply] case={case} level={lev} transpose={tr}")
            y = torch.zeros(J.shape[0], dtype=torch.float64, device="cuda")
            g.irk_level_apply(lev, to_dev(x), y, transpose=tr)
            ref = (J.T if tr else J) @ x
            assert relerr(to_host(y), ref) < 1e-13


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("case", ALL)
def test_sweep_each_level(case, form):
    g, H = gpu_of(case, patch_form=form), oracle_of(case)
    rng = np.random.default_rng(12)
    for lev in range(1, g.nlevels):
        J = H.systems[lev].J
        F, k0 = rng.standard_normal(J.shape[0]), rng.standard_normal(J.shape[0])
        for tr in (False, True):
            say(f"[sweep] case={case} form={form} level={lev} transpose={tr}")
            k = to_dev(k0)
            g.irk_level_sweep(lev, to_dev(F), k, transpose=tr)
            ref = H.smoothers[lev].sweep(F, k0, J.T if tr else J, tr)
            assert relerr(to_host(k), ref) < 1e-11


@pytest.mark.parametrize("case", ALL)
def test_transfers(case):
    g, H = gpu_of(case), oracle_of(case)
    rng = np.random.default_rng(13)
    for lev in range(1, g.nlevels):
        P = H.P[lev]
        xf, xc, base = rng.standard_normal(P.shape[0]), rng.standard_normal(P.shape[1]), rng.standard_normal(P.shape[0])
        say(f"[transfer] case={case} level={lev}")
        out = torch.zeros(P.shape[1], dtype=torch.float64, device="cuda")
        g.irk_level_restrict(lev, to_dev(xf), out)
        assert relerr(to_host(out), P.T @ xf) < 1e-13
        fine = to_dev(base)
        g.irk_level_prolong(lev, to_dev(xc), fine)
        assert relerr(to_host(fine), base + P @ xc) < 1e-13


VCYCLE_TOL = 1e-11
_SKEEL = {}


def coarse_tol(H):
    """max(1e-12, 4 cond_S(J_0) eps) for the pinned coarse operator J_0 of H, with
    Skeel's condition number cond_S(J_0) = || |J_0^{-1}| |J_0| ||_inf."""
    if id(H) not in _SKEEL:
        J = H.ops[0].toarray()
        for q in H.pinned:
            J[q, :] = 0.0
            J[:, q] = 0.0
            J[q, q] = 1.0
        cs = float(np.max(np.abs(np.linalg.inv(J)) @ np.abs(J) @ np.ones(J.shape[0])))
        _SKEEL[id(H)] = (H, max(1e-12, 4 * cs * np.finfo(float).eps))
    return _SKEEL[id(H)][1]


@pytest.mark.parametrize("case", ALL)
def test_coarse_solve(case):
    g, H = gpu_of(case), oracle_of(case)
    J0 = H.systems[0].J
    b = J0 @ np.random.default_rng(14).standard_normal(J0.shape[0])  # consistent
    for tr in (False, True):
        say(f"[coarse] case={case} transpose={tr}")
        x = torch.zeros_like(to_dev(b))
        g.irk_coarse_solve(to_dev(b), x, transpose=tr)
        err = relerr(to_host(x), H.coarse_solve(b, tr))
        say(f"[coarse] case={case} transpose={tr} err={err:.2e} tol={coarse_tol(H):.2e}")
        assert err < coarse_tol(H)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("case", ALL)
def test_vcycle(case, form):
    g, H = gpu_of(case, patch_form=form), oracle_of(case)
    r = np.random.default_rng(15).standard_normal(g.irk_mg_ndofs())
    say(f"[vcycle] case={case} form={form}")
    z = torch.zeros(r.size, dtype=torch.float64, device="cuda")
    g.irk_mg_vcycle(to_dev(r), z)
    err = relerr(to_host(z), H.vcycle(r))
    g.irk_mg_vcycle_transpose(to_dev(r), z)
    err_t = relerr(to_host(z), H.vcycle_transpose(r))
    say(f"[vcycle] case={case} form={form} err={err:.2e} err^T={err_t:.2e} tol={VCYCLE_TOL:.0e}")
    assert err < VCYCLE_TOL and err_t < VCYCLE_TOL


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("case", ALL)
def test_vcycle_bitwise_repeatable(case, form):
    g = gpu_of(case, patch_form=form)
    r = to_dev(np.random.default_rng(16).standard_normal(g.irk_mg_ndofs()))
    say(f"[repeat] case={case} form={form}")
    outs = []
    for _ in range(5):
        z = torch.zeros_like(r)
        g.irk_mg_vcycle(r, z)
        outs.append(to_host(z))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("case", ALL)
def test_fgmres_matches_oracle(case, form):
    from oracle.fgmres import fgmres

    g, H = gpu_of(case, patch_form=form), oracle_of(case)
    S = H.finest
    F = forcing_rhs(case)
    for rtol, maxit in ((1e-8, 200), (1e-30, 4)):
        say(f"[fgmres] case={case} form={form} rtol={rtol} maxit={maxit}")
        k = torch.zeros(F.size, dtype=torch.float64, device="cuda")
        info = g.irk_fgmres_solve(to_dev(F), k, rtol=rtol, maxit=maxit, restart=30)
        xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), rtol, maxit, 30, project=S.project_pressure_mean)
        assert info["iterations"] == io.iterations
        assert relerr(to_host(k), xo) < 1e-10
        if rtol > 1e-20:
            assert info["converged"] and info["rel_residual"] <= rtol


def test_fgmres_restart_and_initial_guess():
    from oracle.fgmres import fgmres

    g, H = gpu_of("c1"), oracle_of("c1")
    S = H.finest
    F = forcing_rhs("c1")
    k0 = np.random.default_rng(17).standard_normal(F.size)
    say("[fgmres-restart] case=c1 restart=3")
    k = to_dev(k0)
    info = g.irk_fgmres_solve(to_dev(F), k, rtol=1e-9, maxit=100, restart=3)
    xo, io = fgmres(S.apply, H.vcycle, F, k0, 1e-9, 100, 3, project=S.project_pressure_mean)
    assert info["iterations"] == io.iterations
    assert relerr(to_host(k), xo) < 1e-10


def test_rhs_and_update():
    from paper_2202_07381_amd import workloads as wl

    g, H = gpu_of("r3"), oracle_of("r3")
    S = H.finest
    rng = np.random.default_rng(18)
    u, p = rng.standard_normal(S.th.nvel), rng.standard_normal(S.th.nverts)
    fn = [rng.standard_normal((S.th.nnodes, S.th.dim)) for _ in range(S.r)]
    say("[rhs] case=r3")
    F = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    g.irk_rhs(to_dev(np.stack(fn).ravel()), to_dev(np.concatenate([u, p])), F)
    assert relerr(to_host(F), S.rhs(fn, u, p)) < 1e-13
    kk = rng.standard_normal(S.n)
    state = to_dev(np.concatenate([u, p]))
    g.irk_update(to_dev(kk), state)
    ref = np.concatenate([u, p]) + sum(S.dt * g.b[j] * kk[j * S.ns:(j + 1) * S.ns] for j in range(S.r))
    assert relerr(to_host(state), ref) < 1e-14


@pytest.mark.parametrize("case", ["r3", "cross"])
def test_rhs_dirichlet(case):
    """Boundary-data terms of the right-hand side (irk_rhs + irk_rhs_dirichlet) against
    the oracle on random node data: 1e-13 of the largest entry."""
    g, H = gpu_of(case), oracle_of(case)
    S = H.finest
    th = S.th
    rng = np.random.default_rng(21)
    u, p = rng.standard_normal(th.nvel), rng.standard_normal(th.nverts)
    fn = [rng.standard_normal((th.nnodes, th.dim)) for _ in range(S.r)]
    gn = rng.standard_normal((th.nnodes, th.dim))
    gst = [rng.standard_normal((th.nnodes, th.dim)) for _ in range(S.r)]
    say(f"[rhs dirichlet] case={case}")
    F = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    g.irk_rhs(to_dev(np.stack(fn).ravel()), to_dev(np.concatenate([u, p])), F)
    g.irk_rhs_dirichlet(to_dev(gn.ravel()), to_dev(np.stack(gst).ravel()), F)
    ref = S.rhs(fn, u, p) + S.rhs_dirichlet(gn, gst)
    assert relerr(to_host(F), ref) < 1e-13


@pytest.mark.parametrize("form", FORMS)
def test_mixed_precision_reaches_tolerance(form):
    g64, g32, H = gpu_of("r3", patch_form=form), gpu_of("r3", precision=1, patch_form=form), oracle_of("r3")
    F = forcing_rhs("r3")
    say("[mixed] case=r3")
    k64 = torch.zeros(F.size, dtype=torch.float64, device="cuda")
    i64 = g64.irk_fgmres_solve(to_dev(F), k64, rtol=1e-8)
    k32 = torch.zeros_like(k64)
    i32 = g32.irk_fgmres_solve(to_dev(F), k32, rtol=1e-8)
    assert i32["converged"] and i32["rel_residual"] <= 1e-8
    S = H.finest
    res = np.linalg.norm(F - S.J @ to_host(k32)) / np.linalg.norm(F)
    assert res <= 1e-8
    say(f"[mixed] its fp64={i64['iterations']} fp32={i32['iterations']} "
        f"rel diff={np.linalg.norm(to_host(k32) - to_host(k64)) / np.linalg.norm(to_host(k64)):.2e}")


def test_error_paths():
    from paper_2202_07381_amd import irkmg

    g = gpu_of("c1")
    F = forcing_rhs("c1")
    say("[errors] case=c1")
    k = torch.zeros(F.size, dtype=torch.float64, device="cuda")
    info = g.irk_fgmres_solve(to_dev(F), k, rtol=1e-12, maxit=1)
    assert info["status"] == irkmg.IRK_ENOCONV and info["iterations"] == 1
    Fn = F.copy()
    Fn[3] = np.nan
    with pytest.raises(irkmg.IrkError) as e:
        g.irk_fgmres_solve(to_dev(Fn), k, rtol=1e-8, maxit=10)
    assert e.value.status == irkmg.IRK_ENAN
    with pytest.raises(ValueError):
        g.irk_mg_vcycle(to_dev(F[:-1]), k)


def test_patch_form_selection():
    """Automatic form: for r >= 2 symmetric factored on Stokes (2D, and 3D with its
    196-unknown patches, four rows per lane), factored for Oseen (a non-symmetric
    operator), dense for r = 1; every form can be forced where it applies, including the
    factored and the symmetric factored forms at r = 1 (one real block, W = 1); forcing
    the symmetric form with a wind is refused."""
    from paper_2202_07381_amd import irkmg

    for case in ALL:
        dim, r, ws = CASES[case][0], CASES[case][4], CASES[case][7]
        want = 0 if r < 2 else (1 if ws is not None else 3)
        assert gpu_of(case, patch_form=2).irk_mg_patch_form() == want, case
        assert gpu_of(case, patch_form=0).irk_mg_patch_form() == 0, case
    rng = np.random.default_rng(19)
    for form in (1, 3):
        g, H = gpu_of("be", patch_form=form), oracle_of("be")
        assert g.irk_mg_patch_form() == form
        for lev in range(1, g.nlevels):
            J = H.systems[lev].J
            F, k0 = rng.standard_normal(J.shape[0]), rng.standard_normal(J.shape[0])
            for tr in (False, True):
                say(f"[form{form} r=1] level={lev} transpose={tr}")
                k = to_dev(k0)
                g.irk_level_sweep(lev, to_dev(F), k, transpose=tr)
                assert relerr(to_host(k), H.smoothers[lev].sweep(F, k0, J.T if tr else J, tr)) < 1e-11
    for case in ("oseen",):
        dim, nc, nl, fam, r, dt, nu, ws = CASES[case]
        A, b, c = irkmg.irk_tableau_builtin(fam, r)
        lv = levels_of(case)
        w = wind_of(case)
        wind = w(irkmg.irk_mesh_p2_nodes(lv[-1])) if w is not None else None
        with pytest.raises(irkmg.IrkError) as e:
            irkmg.IrkMG(lv, A, b, c, dt, nu, wind_nodal=wind, patch_form=3)
        assert e.value.status == irkmg.IRK_EINVAL, case


# ------------------------------------------------------------- edge cases
def _gauss_collocation(r):
    """r-stage Gauss collocation tableau from the Gauss--Legendre nodes: a_ij = int_0^{c_i}
    l_j(t) dt and b_j = int_0^1 l_j(t) dt for the Lagrange basis l_j on the nodes."""
    x, _ = np.polynomial.legendre.leggauss(r)
    c = 0.5 * (x + 1.0)
    V = np.vander(c, r, increasing=True)  # V[i, m] = c_i^m
    Vinv = np.linalg.inv(V)               # l_j(t) = sum_m Vinv[m, j] t^m
    m = np.arange(1, r + 1)
    A = (c[:, None] ** m[None, :] / m[None, :]) @ Vinv
    b = (1.0 / m) @ Vinv
    return A, b, c


def _custom_case(A, b, c, dt, nlev=3):
    from oracle.multigrid import Hierarchy
    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    lv = wl.square_hierarchy(4, nlev)
    H = Hierarchy(lv, A, dt, 1.0)
    return lv, H


@pytest.mark.parametrize("kind", ["gauss4", "sdirk2"])
def test_custom_tableaux(kind):
    """r = 4 (two complex eigenvalue pairs, the largest stage count) and a defective A (a
    2-stage SDIRK, repeated eigenvalue): automatic patch form symmetric factored (a Stokes
    case) resp. dense, the factored form rejected for the defective A; V-cycle and FGMRES
    against the oracle."""
    from oracle.fgmres import fgmres
    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    if kind == "gauss4":
        A, b, c = _gauss_collocation(4)
        form_expected = 3
    else:
        g_ = 1.0 - 1.0 / np.sqrt(2.0)
        A = np.array([[g_, 0.0], [1.0 - g_, g_]])
        b, c = A[-1].copy(), A.sum(axis=1)
        form_expected = 0
        with pytest.raises(irkmg.IrkError):
            irkmg.IrkMG(wl.square_hierarchy(4, 2), A, b, c, 1 / 32, 1.0, patch_form=1)
    lv, H = _custom_case(A, b, c, 1 / 32)
    say(f"[custom] {kind} setup")
    g = irkmg.IrkMG(lv, A, b, c, 1 / 32, 1.0)
    assert g.irk_mg_patch_form() == form_expected
    S = H.finest
    r = np.random.default_rng(41).standard_normal(S.n)
    z = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    g.irk_mg_vcycle(to_dev(r), z)
    err = relerr(to_host(z), H.vcycle(r))
    say(f"[custom] {kind} vcycle err={err:.2e}")
    assert err < VCYCLE_TOL
    f = wl.forcing_2d(1)
    F = S.rhs([S.th.interpolate(f, 0.0)] * S.r, np.zeros(S.th.nvel), np.zeros(S.th.nverts))
    k = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    info = g.irk_fgmres_solve(to_dev(F), k, rtol=1e-8, maxit=200)
    xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 200, 30, project=S.project_pressure_mean)
    say(f"[custom] {kind} its={info['iterations']} oracle={io.iterations}")
    assert info["converged"] and info["iterations"] == io.iterations
    assert relerr(to_host(k), xo) < 1e-10
    g.close()


def test_single_level_hierarchy():
    """One level: the V-cycle is the coarse direct solve, so FGMRES converges in one
    iteration and matches the oracle's solve."""
    from oracle.fgmres import fgmres
    from paper_2202_07381_amd import irkmg

    lv, H = _custom_case(*irkmg.irk_tableau_builtin("radauIIA", 2), 1 / 16, nlev=1)
    A, b, c = irkmg.irk_tableau_builtin("radauIIA", 2)
    g = irkmg.IrkMG(lv, A, b, c, 1 / 16, 1.0)
    S = H.finest
    # a consistent right-hand side (the divergence rows of J k sum to zero per stage)
    F = S.J @ np.random.default_rng(42).standard_normal(S.n)
    k = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    say("[single level] solve")
    info = g.irk_fgmres_solve(to_dev(F), k, rtol=1e-10, maxit=20)
    xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-10, 20, 30, project=S.project_pressure_mean)
    assert info["converged"] and info["iterations"] == io.iterations <= 2
    assert relerr(to_host(k), xo) < coarse_tol(H)
    g.close()

