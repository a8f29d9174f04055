"""The V-cycle of the Newton Jacobian (Sec. 3.2) on the GPU against the oracle's
(oracle.navier_stokes.newton_hierarchy), through the C ABI.

irk_ns_newton_preconditioner rediscretises the stage Jacobian, block (i, j) =
delta_ij M + dt a_ij (K + N'(U_i)), on every level at the stage velocities of (state, k)
injected to the coarser levels, and switches the handle's cycle to it.  Bars as for the
Stokes and Oseen cycles (test_gpu_parity.py): level operators 1e-12 relative to the
largest entry (sums in another order), one sweep 1e-11, the coarse solve 4 cond_S eps
of the pinned coarse Newton Jacobian, the V-cycle 1e-11.  Newton with this
preconditioner rebuilt at every iterate (irk_newton_opts.precond = 1) against the
oracle's Newton with FGMRES and newton_hierarchy: the same Newton and FGMRES
iteration counts at every step, solutions 1e-8 (as for the other Newton tests)."""
import numpy as np
import pytest

from gpu_cases import gpu_of, levels_of, relerr, say, to_dev, to_host
from test_gpu_navier_stokes import _gpu_rhs, _inputs, _oracle_rhs, _stokes
from test_gpu_parity import VCYCLE_TOL, coarse_tol

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _newton_hierarchy(case, ns, S, state, k, gst):
    from oracle.navier_stokes import newton_hierarchy

    U = ns.stage_values(state[:S.th.nvel], k, gst)
    return newton_hierarchy(levels_of(case), S.A, S.dt, S.nu, U)


@pytest.mark.parametrize("case,bnd", [("c1", False), ("lob3", True), ("oseen", False), ("3d2", False)])
def test_newton_vcycle_matches_oracle(case, bnd):
    from paper_2202_07381_amd import irkmg

    g = gpu_of(case)
    ns, S, state, fst, gn, gst = _inputs(case, 31, bnd, 4.0, 1.0)
    k = 0.5 * np.random.default_rng(32).standard_normal(S.n)
    H = _newton_hierarchy(case, ns, S, state, k, gst)
    rv = np.random.default_rng(33).standard_normal(S.n)
    z0 = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    g.irk_mg_vcycle(to_dev(rv), z0)
    before = to_host(z0)
    say(f"[newton-vcycle] case={case} bnd={bnd}")
    g.irk_ns_newton_preconditioner(to_dev(state), to_dev(k), g_stages=None if gst is None else to_dev(gst.reshape(-1)))
    try:
        rng = np.random.default_rng(34)
        for lev in range(g.nlevels):
            J = H.ops[lev]
            x = rng.standard_normal(J.shape[0])
            y = torch.zeros(J.shape[0], dtype=torch.float64, device="cuda")
            g.irk_level_apply(lev, to_dev(x), y)
            assert relerr(to_host(y), J @ x) < 1e-12, lev
            if lev >= 1:
                F, k0 = rng.standard_normal(J.shape[0]), rng.standard_normal(J.shape[0])
                kk = to_dev(k0)
                g.irk_level_sweep(lev, to_dev(F), kk)
                assert relerr(to_host(kk), H.smoothers[lev].sweep(F, k0, J, False)) < 1e-11, lev
        J0 = H.ops[0]
        b = J0 @ rng.standard_normal(J0.shape[0])
        x0 = torch.zeros(J0.shape[0], dtype=torch.float64, device="cuda")
        g.irk_coarse_solve(to_dev(b), x0)
        err_c = relerr(to_host(x0), H.coarse_solve(b))
        z = torch.zeros(S.n, dtype=torch.float64, device="cuda")
        g.irk_mg_vcycle(to_dev(rv), z)
        err = relerr(to_host(z), H.vcycle(rv))
        say(f"[newton-vcycle] case={case} coarse err={err_c:.2e} tol={coarse_tol(H):.2e} vcycle err={err:.2e}")
        assert err_c < coarse_tol(H) and err < VCYCLE_TOL
        with pytest.raises(irkmg.IrkError) as e:
            g.irk_mg_vcycle_transpose(to_dev(rv), z)
        assert e.value.status == irkmg.IRK_EINVAL
    finally:
        g.irk_ns_newton_preconditioner(enable=False)
    # switched back: the handle's own cycle, bitwise as before
    g.irk_mg_vcycle(to_dev(rv), z0)
    assert np.array_equal(to_host(z0), before)


@pytest.mark.parametrize("case", ["c1", "3d2"])
def test_newton_with_newton_vcycle_matches_oracle(case):
    from oracle.fgmres import fgmres
    from oracle.navier_stokes import newton_hierarchy

    g = gpu_of(case)
    amp = {"c1": 8.0, "3d2": 4.0}[case]
    ns, S, state, fst, gn, gst = _inputs(case, 41, False, amp, amp)
    F = _gpu_rhs(g, fst, state)
    k = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    say(f"[newton-precond] case={case} GPU precond=1")
    info = g.irk_ns_newton_solve(F, to_dev(state), k, rtol=1e-10, precond=1)
    k0 = torch.zeros_like(k)
    info0 = g.irk_ns_newton_solve(F, to_dev(state), k0, rtol=1e-10, precond=0)
    Fo = _oracle_rhs(_stokes(ns), fst, state)
    levels = levels_of(case)

    def solve_at(Jm, rhs, eta, U):
        Hn = newton_hierarchy(levels, S.A, S.dt, S.nu, U)
        x, inf = fgmres(lambda v: Jm @ v, Hn.vcycle, rhs, np.zeros_like(rhs), eta, 200, 30,
                        project=S.project_pressure_mean)
        return x, inf.iterations

    say(f"[newton-precond] case={case} oracle")
    ko, oinfo = ns.newton(Fo, state[:S.th.nvel], np.zeros(S.n), rtol=1e-10, linear_solve_at=solve_at)
    say(f"[newton-precond] case={case} newton its gpu={info['iterations']} oracle={oinfo.iterations}; "
        f"linear its gpu={info['linear_its'].tolist()} oracle={oinfo.linear_its}; "
        f"with the Kronecker cycle {info0['linear_its'].tolist()}")
    assert info["converged"] and oinfo.converged
    assert info["iterations"] == oinfo.iterations
    assert info["linear_its"].tolist() == list(oinfo.linear_its)
    pm = S.project_pressure_mean
    assert relerr(pm(to_host(k)), pm(ko)) < 1e-8
    assert relerr(pm(to_host(k)), pm(to_host(k0))) < 1e-8


def test_newton_vcycle_fewer_linear_iterations_at_low_viscosity():
    """At nu = 0.005 (the oracle pin's problem: forcing of amplitude 20, a rough state)
    the Jacobian's own cycle needs fewer FGMRES iterations over the Newton solve than the
    Stokes cycle of the same handle, and both reach the same solution."""
    from oracle.fem import TaylorHood
    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    lv = wl.square_hierarchy(2, 3)
    A, b, c = irkmg.irk_tableau_builtin("radauIIA", 2)
    dt, nu = 0.05, 0.005
    g = irkmg.IrkMG(lv, A, b, c, dt, nu)
    th = TaylorHood(lv[-1].xyz, lv[-1].cells)
    f = wl.forcing_2d(10)
    u_n = 0.5 * np.random.default_rng(10).standard_normal(th.nvel)
    state = to_dev(np.concatenate([u_n, np.zeros(th.nverts)]))
    fn = np.stack([th.interpolate(lambda x, t: 20.0 * f(x, t), ci * dt) for ci in c])
    F = torch.zeros(g.irk_mg_ndofs(), dtype=torch.float64, device="cuda")
    g.irk_rhs(to_dev(fn.ravel()), state, F)
    its, sols = {}, {}
    for pc in (0, 1):
        k = torch.zeros_like(F)
        info = g.irk_ns_newton_solve(F, state, k, rtol=1e-10, precond=pc)
        say(f"[newton-precond] nu=0.005 precond={pc} newton its={info['iterations']} "
            f"linear its={info['linear_its'].tolist()}")
        assert info["converged"]
        its[pc] = info["linear_iterations"]
        sols[pc] = to_host(k)
    assert its[1] < its[0]
    assert relerr(sols[1], sols[0]) < 1e-8
    g.close()
