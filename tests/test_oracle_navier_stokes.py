"""Pins for oracle/navier_stokes.py: the Navier--Stokes stage equations and Newton (Sec. 3.2)."""
import numpy as np
import pytest

from oracle.fem import TaylorHood
from oracle.fgmres import fgmres
from oracle.multigrid import Hierarchy
from oracle.navier_stokes import EWParams, NavierStokesStages, ew_forcing
from oracle.tableau import tableau
from paper_2202_07381_amd import workloads as wl


def _space(dim, n):
    xyz, cells = wl.square_mesh(n) if dim == 2 else wl.cube_mesh(n)
    return TaylorHood(xyz, cells)


def _affine(th, seed):
    """Nodal values of a random affine field x -> alpha + Bm x and (alpha, Bm)."""
    rng = np.random.default_rng(seed)
    alpha = rng.standard_normal(th.dim)
    Bm = rng.standard_normal((th.dim, th.dim))
    return alpha[None, :] + th.node_xyz @ Bm.T, alpha, Bm


def _mass_rows(th, g_nodal):
    """<g, phi_i> for a field g in P2 (nodal values), component-blocked free rows."""
    Mf = th.scalar_mass_full()[th.free]
    return np.concatenate([Mf @ g_nodal[:, c] for c in range(th.dim)])


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
def test_convection_closed_form_affine(dim, n):
    # (a . grad) b = Db (alpha_a + Ba x) is affine, so its P2 interpolant is exact and
    # c(a, b; phi_i) = sum_j M_ij g(x_j); both operand orders (they differ: Ba Db != Db Ba).
    th = _space(dim, n)
    S = NavierStokesStages(th, np.eye(1), 0.1, 1.0)
    a, al_a, Ba = _affine(th, 1)
    b, al_b, Bb = _affine(th, 2)
    ab = (a @ Bb.T)          # (a . grad) b = Bb a
    ba = (b @ Ba.T)          # (b . grad) a = Ba b
    for got, ref in ((S.convection_vector(a, b), _mass_rows(th, ab)),
                     (S.convection_vector(b, a), _mass_rows(th, ba))):
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(_mass_rows(th, ab) - _mass_rows(th, ba)).max() > 1e-3


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
def test_reaction_closed_form_affine(dim, n):
    # (z . grad) U = Bm z for U = alpha + Bm x: R(U) z = [sum_e Bm_ce M z_e]_c
    th = _space(dim, n)
    S = NavierStokesStages(th, np.eye(1), 0.1, 1.0)
    U, _, Bm = _affine(th, 3)
    z = np.random.default_rng(4).standard_normal(dim * th.nfree)
    Mff = th.scalar_mass_full()[th.free][:, th.free]
    zc = [z[c * th.nfree:(c + 1) * th.nfree] for c in range(dim)]
    ref = np.concatenate([sum(Bm[c, e] * (Mff @ zc[e]) for e in range(dim)) for c in range(dim)])
    got = S.reaction_matrix(U) @ z
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_reaction_equals_swapped_convection():
    # R(U) z = c(z, U): two code paths (gradient of U at the points vs of the basis)
    th = _space(2, 4)
    S = NavierStokesStages(th, np.eye(1), 0.1, 1.0)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((th.nnodes, 2))
    z = rng.standard_normal(2 * th.nfree)
    got = S.reaction_matrix(U) @ z
    ref = S.convection_vector(S.free_nodal(z), U)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def _ns(fam="radauIIA", r=3, dim=2, n=4, dt=0.1, nu=0.05):
    th = _space(dim, n)
    A, b, c = tableau(fam, r)
    return NavierStokesStages(th, A, dt, nu), th, b, c


@pytest.mark.parametrize("fam,r,dim,bnd", [("radauIIA", 3, 2, False), ("gauss", 2, 2, True),
                                           ("lobattoIIIC", 2, 3, False)])
def test_jacobian_equals_central_difference(fam, r, dim, bnd):
    # G is quadratic in k, so (G(k + x) - G(k - x)) / 2 = J(k) x up to rounding
    S, th, _, _ = _ns(fam, r, dim, 4 if dim == 2 else 2)
    rng = np.random.default_rng(6)
    k = rng.standard_normal(S.n)
    x = rng.standard_normal(S.n)
    u_n = rng.standard_normal(S.ns)
    F = rng.standard_normal(S.n)
    g = [rng.standard_normal((th.nnodes, dim)) for _ in range(r)] if bnd else None
    fd = 0.5 * (S.residual(F, u_n, k + x, g) - S.residual(F, u_n, k - x, g))
    Jx = S.jacobian(u_n, k, g) @ x
    Jx_mf = S.jacobian_apply(u_n, k, x, g)
    scale = np.abs(fd).max()
    assert np.abs(Jx - fd).max() <= 1e-12 * scale
    assert np.abs(Jx_mf - fd).max() <= 1e-12 * scale


def test_ew_forcing():
    p = EWParams()
    assert ew_forcing(0, 1.0, 1.0, 0.0, p) == p.eta0
    # a fast step: (0.01)^alpha is tiny, the safeguard gamma eta_prev^alpha = 0.3^1.618 = 0.143 > 0.1 holds
    assert ew_forcing(1, 0.01, 1.0, 0.3, p) == pytest.approx(0.3 ** p.alpha)
    # no safeguard when gamma eta_prev^alpha <= 0.1
    assert ew_forcing(2, 1e-4, 1e-2, 0.05, p) == pytest.approx(0.01 ** p.alpha)
    # a stalled step is capped at eta_max
    assert ew_forcing(1, 2.0, 1.0, 0.3, p) == p.eta_max
    # final-step safeguard: never below half the stopping tolerance over the residual
    assert ew_forcing(2, 1e-4, 1e-2, 0.05, p, tau=1e-5) == pytest.approx(0.05)
    assert ew_forcing(2, 1e-4, 1e-2, 0.05, p, tau=1e-9) == pytest.approx(0.01 ** p.alpha)
    assert ew_forcing(2, 1e-4, 1e-2, 0.05, p, tau=1.0) == p.eta_max


def _problem(S, th, seed=7, amp=20.0):
    f = wl.forcing_2d(seed)
    fam = lambda pts, t: amp * f(pts, t)  # noqa: E731
    rng = np.random.default_rng(seed)
    u_n = 0.5 * rng.standard_normal(th.nvel)  # free velocities of the state
    return fam, u_n


def test_newton_solution_satisfies_stage_equations():
    S, th, b, c = _ns("radauIIA", 2, 2, 4, dt=0.1, nu=0.02)
    forcing, u_n = _problem(S, th)
    fn = [th.interpolate(forcing, ci * S.dt) for ci in c]
    F = S.S.rhs(fn, u_n, np.zeros(th.nverts))
    k, info = S.newton(F, u_n, np.zeros(S.n), rtol=1e-13)
    assert info.converged and info.iterations <= 8
    # the stage equations of Sec. 3.2, one stage at a time, with a double loop over a_ij
    St = S.S
    nf = th.nfree
    for i in range(S.r):
        Ui = u_n[:2 * nf].copy()
        for j in range(S.r):
            Ui += S.dt * S.A[i, j] * St.split(k, j)[0]
        Un = S.free_nodal(Ui)
        conv = S.convection_vector(Un, Un)
        kui, _ = St.split(k, i)
        vel = np.concatenate([St.Ms @ kui[cc * nf:(cc + 1) * nf] for cc in range(2)]) + conv
        div = np.zeros(th.nverts)
        for j in range(S.r):
            ku, kp = St.split(k, j)
            vel += S.dt * S.A[i, j] * (np.concatenate([St.Ks @ ku[cc * nf:(cc + 1) * nf] for cc in range(2)]) + St.B @ kp)
            div += S.dt * S.A[i, j] * (St.B.T @ ku)
        Mf = np.concatenate([St.Ms_free_all @ fn[i][:, cc] for cc in range(2)])
        rhs_v = Mf - np.concatenate([St.Ks @ u_n[cc * nf:(cc + 1) * nf] for cc in range(2)])
        assert np.abs(vel - rhs_v).max() <= 1e-10 * np.abs(rhs_v).max()
        assert np.abs(div + St.B.T @ u_n[:2 * nf]).max() <= 1e-10 * np.abs(St.B.T @ u_n[:2 * nf]).max()


def test_newton_converges_quadratically():
    S, th, b, c = _ns("radauIIA", 3, 2, 4, dt=0.1, nu=0.01)
    forcing, u_n = _problem(S, th, seed=8, amp=40.0)
    fn = [th.interpolate(forcing, ci * S.dt) for ci in c]
    F = S.S.rhs(fn, u_n, np.zeros(th.nverts))
    k, info = S.newton(F, u_n, np.zeros(S.n), rtol=1e-14, maxit=30)
    e = np.array(info.norms) / info.norms[0]
    assert info.iterations >= 3  # a genuinely nonlinear problem
    quad = [(e[i], e[i + 1]) for i in range(len(e) - 1) if e[i] < 1e-2 and e[i + 1] > 1e-13]
    assert quad, e
    for a, b_ in quad:
        assert b_ <= 10.0 * a * a, e


def test_newton_reduces_to_stokes_for_small_data():
    # N is quadratic: k(eps F) = eps k_Stokes(F) + O(eps^2)
    S, th, b, c = _ns("gauss", 2, 2, 4, dt=0.1, nu=0.1)
    forcing, _ = _problem(S, th, seed=9, amp=1.0)
    fn = [th.interpolate(forcing, ci * S.dt) for ci in c]
    F = S.S.rhs(fn, np.zeros(th.nvel), np.zeros(th.nverts))
    ks = S.direct_solver()(S.S.J, F, 0.0)[0]
    errs = []
    for eps in (1e-2, 1e-3):
        k, info = S.newton(eps * F, np.zeros(th.nvel), np.zeros(S.n), rtol=1e-13)
        errs.append(np.linalg.norm(k - eps * ks) / np.linalg.norm(eps * ks))
    assert errs[1] < 0.2 * errs[0] and errs[1] < 1e-3


def test_inexact_newton_with_kronecker_multigrid():
    # Newton with FGMRES + the Oseen V-cycle at a frozen wind as preconditioner (a
    # Kronecker operator) and Eisenstat--Walker forcing reaches the exact-Newton solution
    A, b, c = tableau("radauIIA", 2)
    levels = wl.square_hierarchy(2, 3)
    th = TaylorHood(levels[-1].xyz, levels[-1].cells)
    S = NavierStokesStages(th, A, 0.05, 0.02)
    forcing, u_n = _problem(S, th, seed=10, amp=20.0)
    fn = [th.interpolate(forcing, ci * S.dt) for ci in c]
    F = S.S.rhs(fn, u_n, np.zeros(th.nverts))
    k_ex, _ = S.newton(F, u_n, np.zeros(S.n), rtol=1e-12)
    wind_nodal = S.free_nodal(u_n[:th.nvel])

    def wind(pts, t):  # the frozen linearisation point u^n, at the finest nodes
        return wind_nodal
    H = Hierarchy(levels[-1:], A, S.dt, S.S.nu, wind=wind)  # one level: an exact Oseen solve
    Hm = Hierarchy(levels, A, S.dt, S.S.nu)  # Stokes V-cycle

    def mg_solve(H_):
        def solve(Jm, rhs, eta):
            x, inf = fgmres(lambda v: Jm @ v, H_.vcycle, rhs, np.zeros_like(rhs), eta, 200, 30,
                            project=S.S.project_pressure_mean)
            return x, inf.iterations
        return solve
    for H_ in (H, Hm):
        k, info = S.newton(F, u_n, np.zeros(S.n), rtol=1e-10, linear_solve=mg_solve(H_))
        assert info.converged
        assert np.linalg.norm(S.S.project_pressure_mean(k) - S.S.project_pressure_mean(k_ex)) <= \
            1e-7 * np.linalg.norm(k_ex)


def test_mms_inertia_matches_difference_quotients():
    # the manufactured forcing's (u . grad) u against central differences of u
    m = wl.mms_ns_2d(3, 0.1, 2.0)
    x = np.random.default_rng(0).random((7, 2))
    h = 1e-6
    u = m.velocity(x, 0.3)
    ux = (m.velocity(x + [h, 0], 0.3) - m.velocity(x - [h, 0], 0.3)) / (2 * h)
    uy = (m.velocity(x + [0, h], 0.3) - m.velocity(x - [0, h], 0.3)) / (2 * h)
    conv = u[:, :1] * ux + u[:, 1:] * uy
    assert np.abs(conv - m.inertia(x, 0.3)).max() <= 1e-7 * np.abs(conv).max()


def test_newton_time_stepping_temporal_order():
    # RadauIIA(2) is of order 3 for the velocity of the index-2 DAE; on a fixed mesh the
    # error against a run with 1/4 of the smallest step falls by about 2^3 per halving
    th = _space(2, 4)
    A, b, c = tableau("radauIIA", 2)
    mms = wl.mms_ns_2d(3, 0.1, 2.0)
    T = 1.0
    u0 = th.free_velocity(th.interpolate(mms.velocity, 0.0))

    def run(nsteps):
        S = NavierStokesStages(th, A, T / nsteps, 0.1)
        u, p, k = u0.copy(), np.zeros(th.nverts), np.zeros(S.n)
        for n in range(nsteps):
            u, p, k, info = S.step(b, c, mms, n * S.dt, u, p, k, rtol=1e-10, atol=1e-13)
            assert info.converged
        return u
    ref = run(64)
    errs = [np.linalg.norm(run(m) - ref) for m in (4, 8, 16)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.6), (errs, rates)


def test_newton_line_search():
    # a step too large for full Newton steps from k = 0: the backtracking line search
    # converges (Armijo decrease every step, full steps once close), full steps do not
    S, th, b, c = _ns("radauIIA", 3, 2, 4, dt=0.2, nu=0.02)
    forcing, u_n = _problem(S, th, seed=8, amp=30.0)
    fn = [th.interpolate(forcing, ci * S.dt) for ci in c]
    F = S.S.rhs(fn, u_n, np.zeros(th.nverts))
    _, full = S.newton(F, u_n, np.zeros(S.n), rtol=1e-12, maxit=30)
    assert not full.converged
    k, ls = S.newton(F, u_n, np.zeros(S.n), rtol=1e-12, maxit=30, linesearch=True)
    assert ls.converged and ls.iterations <= 15
    assert min(ls.lambdas) < 1.0 and ls.lambdas[-1] == 1.0
    n = np.array(ls.norms)
    lam = np.array(ls.lambdas)
    assert np.all(n[1:] <= (1 - 1e-4 * lam) * n[:-1])
    # on an easy problem every step is a full step: the same iterates as plain Newton
    S2, th2, b2, c2 = _ns("radauIIA", 2, 2, 4, dt=0.1, nu=0.02)
    forcing2, u2 = _problem(S2, th2)
    F2 = S2.S.rhs([th2.interpolate(forcing2, ci * S2.dt) for ci in c2], u2, np.zeros(th2.nverts))
    k1, i1 = S2.newton(F2, u2, np.zeros(S2.n), rtol=1e-13)
    k2, i2 = S2.newton(F2, u2, np.zeros(S2.n), rtol=1e-13, linesearch=True)
    assert i2.lambdas == [1.0] * i2.iterations and np.array_equal(k1, k2)


# ------------------------------------------------ the Newton Jacobian V-cycle
def test_injection_reproduces_coarse_interpolant():
    from oracle.navier_stokes import inject_nodal

    for dim, levels in ((2, wl.square_hierarchy(2, 3)), (3, wl.cube_hierarchy(1, 3))):
        ths = [TaylorHood(m.xyz, m.cells) for m in levels]

        def f(x, t=0.0):  # a quadratic field: its P2 interpolants are exact on every level
            return np.stack([x[:, 0] ** 2 - x[:, 1] + 0.5] + [x[:, 0] * x[:, c] for c in range(1, dim)], axis=1)
        for lc in range(len(ths) - 1):
            got = inject_nodal(ths[lc + 1], ths[lc], ths[lc + 1].interpolate(f))
            assert np.abs(got - ths[lc].interpolate(f)).max() <= 1e-15


def test_newton_cycle_reduces_to_stokes_and_oseen():
    """At U = 0 the Newton Jacobian is the Stokes stage operator, and at a constant U
    (no reaction term, grad U = 0) the Oseen operator with wind U, on every level; the
    cycles then agree with the Kronecker ones to rounding."""
    from oracle.navier_stokes import newton_hierarchy

    A, _, _ = tableau("radauIIA", 2)
    levels = wl.square_hierarchy(2, 3)
    th = TaylorHood(levels[-1].xyz, levels[-1].cells)
    dt, nu = 0.05, 0.02
    rv = np.random.default_rng(3).standard_normal(2 * (2 * th.nfree + th.nverts))
    w = np.array([0.7, -0.4])
    for U, wind in (([np.zeros((th.nnodes, 2))] * 2, None),
                    ([np.tile(w, (th.nnodes, 1))] * 2, lambda x, t=0.0: np.tile(w, (x.shape[0], 1)))):
        Hn = newton_hierarchy(levels, A, dt, nu, U)
        Hk = Hierarchy(levels, A, dt, nu, wind=wind)
        for lev in range(3):
            assert abs(Hn.ops[lev] - Hk.ops[lev]).max() <= 1e-14 * abs(Hk.ops[lev]).max()
        z1, z2 = Hn.vcycle(rv), Hk.vcycle(rv)
        assert np.abs(z1 - z2).max() <= 1e-12 * np.abs(z2).max()


def test_newton_cycle_equals_textbook_propagator():
    """The Newton Jacobian cycle at stage velocities with a reaction term satisfies the
    error-propagator identity of the multigrid pins for its own level operators."""
    from test_oracle_vcycle_propagator import TOL, _check, _Propagator

    from oracle.navier_stokes import newton_hierarchy

    A, _, _ = tableau("radauIIA", 2)
    levels = wl.square_hierarchy(4, 2)
    th = TaylorHood(levels[-1].xyz, levels[-1].cells)
    rng = np.random.default_rng(5)
    U = [3.0 * rng.standard_normal((th.nnodes, 2)) for _ in range(2)]
    H = newton_hierarchy(levels, A, 0.05, 0.02, U)
    _check(H, _Propagator(H, 0.5, True), 24, 13, TOL)


def test_newton_cycle_preconditions_newton():
    """Inexact Newton with FGMRES preconditioned by the Newton Jacobian V-cycle, rebuilt
    at every iterate, reaches the exact-Newton solution; at this Reynolds number it needs
    fewer linear iterations than with the Stokes V-cycle."""
    from oracle.navier_stokes import newton_hierarchy

    A, b, c = tableau("radauIIA", 2)
    levels = wl.square_hierarchy(2, 3)
    th = TaylorHood(levels[-1].xyz, levels[-1].cells)
    S = NavierStokesStages(th, A, 0.05, 0.005)
    forcing, u_n = _problem(S, th, seed=10, amp=20.0)
    fn = [th.interpolate(forcing, ci * S.dt) for ci in c]
    F = S.S.rhs(fn, u_n, np.zeros(th.nverts))
    k_ex, _ = S.newton(F, u_n, np.zeros(S.n), rtol=1e-12)

    def krylov(Jm, rhs, eta, H_):
        x, inf = fgmres(lambda v: Jm @ v, H_.vcycle, rhs, np.zeros_like(rhs), eta, 300, 30,
                        project=S.S.project_pressure_mean)
        return x, inf.iterations

    Hs = Hierarchy(levels, A, S.dt, S.S.nu)
    k1, i1 = S.newton(F, u_n, np.zeros(S.n), rtol=1e-10, linear_solve=lambda J, r, e: krylov(J, r, e, Hs))
    k2, i2 = S.newton(F, u_n, np.zeros(S.n), rtol=1e-10,
                      linear_solve_at=lambda J, r, e, U: krylov(J, r, e, newton_hierarchy(levels, A, S.dt, S.S.nu, U)))
    for k, info in ((k1, i1), (k2, i2)):
        assert info.converged
        assert np.linalg.norm(S.S.project_pressure_mean(k) - S.S.project_pressure_mean(k_ex)) <= \
            1e-7 * np.linalg.norm(k_ex)
    assert sum(i2.linear_its) < sum(i1.linear_its)
