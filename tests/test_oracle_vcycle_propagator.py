"""Pins of the V-cycle's shape (Sec. 4.1) and of the relaxation inside it (Sec. 4.2, 5.1).

The oracle's V-cycle is a recursion over vectors: sweeps from a zero guess, the
residual, restriction, the coarse cycle, prolongation-and-add, sweeps.  Here the same
map is written the textbook way, as an error propagator of dense matrices built from
the level operators J_l, the transfers P_l and the patch index sets alone:

    G_l = I - omega W S J_l,      S = sum_v R_v^T (R_v J_l R_v^T)^{-1} R_v,
    E_l = G_l^post (I - P_l B_{l-1} P_l^T J_l) G_l^pre,
    B_l y = (I - E_l) J_l^+ y     (y in the range of J_l),     B_0 = J_0^+,

with J^+ the Moore--Penrose pseudo-inverse (any solution of the singular but
consistent coarse problems serves: the pressure constants that separate them are
fixed points of every G_l, are annihilated by I - E_l and are removed by the final
pressure-mean projection Pi).  Then V J x = Pi (I - E_L) x for every x, which this
file checks on random probe blocks.  A wrong pre/post count, omega or W on the wrong
side of S, a restriction of b instead of the residual b - J x, a damped coarse
correction or a dropped sweep each change E_L and fail it.

For Chebyshev relaxation (Sec. 5.1) the relaxation's propagator is the polynomial
T_m((theta - S J)/delta) / T_m(theta/delta), evaluated here by the three-term
recurrence of T_m on the matrix argument and the closed form of T_m(theta/delta),
not by the oracle's semi-iteration.

Tolerance: the probes pass through pseudo-inverse solves whose forward error is about
cond * eps, with the level operators' condition numbers on the complement of their
null space at most 1.3e6 in these cases (so cond * eps <= 3e-10).  The bar is 2e-9
relative; each misreading listed above moves the result by more than 1e-4.
"""
import numpy as np
import pytest

from oracle.multigrid import Hierarchy
from oracle.tableau import tableau
from oracle.vanka import multiplicity, patch_dofs
from paper_2202_07381_amd import workloads as wl


TOL = 2e-9


def _dense_S(H, lev, weighted):
    """W sum_v R_v^T A_v^{-1} R_v as a dense matrix, from the patch index sets and J."""
    J = H.ops[lev].toarray()
    sp_ = H.spaces[lev]
    pats = sp_.patches(H.r) if hasattr(sp_, "patches") else patch_dofs(sp_, H.r)
    n = J.shape[0]
    S = np.zeros((n, n))
    for p in pats:
        S[np.ix_(p, p)] += np.linalg.inv(J[np.ix_(p, p)])
    W = 1.0 / multiplicity(pats, n) if weighted else np.ones(n)
    return W[:, None] * S


class _Propagator:
    """E_l and B_l of the module docstring, applied to blocks of column vectors."""

    def __init__(self, H, omega, weighted, relax="sweep", interval=(2.0, 8.0)):
        self.H = H
        self.omega, self.relax, self.interval = omega, relax, interval
        self.J = [J.toarray() for J in H.ops]
        self.Jpinv = [np.linalg.pinv(J) for J in self.J]
        self.S = [None] + [_dense_S(H, lev, weighted) for lev in range(1, len(H.systems))]
        self.P = [None] + [P.toarray() for P in H.P[1:]]

    def relax_prop(self, lev, steps, Z):
        """Error propagator of `steps` relaxation steps applied to Z."""
        SJ = self.S[lev] @ self.J[lev]
        if self.relax == "sweep":
            for _ in range(steps):
                Z = Z - self.omega * (SJ @ Z)
            return Z
        lo, hi = self.interval
        theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
        Y = lambda X: (theta * X - SJ @ X) / delta  # noqa: E731
        t_prev, t = Z, Y(Z)
        if steps == 0:
            return Z
        for _ in range(steps - 1):
            t_prev, t = t, 2.0 * Y(t) - t_prev
        return t / np.cosh(steps * np.arccosh(theta / delta))

    def E(self, lev, Z):
        H = self.H
        Z = self.relax_prop(lev, H.pre, Z)
        Z = Z - self.P[lev] @ self.B(lev - 1, self.P[lev].T @ (self.J[lev] @ Z))
        return self.relax_prop(lev, H.post, Z)

    def B(self, lev, Y):
        X = self.Jpinv[lev] @ Y
        if lev == 0:
            return X
        return X - self.E(lev, X)


def _project(H, X):
    return np.column_stack([H.finest.project_pressure_mean(X[:, j]) for j in range(X.shape[1])])


def _check(H, prop, nprobe, seed, tol):
    S = H.finest
    X = np.random.default_rng(seed).standard_normal((S.n, nprobe))
    JX = H.ops[-1] @ X
    got = np.column_stack([H.vcycle(JX[:, j]) for j in range(nprobe)])
    expect = _project(H, X - prop.E(len(H.systems) - 1, X))
    err = np.abs(got - expect).max() / np.abs(expect).max()
    assert err < tol, err
    return got, expect


CASES = [
    # (n_coarse, nlevels, family, r, dt, nu, wind, omega, weighted, pre, post)
    pytest.param(4, 2, "radauIIA", 2, 1 / 16, 1.0, False, 0.5, True, 2, 2, id="8x8-two-level-radau2"),
    pytest.param(4, 2, "radauIIA", 3, 1e-2, 1.0, False, 0.7, True, 1, 3, id="8x8-two-level-radau3-pre1-post3"),
    pytest.param(4, 2, "gauss", 2, 5e-3, 0.05, True, 0.5, True, 3, 1, id="8x8-two-level-oseen-pre3-post1"),
    pytest.param(4, 2, "radauIIA", 2, 1 / 16, 1.0, False, 0.3, False, 2, 2, id="8x8-two-level-unweighted"),
    pytest.param(4, 3, "radauIIA", 2, 1 / 16, 1.0, False, 0.5, True, 2, 2, id="16x16-three-level-radau2"),
]


@pytest.mark.parametrize("nc,nl,fam,r,dt,nu,wind,omega,weighted,pre,post", CASES)
def test_vcycle_equals_textbook_propagator(nc, nl, fam, r, dt, nu, wind, omega, weighted, pre, post):
    """V J = Pi (I - E_L) with E_L the product of the relaxation and coarse-correction
    propagators (Sec. 4.1 cycle, Sec. 4.2 additive sweep)."""
    A, _, _ = tableau(fam, r)
    kw = dict(wind=wl.wind_2d(3, 16)) if wind else {}
    H = Hierarchy(wl.square_hierarchy(nc, nl), A, dt, nu, omega=omega, weighted=weighted, pre=pre, post=post, **kw)
    prop = _Propagator(H, omega, weighted)
    _check(H, prop, 24, 11, TOL)


def test_propagator_pin_detects_shape_changes():
    """The comparison separates the cycle from plausible misreadings: swapped pre/post
    counts, a different omega, W on the right of S and an undamped coarse correction
    computed from b instead of the residual all give a different map."""
    A, _, _ = tableau("radauIIA", 2)
    H = Hierarchy(wl.square_hierarchy(4, 2), A, 1 / 16, 1.0, omega=0.5, weighted=True, pre=1, post=3)
    good = _Propagator(H, 0.5, True)
    got, expect = _check(H, good, 8, 12, TOL)
    scale = np.abs(expect).max()
    X = np.random.default_rng(12).standard_normal((H.finest.n, 8))

    def err_of(prop):
        return np.abs(got - _project(H, X - prop.E(1, X))).max() / scale

    swapped = _Propagator(H, 0.5, True)
    swapped.H = type("H", (), {"pre": 3, "post": 1})()
    assert err_of(swapped) > 1e-4
    assert err_of(_Propagator(H, 0.6, True)) > 1e-4
    right_W = _Propagator(H, 0.5, True)
    pats = patch_dofs(H.spaces[1], H.r)
    W = 1.0 / multiplicity(pats, H.finest.n)
    right_W.S[1] = (right_W.S[1] / W[:, None]) * W[None, :]
    assert err_of(right_W) > 1e-4
    no_residual = _Propagator(H, 0.5, True)

    def E_b(lev, Z, p=no_residual):
        Z1 = p.relax_prop(lev, 1, Z)
        # coarse correction from the restricted b = J x* instead of the residual
        Z1 = Z1 - p.P[lev] @ p.B(lev - 1, p.P[lev].T @ (p.J[lev] @ X))
        return p.relax_prop(lev, 3, Z1)

    no_residual.E = E_b
    assert err_of(no_residual) > 1e-4


@pytest.mark.parametrize("nl,pre,post", [(2, 2, 2), (2, 1, 3), (3, 2, 2)])
def test_chebyshev_vcycle_equals_polynomial_propagator(nl, pre, post):
    """With Chebyshev relaxation on [2, 8] (Sec. 5.1) each relaxation contributes
    T_m((theta - S J)/delta) / T_m(theta/delta) to the cycle's error propagator."""
    A, _, _ = tableau("radauIIA", 2)
    H = Hierarchy(wl.square_hierarchy(4, nl), A, 1 / 32, 1.0, weighted=False, smoother="chebyshev",
                  pre=pre, post=post)
    prop = _Propagator(H, 1.0, False, relax="chebyshev", interval=(2.0, 8.0))
    _check(H, prop, 16, 13, TOL)


def test_one_sweep_is_the_weighted_additive_step():
    """One damped sweep maps k to k + omega W S (F - J k): with F = J x* the new error is
    G (x* - k) (Sec. 4.2; the partition-of-unity weight W of the damping reading)."""
    A, _, _ = tableau("radauIIA", 3)
    H = Hierarchy(wl.square_hierarchy(4, 2), A, 1e-2, 1.0, omega=0.5, weighted=True)
    S = H.finest
    sm = H.smoothers[1]
    rng = np.random.default_rng(14)
    Sd = _dense_S(H, 1, True)
    J = S.J.toarray()
    for _ in range(3):
        xs, k = rng.standard_normal(S.n), rng.standard_normal(S.n)
        new = sm.sweep(J @ xs, k, S.J)
        expect_err = (xs - k) - 0.5 * (Sd @ (J @ (xs - k)))
        assert np.abs((xs - new) - expect_err).max() < 1e-11 * np.abs(expect_err).max()
    # the exact solution is a fixed point
    xs = rng.standard_normal(S.n)
    assert np.abs(sm.sweep(J @ xs, xs, S.J) - xs).max() < 1e-12 * np.abs(xs).max()


@pytest.mark.parametrize("nc,nl", [(4, 2), (2, 3)])
def test_two_grid_and_vcycle_contraction(nc, nl):
    """The spectral radius of E_L on the complement of the pressure null space is well
    below one (about 0.3, so FGMRES needs a dozen iterations for 1e-8), for the two-grid cycle (4x4 -> 8x8) and the three-level V-cycle
    (2x2 -> 4x4 -> 8x8) alike (Sec. 4.1: a V-cycle contracts about as well as the
    two-grid cycle it approximates)."""
    A, _, _ = tableau("radauIIA", 2)
    H = Hierarchy(wl.square_hierarchy(nc, nl), A, 1 / 16, 1.0)
    prop = _Propagator(H, 0.5, True)
    n = H.finest.n
    E = prop.E(nl - 1, np.eye(n))
    # restrict to the quotient by the null space: Pi E Pi has the same nonzero spectrum
    Pi = _project(H, np.eye(n))
    rho = np.abs(np.linalg.eigvals(Pi @ E @ Pi)).max()
    assert rho < 0.4, rho  # 0.31 (two-grid) and 0.34 (three-level) measured
