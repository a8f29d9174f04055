"""Navier--Stokes IRK stage equations and Newton's method on them (Sec. 3.2).

TEST INFRASTRUCTURE ONLY (oracle).

Inertia enters the weak form as <u . grad u, v>; write the trilinear form
    c(a, b; v) = int ((a . grad) b) . v
and N(U) for the vector of c(U, U; phi) over the free velocity test functions.  With
the stage values U_i = u^n + dt sum_j a_ij k_j^u (the stage velocity of Sec. 2, eq.
"general RK"; at boundary nodes the prescribed data G_i = g(t^n + c_i dt), zero by
default) the stage equations of Sec. 3.2 are, for every stage i,

    M k_i^u + N(U_i) + dt sum_j a_ij (K k_j^u + B k_j^p) = M f_i - K u^n - B p^n,
                       dt sum_j a_ij B^T k_j^u           = -B^T u^n,

i.e. G(k) = J_S k - F + [N(U_i); 0]_i = 0 with J_S, F the Stokes stage operator and
right-hand side of StageSystem (no wind; boundary data through rhs_dirichlet).

Jacobian.  N is quadratic, so its derivative at U along z is c(z, U) + c(U, z):
N'(U) = C(U) + R(U) with C(U) the convection matrix of stage.py (wind U) and
R(U)_{(a,c),(b,e)} = int phi_a phi_b d_e U_c (the reaction term).  Block (i, j) of the
stage Jacobian is delta_ij M + dt a_ij (K + N'(U_i)) plus the B, B^T blocks; since
N'(U_i) depends on the stage, this is not a Kronecker product.

Newton (Sec. 3.2): k <- k + delta with J(k) delta = -G(k), started from the previous
step's stages k^{n-1} (zero at the first step).  Inexact solves stop at
||G + J delta|| <= eta_l ||G|| with the Eisenstat--Walker forcing terms of Sec. 3.2.
The paper names the criterion but not its variant or constants; the reading taken:
Eisenstat and Walker's "choice 2", eta_l = gamma (||G_l|| / ||G_{l-1}||)^alpha, kept at
least gamma eta_{l-1}^alpha when that exceeds a threshold (their safeguard against a
too-fast decrease of eta after a slow step), capped at eta_max, with eta_0 = 0.3,
eta_max = 0.9, gamma = 1, alpha = (1 + sqrt 5)/2, threshold 0.1; and, since a forcing
term far below what the Newton stopping test still needs only makes the last linear
solve grind against rounding, never below 0.5 tau / ||G_l|| (the final-step safeguard of
Kelley's textbook treatment of inexact Newton), tau = max(atol, rtol ||G(k^0)||), the
tolerance at which Newton stops: ||G|| <= tau.

Optional globalisation (not in the paper, off by default): a backtracking line search
on ||G||, k <- k + lam delta with the first lam in 1, 1/2, 1/4, ... (at most ls_maxit
halvings) for which ||G(k + lam delta)|| <= (1 - ls_alpha lam) ||G(k)|| (Armijo's
sufficient decrease, ls_alpha = 1e-4); no such lam ends the iteration unconverged.

Newton Jacobian V-cycle (newton_hierarchy): every level rediscretises the stage
Jacobian at the stage velocities injected from the finest level.  Pinned: injection of
a P2 interpolant equals the coarse interpolant; at U = 0 the cycle equals the Stokes
cycle and at a constant U (no reaction term) the Oseen cycle with that wind, to
rounding; one Vanka sweep with a single patch solves the patch system exactly; and the
cycle satisfies the error-propagator identity of the multigrid module for its own
operators.

Pinned by tests/test_oracle_navier_stokes.py against: closed forms of c(a, b) and of
R(U) z for affine fields (their products are P1, so the integrals equal mass-matrix
products of nodal values); the identity R(U) z = c(z, U) between the two code paths;
central differences of G, which are exact for a quadratic map, against the assembled
Jacobian; the stage equations written out stage by stage with a double loop over a_ij
at the Newton solution; quadratic convergence of the exact-solve iteration; temporal
order 3 of RadauIIA(2) stepping on a manufactured Navier--Stokes solution; and, for the
line search, convergence where full steps diverge, the decrease condition at every
accepted step, and bitwise equality with plain Newton when every step is full.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fem import TaylorHood, p2_basis, simplex_quadrature
from .stage import StageSystem


@dataclass
class EWParams:
    """Eisenstat--Walker choice-2 constants (reading in the module docstring)."""
    eta0: float = 0.3
    eta_max: float = 0.9
    gamma: float = 1.0
    alpha: float = 0.5 * (1.0 + 5.0 ** 0.5)
    threshold: float = 0.1


def ew_forcing(it: int, norm: float, norm_prev: float, eta_prev: float, p: EWParams, tau: float = 0.0) -> float:
    """Forcing term eta_it for the linear solve of Newton step `it` (it = 0: eta0);
    tau: the Newton stopping tolerance on ||G|| (0: no final-step safeguard)."""
    if it == 0:
        eta = min(p.eta0, p.eta_max)
    else:
        eta = p.gamma * (norm / norm_prev) ** p.alpha
        guard = p.gamma * eta_prev ** p.alpha
        if guard > p.threshold:
            eta = max(eta, guard)
        eta = min(eta, p.eta_max)
    if tau > 0.0:
        eta = min(p.eta_max, max(eta, 0.5 * tau / norm))
    return eta


@dataclass
class NewtonInfo:
    iterations: int = 0
    converged: bool = False
    norms: list = field(default_factory=list)   # ||G|| before each step and at exit
    etas: list = field(default_factory=list)    # forcing term of each step
    linear_its: list = field(default_factory=list)
    lambdas: list = field(default_factory=list)  # step length of each step (line search)


class NavierStokesStages:
    """The nonlinear stage system of one mesh level for fixed (tableau, dt, nu)."""

    def __init__(self, th: TaylorHood, A: np.ndarray, dt: float, nu: float):
        self.th = th
        self.S = StageSystem(th, A, dt, nu)  # the Stokes part J_S (no wind)
        self.A = self.S.A
        self.r = self.S.r
        self.dt = self.S.dt
        self.ns = self.S.ns
        self.n = self.S.n

    # ------------------------------------------------------------ stage values
    def stage_values(self, u_n: np.ndarray, k: np.ndarray, g_stages=None) -> list[np.ndarray]:
        """U_i as nodal arrays (nnodes, dim): free nodes from u^n + dt sum_j a_ij k_j^u,
        boundary nodes from g_stages[i] (zero when None)."""
        th = self.th
        d, nf = th.dim, th.nfree
        out = []
        for i in range(self.r):
            Ui = np.array(u_n[: d * nf], dtype=np.float64)
            for j in range(self.r):
                Ui = Ui + self.dt * self.A[i, j] * self.S.split(k, j)[0]
            nod = np.zeros((th.nnodes, d))
            if g_stages is not None:
                nod[th.boundary] = np.asarray(g_stages[i])[th.boundary]
            for c in range(d):
                nod[th.free, c] = Ui[c * nf:(c + 1) * nf]
            out.append(nod)
        return out

    def free_nodal(self, v: np.ndarray) -> np.ndarray:
        """Nodal array (nnodes, dim) of a component-blocked free vector (boundary zero)."""
        th = self.th
        nod = np.zeros((th.nnodes, th.dim))
        for c in range(th.dim):
            nod[th.free, c] = v[c * th.nfree:(c + 1) * th.nfree]
        return nod

    # ---------------------------------------------------------- trilinear form
    def convection_vector(self, a_nodal: np.ndarray, b_nodal: np.ndarray) -> np.ndarray:
        """c(a, b; phi) for every free velocity test function, component-blocked:
        the convection matrix with wind a applied to every component of b (all nodes)."""
        th = self.th
        C = th._assemble_nodes(th.element_convection(a_nodal))[th.free]  # free rows x all nodes
        return np.concatenate([C @ b_nodal[:, c] for c in range(th.dim)])

    def element_reaction(self, U_nodal: np.ndarray) -> np.ndarray:
        """E[cell, a, b, c, e] = int phi_a phi_b d_e U_c (U the P2 interpolant)."""
        th = self.th
        xi, w = simplex_quadrature(th.dim)
        val, gref = p2_basis(th.dim, xi)
        g = np.einsum("cij,qnj->cqni", th.jinvT, gref)  # physical basis gradients
        gU = np.einsum("cqne,cnk->cqke", g, U_nodal[th.cell_nodes])  # d_e U_k at each point
        return np.einsum("q,qa,qb,cqke,c->cabke", w, val, val, gU, th.detj, optimize=True)

    def reaction_matrix(self, U_nodal: np.ndarray) -> sp.csr_matrix:
        """R(U) on component-blocked free velocities."""
        th = self.th
        d = th.dim
        E = self.element_reaction(U_nodal)
        blocks = [[None] * d for _ in range(d)]
        for c in range(d):
            for e in range(d):
                full = th._assemble_nodes(E[:, :, :, c, e])
                blocks[c][e] = full[th.free][:, th.free]
        return sp.bmat(blocks).tocsr()

    def nprime(self, U_nodal: np.ndarray) -> sp.csr_matrix:
        """N'(U) = C(U) + R(U) on component-blocked free velocities."""
        th = self.th
        C = th._assemble_nodes(th.element_convection(U_nodal))[th.free][:, th.free]
        return (sp.kron(sp.identity(th.dim), C) + self.reaction_matrix(U_nodal)).tocsr()

    # ------------------------------------------------------- residual, Jacobian
    def residual(self, F: np.ndarray, u_n: np.ndarray, k: np.ndarray, g_stages=None) -> np.ndarray:
        """G(k) = J_S k - F + [N(U_i); 0]_i."""
        G = self.S.J @ k - F
        nvel = self.th.nvel
        for i, Ui in enumerate(self.stage_values(u_n, k, g_stages)):
            G[i * self.ns:i * self.ns + nvel] += self.convection_vector(Ui, Ui)
        return G

    def jacobian(self, u_n: np.ndarray, k: np.ndarray, g_stages=None) -> sp.csr_matrix:
        """dG/dk at k: J_S plus dt a_ij N'(U_i) in the velocity block (i, j)."""
        return self.jacobian_at(self.stage_values(u_n, k, g_stages))

    def jacobian_at(self, U: list) -> sp.csr_matrix:
        """The stage Jacobian for given nodal stage velocities U_i (nnodes, dim):
        block (i, j) = delta_ij M + dt a_ij (K + N'(U_i)) with the B, B^T blocks."""
        nvel = self.th.nvel
        blocks = [[None] * self.r for _ in range(self.r)]
        for i in range(self.r):
            Np = self.nprime(U[i])
            for j in range(self.r):
                if self.A[i, j] != 0.0:
                    blocks[i][j] = sp.block_diag([self.dt * self.A[i, j] * Np, sp.csr_matrix((self.ns - nvel,) * 2)])
                else:
                    blocks[i][j] = sp.csr_matrix((self.ns, self.ns))
        return (self.S.J + sp.bmat(blocks)).tocsr()

    def jacobian_apply(self, u_n: np.ndarray, k: np.ndarray, x: np.ndarray, g_stages=None) -> np.ndarray:
        """J(k) x without assembling N'(U_i): c(z_i, U_i) + c(U_i, z_i), z_i = sum_j a_ij x_j^u."""
        y = self.S.J @ x
        nvel = self.th.nvel
        U = self.stage_values(u_n, k, g_stages)
        for i in range(self.r):
            z = sum(self.A[i, j] * self.S.split(x, j)[0] for j in range(self.r))
            zn = self.free_nodal(z)
            y[i * self.ns:i * self.ns + nvel] += self.dt * (self.convection_vector(zn, U[i]) +
                                                            self.convection_vector(U[i], zn))
        return y

    # ------------------------------------------------------------------ Newton
    def direct_solver(self):
        """Exact solve of J delta = b with one pinned pressure per stage, pressure means
        removed (the pressure null vectors of the Stokes part are null vectors of J)."""
        pins = [i * self.ns + self.th.nvel for i in range(self.r)]

        def solve(Jmat, b, eta):
            J = Jmat.toarray()
            J[pins, :] = 0.0
            J[:, pins] = 0.0
            J[pins, pins] = 1.0
            rhs = np.array(b, dtype=np.float64)
            rhs[pins] = 0.0
            return self.S.project_pressure_mean(sla.solve(J, rhs)), 0

        return solve

    def newton(self, F: np.ndarray, u_n: np.ndarray, k0: np.ndarray, g_stages=None, rtol: float = 1e-8,
               atol: float = 0.0, maxit: int = 20, ew: EWParams | None = None, linear_solve=None,
               linesearch: bool = False, ls_alpha: float = 1e-4, ls_maxit: int = 12, linear_solve_at=None):
        """Newton's method on G(k) = 0 from k0.  linear_solve(Jmat, b, eta) -> (delta,
        iterations) must satisfy ||b - J delta|| <= eta ||b||; default: exact solves.
        linear_solve_at(Jmat, b, eta, U), if given instead, also receives the nodal stage
        velocities U_i of the iterate (to build a preconditioner for the Jacobian there).
        linesearch: backtracking on ||G|| (module docstring)."""
        ew = ew or EWParams()
        solve = linear_solve or self.direct_solver()
        k = np.array(k0, dtype=np.float64)
        info = NewtonInfo()
        G = self.residual(F, u_n, k, g_stages)
        norm = float(np.linalg.norm(G))
        norm0 = norm
        info.norms.append(norm)
        eta_prev = ew.eta0
        norm_prev = norm
        while True:
            if norm <= max(atol, rtol * norm0):
                info.converged = True
                break
            if info.iterations >= maxit:
                break
            eta = ew_forcing(info.iterations, norm, norm_prev, eta_prev, ew, max(atol, rtol * norm0))
            if linear_solve_at is not None:
                U = self.stage_values(u_n, k, g_stages)
                delta, lits = linear_solve_at(self.jacobian_at(U), -G, eta, U)
            else:
                delta, lits = solve(self.jacobian(u_n, k, g_stages), -G, eta)
            lam = 1.0
            for trial in range(ls_maxit + 1 if linesearch else 1):
                kt = k + lam * delta
                Gt = self.residual(F, u_n, kt, g_stages)
                nt = float(np.linalg.norm(Gt))
                if not linesearch or nt <= (1.0 - ls_alpha * lam) * norm:
                    break
                lam *= 0.5
            else:
                return k, info  # no sufficient decrease: unconverged, k the last iterate
            k, G = kt, Gt
            info.etas.append(eta)
            info.linear_its.append(lits)
            info.lambdas.append(lam)
            info.iterations += 1
            eta_prev, norm_prev = eta, norm
            norm = nt
            info.norms.append(norm)
            if not np.isfinite(norm):
                break
        return k, info

    def step(self, b: np.ndarray, c: np.ndarray, forcing, t: float, u: np.ndarray, p: np.ndarray,
             k_prev: np.ndarray, **newton_kw):
        """One IRK step of the Navier--Stokes DAE: Newton from the previous step's stages,
        then u^{n+1} = u^n + dt sum_j b_j k_j^u (likewise p)."""
        S = self.S
        fn = [self.th.interpolate(forcing, t + ci * S.dt) for ci in c]
        F = S.rhs(fn, u, p)
        k, info = self.newton(F, u, k_prev, **newton_kw)
        u_new, p_new = u.copy(), p.copy()
        for j in range(S.r):
            ku, kp = S.split(k, j)
            u_new += S.dt * b[j] * ku
            p_new += S.dt * b[j] * kp
        return u_new, p_new, k, info


# --------------------------------------------------- the Newton Jacobian V-cycle
def inject_nodal(th_fine: TaylorHood, th_coarse: TaylorHood, U_fine: np.ndarray) -> np.ndarray:
    """A fine-level P2 field's values at the P2 nodes of the next coarser level, which
    are nodes of the fine level (uniform refinement makes every coarse vertex and edge
    midpoint a fine vertex), so the values are the fine field evaluated there."""
    scale = 1.0 + float(np.abs(th_fine.node_xyz).max())
    key = lambda x: tuple(np.round(x / scale * 2.0 ** 40).astype(np.int64))
    where = {key(x): i for i, x in enumerate(th_fine.node_xyz)}
    idx = np.array([where[key(x)] for x in th_coarse.node_xyz])
    return U_fine[idx]


def newton_hierarchy(mesh_levels, A, dt: float, nu: float, U_fine: list, **hierarchy_kw):
    """The V-cycle for the Newton Jacobian of the Navier--Stokes stage equations
    (Sec. 3.2) at the stage velocities U_fine (nodal arrays on the finest level): every
    level rediscretises the Jacobian, block (i, j) = delta_ij M + dt a_ij (K + N'(U_i)),
    with the stage velocities carried to it by injection at its nodes (the reading taken
    for data of the finest level on coarser meshes, as for the wind of the Oseen
    operator); Vanka patches, transfers and the coarse solve as for the Stokes cycle."""
    from .multigrid import Hierarchy

    spaces = [TaylorHood(m.xyz, m.cells) for m in mesh_levels]
    U_lev = [None] * len(spaces)
    U_lev[-1] = [np.asarray(u, dtype=np.float64) for u in U_fine]
    for lev in range(len(spaces) - 2, -1, -1):
        U_lev[lev] = [inject_nodal(spaces[lev + 1], spaces[lev], u) for u in U_lev[lev + 1]]

    def op(lev, system):
        return NavierStokesStages(system.th, A, dt, nu).jacobian_at(U_lev[lev])

    return Hierarchy(mesh_levels, A, dt, nu, level_operators=op, **hierarchy_kw)
