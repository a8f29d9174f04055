"""The stage-coupled IRK system of Sec. 3.1 (Kronecker form) and its right-hand side.

TEST INFRASTRUCTURE ONLY (oracle).

For an r-stage tableau (A, b, c) the stages k = (k_1^u, k_1^p, ..., k_r^u, k_r^p),
ordered by stage with each stage's velocity/pressure pair together, solve

    ( I_r (x) [M 0; 0 0] + dt A (x) [K B; B^T 0] ) k = F,
    F_i = [ M f_i - K u^n - B p^n ; -B^T u^n ],

with f_i the interpolant of the forcing at t^n + c_i dt; then
u^{n+1} = u^n + dt sum_j b_j k_j^u and p^{n+1} = p^n + dt sum_j b_j k_j^p.
For the Oseen operator K is replaced by K + C(w) (Sec. 3.2, linearised inertia with a
prescribed wind).  Within a stage the velocity is component-blocked over free nodes,
then the pressure over all vertices.

Pressure is defined up to a constant per stage (W_h is the zero-mean subspace): with
every velocity boundary node eliminated, J has the null vectors e_i (x) (0, 1_p).
The reading used throughout: remove each stage's arithmetic pressure mean after every
preconditioner application and from the final solution.

Prescribed (non-zero) boundary velocities g(t): the paper does not say how they enter
the stages; the reading here takes the DAE view of Sec. 3.1 and requires every stage
value to equal the data at its stage time, U_{i,b} = g(t^n + c_i dt) = G_i.  The
boundary stage derivatives are then k_b = (dt A)^{-1} (G - 1 (x) g(t^n)), and the
boundary couplings move to the right-hand side: velocity rows get
-M_fb k_{i,b} - K_fb G_i, divergence rows get -B_b^T G_i (rhs_dirichlet).  The state
keeps only free velocities; its boundary values are g at the current time.

Pinned by tests/test_oracle_stage.py against: the stage equations written out stage
by stage as in Sec. 3.1 (a double loop over a_ij) for J and F; the null vectors; a
dense direct solve; for boundary data, a steady P2-P1 Stokes solution (F vanishes) and
a solution linear in time (the exact stage derivatives solve J k = F for every
tableau).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import TaylorHood


class StageSystem:
    """Operators of one mesh level for fixed (tableau, dt, nu, wind)."""

    def __init__(self, th: TaylorHood, A: np.ndarray, dt: float, nu: float, wind_nodal: np.ndarray | None = None):
        self.th = th
        self.A = np.asarray(A, dtype=np.float64)
        self.r = self.A.shape[0]
        self.dt = float(dt)
        self.nu = float(nu)
        self._wind = wind_nodal
        d = th.dim
        M, K, C, Mfa = th.scalar_matrices(nu, wind_nodal)
        self.Ms, self.Ks, self.Cs, self.Ms_free_all = M, K, C, Mfa
        Id = sp.identity(d, format="csr")
        self.Mv = sp.kron(Id, M).tocsr()
        L = K if C is None else (K + C)
        self.Lv = sp.kron(Id, L).tocsr()  # velocity block of the spatial operator
        self.Kv = sp.kron(Id, K).tocsr()
        self.B = th.divergence()
        nv = th.nverts
        self.Mhat = sp.block_diag([self.Mv, sp.csr_matrix((nv, nv))]).tocsr()
        self.Shat = sp.bmat([[self.Lv, self.B], [self.B.T, None]]).tocsr()
        self.J = (sp.kron(sp.identity(self.r), self.Mhat) + self.dt * sp.kron(self.A, self.Shat)).tocsr()
        self.ns = th.nstage
        self.n = self.r * self.ns

    # --------------------------------------------------------------- operators
    def apply(self, k: np.ndarray) -> np.ndarray:
        return self.J @ k

    def apply_transpose(self, k: np.ndarray) -> np.ndarray:
        return self.J.T @ k

    def residual(self, F: np.ndarray, k: np.ndarray) -> np.ndarray:
        return F - self.J @ k

    # ---------------------------------------------------------- right-hand side
    def rhs(self, f_nodal_stages: list[np.ndarray], u_n: np.ndarray, p_n: np.ndarray) -> np.ndarray:
        """F for stage forcings f_i (each (nnodes, d) nodal values), u^n (component-
        blocked free velocity) and p^n (vertex values)."""
        th = self.th
        blocks = []
        for i in range(self.r):
            Mf = np.concatenate([self.Ms_free_all @ f_nodal_stages[i][:, c] for c in range(th.dim)])
            Fu = Mf - self.Lv @ u_n - self.B @ p_n
            Fp = -(self.B.T @ u_n)
            blocks.append(np.concatenate([Fu, Fp]))
        return np.concatenate(blocks)

    # ----------------------------------------------------------------- helpers
    def split(self, k: np.ndarray, i: int) -> tuple[np.ndarray, np.ndarray]:
        blk = k[i * self.ns:(i + 1) * self.ns]
        return blk[: self.th.nvel], blk[self.th.nvel:]

    def project_pressure_mean(self, k: np.ndarray) -> np.ndarray:
        """Remove each stage's arithmetic pressure mean (nullspace reading)."""
        k = k.copy()
        nvel = self.th.nvel
        for i in range(self.r):
            p = k[i * self.ns + nvel:(i + 1) * self.ns]
            p -= p.mean()
        return k

    def nullspace(self) -> np.ndarray:
        Z = np.zeros((self.n, self.r))
        for i in range(self.r):
            Z[i * self.ns + self.th.nvel:(i + 1) * self.ns, i] = 1.0
        return Z


    # ------------------------------------------------------- boundary data terms
    def _boundary_blocks(self):
        if getattr(self, "_bnd", None) is None:
            th = self.th
            f = th.free
            bnd = np.setdiff1d(np.arange(th.nnodes), f)
            Mfull = th.scalar_mass_full()
            Lfull = self.nu * th._assemble_nodes(th.element_stiffness())
            if self.Cs is not None:
                Lfull = Lfull + th._assemble_nodes(th.element_convection(self._wind))
            Bc = th.divergence_full()
            self._bnd = (bnd, Mfull[f][:, bnd].tocsr(), Lfull[f][:, bnd].tocsr(),
                         [B[bnd].T.tocsr() for B in Bc])
        return self._bnd

    def rhs_dirichlet(self, g_n: np.ndarray, g_stages: list[np.ndarray]) -> np.ndarray:
        """Terms the boundary data add to F (reading in the module docstring).
        g_n: (nnodes, dim) data at t^n; g_stages: r arrays (nnodes, dim) at t^n + c_i dt;
        only boundary-node values are used."""
        th = self.th
        bnd, Mfb, Lfb, Btb = self._boundary_blocks()
        G = np.stack([np.asarray(g)[bnd] for g in g_stages])  # (r, nb, dim)
        kb = np.einsum("ij,jbc->ibc", np.linalg.inv(self.dt * self.A), G - np.asarray(g_n)[bnd][None])
        blocks = []
        for i in range(self.r):
            vel = np.concatenate([-(Mfb @ kb[i, :, c]) - (Lfb @ G[i, :, c]) for c in range(th.dim)])
            pre = -sum(Btb[c] @ G[i, :, c] for c in range(th.dim))
            blocks.append(np.concatenate([vel, pre]))
        return np.concatenate(blocks)
