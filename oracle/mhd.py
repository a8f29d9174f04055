"""Linearised 2D MHD stage system and its Vanka multigrid (Sec. 3.3, 4.1, 4.2, Fig. 1 right).

TEST INFRASTRUCTURE ONLY (oracle).

Spaces (Sec. 3.3): velocity u in vector P2 with u = 0 on the boundary, magnetic field B
in lowest-order Nedelec (first kind) with B x n = 0 on the boundary, pressure p in P1
(mean zero), Lagrange multiplier gamma in P1 with gamma = 0 on the boundary.  In 2D the
curl of a vector field is the scalar curl B = d_x B_y - d_y B_x and the products with
it follow the paper's extension to three-dimensional fields with zero third component:
(curl B) x B0 = curl B (-B0_y, B0_x), u x B0 = u_x B0_y - u_y B0_x.

Nedelec degrees of freedom: one per edge, the line integral of the tangential component
along the edge from its lower-numbered to its higher-numbered vertex; on a cell the
basis function of the edge (a, b), a < b, is lam_a grad lam_b - lam_b grad lam_a, with
curl 2 grad lam_a x grad lam_b.

The weak form of Sec. 3.3 is linearised (Newton) at a state (w, B0): u in P2 nodal
values, B0 in Nedelec degrees of freedom on every edge.  The spatial operator S acts on
(u, B, p, gamma) by the bilinear forms, test functions (v, c, q, s):
  (2/Re) (eps(u), eps(v)) + c(w, u; v) + c(u, w; v)                 [viscosity, N'(w)]
  - ((curl B) x B0 + (curl B0) x B) . v                              [Lorentz force]
  - (p, div v),   -(q, div u)                                        [incompressibility]
  (1/Re_m) (curl B, curl c) - (u x B0 + w x B, curl c) - (grad gamma, c)   [induction]
  -(B, grad s)                                                       [solenoidal constraint]
with the mass M = diag(M_u, M_B, 0, 0).  The printed weak form carries a minus sign on
the viscous term; integration by parts of -div((2/Re) eps(u)) gives the plus sign
taken here (with the minus the operator would not be dissipative).  The IRK stage
system (Sec. 3.1 applied to this DAE) is J = I_r (x) M + dt A (x) S.

Unknown order per stage: u (component-blocked over the free P2 nodes, as in the fluid
solver), B (interior edges in edge order), p (every vertex), gamma (interior vertices in
vertex order); stages one after the other.

Transfers (Sec. 4.1): P = diag(P_u, P_B, P_p, P_gamma), P_u and P_p canonical P2 and P1
interpolation, P_gamma the P1 one restricted to interior vertices, P_B the canonical
Nedelec interpolation (a fine degree of freedom is the line integral of the coarse
field along the fine edge, exact by the midpoint rule since the tangential component
of a lowest-order Nedelec function is linear along a segment).  Coarse levels take the
linearisation state by rediscretisation: w injected at their P2 nodes, B0's degrees of
freedom as sums of the fine degrees of freedom along the two halves of each coarse
edge (additivity of the line integral).

Patches (Sec. 4.2, Fig. 1 right): for each vertex v, the free P2 velocity nodes and the
interior edges of the closure of the cells around v, the pressure at v and, for an
interior v, the multiplier at v; all stages.

Pinned by tests/test_oracle_mhd.py against: Nedelec tangential moments (the identity on
every cell), the commuting properties curl grad = 0 and P_B grad_c = grad_f P_1 on
nested meshes, the multiplier coupling -(grad s, c) equal to -(M_B G) for the discrete
gradient G, Nedelec reproduction of constant fields by P_B, the skew coupling
S_uB = -S_Bu^T for constant B0 and w = 0, the rediscretised coarse state against
the coarse interpolant, single-patch exactness, and FGMRES with the V-cycle reaching
the dense direct solve.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fem import LOCAL_EDGES, TaylorHood, p1_basis, p2_basis, simplex_quadrature
from .multigrid import Hierarchy
from .navier_stokes import NavierStokesStages, inject_nodal
from .transfer import _locate, interpolation_matrices
from .vanka import VankaSmoother

_DLAM = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])  # reference gradients of lam_0..2


class MHDSpace:
    """P2 velocity, Nedelec magnetic field, P1 pressure and multiplier on one 2D mesh."""

    def __init__(self, th: TaylorHood):
        assert th.dim == 2, "the MHD spaces are built for triangles"
        self.th = th
        nv = th.nverts
        self.bedge = th.boundary[nv:]
        self.efree = np.flatnonzero(~self.bedge)
        self.nB = self.efree.size
        self.eidx = -np.ones(th.nedges, dtype=np.int64)
        self.eidx[self.efree] = np.arange(self.nB)
        self.vint = np.flatnonzero(~th.boundary[:nv])
        self.ng = self.vint.size
        self.gidx = -np.ones(nv, dtype=np.int64)
        self.gidx[self.vint] = np.arange(self.ng)
        self.nu_ = th.nvel
        self.off_B = self.nu_
        self.off_p = self.off_B + self.nB
        self.off_g = self.off_p + nv
        self.ns = self.off_g + self.ng
        self.cell_edges = th.cell_nodes[:, 3:] - nv  # local edge order LOCAL_EDGES[2]
        # physical gradients of the barycentric coordinates per cell: (nc, 3, 2)
        self.glam = np.einsum("cij,kj->cki", th.jinvT, _DLAM)

    # ------------------------------------------------------------- Nedelec basis
    def _edge_ends(self):
        """Local vertex pairs (lo, hi) of each cell's edges, ordered by global index."""
        cells = self.th.cells
        lo = np.zeros((self.th.ncells, 3), dtype=np.int64)
        hi = np.zeros_like(lo)
        for e, (i, j) in enumerate(LOCAL_EDGES[2]):
            swap = cells[:, i] > cells[:, j]
            lo[:, e] = np.where(swap, j, i)
            hi[:, e] = np.where(swap, i, j)
        return lo, hi

    def nedelec_at(self, lam: np.ndarray):
        """Basis values (nc, nq, 3 edges, 2) at barycentric points lam (nq, 3) of every
        cell, and the curls (nc, 3)."""
        lo, hi = self._edge_ends()
        g = self.glam
        c = np.arange(self.th.ncells)[:, None]
        g_lo, g_hi = g[c, lo], g[c, hi]  # (nc, 3, 2)
        l_lo, l_hi = lam[:, lo], lam[:, hi]  # (nq, nc, 3)
        val = (np.einsum("qce,cek->cqek", l_lo, g_hi) - np.einsum("qce,cek->cqek", l_hi, g_lo))
        curl = 2.0 * (g_lo[..., 0] * g_hi[..., 1] - g_lo[..., 1] * g_hi[..., 0])
        return val, curl

    def _quad(self):
        xi, w = simplex_quadrature(2)
        lam = p1_basis(2, xi)
        val2, gref = p2_basis(2, xi)
        g2 = np.einsum("cij,qnj->cqni", self.th.jinvT, gref)
        nval, ncurl = self.nedelec_at(lam)
        return xi, w, lam, val2, g2, nval, ncurl

    def edge_dofs(self, field, npts: int = 8) -> np.ndarray:
        """Line integrals of a vector field (callable on points (n, 2)) along every edge
        from its lower to its higher vertex (Gauss--Legendre with npts points)."""
        th = self.th
        a, b = th.xyz[th.edges[:, 0]], th.xyz[th.edges[:, 1]]
        g, wg = np.polynomial.legendre.leggauss(npts)
        out = np.zeros(th.nedges)
        for t, wt in zip(0.5 * (g + 1.0), 0.5 * wg):
            out += wt * np.einsum("ek,ek->e", np.asarray(field(a + t * (b - a))), b - a)
        return out

    def edge_mass_all(self) -> sp.csr_matrix:
        """int phi_f . phi_g over every pair of edges (boundary edges included)."""
        xi, w, lam, val2, g2, nval, ncurl = self._quad()
        E = np.einsum("q,cqfk,cqgk,c->cgf", w, nval, nval, self.th.detj, optimize=True)
        n = self.th.nedges
        return self._assemble(E, self.cell_edges, self.cell_edges, (n, n))

    def discrete_gradient(self) -> sp.csr_matrix:
        """Edge degrees of freedom of grad s for s in P1 (all edges x all vertices):
        s_hi - s_lo."""
        th = self.th
        ne = th.nedges
        rows = np.repeat(np.arange(ne), 2)
        cols = th.edges.ravel()
        vals = np.tile([-1.0, 1.0], ne)
        return sp.coo_matrix((vals, (rows, cols)), shape=(ne, th.nverts)).tocsr()

    # ----------------------------------------------------------------- assembly
    def _assemble(self, elem, rows_of, cols_of, shape):
        """Sum element matrices elem (nc, nr, nc_) with global indices rows_of (nc, nr)
        and cols_of (nc, nc_) (negative: dropped)."""
        nr, ncl = elem.shape[1], elem.shape[2]
        R = np.repeat(rows_of, ncl, axis=1).ravel()
        C = np.tile(cols_of, (1, nr)).ravel()
        V = elem.ravel()
        keep = (R >= 0) & (C >= 0)
        return sp.coo_matrix((V[keep], (R[keep], C[keep])), shape=shape).tocsr()

    def operators(self, Re: float, Rem: float, w_nodal: np.ndarray, b0: np.ndarray):
        """Spatial mass M and linearised operator S (ns x ns, unknown order of the module
        docstring) at the state (w_nodal: (nnodes, 2) P2 values; b0: Nedelec degrees of
        freedom on every edge)."""
        th = self.th
        xi, w, lam, val2, g2, nval, ncurl = self._quad()
        detj = th.detj
        nf = th.nfree
        vel_rows = [np.where(th.free_index[th.cell_nodes] >= 0, c * nf + th.free_index[th.cell_nodes], -1)
                    for c in range(2)]
        brow = np.where(self.eidx[self.cell_edges] >= 0, self.off_B + self.eidx[self.cell_edges], -1)
        prow = self.off_p + th.cells
        grow = np.where(self.gidx[th.cells] >= 0, self.off_g + self.gidx[th.cells], -1)
        shape = (self.ns, self.ns)
        # state at the quadrature points
        b0c = b0[self.cell_edges]  # (nc, 3)
        B0q = np.einsum("cqek,ce->cqk", nval, b0c)
        j0 = np.einsum("ce,ce->c", ncurl, b0c)
        # velocity-velocity: (1/Re)(delta_ce grad.grad + d_e phi_a d_c phi_b) + N'(w)
        Mu = np.einsum("q,qa,qb,c->cab", w, val2, val2, detj)
        Kg = np.einsum("q,cqai,cqbi,c->cab", w, g2, g2, detj, optimize=True)
        blocks = []
        for c in range(2):
            for e in range(2):
                Ge = np.einsum("q,cqa,cqb,c->cab", w, g2[:, :, :, e], g2[:, :, :, c], detj, optimize=True)
                ce = (Kg if c == e else 0.0) + Ge
                blocks.append(self._assemble(ce / Re, vel_rows[c], vel_rows[e], shape))
        S = sum(blocks)
        ns_ops = NavierStokesStages(th, np.eye(1), 1.0, 1.0)
        Np = ns_ops.nprime(w_nodal)  # component-blocked free velocities
        S = S + sp.block_diag([Np, sp.csr_matrix((self.ns - self.nu_,) * 2)]).tocsr()
        M = self._assemble(Mu, vel_rows[0], vel_rows[0], shape) + self._assemble(Mu, vel_rows[1], vel_rows[1], shape)
        # Lorentz force: test (a, x): int phi_a (curl phi_f B0_y + j0 phi_f,y); (a, y): -(... B0_x, phi_f,x)
        for c, (k_b0, k_phi, sgn) in enumerate(((1, 1, 1.0), (0, 0, -1.0))):
            E = sgn * (np.einsum("q,qa,ce,cq,c->cae", w, val2, ncurl, B0q[:, :, k_b0], detj, optimize=True)
                       + np.einsum("q,qa,c,cqe,c->cae", w, val2, j0, nval[:, :, :, k_phi], detj, optimize=True))
            S = S + self._assemble(E, vel_rows[c], brow, shape)
        # induction from the velocity: -(u x B0, curl c): trial (b, x): -int phi_b B0_y curl phi_g;
        # (b, y): +int phi_b B0_x curl phi_g
        for e, (k_b0, sgn) in enumerate(((1, -1.0), (0, 1.0))):
            E = sgn * np.einsum("q,qb,cq,cg,c->cgb", w, val2, B0q[:, :, k_b0], ncurl, detj, optimize=True)
            S = S + self._assemble(E, brow, vel_rows[e], shape)
        # magnetic block: (1/Re_m)(curl, curl) - (w x B, curl c), and the mass
        wq = np.einsum("qn,cnk->cqk", val2, w_nodal[th.cell_nodes])
        KB = np.einsum("q,cf,cg,c->cgf", w, ncurl, ncurl, detj) / Rem
        WB = -np.einsum("q,cq,cqf,cg,c->cgf", w, wq[:, :, 0], nval[:, :, :, 1], ncurl, detj, optimize=True) \
            + np.einsum("q,cq,cqf,cg,c->cgf", w, wq[:, :, 1], nval[:, :, :, 0], ncurl, detj, optimize=True)
        S = S + self._assemble(KB + WB, brow, brow, shape)
        MB = np.einsum("q,cqfk,cqgk,c->cgf", w, nval, nval, detj, optimize=True)
        M = M + self._assemble(MB, brow, brow, shape)
        # pressure: -(p, div v) and -(q, div u)
        Dv = sp.coo_matrix(th.divergence())  # component-blocked free velocity x vertices
        rows = np.concatenate([Dv.row, Dv.col + self.off_p])
        cols = np.concatenate([Dv.col + self.off_p, Dv.row])
        S = S + sp.coo_matrix((np.concatenate([Dv.data, Dv.data]), (rows, cols)), shape=shape).tocsr()
        # multiplier: -(grad gamma, c) and -(B, grad s)
        Eg = -np.einsum("q,cqgk,cjk,c->cgj", w, nval, self.glam, detj, optimize=True)  # (nc, 3 edges, 3 vertices)
        S = S + self._assemble(Eg, brow, grow, shape)
        S = S + self._assemble(Eg.transpose(0, 2, 1), grow, brow, shape)
        return M.tocsr(), S.tocsr()

    # --------------------------------------------------------------- patches
    def patches(self, r: int) -> list[np.ndarray]:
        """Sorted global unknowns (stage-major) of every vertex patch."""
        th = self.th
        cells_of_vertex = [[] for _ in range(th.nverts)]
        for c, verts in enumerate(th.cells):
            for v in verts:
                cells_of_vertex[v].append(c)
        out = []
        for v in range(th.nverts):
            cl = cells_of_vertex[v]
            nodes = np.unique(th.cell_nodes[cl].ravel())
            fidx = th.free_index[nodes]
            fidx = fidx[fidx >= 0]
            edges = np.unique(self.cell_edges[cl].ravel())
            eb = self.eidx[edges]
            eb = eb[eb >= 0]
            blk = [c * th.nfree + fidx for c in range(2)] + [self.off_B + eb, np.array([self.off_p + v])]
            if self.gidx[v] >= 0:
                blk.append(np.array([self.off_g + self.gidx[v]]))
            stage = np.concatenate(blk)
            out.append(np.sort(np.concatenate([i * self.ns + stage for i in range(r)])))
        return out

    def project_pressure_mean(self, k: np.ndarray, r: int) -> np.ndarray:
        k = np.array(k, dtype=np.float64)
        for i in range(r):
            p = k[i * self.ns + self.off_p:i * self.ns + self.off_g]
            p -= p.mean()
        return k


def nedelec_prolongation(coarse: MHDSpace, fine: MHDSpace, free_only: bool = True) -> sp.csr_matrix:
    """P_B: fine interior edges x coarse interior edges (every edge with free_only
    False), fine degree of freedom = line integral of the coarse field along the fine
    edge (midpoint rule, exact)."""
    tf = fine.th
    frows = fine.efree if free_only else np.arange(tf.nedges)
    cidx = coarse.eidx if free_only else np.arange(coarse.th.nedges)
    ncol = coarse.nB if free_only else coarse.th.nedges
    a, b = tf.xyz[tf.edges[frows, 0]], tf.xyz[tf.edges[frows, 1]]
    mid = 0.5 * (a + b)
    cell, lam = _locate(coarse.th, mid)
    lo, hi = coarse._edge_ends()
    g = coarse.glam[cell]  # (n, 3, 2)
    rows, cols, vals = [], [], []
    for e in range(3):
        ilo, ihi = lo[cell, e], hi[cell, e]
        n = np.arange(len(cell))
        phi = lam[n, ilo][:, None] * g[n, ihi] - lam[n, ihi][:, None] * g[n, ilo]
        v = np.einsum("nk,nk->n", phi, b - a)
        ce = cidx[coarse.cell_edges[cell, e]]
        keep = ce >= 0
        rows.append(np.arange(len(cell))[keep])
        cols.append(ce[keep])
        vals.append(v[keep])
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(len(frows), ncol)).tocsr()
    P.data[np.abs(P.data) < 1e-14] = 0.0
    P.eliminate_zeros()
    return P


def coarsen_b0(fine: MHDSpace, coarse: MHDSpace, b0_fine: np.ndarray) -> np.ndarray:
    """Degrees of freedom of B0 on the coarse edges: the line integral over each coarse
    edge is the sum over its two fine halves (each traversed from the coarse edge's
    lower to its higher vertex)."""
    tf, tc = fine.th, coarse.th
    scale = 1.0 + float(np.abs(tf.xyz).max())
    key = lambda x: tuple(np.round(x / scale * 2.0 ** 40).astype(np.int64))  # noqa: E731
    vid = {key(x): i for i, x in enumerate(tf.xyz)}
    eid = {(int(p), int(q)): e for e, (p, q) in enumerate(tf.edges)}
    out = np.zeros(tc.nedges)
    for e, (A, B) in enumerate(tc.edges):
        xa, xb = tc.xyz[A], tc.xyz[B]
        fa, fb, fm = vid[key(xa)], vid[key(xb)], vid[key(0.5 * (xa + xb))]
        tot = 0.0
        for s, t in ((fa, fm), (fm, fb)):
            sign = 1.0 if s < t else -1.0
            tot += sign * b0_fine[eid[(min(s, t), max(s, t))]]
        out[e] = tot
    return out


class _MHDLevel:
    """What the V-cycle of multigrid.Hierarchy reads from a level's system."""

    def __init__(self, space: MHDSpace, J: sp.csr_matrix, r: int):
        self.space, self.J, self.r = space, J, r
        self.ns = space.ns
        self.n = r * space.ns

    def apply(self, k):
        return self.J @ k

    def project_pressure_mean(self, k):
        return self.space.project_pressure_mean(k, self.r)


class MHDHierarchy(Hierarchy):
    """The V-cycle of Sec. 4.1 for the linearised MHD stage system: rediscretisation on
    every level, the Vanka patches of Fig. 1 (right), damped additive sweeps (smoother
    "sweep") or Chebyshev relaxation on `interval` (smoother "chebyshev", Sec. 5.1; the
    paper's MHD runs take 3 / 3 steps on [2, 10]), I_r (x) P transfers and a dense coarse
    solve with the pressure of vertex 0 pinned per stage; the cycle itself is
    multigrid.Hierarchy's."""

    def __init__(self, mesh_levels, A, dt, Re, Rem, w_fine, b0_fine, omega=0.5, weighted=True, pre=2, post=2,
                 smoother="sweep", interval=(2.0, 10.0)):
        self.A = np.asarray(A, dtype=np.float64)
        self.r = r = self.A.shape[0]
        self.pre, self.post = pre, post
        self.smoother, self.interval = smoother, tuple(interval)
        self.dtype = np.float64
        ths = [TaylorHood(m.xyz, m.cells) for m in mesh_levels]
        self.spaces = [MHDSpace(t) for t in ths]
        L = len(ths)
        ws, bs = [None] * L, [None] * L
        ws[-1], bs[-1] = np.asarray(w_fine, dtype=np.float64), np.asarray(b0_fine, dtype=np.float64)
        for lev in range(L - 2, -1, -1):
            ws[lev] = inject_nodal(ths[lev + 1], ths[lev], ws[lev + 1])
            bs[lev] = coarsen_b0(self.spaces[lev + 1], self.spaces[lev], bs[lev + 1])
        self.states = list(zip(ws, bs))
        self.M, self.S, self.ops = [], [], []
        for lev, sp_ in enumerate(self.spaces):
            M, S = sp_.operators(Re, Rem, ws[lev], bs[lev])
            self.M.append(M)
            self.S.append(S)
            self.ops.append((sp.kron(sp.identity(r), M) + dt * sp.kron(self.A, S)).tocsr())
        self.systems = [_MHDLevel(s, J, r) for s, J in zip(self.spaces, self.ops)]
        self.dim = 2
        self.P = [None]
        for lev in range(L - 1):
            c, f = self.spaces[lev], self.spaces[lev + 1]
            Pu, Pp = interpolation_matrices(c.th, f.th)
            Pg = Pp[f.vint][:, c.vint]
            P1 = sp.block_diag([sp.kron(sp.identity(2), Pu), nedelec_prolongation(c, f), Pp, Pg])
            self.P.append(sp.kron(sp.identity(r), P1).tocsr())
        self.Jw = list(self.ops)
        self.Pw = list(self.P)
        self.smoothers = [None] + [VankaSmoother(self.ops[lev], self.spaces[lev].patches(r), omega, weighted)
                                   for lev in range(1, L)]
        s0 = self.spaces[0]
        Jc = self.ops[0].toarray()
        self.pinned = [i * s0.ns + s0.off_p for i in range(r)]
        for q in self.pinned:
            Jc[q, :] = 0.0
            Jc[:, q] = 0.0
            Jc[q, q] = 1.0
        self.coarse_lu = sla.lu_factor(Jc)
        self.coarse_luT = sla.lu_factor(Jc.T.copy())


def island_state(space: MHDSpace, k: float = 0.2, perturb: bool = True):
    """The island-coalescence equilibrium of Sec. 5.3 with the perturbation of its
    initial condition, evaluated at X = 2x - 1 on the unit square (the paper's domain is
    (-1, 1)^2 with periodic sides; here the square of the meshes with the boundary
    conditions of Sec. 3.3): w = 0 (P2 nodal) and B0's Nedelec degrees of freedom."""
    def B(x):
        X, Y = 2.0 * x[:, 0] - 1.0, 2.0 * x[:, 1] - 1.0
        den = np.cosh(2 * np.pi * Y) + k * np.cos(2 * np.pi * X)
        b = np.stack([np.sinh(2 * np.pi * Y), k * np.sin(2 * np.pi * X)], axis=1) / den[:, None]
        if perturb:
            b += (-0.01 / np.pi) * np.stack([-np.cos(np.pi * X) * np.sin(np.pi * Y / 2) / 2,
                                             np.cos(np.pi * Y / 2) * np.sin(np.pi * X)], axis=1)
        return b
    return np.zeros((space.th.nnodes, 2)), space.edge_dofs(B)
