"""Taylor--Hood P2-P1 discretization on simplices (Sec. 3.1).

TEST INFRASTRUCTURE ONLY (oracle).

Velocity lives in vector P2 with homogeneous Dirichlet conditions, pressure in P1 on
the vertices (Sec. 3.1, spaces V_h and W_h).  The semi-discrete system is
[M u_t; 0] + [K B; B^T 0][u; p] = [M f; 0] with
  M_ij       = int phi_i phi_j                       (mass, per component)
  K_ij       = nu int grad phi_i . grad phi_j          (stiffness, per component)
  B_(i,c),q  = - int psi_q d_c phi_i                   (weak gradient; -<p, div v>)
and, for the linearised Navier--Stokes (Oseen) operator of Sec. 3.2, the convection
  C_ij       = int (w . grad phi_j) phi_i              (prescribed wind w in P2).

Numbering (shared convention with the HIP library, fixed by its public header):
P2 nodes are the vertices in input order followed by the edges sorted by
(smaller vertex, larger vertex).  A node is on the boundary when it lies on a facet
that belongs to exactly one cell.  Free velocity nodes are the interior nodes in
ascending node order.  Dirichlet nodes are eliminated (the paper does not say how
boundary conditions are imposed; elimination is the reading taken here).

Quadrature: Duffy-collapsed Gauss--Legendre with 5 points per direction on the
reference simplex, exact for polynomial integrands of degree <= 7 (3D) and <= 8 (2D),
so every integral here (degree <= 5) is exact.

Pinned by tests/test_oracle_fem.py against: the textbook P2 element mass matrix on a
triangle (|T|/180 [6 -1 -1 0 -4 0; ...]); sum of the full mass matrix = |Omega|;
K 1 = 0; q^T B^T u = -int q div u for polynomial u, q computed in closed form;
B 1_p = 0 after elimination; x^T C x = 0 for a constant wind; entity counts.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

LOCAL_EDGES = {
    2: [(0, 1), (0, 2), (1, 2)],
    3: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
}


# --------------------------------------------------------------------- quadrature
def simplex_quadrature(dim: int, npts: int = 5) -> tuple[np.ndarray, np.ndarray]:
    """Collapsed (Duffy) Gauss--Legendre rule on the reference simplex
    {xi >= 0, sum xi <= 1}.  Returns points (nq, dim) and weights (nq,)."""
    g, w = np.polynomial.legendre.leggauss(npts)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    if dim == 2:
        for (u, wu), (v, wv) in itertools.product(zip(g, w), zip(g, w)):
            pts.append((u, v * (1 - u)))
            wts.append(wu * wv * (1 - u))
    else:
        for (u, wu), (v, wv), (s, ws) in itertools.product(zip(g, w), zip(g, w), zip(g, w)):
            pts.append((u, v * (1 - u), s * (1 - u) * (1 - v)))
            wts.append(wu * wv * ws * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


def p2_basis(dim: int, xi: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """P2 Lagrange basis on the reference simplex at points xi (nq, dim).

    Local order: vertices 0..dim, then edges LOCAL_EDGES[dim].  In barycentric
    coordinates lam the vertex function is lam_i (2 lam_i - 1) and the edge function
    4 lam_i lam_j.  Returns values (nq, nloc) and reference gradients (nq, nloc, dim).
    """
    nq = xi.shape[0]
    lam = np.hstack([1.0 - xi.sum(axis=1, keepdims=True), xi])
    dlam = np.vstack([-np.ones((1, dim)), np.eye(dim)])  # (dim+1, dim)
    edges = LOCAL_EDGES[dim]
    nloc = dim + 1 + len(edges)
    val = np.zeros((nq, nloc))
    grad = np.zeros((nq, nloc, dim))
    for i in range(dim + 1):
        val[:, i] = lam[:, i] * (2 * lam[:, i] - 1)
        grad[:, i, :] = (4 * lam[:, i] - 1)[:, None] * dlam[i][None, :]
    for e, (i, j) in enumerate(edges):
        val[:, dim + 1 + e] = 4 * lam[:, i] * lam[:, j]
        grad[:, dim + 1 + e, :] = 4 * (lam[:, i][:, None] * dlam[j][None, :] + lam[:, j][:, None] * dlam[i][None, :])
    return val, grad


def p1_basis(dim: int, xi: np.ndarray) -> np.ndarray:
    return np.hstack([1.0 - xi.sum(axis=1, keepdims=True), xi])


# ------------------------------------------------------------------------ spaces
class TaylorHood:
    """P2 (velocity) / P1 (pressure) spaces on one simplicial mesh."""

    def __init__(self, xyz: np.ndarray, cells: np.ndarray):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.cells = np.asarray(cells, dtype=np.int64)
        self.dim = self.cells.shape[1] - 1
        d = self.dim
        self.nverts = self.xyz.shape[0]
        self.ncells = self.cells.shape[0]
        le = LOCAL_EDGES[d]
        pairs = np.concatenate([np.sort(self.cells[:, [a, b]], axis=1) for a, b in le])
        self.edges, inv = np.unique(pairs, axis=0, return_inverse=True)
        inv = np.asarray(inv).ravel()
        self.nedges = self.edges.shape[0]
        cell_edges = inv.reshape(len(le), self.ncells).T
        self.cell_nodes = np.hstack([self.cells, self.nverts + cell_edges])
        self.nnodes = self.nverts + self.nedges
        self.node_xyz = np.vstack([self.xyz, 0.5 * (self.xyz[self.edges[:, 0]] + self.xyz[self.edges[:, 1]])])

        # boundary facets: facets that belong to exactly one cell
        facets = np.concatenate([np.sort(self.cells[:, list(f)], axis=1) for f in itertools.combinations(range(d + 1), d)])
        uniq, counts = np.unique(facets, axis=0, return_counts=True)
        bfac = uniq[counts == 1]
        bmask = np.zeros(self.nnodes, dtype=bool)
        bmask[np.unique(bfac)] = True
        keys = self.edges[:, 0] * self.nverts + self.edges[:, 1]
        for a, b in itertools.combinations(range(d), 2):
            ek = np.minimum(bfac[:, a], bfac[:, b]) * self.nverts + np.maximum(bfac[:, a], bfac[:, b])
            idx = np.searchsorted(keys, ek)
            assert np.all(keys[idx] == ek)
            bmask[self.nverts + idx] = True
        self.boundary = bmask
        self.free = np.flatnonzero(~bmask)
        self.nfree = self.free.size
        self.free_index = -np.ones(self.nnodes, dtype=np.int64)
        self.free_index[self.free] = np.arange(self.nfree)

        # affine maps
        x0 = self.xyz[self.cells[:, 0]]
        self.jac = np.stack([self.xyz[self.cells[:, k + 1]] - x0 for k in range(d)], axis=2)  # (nc, d, d)
        self.detj = np.abs(np.linalg.det(self.jac))
        self.jinvT = np.linalg.inv(self.jac).transpose(0, 2, 1)

    # per-stage vector sizes in the public (component-blocked) layout
    @property
    def nvel(self) -> int:
        return self.dim * self.nfree

    @property
    def nstage(self) -> int:
        return self.dim * self.nfree + self.nverts

    def interpolate(self, field, t: float = 0.0) -> np.ndarray:
        """Nodal P2 interpolant of a vector field at every node: (nnodes, dim)."""
        return np.asarray(field(self.node_xyz, t), dtype=np.float64)

    def free_velocity(self, nodal: np.ndarray) -> np.ndarray:
        """Component-blocked free-node vector from (nnodes, dim) nodal values."""
        return np.concatenate([nodal[self.free, c] for c in range(self.dim)])

    # ------------------------------------------------------------- element data
    def _quad(self):
        xi, w = simplex_quadrature(self.dim)
        val, gref = p2_basis(self.dim, xi)
        gphys = np.einsum("cij,qnj->cqni", self.jinvT, gref)  # (nc, nq, nloc, d)
        return xi, w, val, gphys

    def element_mass(self) -> np.ndarray:
        xi, w, val, _ = self._quad()
        return np.einsum("q,qa,qb,c->cab", w, val, val, self.detj)

    def element_stiffness(self) -> np.ndarray:
        xi, w, val, g = self._quad()
        return np.einsum("q,cqai,cqbi,c->cab", w, g, g, self.detj, optimize=True)

    def element_divergence(self) -> np.ndarray:
        """E[c, a, comp, i] = -int psi_i d_comp phi_a over cell c."""
        xi, w, val, g = self._quad()
        psi = p1_basis(self.dim, xi)
        return -np.einsum("q,qi,cqak,c->caki", w, psi, g, self.detj, optimize=True)

    def element_convection(self, wind_nodal: np.ndarray) -> np.ndarray:
        """C[c, a, b] = int (w . grad phi_b) phi_a, w the P2 interpolant of the wind."""
        xi, w, val, g = self._quad()
        wloc = wind_nodal[self.cell_nodes]  # (nc, nloc, d)
        wq = np.einsum("qn,cnk->cqk", val, wloc)
        return np.einsum("q,qa,cqk,cqbk,c->cab", w, val, wq, g, self.detj, optimize=True)

    # ---------------------------------------------------------------- assembly
    def _assemble_nodes(self, elem: np.ndarray) -> sp.csr_matrix:
        nl = self.cell_nodes.shape[1]
        rows = np.repeat(self.cell_nodes, nl, axis=1).ravel()
        cols = np.tile(self.cell_nodes, (1, nl)).ravel()
        return sp.coo_matrix((elem.ravel(), (rows, cols)), shape=(self.nnodes, self.nnodes)).tocsr()

    def scalar_mass_full(self) -> sp.csr_matrix:
        return self._assemble_nodes(self.element_mass())

    def scalar_matrices(self, nu: float, wind_nodal: np.ndarray | None = None):
        """Free-free scalar P2 matrices: M, nu*K, C (C is None without wind), plus the
        free-rows/all-columns mass used for the forcing term."""
        Mfull = self.scalar_mass_full()
        Kfull = self._assemble_nodes(self.element_stiffness())
        f = self.free
        M = Mfull[f][:, f].tocsr()
        K = (nu * Kfull[f][:, f]).tocsr()
        C = None
        if wind_nodal is not None:
            C = self._assemble_nodes(self.element_convection(wind_nodal))[f][:, f].tocsr()
        return M, K, C, Mfull[f].tocsr()

    def divergence_full(self) -> list[sp.csr_matrix]:
        """B_c over all P2 nodes (rows) and vertices (columns), one per component."""
        E = self.element_divergence()
        nl = self.cell_nodes.shape[1]
        out = []
        for k in range(self.dim):
            rows = np.repeat(self.cell_nodes, self.dim + 1, axis=1).ravel()
            cols = np.tile(self.cells, (1, nl)).ravel()
            out.append(sp.coo_matrix((E[:, :, k, :].ravel(), (rows, cols)), shape=(self.nnodes, self.nverts)).tocsr())
        return out

    def divergence(self) -> sp.csr_matrix:
        """B: component-blocked free velocity rows x vertex columns."""
        Bc = self.divergence_full()
        return sp.vstack([B[self.free] for B in Bc]).tocsr()

    # ------------------------------------------------------------------ errors
    def l2_norm_p2(self, nodal: np.ndarray, exact=None, t: float = 0.0) -> float:
        """L2 norm of (P2 field given by nodal values) - exact (callable or None)."""
        xi, w = simplex_quadrature(self.dim)
        val, _ = p2_basis(self.dim, xi)
        uq = np.einsum("qn,cnk->cqk", val, nodal[self.cell_nodes])
        if exact is not None:
            x0 = self.xyz[self.cells[:, 0]]
            xq = x0[:, None, :] + np.einsum("cij,qj->cqi", self.jac, xi)
            ex = exact(xq.reshape(-1, self.dim), t).reshape(uq.shape)
            uq = uq - ex
        return float(np.sqrt(np.einsum("q,cqk,c->", w, uq**2, self.detj)))

    def p1_integral(self, p: np.ndarray) -> float:
        return float(np.sum(p[self.cells].mean(axis=1) * self.detj) / np.prod(range(1, self.dim + 1)))

    def l2_norm_p1(self, p: np.ndarray) -> float:
        xi, w = simplex_quadrature(self.dim)
        psi = p1_basis(self.dim, xi)
        pq = np.einsum("qi,ci->cq", psi, p[self.cells])
        return float(np.sqrt(np.einsum("q,cq,c->", w, pq**2, self.detj)))

    def volume(self) -> float:
        return float(self.detj.sum() / np.prod(range(1, self.dim + 1)))
