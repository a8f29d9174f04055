"""Canonical finite-element interpolation between nested meshes (Sec. 4.1).

TEST INFRASTRUCTURE ONLY (oracle).

P = diag(P_u, P_p): P_u evaluates a coarse P2 function at the fine P2 nodes (per
component), P_p a coarse P1 function at the fine vertices.  The stage operator is
I_r (x) P and restriction is its transpose.  Coarse cells are found by point location
(nearest coarse centroids, then the barycentric inside-test) — the fine mesh's parent
map is deliberately not used.  Rows and columns of eliminated (boundary) velocity
nodes are dropped: a fine boundary node lies on a coarse boundary facet, so its
interpolated value involves coarse boundary nodes only, all zero.

Pinned by tests/test_oracle_transfer.py against: exact reproduction of coarse
quadratics / linears at fine nodes; the Galerkin identity P^T J_f P = J_c (the paper
notes that rediscretisation equals Galerkin coarsening for compatible quadrature).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .fem import LOCAL_EDGES, TaylorHood


def _locate(coarse: TaylorHood, pts: np.ndarray, k: int = 12) -> tuple[np.ndarray, np.ndarray]:
    """Containing coarse cell and barycentric coordinates for each point."""
    d = coarse.dim
    cen = coarse.xyz[coarse.cells].mean(axis=1)
    tree = cKDTree(cen)
    _, cand = tree.query(pts, k=min(k, coarse.ncells))
    cell = -np.ones(len(pts), dtype=np.int64)
    bary = np.zeros((len(pts), d + 1))
    best = np.full(len(pts), -np.inf)
    for j in range(cand.shape[1]):
        c = cand[:, j]
        x0 = coarse.xyz[coarse.cells[c, 0]]
        jinv = np.linalg.inv(coarse.jac[c])
        xi = np.einsum("pij,pj->pi", jinv, pts - x0)
        lam = np.hstack([1.0 - xi.sum(axis=1, keepdims=True), xi])
        score = lam.min(axis=1)
        better = score > best
        best[better] = score[better]
        cell[better] = c[better]
        bary[better] = lam[better]
    assert np.all(best > -1e-10), "point location failed"
    return cell, bary


def p2_values(lam: np.ndarray, dim: int) -> np.ndarray:
    """P2 basis values from barycentric coordinates (npts, dim+1)."""
    vals = [lam[:, i] * (2 * lam[:, i] - 1) for i in range(dim + 1)]
    vals += [4 * lam[:, i] * lam[:, j] for i, j in LOCAL_EDGES[dim]]
    return np.stack(vals, axis=1)


def interpolation_matrices(coarse: TaylorHood, fine: TaylorHood) -> tuple[sp.csr_matrix, sp.csr_matrix]:
    """Scalar P2 interpolation (fine free nodes x coarse free nodes) and P1
    interpolation (fine vertices x coarse vertices)."""
    d = coarse.dim
    cell, lam = _locate(coarse, fine.node_xyz[fine.free])
    w = p2_values(lam, d)
    cols = coarse.cell_nodes[cell]
    rows = np.repeat(np.arange(fine.nfree), cols.shape[1])
    full = sp.coo_matrix((w.ravel(), (rows, cols.ravel())), shape=(fine.nfree, coarse.nnodes)).tocsr()
    Pu = full[:, coarse.free].tocsr()
    Pu.data[np.abs(Pu.data) < 1e-14] = 0.0
    Pu.eliminate_zeros()

    cell, lam = _locate(coarse, fine.xyz)
    cols = coarse.cells[cell]
    rows = np.repeat(np.arange(fine.nverts), d + 1)
    Pp = sp.coo_matrix((lam.ravel(), (rows, cols.ravel())), shape=(fine.nverts, coarse.nverts)).tocsr()
    Pp.data[np.abs(Pp.data) < 1e-14] = 0.0
    Pp.eliminate_zeros()
    return Pu, Pp


def stage_prolongation(Pu: sp.csr_matrix, Pp: sp.csr_matrix, dim: int, r: int) -> sp.csr_matrix:
    """I_r (x) diag(I_d (x) P_u, P_p) in the stage-major, component-blocked layout."""
    P1 = sp.block_diag([sp.kron(sp.identity(dim), Pu), Pp])
    return sp.kron(sp.identity(r), P1).tocsr()
