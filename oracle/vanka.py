"""Vertex-star Vanka patches and the additive Schwarz sweep (Sec. 4.2).

TEST INFRASTRUCTURE ONLY (oracle).

Patch S_v (Sec. 4.2, Fig. 1): every free velocity DOF on the closure of the cells
around vertex v, plus the single pressure DOF at v, for every RK stage.  One patch per
vertex, boundary vertices included.  With R_v the restriction to S_v, one sweep is

    k <- k + omega * W * sum_v R_v^T (R_v J R_v^T)^{-1} R_v (F - J k),

the weighted stationary iteration of Sec. 4.2.  W = I is the literal form.  The paper
wraps the undamped operator in Chebyshev acceleration; for the plain damped sweep the
reading taken here also offers W = D^{-1}, D the number of patches containing each
DOF (a partition of unity), because the undamped operator has eigenvalues up to the
overlap count (about 7 in 2D) and omega = 0.5 alone then amplifies the top modes.
The transposed sweep (for adjoint solves) uses omega * sum_v R_v^T A_v^{-T} R_v W.

Pinned by tests/test_oracle_vanka.py against: Fig. 1's patch (19 velocity nodes and
one pressure node for an interior vertex); the DOF cover; single-patch exactness
(R_v^T A_v^{-1} R_v J e = e for e supported on S_v); multiplicity bounds.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import TaylorHood


def patch_dofs(th: TaylorHood, r: int) -> list[np.ndarray]:
    """Sorted global DOF indices (stage-major layout) of every vertex patch."""
    ns = th.nstage
    nvel = th.nvel
    cells_of_vertex = [[] for _ in range(th.nverts)]
    for c, verts in enumerate(th.cells):
        for v in verts:
            cells_of_vertex[v].append(c)
    out = []
    for v in range(th.nverts):
        nodes = np.unique(th.cell_nodes[cells_of_vertex[v]].ravel())
        fidx = th.free_index[nodes]
        fidx = fidx[fidx >= 0]
        stage_block = np.concatenate([c * th.nfree + fidx for c in range(th.dim)] + [np.array([nvel + v])])
        out.append(np.sort(np.concatenate([i * ns + stage_block for i in range(r)])))
    return out


def multiplicity(patches: list[np.ndarray], n: int) -> np.ndarray:
    D = np.zeros(n)
    for idx in patches:
        D[idx] += 1.0
    return D


class VankaSmoother:
    """Stored dense patch inverses for one level, grouped by patch size so that the
    sum over patches can use batched products; the sum itself is unchanged."""

    def __init__(self, J: sp.csr_matrix, patches: list[np.ndarray], omega: float, weighted: bool, dtype=np.float64):
        self.J = J
        self.omega = float(omega)
        self.n = J.shape[0]
        self.weighted = weighted
        self.W = 1.0 / multiplicity(patches, self.n) if weighted else np.ones(self.n)
        self.dtype = dtype
        groups: dict[int, list[int]] = {}
        for p, idx in enumerate(patches):
            groups.setdefault(idx.size, []).append(p)
        self.groups = []
        Jc = J.tocsr()
        for size, plist in sorted(groups.items()):
            idx = np.stack([patches[p] for p in plist])
            mats = np.stack([Jc[i][:, i].toarray() for i in idx])
            inv = np.linalg.inv(mats).astype(dtype)
            self.groups.append((idx, inv))

    def patch_sum(self, res: np.ndarray, transpose: bool = False) -> np.ndarray:
        """sum_v R_v^T A_v^{-1} R_v res (A_v^{-T} when transpose), in self.dtype."""
        out = np.zeros(self.n, dtype=self.dtype)
        res = res.astype(self.dtype)
        for idx, inv in self.groups:
            loc = res[idx]
            sub = "pji,pj->pi" if transpose else "pij,pj->pi"
            np.add.at(out, idx, np.einsum(sub, inv, loc))
        return out

    def sweep(self, F: np.ndarray, k: np.ndarray, Jop, transpose: bool = False) -> np.ndarray:
        """One additive sweep on k, returning the new k.  Jop is the level operator in
        the working precision (J itself, or J^T for the transposed smoother)."""
        W = self.W.astype(self.dtype)
        res = F - Jop @ k
        if transpose:
            return k + self.dtype(self.omega) * self.patch_sum(W * res, transpose=True)
        return k + self.dtype(self.omega) * (W * self.patch_sum(res))
