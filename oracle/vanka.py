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

Chebyshev relaxation (Sec. 5.1): the paper accelerates the undamped additive operator
S = sum_v R_v^T A_v^{-1} R_v with Chebyshev polynomials of the first kind on a fixed
interval [lo, hi] of the spectrum of S J ([2, 8] for its 2D Stokes runs).  The steps
follow the classical Chebyshev semi-iteration: with theta = (hi + lo)/2,
delta = (hi - lo)/2, sigma = theta/delta and r_j = F - J k_j,
    d_0 = S r_0 / theta,                 rho_0 = 1/sigma,
    rho_j = 1/(2 sigma - rho_{j-1}),     d_j = rho_j rho_{j-1} d_{j-1} + (2 rho_j/delta) S r_j,
    k_{j+1} = k_j + d_j,
so that after m steps the error is T_m((theta - S J)/delta) / T_m(theta/delta) times
the initial error (T_m the Chebyshev polynomial of the first kind).  The transposed
relaxation (adjoint) is the same recurrence with J^T and S^T.

GMRES relaxation (Sec. 4.2: several steps of a Vanka-preconditioned GMRES iteration as
the relaxation; Sec. 5.4 uses 3 such pre- and post-steps for its convective problem).
The paper leaves the GMRES variant open; the reading here is one cycle of m steps of
left-preconditioned GMRES on J k = F with the additive operator S, from the current k:
with r_0 = F - J k and beta = ||S r_0||, v_0 = S r_0 / beta and for j < m the Arnoldi
step w = S J v_j, h_ij = <w, v_i> for i <= j against the unmodified w (classical
Gram--Schmidt), w -= sum_i h_ij v_i, h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j};
then y minimises ||beta e_1 - H y|| over the (m+1) x m Hessenberg H and
k <- k + sum_j y_j v_j.  A zero h_{j+1,j} (the Krylov space is invariant) ends the
cycle with the j+1 steps taken; beta = 0 leaves k unchanged.  The result depends
nonlinearly on F, so the V-cycle is a nonlinear preconditioner and the outer
iteration must be flexible (Sec. 4.1).  The transposed relaxation uses J^T and S^T.

Spectrum estimate for the Chebyshev interval (Sec. 5.1 takes [lambda_max/4, lambda_max],
lambda_max the largest eigenvalue of S J): m Arnoldi steps on M = S J from a given
start vector, classical Gram--Schmidt as in the GMRES relaxation, and the Ritz values,
the eigenvalues of the leading m x m block of the Hessenberg matrix.

Pinned by tests/test_oracle_vanka.py against: Fig. 1's patch (19 velocity nodes and
one pressure node for an interior vertex); the DOF cover; single-patch exactness
(R_v^T A_v^{-1} R_v J e = e for e supported on S_v); multiplicity bounds; the
Chebyshev error polynomial in closed form on a diagonal operator; the Ritz values
against the eigenvalues of V^T M V for an orthonormal basis V of the Krylov space built
from its power basis, and against the exact spectrum when m reaches the dimension; the GMRES relaxation
against the minimal-residual step in closed form (m = 1), against a least-squares
solve over the power basis of the Krylov space (m = 3), and against the exact solution
when m reaches the dimension.
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

    def apply_S(self, res: np.ndarray, transpose: bool = False) -> np.ndarray:
        """The (weighted) additive operator W sum_v R_v^T A_v^{-1} R_v, or its transpose."""
        W = self.W.astype(self.dtype)
        if transpose:
            return self.patch_sum(W * res, transpose=True)
        return W * self.patch_sum(res)

    def chebyshev(self, F: np.ndarray, k: np.ndarray, Jop, steps: int, lo: float, hi: float,
                  transpose: bool = False) -> np.ndarray:
        """Chebyshev relaxation (Sec. 5.1) on [lo, hi] with the additive operator; Jop is
        J (or J^T for the transposed relaxation) in the working precision."""
        return chebyshev_iteration(lambda x: Jop @ x, lambda r: self.apply_S(r, transpose), F, k, steps, lo, hi,
                                   self.dtype)

    def gmres(self, F: np.ndarray, k: np.ndarray, Jop, steps: int, transpose: bool = False) -> np.ndarray:
        """GMRES relaxation (module docstring) with the additive operator; Jop is J (or
        J^T for the transposed relaxation) in the working precision."""
        return gmres_relaxation(lambda x: Jop @ x, lambda r: self.apply_S(r, transpose), F, k, steps, self.dtype)

    def sweep(self, F: np.ndarray, k: np.ndarray, Jop, transpose: bool = False) -> np.ndarray:
        """One additive sweep on k, returning the new k.  Jop is the level operator in
        the working precision (J itself, or J^T for the transposed smoother)."""
        W = self.W.astype(self.dtype)
        res = F - Jop @ k
        if transpose:
            return k + self.dtype(self.omega) * self.patch_sum(W * res, transpose=True)
        return k + self.dtype(self.omega) * (W * self.patch_sum(res))


def chebyshev_iteration(apply_J, apply_S, F, k, steps: int, lo: float, hi: float, dtype=np.float64):
    """`steps` Chebyshev-accelerated steps for J k = F preconditioned by S, for the
    spectrum interval [lo, hi] of S J (recurrence in the module docstring)."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    k = np.array(k, dtype=dtype)
    d = None
    rho = None
    for j in range(steps):
        z = apply_S(np.asarray(F, dtype=dtype) - apply_J(k))
        if j == 0:
            rho = 1.0 / sigma
            d = dtype(1.0 / theta) * z
        else:
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = dtype(rho_new * rho) * d + dtype(2.0 * rho_new / delta) * z
            rho = rho_new
        k = k + d
    return k


def gmres_relaxation(apply_J, apply_S, F, k, steps: int, dtype=np.float64):
    """One cycle of `steps` left-preconditioned GMRES steps for J k = F from k
    (Arnoldi with classical Gram--Schmidt, Hessenberg least squares; module docstring).
    Vectors are kept in `dtype`, inner products and the small problem in float64."""
    k = np.array(k, dtype=dtype)
    z = apply_S(np.asarray(F, dtype=dtype) - apply_J(k))
    beta = float(np.linalg.norm(z.astype(np.float64)))
    if steps <= 0 or beta == 0.0:
        return k
    V = [(z / dtype(beta)).astype(dtype)]
    H = np.zeros((steps + 1, steps))
    m = steps
    for j in range(steps):
        w = apply_S(apply_J(V[j]))
        h = np.array([float(np.dot(V[i].astype(np.float64), w.astype(np.float64))) for i in range(j + 1)])
        for i in range(j + 1):
            w = w - dtype(h[i]) * V[i]
        H[:j + 1, j] = h
        H[j + 1, j] = float(np.linalg.norm(w.astype(np.float64)))
        if H[j + 1, j] == 0.0:
            m = j + 1
            break
        V.append((w / dtype(H[j + 1, j])).astype(dtype))
    e1 = np.zeros(m + 1)
    e1[0] = beta
    y = np.linalg.lstsq(H[:m + 1, :m], e1, rcond=None)[0]
    for j in range(m):
        k = k + dtype(y[j]) * V[j]
    return k


def arnoldi_ritz(apply_J, apply_S, v0, steps: int):
    """Hessenberg matrix H ((steps+1) x steps) of `steps` Arnoldi steps on M = S J from v0
    (classical Gram--Schmidt) and the Ritz values, eigenvalues of H[:steps, :steps] sorted
    by decreasing real part (module docstring).  Stops early at an invariant subspace."""
    v = np.asarray(v0, dtype=np.float64)
    V = [v / np.linalg.norm(v)]
    H = np.zeros((steps + 1, steps))
    m = steps
    for j in range(steps):
        w = apply_S(apply_J(V[j]))
        h = np.array([V[i] @ w for i in range(j + 1)])
        for i in range(j + 1):
            w = w - h[i] * V[i]
        H[:j + 1, j] = h
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:
            m = j + 1
            break
        V.append(w / H[j + 1, j])
    ritz = np.linalg.eigvals(H[:m, :m])
    return H[:m + 1, :m], ritz[np.argsort(-ritz.real, kind="stable")]
