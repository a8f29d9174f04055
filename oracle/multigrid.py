"""Monolithic geometric multigrid V-cycle for the stage system (Sec. 4.1-4.2, 5.1).

TEST INFRASTRUCTURE ONLY (oracle).

Hierarchy from uniform refinement; coarse operators by rediscretisation (assembly of
the stage system on every level, Sec. 4.1); interpolation I_r (x) P, restriction its
transpose; additive Vanka relaxation with `pre` and `post` sweeps, Chebyshev
steps (Sec. 5.1 uses 2 and 2) or GMRES steps (Sec. 5.4 uses 3 and 3); direct solve
on the coarsest level (Sec. 4.1 uses a
sparse direct solver; here a dense LU with partial pivoting).

Readings where the paper is silent:
  * cycle shape: on each level, pre-sweeps from a zero guess, residual, restrict,
    recurse, prolongate-and-add without damping, post-sweeps;
  * pressure nullspace: the coarse LU pins the pressure at vertex 0 of every stage
    (its row and column replaced by the identity, right-hand side entry 0), and the
    V-cycle output has each stage's pressure mean removed;
  * the wind of the Oseen operator is interpolated on each level (evaluated at that
    level's P2 nodes).

Mixed precision: with dtype=float32 the level operators, patch inverses and
vectors of the V-cycle are float32 and the coarse solve stays float64, as in the
FP32-patch variant of the HIP library.

Pinned by tests/test_oracle_vcycle_propagator.py: V J equals the textbook error
propagator G^post (I - P B_c P^T J) G^pre (G = I - omega W S J, B_c the coarser cycle),
assembled from dense matrices, for two- and three-level cycles, unequal pre/post
counts, Oseen operators and Chebyshev relaxation (whose factor is the closed-form
Chebyshev polynomial of S J); one sweep against k + omega W S (F - J k); two-grid and
V-cycle contraction (spectral radius about 0.3).  By tests/test_oracle_multigrid.py:
coarse solve residual; FGMRES-MG solution equal to the dense direct solve;
mesh-independent iteration counts.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fem import TaylorHood
from .stage import StageSystem
from .transfer import interpolation_matrices, stage_prolongation
from .vanka import VankaSmoother, patch_dofs

# Optional callable(str) told when each stage of a hierarchy's construction finishes (for
# callers that must show progress during a long setup); it does not affect the results.
PROGRESS = None


def _progress(msg):
    if PROGRESS is not None:
        PROGRESS(msg)


class Hierarchy:
    def __init__(self, mesh_levels, A, dt, nu, wind=None, omega=0.5, weighted=True, pre=2, post=2,
                 dtype=np.float64, smoother="sweep", interval=(2.0, 8.0), level_operators=None):
        """mesh_levels: coarse-to-fine sequence of objects with .xyz and .cells.
        wind: callable (points, t) -> (npts, dim) or None (Stokes).
        smoother: "sweep" (damped additive sweeps, omega and weighting), "chebyshev"
        (Chebyshev relaxation on `interval` with the additive operator, Sec. 5.1) or
        "gmres" (`pre`/`post` steps of GMRES preconditioned by the additive operator,
        Sec. 4.2, 5.4).
        level_operators: None (each level's operator is its StageSystem's J) or a
        callable (level, StageSystem) -> sparse operator of that level with the same
        unknowns, e.g. the Newton Jacobian of Sec. 3.2 rediscretised on the level; the
        relaxation, the coarse solve and the cycle then use those operators (self.ops)."""
        self.A = np.asarray(A, dtype=np.float64)
        self.r = self.A.shape[0]
        self.pre, self.post = pre, post
        if smoother not in ("sweep", "chebyshev", "gmres"):
            raise ValueError("smoother must be 'sweep', 'chebyshev' or 'gmres'")
        self.smoother, self.interval = smoother, (float(interval[0]), float(interval[1]))
        self.dtype = dtype
        self.spaces = [TaylorHood(m.xyz, m.cells) for m in mesh_levels]
        self.systems = []
        for th in self.spaces:
            wn = th.interpolate(wind) if wind is not None else None
            self.systems.append(StageSystem(th, self.A, dt, nu, wn))
            _progress(f"oracle: level with {th.ncells} cells assembled")
        self.dim = self.spaces[0].dim
        self.P = [None]
        for lc in range(len(self.spaces) - 1):
            Pu, Pp = interpolation_matrices(self.spaces[lc], self.spaces[lc + 1])
            self.P.append(stage_prolongation(Pu, Pp, self.dim, self.r))
        self.smoothers = [None]
        if level_operators is None:
            self.ops = [s.J for s in self.systems]
        else:
            self.ops = [level_operators(lev, s).tocsr() for lev, s in enumerate(self.systems)]
        self.Jw = [J.astype(dtype) for J in self.ops]
        self.Pw = [None] + [P.astype(dtype) for P in self.P[1:]]
        for lev in range(1, len(self.spaces)):
            pat = patch_dofs(self.spaces[lev], self.r)
            self.smoothers.append(VankaSmoother(self.ops[lev], pat, omega, weighted, dtype))
            _progress(f"oracle: patch inverses of level {lev} computed")
        # coarse LU with one pinned pressure per stage
        s0 = self.systems[0]
        Jc = self.ops[0].toarray()
        self.pinned = [i * s0.ns + s0.th.nvel for i in range(self.r)]
        for q in self.pinned:
            Jc[q, :] = 0.0
            Jc[:, q] = 0.0
            Jc[q, q] = 1.0
        self.coarse_lu = sla.lu_factor(Jc)
        self.coarse_luT = sla.lu_factor(Jc.T.copy())

    @property
    def finest(self) -> StageSystem:
        return self.systems[-1]

    def coarse_solve(self, b: np.ndarray, transpose: bool = False) -> np.ndarray:
        b = np.array(b, dtype=np.float64)
        b[self.pinned] = 0.0
        return sla.lu_solve(self.coarse_luT if transpose else self.coarse_lu, b)

    def _cycle(self, lev: int, b: np.ndarray, transpose: bool) -> np.ndarray:
        if lev == 0:
            return self.coarse_solve(b, transpose).astype(self.dtype)
        Jop = self.Jw[lev].T if transpose else self.Jw[lev]
        sm = self.smoothers[lev]
        npre, npost = (self.post, self.pre) if transpose else (self.pre, self.post)
        x = np.zeros_like(b)
        x = self._relax(sm, b, x, Jop, npre, transpose)
        res = b - Jop @ x
        bc = self.Pw[lev].T @ res
        x = x + self.Pw[lev] @ self._cycle(lev - 1, bc, transpose)
        return self._relax(sm, b, x, Jop, npost, transpose)

    def _relax(self, sm, b, x, Jop, steps, transpose):
        if self.smoother == "chebyshev":
            return sm.chebyshev(b, x, Jop, steps, *self.interval, transpose) if steps > 0 else x
        if self.smoother == "gmres":
            return sm.gmres(b, x, Jop, steps, transpose) if steps > 0 else x
        for _ in range(steps):
            x = sm.sweep(b, x, Jop, transpose)
        return x

    def vcycle(self, b: np.ndarray) -> np.ndarray:
        """z = V b from a zero initial guess, pressure means removed."""
        z = self._cycle(len(self.spaces) - 1, np.asarray(b).astype(self.dtype), False).astype(np.float64)
        return self.finest.project_pressure_mean(z)

    def vcycle_transpose(self, b: np.ndarray) -> np.ndarray:
        """V^T b: the transpose of vcycle as a linear map (projection first, then the
        V-cycle of J^T with transposed patch solves and swapped sweep counts)."""
        b = self.finest.project_pressure_mean(np.asarray(b, dtype=np.float64))
        return self._cycle(len(self.spaces) - 1, b.astype(self.dtype), True).astype(np.float64)
