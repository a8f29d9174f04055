"""Seeded synthetic workloads: meshes, random coefficients and analytic fields.

This module is the only code that both the HIP path and the CPU checker use.  It
holds workload *definitions* only: structured simplicial meshes of the unit square
and unit cube with the parent maps of their nested refinements, the random draws
that fix each synthetic problem, and analytic vector fields (forcing, manufactured
solution, wind) evaluated at caller-supplied points.  It contains none of the
solver's arithmetic: no finite-element basis, quadrature, assembly, interpolation
operator, Runge--Kutta tableau or linear algebra.

Meshes follow Sec. 4.1 of the paper (hierarchies from uniform refinement of a
coarsest grid).  The 2D mesh splits every quad along the diagonal from its
lower-right to its upper-left corner, the orientation drawn in Fig. 1; the 3D mesh
is the Kuhn split of each cube into 6 tetrahedra (Sec. 5.4 cuts hexahedra into six).
Both families are nested: the mesh at 2n is the red refinement of the mesh at n.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np


@dataclass
class MeshLevel:
    """One level of a nested simplicial hierarchy.

    xyz:    (nverts, dim) float64 vertex coordinates.
    cells:  (ncells, dim+1) int64 vertex indices.
    parent: (ncells,) int64 index of the coarse cell containing each cell, or None
            on the coarsest level.
    """

    dim: int
    xyz: np.ndarray
    cells: np.ndarray
    parent: np.ndarray | None


# ----------------------------------------------------------------------------- 2D
def square_mesh(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n x n quads of the unit square, each cut into two triangles.

    Vertex (i, j) has index j*(n+1) + i and sits at (i/n, j/n).  Quad (i, j) gives
    cells 2*(j*n+i) (lower-left triangle) and 2*(j*n+i)+1 (upper-right triangle),
    split along the diagonal (i+1, j)-(i, j+1).
    """
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    xyz = np.stack([ii.ravel() / n, jj.ravel() / n], axis=1).astype(np.float64)
    qi, qj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    v00 = (qj * (n + 1) + qi).ravel()
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    lower = np.stack([v00, v10, v01], axis=1)
    upper = np.stack([v10, v11, v01], axis=1)
    cells = np.empty((2 * n * n, 3), dtype=np.int64)
    cells[0::2] = lower
    cells[1::2] = upper
    return xyz, cells


def _square_parent(n_fine: int) -> np.ndarray:
    """Coarse cell (mesh at n_fine/2) containing each cell of the mesh at n_fine."""
    nc = n_fine // 2
    xyz, cells = square_mesh(n_fine)
    cen = xyz[cells].mean(axis=1) * nc  # centroid in coarse-quad units
    qi = np.floor(cen[:, 0]).astype(np.int64)
    qj = np.floor(cen[:, 1]).astype(np.int64)
    fx = cen[:, 0] - qi
    fy = cen[:, 1] - qj
    upper = (fx + fy > 1.0).astype(np.int64)
    return 2 * (qj * nc + qi) + upper


def square_hierarchy(n_coarse: int, nlevels: int) -> list[MeshLevel]:
    """Nested square meshes n_coarse * 2**l, l = 0..nlevels-1 (coarse to fine)."""
    levels = []
    for lev in range(nlevels):
        n = n_coarse * 2**lev
        xyz, cells = square_mesh(n)
        parent = _square_parent(n) if lev > 0 else None
        levels.append(MeshLevel(2, xyz, cells, parent))
    return levels


def crossed_mesh(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n x n quads of the unit square, each cut into four triangles by a vertex at its
    centre (the "crossed" mesh of Sec. 5.1).

    Corner vertex (i, j) has index j*(n+1) + i; the centre of quad (i, j) has index
    (n+1)**2 + j*n + i.  Quad (i, j) gives cells 4*(j*n+i) + 0..3: bottom, right, top,
    left, each listed counter-clockwise with the centre last.
    """
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    corners = np.stack([ii.ravel() / n, jj.ravel() / n], axis=1)
    qi, qj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    centres = np.stack([(qi.ravel() + 0.5) / n, (qj.ravel() + 0.5) / n], axis=1)
    xyz = np.concatenate([corners, centres]).astype(np.float64)
    v00 = (qj * (n + 1) + qi).ravel()
    v10, v01 = v00 + 1, v00 + (n + 1)
    v11 = v01 + 1
    c = (n + 1) ** 2 + (qj * n + qi).ravel()
    cells = np.empty((4 * n * n, 3), dtype=np.int64)
    cells[0::4] = np.stack([v00, v10, c], axis=1)
    cells[1::4] = np.stack([v10, v11, c], axis=1)
    cells[2::4] = np.stack([v11, v01, c], axis=1)
    cells[3::4] = np.stack([v01, v00, c], axis=1)
    return xyz, cells


def red_refine(xyz: np.ndarray, cells: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Uniform (red) refinement of a triangle mesh: every cell [a, b, c] becomes
    [a, m_ab, m_ca], [m_ab, b, m_bc], [m_ca, m_bc, c], [m_ab, m_bc, m_ca] (children
    4*cell + 0..3, orientation kept).  Coarse vertices keep their indices; edge midpoints
    follow in the order of the sorted edge list.  Returns (xyz, cells, parent)."""
    nv = xyz.shape[0]
    e = np.concatenate([cells[:, [0, 1]], cells[:, [1, 2]], cells[:, [2, 0]]])
    key = np.sort(e, axis=1)
    code = key[:, 0] * nv + key[:, 1]
    uniq, inv = np.unique(code, return_inverse=True)
    a, b = uniq // nv, uniq % nv
    mid = 0.5 * (xyz[a] + xyz[b])
    nc = cells.shape[0]
    m_ab, m_bc, m_ca = (nv + inv[:nc]), (nv + inv[nc:2 * nc]), (nv + inv[2 * nc:])
    c0, c1, c2 = cells[:, 0], cells[:, 1], cells[:, 2]
    fine = np.empty((4 * nc, 3), dtype=np.int64)
    fine[0::4] = np.stack([c0, m_ab, m_ca], axis=1)
    fine[1::4] = np.stack([m_ab, c1, m_bc], axis=1)
    fine[2::4] = np.stack([m_ca, m_bc, c2], axis=1)
    fine[3::4] = np.stack([m_ab, m_bc, m_ca], axis=1)
    parent = np.repeat(np.arange(nc, dtype=np.int64), 4)
    return np.concatenate([xyz, mid]), fine, parent


def crossed_hierarchy(n_coarse: int, nlevels: int) -> list[MeshLevel]:
    """The crossed n_coarse x n_coarse mesh and nlevels-1 uniform refinements of it
    (Sec. 5.1 uses n_coarse = 8 and refinement levels l = 5, 6, 7)."""
    xyz, cells = crossed_mesh(n_coarse)
    levels = [MeshLevel(2, xyz, cells, None)]
    for _ in range(nlevels - 1):
        xyz, cells, parent = red_refine(xyz, cells)
        levels.append(MeshLevel(2, xyz, cells, parent))
    return levels


def mesh_edges(cells: np.ndarray, nverts: int) -> np.ndarray:
    """(nedges, 2) vertex pairs (smaller, larger) of a simplicial mesh, sorted: the edge
    numbering of the library and the checker."""
    nb = cells.shape[1]
    pairs = np.concatenate([cells[:, [a, b]] for a in range(nb) for b in range(a + 1, nb)])
    key = np.sort(pairs, axis=1)
    code = np.unique(key[:, 0] * nverts + key[:, 1])
    return np.stack([code // nverts, code % nverts], axis=1)


def island_field(x: np.ndarray, k: float = 0.2, perturb: bool = True) -> np.ndarray:
    """The island-coalescence magnetic field of Sec. 5.3 (the equilibrium and, with
    perturb, the perturbation of its initial condition) at points x of the unit square,
    in the coordinates X = 2x - 1 of the paper's square (-1, 1)^2: (n, 2)."""
    X, Y = 2.0 * x[:, 0] - 1.0, 2.0 * x[:, 1] - 1.0
    den = np.cosh(2 * np.pi * Y) + k * np.cos(2 * np.pi * X)
    b = np.stack([np.sinh(2 * np.pi * Y), k * np.sin(2 * np.pi * X)], axis=1) / den[:, None]
    if perturb:
        b += (-0.01 / np.pi) * np.stack([-np.cos(np.pi * X) * np.sin(np.pi * Y / 2) / 2,
                                         np.cos(np.pi * Y / 2) * np.sin(np.pi * X)], axis=1)
    return b


def island_coalescence(xyz: np.ndarray, cells: np.ndarray, k: float = 0.2, perturb: bool = True,
                       npts: int = 8) -> tuple[np.ndarray, np.ndarray]:
    """Linearisation state of the 2D MHD workload on one mesh: the velocity w = 0 at the
    P2 nodes (vertices, then edges), (nverts + nedges, 2), and the line integrals of the
    island field along every edge from its smaller to its larger vertex (Gauss--Legendre
    with npts points), (nedges,)."""
    nv = xyz.shape[0]
    edges = mesh_edges(cells, nv)
    a, b = xyz[edges[:, 0]], xyz[edges[:, 1]]
    g, wg = np.polynomial.legendre.leggauss(npts)
    b0 = np.zeros(edges.shape[0])
    for t, wt in zip(0.5 * (g + 1.0), 0.5 * wg):
        b0 += wt * np.einsum("ek,ek->e", island_field(a + t * (b - a), k, perturb), b - a)
    return np.zeros((nv + edges.shape[0], 2)), b0


# ----------------------------------------------------------------------------- 3D
_KUHN_PERMS = list(itertools.permutations(range(3)))


def cube_mesh(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n^3 cubes of the unit cube, each split into the 6 Kuhn tetrahedra.

    Vertex (i, j, k) has index (k*(n+1) + j)*(n+1) + i.  Cube c, permutation p of
    (x, y, z) gives cell 6*c + p with vertices on the monotone lattice path
    corner -> corner+e_p0 -> corner+e_p0+e_p1 -> corner+(1,1,1).
    """
    g = np.arange(n + 1)
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64) / n
    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()

    def vid(i, j, k):
        return (k * (n + 1) + j) * (n + 1) + i

    cells = np.empty((6 * n**3, 4), dtype=np.int64)
    for p, perm in enumerate(_KUHN_PERMS):
        pos = np.zeros((3, ci.size), dtype=np.int64)
        path = [vid(ci, cj, ck)]
        for ax in perm:
            pos[ax] += 1
            path.append(vid(ci + pos[0], cj + pos[1], ck + pos[2]))
        cells[p::6] = np.stack(path, axis=1)
    return xyz, cells


def _cube_parent(n_fine: int) -> np.ndarray:
    nc = n_fine // 2
    xyz, cells = cube_mesh(n_fine)
    cen = xyz[cells].mean(axis=1) * nc
    q = np.floor(cen).astype(np.int64)
    f = cen - q
    # the Kuhn tetrahedron of a cube holding a point orders its local coordinates
    order = np.argsort(-f, axis=1, kind="stable")
    perm_index = {perm: idx for idx, perm in enumerate(_KUHN_PERMS)}
    p = np.array([perm_index[tuple(o)] for o in order], dtype=np.int64)
    cube = (q[:, 2] * nc + q[:, 1]) * nc + q[:, 0]
    return 6 * cube + p


def cube_hierarchy(n_coarse: int, nlevels: int) -> list[MeshLevel]:
    levels = []
    for lev in range(nlevels):
        n = n_coarse * 2**lev
        xyz, cells = cube_mesh(n)
        parent = _cube_parent(n) if lev > 0 else None
        levels.append(MeshLevel(3, xyz, cells, parent))
    return levels


# ------------------------------------------------------------------ analytic fields
@dataclass
class ModeForcing:
    """f(x) = sum_m sum_d theta[m, d] * prod_k trig_{m,d,k}(a[m,k] pi x_k) e_d.

    2D (the small-problem and Oseen forcing): component 0 uses sin(a x) cos(b y),
    component 1 uses cos(a x) sin(b y).  3D: every component uses
    sin(a x) sin(b y) sin(c z).  The field does not depend on time.
    """

    dim: int
    freqs: np.ndarray  # (nmodes, dim) integer frequencies
    theta: np.ndarray  # (nmodes, dim) coefficients

    def __call__(self, pts: np.ndarray, t: float = 0.0) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64)
        out = np.zeros((pts.shape[0], self.dim))
        for m in range(self.freqs.shape[0]):
            arg = np.pi * self.freqs[m][None, :] * pts
            s, c = np.sin(arg), np.cos(arg)
            if self.dim == 2:
                out[:, 0] += self.theta[m, 0] * s[:, 0] * c[:, 1]
                out[:, 1] += self.theta[m, 1] * c[:, 0] * s[:, 1]
            else:
                prod = s[:, 0] * s[:, 1] * s[:, 2]
                for d in range(3):
                    out[:, d] += self.theta[m, d] * prod
        return out

    def with_theta(self, theta: np.ndarray) -> "ModeForcing":
        return ModeForcing(self.dim, self.freqs, np.asarray(theta, dtype=np.float64).reshape(self.theta.shape))


def forcing_2d(seed: int) -> ModeForcing:
    """Eight modes, frequencies the first 8 pairs of {1,2,3}^2 in lexicographic
    order, 16 coefficients drawn N(0,1) from PCG64(seed) as an (8, 2) array."""
    pairs = np.array(list(itertools.product((1, 2, 3), repeat=2))[:8], dtype=np.int64)
    theta = np.random.default_rng(seed).standard_normal((8, 2))
    return ModeForcing(2, pairs, theta)


def forcing_3d(seed: int) -> ModeForcing:
    """Nine modes, frequencies the first 9 triples of {1,2,3}^3 ordered by
    (a+b+c, then lexicographic); 27 coefficients N(0,1) from PCG64(seed)."""
    trip = sorted(itertools.product((1, 2, 3), repeat=3), key=lambda t: (sum(t), t))[:9]
    theta = np.random.default_rng(seed).standard_normal((9, 3))
    return ModeForcing(3, np.array(trip, dtype=np.int64), theta)


@dataclass
class StreamMMS:
    """Manufactured Stokes solution from a stream function (2D).

    psi(x, y, t) = exp(-t) sum_m c_m sin^2(a_m pi x) sin^2(b_m pi y),
    u = (d psi/dy, -d psi/dx) (zero on the boundary, divergence free), p = 0,
    f = u_t - nu * Laplacian(u).
    """

    a: np.ndarray
    b: np.ndarray
    c: np.ndarray
    nu: float

    @staticmethod
    def _s(k, x):
        w = k * np.pi
        return (np.sin(w * x) ** 2, w * np.sin(2 * w * x), 2 * w**2 * np.cos(2 * w * x), -4 * w**3 * np.sin(2 * w * x))

    def velocity(self, pts: np.ndarray, t: float) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64)
        u = np.zeros((pts.shape[0], 2))
        for a, b, c in zip(self.a, self.b, self.c):
            sx = self._s(a, pts[:, 0])
            sy = self._s(b, pts[:, 1])
            u[:, 0] += c * sx[0] * sy[1]
            u[:, 1] -= c * sx[1] * sy[0]
        return np.exp(-t) * u

    def laplacian(self, pts: np.ndarray, t: float) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64)
        lap = np.zeros((pts.shape[0], 2))
        for a, b, c in zip(self.a, self.b, self.c):
            sx = self._s(a, pts[:, 0])
            sy = self._s(b, pts[:, 1])
            lap[:, 0] += c * (sx[2] * sy[1] + sx[0] * sy[3])
            lap[:, 1] -= c * (sx[3] * sy[0] + sx[1] * sy[2])
        return np.exp(-t) * lap

    def __call__(self, pts: np.ndarray, t: float = 0.0) -> np.ndarray:
        """The forcing f = u_t - nu Laplacian(u) (u_t = -u here)."""
        return -self.velocity(pts, t) - self.nu * self.laplacian(pts, t)


@dataclass
class StreamMMSInertial(StreamMMS):
    """The same velocity and pressure (p = 0) as an exact solution of the Navier--Stokes
    equations: f = u_t + (u . grad) u - nu Laplacian(u), with (u . grad) u written out
    from the stream function (u = (psi_y, -psi_x))."""

    amp: float = 1.0

    def velocity(self, pts: np.ndarray, t: float) -> np.ndarray:
        return self.amp * super().velocity(pts, t)

    def laplacian(self, pts: np.ndarray, t: float) -> np.ndarray:
        return self.amp * super().laplacian(pts, t)

    def inertia(self, pts: np.ndarray, t: float) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64)
        px, py, pxx, pyy, pxy = (np.zeros(pts.shape[0]) for _ in range(5))
        for a, b, c in zip(self.a, self.b, self.c):
            sx = self._s(a, pts[:, 0])
            sy = self._s(b, pts[:, 1])
            px += c * sx[1] * sy[0]
            py += c * sx[0] * sy[1]
            pxx += c * sx[2] * sy[0]
            pyy += c * sx[0] * sy[2]
            pxy += c * sx[1] * sy[1]
        g = self.amp * np.exp(-t)
        px, py, pxx, pyy, pxy = (g * v for v in (px, py, pxx, pyy, pxy))
        out = np.zeros((pts.shape[0], 2))
        out[:, 0] = py * pxy - px * pyy
        out[:, 1] = -py * pxx + px * pxy
        return out

    def __call__(self, pts: np.ndarray, t: float = 0.0) -> np.ndarray:
        return -self.velocity(pts, t) - self.nu * self.laplacian(pts, t) + self.inertia(pts, t)


def mms_ns_2d(seed: int, nu: float, amp: float, nmodes: int = 4) -> StreamMMSInertial:
    """Draws as mms_2d (fewer modes by default), velocity scaled by amp."""
    m = mms_2d(seed, nu, nmodes)
    return StreamMMSInertial(m.a, m.b, m.c, nu, amp)


def mms_2d(seed: int, nu: float = 1.0, nmodes: int = 16) -> StreamMMS:
    """Draw order from PCG64(seed): a (nmodes ints in 1..4), b (same), then
    c ~ N(0,1), scaled by 1/(a^2+b^2)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(1, 5, nmodes)
    b = rng.integers(1, 5, nmodes)
    c = rng.standard_normal(nmodes) / (a**2 + b**2)
    return StreamMMS(a.astype(np.float64), b.astype(np.float64), c, nu)


@dataclass
class StreamWind:
    """w = scale * curl psi_w, psi_w = sum_m c_m sin(a_m pi x) sin(b_m pi y)."""

    a: np.ndarray
    b: np.ndarray
    c: np.ndarray
    scale: float

    def __call__(self, pts: np.ndarray, t: float = 0.0) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64)
        w = np.zeros((pts.shape[0], 2))
        for a, b, c in zip(self.a, self.b, self.c):
            ax, by = a * np.pi, b * np.pi
            w[:, 0] += c * by * np.sin(ax * pts[:, 0]) * np.cos(by * pts[:, 1])
            w[:, 1] -= c * ax * np.cos(ax * pts[:, 0]) * np.sin(by * pts[:, 1])
        return self.scale * w


def wind_2d(seed: int, n_lattice: int, nmodes: int = 32) -> StreamWind:
    """Draw order from PCG64(seed): a, b (ints in 1..8), c ~ N(0,1)/(a^2+b^2)^1.5.
    The field is scaled so that its largest speed over the lattice of spacing
    1/(2 n_lattice) is 1 (for the n_lattice x n_lattice mesh these lattice points
    are exactly the quadratic nodes)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(1, 9, nmodes).astype(np.float64)
    b = rng.integers(1, 9, nmodes).astype(np.float64)
    c = rng.standard_normal(nmodes) / (a**2 + b**2) ** 1.5
    raw = StreamWind(a, b, c, 1.0)
    g = np.arange(2 * n_lattice + 1) / (2 * n_lattice)
    gx, gy = np.meshgrid(g, g, indexing="xy")
    speed = np.linalg.norm(raw(np.stack([gx.ravel(), gy.ravel()], axis=1)), axis=1)
    return StreamWind(a, b, c, 1.0 / speed.max())


@dataclass
class ConstantField:
    value: np.ndarray

    def __call__(self, pts: np.ndarray, t: float = 0.0) -> np.ndarray:
        return np.broadcast_to(np.asarray(self.value, dtype=np.float64), (np.asarray(pts).shape[0], len(self.value))).copy()


def random_vector(n: int, seed: int) -> np.ndarray:
    """N(0,1) draws from PCG64(seed), used as residuals and initial guesses."""
    return np.random.default_rng(seed).standard_normal(n)


@dataclass
class BatchSolveSpec:
    n: int        # finest mesh is n x n (levels from a 4 x 4 coarsest mesh)
    r: int        # RadauIIA stages
    nu: float
    dt: float
    forcing_seed: int


def batch_specs(seed: int = 4, count: int = 64, dt: float = 1e-2) -> list[BatchSolveSpec]:
    """Uneven batch: n ~ U{32, 64, 128, 256}, r ~ U{2, 3}, nu = 10^U(-2, 0), drawn in
    that order per solve from PCG64(seed); solve j uses the 2D forcing with seed
    4000 + j."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(rng.choice([32, 64, 128, 256]))
        r = int(rng.integers(2, 4))
        nu = float(10.0 ** rng.uniform(-2.0, 0.0))
        out.append(BatchSolveSpec(n, r, nu, dt, 4000 + j))
    return out
