"""Thin ctypes binding of libirkmg (include/irk_mg.h, include/irk_mhd.h).

Argument marshalling only: every step of the method runs in the HIP library.  Names
follow the C ABI.  Device vectors are torch float64 CUDA tensors; the current torch
stream is passed to every call.  Importing this module loads ``libirkmg.so`` and fails
loudly if it has not been built (``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

# torch is imported before libirkmg.so is loaded: torch ships its own HIP runtime under
# the same soname (libamdhip64.so.7) but links it by another name, so loading
# libirkmg.so first (which resolves ROCm's copy) would put two HIP and HSA runtimes in
# one process and leave the GPU unusable (hipErrorNoDevice).  Loaded in this order, the
# library binds to the runtime torch already holds and both share its device pointers
# and streams.
import torch  # noqa: F401,E402

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libirkmg.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "irk_mg.h")
MHD_HEADER = os.path.join(os.path.dirname(_HERE), "include", "irk_mhd.h")

IRK_OK, IRK_EINVAL, IRK_ENOMEM, IRK_EHIP, IRK_ESINGULAR, IRK_ENAN, IRK_ENOCONV = 0, -1, -2, -3, -4, -5, 1
FAMILIES = {"radauIIA": 0, "gauss": 1, "lobattoIIIC": 2}


class IrkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"irk status {status}: {msg}")
        self.status = status


class irk_mesh_level(C.Structure):
    _fields_ = [("dim", C.c_int), ("nverts", C.c_int64), ("ncells", C.c_int64),
                ("xyz", C.c_void_p), ("cells", C.c_void_p), ("parent", C.c_void_p)]


class irk_tableau(C.Structure):
    _fields_ = [("r", C.c_int), ("A", C.c_void_p), ("b", C.c_void_p), ("c", C.c_void_p)]


class irk_mg_opts(C.Structure):
    _fields_ = [("pre", C.c_int), ("post", C.c_int), ("omega", C.c_double),
                ("weighting", C.c_int), ("precision", C.c_int), ("patch_form", C.c_int),
                ("smoother", C.c_int), ("cheb_lo", C.c_double), ("cheb_hi", C.c_double)]


class irk_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("rel_residual", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int),
                ("ms_vcycle", C.c_double), ("ms_total", C.c_double)]


class irk_batch_opts(C.Structure):
    _fields_ = [("rows_per_item", C.c_int), ("patches_per_wave", C.c_int), ("workgroups_per_cu", C.c_int),
                ("autotune", C.c_int), ("mode", C.c_int), ("streams", C.c_int)]


class irk_kernel_stats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms_total", C.c_double), ("bytes_per_launch", C.c_double)]


class irk_newton_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("maxit", C.c_int), ("linear_maxit", C.c_int),
                ("restart", C.c_int), ("eta0", C.c_double), ("eta_max", C.c_double), ("ew_gamma", C.c_double),
                ("ew_alpha", C.c_double), ("ew_threshold", C.c_double), ("eta_fixed", C.c_double),
                ("linesearch", C.c_int), ("ls_maxit", C.c_int), ("ls_alpha", C.c_double), ("precond", C.c_int)]


class irk_mhd_opts(C.Structure):
    _fields_ = [("pre", C.c_int), ("post", C.c_int), ("omega", C.c_double), ("weighting", C.c_int),
                ("patch_form", C.c_int), ("smoother", C.c_int), ("cheb_lo", C.c_double), ("cheb_hi", C.c_double)]


class irk_newton_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("linear_iterations", C.c_int),
                ("norm0", C.c_double), ("norm", C.c_double), ("history", C.POINTER(C.c_double)),
                ("etas", C.POINTER(C.c_double)), ("linear_its", C.POINTER(C.c_int)), ("history_cap", C.c_int),
                ("ms_linear", C.c_double), ("ms_wall", C.c_double), ("lambdas", C.POINTER(C.c_double))]


KERNELS = {"patch_apply": 0, "residual": 1, "gather_update": 2, "ns_element": 3, "ns_gather": 4}


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    vp, i64, d, i = C.c_void_p, C.c_int64, C.c_double, C.c_int
    sig = {
        "irk_mg_default_opts": (None, [vp]),
        "irk_tableau_builtin": (i, [i, i, vp, vp, vp]),
        "irk_mesh_p2_nodes": (i, [vp, vp, vp]),
        "irk_mg_setup": (i, [vp, i, vp, d, d, vp, vp, vp, vp]),
        "irk_mg_destroy": (None, [vp]),
        "irk_mg_patch_form": (i, [vp]),
        "irk_stage_basis": (i, [i, vp, vp, vp, vp]),
        "irk_hessenberg_eigs": (i, [i, vp, i, vp, vp]),
        "irk_mg_ritz": (i, [vp, i, i, vp, vp, vp, vp, vp, vp]),
        "irk_mg_ritz_noalloc": (i, [vp, i, i, vp, vp, vp, vp, vp, vp]),
        "irk_mg_set_interval": (i, [vp, d, d]),
        "irk_mg_ndofs": (i64, [vp, i]),
        "irk_mg_sizes": (i, [vp, i, vp]),
        "irk_mg_layout": (i, [vp, i, vp, vp]),
        "irk_mg_p2_nodes": (i, [vp, i, vp, vp]),
        "irk_mg_apply": (i, [vp, vp, vp, i, vp]),
        "irk_mg_vcycle": (i, [vp, vp, vp, vp]),
        "irk_mg_vcycle_transpose": (i, [vp, vp, vp, vp]),
        "irk_fgmres_solve": (i, [vp, vp, vp, d, i, i, vp, vp]),
        "irk_adjoint_solve": (i, [vp, vp, vp, d, i, i, vp, vp]),
        "irk_rhs": (i, [vp, vp, vp, vp, vp]),
        "irk_update": (i, [vp, vp, vp, vp]),
        "irk_rhs_dirichlet": (i, [vp, vp, vp, vp, vp]),
        "irk_level_apply": (i, [vp, i, i, vp, vp, vp]),
        "irk_level_sweep": (i, [vp, i, i, vp, vp, vp]),
        "irk_level_restrict": (i, [vp, i, vp, vp, vp]),
        "irk_level_prolong": (i, [vp, i, vp, vp, vp]),
        "irk_coarse_solve": (i, [vp, i, vp, vp, vp]),
        "irk_rhs_adjoint": (i, [vp, vp, vp, vp, i, vp]),
        "irk_update_adjoint": (i, [vp, vp, vp, vp]),
        "irk_nu_sensitivity": (i, [vp, vp, vp, vp, vp, i, vp]),
        "irk_mass_apply": (i, [vp, vp, vp, vp]),
        "irk_tracking_loss": (i, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "irk_ns_residual": (i, [vp, vp, vp, vp, vp, vp, vp]),
        "irk_ns_jacobian_apply": (i, [vp, vp, vp, vp, vp, vp, vp]),
        "irk_newton_default_opts": (None, [vp]),
        "irk_ns_newton_solve": (i, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "irk_ns_newton_preconditioner": (i, [vp, vp, vp, vp, i, vp]),
        "irk_batch_default_opts": (None, [vp]),
        "irk_batch_create": (i, [vp, i, vp, vp, vp]),
        "irk_batch_fgmres_solve": (i, [vp, vp, vp, d, i, i, vp, vp, vp]),
        "irk_batch_get_opts": (i, [vp, vp]),
        "irk_batch_destroy": (None, [vp]),
        "irk_mg_profile": (i, [vp, i]),
        "irk_mg_kernel_stats": (i, [vp, i, i, vp]),
        "irk_last_error": (C.c_char_p, []),
        "irk_mhd_default_opts": (None, [vp]),
        "irk_mhd_setup": (i, [vp, i, vp, d, d, d, vp, vp, vp, vp, vp]),
        "irk_mhd_destroy": (None, [vp]),
        "irk_mhd_host_operators": (i, [vp, i, i, d, d, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "irk_mhd_ndofs": (i64, [vp, i]),
        "irk_mhd_patch_form": (i, [vp]),
        "irk_mhd_layout": (i, [vp, i, vp]),
        "irk_mhd_apply": (i, [vp, i, vp, vp, vp]),
        "irk_mhd_sweep": (i, [vp, i, vp, vp, vp]),
        "irk_mhd_restrict": (i, [vp, i, vp, vp, vp]),
        "irk_mhd_prolong": (i, [vp, i, vp, vp, vp]),
        "irk_mhd_coarse_solve": (i, [vp, vp, vp, vp]),
        "irk_mhd_vcycle": (i, [vp, vp, vp, vp]),
        "irk_mhd_fgmres_solve": (i, [vp, vp, vp, d, i, i, vp, vp]),
        "irk_mhd_profile": (i, [vp, i]),
        "irk_mhd_kernel_stats": (i, [vp, i, i, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def header_functions() -> list[str]:
    """Names of the functions the public headers declare."""
    txt = open(HEADER).read() + open(MHD_HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:irk_status|void|int64_t|int|const char\*)\s+(irk_\w+)\s*\(", txt, re.M)))


def _check(status: int, ok=(IRK_OK,)) -> int:
    if status not in ok:
        raise IrkError(status, lib.irk_last_error().decode())
    return status


def irk_tableau_builtin(family: str, r: int):
    A, b, c = np.zeros(16), np.zeros(4), np.zeros(4)
    _check(lib.irk_tableau_builtin(FAMILIES[family], r, A.ctypes.data, b.ctypes.data, c.ctypes.data))
    return A[: r * r].reshape(r, r).copy(), b[:r].copy(), c[:r].copy()


def _mesh_struct(level) -> tuple[irk_mesh_level, list]:
    xyz = np.ascontiguousarray(level.xyz, dtype=np.float64)
    cells = np.ascontiguousarray(level.cells, dtype=np.int64)
    keep = [xyz, cells]
    par = None
    if getattr(level, "parent", None) is not None:
        par = np.ascontiguousarray(level.parent, dtype=np.int64)
        keep.append(par)
    s = irk_mesh_level(level.dim, xyz.shape[0], cells.shape[0], xyz.ctypes.data, cells.ctypes.data,
                       par.ctypes.data if par is not None else None)
    return s, keep


def irk_stage_basis(A):
    """(W, Winv, T) with A = W T W^{-1}, T real block diagonal (irk_stage_basis)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    r = A.shape[0]
    W, Wi, T = (np.zeros((r, r)) for _ in range(3))
    _check(lib.irk_stage_basis(r, A.ctypes.data, W.ctypes.data, Wi.ctypes.data, T.ctypes.data))
    return W, Wi, T


def irk_hessenberg_eigs(H, m=None):
    """Eigenvalues (complex array, decreasing real part) of the leading m x m block of an
    upper Hessenberg matrix (irk_hessenberg_eigs; host only)."""
    H = np.asfortranarray(H, dtype=np.float64)
    m = H.shape[1] if m is None else int(m)
    wr, wi = np.zeros(m), np.zeros(m)
    _check(lib.irk_hessenberg_eigs(m, H.ctypes.data, H.shape[0], wr.ctypes.data, wi.ctypes.data))
    return wr + 1j * wi


def irk_mesh_p2_nodes(level) -> np.ndarray:
    s, keep = _mesh_struct(level)
    n = C.c_int64(0)
    _check(lib.irk_mesh_p2_nodes(C.byref(s), C.byref(n), None))
    xyz = np.zeros((n.value, level.dim))
    _check(lib.irk_mesh_p2_nodes(C.byref(s), C.byref(n), xyz.ctypes.data))
    return xyz


def _stream(stream=None) -> int:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t, n: int, name: str) -> int:
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return t.data_ptr()


class IrkMG:
    """Handle of one hierarchy (irk_mg_setup ... irk_mg_destroy)."""

    def __init__(self, levels, A, b, c, dt: float, nu: float, wind_nodal=None, pre=2, post=2,
                 omega=0.5, weighting=1, precision=0, patch_form=2, smoother=0, interval=(2.0, 8.0),
                 stream=None):
        structs, keep = [], []
        for lv in levels:
            s, k = _mesh_struct(lv)
            structs.append(s)
            keep += k
        arr = (irk_mesh_level * len(structs))(*structs)
        A = np.ascontiguousarray(A, dtype=np.float64)
        self.A, self.b, self.c = A, np.ascontiguousarray(b, dtype=np.float64), np.ascontiguousarray(c, dtype=np.float64)
        self.r = len(self.b)
        tab = irk_tableau(self.r, A.ctypes.data, self.b.ctypes.data, self.c.ctypes.data)
        opts = irk_mg_opts(pre, post, omega, weighting, precision, patch_form, smoother, interval[0], interval[1])
        w = None
        if wind_nodal is not None:
            w = np.ascontiguousarray(wind_nodal, dtype=np.float64)
        h = C.c_void_p()
        _check(lib.irk_mg_setup(arr, len(structs), C.byref(tab), dt, nu, w.ctypes.data if w is not None else None,
                                C.byref(opts), _stream(stream), C.byref(h)))
        self.h = h
        self.dt, self.nu, self.precision = dt, nu, precision
        self.nlevels = len(structs)
        self.dim = levels[0].dim

    def close(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "h", None) and lib is not None:
            lib.irk_mg_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # ----------------------------------------------------- relaxation spectrum
    def irk_mg_ritz(self, level, steps, v0, stream=None):
        """(H, Ritz values) of `steps` Arnoldi steps on W S J_level from v0 (device,
        ABI layout of the level); the Ritz values past an early invariant space are dropped."""
        n = self.irk_mg_ndofs(level)
        H = np.zeros((steps + 1, steps), order="F")
        wr, wi = np.zeros(steps), np.zeros(steps)
        m = C.c_int(0)
        _check(lib.irk_mg_ritz(self.h, level, steps, _dev(v0, n, "v0"), H.ctypes.data, wr.ctypes.data,
                               wi.ctypes.data, C.byref(m), _stream(stream)))
        return H, (wr + 1j * wi)[: m.value]

    def irk_mg_ritz_noalloc(self, level, steps, v0, stream=None):
        """irk_mg_ritz with the library's static device scratch instead of allocations."""
        n = self.irk_mg_ndofs(level)
        H = np.zeros((steps + 1, steps), order="F")
        wr, wi = np.zeros(steps), np.zeros(steps)
        m = C.c_int(0)
        _check(lib.irk_mg_ritz_noalloc(self.h, level, steps, _dev(v0, n, "v0"), H.ctypes.data, wr.ctypes.data,
                                       wi.ctypes.data, C.byref(m), _stream(stream)))
        return H, (wr + 1j * wi)[: m.value]

    def irk_mg_set_interval(self, lo, hi):
        _check(lib.irk_mg_set_interval(self.h, float(lo), float(hi)))

    # ---------------------------------------------------------------- sizes
    def irk_mg_patch_form(self) -> int:
        """0: dense patch inverses; 1: factored through the stage eigenbasis; 3: symmetric
        factored (wrapped diagonals of each block inverse, Stokes)."""
        return int(lib.irk_mg_patch_form(self.h))

    def irk_mg_ndofs(self, level: int = -1) -> int:
        return int(lib.irk_mg_ndofs(self.h, level))

    def irk_mg_sizes(self, level: int = -1) -> dict:
        out = np.zeros(5, dtype=np.int64)
        _check(lib.irk_mg_sizes(self.h, level, out.ctypes.data))
        return dict(nverts=int(out[0]), nnodes=int(out[1]), nfree=int(out[2]), ns=int(out[3]), nlevels=int(out[4]))

    def irk_mg_layout(self, level: int = -1) -> tuple[np.ndarray, np.ndarray]:
        """(offsets, lengths): offsets[s, c] is where velocity component c (c < dim) or the
        pressure (c = dim) of stage s starts in the ABI layout; lengths[c] its length."""
        off = np.zeros((self.r, self.dim + 1), dtype=np.int64)
        ln = np.zeros(self.dim + 1, dtype=np.int64)
        _check(lib.irk_mg_layout(self.h, level, off.ctypes.data, ln.ctypes.data))
        return off, ln

    def irk_mg_p2_nodes(self, level: int = -1):
        sz = self.irk_mg_sizes(level)
        xyz = np.zeros((sz["nnodes"], self.dim))
        free = np.zeros(sz["nfree"], dtype=np.int64)
        _check(lib.irk_mg_p2_nodes(self.h, level, xyz.ctypes.data, free.ctypes.data))
        return xyz, free

    # ------------------------------------------------------------- operators
    def irk_mg_apply(self, x, y, transpose=False, stream=None):
        n = self.irk_mg_ndofs()
        _check(lib.irk_mg_apply(self.h, _dev(x, n, "x"), _dev(y, n, "y"), int(transpose), _stream(stream)))

    def irk_mg_vcycle(self, r, z, stream=None):
        n = self.irk_mg_ndofs()
        _check(lib.irk_mg_vcycle(self.h, _dev(r, n, "r"), _dev(z, n, "z"), _stream(stream)))

    def irk_mg_vcycle_transpose(self, r, z, stream=None):
        n = self.irk_mg_ndofs()
        _check(lib.irk_mg_vcycle_transpose(self.h, _dev(r, n, "r"), _dev(z, n, "z"), _stream(stream)))

    def _solve(self, fn, F, k, rtol, maxit, restart, history_cap, stream):
        n = self.irk_mg_ndofs()
        hist = np.zeros(max(1, history_cap))
        info = irk_solve_info(0, 0, 0.0, hist.ctypes.data_as(C.POINTER(C.c_double)), history_cap, 0.0, 0.0)
        st = _check(fn(self.h, _dev(F, n, "F"), _dev(k, n, "k"), rtol, maxit, restart, C.byref(info), _stream(stream)),
                    ok=(IRK_OK, IRK_ENOCONV))
        its = info.iterations
        return dict(status=st, iterations=its, converged=bool(info.converged), rel_residual=info.rel_residual,
                    history=hist[: min(history_cap, its + 1)].copy(), ms_vcycle=info.ms_vcycle, ms_total=info.ms_total)

    def irk_fgmres_solve(self, F, k, rtol=1e-8, maxit=1000, restart=30, history_cap=1024, stream=None):
        return self._solve(lib.irk_fgmres_solve, F, k, rtol, maxit, restart, history_cap, stream)

    def irk_adjoint_solve(self, G, lam, rtol=1e-8, maxit=1000, restart=30, history_cap=1024, stream=None):
        return self._solve(lib.irk_adjoint_solve, G, lam, rtol, maxit, restart, history_cap, stream)

    def irk_rhs(self, f_nodal, state, F, stream=None):
        sz = self.irk_mg_sizes()
        _check(lib.irk_rhs(self.h, _dev(f_nodal, self.r * sz["nnodes"] * self.dim, "f"), _dev(state, sz["ns"], "state"),
                           _dev(F, self.irk_mg_ndofs(), "F"), _stream(stream)))

    def irk_rhs_dirichlet(self, g_n, g_stages, F, stream=None):
        sz = self.irk_mg_sizes()
        nn = sz["nnodes"] * self.dim
        _check(lib.irk_rhs_dirichlet(self.h, _dev(g_n, nn, "g_n"), _dev(g_stages, self.r * nn, "g_stages"),
                                     _dev(F, self.irk_mg_ndofs(), "F"), _stream(stream)))

    def irk_update(self, k, state, stream=None):
        sz = self.irk_mg_sizes()
        _check(lib.irk_update(self.h, _dev(k, self.irk_mg_ndofs(), "k"), _dev(state, sz["ns"], "state"), _stream(stream)))

    # -------------------------------------------------------------- adjoint
    def irk_rhs_adjoint(self, lam, gf, gstate, accumulate=False, stream=None):
        sz = self.irk_mg_sizes()
        _check(lib.irk_rhs_adjoint(self.h, _dev(lam, self.irk_mg_ndofs(), "lam"),
                                   _dev(gf, self.r * sz["nnodes"] * self.dim, "gf"), _dev(gstate, sz["ns"], "gstate"),
                                   int(accumulate), _stream(stream)))

    def irk_update_adjoint(self, gstate, G, stream=None):
        sz = self.irk_mg_sizes()
        _check(lib.irk_update_adjoint(self.h, _dev(gstate, sz["ns"], "gstate"), _dev(G, self.irk_mg_ndofs(), "G"),
                                      _stream(stream)))

    def irk_nu_sensitivity(self, lam, k, state, out, accumulate=False, stream=None):
        sz = self.irk_mg_sizes()
        n = self.irk_mg_ndofs()
        _check(lib.irk_nu_sensitivity(self.h, _dev(lam, n, "lam"), _dev(k, n, "k"), _dev(state, sz["ns"], "state"),
                                      _dev(out, 1, "out"), int(accumulate), _stream(stream)))

    def irk_tracking_loss(self, state, target, loss=None, grad_state=None, grad_target=None, scale=None,
                          stream=None):
        """loss (1 value) = 1/2 e^T M e, e the velocity part of state - target;
        grad_state / grad_target (ns values) = +- scale [M e; 0]; any output may be None."""
        ns = self.irk_mg_sizes()["ns"]

        def opt(t, m, name):
            return None if t is None else _dev(t, m, name)

        _check(lib.irk_tracking_loss(self.h, _dev(state, ns, "state"), _dev(target, ns, "target"),
                                     opt(scale, 1, "scale"), opt(loss, 1, "loss"), opt(grad_state, ns, "grad_state"),
                                     opt(grad_target, ns, "grad_target"), _stream(stream)))

    def irk_mass_apply(self, state, out, stream=None):
        sz = self.irk_mg_sizes()
        _check(lib.irk_mass_apply(self.h, _dev(state, sz["ns"], "state"), _dev(out, sz["ns"], "out"), _stream(stream)))

    # ------------------------------------------------ Navier--Stokes, Newton
    def _ns_common(self, state, g_stages):
        sz = self.irk_mg_sizes()
        g = None if g_stages is None else _dev(g_stages, self.r * sz["nnodes"] * self.dim, "g_stages")
        return _dev(state, sz["ns"], "state"), g

    def irk_ns_residual(self, F, state, k, R, g_stages=None, stream=None):
        n = self.irk_mg_ndofs()
        st, g = self._ns_common(state, g_stages)
        _check(lib.irk_ns_residual(self.h, _dev(F, n, "F"), st, g, _dev(k, n, "k"), _dev(R, n, "R"),
                                   _stream(stream)))

    def irk_ns_jacobian_apply(self, state, k, x, y, g_stages=None, stream=None):
        n = self.irk_mg_ndofs()
        st, g = self._ns_common(state, g_stages)
        _check(lib.irk_ns_jacobian_apply(self.h, st, g, _dev(k, n, "k"), _dev(x, n, "x"), _dev(y, n, "y"),
                                         _stream(stream)))

    def irk_ns_newton_preconditioner(self, state=None, k=None, g_stages=None, enable=True, stream=None):
        """Switch the V-cycle to the Newton Jacobian's operators at (state, k) (enable) or
        back to the handle's own operator."""
        if not enable:
            _check(lib.irk_ns_newton_preconditioner(self.h, None, None, None, 0, _stream(stream)))
            return
        st, g = self._ns_common(state, g_stages)
        _check(lib.irk_ns_newton_preconditioner(self.h, st, g, _dev(k, self.irk_mg_ndofs(), "k"), 1,
                                                _stream(stream)))

    def irk_ns_newton_solve(self, F, state, k, g_stages=None, history_cap=64, stream=None, **opts):
        """Newton on the Navier--Stokes stage equations; opts: fields of irk_newton_opts."""
        n = self.irk_mg_ndofs()
        st, g = self._ns_common(state, g_stages)
        o = irk_newton_opts()
        lib.irk_newton_default_opts(C.byref(o))
        for key, val in opts.items():
            if key not in dict(irk_newton_opts._fields_):
                raise TypeError(f"unknown Newton option {key}")
            setattr(o, key, val)
        cap = max(1, history_cap)
        hist, etas, lits, lams = np.zeros(cap), np.zeros(cap), np.zeros(cap, dtype=np.int32), np.zeros(cap)
        info = irk_newton_info(0, 0, 0, 0.0, 0.0, hist.ctypes.data_as(C.POINTER(C.c_double)),
                               etas.ctypes.data_as(C.POINTER(C.c_double)), lits.ctypes.data_as(C.POINTER(C.c_int)),
                               cap, 0.0, 0.0, lams.ctypes.data_as(C.POINTER(C.c_double)))
        status = _check(lib.irk_ns_newton_solve(self.h, _dev(F, n, "F"), st, g, _dev(k, n, "k"), C.byref(o),
                                                C.byref(info), _stream(stream)), ok=(IRK_OK, IRK_ENOCONV))
        its = info.iterations
        return dict(status=status, iterations=its, converged=bool(info.converged),
                    linear_iterations=info.linear_iterations, norm0=info.norm0, norm=info.norm,
                    history=hist[: min(cap, its + 1)].copy(), etas=etas[: min(cap, its)].copy(),
                    linear_its=lits[: min(cap, its)].copy(), lambdas=lams[: min(cap, its)].copy(),
                    ms_linear=info.ms_linear, ms_wall=info.ms_wall)

    # ---------------------------------------------------------- measurement
    def irk_mg_profile(self, mode):
        """0 (or False) off; 1 (or True) finest-level patch apply; 2 finest-level kernels; 3 all."""
        _check(lib.irk_mg_profile(self.h, int(mode)))

    def irk_mg_kernel_stats(self, kernel: str, level: int = -1) -> dict:
        st = irk_kernel_stats()
        _check(lib.irk_mg_kernel_stats(self.h, KERNELS[kernel], level, C.byref(st)))
        return dict(launches=int(st.launches), ms_total=float(st.ms_total), bytes_per_launch=float(st.bytes_per_launch))

    # ------------------------------------------------------------ per level
    def irk_level_apply(self, level, x, y, transpose=False, stream=None):
        n = self.irk_mg_ndofs(level)
        _check(lib.irk_level_apply(self.h, level, int(transpose), _dev(x, n, "x"), _dev(y, n, "y"), _stream(stream)))

    def irk_level_sweep(self, level, F, k, transpose=False, stream=None):
        n = self.irk_mg_ndofs(level)
        _check(lib.irk_level_sweep(self.h, level, int(transpose), _dev(F, n, "F"), _dev(k, n, "k"), _stream(stream)))

    def irk_level_restrict(self, level, xf, xc, stream=None):
        _check(lib.irk_level_restrict(self.h, level, _dev(xf, self.irk_mg_ndofs(level), "xf"),
                                      _dev(xc, self.irk_mg_ndofs(level - 1), "xc"), _stream(stream)))

    def irk_level_prolong(self, level, xc, xf, stream=None):
        _check(lib.irk_level_prolong(self.h, level, _dev(xc, self.irk_mg_ndofs(level - 1), "xc"),
                                     _dev(xf, self.irk_mg_ndofs(level), "xf"), _stream(stream)))

    def irk_coarse_solve(self, b, x, transpose=False, stream=None):
        n = self.irk_mg_ndofs(0)
        _check(lib.irk_coarse_solve(self.h, int(transpose), _dev(b, n, "b"), _dev(x, n, "x"), _stream(stream)))


class IrkBatch:
    """Batched solves of several handles (irk_batch_*): one persistent launch (mode 0)
    or concurrent streams (mode 1); autotuning picks the faster schedule."""

    def __init__(self, solvers, rows_per_item=1, patches_per_wave=1, workgroups_per_cu=2, autotune=True, mode=0,
                 streams=4, stream=None):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        opts = irk_batch_opts(rows_per_item, patches_per_wave, workgroups_per_cu, int(autotune), mode, streams)
        h = C.c_void_p()
        _check(lib.irk_batch_create(arr, len(self.solvers), C.byref(opts), _stream(stream), C.byref(h)))
        self.h = h

    def close(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "h", None) and lib is not None:
            lib.irk_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def irk_batch_get_opts(self) -> dict:
        o = irk_batch_opts()
        _check(lib.irk_batch_get_opts(self.h, C.byref(o)))
        return dict(rows_per_item=o.rows_per_item, patches_per_wave=o.patches_per_wave,
                    workgroups_per_cu=o.workgroups_per_cu, autotune=o.autotune, mode=o.mode, streams=o.streams)

    def irk_batch_fgmres_solve(self, Fs, ks, rtol=1e-8, maxit=1000, restart=30, stream=None):
        n = len(self.solvers)
        if len(Fs) != n or len(ks) != n:
            raise ValueError("one F and one k per solver")
        Fp = (C.c_void_p * n)(*[_dev(F, s.irk_mg_ndofs(), "F") for F, s in zip(Fs, self.solvers)])
        kp = (C.c_void_p * n)(*[_dev(k, s.irk_mg_ndofs(), "k") for k, s in zip(ks, self.solvers)])
        infos = (irk_solve_info * n)()
        lat = np.zeros(n)
        st = _check(lib.irk_batch_fgmres_solve(self.h, Fp, kp, rtol, maxit, restart, infos, lat.ctypes.data,
                                               _stream(stream)), ok=(IRK_OK, IRK_ENOCONV))
        out = [dict(iterations=i.iterations, converged=bool(i.converged), rel_residual=i.rel_residual,
                    latency_ms=float(l)) for i, l in zip(infos, lat)]
        return st, out, float(infos[0].ms_total)


def irk_mhd_host_operators(levels, level, Re, Rem, w, b0):
    """(M, S, P) of one level as scipy CSR matrices, assembled by the library on the host
    (irk_mhd_host_operators; P is None on level 0)."""
    import scipy.sparse as sp

    structs, keep = [], []
    for lv in levels:
        s, k = _mesh_struct(lv)
        structs.append(s)
        keep += k
    arr = (irk_mesh_level * len(structs))(*structs)
    w = np.ascontiguousarray(w, dtype=np.float64)
    b0 = np.ascontiguousarray(b0, dtype=np.float64)
    sizes = np.zeros(4, dtype=np.int64)
    args = (arr, len(structs), level, Re, Rem, w.ctypes.data, b0.ctypes.data, sizes.ctypes.data)
    _check(lib.irk_mhd_host_operators(*args, None, None, None, None, None, None, None))
    ns, nnz, nnzp, nsc = (int(v) for v in sizes)
    ptr, col = np.zeros(ns + 1, np.int32), np.zeros(nnz, np.int32)
    mv, sv = np.zeros(nnz), np.zeros(nnz)
    pp, pc, pv = np.zeros(ns + 1, np.int32), np.zeros(max(nnzp, 1), np.int32), np.zeros(max(nnzp, 1))
    _check(lib.irk_mhd_host_operators(*args, ptr.ctypes.data, col.ctypes.data, mv.ctypes.data, sv.ctypes.data,
                                      pp.ctypes.data, pc.ctypes.data, pv.ctypes.data))
    M = sp.csr_matrix((mv, col, ptr), shape=(ns, ns))
    S = sp.csr_matrix((sv, col, ptr), shape=(ns, ns))
    P = sp.csr_matrix((pv[:nnzp], pc[:nnzp], pp), shape=(ns, nsc)) if nsc > 0 else None
    return M, S, P


class IrkMHD:
    """Handle of the linearised 2D MHD stage solver (irk_mhd_setup ... irk_mhd_destroy).
    w: finest P2 nodes x 2 (the velocity of the linearisation); b0: Nedelec degrees of
    freedom of B0 on every finest edge."""

    def __init__(self, levels, A, dt: float, Re: float, Rem: float, w, b0, pre=2, post=2, omega=0.5, weighting=1,
                 patch_form=2, smoother=0, interval=(2.0, 10.0), stream=None):
        structs, keep = [], []
        for lv in levels:
            s, k = _mesh_struct(lv)
            structs.append(s)
            keep += k
        arr = (irk_mesh_level * len(structs))(*structs)
        self.A = np.ascontiguousarray(A, dtype=np.float64)
        self.r = self.A.shape[0]
        zero = np.zeros(self.r)
        tab = irk_tableau(self.r, self.A.ctypes.data, zero.ctypes.data, zero.ctypes.data)
        opts = irk_mhd_opts(pre, post, omega, weighting, patch_form, smoother, interval[0], interval[1])
        w = np.ascontiguousarray(w, dtype=np.float64)
        b0 = np.ascontiguousarray(b0, dtype=np.float64)
        h = C.c_void_p()
        _check(lib.irk_mhd_setup(arr, len(structs), C.byref(tab), dt, Re, Rem, w.ctypes.data, b0.ctypes.data,
                                 C.byref(opts), _stream(stream), C.byref(h)))
        self.h = h
        self.nlevels = len(structs)

    def close(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "h", None) and lib is not None:
            lib.irk_mhd_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def irk_mhd_ndofs(self, level: int = -1) -> int:
        return int(lib.irk_mhd_ndofs(self.h, level))

    def irk_mhd_patch_form(self) -> int:
        return int(lib.irk_mhd_patch_form(self.h))

    def irk_mhd_layout(self, level: int = -1) -> dict:
        out = np.zeros(7, dtype=np.int64)
        _check(lib.irk_mhd_layout(self.h, level, out.ctypes.data))
        return dict(zip(("u_x", "u_y", "B", "p", "gamma", "ns", "r"), (int(v) for v in out)))

    def irk_mhd_apply(self, level, x, y, stream=None):
        n = self.irk_mhd_ndofs(level)
        _check(lib.irk_mhd_apply(self.h, level, _dev(x, n, "x"), _dev(y, n, "y"), _stream(stream)))

    def irk_mhd_sweep(self, level, F, k, stream=None):
        n = self.irk_mhd_ndofs(level)
        _check(lib.irk_mhd_sweep(self.h, level, _dev(F, n, "F"), _dev(k, n, "k"), _stream(stream)))

    def irk_mhd_restrict(self, level, xf, xc, stream=None):
        _check(lib.irk_mhd_restrict(self.h, level, _dev(xf, self.irk_mhd_ndofs(level), "xf"),
                                    _dev(xc, self.irk_mhd_ndofs(level - 1), "xc"), _stream(stream)))

    def irk_mhd_prolong(self, level, xc, xf, stream=None):
        _check(lib.irk_mhd_prolong(self.h, level, _dev(xc, self.irk_mhd_ndofs(level - 1), "xc"),
                                   _dev(xf, self.irk_mhd_ndofs(level), "xf"), _stream(stream)))

    def irk_mhd_coarse_solve(self, b, x, stream=None):
        n = self.irk_mhd_ndofs(0)
        _check(lib.irk_mhd_coarse_solve(self.h, _dev(b, n, "b"), _dev(x, n, "x"), _stream(stream)))

    def irk_mhd_vcycle(self, r, z, stream=None):
        n = self.irk_mhd_ndofs()
        _check(lib.irk_mhd_vcycle(self.h, _dev(r, n, "r"), _dev(z, n, "z"), _stream(stream)))

    def irk_mhd_fgmres_solve(self, F, k, rtol=1e-8, maxit=1000, restart=30, history_cap=1024, stream=None):
        n = self.irk_mhd_ndofs()
        hist = np.zeros(max(1, history_cap))
        info = irk_solve_info(0, 0, 0.0, hist.ctypes.data_as(C.POINTER(C.c_double)), history_cap, 0.0, 0.0)
        st = _check(lib.irk_mhd_fgmres_solve(self.h, _dev(F, n, "F"), _dev(k, n, "k"), rtol, maxit, restart,
                                             C.byref(info), _stream(stream)), ok=(IRK_OK, IRK_ENOCONV))
        its = info.iterations
        return dict(status=st, iterations=its, converged=bool(info.converged), rel_residual=info.rel_residual,
                    history=hist[: min(history_cap, its + 1)].copy(), ms_vcycle=info.ms_vcycle, ms_total=info.ms_total)

    def irk_mhd_profile(self, mode):
        _check(lib.irk_mhd_profile(self.h, int(mode)))

    def irk_mhd_kernel_stats(self, kernel: str, level: int = -1) -> dict:
        kid = {"patch_apply": 0, "residual": 1, "gather_update": 2}[kernel]
        st = irk_kernel_stats()
        _check(lib.irk_mhd_kernel_stats(self.h, kid, level, C.byref(st)))
        return dict(launches=st.launches, ms_total=st.ms_total, bytes_per_launch=st.bytes_per_launch)
