"""Shared set-up for GPU parity tests: the same seeded workload handed to the HIP
library (through the C ABI) and to the CPU oracle."""
import functools
import sys

import numpy as np

from oracle.multigrid import Hierarchy
from oracle.tableau import tableau
from paper_2202_07381_amd import workloads as wl

CASES = {
    # name: (dim, n_coarse, nlevels, family, r, dt, nu, wind seed or None)
    "c1": (2, 4, 3, "radauIIA", 2, 1 / 16, 1.0, None),
    "r3": (2, 4, 4, "radauIIA", 3, 1e-2, 1.0, None),
    "oseen": (2, 4, 3, "gauss", 2, 5e-3, 0.01, 3),
    "be": (2, 2, 3, "radauIIA", 1, 0.05, 0.3, None),
    "lob3": (2, 2, 3, "lobattoIIIC", 3, 0.02, 1.0, None),
    "3d2": (3, 2, 2, "radauIIA", 2, 1e-2, 1.0, None),
    "3d3": (3, 2, 3, "radauIIA", 2, 1e-2, 1.0, None),
    "cross": (2, 2, 3, "radauIIA", 3, 1 / 64, 1.0, None),
    # the 7-level benchmark workload one level down: 128^2, 6 levels, 16,641 finest
    # patches (above the count from which the library streams patch factors with
    # non-temporal loads), 440,073 unknowns; its oracle takes about half a minute
    "s128": (2, 4, 6, "radauIIA", 3, 1e-2, 1.0, None),
    # the benchmark workload itself: 256^2, 7 levels, 1,764,873 unknowns; its oracle needs
    # about 35 GB and a few minutes (test_gpu_parity_256.py, run on request)
    "s256": (2, 4, 7, "radauIIA", 3, 1e-2, 1.0, None),
}
# cases whose oracle is too slow for the per-step sweeps over every level
LARGE = {"s128", "s256"}
SMALL = [c for c in CASES if c not in LARGE]
# cases on the crossed mesh of Sec. 5.1 (four triangles per quad) instead of the
# diagonal split
CROSSED = {"cross"}


# Set by an autouse fixture in conftest.py so that progress lines reach the terminal
# while pytest captures output (a long test must not look silent).
_sink = None


def say(msg):
    if _sink is not None:
        _sink(msg)
        return
    print(msg, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch

    return torch.device("cuda:0")


def levels_of(case):
    dim, nc, nl = CASES[case][:3]
    if case in CROSSED:
        return wl.crossed_hierarchy(nc, nl)
    return wl.square_hierarchy(nc, nl) if dim == 2 else wl.cube_hierarchy(nc, nl)


def wind_of(case):
    dim, nc, nl, fam, r, dt, nu, ws = CASES[case]
    if ws is None:
        return None
    return wl.wind_2d(ws, nc * 2 ** (nl - 1))


@functools.lru_cache(maxsize=None)
def oracle_of(case, dtype=np.float64, smoother="sweep"):
    """Oracle hierarchy; smoother "chebyshev" is the paper's relaxation (unweighted
    additive operator, interval [2, 8]); "gmres" two GMRES steps per relaxation with the
    weighted additive operator."""
    dim, nc, nl, fam, r, dt, nu, ws = CASES[case]
    A, b, c = tableau(fam, r)
    if smoother == "chebyshev":
        return Hierarchy(levels_of(case), A, dt, nu, wind=wind_of(case), dtype=dtype, weighted=False,
                         smoother="chebyshev", interval=(2.0, 8.0))
    if smoother == "gmres":
        return Hierarchy(levels_of(case), A, dt, nu, wind=wind_of(case), dtype=dtype, smoother="gmres")
    return Hierarchy(levels_of(case), A, dt, nu, wind=wind_of(case), dtype=dtype)


_GPU = {}


def gpu_of(case, precision=0, patch_form=2, smoother=0):
    key = (case, precision, patch_form, smoother)
    if key not in _GPU:
        from paper_2202_07381_amd import irkmg

        dim, nc, nl, fam, r, dt, nu, ws = CASES[case]
        lv = levels_of(case)
        A, b, c = irkmg.irk_tableau_builtin(fam, r)
        wind = wind_of(case)
        wn = wind(irkmg.irk_mesh_p2_nodes(lv[-1])) if wind is not None else None
        say(f"[setup] case={case} precision={precision} patch_form={patch_form} smoother={smoother}")
        extra = {1: dict(smoother=1, weighting=0, interval=(2.0, 8.0)), 2: dict(smoother=2)}.get(smoother, {})
        _GPU[key] = irkmg.IrkMG(lv, A, b, c, dt, nu, wind_nodal=wn, precision=precision, patch_form=patch_form,
                                **extra)
        say(f"[setup] done case={case} N={_GPU[key].irk_mg_ndofs()} form={_GPU[key].irk_mg_patch_form()}")
    return _GPU[key]


def to_dev(x):
    import torch

    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=torch_dev())


def to_host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def forcing_rhs(case):
    """F of the first step from rest with the seeded forcing (oracle side)."""
    H = oracle_of(case)
    S = H.finest
    f = wl.forcing_2d(1) if S.th.dim == 2 else wl.forcing_3d(5)
    return S.rhs([S.th.interpolate(f, 0.0)] * S.r, np.zeros(S.th.nvel), np.zeros(S.th.nverts))
