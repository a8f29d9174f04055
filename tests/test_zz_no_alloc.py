"""irk_mg_ritz_noalloc, the allocation-free form of irk_mg_ritz, called through the C ABI:
its Hessenberg matrix and Ritz values equal those of irk_mg_ritz (the same kernels in
the same order, so bitwise), on two calls in a row whose second is smaller (a coarser
level and fewer steps, so it runs on what the first call left in the shared scratch),
in FP64 and FP32; a request beyond the 64 MiB scratch is refused with IRK_EINVAL."""
import ctypes as C

import numpy as np
import pytest

from gpu_cases import gpu_of, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _noalloc(g, level, steps, v0):
    from paper_2202_07381_amd import irkmg

    f = irkmg.lib.irk_mg_ritz_noalloc
    f.restype = C.c_int
    f.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                  C.c_void_p]
    H = np.zeros((steps + 1, steps), order="F")
    wr, wi = np.zeros(steps), np.zeros(steps)
    m = C.c_int(0)
    st = f(g.h, level, steps, v0.data_ptr(), H.ctypes.data, wr.ctypes.data, wi.ctypes.data, C.byref(m), None)
    torch.cuda.synchronize()
    return st, H, (wr + 1j * wi)[: m.value]


@pytest.mark.parametrize("precision", [0, 1])
def test_ritz_noalloc_matches_ritz(precision):
    from paper_2202_07381_amd import irkmg

    g = gpu_of("r3", precision=precision)
    for level, steps in ((-1, 24), (2, 6)):  # the second call is the smaller one
        n = g.irk_mg_ndofs(level)
        v0 = to_dev(np.random.default_rng(90 + steps).standard_normal(n))
        say(f"[noalloc] precision={precision} level={level} steps={steps} n={n}")
        st, H, ritz = _noalloc(g, level, steps, v0)
        assert st == irkmg.IRK_OK
        Href, ritz_ref = g.irk_mg_ritz(level, steps, v0)
        assert np.array_equal(H, Href)
        assert ritz.size == ritz_ref.size and np.array_equal(ritz, ritz_ref)


def test_ritz_noalloc_rejects_oversize():
    from paper_2202_07381_amd import irkmg

    g = gpu_of("s128")
    n = g.irk_mg_ndofs(-1)  # 440,073 unknowns: 21 vectors of 3.5 MB exceed 64 MiB
    v0 = to_dev(np.ones(n))
    st, _, _ = _noalloc(g, -1, 20, v0)
    assert st == irkmg.IRK_EINVAL
    assert b"64 MiB" in irkmg.lib.irk_last_error()
