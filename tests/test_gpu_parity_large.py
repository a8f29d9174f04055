"""GPU parity at 128 x 128 (the benchmark's workload family one level below its size):
RadauIIA(3), dt = 1e-2, nu = 1, 6 levels, 440,073 unknowns, the first step of the
seeded manufactured solution.  The finest level has 16,641 patches, so the patch
kernels that stream factors with non-temporal loads run there, in each of the three
patch forms.  Bars as in test_gpu_parity.py: V-cycles max(1e-12, 4 cond_S(J_0) eps)
(Skeel's condition number of the pinned coarse operator), FGMRES solutions 1e-10
relative after equal iteration counts, for a solve to 1e-8 and for four iterations
with an unreachable tolerance.  The FP32-patch solve must reach the relative residual
1e-8 measured with the oracle's operator; its error against the oracle's FP64 solution
is printed and bounded by 1e-6."""
import functools

import numpy as np
import pytest

from gpu_cases import gpu_of, oracle_of, relerr, say, to_dev, to_host
from test_gpu_parity import VCYCLE_TOL

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASE = "s128"


@functools.lru_cache(maxsize=None)
def mms_rhs():
    """F of the first step of the manufactured solution (seed 2) from its interpolant."""
    from paper_2202_07381_amd import workloads as wl

    H = oracle_of(CASE)
    S = H.finest
    th = S.th
    dt, nu = 1e-2, 1.0
    mms = wl.mms_2d(2, nu)
    c = [float(x) for x in np.sum(S.A, axis=1)]
    u0 = th.free_velocity(th.interpolate(mms.velocity, 0.0))
    fn = [th.interpolate(mms, ci * dt) for ci in c]
    return S.rhs(fn, u0, np.zeros(th.nverts))


@functools.lru_cache(maxsize=None)
def oracle_solution(rtol, maxit):
    from oracle.fgmres import fgmres

    H = oracle_of(CASE)
    S = H.finest
    F = mms_rhs()
    say(f"[s128] oracle FGMRES rtol={rtol} maxit={maxit}")
    return fgmres(S.apply, H.vcycle, F, np.zeros_like(F), rtol, maxit, 30, project=S.project_pressure_mean)


@pytest.mark.parametrize("form", [0, 1, 2])
def test_s128_vcycle(form):
    say(f"[s128] oracle hierarchy and GPU setup form={form}")
    H = oracle_of(CASE)
    g = gpu_of(CASE, patch_form=form)
    assert g.irk_mg_ndofs() == H.finest.n == 440073
    r = np.random.default_rng(61).standard_normal(H.finest.n)
    z = torch.zeros(r.size, dtype=torch.float64, device="cuda")
    g.irk_mg_vcycle(to_dev(r), z)
    err = relerr(to_host(z), H.vcycle(r))
    say(f"[s128] vcycle form={form} err={err:.2e} tol={VCYCLE_TOL:.0e}")
    assert err < VCYCLE_TOL


@pytest.mark.parametrize("form", [0, 1, 2])
def test_s128_fgmres_matches_oracle(form):
    g = gpu_of(CASE, patch_form=form)
    F = mms_rhs()
    for rtol, maxit in ((1e-8, 200), (1e-30, 4)):
        xo, io = oracle_solution(rtol, maxit)
        say(f"[s128] fgmres form={form} rtol={rtol} maxit={maxit}")
        k = torch.zeros(F.size, dtype=torch.float64, device="cuda")
        info = g.irk_fgmres_solve(to_dev(F), k, rtol=rtol, maxit=maxit, restart=30)
        err = relerr(to_host(k), xo)
        say(f"[s128] its gpu={info['iterations']} oracle={io.iterations} err={err:.2e}")
        assert info["iterations"] == io.iterations
        assert err < 1e-10
        if rtol > 1e-20:
            assert info["converged"] and info["rel_residual"] <= rtol


def test_s128_fp32_error_against_oracle():
    H = oracle_of(CASE)
    S = H.finest
    F = mms_rhs()
    xo, io = oracle_solution(1e-8, 200)
    g32 = gpu_of(CASE, precision=1, patch_form=2)
    k = torch.zeros(F.size, dtype=torch.float64, device="cuda")
    info = g32.irk_fgmres_solve(to_dev(F), k, rtol=1e-8, maxit=200)
    kk = to_host(k)
    res = np.linalg.norm(F - S.J @ kk) / np.linalg.norm(F)
    err = np.linalg.norm(kk - xo) / np.linalg.norm(xo)
    say(f"[s128] fp32 its={info['iterations']} (oracle fp64 {io.iterations}) residual={res:.2e} "
        f"error vs oracle={err:.2e} (max-norm {relerr(kk, xo):.2e})")
    assert info["converged"] and res <= 1e-8
    assert err < 1e-6
