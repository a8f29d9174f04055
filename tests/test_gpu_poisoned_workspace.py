"""Regression test: no kernel may read a workspace entry it has not written.

Every device allocation of the handles built here is filled with the byte 0xFF (a NaN
in FP64 and FP32) by the library's IRK_MG_POISON_ALLOC switch, and the caching
allocator of torch is filled with NaN and released before, so that the caller's fresh
vectors start on NaN-filled memory too.  A kernel that multiplies a stale workspace
value by zero (0 * NaN = NaN; the case once hit when the first Krylov basis vector
was formed from the previous contents of the basis buffer) then turns the result
non-finite.  Solves with the damped, Chebyshev and GMRES relaxations, the FP32 form and
the adjoint solve must match the oracle exactly as on clean memory: equal iteration
counts and 1e-10 relative."""
import os

import numpy as np
import pytest

from gpu_cases import CASES, forcing_rhs, levels_of, oracle_of, relerr, say, to_dev, to_host, wind_of

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture
def poisoned():
    junk = torch.full((64 << 20,), float("nan"), dtype=torch.float64, device="cuda")  # 512 MiB
    del junk
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    old = os.environ.get("IRK_MG_POISON_ALLOC")
    os.environ["IRK_MG_POISON_ALLOC"] = "1"
    try:
        yield
    finally:
        if old is None:
            del os.environ["IRK_MG_POISON_ALLOC"]
        else:
            os.environ["IRK_MG_POISON_ALLOC"] = old


def _handle(case, **kw):
    from paper_2202_07381_amd import irkmg

    dim, nc, nl, fam, r, dt, nu, ws = CASES[case]
    lv = levels_of(case)
    A, b, c = irkmg.irk_tableau_builtin(fam, r)
    w = wind_of(case)
    wn = w(irkmg.irk_mesh_p2_nodes(lv[-1])) if w is not None else None
    return irkmg.IrkMG(lv, A, b, c, dt, nu, wind_nodal=wn, **kw)


@pytest.mark.parametrize("case,smoother,precision", [("c1", "sweep", 0), ("oseen", "gmres", 0),
                                                     ("r3", "chebyshev", 0), ("3d2", "sweep", 0),
                                                     ("r3", "sweep", 1)])
def test_solve_on_poisoned_memory(poisoned, case, smoother, precision):
    from oracle.fgmres import fgmres

    kw = {"sweep": {}, "gmres": dict(smoother=2),
          "chebyshev": dict(smoother=1, weighting=0, interval=(2.0, 8.0))}[smoother]
    say(f"[poison] case={case} smoother={smoother} precision={precision}")
    g = _handle(case, precision=precision, **kw)
    H = oracle_of(case, smoother=smoother)
    S = H.finest
    F = forcing_rhs(case)
    k = torch.full((F.size,), float("nan"), dtype=torch.float64, device="cuda")
    k.zero_()
    info = g.irk_fgmres_solve(to_dev(F), k, rtol=1e-8, maxit=200, restart=30)
    kk = to_host(k)
    assert np.all(np.isfinite(kk)) and info["converged"]
    if precision == 0:
        xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 200, 30, project=S.project_pressure_mean)
        say(f"[poison] its gpu={info['iterations']} oracle={io.iterations} err={relerr(kk, xo):.2e}")
        assert info["iterations"] == io.iterations and relerr(kk, xo) < 1e-10
    else:
        assert np.linalg.norm(F - S.J @ kk) <= 1e-8 * np.linalg.norm(F)
    # the adjoint solve and a preconditioner application on the same poisoned handle
    G = np.concatenate([S.dt * g.b[i] * np.random.default_rng(71).standard_normal(S.ns) for i in range(S.r)])
    for i in range(S.r):
        G[i * S.ns + S.th.nvel:(i + 1) * S.ns] = 0.0  # zero pressure part: consistent for J^T
    lam = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    ia = g.irk_adjoint_solve(to_dev(G), lam, rtol=1e-8, maxit=200)
    assert ia["converged"] and np.all(np.isfinite(to_host(lam)))
    z = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    g.irk_mg_vcycle(to_dev(F), z)
    assert np.all(np.isfinite(to_host(z)))
    g.close()


@pytest.mark.parametrize("case", ["mx", "mc"])
def test_mhd_solve_on_poisoned_memory(poisoned, case):
    """The linearised MHD solver (damped sweeps and Chebyshev relaxation) on poisoned
    memory: FGMRES equal to the oracle's, equal iterations, 1e-10."""
    from oracle.fgmres import fgmres
    from test_gpu_mhd import CASES as MHD, _levels, _state, oracle_of as mhd_oracle
    from oracle.tableau import tableau
    from paper_2202_07381_amd import irkmg

    c = MHD[case]
    A, _, _ = tableau(c["fam"], c["r"])
    w0, b0 = _state(case)
    relax = dict(pre=3, post=3, weighting=0, smoother=1, interval=(2.0, 10.0)) if c.get("cheb") else {}
    say(f"[poison] mhd case={case}")
    g = irkmg.IrkMHD(_levels(case), A, c["dt"], c["Re"], c["Rem"], w0, b0, **relax)
    H = mhd_oracle(case)
    S = H.systems[-1]
    F = S.J @ np.random.default_rng(27).standard_normal(S.n)
    k = torch.zeros(F.size, dtype=torch.float64, device="cuda")
    info = g.irk_mhd_fgmres_solve(to_dev(F), k, rtol=1e-8, maxit=200, restart=30)
    xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 200, 30, project=S.project_pressure_mean)
    x = to_host(k)
    assert np.all(np.isfinite(x))
    assert info["iterations"] == io.iterations
    assert relerr(x, xo) < 1e-10
    z = torch.zeros(F.size, dtype=torch.float64, device="cuda")
    g.irk_mhd_vcycle(to_dev(F), z)
    assert relerr(to_host(z), H.vcycle(F)) < 1e-11
    g.close()
