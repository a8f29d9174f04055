"""Batched solves in one persistent launch: every solve of the batch against the
oracle's FGMRES (equal iteration counts, solutions within 1e-10 relative)."""
import numpy as np
import pytest

from gpu_cases import forcing_rhs, gpu_of, oracle_of, relerr, say, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BATCH = ["c1", "r3", "oseen", "be", "lob3"]


@pytest.mark.parametrize("autotune", [False, True])
def test_batch_matches_oracle(autotune):
    from oracle.fgmres import fgmres
    from paper_2202_07381_amd import irkmg

    gs = [gpu_of(c) for c in BATCH]
    Fs = [forcing_rhs(c) for c in BATCH]
    say(f"[batch] create autotune={autotune} n={len(gs)}")
    b = irkmg.IrkBatch(gs, autotune=autotune)
    ks = [torch.zeros(F.size, dtype=torch.float64, device="cuda") for F in Fs]
    say("[batch] solve")
    st, infos, ms = b.irk_batch_fgmres_solve([to_dev(F) for F in Fs], ks, rtol=1e-8, maxit=200, restart=30)
    say(f"[batch] done status={st} ms={ms:.2f} opts={b.irk_batch_get_opts()}")
    for c, info in zip(BATCH, infos):
        say(f"[batch] case={c} {info}")
    assert st == irkmg.IRK_OK
    for c, F, k, info in zip(BATCH, Fs, ks, infos):
        H = oracle_of(c)
        S = H.finest
        xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 200, 30, project=S.project_pressure_mean)
        say(f"[batch] case={c} its={info['iterations']} oracle={io.iterations} lat={info['latency_ms']:.3f}ms")
        assert info["converged"] and info["iterations"] == io.iterations
        assert info["rel_residual"] <= 1e-8
        assert relerr(to_host(k), xo) < 1e-10
    b.close()


def test_batch_maxit_and_restart():
    from paper_2202_07381_amd import irkmg

    gs = [gpu_of(c) for c in ("c1", "be")]
    Fs = [forcing_rhs(c) for c in ("c1", "be")]
    b = irkmg.IrkBatch(gs, autotune=False)
    ks = [torch.zeros(F.size, dtype=torch.float64, device="cuda") for F in Fs]
    say("[batch] maxit=2")
    st, infos, _ = b.irk_batch_fgmres_solve([to_dev(F) for F in Fs], ks, rtol=1e-12, maxit=2, restart=30)
    assert st == irkmg.IRK_ENOCONV and all(i["iterations"] == 2 for i in infos)
    # restart 4 with the individual solver as reference (same algorithm)
    say("[batch] restart=4")
    ks = [torch.zeros(F.size, dtype=torch.float64, device="cuda") for F in Fs]
    st, infos, _ = b.irk_batch_fgmres_solve([to_dev(F) for F in Fs], ks, rtol=1e-9, maxit=100, restart=4)
    for g, F, k, info in zip(gs, Fs, ks, infos):
        kk = torch.zeros_like(k)
        ref = g.irk_fgmres_solve(to_dev(F), kk, rtol=1e-9, maxit=100, restart=4)
        assert info["iterations"] == ref["iterations"]
        assert relerr(to_host(k), to_host(kk)) < 1e-11
    b.close()


def test_batch_bitwise_repeatable():
    """Work items may run on any workgroup in any order; every result must still be
    bitwise identical from one launch to the next (reductions are in item order)."""
    from paper_2202_07381_amd import irkmg

    gs = [gpu_of(c) for c in BATCH]
    Fs = [to_dev(forcing_rhs(c)) for c in BATCH]
    for wg in (1,):
        b = irkmg.IrkBatch(gs, workgroups_per_cu=wg, autotune=False)
        ref = None
        for rep in range(5):
            say(f"[batch-repeat] workgroups_per_cu={wg} rep={rep}")
            ks = [torch.zeros_like(F) for F in Fs]
            st, infos, _ = b.irk_batch_fgmres_solve(Fs, ks, rtol=1e-8, maxit=200, restart=30)
            assert st == irkmg.IRK_OK
            out = [to_host(k) for k in ks]
            if ref is None:
                ref = out
            else:
                assert all(np.array_equal(a, c) for a, c in zip(out, ref))
        b.close()


def test_batch_streams_mode_matches_one_by_one():
    """Concurrent-streams schedule on handles the persistent kernel does not run (FP32
    patches, Chebyshev relaxation, 3D) beside ordinary ones: every solution equals the
    one-by-one solve bitwise (the same deterministic kernels on another stream); with
    autotuning such a batch is scheduled on streams."""
    from paper_2202_07381_amd import irkmg

    cases = [("r3", dict(precision=1)), ("c1", dict(smoother=1)), ("3d2", {}), ("oseen", {}), ("lob3", {})]
    gs = [gpu_of(c, **kw) for c, kw in cases]
    Fs = [to_dev(forcing_rhs(c)) for c, _ in cases]
    ref = []
    for g, F in zip(gs, Fs):
        k = torch.zeros_like(F)
        info = g.irk_fgmres_solve(F, k, rtol=1e-8, maxit=200, restart=30)
        ref.append((to_host(k), info["iterations"]))
    for autotune in (False, True):
        say(f"[batch streams] autotune={autotune}")
        b = irkmg.IrkBatch(gs, autotune=autotune, mode=1, streams=3)
        ks = [torch.zeros_like(F) for F in Fs]
        st, infos, _ = b.irk_batch_fgmres_solve(Fs, ks, rtol=1e-8, maxit=200, restart=30)
        assert st == irkmg.IRK_OK and b.irk_batch_get_opts()["mode"] == 1
        for (kr, itr), k, info in zip(ref, ks, infos):
            assert info["converged"] and info["iterations"] == itr
            assert np.array_equal(to_host(k), kr)
        b.close()
    with pytest.raises(irkmg.IrkError):
        irkmg.IrkBatch(gs, autotune=False, mode=0)


# members of the uneven 64-solve batch (seed 4) with meshes up to 128 x 128: both stage
# counts, viscosities from 0.018 to 0.77
C4_SUBSET = [2, 9, 10, 11, 17, 19, 22]


def test_batch_c4_subset_persistent_matches_oracle():
    """The persistent launch (mode 0, no autotuning, so the one-launch schedule is the
    one that runs) on seven members of the uneven batch workload, each against the
    oracle's FGMRES: equal iteration counts, solutions within 1e-10 relative."""
    from oracle.fgmres import fgmres
    from oracle.multigrid import Hierarchy
    from oracle.tableau import tableau
    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    specs = wl.batch_specs()
    gs, Fs, Hs = [], [], []
    for j in C4_SUBSET:
        sp = specs[j]
        nl = int(np.log2(sp.n // 4)) + 1
        lv = wl.square_hierarchy(4, nl)
        A, b, c = irkmg.irk_tableau_builtin("radauIIA", sp.r)
        say(f"[batch-c4] member {j}: n={sp.n} r={sp.r} nu={sp.nu:.4f} levels={nl}")
        gs.append(irkmg.IrkMG(lv, A, b, c, sp.dt, sp.nu))
        H = Hierarchy(lv, tableau("radauIIA", sp.r)[0], sp.dt, sp.nu)
        S = H.finest
        f = wl.forcing_2d(sp.forcing_seed)
        Fs.append(S.rhs([S.th.interpolate(f, 0.0)] * S.r, np.zeros(S.th.nvel), np.zeros(S.th.nverts)))
        Hs.append(H)
    b = irkmg.IrkBatch(gs, autotune=False, mode=0)
    assert b.irk_batch_get_opts()["mode"] == 0
    ks = [torch.zeros(F.size, dtype=torch.float64, device="cuda") for F in Fs]
    say("[batch-c4] persistent solve")
    st, infos, ms = b.irk_batch_fgmres_solve([to_dev(F) for F in Fs], ks, rtol=1e-8, maxit=200, restart=30)
    assert st == irkmg.IRK_OK
    for j, H, F, k, info in zip(C4_SUBSET, Hs, Fs, ks, infos):
        S = H.finest
        xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 200, 30, project=S.project_pressure_mean)
        err = relerr(to_host(k), xo)
        say(f"[batch-c4] member {j}: its={info['iterations']} oracle={io.iterations} err={err:.2e} "
            f"latency={info['latency_ms']:.2f} ms")
        assert info["converged"] and info["iterations"] == io.iterations
        assert err < 1e-10
    b.close()
    for g in gs:
        g.close()
