#!/usr/bin/env python3
"""Benchmark of the stage-coupled Vanka multigrid path on one MI355X.

Workload (all inputs seeded and synthetic): 2D Stokes on the 256 x 256 triangulated
unit square, Taylor--Hood P2-P1 (588,291 unknowns per stage), 3-stage RadauIIA,
dt = 1e-2, nu = 1, manufactured solution from a 16-mode stream function (seed 2);
7-level geometric V-cycle (4 x 4 coarsest mesh) with 2 pre- and 2 post-sweeps of
the additive vertex-star Vanka smoother, omega = 0.5, preconditioning FGMRES(30) to a
relative residual of 1e-8.

A step is one IRK time step: right-hand side, FGMRES solve from a zero initial guess
(every V-cycle inside it: residuals, patch solves, transfers, coarse solve), and the
stage update.  Inputs (forcing at every stage time of every step) are resident in
device memory before the timed region.  The FP64 path gives the headline value; the
FP32-patch path (FP32 patch factors and V-cycle inside FP64 FGMRES) is reported
beside it, with its speedup and its solution difference from the FP64 path.

value = stage-DOF updates per second = (unknowns of the finest level) x (V-cycles
applied in the timed steps) / (timed wall time), so FGMRES, right-hand-side and
update work are charged to the V-cycles.

The roofline object is for the dominant kernel, the finest-level patch apply, timed
with HIP events around each of its launches on its own stream inside the timed
region; achieved = algorithmic bytes per launch / average launch time.
The cpu_baseline object times the CPU oracle on a bounded sample (the same workload on
the 128 x 128 mesh, 6 levels, by default; --cpu-n 256 for the benchmark mesh itself):
setup, one V-cycle and the full solve of the first step, BLAS on every core the
process may use.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Vanka V-cycle stage-DOF updates/s + time to 1e-8 rel. residual, FP32 vs FP64"
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_precision(precision, levels, A, b, c, dt, nu, mms, nodes, steps, warmup, profile):
    import numpy as np
    import torch

    from paper_2202_07381_amd import irkmg

    t0 = time.time()
    g = irkmg.IrkMG(levels, A, b, c, dt, nu, precision=precision)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    sz = g.irk_mg_sizes()
    _, free = g.irk_mg_p2_nodes()
    N = g.irk_mg_ndofs()
    r = len(b)
    log(f"precision={precision} setup {setup_s:.2f}s N={N}")
    u0 = mms.velocity(nodes[free], 0.0)
    state = torch.tensor(np.concatenate([u0[:, 0], u0[:, 1], np.zeros(sz["nverts"])]), device="cuda")
    nsteps = warmup + steps
    fdev = []
    for n in range(nsteps):
        fn = np.stack([mms(nodes, (n + ci) * dt) for ci in c])  # (r, nnodes, 2)
        fdev.append(torch.tensor(fn.ravel(), device="cuda"))
    F = torch.zeros(N, dtype=torch.float64, device="cuda")
    k = torch.zeros_like(F)
    its = []

    def step(n):
        g.irk_rhs(fdev[n], state, F)
        k.zero_()
        info = g.irk_fgmres_solve(F, k, rtol=1e-8, maxit=300, restart=30, history_cap=0)
        if not info["converged"]:
            raise RuntimeError(f"FGMRES did not converge at step {n}: {info}")
        g.irk_update(k, state)
        return info

    for n in range(warmup):
        step(n)
        log(f"precision={precision} warmup step {n} done")
    torch.cuda.synchronize()
    if profile:
        g.irk_mg_profile(1)  # events around the finest-level patch apply only
    t0 = time.perf_counter()
    infos = []
    for n in range(warmup, nsteps):
        infos.append(step(n))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if profile:
        g.irk_mg_profile(False)
    its = [i["iterations"] for i in infos]
    log(f"precision={precision} timed {steps} steps in {elapsed:.3f}s, iterations {its}")
    out = dict(
        N=N, setup_s=setup_s, elapsed_s=elapsed, iterations=its,
        rel_residual=max(i["rel_residual"] for i in infos),
        ms_per_step=1000.0 * elapsed / steps,
        value=N * sum(its) / elapsed,
        state=state.cpu().numpy(),
    )
    if profile:
        out["stats"] = {"patch_apply": g.irk_mg_kernel_stats("patch_apply", -1)}
        # the other finest-level kernels, from a separate profiled pass of 5 V-cycles
        rv0 = torch.tensor(np.random.default_rng(9).standard_normal(N), device="cuda")
        z0 = torch.zeros_like(rv0)
        g.irk_mg_profile(2)
        for _ in range(5):
            g.irk_mg_vcycle(rv0, z0)
        torch.cuda.synchronize()
        g.irk_mg_profile(False)
        for kname in ("residual", "gather_update"):
            out["stats"][kname] = g.irk_mg_kernel_stats(kname, -1)
    # V-cycle alone (preconditioner application on a fixed residual)
    rv = torch.tensor(np.random.default_rng(7).standard_normal(N), device="cuda")
    z = torch.zeros_like(rv)
    for _ in range(2):
        g.irk_mg_vcycle(rv, z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nv = 10
    e0.record()
    for _ in range(nv):
        g.irk_mg_vcycle(rv, z)
    e1.record()
    torch.cuda.synchronize()
    out["vcycle_ms"] = e0.elapsed_time(e1) / nv
    out["vcycle_updates_per_s"] = N / (out["vcycle_ms"] * 1e-3)
    g.close()
    return out


def run_mhd(base=5, nlevels=7, Re=5000.0, nv=5, relax="chebyshev"):
    """The linearised 2D MHD stage system (Sec. 3.3) of the island-coalescence workload
    (Sec. 5.3): LobattoIIIC(2), Re = Rem, dt = 0.025 at the paper's level l = 4 (halved
    per level), the crossed base x base mesh refined nlevels - 1 times (5 -> 320: the
    paper's l = 4 finest mesh size, 2.66M unknowns per stage), state w = 0 and the
    perturbed island field.  Relaxation: the paper's for its MHD runs, 3 / 3 Chebyshev
    steps on [2, 10] with the unweighted operator (relax "chebyshev"), or 2 / 2 damped
    weighted sweeps (relax "sweep").  Times the V-cycle, one FGMRES(30) solve to 1e-8 of
    J k = J x (x seeded N(0, 1)) from zero, and the finest level's kernels."""
    import numpy as np
    import torch

    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    lv = wl.crossed_hierarchy(base, nlevels)
    nfine = base * 2 ** (nlevels - 1)
    ell = int(round(np.log2(nfine / 20)))
    dt = 0.025 * 2.0 ** (4 - ell)
    w0, b0 = wl.island_coalescence(lv[-1].xyz, lv[-1].cells)
    A, _, _ = irkmg.irk_tableau_builtin("lobattoIIIC", 2)
    t0 = time.time()
    opts = dict(pre=3, post=3, weighting=0, smoother=1, interval=(2.0, 10.0)) if relax == "chebyshev" else {}
    g = irkmg.IrkMHD(lv, A, dt, Re, Re, w0, b0, **opts)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    n = g.irk_mhd_ndofs()
    log(f"mhd setup {setup_s:.1f}s N={n}")
    gen = torch.Generator(device="cuda").manual_seed(5)
    xt = torch.randn(n, dtype=torch.float64, device="cuda", generator=gen)
    F = torch.zeros_like(xt)
    g.irk_mhd_apply(-1, xt, F)
    z = torch.zeros_like(xt)
    for _ in range(2):
        g.irk_mhd_vcycle(xt, z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(nv):
        g.irk_mhd_vcycle(xt, z)
    e1.record()
    torch.cuda.synchronize()
    vms = e0.elapsed_time(e1) / nv
    k = torch.zeros_like(F)
    info = g.irk_mhd_fgmres_solve(F, k, rtol=1e-8, maxit=300, restart=30, history_cap=0)
    torch.cuda.synchronize()
    g.irk_mhd_profile(1)
    for _ in range(nv):
        g.irk_mhd_vcycle(xt, z)
    torch.cuda.synchronize()
    kern = {}
    for kname in ("patch_apply", "residual", "gather_update"):
        st = g.irk_mhd_kernel_stats(kname, -1)
        avg = st["ms_total"] / max(1, st["launches"])
        gbs = st["bytes_per_launch"] / max(1e-12, avg * 1e-3) / 1e9
        kern[kname] = {"launches": st["launches"], "avg_ms": avg, "bytes_per_launch": st["bytes_per_launch"],
                       "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS}
    g.irk_mhd_profile(0)
    lay = g.irk_mhd_layout()
    g.close()
    log(f"mhd V-cycle {vms:.2f} ms, FGMRES {info['iterations']} its {info['ms_total']:.1f} ms")
    rdesc = ("3/3 Chebyshev [2, 10] on the unweighted additive Vanka operator" if relax == "chebyshev"
             else "2/2 additive Vanka omega=0.5")
    return {
        "workload": f"linearised 2D MHD (island coalescence, w=0, perturbed B0), crossed {base}x{base} refined "
                    f"{nlevels - 1}x to {nfine}x{nfine}, P2/Nedelec/P1/P1, LobattoIIIC(2), dt={dt}, Re=Rem={Re:g}, "
                    f"{nlevels}-level V-cycle {rdesc}, patches factored through the stage eigenbasis, "
                    f"FGMRES(30) to 1e-8",
        "unknowns": n, "unknowns_per_stage": lay["ns"], "setup_s": setup_s,
        "vcycle_ms": vms, "vcycle_updates_per_s": n / (vms * 1e-3),
        "fgmres": {"iterations": info["iterations"], "ms": info["ms_total"], "rel_residual": info["rel_residual"],
                   "converged": info["converged"]},
        "kernels_finest_level": kern,
    }


def cpu_baseline(A, c, dt, nu, n):
    """The oracle on the host cores: setup (assembly of every level and the patch
    inverses), one V-cycle (mean of 2 after a warm-up) and the full FGMRES(30) solve
    of the first step to 1e-8, on the n x n member of the benchmark's workload family
    (same tableau, dt, nu and manufactured solution), with the BLAS thread pool set to
    the cores this process may run on."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.fgmres import fgmres
    from oracle.multigrid import Hierarchy
    from paper_2202_07381_amd import workloads as wl

    cores = len(os.sched_getaffinity(0))
    nlev = int(round(np.log2(n // 4))) + 1
    levels = wl.square_hierarchy(4, nlev)
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        H = Hierarchy(levels, A, dt, nu)
        setup_s = time.perf_counter() - t0
        log(f"oracle setup ({n}x{n}, {cores} threads) {setup_s:.1f}s")
        S = H.finest
        th = S.th
        N = S.n
        mms = wl.mms_2d(2, nu)
        u0 = th.free_velocity(th.interpolate(mms.velocity, 0.0))
        F = S.rhs([th.interpolate(mms, ci * dt) for ci in c], u0, np.zeros(th.nverts))
        rv = np.random.default_rng(7).standard_normal(N)
        H.vcycle(rv)
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            H.vcycle(rv)
        vcycle_s = (time.perf_counter() - t0) / reps
        log(f"oracle V-cycle {vcycle_s:.2f}s")
        t0 = time.perf_counter()
        _, info = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), 1e-8, 200, 30, project=S.project_pressure_mean)
        solve_s = time.perf_counter() - t0
        log(f"oracle FGMRES solve {solve_s:.1f}s, {info.iterations} iterations")
    out = {"value": N / vcycle_s, "unit": "stage-DOF updates/s", "cores": cores, "kind": "oracle",
           "sample": f"the oracle (NumPy/SciPy, FP64) on the {n}x{n} member of the benchmark workload "
                     f"({nlev} levels, {N} unknowns, RadauIIA(3), dt=1e-2, nu=1, MMS seed 2): setup, one "
                     f"V-cycle (value = unknowns / V-cycle time, the benchmark's unit) and the full "
                     f"FGMRES(30) solve of the first step to 1e-8; BLAS threads = {cores} (the patch "
                     f"inverses and sparse products run on one thread)",
           "n": n, "unknowns": N, "setup_s": setup_s, "vcycle_s": vcycle_s, "solve_s": solve_s,
           "solve_iterations": info.iterations}
    if n != 256:
        f = 4.0 ** round(np.log2(256 / n))
        out["extrapolated_to_256"] = {"factor": f, "setup_s": f * setup_s, "vcycle_s": f * vcycle_s,
                                      "solve_s": f * solve_s,
                                      "note": "every oracle step is linear in the number of unknowns"}
    return out


# ------------------------------------------------------------ HBM traffic (PMC)
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "patch_apply_traffic_stokes256_radau3.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2202_07381_amd", "csrc", f) for f in ("device_ops.h", "kernels.hip")]
CALIB_ELEMS = 1 << 27  # doubles per calibration copy (1 GiB read + 1 GiB written)


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def calibration_copies():
    """Plain elementwise copies of known size for scaling the FETCH/WRITE counters."""
    import torch

    src = torch.ones(CALIB_ELEMS, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log(f"calibration copies done: 3 x {CALIB_ELEMS * 8} bytes read and written")


def _pmc_rows(d, counter):
    import csv
    import glob

    out = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") != counter:
                continue
            key = (r["Kernel_Name"], int(r.get("Grid_Size") or 0))
            out.setdefault(key, []).append(float(r["Counter_Value"]))
    return out


PATCH_KERNELS = ("k_patch_apply_sym<double, 128", "k_patch_apply_eig<double, 1, 128")


def summarize_pmc(fetch_dir, write_dir, tags=PATCH_KERNELS):
    """Per-launch HBM bytes of the finest-level patch apply (the first kernel whose name
    contains one of tags) from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch), each scaled by what the same counter reads for the calibration copies
    (CALIB_ELEMS doubles in and out)."""
    res = {}
    for name, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _pmc_rows(d, counter)
        cal = [v for (k, g), vals in rows.items() if "neg_kernel" in k for v in vals]
        pa = {}
        for tag in tags:  # the form the workload uses (symmetric for Stokes)
            pa = {(k, g): vals for (k, g), vals in rows.items() if tag in k}
            if pa:
                res["kernel"] = tag
                break
        if not cal or not pa:
            raise SystemExit(f"{counter}: calibration or patch-apply dispatches missing in {d}")
        ideal_kib = CALIB_ELEMS * 8 / 1024.0
        scale = ideal_kib / (sum(cal) / len(cal))
        key = max(pa, key=lambda kg: kg[1])  # finest level: largest grid
        vals = pa[key]
        res[name] = dict(counter=counter, calib_measured_kib=sum(cal) / len(cal), calib_ideal_kib=ideal_kib,
                         scale=scale, dispatches=len(vals), grid=key[1],
                         raw_kib_per_launch=sum(vals) / len(vals),
                         bytes_per_launch=scale * 1024.0 * sum(vals) / len(vals))
    rec = {"kernel_source_sha256_16": kernel_source_hash(), "kernel": res.pop("kernel") + "> finest level",
           "traffic_bytes_per_launch": res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"],
           "fetch": res["fetch"], "write": res["write"]}
    print("traffic-record: " + json.dumps(rec))


def stored_traffic():
    """Calibrated HBM bytes per finest-level patch-apply launch from the committed PMC
    summary, or None when the kernel sources changed since the counters were taken."""
    try:
        for line in open(TRAFFIC_RECORD):
            if line.startswith("traffic-record: "):
                rec = json.loads(line[len("traffic-record: "):])
                if rec.get("kernel_source_sha256_16") == kernel_source_hash():
                    return rec["traffic_bytes_per_launch"]
                log("kernel sources changed since the PMC counters were taken: traffic = null")
                return None
    except OSError:
        pass
    return None


# ------------------------------------------------ mirror of the paper's 2D Stokes table
# Iterations per time step reported in Table 1 (2D Stokes, crossed 8x8 mesh refined l
# times, dt = 0.5/2^(l+3), Chebyshev [2, 8] with 2/2 steps): {(r, l): its/step}.
PAPER_T1_RADAU_ITS = {(2, 5): 8.70, (2, 6): 10.99, (2, 7): 14.22, (3, 5): 9.32, (3, 6): 12.40, (3, 7): 13.91}
# Table 3 (the same runs with the time step fixed at 0.5/2^8): iterations per step by
# (family, stages, level)
PAPER_T3_ITS = {("radauIIA", 2, 5): 8.70, ("radauIIA", 2, 6): 12.18, ("radauIIA", 2, 7): 18.04,
                ("radauIIA", 3, 5): 9.32, ("radauIIA", 3, 6): 14.22, ("radauIIA", 3, 7): 17.30,
                ("lobattoIIIC", 3, 5): 9.61, ("lobattoIIIC", 3, 6): 14.60, ("lobattoIIIC", 3, 7): 17.47}


def p2p1_errors(level, vel, p, exact):
    """L2 error of a P2 velocity field (nodal values at every node, numbering of the
    library: vertices, then edges sorted by (smaller, larger) vertex) against `exact`,
    by 25-point collapsed Gauss quadrature per cell; and the L2 norm of the P1 pressure
    after removing its integral mean (the exact pressure is zero)."""
    import numpy as np

    xyz, cells = level.xyz, level.cells
    nv = xyz.shape[0]
    pairs = [(0, 1), (1, 2), (0, 2)]
    keys = np.concatenate([np.sort(cells[:, [a, b]], axis=1) for a, b in pairs])
    code = keys[:, 0] * nv + keys[:, 1]
    _, inv = np.unique(code, return_inverse=True)
    edge_node = nv + inv.reshape(3, -1).T  # (nc, 3) nodes of edges 01, 12, 02
    gx, gw = np.polynomial.legendre.leggauss(5)
    gx, gw = 0.5 * (gx + 1.0), 0.5 * gw
    s_, t_ = np.meshgrid(gx, gx, indexing="ij")
    w2 = np.outer(gw, gw)
    l1 = s_ * (1.0 - t_)  # collapsed (Duffy) map to the reference triangle
    l2 = s_ * t_
    w = (w2 * s_).ravel()
    l1, l2 = l1.ravel(), l2.ravel()
    l0 = 1.0 - l1 - l2
    lam = np.stack([l0, l1, l2], axis=1)  # (nq, 3)
    phi_v = lam * (2.0 * lam - 1.0)
    phi_e = np.stack([4 * l0 * l1, 4 * l1 * l2, 4 * l0 * l2], axis=1)
    P = xyz[cells]  # (nc, 3, 2)
    det = np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                 - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1]))
    xq = np.einsum("qk,ckd->cqd", lam, P)
    uh = np.einsum("qk,ckd->cqd", phi_v, vel[cells]) + np.einsum("qk,ckd->cqd", phi_e, vel[edge_node])
    ue = exact(xq.reshape(-1, 2)).reshape(uh.shape)
    vel_err = np.sqrt(np.einsum("q,cqd,c->", w, (uh - ue) ** 2, det))
    area = 0.5 * det
    pc = p[cells]
    mean = np.sum(area * pc.sum(axis=1) / 3.0) / area.sum()
    pc = pc - mean
    p_err = np.sqrt(np.sum(area / 12.0 * (np.sum(pc ** 2, axis=1) + np.sum(pc, axis=1) ** 2)))
    return float(vel_err), float(p_err)


def run_t1(ell, r, precision=0, max_steps=None, log_every=32, fixed_rtol=None, auto_interval=False,
           family="radauIIA", dt_level=None):
    """The paper's 2D Stokes experiment (Sec. 5.1, Table 1): exact solution
    u = (sin(pi x) cos(pi y), -cos(pi x) sin(pi y)) e^{-2 pi^2 t}, p = 0 (so f = 0 and the
    boundary data drive the flow), nu = 1, RadauIIA(r) (or LobattoIIIC(r)), FGMRES with the
    Chebyshev-relaxed V-cycle, stopping at an absolute residual below 1e-2 N^-3 or a
    relative 1e-8.  dt = 0.5/2^(dt_level+3) with dt_level = ell (Table 1) or fixed at 5
    (Table 3: dt = 0.5/2^8 on every level)."""
    import math

    import numpy as np
    import torch

    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    levels = wl.crossed_hierarchy(8, ell + 1)
    A, b, c = irkmg.irk_tableau_builtin(family, r)
    nsteps = 2 ** ((ell if dt_level is None else dt_level) + 3)
    dt = 0.5 / nsteps
    t0 = time.time()
    g = irkmg.IrkMG(levels, A, b, c, dt, 1.0, weighting=0, precision=precision, smoother=1, interval=(2.0, 8.0))
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    interval = (2.0, 8.0)
    if auto_interval:
        # Sec. 5.1's rule [lambda/4, lambda], lambda the largest eigenvalue of S J, from 20
        # Arnoldi steps on the finest level (the paper tuned its interval by hand)
        top = len(levels) - 1
        v0 = torch.tensor(np.random.default_rng(5).standard_normal(g.irk_mg_ndofs(top)), device="cuda")
        _, ritz = g.irk_mg_ritz(top, 20, v0)
        lam = float(ritz[0].real)
        interval = (lam / 4, lam)
        g.irk_mg_set_interval(*interval)
        log(f"t1 interval from the Ritz estimate: [{interval[0]:.4f}, {interval[1]:.4f}]")
    nodes, free = g.irk_mg_p2_nodes()
    sz = g.irk_mg_sizes()
    N = g.irk_mg_ndofs()
    log(f"t1 l={ell} r={r} precision={precision} setup {setup_s:.1f}s unknowns {N} ({N // r} per stage)")

    def shape(x):  # spatial factor of the exact velocity
        return np.stack([np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1]),
                         -np.cos(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])], axis=1)

    u0 = shape(nodes)
    g0 = torch.tensor(u0.ravel(), device="cuda")
    decay = lambda t: math.exp(-2.0 * math.pi ** 2 * t)
    uf = u0[free]
    state = torch.tensor(np.concatenate([uf[:, 0], uf[:, 1], np.zeros(sz["nverts"])]), device="cuda")
    fzero = torch.zeros(r * sz["nnodes"] * 2, dtype=torch.float64, device="cuda")
    gst = torch.empty(r * sz["nnodes"] * 2, dtype=torch.float64, device="cuda")
    gn = torch.empty_like(g0)
    F = torch.zeros(N, dtype=torch.float64, device="cuda")
    k = torch.zeros_like(F)
    atol = 1e-2 * float(nsteps) ** -3
    steps = nsteps if max_steps is None else min(nsteps, max_steps)
    its = []
    torch.cuda.synchronize()
    tstart = time.perf_counter()
    for n in range(steps):
        tn = n * dt
        gn.copy_(g0).mul_(decay(tn))
        for i in range(r):
            gst[i * g0.numel():(i + 1) * g0.numel()].copy_(g0).mul_(decay(tn + float(c[i]) * dt))
        g.irk_rhs(fzero, state, F)
        g.irk_rhs_dirichlet(gn, gst, F)
        normF = float(torch.linalg.vector_norm(F))
        rtol = max(1e-8, atol / normF) if normF > 0 else 1e-8
        if fixed_rtol is not None:
            rtol = fixed_rtol
        k.zero_()
        info = g.irk_fgmres_solve(F, k, rtol=rtol, maxit=300, restart=30, history_cap=0)
        if not info["converged"]:
            raise RuntimeError(f"t1 step {n} did not converge: {info}")
        g.irk_update(k, state)
        its.append(info["iterations"])
        if (n + 1) % log_every == 0:
            log(f"t1 step {n + 1}/{steps}: mean its {sum(its) / len(its):.2f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - tstart
    T = steps * dt
    st = state.cpu().numpy()
    nf = sz["nfree"]
    vel = u0 * decay(T)  # boundary nodes keep the exact data
    vel[free, 0], vel[free, 1] = st[:nf], st[nf:2 * nf]
    vel_err, p_err = p2p1_errors(levels[-1], vel, st[2 * nf:], lambda x: shape(x) * decay(T))
    vel_err /= math.sqrt(0.5) * decay(T)  # exact L2 norm of u(T)
    mean_its = sum(its) / len(its)
    g.close()
    return {
        "metric": "paper 2D Stokes table mirror: FGMRES iterations per time step, time, t/K (Sec. 5.1, Table 1)",
        "value": mean_its, "unit": "iterations per step", "higher_is_better": False,
        "n_gpus": 1, "steps": steps, "dtype": "f64" if precision == 0 else "f64 (FP32 patches)",
        "data": "synthetic (the paper's exact solution)",
        "config": {"workload": f"2D Stokes, crossed 8x8 refined l={ell} times, {family}({r}), dt=0.5/{nsteps}, "
                               f"Chebyshev [{interval[0]:.4g},{interval[1]:.4g}] 2/2, unweighted additive Vanka, "
                               + (f"stop at {fixed_rtol:g} rel" if fixed_rtol is not None
                                  else "stop at 1e-2 N^-3 abs or 1e-8 rel"),
                   "l": ell, "stages": r, "unknowns": N, "dofs_per_stage": N // r, "time_steps_total": nsteps},
        "iterations_per_step_mean": mean_its, "iterations_min_max": [min(its), max(its)],
        "paper_iterations_per_step": (PAPER_T1_RADAU_ITS.get((r, ell)) if family == "radauIIA" and dt_level is None
                                      else PAPER_T3_ITS.get((family, r, ell)) if dt_level == 5 else None),
        "time_s": elapsed, "setup_s": setup_s, "t_per_krylov_it_ms": 1e3 * elapsed / sum(its),
        "final_time": T, "velocity_rel_l2_error": vel_err, "pressure_l2_error": p_err,
    }


def run_batch(count, log_every=8):
    """Uneven batch of independent solves through the batch entry point (autotuned over
    concurrent streams and the persistent kernel's tiles), beside the same solves one
    after another and the persistent one-launch schedule on its own."""
    import numpy as np
    import torch

    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    specs = wl.batch_specs(4, count)
    handles, Fs = [], []
    t0 = time.time()
    for j, sp in enumerate(specs):
        levels = wl.square_hierarchy(4, int(round(np.log2(sp.n // 4))) + 1)
        A, b, c = irkmg.irk_tableau_builtin("radauIIA", sp.r)
        g = irkmg.IrkMG(levels, A, b, c, sp.dt, sp.nu)
        nodes = irkmg.irk_mesh_p2_nodes(levels[-1])
        f = wl.forcing_2d(sp.forcing_seed)
        fn = np.stack([f(nodes)] * sp.r)
        sz = g.irk_mg_sizes()
        F = torch.zeros(g.irk_mg_ndofs(), dtype=torch.float64, device="cuda")
        g.irk_rhs(torch.tensor(fn.ravel(), device="cuda"), torch.zeros(sz["ns"], dtype=torch.float64, device="cuda"), F)
        handles.append(g)
        Fs.append(F)
        if (j + 1) % log_every == 0:
            log(f"batch setup {j + 1}/{count} ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()
    total_unknowns = sum(g.irk_mg_ndofs() for g in handles)
    # one after another
    ks = [torch.zeros_like(F) for F in Fs]
    for g, F, k in zip(handles[:2], Fs[:2], ks[:2]):
        g.irk_fgmres_solve(F, k, rtol=1e-8, maxit=300)
    torch.cuda.synchronize()
    seq_lat, seq_its = [], []
    t0 = time.perf_counter()
    for g, F, k in zip(handles, Fs, ks):
        k.zero_()
        info = g.irk_fgmres_solve(F, k, rtol=1e-8, maxit=300, history_cap=0)
        seq_its.append(info["iterations"])
        seq_lat.append((time.perf_counter() - t0) * 1e3)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    log(f"sequential {seq_s * 1e3:.1f} ms")
    # batched
    bt = irkmg.IrkBatch(handles, autotune=True)
    kb = [torch.zeros_like(F) for F in Fs]
    st, infos, _ = bt.irk_batch_fgmres_solve(Fs, kb, rtol=1e-8, maxit=300, restart=30)  # includes autotuning
    for k in kb:
        k.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, infos, ms = bt.irk_batch_fgmres_solve(Fs, kb, rtol=1e-8, maxit=300, restart=30)
    torch.cuda.synchronize()
    bat_s = time.perf_counter() - t0
    log(f"batched {bat_s * 1e3:.1f} ms, schedule {bt.irk_batch_get_opts()}")
    lat = np.array([i["latency_ms"] for i in infos])
    diff = max(float((kb[q] - ks[q]).norm() / ks[q].norm()) for q in range(count))
    # the persistent one-launch schedule alone, with its autotuned tiles
    bp = irkmg.IrkBatch(handles, autotune=False, mode=0, rows_per_item=4, patches_per_wave=4, workgroups_per_cu=1)
    kp = [torch.zeros_like(F) for F in Fs]
    bp.irk_batch_fgmres_solve(Fs, kp, rtol=1e-8, maxit=300, restart=30)
    for k in kp:
        k.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stp, infp, _ = bp.irk_batch_fgmres_solve(Fs, kp, rtol=1e-8, maxit=300, restart=30)
    torch.cuda.synchronize()
    per_s = time.perf_counter() - t0
    latp = np.array([i["latency_ms"] for i in infp])
    log(f"persistent one-launch {per_s * 1e3:.1f} ms")
    bp.close()
    its = [i["iterations"] for i in infos]
    vcycles = sum(its)
    line = {
        "metric": METRIC + " (batched workload)",
        "value": sum(g.irk_mg_ndofs() * i for g, i in zip(handles, its)) / bat_s,
        "unit": "stage-DOF updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": bat_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{count} independent 2D Stokes IRK solves, n in {{32,64,128,256}}, RadauIIA r in {{2,3}}, "
                               f"nu log-uniform [1e-2,1], dt=1e-2, seeds 4 / 4000+j, FGMRES(30) to 1e-8, batch entry point "
                               f"(autotuned schedule)",
                   "solves": count, "unknowns_total": total_unknowns},
        "status": st, "all_converged": all(i["converged"] for i in infos),
        "iterations_total": vcycles, "latency_ms_p50": float(np.percentile(lat, 50)),
        "latency_ms_p99": float(np.percentile(lat, 99)), "latency_ms_max": float(lat.max()),
        "sequential_ms": seq_s * 1e3, "speedup_vs_sequential": seq_s / bat_s,
        "sequential_latency_ms_p50": float(np.percentile(seq_lat, 50)),
        "sequential_latency_ms_p99": float(np.percentile(seq_lat, 99)),
        "max_rel_diff_vs_sequential": diff, "schedule": bt.irk_batch_get_opts(),
        "iterations_match_sequential": its == seq_its,
        "persistent_one_launch": {"ms": per_s * 1e3, "status": stp, "speedup_vs_sequential": seq_s / per_s,
                                  "latency_ms_p50": float(np.percentile(latp, 50)),
                                  "latency_ms_p99": float(np.percentile(latp, 99)),
                                  "schedule": {"rows_per_item": 4, "patches_per_wave": 4, "workgroups_per_cu": 1}},
    }
    print(json.dumps(line), flush=True)


def run_relax(n):
    """The three relaxations side by side (Sec. 4.2: Chebyshev or GMRES acceleration of
    the additive Vanka operator; the damped sweep): FGMRES(30) to 1e-8 on the 2D Oseen
    problem (n x n, Gauss(2), nu = 0.01, dt = 5e-3, unit-speed wind) and on the 2D Stokes
    problem of the headline line, FP64; iterations, time per solve and per V-cycle."""
    import numpy as np
    import torch

    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    relaxations = {"sweep": dict(smoother=0), "chebyshev": dict(smoother=1, weighting=0, interval=(2.0, 8.0)),
                   "gmres": dict(smoother=2)}
    problems = {
        f"oseen{n}": ("gauss", 2, 5e-3, 0.01, True),
        "stokes256": ("radauIIA", 3, 1e-2, 1.0, False),
    }
    out = {}
    for pname, (fam, r, dt, nu, convective) in problems.items():
        nn = n if convective else 256
        levels = wl.square_hierarchy(4, int(round(np.log2(nn // 4))) + 1)
        A, b, c = irkmg.irk_tableau_builtin(fam, r)
        nodes = irkmg.irk_mesh_p2_nodes(levels[-1])
        wind = wl.wind_2d(3, nn)(nodes) if convective else None
        f = wl.forcing_2d(3)
        for rname, kw in relaxations.items():
            t0 = time.time()
            g = irkmg.IrkMG(levels, A, b, c, dt, nu, wind_nodal=wind, **kw)
            torch.cuda.synchronize()
            setup = time.time() - t0
            N = g.irk_mg_ndofs()
            sz = g.irk_mg_sizes()
            F = torch.zeros(N, dtype=torch.float64, device="cuda")
            g.irk_rhs(torch.tensor(np.stack([f(nodes)] * r).ravel(), device="cuda"),
                      torch.zeros(sz["ns"], dtype=torch.float64, device="cuda"), F)
            k = torch.zeros_like(F)
            g.irk_fgmres_solve(F, k, rtol=1e-8, maxit=300)  # warm-up
            k.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            info = g.irk_fgmres_solve(F, k, rtol=1e-8, maxit=300)
            torch.cuda.synchronize()
            solve_ms = 1e3 * (time.perf_counter() - t1)
            z = torch.zeros_like(F)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for _ in range(5):
                g.irk_mg_vcycle(F, z)
            torch.cuda.synchronize()
            vc_ms = 1e3 * (time.perf_counter() - t2) / 5
            out.setdefault(pname, {})[rname] = {
                "converged": bool(info["converged"]), "iterations": info["iterations"],
                "rel_residual": info["rel_residual"], "solve_ms": solve_ms, "vcycle_ms": vc_ms, "setup_s": setup}
            log(f"relax {pname} {rname}: its {info['iterations']} solve {solve_ms:.1f} ms vcycle {vc_ms:.2f} ms")
            g.close()
    return {"metric": "FGMRES iterations and time to 1e-8 by relaxation (damped sweep, Chebyshev, GMRES)",
            "unit": "iterations / ms", "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"2D Oseen {n}x{n} Gauss(2) nu=0.01 dt=5e-3 unit wind; 2D Stokes 256x256 "
                                   "RadauIIA(3) dt=1e-2; 2/2 relaxation steps, FGMRES(30) to 1e-8"},
            "results": out}


def ns_element_flops(dim, r, ncells):
    """Algorithmic FP64 flops (an FMA counts 2) of one Jacobian-mode launch of the
    Navier--Stokes element kernel: per (cell, stage) the stage mix of the direction
    (nloc dim r FMAs) and, at each quadrature point (7 in 2D, 14 in 3D), the wind and z
    at the point (2 nloc dim), their components along the dim+1 gradients of the
    barycentric coordinates (2 (dim+1) dim), the barycentric derivatives of z and U
    (2 (dim+1)(1+dim) dim: 1 + dim nonzero basis derivatives per coordinate), the two
    directional derivatives (2 (dim+1) dim), the weighted test functions (nloc) and the
    accumulation (nloc dim)."""
    nl, nb, nq = (6, 3, 7) if dim == 2 else (10, 4, 14)
    per_point = 2 * nl * dim + 2 * nb * dim + 2 * nb * (1 + dim) * dim + 2 * nb * dim + nl + nl * dim
    fma = nq * per_point + nl * dim * r
    return 2.0 * fma * ncells * r


def run_ns(n, nsteps, smoother, precond="oseen", dt=1.0 / 400, dim=2, nu=0.01, eta_fixed=0.0):
    """Navier--Stokes time stepping (Sec. 3.2): Newton with Eisenstat--Walker forcing,
    FGMRES preconditioned by the V-cycle of the Oseen operator linearised at the initial
    state (precond "oseen"; set up once, kept for every step), of the Stokes operator
    ("stokes"), or of the Newton Jacobian itself, rediscretised on every level at each
    Newton iterate ("newton", Sec. 3.2; its set-up time is part of the step), 2D n x n, RadauIIA(3), nu = 0.01 (Re = 100 for unit speed and length),
    dt = 1/400 (the paper's cylinder run), a unit-speed divergence-free initial state and a
    smooth body force, all synthetic.  dim = 3: the n^3 cube (Kuhn tetrahedra), RadauIIA(2),
    initial state and force from the 3D forcing modes."""
    import numpy as np
    import torch

    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    fam, r = "radauIIA", 3 if dim == 2 else 2
    if dim == 2:
        levels = wl.square_hierarchy(4, int(round(np.log2(n // 4))) + 1)
    else:
        levels = wl.cube_hierarchy(2, int(round(np.log2(n // 2))) + 1)
    A, b, c = irkmg.irk_tableau_builtin(fam, r)
    nodes = irkmg.irk_mesh_p2_nodes(levels[-1])
    if dim == 2:
        u0 = wl.wind_2d(3, n)(nodes)
    else:
        u0 = wl.forcing_3d(4)(nodes, 0.0)
        u0 /= np.abs(u0).max()
    kw = {"sweep": dict(smoother=0), "chebyshev": dict(smoother=1, weighting=0, interval=(1.5, 8.0)),
          "gmres": dict(smoother=2)}[smoother]
    t0 = time.time()
    g = irkmg.IrkMG(levels, A, b, c, dt, nu, wind_nodal=u0 if precond == "oseen" else None, **kw)
    pc = 1 if precond == "newton" else 0
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    form = g.irk_mg_patch_form()
    sz = g.irk_mg_sizes()
    N = g.irk_mg_ndofs()
    free = g.irk_mg_p2_nodes()[1]
    state = torch.zeros(sz["ns"], dtype=torch.float64, device="cuda")
    state[: dim * sz["nfree"]] = torch.tensor(np.concatenate([u0[free, d] for d in range(dim)]), device="cuda")
    f = wl.forcing_2d(3) if dim == 2 else wl.forcing_3d(3)
    fst = torch.tensor(np.stack([f(nodes)] * r).ravel(), device="cuda")
    k = torch.zeros(N, dtype=torch.float64, device="cuda")
    F = torch.zeros_like(k)
    log(f"ns {n}^{dim}: N={N} setup {setup_s:.1f} s")
    steps = []
    for it in range(nsteps):
        if it == 1:
            g.irk_mg_profile(2)  # kernel times from the second step on
        g.irk_rhs(fst, state, F)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = g.irk_ns_newton_solve(F, state, k, rtol=1e-8, eta_fixed=eta_fixed, precond=pc)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t1)
        g.irk_update(k, state)
        steps.append({"newton": info["iterations"], "linear": info["linear_its"].tolist(), "ms": ms,
                      "converged": info["converged"]})
        log(f"ns step {it}: newton {info['iterations']} linear {info['linear_its'].tolist()} {ms:.1f} ms")
    pa = g.irk_mg_kernel_stats("patch_apply")
    # the element kernel and its gather in Jacobian mode alone (the residual mode does one
    # of the two tensor contractions): 20 Jacobian actions at the last iterate
    g.irk_mg_profile(2)
    x = torch.ones_like(k)
    y = torch.empty_like(k)
    for _ in range(20):
        g.irk_ns_jacobian_apply(state, k, x, y)
    se, sg = g.irk_mg_kernel_stats("ns_element"), g.irk_mg_kernel_stats("ns_gather")
    g.irk_mg_profile(0)
    e_ms = se["ms_total"] / max(1, se["launches"])
    gat_ms = sg["ms_total"] / max(1, sg["launches"])
    ncells = levels[-1].cells.shape[0]
    flops = ns_element_flops(dim, r, ncells)
    g.close()
    t = steps[1:] if len(steps) > 1 else steps
    return {"metric": "Navier--Stokes IRK time step (Newton-Krylov-multigrid)", "unit": "ms / step",
            "value": float(np.mean([s["ms"] for s in t])), "higher_is_better": False, "n_gpus": 1,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{dim}D Navier-Stokes {n}^{dim} RadauIIA({r}) nu={nu:g} dt={dt:g}, relaxation {smoother}, "
                                   f"{precond} preconditioner (Oseen: linearised at the initial state), "
                                   "Newton to 1e-8"},
            "patch_form": form,
            "setup_s": setup_s, "steps": steps,
            "newton_per_step": float(np.mean([s["newton"] for s in t])),
            "linear_per_step": float(np.mean([sum(s["linear"]) for s in t])),
            "kernels": {"ns_element_us": 1e3 * e_ms, "ns_element_launches": se["launches"],
                        "ns_gather_us": 1e3 * gat_ms, "ns_gather_bytes": sg["bytes_per_launch"],
                        "patch_apply_us": 1e3 * pa["ms_total"] / max(1, pa["launches"])},
            "roofline_ns_element": {"bound": "alu", "achieved": flops / (e_ms * 1e-3) / 1e12, "peak": 78.6,
                                    "unit": "TFLOP/s", "frac": flops / (e_ms * 1e-3) / 1e12 / 78.6,
                                    "flops_per_launch": flops,
                                    "bytes_per_launch": se["bytes_per_launch"],
                                    "hbm_GBps": se["bytes_per_launch"] / (e_ms * 1e-3) / 1e9},
            "roofline_ns_gather": {"bound": "hbm", "achieved": sg["bytes_per_launch"] / (gat_ms * 1e-3) / 1e9,
                                   "peak": 8000.0, "unit": "GB/s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="finest mesh size (power-of-two multiple of 4)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=128,
                    help="mesh of the oracle timing (256: the benchmark mesh itself, about 35 GB and minutes)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-mhd", action="store_true", help="skip the linearised MHD measurement")
    ap.add_argument("--mhd-relax", default="chebyshev", choices=["chebyshev", "sweep"],
                    help="mhd: the paper's 3/3 Chebyshev [2, 10] or 2/2 damped sweeps")
    ap.add_argument("--mhd-re", type=float, default=5000.0, help="mhd: Re = Rem")
    ap.add_argument("--workload", default="stokes256", choices=["stokes256", "batch64", "t1", "relax", "ns", "mhd"],
                    help="stokes256: the headline line; batch64: the uneven batched workload; t1: the paper's "
                         "2D Stokes table; relax: the three relaxations side by side; ns: Navier-Stokes "
                         "time steps with Newton")
    ap.add_argument("--ns-n", type=int, default=256, help="ns: finest mesh size")
    ap.add_argument("--ns-steps", type=int, default=6, help="ns: time steps")
    ap.add_argument("--ns-relax", default="sweep", choices=["sweep", "chebyshev", "gmres"], help="ns: relaxation")
    ap.add_argument("--ns-dim", type=int, default=2, choices=[2, 3], help="ns: 2 (square) or 3 (cube)")
    ap.add_argument("--ns-nu", type=float, default=0.01, help="ns: viscosity (1/Re for unit speed and length)")
    ap.add_argument("--ns-eta-fixed", type=float, default=0.0,
                    help="ns: constant forcing term instead of Eisenstat-Walker (e.g. 1e-8 to count iterations "
                         "of tight linear solves)")
    ap.add_argument("--ns-dt", type=float, default=1.0 / 400, help="ns: time step (default the cylinder run's 1/400)")
    ap.add_argument("--ns-precond", default="oseen", choices=["oseen", "stokes", "newton"],
                    help="ns: operator of the V-cycle (Oseen at the initial state, Stokes, or the Newton "
                         "Jacobian at every iterate)")
    ap.add_argument("--relax-n", type=int, default=512, help="relax: finest mesh size of the Oseen problem")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--t1-level", type=int, default=5, help="t1: refinement level l of the crossed 8x8 mesh")
    ap.add_argument("--t1-stages", type=int, default=2, choices=[2, 3], help="t1: RadauIIA stages")
    ap.add_argument("--t1-family", default="radauIIA", choices=["radauIIA", "gauss", "lobattoIIIC"],
                    help="t1: IRK family")
    ap.add_argument("--t1-dt-level", type=int, default=None,
                    help="t1: dt = 0.5/2^(this+3) instead of the level's own (5: the fixed step of Table 3)")
    ap.add_argument("--t1-max-steps", type=int, default=None, help="t1: stop after this many time steps")
    ap.add_argument("--t1-fp32", action="store_true", help="t1: FP32 patch factors")
    ap.add_argument("--t1-auto-interval", action="store_true",
                    help="t1: Chebyshev interval [lambda/4, lambda] from a Ritz estimate instead of [2, 8]")
    ap.add_argument("--t1-rtol", type=float, default=None,
                    help="t1: fixed relative tolerance instead of the paper's stopping rule")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run plain copies of known size (for scaling PMC byte counters)")
    ap.add_argument("--pmc-kernel", action="append", default=None,
                    help="with --summarize-pmc: kernel name fragment(s) to summarise (default: the patch apply "
                         "of the headline workload)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the traffic record from two rocprofv3 --pmc output directories and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, tags=tuple(args.pmc_kernel) if args.pmc_kernel else PATCH_KERNELS)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(one process per GPU, sharded by subdomain, is the design); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batch64":
        run_batch(args.batch_count)
        return
    if args.workload == "relax":
        print(json.dumps(run_relax(args.relax_n)), flush=True)
        return
    if args.workload == "ns":
        print(json.dumps(run_ns(args.ns_n, args.ns_steps, args.ns_relax, args.ns_precond, args.ns_dt, args.ns_dim,
                                args.ns_nu, args.ns_eta_fixed)), flush=True)
        return
    if args.workload == "mhd":
        print(json.dumps(run_mhd(Re=args.mhd_re, relax=args.mhd_relax)), flush=True)
        if args.calibrate_copy:
            calibration_copies()
        return
    if args.workload == "t1":
        print(json.dumps(run_t1(args.t1_level, args.t1_stages, 1 if args.t1_fp32 else 0, args.t1_max_steps,
                                family=args.t1_family, dt_level=args.t1_dt_level,
                                fixed_rtol=args.t1_rtol, auto_interval=args.t1_auto_interval)), flush=True)
        return
    nlev = int(round(np.log2(args.n // 4))) + 1
    levels = wl.square_hierarchy(4, nlev)
    A, b, c = irkmg.irk_tableau_builtin("radauIIA", 3)
    dt, nu = 1e-2, 1.0
    mms = wl.mms_2d(2, nu)
    nodes = irkmg.irk_mesh_p2_nodes(levels[-1])

    r64 = run_precision(0, levels, A, b, c, dt, nu, mms, nodes, args.steps, args.warmup, profile=True)
    r32 = None if args.no_fp32 else run_precision(1, levels, A, b, c, dt, nu, mms, nodes, args.steps, args.warmup,
                                                  profile=True)
    st = r64["stats"]["patch_apply"]
    avg_ms = st["ms_total"] / max(1, st["launches"])
    achieved = st["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "stage-DOF updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D Stokes {args.n}x{args.n} P2-P1, RadauIIA(3), dt=1e-2, nu=1, MMS seed 2, "
                        f"{nlev}-level V-cycle 2/2 additive Vanka omega=0.5, FGMRES(30) to 1e-8",
            "n": args.n, "levels": nlev, "stages": 3, "unknowns": r64["N"],
        },
        "time_to_1e-8_ms": r64["ms_per_step"],
        "iterations_per_step": r64["iterations"],
        "max_rel_residual": r64["rel_residual"],
        "vcycle_ms": r64["vcycle_ms"],
        "vcycle_only_updates_per_s": r64["vcycle_updates_per_s"],
        "setup_s": r64["setup_s"],
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(),
            "kernel": "patch_apply (finest level)", "avg_launch_ms": avg_ms, "launches": st["launches"],
            "bytes_per_launch": st["bytes_per_launch"],
        },
        "kernels_finest_level": {k: {"launches": v["launches"], "avg_ms": v["ms_total"] / max(1, v["launches"]),
                                     "GB/s": v["bytes_per_launch"] / max(1e-12, v["ms_total"] / max(1, v["launches"]) * 1e-3) / 1e9}
                                 for k, v in r64["stats"].items()},
    }
    if r32 is not None:
        s32 = r32["stats"]["patch_apply"]
        ms32 = s32["ms_total"] / max(1, s32["launches"])
        diff = float(np.linalg.norm(r32["state"] - r64["state"]) / np.linalg.norm(r64["state"]))
        line["fp32_patch"] = {
            "value": r32["value"], "ms_per_step": r32["ms_per_step"], "iterations_per_step": r32["iterations"],
            "max_rel_residual": r32["rel_residual"], "vcycle_ms": r32["vcycle_ms"],
            "vcycle_only_updates_per_s": r32["vcycle_updates_per_s"],
            "speedup_vs_fp64_step": r64["ms_per_step"] / r32["ms_per_step"],
            "speedup_vs_fp64_vcycle": r64["vcycle_ms"] / r32["vcycle_ms"],
            "state_rel_diff_vs_fp64": diff,
            "patch_apply_GB/s": s32["bytes_per_launch"] / (ms32 * 1e-3) / 1e9,
        }
    if not args.no_mhd:
        line["mhd"] = run_mhd(Re=args.mhd_re, relax=args.mhd_relax)
    if args.calibrate_copy:
        calibration_copies()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(A, c, dt, nu, args.cpu_n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
