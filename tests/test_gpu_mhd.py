"""GPU parity of the linearised 2D MHD stage solver (irk_mhd_*, include/irk_mhd.h) against
the oracle (oracle/mhd.py; Sec. 3.3, 4.1, 4.2, Fig. 1 right), through the C ABI.

Cases: a diagonal-split hierarchy 2 -> 8 with LobattoIIIC(2), a random linearisation
velocity and the island-coalescence field; the same with RadauIIA(1) (implicit Euler); a diagonal-split 2 -> 16 hierarchy with
RadauIIA(3) (stage-coupled patches of up to 156 unknowns: the factorisation takes the
blocked global-memory path); a crossed 2 -> 8 hierarchy (vertices of valence 8 and 4, the
mesh family of the paper's island-coalescence runs) at Re = Rem = 5000, with the damped
sweep and with the paper's MHD relaxation (3 / 3 Chebyshev steps on [2, 10], Sec. 5.1,
5.3; a level sweep is then one Chebyshev step).
Tolerances as for the fluid solver: single operator applications 1e-13 relative to the
largest entry; patch sweeps 1e-11; the coarse solve max(1e-12, 4 cond_S(J_0) eps)
(Skeel's componentwise condition number of the pinned coarse operator); V-cycles 1e-11;
FGMRES solutions after equal iteration counts 1e-10.  Sweeps, V-cycles and solves run
with both patch forms: dense inverses (0) and the automatic choice (2), which for r >= 2
stores each inverse factored through the stage eigenbasis (the same operator up to
rounding)."""
import numpy as np
import pytest

from gpu_cases import relerr, say, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "m2": dict(mesh="square", nc=2, nl=3, fam="lobattoIIIC", r=2, dt=0.025, Re=100.0, Rem=50.0, seed=3),
    "m3": dict(mesh="square", nc=2, nl=4, fam="radauIIA", r=3, dt=0.01, Re=1000.0, Rem=1000.0, seed=None),
    "mx": dict(mesh="crossed", nc=2, nl=3, fam="lobattoIIIC", r=2, dt=0.025, Re=5000.0, Rem=5000.0, seed=None),
    "m1": dict(mesh="square", nc=2, nl=3, fam="radauIIA", r=1, dt=0.05, Re=100.0, Rem=100.0, seed=5),
    # the paper's MHD relaxation: 3 / 3 Chebyshev steps on [2, 10], unweighted operator
    "mc": dict(mesh="crossed", nc=2, nl=3, fam="lobattoIIIC", r=2, dt=0.025, Re=5000.0, Rem=5000.0, seed=None,
               cheb=True),
}
_G, _H = {}, {}
FORMS = [0, 2]


def _levels(case):
    from paper_2202_07381_amd import workloads as wl

    c = CASES[case]
    return (wl.square_hierarchy if c["mesh"] == "square" else wl.crossed_hierarchy)(c["nc"], c["nl"])


def _state(case):
    from paper_2202_07381_amd import workloads as wl

    lv = _levels(case)
    w0, b0 = wl.island_coalescence(lv[-1].xyz, lv[-1].cells)
    if CASES[case]["seed"] is not None:
        w0 = 0.3 * np.random.default_rng(CASES[case]["seed"]).standard_normal(w0.shape)
    return w0, b0


def oracle_of(case):
    if case not in _H:
        from oracle.mhd import MHDHierarchy
        from oracle.tableau import tableau

        c = CASES[case]
        A, _, _ = tableau(c["fam"], c["r"])
        w0, b0 = _state(case)
        if c.get("cheb"):
            _H[case] = MHDHierarchy(_levels(case), A, c["dt"], c["Re"], c["Rem"], w0, b0, weighted=False, pre=3,
                                    post=3, smoother="chebyshev", interval=(2.0, 10.0))
        else:
            _H[case] = MHDHierarchy(_levels(case), A, c["dt"], c["Re"], c["Rem"], w0, b0)
    return _H[case]


def gpu_of(case, form=2):
    if (case, form) not in _G:
        from oracle.tableau import tableau
        from paper_2202_07381_amd import irkmg

        c = CASES[case]
        A, _, _ = tableau(c["fam"], c["r"])
        w0, b0 = _state(case)
        say(f"[mhd-setup] case={case} form={form}")
        relax = dict(pre=3, post=3, weighting=0, smoother=1, interval=(2.0, 10.0)) if c.get("cheb") else {}
        _G[(case, form)] = irkmg.IrkMHD(_levels(case), A, c["dt"], c["Re"], c["Rem"], w0, b0, patch_form=form,
                                        **relax)
    return _G[(case, form)]


def _skeel_tol(H):
    J = H.ops[0].toarray()
    for q in H.pinned:
        J[q, :] = 0.0
        J[:, q] = 0.0
        J[q, q] = 1.0
    cs = float(np.max(np.abs(np.linalg.inv(J)) @ np.abs(J) @ np.ones(J.shape[0])))
    return max(1e-12, 4 * cs * np.finfo(float).eps)


@pytest.mark.parametrize("case", list(CASES))
def test_layout_and_sizes(case):
    g, H = gpu_of(case), oracle_of(case)
    for lev, s in enumerate(H.spaces):
        lay = g.irk_mhd_layout(lev)
        assert (lay["u_x"], lay["u_y"], lay["B"], lay["p"], lay["gamma"], lay["ns"]) == (
            0, s.nu_ // 2, s.off_B, s.off_p, s.off_g, s.ns)
        assert lay["r"] == H.r and g.irk_mhd_ndofs(lev) == H.r * s.ns


@pytest.mark.parametrize("case", list(CASES))
def test_apply_all_levels(case):
    g, H = gpu_of(case), oracle_of(case)
    rng = np.random.default_rng(21)
    for lev in range(g.nlevels):
        J = H.systems[lev].J
        x = rng.standard_normal(J.shape[0])
        say(f"[mhd-apply] case={case} level={lev}")
        y = torch.zeros(J.shape[0], dtype=torch.float64, device="cuda")
        g.irk_mhd_apply(lev, to_dev(x), y)
        assert relerr(to_host(y), J @ x) < 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_transfers(case):
    g, H = gpu_of(case), oracle_of(case)
    rng = np.random.default_rng(22)
    for lev in range(1, g.nlevels):
        P = H.P[lev]
        xf, xc, base = rng.standard_normal(P.shape[0]), rng.standard_normal(P.shape[1]), rng.standard_normal(P.shape[0])
        say(f"[mhd-transfer] case={case} level={lev}")
        out = torch.zeros(P.shape[1], dtype=torch.float64, device="cuda")
        g.irk_mhd_restrict(lev, to_dev(xf), out)
        assert relerr(to_host(out), P.T @ xf) < 1e-13
        fine = to_dev(base)
        g.irk_mhd_prolong(lev, to_dev(xc), fine)
        assert relerr(to_host(fine), base + P @ xc) < 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_coarse_solve(case):
    g, H = gpu_of(case), oracle_of(case)
    J0 = H.systems[0].J
    b = J0 @ np.random.default_rng(23).standard_normal(J0.shape[0])
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    g.irk_mhd_coarse_solve(to_dev(b), x)
    err, tol = relerr(to_host(x), H.coarse_solve(b)), _skeel_tol(H)
    say(f"[mhd-coarse] case={case} err={err:.2e} tol={tol:.2e}")
    assert err < tol


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("case", list(CASES))
def test_sweep_each_level(case, form):
    g, H = gpu_of(case, form), oracle_of(case)
    # the automatic form factors through the stage eigenbasis for r >= 2 only
    assert g.irk_mhd_patch_form() == (1 if form == 2 and CASES[case]["r"] >= 2 else 0)
    rng = np.random.default_rng(24)
    for lev in range(1, g.nlevels):
        J = H.systems[lev].J
        F, k0 = rng.standard_normal(J.shape[0]), rng.standard_normal(J.shape[0])
        say(f"[mhd-sweep] case={case} form={form} level={lev}")
        k = to_dev(k0)
        g.irk_mhd_sweep(lev, to_dev(F), k)
        if CASES[case].get("cheb"):
            ref = H.smoothers[lev].chebyshev(F, k0, J, 1, 2.0, 10.0)
        else:
            ref = H.smoothers[lev].sweep(F, k0, J)
        err = relerr(to_host(k), ref)
        say(f"[mhd-sweep] case={case} form={form} level={lev} err={err:.2e}")
        assert err < 1e-11


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("case", list(CASES))
def test_vcycle(case, form):
    g, H = gpu_of(case, form), oracle_of(case)
    r = np.random.default_rng(25).standard_normal(g.irk_mhd_ndofs())
    say(f"[mhd-vcycle] case={case}")
    z = torch.zeros(r.size, dtype=torch.float64, device="cuda")
    g.irk_mhd_vcycle(to_dev(r), z)
    err = relerr(to_host(z), H.vcycle(r))
    say(f"[mhd-vcycle] case={case} form={form} err={err:.2e}")
    assert err < 1e-11


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("case", list(CASES))
def test_fgmres_matches_oracle(case, form):
    from oracle.fgmres import fgmres

    g, H = gpu_of(case, form), oracle_of(case)
    S = H.systems[-1]
    F = S.J @ np.random.default_rng(26).standard_normal(S.n)
    for rtol, maxit in ((1e-8, 200), (1e-30, 4)):
        say(f"[mhd-fgmres] case={case} rtol={rtol} maxit={maxit}")
        k = torch.zeros(F.size, dtype=torch.float64, device="cuda")
        info = g.irk_mhd_fgmres_solve(to_dev(F), k, rtol=rtol, maxit=maxit, restart=30)
        xo, io = fgmres(S.apply, H.vcycle, F, np.zeros_like(F), rtol, maxit, 30, project=S.project_pressure_mean)
        err = relerr(to_host(k), xo)
        say(f"[mhd-fgmres] case={case} form={form} its={info['iterations']} oracle_its={io.iterations} "
            f"err={err:.2e}")
        assert info["iterations"] == io.iterations
        assert err < 1e-10
        if rtol > 1e-20:
            assert info["converged"] and info["rel_residual"] <= rtol


def test_argument_errors():
    from paper_2202_07381_amd import irkmg

    g = gpu_of("m2")
    n = g.irk_mhd_ndofs()
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    x0 = torch.zeros(g.irk_mhd_ndofs(0), dtype=torch.float64, device="cuda")
    with pytest.raises(irkmg.IrkError) as e:  # no sweep on the coarsest level
        g.irk_mhd_sweep(0, x0, x0.clone())
    assert e.value.status == irkmg.IRK_EINVAL
    with pytest.raises(irkmg.IrkError) as e:
        g.irk_mhd_vcycle(x, x)
    assert e.value.status == irkmg.IRK_EINVAL
    with pytest.raises(ValueError):
        g.irk_mhd_apply(-1, torch.zeros(n + 1, dtype=torch.float64, device="cuda"), x)
