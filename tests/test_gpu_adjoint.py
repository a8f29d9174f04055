"""GPU parity of the adjoint path (transposed solves and gradient assembly) against the
CPU oracle, and of the autograd gradient against finite differences.

Tolerances: building blocks 1e-13 relative; adjoint FGMRES after equal iteration
counts 1e-10; gradients of the 4-step tracking loss 1e-8 relative to the oracle's
(both sides solve to rtol 1e-13 / directly) and 1e-6 relative to central finite
differences with h = 1e-6 (the target stated for the method; the loss is quadratic in
the forcing, so there the difference quotient is exact up to solver error / h)."""
import numpy as np
import pytest

from gpu_cases import gpu_of, levels_of, oracle_of, relerr, say, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("case", ["c1", "oseen", "3d2"])
def test_adjoint_building_blocks(case):
    g, H = gpu_of(case), oracle_of(case)
    S = H.finest
    th = S.th
    rng = np.random.default_rng(31)
    lam = rng.standard_normal(S.n)
    say(f"[adj-blocks] case={case}")
    gf = torch.zeros(S.r * th.nnodes * th.dim, dtype=torch.float64, device="cuda")
    gs = torch.zeros(S.ns, dtype=torch.float64, device="cuda")
    g.irk_rhs_adjoint(to_dev(lam), gf, gs)
    lu = [lam[i * S.ns:i * S.ns + th.nvel] for i in range(S.r)]
    lp = [lam[i * S.ns + th.nvel:(i + 1) * S.ns] for i in range(S.r)]
    ref_f = np.stack([np.stack([S.Ms_free_all.T @ lu[i][c * th.nfree:(c + 1) * th.nfree] for c in range(th.dim)], 1)
                      for i in range(S.r)])
    assert relerr(to_host(gf).reshape(ref_f.shape), ref_f) < 1e-13
    su, sp = sum(lu), sum(lp)
    ref_s = np.concatenate([-(S.Lv.T @ su) - S.B @ sp, -(S.B.T @ su)])
    assert relerr(to_host(gs), ref_s) < 1e-13
    gbar = rng.standard_normal(S.ns)
    G = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    g.irk_update_adjoint(to_dev(gbar), G)
    assert relerr(to_host(G), np.concatenate([S.dt * g.b[i] * gbar for i in range(S.r)])) < 1e-15
    kk, st = rng.standard_normal(S.n), rng.standard_normal(S.ns)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    g.irk_nu_sensitivity(to_dev(lam), to_dev(kk), to_dev(st), out)
    K1v = S.Kv / S.nu
    ref = 0.0
    for i in range(S.r):
        ref -= lu[i] @ (K1v @ st[:th.nvel])
        for j in range(S.r):
            ref -= S.dt * S.A[i, j] * (lu[i] @ (K1v @ kk[j * S.ns:j * S.ns + th.nvel]))
    assert abs(to_host(out)[0] - ref) < 1e-12 * abs(ref)
    Mo = torch.zeros(S.ns, dtype=torch.float64, device="cuda")
    g.irk_mass_apply(to_dev(st), Mo)
    assert relerr(to_host(Mo), np.concatenate([S.Mv @ st[:th.nvel], np.zeros(th.nverts)])) < 1e-13
    # accumulating forms: the state adjoint and the viscosity sensitivity added in place
    pre = rng.standard_normal(S.ns)
    gs = to_dev(pre)
    g.irk_rhs_adjoint(to_dev(lam), gf, gs, accumulate=True)
    assert relerr(to_host(gs), pre + ref_s) < 1e-13
    out = to_dev(np.array([2.5]))
    g.irk_nu_sensitivity(to_dev(lam), to_dev(kk), to_dev(st), out, accumulate=True)
    assert abs(to_host(out)[0] - (2.5 + ref)) < 1e-12 * abs(2.5 + ref)
    # tracking loss 1/2 e^T M e (velocity part of state - target) and its gradients
    from oracle.adjoint import loss as oracle_loss

    tgt = rng.standard_normal(S.ns)
    Lg = torch.zeros(1, dtype=torch.float64, device="cuda")
    gsd, gtd = torch.zeros(S.ns, dtype=torch.float64, device="cuda"), torch.zeros(S.ns, dtype=torch.float64, device="cuda")
    g.irk_tracking_loss(to_dev(st), to_dev(tgt), loss=Lg, grad_state=gsd, grad_target=gtd,
                        scale=to_dev(np.array([0.75])))
    Lref = oracle_loss(S, st, tgt[:th.nvel])
    assert abs(to_host(Lg)[0] - Lref) < 1e-13 * abs(Lref)
    Me = np.concatenate([S.Mv @ (st[:th.nvel] - tgt[:th.nvel]), np.zeros(th.nverts)])
    assert relerr(to_host(gsd), 0.75 * Me) < 1e-13 and relerr(to_host(gtd), -0.75 * Me) < 1e-13
    # field offsets of the ABI layout
    off, ln = g.irk_mg_layout()
    assert list(ln) == [th.nfree] * th.dim + [th.nverts]
    for i in range(S.r):
        assert list(off[i]) == [i * S.ns + c * th.nfree for c in range(th.dim)] + [i * S.ns + th.nvel]


@pytest.mark.parametrize("case", ["c1", "oseen", "3d3"])
def test_adjoint_solve_matches_oracle(case):
    from oracle.fgmres import fgmres

    g, H = gpu_of(case), oracle_of(case)
    S = H.finest
    G = S.J.T @ np.random.default_rng(32).standard_normal(S.n)  # consistent right-hand side
    for rtol, maxit in ((1e-8, 200), (1e-30, 5)):
        say(f"[adj-solve] case={case} rtol={rtol}")
        lam = torch.zeros(S.n, dtype=torch.float64, device="cuda")
        info = g.irk_adjoint_solve(to_dev(G), lam, rtol=rtol, maxit=maxit)
        xo, io = fgmres(S.apply_transpose, H.vcycle_transpose, G, np.zeros_like(G), rtol, maxit, 30,
                        project=S.project_pressure_mean)
        assert info["iterations"] == io.iterations
        assert relerr(to_host(lam), xo) < 1e-10


def _theta_basis(th_nodes, dim):
    from paper_2202_07381_amd import workloads as wl

    base = wl.forcing_3d(5) if dim == 3 else wl.forcing_2d(1)
    m, d = base.theta.shape
    Phi = np.zeros((m * d, th_nodes.shape[0], dim))
    for q in range(m * d):
        e = np.zeros(m * d)
        e[q] = 1.0
        Phi[q] = base.with_theta(e.reshape(m, d))(th_nodes)
    return base.theta.ravel(), Phi


def _gpu_loss(g, Phi_t, theta_t, nu_t, s0, target, nsteps, rtol=1e-13):
    from paper_2202_07381_amd.adjoint import IrkSteps, tracking_loss

    f = torch.einsum("q,qnd->nd", theta_t, Phi_t)
    f_all = f.unsqueeze(0).unsqueeze(0).expand(nsteps, g.r, -1, -1)
    sN = IrkSteps.apply(f_all, nu_t, s0, g, rtol, 500)
    return tracking_loss(sN, target, g)


def test_gradient_matches_oracle_and_fd():
    from oracle.adjoint import gradient
    from oracle.timestep import dense_solver
    from paper_2202_07381_amd import irkmg
    from paper_2202_07381_amd import workloads as wl

    case, nsteps = "3d3", 4
    g, H = gpu_of(case), oracle_of(case)
    S = H.finest
    th = S.th
    theta0, Phi = _theta_basis(th.node_xyz, th.dim)
    target = np.zeros(S.ns)
    target[:th.nvel] = 0.01 * wl.random_vector(th.nvel, 50)
    s0 = np.zeros(S.ns)
    # oracle gradient (dense solves)
    f0 = np.einsum("q,qnd->nd", theta0, Phi)
    L_o, gf_o, gnu_o, _ = gradient(S, g.b, [[f0] * S.r] * nsteps, s0, target[:th.nvel], dense_solver(S),
                                   dense_solver(S, transpose=True))
    gtheta_o = np.array([sum(float(np.sum(gf_o[n][i] * Phi[q])) for n in range(nsteps) for i in range(S.r))
                         for q in range(Phi.shape[0])])
    # GPU gradient through autograd
    say("[adj-grad] case=3d3 autograd")
    Phi_t = to_dev(Phi)
    theta_t = to_dev(theta0).requires_grad_(True)
    nu_t = torch.tensor(g.nu, dtype=torch.float64, device="cuda", requires_grad=True)
    L = _gpu_loss(g, Phi_t, theta_t, nu_t, to_dev(s0), to_dev(target), nsteps)
    L.backward()
    torch.cuda.synchronize()
    assert abs(L.item() - L_o) < 1e-10 * abs(L_o)
    assert relerr(theta_t.grad.cpu().numpy(), gtheta_o) < 1e-8
    assert abs(nu_t.grad.item() - gnu_o) < 1e-8 * abs(gnu_o)
    # central finite differences on the GPU, h = 1e-6
    h = 1e-6
    v = np.random.default_rng(33).standard_normal(theta0.size)
    with torch.no_grad():
        say("[adj-grad] case=3d3 FD theta")
        Lp = _gpu_loss(g, Phi_t, to_dev(theta0 + h * v), nu_t.detach(), to_dev(s0), to_dev(target), nsteps).item()
        Lm = _gpu_loss(g, Phi_t, to_dev(theta0 - h * v), nu_t.detach(), to_dev(s0), to_dev(target), nsteps).item()
        fd = (Lp - Lm) / (2 * h)
        ad = float(theta_t.grad.cpu().numpy() @ v)
        assert abs(fd - ad) <= 1e-6 * abs(ad)
        say("[adj-grad] case=3d3 FD nu")
        lv = levels_of(case)
        A, b, c = irkmg.irk_tableau_builtin("radauIIA", 2)
        Ls = []
        for nu in (g.nu + h, g.nu - h):
            gg = irkmg.IrkMG(lv, A, b, c, g.dt, nu)
            Ls.append(_gpu_loss(gg, Phi_t, to_dev(theta0), torch.tensor(nu, dtype=torch.float64), to_dev(s0),
                                to_dev(target), nsteps).item())
            gg.close()
        fdn = (Ls[0] - Ls[1]) / (2 * h)
        assert abs(fdn - nu_t.grad.item()) <= 1e-6 * abs(nu_t.grad.item())
