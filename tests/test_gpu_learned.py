"""GPU parity of the learned correction: the network's HIP kernels (forward, gradients, input
features) against the CPU reference oracle/learned_ref.py, and the learned solve against the plain
solve and against a CPU emulation built from the two CPU references.

Tolerances.  Both sides round the same convolution operands to BF16; the GPU sums in FP32 (MFMA)
where the reference sums exactly, so a layer output differs by ~1e-6 relative, and an activation
that lies within that distance of a BF16 rounding boundary rounds the other way on one side (one
BF16 unit, 2^-8 relative, in a fraction ~1e-4 of the elements).  Forward outputs therefore agree to
~1e-4 relative L2 (bound used: 1e-3).  The backward pass rounds the upstream gradient to BF16 once
per layer, so the flips compound towards the first layer: a variant of the reference that only
accumulates in FP32 instead of exactly differs from it, at n = 33 with these parameters, by 1.4e-3
to 2.2e-3 (first layer), 5e-4 to 7e-4 (second), 3e-4 to 6e-4 (third) and 3e-5 to 5e-5 (last) in
relative L2.  Bound used for every layer: 1e-2.
"""
import sys

import numpy as np
import pytest

from oracle import learned_ref as L
from oracle.asdsm_oracle import Oracle, mesh_coeffs, permutation
from paper_2303_01163_amd.workloads import make_problem

pytestmark = pytest.mark.gpu

TOL_FWD = 1e-3
TOL_GRAD = 1e-2


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    from paper_2303_01163_amd import asdsm
    if not asdsm.LIB_PATH.exists():
        from paper_2303_01163_amd.build import build_library
        build_library()
    asdsm.load_library()
    return torch, torch.device("cuda", 0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _params(net, seed, scale=0.15):
    """Random parameters (padded channels zero) loaded into the network; returns them."""
    rng = np.random.default_rng(seed)
    lay, total = L.param_layout()
    assert total == net.n_params
    p = rng.normal(0.0, scale, total)
    for l, (w, b) in enumerate(L.unflatten(p)):
        cin_real = L.IN_CHANNELS if l == 0 else L.COUT[l - 1]
        w[L.COUT[l]:] = 0.0
        w[:, :, cin_real:] = 0.0
        b[L.COUT[l]:] = 0.0
    p = p.astype(np.float32)
    net.set_params(p)
    assert np.array_equal(net.get_params(), p)
    return p


def _input(n, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, n, n, 16), dtype=np.float32)
    x[..., :L.IN_CHANNELS] = rng.normal(size=(n, n, n, L.IN_CHANNELS))
    return x


def _dev32(torch_dev, a):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).ravel()).to(dev)


def _dev64(torch_dev, a):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


@pytest.mark.parametrize("n", [13, 67])
def test_forward_parity(torch_dev, n):
    """n = 13: one ragged x tile; n = 67: two x tiles, the second ragged."""
    from paper_2303_01163_amd.asdsm import Net
    _say("net forward", n)
    net = Net(n, seed=3)
    p = _params(net, 30)
    x = _input(n, 4)
    out = net.forward(_dev32(torch_dev, x)).cpu().numpy().reshape(n, n, n)
    ref, _ = L.forward(p, x, rounded=True)
    assert _rel(out, ref) <= TOL_FWD
    exact, _ = L.forward(p, x, rounded=False)
    assert _rel(out, exact) <= 0.05   # the BF16 operands themselves (sanity, not parity)


def _bound_plan(level, seed=0):
    from paper_2303_01163_amd.asdsm import Plan
    P = make_problem("sinbump3d", level, seed=seed)
    return P, Plan(3, P.alpha, P.beta, level, 0, seed=seed)


def _stencil_of(P, level):
    o = Oracle(3, P.alpha, P.beta, level)
    return L.operator_stencil(mesh_coeffs(o.grid, P.alpha, P.beta, ()), o.grid.h ** 2 / np.mean(P.alpha))


@pytest.mark.parametrize("kind,n,level", [("mse", 13, 5), ("mse", 33, 6), ("residual", 13, 5),
                                          ("residual", 33, 6)])
def test_gradient_parity(torch_dev, kind, n, level):
    from paper_2303_01163_amd.asdsm import Net
    _say("net gradient", kind, n)
    net = Net(n, seed=5)
    p = _params(net, 31)
    x = _input(n, 6)
    t = np.random.default_rng(7).normal(size=(n, n, n)).astype(np.float32)
    K = None
    if kind == "residual":
        P, plan = _bound_plan(level)
        net.bind(plan)
        K = _stencil_of(P, level)
    loss, grad = net.gradient(_dev32(torch_dev, x), _dev32(torch_dev, t), loss=kind)
    ref_loss, ref_grad = L.loss_and_grad(p, x, t, K, rounded=True)
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    lay, total = L.param_layout()
    for l, (wo, bo) in enumerate(lay):
        assert _rel(grad[wo:bo], ref_grad[wo:bo]) <= TOL_GRAD, ("weights", l)
        nb = L.COUT_P[l]
        assert _rel(grad[bo:bo + nb], ref_grad[bo:bo + nb]) <= TOL_GRAD, ("bias", l)
    # padded parameters get exactly zero gradient
    for l, (w, b) in enumerate(L.unflatten(grad.astype(np.float64))):
        cin_real = L.IN_CHANNELS if l == 0 else L.COUT[l - 1]
        assert not np.any(w[L.COUT[l]:]) and not np.any(w[:, :, cin_real:]) and not np.any(b[L.COUT[l]:])


def test_adam_step_matches_formula(torch_dev):
    from paper_2303_01163_amd.asdsm import Net
    n = 9
    net = Net(n, seed=8)
    p0 = _params(net, 32).astype(np.float64)
    x = _input(n, 9)
    t = np.random.default_rng(10).normal(size=(n, n, n)).astype(np.float32)
    _, g1 = net.gradient(_dev32(torch_dev, x), _dev32(torch_dev, t))
    net.adam(1e-3)
    p1 = net.get_params().astype(np.float64)
    g1 = g1.astype(np.float64)
    # first Adam step: m = (1 - b1) g, v = (1 - b2) g^2, bias-corrected -> p - lr g / (|g| + eps)
    ref = p0 - 1e-3 * g1 / (np.abs(g1) + 1e-8)
    assert np.max(np.abs(p1 - ref)) <= 1e-6


@pytest.mark.parametrize("n,offset", [(31, (0, 0, 0)), (20, (3, 5, 7))])
def test_features_parity(torch_dev, n, offset):
    from paper_2303_01163_amd.asdsm import Net
    P, plan = _bound_plan(5, seed=2)
    net = Net(n)
    net.bind(plan)
    r = np.random.default_rng(11).normal(size=plan.n_fine)
    rn2 = float(r @ r)
    x, rhat = net.features(_dev64(torch_dev, r), rn2, offset)
    g = Oracle(3, P.alpha, P.beta, 5).grid
    pe = P.beta * g.h / (2 * P.alpha)
    ref = L.features(r, rn2, g.Nf, g.n, pe, offset, n)
    xg = x.cpu().numpy().reshape(n, n, n, 16)
    assert _rel(xg, ref) <= 1e-6
    assert np.array_equal(rhat.cpu().numpy().reshape(n, n, n), xg[..., 0])


def _zero_net(n):
    from paper_2303_01163_amd.asdsm import Net
    net = Net(n)
    net.set_params(np.zeros(net.n_params, dtype=np.float32))
    return net


@pytest.mark.parametrize("eager", [False, True])
def test_zero_network_gives_the_plain_solve(torch_dev, eager):
    """A network that proposes nothing is never accepted: the learned solve is the plain one,
    bit for bit."""
    from paper_2303_01163_amd.asdsm import solve_learned
    P, plan = _bound_plan(5, seed=3)
    net = _zero_net(plan.n_f)
    net.bind(plan)
    s, g = _dev64(torch_dev, P.s_flat()), _dev64(torch_dev, P.g_flat())
    u0, i0 = plan.solve(s, g, max_iter=6, rtol=0, stag_window=0, eager=eager)
    u1, i1 = solve_learned(plan, net, s, g, max_iter=6, rtol=0, stag_window=0, eager=eager)
    assert i1["accepted"] == 0
    assert i1["iterations"] == i0["iterations"] == 6
    assert np.array_equal(u0.cpu().numpy(), u1.cpu().numpy())
    assert i0["res_hist"] == i1["res_hist"]


def test_learned_solve_matches_cpu_emulation(torch_dev):
    """31^3, a briefly trained network and a low acceptance factor (so that proposals are taken):
    every iterate against an emulation that uses oracle/learned_ref.py for the proposals and the
    ASDSM oracle for Algorithm 1, the residuals and the plain steps."""
    from paper_2303_01163_amd.asdsm import Net, solve_learned
    level, seed, factor, K = 5, 4, 1.05, 5
    P, plan = _bound_plan(level, seed=seed)
    net = Net(plan.n_f, seed=12)
    net.bind(plan)
    s, g = _dev64(torch_dev, P.s_flat()), _dev64(torch_dev, P.g_flat())
    # a few training steps on this problem's own residuals
    u, _ = plan.solve(s, g, max_iter=0)
    for _ in range(30):
        r, rn = plan.residual(u, s, g)
        x, rhat = net.features(r, rn * rn)
        net.gradient(x, rhat, loss="residual", want_grad=False)
        net.adam(1e-3)
    params = net.get_params()
    ug, info = solve_learned(plan, net, s, g, factor=factor, max_iter=K, rtol=0, stag_window=0)
    # emulation
    o = Oracle(3, P.alpha, P.beta, level, seed=seed)
    gr = o.grid
    pe = P.beta * gr.h / (2 * P.alpha)
    h2a = gr.h ** 2 / np.mean(P.alpha)
    u, b = o.initial_guess(P.s, P.g)
    accepted = 0
    hist = [float(np.linalg.norm(o.residual(u, b)))]
    for k in range(K):
        r = o.residual(u, b)
        rf = r.reshape(-1, order="F")
        rn2 = float(rf @ rf)
        F = L.features(rf, rn2, gr.Nf, gr.n, pe, (0, 0, 0), gr.Nf)
        out, _ = L.forward(params, F, rounded=True)
        sig = np.sqrt(rn2 / gr.Nf ** 3)
        e = np.transpose(out, (2, 1, 0)) * sig * h2a          # [z,y,x] -> oracle [x,y,z]
        q = o.apply_A(e)
        rq, qq = float(np.sum(r * q)), float(np.sum(q * q))
        if qq > 0 and rq > 0 and (rn2 - rq * rq / qq) * factor ** 2 <= rn2:
            u = u + (rq / qq) * e
            accepted += 1
        else:
            e, _ = o.error_guess(r, permutation(o.seed, k, 3))
            q = o.apply_A(e)
            shat = max(0.0, float(np.sum(r * q)) / float(np.sum(q * q)))
            u = u + shat * e
        hist.append(float(np.linalg.norm(o.residual(u, b))))
    _say("learned emulation accepted", accepted, "gpu", info["accepted"])
    assert info["accepted"] == accepted
    assert accepted >= 1
    # the proposals agree to the forward tolerance, and so do the iterates and residuals
    assert _rel(ug.cpu().numpy(), u.reshape(-1, order="F")) <= TOL_FWD
    for k in range(K + 1):
        assert abs(info["res_hist"][k] - hist[k]) <= 2 * TOL_FWD * hist[k], k


def test_accepted_steps_meet_the_factor(torch_dev):
    """Whatever the network proposes, an accepted step lowers ||r|| by at least the factor and a
    refused one is the plain step (checked through the residual history)."""
    from paper_2303_01163_amd.asdsm import Net, solve_learned
    P, plan = _bound_plan(5, seed=6)
    net = Net(plan.n_f, seed=13)
    net.bind(plan)
    s, g = _dev64(torch_dev, P.s_flat()), _dev64(torch_dev, P.g_flat())
    u, _ = plan.solve(s, g, max_iter=0)
    for _ in range(30):
        r, rn = plan.residual(u, s, g)
        x, rhat = net.features(r, rn * rn)
        net.gradient(x, rhat, loss="residual", want_grad=False)
        net.adam(1e-3)
    factor = 1.5
    _, info = solve_learned(plan, net, s, g, factor=factor, max_iter=8, rtol=0, stag_window=0)
    h = info["res_hist"]
    big_drops = sum(1 for k in range(len(h) - 1) if h[k + 1] * factor <= h[k] * (1 + 1e-12))
    assert big_drops >= info["accepted"]


def test_initial_network_proposes_nothing(torch_dev):
    from paper_2303_01163_amd.asdsm import Net
    net = Net(9, seed=1)
    out = net.forward(_dev32(torch_dev, _input(9, 2))).cpu().numpy()
    assert not np.any(out)
    p = net.get_params()
    lay, _ = L.param_layout()
    assert np.any(p[lay[0][0]:lay[0][1]]) and not np.any(p[lay[-1][0]:])


def test_training_lowers_the_residual_loss(torch_dev):
    """The trainer on 31^3 windows of 31^3 problems: the residual loss (1 for c = 0) falls."""
    from paper_2303_01163_amd.asdsm import Net
    from paper_2303_01163_amd.learn import TrainConfig, train_correction
    net = Net(31, seed=14)
    cfg = TrainConfig(level=5, plans=2, sources=3, iters=10, windows=2, lr=1e-3, lr_final=1e-4,
                      seed=77, log_every=20)
    res = train_correction(net, cfg, log=_say)
    h = res["loss_hist"]
    assert res["pairs"] == cfg.pairs == 120
    # full-volume windows and c = 0 at the start: the first loss is mean(rhat^2) = 1
    assert abs(res["first_loss"] - 1.0) <= 1e-5
    assert h[-1] < 0.5 * h[0]


def test_trained_network_lowers_the_stagnation_level(torch_dev):
    """What the trained network gains over the method without it: a network trained on 1024
    residual windows (31^3) of plain ASDSM runs at 63^3, then plain and learned solves (acceptance
    factor 1.1) of held-out problems whose exact discrete solution is known.  After 50 steps the
    learned solve reaches a residual at least 2x below the plain method's (which stagnates) and a
    lower algebraic error.  (The proposals mostly remove the rough part of the residual, which
    carries little of the error, so the error falls by less than the residual.)"""
    import torch
    from paper_2303_01163_amd.asdsm import Net, Plan, solve_learned
    from paper_2303_01163_amd.learn import TrainConfig, discrete_manufactured, train_correction
    net = Net(31, seed=21)
    cfg = TrainConfig(level=6, plans=4, sources=4, iters=32, windows=2, seed=500, log_every=256)
    res = train_correction(net, cfg, log=_say)
    big = Net(63)
    big.set_params(net.get_params())
    for seed in (0, 9):
        P = make_problem("sinbump3d", 6, seed=seed)
        plan = Plan(3, P.alpha, P.beta, 6, 0, seed=seed)
        big.bind(plan)
        s, g, uex = discrete_manufactured(plan, P, torch_dev[1])
        u0, i0 = plan.solve(s, g, max_iter=50, rtol=1e-12, stag_window=0)
        u1, i1 = solve_learned(plan, big, s, g, factor=1.1, max_iter=50, rtol=1e-12, stag_window=0)
        e0 = float(torch.linalg.norm(u0 - uex) / torch.linalg.norm(uex))
        e1 = float(torch.linalg.norm(u1 - uex) / torch.linalg.norm(uex))
        r0, r1 = min(i0["res_hist"]) / i0["bnorm"], min(i1["res_hist"]) / i1["bnorm"]
        _say("seed", seed, "plain res %.3e err %.3e | learned res %.3e err %.3e accepted %d/%d" %
             (r0, e0, r1, e1, i1["accepted"], i1["iterations"]))
        assert i1["accepted"] >= 1
        assert r1 <= 0.5 * r0 and e1 < e0
        plan.close()


def test_net_argument_errors(torch_dev):
    from paper_2303_01163_amd.asdsm import AsdsmError, Net, solve_learned
    P, plan = _bound_plan(5, seed=0)
    net = Net(20)
    s, g = _dev64(torch_dev, P.s_flat()), _dev64(torch_dev, P.g_flat())
    with pytest.raises(AsdsmError):
        solve_learned(plan, net, s, g)                 # not bound
    net.bind(plan)
    with pytest.raises(AsdsmError):
        solve_learned(plan, net, s, g)                 # 20 != N_f = 31
    r = _dev64(torch_dev, np.zeros(plan.n_fine))
    with pytest.raises(AsdsmError):
        net.features(r, 1.0, (12, 0, 0))               # 12 + 20 > 31
    net31 = Net(31)
    net31.bind(plan)
    with pytest.raises(AsdsmError):
        solve_learned(plan, net31, s, g, factor=1.0)   # factor must exceed 1


def test_learned_solve_with_fp32_guesses_and_resume(torch_dev):
    """The learned step composes with FP32 error guesses and with resuming: accepted proposals still
    meet the factor and a resumed learned solve continues from the given iterate."""
    from paper_2303_01163_amd.asdsm import Net, solve_learned
    P, plan = _bound_plan(5, seed=7)
    net = Net(plan.n_f, seed=15)
    net.bind(plan)
    s, g = _dev64(torch_dev, P.s_flat()), _dev64(torch_dev, P.g_flat())
    u, _ = plan.solve(s, g, max_iter=0)
    for _ in range(20):
        r, rn = plan.residual(u, s, g)
        x, rhat = net.features(r, rn * rn)
        net.gradient(x, rhat, loss="residual", want_grad=False, want_loss=False)
        net.adam(1e-3)
    for prec in ("fp64", "fp32"):
        u1, info = solve_learned(plan, net, s, g, factor=1.2, max_iter=6, rtol=0, stag_window=0, precision=prec)
        h = info["res_hist"]
        assert sum(1 for k in range(len(h) - 1) if h[k + 1] * 1.2 <= h[k] * (1 + 1e-12)) >= info["accepted"]
        u2, info2 = solve_learned(plan, net, s, g, u=u1.clone(), factor=1.2, max_iter=2, rtol=0, stag_window=0,
                                  precision=prec, resume=True, k0=6)
        assert info2["iterations"] == 2
        assert abs(info2["res_hist"][0] - h[-1]) <= 1e-9 * h[-1]
