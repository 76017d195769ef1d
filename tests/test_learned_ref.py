"""Pins of the CPU reference of the correction network (oracle/learned_ref.py) against definitions
that do not come from the reference itself: a brute-force convolution loop, scipy's correlate,
hand-computed BF16 roundings, central finite differences of the float64 network and the ASDSM fine
operator of the main CPU oracle."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import learned_ref as L
from oracle.asdsm_oracle import Grid, apply_operator, mesh_coeffs


def _params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    lay, total = L.param_layout()
    p = rng.normal(0.0, scale, total)
    # padded channels stay zero, as in the network's own initialisation
    for l, (w, b) in enumerate(L.unflatten(p)):
        cin_real = L.IN_CHANNELS if l == 0 else L.COUT[l - 1]
        w[L.COUT[l]:] = 0.0
        w[:, :, cin_real:] = 0.0
        b[L.COUT[l]:] = 0.0
    return p


def _input(n, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, n, n, 16))
    x[..., :L.IN_CHANNELS] = rng.normal(size=(n, n, n, L.IN_CHANNELS))
    return x


def test_conv3d_matches_brute_force_loop():
    rng = np.random.default_rng(1)
    n, ci, co = 3, 2, 2
    x = rng.normal(size=(n, n, n, ci))
    w = rng.normal(size=(co, 27, ci))
    b = rng.normal(size=co)
    out = L.conv3d(x, w, b)
    for z in range(n):
        for y in range(n):
            for xx in range(n):
                for o in range(co):
                    s = b[o]
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, yy, x2 = z + dz, y + dy, xx + dx
                                if 0 <= zz < n and 0 <= yy < n and 0 <= x2 < n:
                                    tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                    s += sum(w[o, tap, c] * x[zz, yy, x2, c] for c in range(ci))
                    assert abs(out[z, y, xx, o] - s) <= 1e-12 * (1 + abs(s))


def test_conv3d_matches_scipy_correlate():
    rng = np.random.default_rng(2)
    n, ci, co = 6, 3, 2
    x = rng.normal(size=(n, n, n, ci))
    w = rng.normal(size=(co, 27, ci))
    out = L.conv3d(x, w)
    for o in range(co):
        ref = sum(ndimage.correlate(x[..., c], w[o, :, c].reshape(3, 3, 3), mode="constant", cval=0.0)
                  for c in range(ci))
        assert np.max(np.abs(out[..., o] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_bf16_rounding_values():
    one = 1.0
    assert L.round_bf16(one) == 1.0
    assert L.round_bf16(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7          # representable
    assert L.round_bf16(1.0 + 2.0 ** -8) == 1.0                      # tie -> even (1.0)
    assert L.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie -> even (1 + 2^-6)
    assert L.round_bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7  # above the tie
    assert L.round_bf16(3.0 + 3 * 2.0 ** -8) == 3.0 + 2.0 ** -6       # spacing 2^-6 on [2, 4)
    assert L.round_bf16(-(3.0 + 3 * 2.0 ** -8)) == -(3.0 + 2.0 ** -6)  # sign-symmetric
    assert L.round_bf16(0.0) == 0.0
    # relative error at most 2^-8 (half a unit in the 8th significant bit)
    v = np.random.default_rng(3).normal(size=1000)
    assert np.max(np.abs(L.round_bf16(v) - v) / np.abs(v)) <= 2.0 ** -8 + 1e-15


@pytest.mark.parametrize("kind", ["mse", "residual"])
def test_backward_matches_finite_differences(kind):
    n = 4
    p = _params(5)
    x = _input(n, 6)
    t = np.random.default_rng(7).normal(size=(n, n, n))
    K = None
    if kind == "residual":
        g = Grid(3, 3)
        K = L.operator_stencil(mesh_coeffs(g, np.array([0.3, 1.0, 0.5]), np.array([2.0, -1.0, 4.0]), ()),
                               g.h ** 2 / 0.6)
    loss, grad = L.loss_and_grad(p, x, t, K, rounded=False)
    rng = np.random.default_rng(8)
    lay, total = L.param_layout()
    # a few weights and biases of every layer, each away from ReLU kinks with high probability
    picks = []
    for l, (wo, bo) in enumerate(lay):
        w, b = L.unflatten(p)[l]
        for _ in range(6):
            co = rng.integers(L.COUT[l])
            ci = rng.integers(L.IN_CHANNELS if l == 0 else L.COUT[l - 1])
            picks.append(wo + (co * 27 + rng.integers(27)) * L.CIN_P[l] + ci)
        picks.append(bo + rng.integers(L.COUT[l]))
    eps = 1e-6
    for i in picks:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (L.loss_and_grad(pp, x, t, K, rounded=False)[0] - L.loss_and_grad(pm, x, t, K, rounded=False)[0]) / (2 * eps)
        assert abs(fd - grad[i]) <= 1e-6 * (abs(fd) + 1e-3), (i, fd, grad[i])


def test_padded_parameters_get_zero_gradient():
    n = 4
    p = _params(9)
    _, grad = L.loss_and_grad(p, _input(n, 10), np.ones((n, n, n)), rounded=True)
    for l, (w, b) in enumerate(L.unflatten(grad)):
        cin_real = L.IN_CHANNELS if l == 0 else L.COUT[l - 1]
        assert not np.any(w[L.COUT[l]:]) and not np.any(w[:, :, cin_real:]) and not np.any(b[L.COUT[l]:])


def test_residual_loss_uses_the_asdsm_operator():
    """mean (t - K o)^2 with K = operator_stencil equals the loss written with the main oracle's
    fine operator (apply_operator on arrays indexed [axis 0, axis 1, axis 2])."""
    n = 5
    g = Grid(3, 3)  # N_f = 7 >= n
    alpha, beta = np.array([0.2, 0.7, 1.0]), np.array([-3.0, 1.5, 4.5])
    coeffs = mesh_coeffs(g, alpha, beta, ())
    h2a = g.h ** 2 / alpha.mean()
    K = L.operator_stencil(coeffs, h2a)
    p = _params(11)
    x = _input(n, 12)
    t = np.random.default_rng(13).normal(size=(n, n, n))
    loss, _ = L.loss_and_grad(p, x, t, K, rounded=False)
    o, _ = L.forward(p, x, rounded=False)
    # [z, y, x] -> [x, y, z] for apply_operator (array axis j = equation axis j)
    Ao = np.transpose(apply_operator(np.transpose(o, (2, 1, 0)), coeffs), (2, 1, 0)) * h2a
    assert abs(loss - np.mean((t - Ao) ** 2)) <= 1e-12 * loss
    # the identity stencil is the mean squared error
    mse, _ = L.loss_and_grad(p, x, t, None, rounded=False)
    assert abs(mse - np.mean((t - o) ** 2)) <= 1e-12 * mse


def test_features_channels():
    g = Grid(3, 5)  # N_f = 31, coarse planes every 8 fine points
    rng = np.random.default_rng(14)
    r = rng.normal(size=g.Nf ** 3)
    rn2 = float(r @ r)
    F = L.features(r, rn2, g.Nf, g.n, (0.1, -0.2, 0.3), (3, 5, 7), 20)
    R = r.reshape(g.Nf, g.Nf, g.Nf)
    sig = np.sqrt(rn2 / g.Nf ** 3)
    assert np.allclose(F[..., 0], R[7:27, 5:25, 3:23] / sig)
    assert np.array_equal(F[0, 0, :, 1] > 0, g.is_coarse_1d[3:23])
    assert np.array_equal(F[0, :, 0, 2] > 0, g.is_coarse_1d[5:25])
    assert np.array_equal(F[:, 0, 0, 3] > 0, g.is_coarse_1d[7:27])
    assert np.all(F[..., 4] == 0.1) and np.all(F[..., 6] == 0.3) and not np.any(F[..., 7:])
