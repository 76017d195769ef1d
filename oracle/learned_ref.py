"""CPU reference of the learned-correction network: forward pass, losses and backward pass.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the product path never imports, links or calls it, and it imports
nothing from the product path.

The network is the one the learned correction of the refinement loop uses (the loop itself is
Algorithm 4; the correction is motivated by the stagnation diagnosis of Section 4, Example 2): four
3x3x3 convolutions with zero padding, channels 7 (stored as 16) -> 32 -> 32 -> 32 -> 1, ReLU after the
first three.  Everything is written from the definitions, in float64:

* conv3d:  out[z, y, x, co] = b[co] + sum_{tap, ci} w[co, tap, ci] in[z + dz, y + dy, x + dx, ci],
  tap = (dz + 1) 9 + (dy + 1) 3 + (dx + 1), zero outside the volume.
* The GPU computes the convolutions on BF16 operands (weights and activations rounded to nearest,
  ties to even, 8 significant bits) with FP32 accumulation and stores activations as FP32.  With
  ``rounded=True`` this reference rounds the same operands (activations first to FP32, as stored,
  then to BF16) and sums exactly in float64; ``rounded=False`` gives the exact float64 network (for
  the finite-difference check of the backward pass).
* Losses: mean (t - K o)^2 over the voxels with a 7-point stencil K (centre, x-, x+, y-, y+, z-, z+;
  zero outside the volume); K = identity is the mean squared error.
* Backward: dL/do = -(2/N) K^T rho; per layer dW = sum_v g (x) in (in = the layer input as the
  forward pass used it: BF16-rounded when ``rounded``; g as stored, FP32), db = sum_v g, and the
  data gradient, a convolution of g with the spatially flipped, channel-transposed weights,
  computed on BF16-rounded g and weights when ``rounded`` (as the GPU does), followed by the ReLU
  mask.

Parity status: conv3d is pinned by a brute-force loop and by scipy.ndimage.correlate; the rounding
by hand-computed BF16 values (ties to even); the backward pass by central finite differences of the
float64 network; the residual loss by the ASDSM operator of asdsm_oracle.apply_operator.
"""
from __future__ import annotations

import numpy as np

__all__ = ["LAYERS", "CIN_P", "COUT", "COUT_P", "param_layout", "unflatten", "round_bf16",
           "conv3d", "forward", "loss_and_grad", "features", "identity_stencil", "operator_stencil"]

LAYERS = 4
CIN_P = (16, 32, 32, 32)    # stored input channels per layer
COUT = (32, 32, 32, 1)      # real output channels
COUT_P = (32, 32, 32, 16)   # padded output channels of the stored weights
IN_CHANNELS = 7


def param_layout():
    """Offsets of (weights, biases) of each layer in the flat parameter vector: per layer the
    weights w[co][tap][ci] (co < COUT_P, ci < CIN_P) followed by COUT_P biases."""
    off = 0
    out = []
    for l in range(LAYERS):
        nw = COUT_P[l] * 27 * CIN_P[l]
        out.append((off, off + nw))
        off += nw + COUT_P[l]
    return out, off


def unflatten(params):
    """[(w (COUT_P, 27, CIN_P), b (COUT_P,)), ...] as float64 views of a flat parameter vector."""
    lay, total = param_layout()
    p = np.asarray(params, dtype=np.float64)
    assert p.size == total
    res = []
    for l, (wo, bo) in enumerate(lay):
        w = p[wo:bo].reshape(COUT_P[l], 27, CIN_P[l])
        b = p[bo:bo + COUT_P[l]]
        res.append((w, b))
    return res


def round_bf16(a):
    """Round to the nearest value with 8 significant bits, ties to even (BF16 has float32's
    exponent range; the values here are normal numbers).  Uses frexp/ldexp and numpy's
    round-half-to-even, not the bit pattern."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                 # a = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0) / 256.0, e)


def _q(a, rounded):
    """Operand of a convolution on the GPU: stored as FP32, fed to the MFMA as BF16."""
    if not rounded:
        return np.asarray(a, dtype=np.float64)
    return round_bf16(np.asarray(a, dtype=np.float32).astype(np.float64))


def _taps():
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yield (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1), dz, dy, dx


def conv3d(x, w, b=None):
    """x: (n, n, n, Cin) indexed [z, y, x, c]; w: (Cout, 27, Cin); b: (Cout,) or None."""
    n = x.shape[0]
    xp = np.zeros((n + 2, n + 2, n + 2, x.shape[3]), dtype=np.float64)
    xp[1:-1, 1:-1, 1:-1] = x
    out = np.zeros((n, n, n, w.shape[0]), dtype=np.float64)
    for tap, dz, dy, dx in _taps():
        sh = xp[1 + dz:1 + dz + n, 1 + dy:1 + dy + n, 1 + dx:1 + dx + n]
        out += np.tensordot(sh, w[:, tap, :], axes=([3], [1]))
    if b is not None:
        out += b
    return out


def forward(params, x16, rounded=True):
    """x16: (n, n, n, 16).  Returns (output (n, n, n), list of layer inputs as stored: FP32 values
    when rounded, float64 otherwise)."""
    layers = unflatten(params)
    acts = []
    a = np.asarray(x16, dtype=np.float64)
    if rounded:
        a = a.astype(np.float32).astype(np.float64)
    for l, (w, b) in enumerate(layers):
        acts.append(a)
        y = conv3d(_q(a, rounded), _q(w, rounded), b)
        if l == LAYERS - 1:
            y = y[..., :COUT[l]]
        else:
            y = np.maximum(y, 0.0)
        if rounded:
            y = y.astype(np.float32).astype(np.float64)
        a = y
    return a[..., 0], acts


def identity_stencil():
    return np.array([1.0, 0, 0, 0, 0, 0, 0])


def operator_stencil(coeffs, h2a):
    """Stencil of the fine ASDSM operator (per-axis (sub, diag, super) triples, axis 0 = x) scaled by
    h2a: centre sum_j diag_j, neighbours i - 1 / i + 1 of axis j the sub / super coefficient."""
    K = np.zeros(7)
    for j, (a, b, c) in enumerate(coeffs):
        K[0] += b * h2a
        K[1 + 2 * j] = a * h2a
        K[2 + 2 * j] = c * h2a
    return K


def _apply_stencil(f, K):
    """(K f) on an (n, n, n) array indexed [z, y, x], zero outside."""
    out = K[0] * f
    n = f.shape[0]
    # axis 0 = x = last array index, axis 1 = y, axis 2 = z
    for j, ax in enumerate((2, 1, 0)):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(1, n)
        hi[ax] = slice(0, n - 1)
        out[tuple(lo)] += K[1 + 2 * j] * f[tuple(hi)]   # neighbour i - 1
        out[tuple(hi)] += K[2 + 2 * j] * f[tuple(lo)]   # neighbour i + 1
    return out


def _transpose_stencil(K):
    KT = K.copy()
    for j in range(3):
        KT[1 + 2 * j], KT[2 + 2 * j] = K[2 + 2 * j], K[1 + 2 * j]
    return KT


def loss_and_grad(params, x16, target, K=None, rounded=True):
    """Loss mean (t - K o)^2 and its gradient with respect to the flat parameters (float64)."""
    K = identity_stencil() if K is None else np.asarray(K, dtype=np.float64)
    layers = unflatten(params)
    o, acts = forward(params, x16, rounded)
    t = np.asarray(target, dtype=np.float64)
    N = o.size
    rho = t - _apply_stencil(o, K)
    loss = float(np.mean(rho * rho))
    g = -(2.0 / N) * _apply_stencil(rho, _transpose_stencil(K))
    if rounded:
        g = g.astype(np.float32).astype(np.float64)
    lay, total = param_layout()
    grad = np.zeros(total)
    # upstream gradient with the padded output channels of the last layer
    gl = np.zeros(o.shape + (COUT_P[-1],))
    gl[..., 0] = g
    for l in range(LAYERS - 1, -1, -1):
        w, _ = layers[l]
        x = _q(acts[l], rounded)  # the operand the forward pass used
        n = x.shape[0]
        xp = np.zeros((n + 2, n + 2, n + 2, x.shape[3]))
        xp[1:-1, 1:-1, 1:-1] = x
        dw = np.zeros_like(w)
        for tap, dz, dy, dx in _taps():
            sh = xp[1 + dz:1 + dz + n, 1 + dy:1 + dy + n, 1 + dx:1 + dx + n]
            dw[:, tap, :] = np.tensordot(gl, sh, axes=([0, 1, 2], [0, 1, 2]))
        wo, bo = lay[l]
        grad[wo:bo] = dw.ravel()
        db = gl.sum(axis=(0, 1, 2))
        db[COUT[l]:] = 0.0
        grad[bo:bo + COUT_P[l]] = db
        if l == 0:
            break
        # data gradient: flipped taps, transposed channels
        wt = np.transpose(w[:, ::-1, :], (2, 1, 0))          # (ci, tap, co)
        dx_ = conv3d(_q(gl, rounded), _q(wt, rounded))
        if rounded:
            dx_ = dx_.astype(np.float32).astype(np.float64)
        mask = np.zeros(dx_.shape[-1], dtype=bool)
        mask[:COUT[l - 1]] = True
        gl = np.where((acts[l] > 0.0) & mask, dx_, 0.0)
    return loss, grad


def features(r, rnorm2, Nf, nsp, peclet, offset, n):
    """Network input for the window [offset_j, offset_j + n) of a fine residual r given as the flat
    x-fastest vector of N_f^3 values: channel 0 r / sigma (sigma^2 = rnorm2 / N_f^3), channels 1..3
    coarse-plane indicators of axes x, y, z (0-based fine index i on a coarse plane when
    (i + 1) % nsp == 0), channels 4..6 the cell Peclet numbers, 7..15 zero.  Returns (n, n, n, 16)
    indexed [z, y, x, c]."""
    R = np.asarray(r, dtype=np.float64).reshape(Nf, Nf, Nf)   # [z, y, x]
    ox, oy, oz = offset
    w = R[oz:oz + n, oy:oy + n, ox:ox + n]
    sig = np.sqrt(rnorm2 / float(Nf) ** 3)
    F = np.zeros((n, n, n, 16))
    F[..., 0] = w / sig if sig > 0 else 0.0
    on = lambda i: ((i + 1) % nsp == 0).astype(np.float64)
    idx = np.arange(n)
    F[..., 1] = on(idx + ox)[None, None, :]
    F[..., 2] = on(idx + oy)[None, :, None]
    F[..., 3] = on(idx + oz)[:, None, None]
    for j in range(3):
        F[..., 4 + j] = peclet[j]
    return F
