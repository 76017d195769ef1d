"""Seeded manufactured-solution problems for the steady advection-diffusion equation.

This module builds problem *data* only: the coefficients alpha_i, beta_i, the source s and the
Dirichlet data g of eq. (1) of the paper, derived analytically from a manufactured solution u.
It contains none of the solver's arithmetic (no finite differences, no submeshes, no merge) and
imports nothing from the solver or from the reference implementation used by the tests, so the
same arrays can be fed to both.

Layouts (shared by every consumer):

* ``s``: fine interior mesh, ``N_f = 2**level - 1`` points per axis, flattened with x_1 fastest
  (the ordering of Section 2.2).  Here it is returned as a float64 array of shape ``(N_f,)*d``
  indexed ``[i_1, ..., i_d]`` -- flatten with ``order='F'`` for the x_1-fastest vector.
* ``g``: ``2*d`` faces, ordered axis j = 1..d and, for each axis, side x_j = 0 then x_j = 1.
  Face (j, side) holds u on the N_f**(d-1) interior points of the other axes, in increasing axis
  order, lowest axis fastest.  Returned as an array of shape ``(2*d, N_f**(d-1))``.

Workload families (draw order from ``numpy.random.default_rng(seed)``: alpha, beta, frequencies,
bump centre):

* ``sinprod2d``: d=2, alpha=(1,1), beta ~ U[-1,1]^2, k_i in {1..4};
  u = prod_i sin(pi k_i x_i)  (so g = 0).
* ``sinbump3d``: d=3, alpha_i = 10**U[-1,0], beta_i ~ U[-5,5], k_i in {1..8};
  u = prod_i sin(pi k_i x_i) + exp(-|x-c|^2 / (2*0.1^2)), c ~ U[0.2,0.8]^3 (g != 0).
* ``sinbump_wide``: d = 3 or 4 (default 3), the advection-dominated batch draws: alpha_i =
  10**U[-2,0], beta_i ~ U[-10,10], k_i in {1..8}; u = prod_i sin(pi k_i x_i) + a Gaussian bump of
  width 0.1 at c ~ U[0.2,0.8]^d (g != 0).
* ``paper_smooth``: alpha_i = beta_i = 1, u = sin(pi*sum_i x_i) (Example 1 / Example 4, setting 1).
* ``quadratic``: a product of quadratics with seeded coefficients (exact for the centred scheme).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Problem", "make_problem", "fine_coords"]


@dataclass
class Problem:
    d: int
    level: int
    alpha: np.ndarray          # (d,)
    beta: np.ndarray           # (d,)
    s: np.ndarray              # (N_f,)*d, index [i_1..i_d]
    g: np.ndarray              # (2d, N_f**(d-1))
    u_exact: np.ndarray        # (N_f,)*d, manufactured solution at the fine interior points
    family: str = ""
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_f(self) -> int:
        return 2 ** self.level - 1

    def s_flat(self) -> np.ndarray:
        return np.ascontiguousarray(self.s.reshape(-1, order="F"))

    def g_flat(self) -> np.ndarray:
        return np.ascontiguousarray(self.g.reshape(-1))


def fine_coords(level: int) -> np.ndarray:
    n_f = 2 ** level - 1
    return np.arange(1, n_f + 1, dtype=np.float64) / (n_f + 1)


class _Manufactured:
    """u(x) together with its first and second partial derivatives along each axis."""

    def __init__(self, d: int):
        self.d = d

    def value(self, xs):  # xs: list of d broadcastable coordinate arrays
        raise NotImplementedError

    def d1(self, xs, j):
        raise NotImplementedError

    def d2(self, xs, j):
        raise NotImplementedError


class _SinProduct(_Manufactured):
    def __init__(self, d, k):
        super().__init__(d)
        self.k = np.asarray(k, dtype=np.float64)

    def _f(self, xs, j, der):
        w = math.pi * self.k[j]
        if der == 0:
            return np.sin(w * xs[j])
        if der == 1:
            return w * np.cos(w * xs[j])
        return -(w * w) * np.sin(w * xs[j])

    def _prod(self, xs, j, der):
        out = self._f(xs, j, der)
        for i in range(self.d):
            if i != j:
                out = out * self._f(xs, i, 0)
        return out

    def value(self, xs):
        return self._prod(xs, 0, 0)

    def d1(self, xs, j):
        return self._prod(xs, j, 1)

    def d2(self, xs, j):
        return self._prod(xs, j, 2)


class _Bump(_Manufactured):
    def __init__(self, d, centre, width):
        super().__init__(d)
        self.c = np.asarray(centre, dtype=np.float64)
        self.w2 = width * width

    def value(self, xs):
        r2 = 0.0
        for j in range(self.d):
            r2 = r2 + (xs[j] - self.c[j]) ** 2
        return np.exp(-r2 / (2.0 * self.w2))

    def d1(self, xs, j):
        return -(xs[j] - self.c[j]) / self.w2 * self.value(xs)

    def d2(self, xs, j):
        t = xs[j] - self.c[j]
        return (t * t / (self.w2 * self.w2) - 1.0 / self.w2) * self.value(xs)


class _SinOfSum(_Manufactured):
    def __init__(self, d, freq=1.0):
        super().__init__(d)
        self.w = math.pi * freq

    def value(self, xs):
        t = 0.0
        for j in range(self.d):
            t = t + xs[j]
        return np.sin(self.w * t)

    def d1(self, xs, j):
        t = 0.0
        for i in range(self.d):
            t = t + xs[i]
        return self.w * np.cos(self.w * t)

    def d2(self, xs, j):
        return -(self.w ** 2) * self.value(xs)


class _QuadProduct(_Manufactured):
    """prod_j (c0_j + c1_j x_j + c2_j x_j^2)."""

    def __init__(self, d, coef):
        super().__init__(d)
        self.coef = np.asarray(coef, dtype=np.float64)  # (d, 3)

    def _f(self, xs, j, der):
        c0, c1, c2 = self.coef[j]
        x = xs[j]
        if der == 0:
            return c0 + c1 * x + c2 * x * x
        if der == 1:
            return c1 + 2.0 * c2 * x
        return 2.0 * c2 + 0.0 * x

    def _prod(self, xs, j, der):
        out = self._f(xs, j, der)
        for i in range(self.d):
            if i != j:
                out = out * self._f(xs, i, 0)
        return out

    def value(self, xs):
        return self._prod(xs, 0, 0)

    def d1(self, xs, j):
        return self._prod(xs, j, 1)

    def d2(self, xs, j):
        return self._prod(xs, j, 2)


class _Sum(_Manufactured):
    def __init__(self, parts):
        super().__init__(parts[0].d)
        self.parts = parts

    def value(self, xs):
        return sum(p.value(xs) for p in self.parts)

    def d1(self, xs, j):
        return sum(p.d1(xs, j) for p in self.parts)

    def d2(self, xs, j):
        return sum(p.d2(xs, j) for p in self.parts)


def _grid(d, x1d):
    # one broadcastable coordinate array per axis (no full meshgrid copies)
    return [x1d.reshape([-1 if i == j else 1 for i in range(d)]) for j in range(d)]


def _source(man, alpha, beta, xs):
    # eq. (1): -sum_i alpha_i d2u/dx_i^2 + sum_i beta_i du/dx_i = s
    s = 0.0
    for j in range(man.d):
        s = s - alpha[j] * man.d2(xs, j) + beta[j] * man.d1(xs, j)
    return s


def _faces(man, d, x1d):
    n = x1d.size
    faces = np.empty((2 * d, n ** (d - 1)), dtype=np.float64)
    for j in range(d):
        others = [i for i in range(d) if i != j]
        for side in (0, 1):
            xs = [None] * d
            for pos, ax in enumerate(others):
                xs[ax] = x1d.reshape([-1 if q == pos else 1 for q in range(d - 1)])
            xs[j] = np.full((1,) * (d - 1), float(side))
            val = np.broadcast_to(man.value(xs), (n,) * (d - 1))
            # lowest remaining axis fastest -> Fortran flatten of an array indexed by those axes
            faces[2 * j + side] = np.asarray(val, dtype=np.float64).reshape(-1, order="F")
    return faces


def make_problem(family: str, level: int, seed: int = 0, d: int | None = None,
                 alpha=None, beta=None) -> Problem:
    """Seeded problem of the given family; ``alpha``/``beta`` override the drawn coefficients
    (the draws still happen, so the other seeded quantities do not change)."""
    alpha_override, beta_override = alpha, beta
    rng = np.random.default_rng(seed)
    meta = {}
    if family == "sinprod2d":
        d = 2
        alpha = np.ones(2)
        beta = rng.uniform(-1.0, 1.0, size=2)
        k = rng.integers(1, 5, size=2)
        man = _SinProduct(2, k)
        meta["k"] = k.tolist()
    elif family == "sinbump3d":
        d = 3
        alpha = 10.0 ** rng.uniform(-1.0, 0.0, size=3)
        beta = rng.uniform(-5.0, 5.0, size=3)
        k = rng.integers(1, 9, size=3)
        c = rng.uniform(0.2, 0.8, size=3)
        man = _Sum([_SinProduct(3, k), _Bump(3, c, 0.1)])
        meta["k"] = k.tolist()
        meta["centre"] = c.tolist()
    elif family == "sinbump_wide":
        d = d or 3
        alpha = 10.0 ** rng.uniform(-2.0, 0.0, size=d)
        beta = rng.uniform(-10.0, 10.0, size=d)
        k = rng.integers(1, 9, size=d)
        c = rng.uniform(0.2, 0.8, size=d)
        man = _Sum([_SinProduct(d, k), _Bump(d, c, 0.1)])
        meta["k"] = k.tolist()
        meta["centre"] = c.tolist()
    elif family == "paper_smooth":
        d = d or 2
        alpha = np.ones(d)
        beta = np.ones(d)
        man = _SinOfSum(d, 1.0)
    elif family == "quadratic":
        d = d or 2
        alpha = 10.0 ** rng.uniform(-1.0, 0.0, size=d)
        beta = rng.uniform(-2.0, 2.0, size=d)
        coef = rng.uniform(-1.0, 1.0, size=(d, 3))
        man = _QuadProduct(d, coef)
    elif family == "sinprod":
        d = d or 2
        alpha = 10.0 ** rng.uniform(-1.0, 0.0, size=d)
        beta = rng.uniform(-2.0, 2.0, size=d)
        k = rng.integers(1, 4, size=d)
        man = _SinProduct(d, k)
        meta["k"] = k.tolist()
    else:
        raise ValueError(f"unknown workload family {family!r}")
    if alpha_override is not None:
        alpha = np.asarray(alpha_override, dtype=np.float64)
    if beta_override is not None:
        beta = np.asarray(beta_override, dtype=np.float64)
    x1d = fine_coords(level)
    xs = _grid(d, x1d)
    shape = (x1d.size,) * d
    s = np.array(np.broadcast_to(_source(man, alpha, beta, xs), shape), dtype=np.float64)
    u = np.array(np.broadcast_to(man.value(xs), shape), dtype=np.float64)
    g = _faces(man, d, x1d)
    return Problem(d=d, level=level, alpha=np.asarray(alpha, np.float64),
                   beta=np.asarray(beta, np.float64), s=s, g=g, u_exact=u,
                   family=family, seed=seed, meta=meta)
