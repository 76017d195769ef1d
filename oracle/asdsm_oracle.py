"""Plain FP64 CPU oracle of the Anisotropic Submeshes Domain Splitting Method (ASDSM).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  The product path (the HIP library and its Python binding) never
imports, links or calls anything here, and this module imports nothing from the product path.

It is written to be checked against the paper by eye, not to be fast:

* Meshes follow eqs. (3)-(5) (Section 2.1), generalised to d axes as in Section 3.5: for a subset S
  of axes, mesh M_S has the coarse spacing H on the axes in S and the fine spacing h elsewhere.
  M_{{k}} are the anisotropic ("denser") meshes, M_S with |S| >= 2 are intersection meshes and
  M_{all axes} is the coarse mesh.  Holes are the fine points with no coordinate on a coarse line.
* Every linear system is the centred second-order finite-difference discretisation of eq. (1) on
  that mesh, assembled literally as the Kronecker sum of Section 2.3 (alpha_j L/h_j^2 plus
  beta_j D/(2 h_j) per axis, x_1 fastest).  Dirichlet data are moved to the right-hand side with
  each mesh's own spacing.
* Submesh, coarse and hole systems are solved by banded LU with partial pivoting (LAPACK
  dgbtrf/dgbtrs), factorised once per distinct box.
* InitialGuess (Algorithm 1), Skeleton (Algorithm 2), Filler (Algorithm 3) and the outer iteration
  (Algorithm 4) follow the paper's steps in order.  Where the paper is silent the readings used are
  stated next to the code (cross-point extrapolation, spline type, multi-axis spline, random choice,
  norm, line search, stopping rule).

Array convention: a vector on a mesh with per-axis extents (n_1..n_d) is a float64 array of shape
(n_1, ..., n_d) indexed [i_1, ..., i_d] (0-based); the paper's x_1-fastest vector is its
Fortran-order flattening.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
  op1d / assemble_operator / apply_operator -- Q2-polynomial exactness, 1D closed form,
      O(h^2) convergence, tensor-eigenvector right-hand sides, pointwise stencil loops.
  BandedBoxSolver -- tensor-eigenvector right-hand sides, 1D closed form, residual of dense solve.
  spline_matrix -- exact on cubics vanishing at 0 and 1; unit rows at knots.
  boolean_sum_extend -- exact on tensor products of such cubics; reproduces data on every line.
  cross-point extrapolation -- O(H^4) convergence to the fine discrete solution; exact on Q2.
  skeleton (Algorithm 2 steps 4-6) -- submesh values shifted by spline-reproducible functions are
      restored exactly; the skeleton of u^(0) is O(H^4)-close to u_ff on smooth non-Q2 solutions.
  chosen cross points (Algorithm 2 step 3) -- a hand-computed d = 3 case for two axis orders.
  error-phase normalisation (Algorithm 1 steps 2.1/2.2) -- unit 2-norm over the submesh, invariance
      under scaling of the residual.
  filler -- Proposition 3.2(1): Filler(skeleton of u_ff) = u_ff.
  asdsm iteration -- Proposition 3.2(2) (zero hole residual), Remark 3.4 (monotone residual),
      convergence towards a direct fine solve on tiny grids.
  permutation (splitmix64) -- published splitmix64 output for seed 0.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.interpolate import CubicSpline

__all__ = [
    "Grid", "op1d", "assemble_operator", "apply_operator", "BandedBoxSolver", "rhs_on_mesh",
    "spline_matrix", "boolean_sum_extend", "splitmix64_stream", "permutation",
    "Oracle", "AsdsmResult", "fine_direct_solve", "fine_reference_solve",
]

_MASK64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


# --------------------------------------------------------------------------------------------
# Geometry: eqs. (3)-(5), Proposition 2.1, Section 3.5
# --------------------------------------------------------------------------------------------
class Grid:
    """Fine level L and coarse level L_c, identical on every axis.

    N_f = 2^L - 1 and N_c = 2^Lc - 1 interior points, h = 2^-L, H = 2^-Lc, n = H/h, so that
    N_f + 1 = n (N_c + 1) -- the nesting condition eq. (3).  Coarse lines sit at the 1-based fine
    indices n, 2n, ..., N_c n.
    """

    def __init__(self, d: int, level: int, coarse_level: int | None = None):
        if coarse_level is None or coarse_level == 0:
            coarse_level = level // 2
        if not (1 <= coarse_level < level):
            raise ValueError("need 1 <= coarse_level < level (eq. (3))")
        self.d = d
        self.level = level
        self.coarse_level = coarse_level
        self.Nf = 2 ** level - 1
        self.Nc = 2 ** coarse_level - 1
        self.n = 2 ** (level - coarse_level)
        self.h = 1.0 / (self.Nf + 1)
        self.H = 1.0 / (self.Nc + 1)
        assert self.Nf + 1 == self.n * (self.Nc + 1)
        # 0-based fine indices of the coarse lines
        self.cidx = np.arange(1, self.Nc + 1) * self.n - 1
        self.is_coarse_1d = np.zeros(self.Nf, dtype=bool)
        self.is_coarse_1d[self.cidx] = True

    # mesh M_S: per-axis extents and spacings
    def mesh_dims(self, S) -> tuple:
        return tuple(self.Nc if j in S else self.Nf for j in range(self.d))

    def mesh_spacings(self, S) -> tuple:
        return tuple(self.H if j in S else self.h for j in range(self.d))

    def mesh_fine_index(self, S):
        """0-based fine indices of M_S's points along each axis (its injection into the fine mesh)."""
        return [self.cidx if j in S else np.arange(self.Nf) for j in range(self.d)]

    def coarse_count(self) -> np.ndarray:
        """|S(p)| for every fine point p: the number of coordinates lying on a coarse line."""
        cnt = np.zeros((self.Nf,) * self.d, dtype=np.int64)
        for j in range(self.d):
            shape = [1] * self.d
            shape[j] = self.Nf
            cnt = cnt + self.is_coarse_1d.reshape(shape).astype(np.int64)
        return cnt

    def coarse_mask(self, j) -> np.ndarray:
        shape = [1] * self.d
        shape[j] = self.Nf
        return np.broadcast_to(self.is_coarse_1d.reshape(shape), (self.Nf,) * self.d)

    def hole_mask(self) -> np.ndarray:
        return self.coarse_count() == 0

    def restrict(self, v_fine: np.ndarray, S) -> np.ndarray:
        """Projector of Definition 2.3: keep the fine components lying on M_S."""
        return v_fine[np.ix_(*self.mesh_fine_index(S))]

    def prolong(self, v_mesh: np.ndarray, S) -> np.ndarray:
        """Transpose of the projector: zero extension to the fine mesh."""
        out = np.zeros((self.Nf,) * self.d)
        out[np.ix_(*self.mesh_fine_index(S))] = v_mesh
        return out

    def hole_starts(self) -> np.ndarray:
        """0-based fine index of the first point of each hole along one axis (Section 2.1 holes)."""
        return np.arange(self.Nc + 1) * self.n

    @property
    def hole_len(self) -> int:
        return self.n - 1


# --------------------------------------------------------------------------------------------
# Discretisation: Section 2.3
# --------------------------------------------------------------------------------------------
def op1d(alpha: float, beta: float, h: float):
    """Row of alpha/h^2 L_N + beta/(2h) D_N: (sub, diag, super) coefficients.

    L_N = tridiag(-1, 2, -1), D_N = tridiag(-1, 0, 1) (Section 2.3).
    """
    sub = -alpha / h ** 2 - beta / (2.0 * h)
    dia = 2.0 * alpha / h ** 2
    sup = -alpha / h ** 2 + beta / (2.0 * h)
    return sub, dia, sup


def _tridiag_sparse(n, coeffs):
    a, b, c = coeffs
    return sp.diags([np.full(n - 1, a), np.full(n, b), np.full(n - 1, c)], [-1, 0, 1],
                    shape=(n, n), format="csr")


def assemble_operator(dims, coeffs) -> sp.csr_matrix:
    """Kronecker sum sum_j I (x) ... (x) T_j (x) ... (x) I with x_1 fastest (Section 2.3).

    dims: per-axis extents (n_1..n_d); coeffs: per-axis (sub, diag, super) triples.
    """
    d = len(dims)
    total = int(np.prod(dims))
    A = sp.csr_matrix((total, total))
    for j in range(d):
        fast = int(np.prod(dims[:j])) if j > 0 else 1
        slow = int(np.prod(dims[j + 1:])) if j < d - 1 else 1
        Tj = _tridiag_sparse(dims[j], coeffs[j])
        A = A + sp.kron(sp.identity(slow, format="csr"),
                        sp.kron(Tj, sp.identity(fast, format="csr"), format="csr"), format="csr")
    return A.tocsr()


def apply_operator(u: np.ndarray, coeffs) -> np.ndarray:
    """(A u) for an array u on a box, with zero values outside it (the (2d+1)-point stencil)."""
    out = np.zeros_like(u)
    for j, (a, b, c) in enumerate(coeffs):
        out += b * u
        lo = [slice(None)] * u.ndim
        hi = [slice(None)] * u.ndim
        lo[j] = slice(1, None)
        hi[j] = slice(0, -1)
        out[tuple(lo)] += a * u[tuple(hi)]     # neighbour i-1
        out[tuple(hi)] += c * u[tuple(lo)]     # neighbour i+1
    return out


def mesh_coeffs(grid: Grid, alpha, beta, S):
    return [op1d(alpha[j], beta[j], sp_) for j, sp_ in enumerate(grid.mesh_spacings(S))]


def _face_value(grid: Grid, g_faces: np.ndarray, j: int, side: int, pts):
    """Dirichlet value on face (axis j, side) at the given 0-based fine indices of the other axes.

    Face layout: N_f^(d-1) values over the remaining axes in increasing order, lowest fastest.
    """
    d = grid.d
    others = [i for i in range(d) if i != j]
    face = g_faces[2 * j + side].reshape((grid.Nf,) * (d - 1), order="F") if d > 1 else g_faces[2 * j + side]
    return face[tuple(pts[i] for i in others)]


def rhs_on_mesh(grid: Grid, S, s_fine: np.ndarray, g_faces: np.ndarray, alpha, beta) -> np.ndarray:
    """Right-hand side b on M_S: the source injected from the fine mesh plus, for every point whose
    stencil neighbour along axis j lies on the boundary, -(sub or super coefficient) * g there,
    using M_S's own spacing on that axis (Section 2.3; the Dirichlet placement is the standard one,
    the paper lists only s)."""
    idx = grid.mesh_fine_index(S)
    b = s_fine[np.ix_(*idx)].copy()
    dims = grid.mesh_dims(S)
    coeffs = mesh_coeffs(grid, alpha, beta, S)
    d = grid.d
    for j in range(d):
        a_j, _, c_j = coeffs[j]
        for side, coef, pos in ((0, a_j, 0), (1, c_j, dims[j] - 1)):
            # points of M_S adjacent to face (j, side)
            sl = [slice(None)] * d
            sl[j] = slice(pos, pos + 1)
            grids = np.meshgrid(*[idx[i] if i != j else np.array([idx[j][pos]]) for i in range(d)],
                                indexing="ij")
            gv = _face_value(grid, g_faces, j, side, grids)
            b[tuple(sl)] -= coef * gv
    return b


# --------------------------------------------------------------------------------------------
# Banded LU box solver
# --------------------------------------------------------------------------------------------
class BandedBoxSolver:
    """Direct solver for the Kronecker-sum operator on a box, by banded LU with partial pivoting.

    The axes are reordered so the longest axis is slowest (smallest bandwidth); the matrix is
    factorised once, and solve() accepts one right-hand side array or a batch along a trailing axis.
    """

    def __init__(self, dims, coeffs):
        self.dims = tuple(int(x) for x in dims)
        d = len(self.dims)
        self.perm = sorted(range(d), key=lambda j: (self.dims[j], j))  # fastest first
        pdims = tuple(self.dims[j] for j in self.perm)
        pcoeffs = [coeffs[j] for j in self.perm]
        A = assemble_operator(pdims, pcoeffs).tocoo()
        self.n = A.shape[0]
        bw = int(np.prod(pdims[:-1])) if d > 1 else 1
        self.kl = self.ku = bw
        ab = np.zeros((2 * self.kl + self.ku + 1, self.n))
        ab[self.kl + self.ku + A.row - A.col, A.col] = A.data
        self.lub, self.piv, info = sla.lapack.dgbtrf(ab, self.kl, self.ku)
        if info != 0:
            raise np.linalg.LinAlgError(f"dgbtrf info={info}")
        self.pdims = pdims

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        d = len(self.dims)
        batched = rhs.ndim == d + 1
        arr = rhs if batched else rhs[..., None]
        nb = arr.shape[-1]
        t = np.transpose(arr, self.perm + [d])
        flat = t.reshape(self.n, nb, order="F")
        x, info = sla.lapack.dgbtrs(self.lub, self.kl, self.ku, np.asfortranarray(flat), self.piv)
        if info != 0:
            raise np.linalg.LinAlgError(f"dgbtrs info={info}")
        t = x.reshape(self.pdims + (nb,), order="F")
        inv = np.argsort(self.perm + [d])
        out = np.transpose(t, inv)
        return out if batched else out[..., 0]


# --------------------------------------------------------------------------------------------
# Spline prolongation of the cross-point discrepancy (Algorithm 2, step 5)
# --------------------------------------------------------------------------------------------
def spline_matrix(grid: Grid) -> np.ndarray:
    """N_f x N_c matrix of the cubic not-a-knot spline through the knots 0, H, ..., N_c H, 1 with
    value 0 at 0 and 1 ("high order spline ... with zero BCs"), evaluated at the fine points i h.
    With only three knots (N_c = 1) it is the parabola through them."""
    knots = np.concatenate(([0.0], (np.arange(1, grid.Nc + 1)) * grid.H, [1.0]))
    xf = np.arange(1, grid.Nf + 1) * grid.h
    Sp = np.empty((grid.Nf, grid.Nc))
    for c in range(grid.Nc):
        y = np.zeros(grid.Nc + 2)
        y[c + 1] = 1.0
        if grid.Nc == 1:
            coef = np.polyfit(knots, y, 2)
            Sp[:, c] = np.polyval(coef, xf)
        else:
            Sp[:, c] = CubicSpline(knots, y, bc_type="not-a-knot")(xf)
    return Sp


def boolean_sum_extend(delta_lines: dict, axes: list, Sp: np.ndarray, grid: Grid,
                       out_shape: tuple) -> np.ndarray:
    """Extend a discrepancy known on the intersection lines of a submesh to the whole submesh.

    For fine axes F of the submesh, the transfinite (Boolean-sum) interpolant
        sum_{T subset F, T nonempty} (-1)^(|T|+1) (prod_{j in T} Sp_j) delta|_{axes T coarse}
    is used (for one fine axis it is the plain 1D spline of Algorithm 2, step 5).
    delta_lines[T] is delta restricted to the points whose axes in T are at coarse indices (shape:
    N_c on the axes in T, full extent elsewhere).
    """
    out = np.zeros(out_shape)
    for r in range(1, len(axes) + 1):
        for T in itertools.combinations(axes, r):
            term = delta_lines[T]
            for j in T:
                term = np.moveaxis(np.tensordot(Sp, term, axes=([1], [j])), 0, j)
            out += ((-1.0) ** (r + 1)) * term
    return out


# --------------------------------------------------------------------------------------------
# Counter-based random choice of the error cross-points (Algorithm 2 step 3, Section 3.2)
# --------------------------------------------------------------------------------------------
def _mix64(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def splitmix64_stream(state: int, count: int) -> list:
    """splitmix64 (Steele, Lea, Flood 2014): state += golden gamma, output = mix(state)."""
    out = []
    for _ in range(count):
        state = (state + _GOLDEN) & _MASK64
        out.append(_mix64(state))
    return out


def permutation(seed: int, k: int, d: int) -> list:
    """pi_k: Fisher-Yates shuffle of the axes (0-based) driven by a splitmix64 stream whose start
    state is seed XOR ((k+1) * golden gamma) mod 2^64.  For i = d-1 down to 1: j = draw mod (i+1),
    swap positions i and j."""
    state = (seed ^ (((k + 1) * _GOLDEN) & _MASK64)) & _MASK64
    draws = splitmix64_stream(state, d - 1)
    p = list(range(d))
    for t, i in enumerate(range(d - 1, 0, -1)):
        j = draws[t] % (i + 1)
        p[i], p[j] = p[j], p[i]
    return p


# --------------------------------------------------------------------------------------------
# ASDSM
# --------------------------------------------------------------------------------------------
STATUS_OK, STATUS_STAGNATED, STATUS_MAXITER = 0, 1, 2


@dataclass
class AsdsmResult:
    u: np.ndarray
    status: int
    iterations: int
    bnorm: float
    res_hist: list = field(default_factory=list)     # ||r_k||_2, k = 0..K
    step_hist: list = field(default_factory=list)    # s_hat_k
    perm_hist: list = field(default_factory=list)    # pi_k
    iterates: list = field(default_factory=list)     # u^(k) if requested


class Oracle:
    """One problem instance: grid, coefficients, factorised box solvers and the spline matrix."""

    def __init__(self, d: int, alpha, beta, level: int, coarse_level: int | None = None,
                 seed: int = 0):
        self.grid = Grid(d, level, coarse_level)
        self.d = d
        self.alpha = np.asarray(alpha, dtype=np.float64)
        self.beta = np.asarray(beta, dtype=np.float64)
        self.seed = int(seed) & _MASK64
        g = self.grid
        self.fine_coeffs = mesh_coeffs(g, self.alpha, self.beta, ())
        self.A_ff = assemble_operator((g.Nf,) * d, self.fine_coeffs)
        self.Sp = spline_matrix(g)
        self._solvers = {}

    # ---- box solvers, factorised lazily and cached per distinct mesh
    def _solver(self, S):
        key = tuple(sorted(S))
        if key not in self._solvers:
            g = self.grid
            if key == ("hole",):
                dims = (g.hole_len,) * self.d
                coeffs = self.fine_coeffs
            else:
                dims = g.mesh_dims(key)
                coeffs = mesh_coeffs(g, self.alpha, self.beta, key)
            self._solvers[key] = BandedBoxSolver(dims, coeffs)
        return self._solvers[key]

    def solve_mesh(self, S, rhs):
        return self._solver(S).solve(rhs)

    # ---- right-hand sides (a1)
    def rhs(self, S, s_fine, g_faces):
        return rhs_on_mesh(self.grid, tuple(S), s_fine, g_faces, self.alpha, self.beta)

    def fine_rhs(self, s_fine, g_faces):
        return self.rhs((), s_fine, g_faces)

    # ---- fine residual (Algorithm 4, step 3)
    def residual(self, u, b_ff):
        flat = u.reshape(-1, order="F")
        r = b_ff.reshape(-1, order="F") - self.A_ff @ flat
        return r.reshape(u.shape, order="F")

    def apply_A(self, v):
        return (self.A_ff @ v.reshape(-1, order="F")).reshape(v.shape, order="F")

    # ---- Skeleton builder (Algorithm 2)
    def skeleton(self, sols: dict, uhat: np.ndarray) -> np.ndarray:
        """Merge the submesh solutions sols[(k,)] into a fine vector that is zero on the holes.

        uhat: fine-shaped array holding the chosen/extrapolated cross-point values at every point
        with |S(p)| >= 2 (ignored elsewhere).
        Step 4: delta_k = uhat - u_k on the intersection points of M_k.
        Step 5: extend delta_k over M_k with the spline (Boolean sum over its fine axes) and add.
        Step 6: merge -- skeleton points lying on one submesh only take the corrected submesh
        value, intersection points take uhat, holes are zero.
        """
        g = self.grid
        d = self.d
        cnt = g.coarse_count()
        out = np.zeros((g.Nf,) * d)
        for k in range(d):
            Sk = (k,)
            uk = sols[Sk]
            fine_axes = [j for j in range(d) if j != k]
            uhat_k = g.restrict(uhat, Sk)             # uhat seen on M_k's points
            delta = uhat_k - uk                        # meaningful on intersection points only
            lines = {}
            for r in range(1, len(fine_axes) + 1):
                for T in itertools.combinations(fine_axes, r):
                    sel = [slice(None)] * d
                    for j in T:
                        sel[j] = g.cidx
                    # pick rows axis by axis (np.ix_-like selection)
                    arr = delta
                    for j in T:
                        arr = np.take(arr, g.cidx, axis=j)
                    lines[T] = arr
            corr = boolean_sum_extend(lines, fine_axes, self.Sp, g, uk.shape)
            ut = uk + corr                               # corrected submesh solution u~_k
            ut_f = g.prolong(ut, Sk)
            only_k = (cnt == 1) & g.coarse_mask(k)
            out[only_k] = ut_f[only_k]
        inter = cnt >= 2
        out[inter] = uhat[inter]
        return out

    # ---- Filler (Algorithm 3)
    def filler(self, skel: np.ndarray, b_ff: np.ndarray | None) -> np.ndarray:
        """c = -P_h A u~ ; v = (P_h A P_h^T)^-1 (P_h b + c) ; u~ += P_h^T v.
        P_h A P_h^T is block diagonal with one identical block per hole (Remark 2.5), so every hole
        is solved with the same factorised hole matrix."""
        g = self.grid
        d = self.d
        c = -self.apply_A(skel)
        rhs_fine = c if b_ff is None else b_ff + c
        L = g.hole_len
        starts = g.hole_starts()
        boxes = []
        corners = list(itertools.product(starts, repeat=d))
        for st in corners:
            sl = tuple(slice(s0, s0 + L) for s0 in st)
            boxes.append(rhs_fine[sl])
        batch = np.stack(boxes, axis=-1)
        sol = self.solve_mesh(("hole",), batch)
        out = skel.copy()
        for t, st in enumerate(corners):
            sl = tuple(slice(s0, s0 + L) for s0 in st)
            out[sl] = out[sl] + sol[..., t]
        return out

    # ---- cross-point values
    def extrapolated_crosspoints(self, sols: dict) -> np.ndarray:
        """Initial-guess cross points (Algorithm 2, step 2, "RE"): at a point p lying on the submeshes
        k in S(p), |S(p)| >= 2, uhat = (sum_{k in S(p)} u_k(p) - u_{S(p)}(p)) / (|S(p)| - 1), which for
        d = 2 is P u_fc + P u_cf - u_cc.  It targets the fine discrete solution (error model
        a_1 H^2 + ... on each submesh) and uses the solution on the intersection mesh M_{S(p)}."""
        g = self.grid
        d = self.d
        uhat = np.zeros((g.Nf,) * d)
        for r in range(2, d + 1):
            for S in itertools.combinations(range(d), r):
                # points whose coarse-axis set is exactly S
                mask = np.ones((g.Nf,) * d, dtype=bool)
                for j in range(d):
                    mj = g.coarse_mask(j)
                    mask &= mj if j in S else ~mj
                acc = -g.prolong(sols[S], S)
                for k in S:
                    acc = acc + g.prolong(sols[(k,)], (k,))
                uhat[mask] = acc[mask] / (r - 1)
        return uhat

    def chosen_crosspoints(self, sols: dict, perm: list) -> np.ndarray:
        """Error-phase cross points (Algorithm 2, step 3): one random choice per iteration, given
        as a permutation of the axes; a point p takes the value of the first submesh of the
        permutation that contains it."""
        g = self.grid
        d = self.d
        uhat = np.zeros((g.Nf,) * d)
        cnt = g.coarse_count()
        done = np.zeros((g.Nf,) * d, dtype=bool)
        for k in perm:
            on_k = g.coarse_mask(k) & (cnt >= 2) & ~done
            vk = g.prolong(sols[(k,)], (k,))
            uhat[on_k] = vk[on_k]
            done |= on_k
        return uhat

    # ---- InitialGuess (Algorithm 1)
    def initial_guess(self, s_fine, g_faces):
        d = self.d
        b_ff = self.fine_rhs(s_fine, g_faces)
        sols = {}
        # steps 1.1/1.2 (anisotropic) and 1.3 (coarse and, for d >= 3, the other intersections)
        for r in range(1, d + 1):
            for S in itertools.combinations(range(d), r):
                sols[S] = self.solve_mesh(S, self.rhs(S, s_fine, g_faces))
        uhat = self.extrapolated_crosspoints(sols)
        skel = self.skeleton(sols, uhat)
        return self.filler(skel, b_ff), b_ff

    def error_guess(self, r_ff, perm):
        """InitialGuess(0 * b_ff, P r, ...): submesh solves of the projected residual (zero Dirichlet
        data), normalisation (steps 2.1/2.2), random cross-point choice, skeleton, homogeneous
        filler."""
        d = self.d
        g = self.grid
        sols = {}
        norms = []
        for k in range(d):
            ek = self.solve_mesh((k,), g.restrict(r_ff, (k,)))
            nk = float(np.sqrt(np.sum(ek * ek)))
            norms.append(nk)
            sols[(k,)] = ek / nk if nk > 0.0 else ek
        uhat = self.chosen_crosspoints(sols, perm)
        skel = self.skeleton(sols, uhat)
        return self.filler(skel, None), norms

    # ---- ASDSM (Algorithm 4)
    def solve(self, s_fine, g_faces, max_iter=50, rtol=1e-10, stag_window=3, stag_eta=1e-3,
              keep_iterates=False, u0=None, k0=0) -> AsdsmResult:
        """Outer iteration.  Continue while ||r_k||/||b|| > rtol, k < max_iter and not stagnated;
        stagnated means ||r_{k+1}|| > (1 - eta) ||r_k|| for stag_window consecutive iterations
        (stag_window = 0 disables the test).  A zero step s_hat = 0 leaves u unchanged and counts as
        one such iteration; it does not end the loop by itself, since the next iteration draws a
        new random choice of the cross points (Algorithm 2 step 3)."""
        if u0 is None:
            u, b_ff = self.initial_guess(s_fine, g_faces)
        else:
            u = np.array(u0, dtype=np.float64, copy=True)
            b_ff = self.fine_rhs(s_fine, g_faces)
        bnorm = float(np.linalg.norm(b_ff))
        r = self.residual(u, b_ff)
        rn = float(np.linalg.norm(r))
        res = AsdsmResult(u=u, status=STATUS_MAXITER, iterations=0, bnorm=bnorm, res_hist=[rn])
        if keep_iterates:
            res.iterates.append(u.copy())
        k = k0
        it = 0
        stag = 0
        status = STATUS_MAXITER
        while True:
            if bnorm > 0 and rn <= rtol * bnorm:
                status = STATUS_OK
                break
            if bnorm == 0.0 and rn == 0.0:
                status = STATUS_OK
                break
            if it >= max_iter:
                status = STATUS_MAXITER
                break
            perm = permutation(self.seed, k, self.d)
            e, _ = self.error_guess(r, perm)
            q = self.apply_A(e)
            qq = float(np.sum(q * q))
            rq = float(np.sum(r * q))
            shat = max(0.0, rq / qq) if qq > 0.0 else 0.0
            u = u + shat * e
            r = self.residual(u, b_ff)
            rn_new = float(np.linalg.norm(r))
            res.step_hist.append(shat)
            res.perm_hist.append(perm)
            res.res_hist.append(rn_new)
            if keep_iterates:
                res.iterates.append(u.copy())
            stag = stag + 1 if rn_new > (1.0 - stag_eta) * rn else 0
            rn = rn_new
            k += 1
            it += 1
            if stag_window > 0 and stag >= stag_window:
                status = STATUS_STAGNATED
                break
        res.u = u
        res.status = status
        res.iterations = it
        return res


def fine_direct_solve(d, alpha, beta, level, s_fine, g_faces) -> np.ndarray:
    """u_ff = A_ff^-1 b_ff by banded LU on the whole fine mesh (small grids only)."""
    g = Grid(d, level, 1)
    coeffs = mesh_coeffs(g, alpha, beta, ())
    b = rhs_on_mesh(g, (), s_fine, g_faces, alpha, beta)
    return BandedBoxSolver((g.Nf,) * d, coeffs).solve(b)


# --------------------------------------------------------------------------------------------
# Reference fine solution u_ff = A_ff^-1 b_ff at any size (used only to measure errors)
# --------------------------------------------------------------------------------------------
def _along(x: np.ndarray, M: np.ndarray, j: int) -> np.ndarray:
    """y = M applied along axis j of x: y[.., i, ..] = sum_m M[i, m] x[.., m, ..]."""
    return np.moveaxis(np.tensordot(M, x, axes=([1], [j])), 0, j)


class _TensorPreconditioner:
    """Approximate inverse of a Kronecker-sum operator (Section 2.3) on a box.

    Every axis except `line_axis` is diagonalised with the eigen-decomposition of its 1D operator
    (LAPACK, complex where the spectrum is complex); with line_axis = None every axis is, and each
    mode is divided by the sum of its eigenvalues.  Otherwise each mode of the diagonalised axes
    leaves a shifted tridiagonal system along line_axis, solved by banded LU with partial pivoting.
    In exact arithmetic both forms are the exact inverse; in floating point they lose accuracy with
    the condition numbers of the eigenvector matrices, which is why they only precondition the
    Krylov iteration of fine_reference_solve."""

    def __init__(self, dims, coeffs, line_axis=None):
        self.dims = tuple(dims)
        self.coeffs = coeffs
        self.line = line_axis
        self.eig = []
        for j, (n, (a, b, c)) in enumerate(zip(dims, coeffs)):
            if j == line_axis:
                self.eig.append(None)
                continue
            T = np.diag(np.full(n, b)) + np.diag(np.full(n - 1, a), -1) + np.diag(np.full(n - 1, c), 1)
            lam, V = np.linalg.eig(T)
            self.eig.append((lam, V, np.linalg.inv(V)))

    def __call__(self, f: np.ndarray) -> np.ndarray:
        d = len(self.dims)
        y = f.astype(np.complex128)
        shift = np.zeros((1,) * d, dtype=np.complex128)
        for j in range(d):
            if self.eig[j] is None:
                continue
            lam, _, Vinv = self.eig[j]
            y = _along(y, Vinv, j)
            shape = [1] * d
            shape[j] = self.dims[j]
            shift = shift + lam.reshape(shape)
        if self.line is None:
            y = y / shift
        else:
            L = self.line
            a, b, c = self.coeffs[L]
            n = self.dims[L]
            ym = np.moveaxis(y, L, 0)
            rest = ym.shape[1:]
            ym = ym.reshape(n, -1)
            # the shift of every mode, in the same order as the columns of ym
            sh = np.moveaxis(np.broadcast_to(shift, y.shape), L, 0)[0].reshape(-1)
            out = np.empty_like(ym)
            ab = np.zeros((3, n), dtype=np.complex128)
            ab[0, 1:] = c
            ab[2, :-1] = a
            for q in range(ym.shape[1]):
                ab[1, :] = b + sh[q]
                out[:, q] = sla.solve_banded((1, 1), ab, ym[:, q])
            y = np.moveaxis(out.reshape((n,) + rest), 0, L)
        for j in range(d):
            if self.eig[j] is None:
                continue
            y = _along(y, self.eig[j][1], j)
        return y.real


def fine_reference_solve(d, alpha, beta, level, s_fine, g_faces, precond="fdm", tol=1e-14,
                         max_outer=12):
    """Reference fine solution u_ff = A_ff^-1 b_ff (Section 2.3 system) for grids too large for
    banded LU, used only to measure the error of ASDSM iterates, never inside ASDSM.

    Preconditioned GMRES (scipy) inside FP64 iterative refinement: the outer loop forms the true
    residual r = b - A x with the assembled sparse A_ff, GMRES solves A dx = r to a modest relative
    accuracy with a tensor-product preconditioner, and x += dx; it stops once ||r||_2 <= tol ||b||_2
    or the residual stops falling (the rounding floor of forming b - A x).  precond = "fdm" (all axes
    diagonalised) or "line" (the axis with the worst-conditioned eigenvectors solved by banded LU)
    gives two different preconditioners whose results must agree.  Returns (u_ff, ||r||/||b||)."""
    from scipy.sparse.linalg import LinearOperator, gmres
    g = Grid(d, level, 1)
    dims = (g.Nf,) * d
    coeffs = mesh_coeffs(g, np.asarray(alpha, float), np.asarray(beta, float), ())
    b = rhs_on_mesh(g, (), s_fine, g_faces, alpha, beta)
    A = assemble_operator(dims, coeffs)
    if precond == "fdm":
        pre = _TensorPreconditioner(dims, coeffs)
    elif precond == "line":
        conds = []
        for (a_, b_, c_) in coeffs:
            ratio = abs(a_ / c_) if c_ != 0.0 else np.inf
            conds.append(abs(np.log(ratio)) if ratio > 0 else np.inf)
        pre = _TensorPreconditioner(dims, coeffs, line_axis=int(np.argmax(conds)))
    else:
        raise ValueError("precond must be 'fdm' or 'line'")
    n = A.shape[0]

    def mv(v):
        return pre(np.asarray(v).reshape(dims, order="F")).reshape(-1, order="F")

    M = LinearOperator((n, n), matvec=mv, dtype=np.float64)
    bf = b.reshape(-1, order="F")
    bn = float(np.linalg.norm(bf))
    x = np.zeros(n)
    if bn == 0.0:
        return x.reshape(dims, order="F"), 0.0
    r = bf.copy()
    rn = bn
    for _ in range(max_outer):
        dx, _info = gmres(A, r, rtol=1e-6, atol=0.0, restart=40, maxiter=20, M=M)
        x_new = x + dx
        r_new = bf - A @ x_new
        rn_new = float(np.linalg.norm(r_new))
        if rn_new >= rn:          # rounding floor reached: keep the better iterate
            break
        x, r, rn = x_new, r_new, rn_new
        if rn <= tol * bn:
            break
    if not rn <= 1e-11 * bn:
        raise RuntimeError(f"fine_reference_solve: preconditioner '{precond}' reached only "
                           f"||r||/||b|| = {rn / bn:.3e}")
    return x.reshape(dims, order="F"), rn / bn
