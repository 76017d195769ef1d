"""GPU parity: the HIP path (libasdsm.so through its C ABI) against the FP64 CPU oracle.

Tolerances: FP64 throughout; single operations (residual, submesh solves) agree to <= 1e-11
relative L2, iterates to <= 1e-10 relative L2 (the bar fixed for the FP64 GPU path).  The two
sides differ only in rounding order: banded LU vs fast diagonalisation, summation order of the
stencil, spline and reductions.
"""
import itertools
import sys

import numpy as np
import pytest

from oracle.asdsm_oracle import Oracle, apply_operator, fine_direct_solve, mesh_coeffs
from paper_2303_01163_amd.workloads import make_problem

pytestmark = pytest.mark.gpu

TOL_OP = 1e-11
TOL_ITER = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    from paper_2303_01163_amd import asdsm
    if not asdsm.LIB_PATH.exists():
        from paper_2303_01163_amd.build import build_library
        build_library()
    asdsm.load_library()
    return torch, torch.device("cuda", 0)


def _t(torch_dev, a):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _canon(d, S, arr):
    order = [j for j in range(d) if j not in S] + list(S)
    return np.transpose(arr, order).reshape(-1, order="F")


def _uncanon(grid, S, flat):
    d = grid.d
    order = [j for j in range(d) if j not in S] + list(S)
    shape = [grid.Nc if j in S else grid.Nf for j in order]
    return np.transpose(flat.reshape(shape, order="F"), np.argsort(order))


def _plan(P, L, Lc=0, seed=0):
    from paper_2303_01163_amd.asdsm import Plan
    return Plan(P.d, P.alpha, P.beta, L, Lc, seed=seed)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [  # (family, level, coarse_level, d, seed)
    ("sinprod2d", 6, 0, None, 0),      # 63^2, H = 1/8: the small 2D workload
    ("sinprod2d", 6, 2, None, 3),      # coarser submeshes, 15^2 holes
    ("sinprod", 5, 3, 2, 5),           # n = 4
    ("sinbump3d", 5, 0, None, 2),      # 31^3, H = 1/4, g != 0
    ("sinprod", 5, 3, 3, 1),           # 31^3, 7 coarse planes, 3^3 holes
    ("sinbump3d", 6, 3, None, 4),      # 63^3
    ("sinbump3d", 6, 4, None, 6),      # 63^3, 15 coarse planes per axis, 3^3 holes
    ("sinprod2d", 8, 4, None, 1),      # 255^2, 15 coarse lines per axis, 15^2 holes
    ("sinprod", 3, 1, 4, 14),          # d = 4: 7^4, one coarse plane per axis, 3^4 holes
    ("sinprod", 4, 2, 4, 6),           # 15^4, 3 coarse planes per axis, 3^4 holes
    ("sinprod", 4, 3, 4, 7),           # 15^4, 7 coarse planes per axis, single-point holes
    ("sinprod", 4, 1, 4, 8),           # 15^4, one coarse plane per axis, 7^4 holes
    ("sinprod", 5, 4, 3, 9),           # 31^3, 15 coarse planes per axis, single-point holes
]


@pytest.mark.parametrize("fam,L,Lc,d,seed", CASES)
def test_residual_parity(torch_dev, fam, L, Lc, d, seed):
    _say("residual", fam, L, Lc, seed)
    P = make_problem(fam, L, seed=seed, d=d)
    o = Oracle(P.d, P.alpha, P.beta, L, Lc or None)
    rng = np.random.default_rng(seed)
    u = P.u_exact + 0.1 * rng.standard_normal(P.u_exact.shape)
    b = o.fine_rhs(P.s, P.g)
    r_or = o.residual(u, b).reshape(-1, order="F")
    pl = _plan(P, L, Lc)
    r, nrm = pl.residual(_t(torch_dev, u.reshape(-1, order="F")), _t(torch_dev, P.s_flat()),
                         _t(torch_dev, P.g_flat()))
    assert _rel(r.cpu().numpy(), r_or) <= TOL_OP
    assert abs(nrm - np.linalg.norm(r_or)) <= 1e-12 * np.linalg.norm(r_or)


@pytest.mark.parametrize("fam,L,Lc,d,seed", CASES)
def test_mesh_solve_parity(torch_dev, fam, L, Lc, d, seed):
    """Every submesh / intersection / coarse system against the oracle's banded LU."""
    P = make_problem(fam, L, seed=seed, d=d)
    o = Oracle(P.d, P.alpha, P.beta, L, Lc or None)
    pl = _plan(P, L, Lc)
    rng = np.random.default_rng(100 + seed)
    for r_ in range(1, P.d + 1):
        for S in itertools.combinations(range(P.d), r_):
            _say("mesh", fam, L, Lc, seed, S)
            mask = sum(1 << j for j in S)
            rhs = rng.standard_normal(o.grid.mesh_dims(S))
            x_or = o.solve_mesh(S, rhs)
            x = pl.mesh_solve(mask, _t(torch_dev, _canon(P.d, S, rhs))).cpu().numpy()
            assert _rel(_uncanon(o.grid, S, x), x_or) <= TOL_OP, S


@pytest.mark.parametrize("fam,L,Lc,d,seed", CASES)
def test_iterate_parity(torch_dev, fam, L, Lc, d, seed):
    """u^(0) (Algorithm 1) and u^(1..5) (Algorithm 4) with the same seed, iterate by iterate."""
    _say("iterates", fam, L, Lc, seed)
    P = make_problem(fam, L, seed=seed, d=d)
    o = Oracle(P.d, P.alpha, P.beta, L, Lc or None, seed=seed + 17)
    ref = o.solve(P.s, P.g, max_iter=5, rtol=0, stag_window=0, keep_iterates=True)
    pl = _plan(P, L, Lc, seed=seed + 17)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    b = o.fine_rhs(P.s, P.g)
    # relative rounding of r_k (and of s_k): 100 eps * scale / ||r_k||, see _rounding_scale_of_residual
    rtol_r = [100 * 2.2e-16 * _rounding_scale_of_residual(o, ref.iterates[k], b) / ref.res_hist[k]
              for k in range(6)]
    for K in range(0, 6):
        u, info = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0)
        assert info["iterations"] == K
        assert _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F")) <= TOL_ITER, K
        for k in range(K + 1):
            assert abs(info["res_hist"][k] - ref.res_hist[k]) <= 1e-9 * ref.res_hist[k] + rtol_r[k] * ref.res_hist[k], k
        # the step also carries the rounding of the two inner products over ~N_f^d terms
        for k in range(K):
            assert abs(info["step_hist"][k] - ref.step_hist[k]) <= (1e-8 + rtol_r[k]) * abs(ref.step_hist[k]) + 1e-300, k


def _rounding_scale_of_residual(o, u, b):
    """|| |b| + |A| |u| ||_2: r = b - A u is computed to about eps times this (any summation order),
    so ||r|| and the step s = <r,q>/<q,q> that is built from r carry a relative rounding of about
    eps * scale / ||r||, which grows as the residual falls."""
    coeffs = [(abs(a), abs(b_), abs(c)) for a, b_, c in mesh_coeffs(o.grid, o.alpha, o.beta, ())]
    return np.linalg.norm(np.abs(b) + apply_operator(np.abs(u), coeffs))


def test_small_2d_workload_error_vs_fine_solution(torch_dev):
    """The 63^2 workload with 5 refinement iterations: GPU result equals the oracle's and its error
    against the direct fine solution is the oracle's (stagnation level of the method)."""
    P = make_problem("sinprod2d", 6, seed=0)
    o = Oracle(2, P.alpha, P.beta, 6, seed=0)
    ref = o.solve(P.s, P.g, max_iter=5, rtol=0, stag_window=0)
    pl = _plan(P, 6, 0, seed=0)
    u, info = pl.solve(_t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat()), max_iter=5, rtol=0,
                       stag_window=0)
    ug = u.cpu().numpy()
    assert _rel(ug, ref.u.reshape(-1, order="F")) <= TOL_ITER
    uff = fine_direct_solve(2, P.alpha, P.beta, 6, P.s, P.g).reshape(-1, order="F")
    assert abs(_rel(ug, uff) - _rel(ref.u.reshape(-1, order="F"), uff)) <= 1e-9


def test_full_size_3d_parity(torch_dev):
    """127^3 (h = 1/128), alpha log-uniform in [0.1,1], beta in [-5,5], sinusoids + bump: the GPU
    iterates u^(0..2) against the oracle at full size."""
    _say("full size 127^3")
    P = make_problem("sinbump3d", 7, seed=0)
    o = Oracle(3, P.alpha, P.beta, 7, seed=0)
    ref = o.solve(P.s, P.g, max_iter=2, rtol=0, stag_window=0, keep_iterates=True)
    pl = _plan(P, 7, 0, seed=0)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    for K in (0, 2):
        u, info = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0)
        assert _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F")) <= TOL_ITER, K


def test_full_size_3d_properties(torch_dev):
    """Properties that hold at any size, in the benchmark's configuration (127^3, default coarse
    level, stagnation rule on): residual zero on the holes for the returned iterate
    (Proposition 3.2(2)), non-increasing residual history (Remark 3.4), submesh solves satisfy their
    equations."""
    _say("full size properties 127^3")
    P = make_problem("sinbump3d", 7, seed=0)
    pl = _plan(P, 7, 0, seed=0)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u, info = pl.solve(s, g, max_iter=12, rtol=1e-10, stag_window=3)
    h = info["res_hist"]
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(len(h) - 1))
    o = Oracle(3, P.alpha, P.beta, 7)
    r, nrm = pl.residual(u, s, g)
    rr = r.cpu().numpy().reshape((127,) * 3, order="F")
    holes = o.grid.hole_mask()
    assert np.max(np.abs(rr[holes])) <= 1e-10 * info["bnorm"] / 127 ** 1.5 * 1e3
    assert abs(nrm - h[-1]) <= 1e-9 * h[-1]
    rng = np.random.default_rng(7)
    for S in ((0,), (1,), (2,), (0, 2), (0, 1, 2)):
        mask = sum(1 << j for j in S)
        rhs = rng.standard_normal(o.grid.mesh_dims(S))
        x = _uncanon(o.grid, S, pl.mesh_solve(mask, _t(torch_dev, _canon(3, S, rhs))).cpu().numpy())
        res = apply_operator(x, mesh_coeffs(o.grid, P.alpha, P.beta, S)) - rhs
        assert np.linalg.norm(res) <= 1e-11 * np.linalg.norm(rhs) * 1e2, S


def test_large_2d_parity(torch_dev):
    """The largest fine level (1023^2) with 31 coarse lines per axis: iterates u^(0), u^(2)."""
    _say("2D level 10")
    P = make_problem("sinprod2d", 10, seed=8)
    o = Oracle(2, P.alpha, P.beta, 10, 5, seed=8)
    ref = o.solve(P.s, P.g, max_iter=2, rtol=0, stag_window=0, keep_iterates=True)
    pl = _plan(P, 10, 5, seed=8)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    for K in (0, 2):
        u, _ = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0)
        assert _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F")) <= TOL_ITER, K


# ----------------------------------------------------------------------------- edge cases
@pytest.mark.parametrize("d,L,Lc", [(2, 3, 1), (2, 5, 4), (3, 3, 1), (3, 4, 3), (3, 3, 2)])
def test_degenerate_meshes(torch_dev, d, L, Lc):
    """N_c = 1 (the spline is a parabola), n = 2 (one-point holes), tiny grids."""
    _say("degenerate", d, L, Lc)
    fam = "sinprod2d" if d == 2 else "sinbump3d"
    P = make_problem(fam, L, seed=L + Lc)
    o = Oracle(d, P.alpha, P.beta, L, Lc, seed=5)
    ref = o.solve(P.s, P.g, max_iter=3, rtol=0, stag_window=0, keep_iterates=True)
    pl = _plan(P, L, Lc, seed=5)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    for K in (0, 3):
        u, _ = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0)
        assert _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F")) <= TOL_ITER, K


def test_q2_converges_at_initial_guess(torch_dev):
    """A Q2 solution is reproduced by Algorithm 1; the stopping rule ends with status OK and 0 steps."""
    P = make_problem("quadratic", 5, seed=2, d=3)
    pl = _plan(P, 5, 0)
    u, info = pl.solve(_t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat()), max_iter=10, rtol=1e-10)
    assert info["status"] == 0 and info["iterations"] == 0
    assert np.max(np.abs(u.cpu().numpy() - P.u_exact.reshape(-1, order="F"))) <= 1e-11


def test_resume_and_determinism(torch_dev):
    P = make_problem("sinbump3d", 5, seed=3)
    pl = _plan(P, 5, 0, seed=99)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u5, _ = pl.solve(s, g, max_iter=5, rtol=0, stag_window=0)
    u5b, _ = pl.solve(s, g, max_iter=5, rtol=0, stag_window=0)
    assert bool((u5 == u5b).all())                       # fixed-order reductions: bitwise equal
    u3, _ = pl.solve(s, g, max_iter=3, rtol=0, stag_window=0)
    u32, _ = pl.solve(s, g, u=u3.clone(), max_iter=2, rtol=0, stag_window=0, resume=True, k0=3)
    assert bool((u32 == u5).all())


def test_stagnation_and_maxiter_status(torch_dev):
    P = make_problem("sinprod2d", 6, seed=0)
    pl = _plan(P, 6, 0)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    _, info = pl.solve(s, g, max_iter=3, rtol=0, stag_window=0)
    assert info["status"] == 2 and info["iterations"] == 3
    _, info = pl.solve(s, g, max_iter=400, rtol=0, stag_window=1, stag_eta=0.5)
    assert info["status"] == 1 and info["iterations"] < 400


def test_error_codes(torch_dev):
    from paper_2303_01163_amd.asdsm import AsdsmError, Plan
    with pytest.raises(AsdsmError) as e:
        Plan(2, [1.0, -1.0], [0.0, 0.0], 5)
    assert e.value.code == -1
    with pytest.raises(AsdsmError) as e:
        Plan(2, [1.0, 1.0], [0.0, 0.0], 5, 5)
    assert e.value.code == -2
    with pytest.raises(AsdsmError) as e:              # cell Peclet 1.17 on every fine axis at 255^3,
        Plan(3, [0.5, 0.5, 0.5], [300.0, 300.0, 300.0], 8)   # 18.75 on the coarse ones
    assert e.value.code == -6
    with pytest.raises(AsdsmError) as e:             # d outside 2..4
        Plan(5, [1.0] * 5, [0.0] * 5, 3)
    assert e.value.code == -1
    P = make_problem("sinprod2d", 5, seed=0)
    pl = _plan(P, 5, 0)
    bad = P.s_flat().copy()
    bad[7] = np.nan
    with pytest.raises(AsdsmError) as e:
        pl.solve(_t(torch_dev, bad), _t(torch_dev, P.g_flat()), max_iter=2)
    assert e.value.code == -4


# ----------------------------------------------------------------------------- conditioning
def test_ill_conditioned_axis_refinement(torch_dev):
    """One fine axis with cell Peclet 0.35 (eigenvector matrix condition ~1e10 at N_f = 63): the
    plan adds FP64 refinement sweeps around the fast-diagonalisation solves, and submesh solves and
    iterates still match the banded-LU oracle."""
    _say("ill-conditioned axis")
    P = make_problem("sinbump3d", 6, seed=1, alpha=[0.1, 0.5, 0.8], beta=[4.5, 1.0, -1.0])
    o = Oracle(3, P.alpha, P.beta, 6, seed=4)
    pl = _plan(P, 6, 0, seed=4)
    rng = np.random.default_rng(3)
    for S in ((0,), (1,), (2,), (0, 1), (1, 2)):
        mask = sum(1 << j for j in S)
        rhs = rng.standard_normal(o.grid.mesh_dims(S))
        x = pl.mesh_solve(mask, _t(torch_dev, _canon(3, S, rhs))).cpu().numpy()
        assert _rel(_uncanon(o.grid, S, x), o.solve_mesh(S, rhs)) <= TOL_OP, S
    ref = o.solve(P.s, P.g, max_iter=3, rtol=0, stag_window=0, keep_iterates=True)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    for K in (0, 3):
        u, _ = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0)
        assert _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F")) <= TOL_ITER, K


def test_two_ill_conditioned_axes_use_a_line_axis(torch_dev):
    """Two fine axes with cell Peclet 0.47 at N_f = 63 (eigenvector matrices of condition 5.6e13
    each): the submesh with both as fine axes cannot be diagonalised on both, so each anisotropic
    mesh eliminates its worst fine axis by block cyclic reduction and transforms the other (with
    refinement sweeps); submesh solves and iterates match the banded-LU oracle."""
    _say("two ill-conditioned axes")
    P = make_problem("sinbump3d", 6, seed=1, alpha=[0.1, 0.1, 0.8], beta=[6.0, -6.0, 1.0])
    o = Oracle(3, P.alpha, P.beta, 6, seed=4)
    pl = _plan(P, 6, 0, seed=4)
    info = pl.line_axes()
    assert info[1 << 2][0] in (0, 1) and info[1 << 2][1] >= 1   # M_2: one of the two, with sweeps
    rng = np.random.default_rng(5)
    for S in ((0,), (1,), (2,), (0, 1), (1, 2), (0, 2)):
        mask = sum(1 << j for j in S)
        rhs = rng.standard_normal(o.grid.mesh_dims(S))
        x = pl.mesh_solve(mask, _t(torch_dev, _canon(3, S, rhs))).cpu().numpy()
        assert _rel(_uncanon(o.grid, S, x), o.solve_mesh(S, rhs)) <= TOL_OP, S
    ref = o.solve(P.s, P.g, max_iter=3, rtol=0, stag_window=0, keep_iterates=True)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u, _ = pl.solve(s, g, max_iter=3, rtol=0, stag_window=0)
    assert _rel(u.cpu().numpy(), ref.iterates[3].reshape(-1, order="F")) <= TOL_ITER


def _two_axes_parity(torch_dev, P, L, Lc, seed):
    o = Oracle(3, P.alpha, P.beta, L, Lc, seed=seed)
    pl = _plan(P, L, Lc, seed=seed)
    rng = np.random.default_rng(5)
    for S in ((0,), (1,), (2,), (0, 1), (1, 2), (0, 2), (0, 1, 2)):
        _say("two complex axes: mesh", L, S)
        mask = sum(1 << j for j in S)
        rhs = rng.standard_normal(o.grid.mesh_dims(S))
        x = pl.mesh_solve(mask, _t(torch_dev, _canon(3, S, rhs))).cpu().numpy()
        assert _rel(_uncanon(o.grid, S, x), o.solve_mesh(S, rhs)) <= TOL_OP, S
    ref = o.solve(P.s, P.g, max_iter=3, rtol=0, stag_window=0, keep_iterates=True)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    for skeleton in (False, True):
        _say("two complex axes: iterates", L, "skeleton" if skeleton else "fine")
        for K in (0, 1, 3):
            u, info = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0, skeleton=skeleton)
            assert info["iterations"] == K
            assert _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F")) <= TOL_ITER, (skeleton, K)
    return pl


def test_two_complex_axes_take_both_on_the_line_solve(torch_dev):
    """63^3 with two fine axes of cell Peclet 1.02 (complex 1D spectra): the anisotropic mesh with
    both as fine axes solves along one with the other and the coarse axis as its 441-point block
    (block cyclic reduction as GEMMs per level), and the holes (7^3, two such axes) apply their
    operator's inverse; every submesh solve and the iterates, fine-mesh and skeleton-sparse, match
    the banded-LU oracle."""
    P = make_problem("sinbump3d", 6, seed=1, alpha=[0.1, 0.1, 0.8], beta=[13.0, -13.0, 1.0])
    pl = _two_axes_parity(torch_dev, P, 6, 3, 4)
    assert pl.line_axes()[1 << 2][0] == 0   # M_2: the line along axis 0, axis 1 in the block


def test_three_complex_axes_at_31(torch_dev):
    """31^3 with every axis advection-dominated (cell Peclet 4.7 to 7.8 at h = 1/32, the range of
    the advection-dominated family): every anisotropic mesh takes both fine axes on its line solve
    (93-point blocks), the intersection meshes their one fine axis, and the holes (7^3, three such
    axes) the dense inverse; submesh solves and iterates match the oracle."""
    P = make_problem("sinbump3d", 5, seed=2, alpha=[0.02, 0.02, 0.02], beta=[10.0, -9.0, 6.0])
    pl = _two_axes_parity(torch_dev, P, 5, 2, 6)
    axes = pl.line_axes()
    for k in range(3):
        assert axes[1 << k][0] == (1 if k == 0 else 0)   # position 0 of M_k: its first fine axis


def test_two_ill_conditioned_axes_at_127_diagonalise_the_coarse_axis(torch_dev):
    """127^3 with two fine axes at cell Peclet 0.27 (eigenvector matrices of condition ~1e15, past
    what refinement sweeps recover; the 15^3 holes still take them): the mesh with both as fine axes
    would need a 127 * 7-point block, so it diagonalises its coarse axis instead and solves, per
    coarse mode, along one fine axis with the other (127 points) as the block; every submesh solve
    and the iterates, fine-mesh and skeleton-sparse, match the banded-LU oracle."""
    P = make_problem("sinbump3d", 7, seed=3, alpha=[0.1, 0.1, 1.0], beta=[7.0, -7.0, 1.0])
    pl = _two_axes_parity(torch_dev, P, 7, 3, 8)
    assert pl.line_axes()[1 << 2] == (0, 0)   # M_2: the line along axis 0, no sweeps


def test_two_complex_axes_at_127_holes_take_the_line_solve(torch_dev):
    """127^3 with two fine axes of cell Peclet 1.02 (complex 1D spectra): the 15^3 holes eliminate
    along one hole axis with the other two (225 points) as the block, one table for every hole, as
    batched GEMMs over the holes; the mesh with both as fine axes diagonalises its coarse axis.
    Every submesh solve and the iterates, fine-mesh and skeleton-sparse (whose layer-mode fill runs
    the same hole solve), match the banded-LU oracle."""
    P = make_problem("sinbump3d", 7, seed=4, alpha=[0.1, 0.1, 0.8], beta=[26.0, -26.0, 1.0])
    pl = _two_axes_parity(torch_dev, P, 7, 3, 9)
    assert pl.line_axes()[1 << 2] == (0, 0)   # M_2: the line along axis 0, coarse axis diagonalised


def test_three_complex_axes_at_127(torch_dev):
    """127^3 with every axis advection-dominated (cell Peclet 1.02 at h = 1/128, 16 at the coarse
    spacing): no coarse axis can be diagonalised, so each anisotropic mesh takes its two fine axes
    and its coarse axis on one line solve (889-point blocks), and the holes (15^3, three such axes)
    the hole line solve; every submesh solve and the iterates, fine-mesh and skeleton-sparse, match
    the banded-LU oracle."""
    P = make_problem("sinbump3d", 7, seed=5, alpha=[0.1, 0.1, 0.1], beta=[26.0, -26.0, 26.0])
    pl = _two_axes_parity(torch_dev, P, 7, 3, 10)
    axes = pl.line_axes()
    for k in range(3):
        assert axes[1 << k] == (1 if k == 0 else 0, 0)   # position 0 of M_k: its first fine axis


def test_two_complex_axes_beyond_the_limits_are_refused(torch_dev):
    """Beyond what is built: every axis with |cell Peclet| > 1 at 255^3 (fine and coarse spacing:
    a 255 * 15-point block whose coarse axis cannot be diagonalised either) reports
    ASDSM_E_UNSUPPORTED instead of returning inaccurate solves; so does d = 4 with two such axes."""
    from paper_2303_01163_amd.asdsm import AsdsmError, Plan
    with pytest.raises(AsdsmError) as e:
        Plan(3, [0.05, 0.05, 0.05], [26.0, -26.0, 26.0], 8)
    assert e.value.code == -6
    with pytest.raises(AsdsmError) as e:
        Plan(4, [0.05, 0.05, 0.8, 0.8], [8.0, -8.0, 1.0, 1.0], 5, 2)
    assert e.value.code == -6


def test_graph_replay_matches_eager(torch_dev):
    """The refinement loop replays a captured HIP graph of two gated steps; every replayed solve must
    equal the eager (kernel-by-kernel) solve bitwise, with eager work and synchronisations between the
    replays, for odd and even step counts and when the stopping rule fires inside a graph."""
    torch, dev = torch_dev
    P = make_problem("sinbump3d", 5, seed=6)
    pl = _plan(P, 5, 0, seed=6)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    for K in (1, 4, 7):
        ue, ie = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0, eager=True)
        u = torch.empty_like(ue)
        for rep in range(3):
            ug, ig = pl.solve(s, g, u=u, max_iter=K, rtol=0, stag_window=0)
            assert ig["iterations"] == ie["iterations"] == K
            assert bool((ug == ue).all()), (K, rep)
            assert ig["res_hist"] == ie["res_hist"]
            torch.cuda.synchronize()
            _, _ = pl.residual(ug, s, g)                  # eager work between replays
    ue, ie = pl.solve(s, g, max_iter=40, rtol=0, stag_window=1, stag_eta=0.3, eager=True)
    ug, ig = pl.solve(s, g, max_iter=40, rtol=0, stag_window=1, stag_eta=0.3)
    assert ie["status"] == ig["status"] == 1 and ie["iterations"] == ig["iterations"] < 40
    assert bool((ug == ue).all())


# ---- mixed-precision error guesses (FP32 submesh solves in the refinement steps)
MIXED_CASES = [  # (family, level, coarse_level, d, seed): every anisotropic mesh FP32-eligible
    ("sinprod2d", 6, 0, None, 0),
    ("sinbump3d", 6, 3, None, 4),
    ("sinbump3d", 7, 0, None, 1),
    ("sinprod", 4, 1, 4, 8),           # d = 4: 15^4, holes of 7^4
    ("sinprod", 4, 2, 4, 6),           # d = 4: 15^4, 3 coarse planes per axis
]


@pytest.mark.parametrize("fam,L,Lc,d,seed", MIXED_CASES)
def test_mixed_precision_iterates(torch_dev, fam, L, Lc, d, seed):
    """FP32 error guesses against the FP64 oracle.  The plan admits FP32 only where the FP32
    solves are accurate to delta <= 1e-3 (6e-8 * prod cond(V_j)), so each update s_k e_k carries an
    error of at most ~delta of itself: u_K differs from the oracle's by at most
    delta * sum_k ||u_{k+1} - u_k||.  The initial guess is FP64 in both modes."""
    _say("mixed", fam, L, Lc, seed)
    P = make_problem(fam, L, seed=seed, d=d)
    o = Oracle(P.d, P.alpha, P.beta, L, Lc or None, seed=seed + 17)
    K = 5
    ref = o.solve(P.s, P.g, max_iter=K, rtol=0, stag_window=0, keep_iterates=True)
    pl = _plan(P, L, Lc, seed=seed + 17)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u0, info0 = pl.solve(s, g, max_iter=0, rtol=0, stag_window=0, precision="fp32")
    assert _rel(u0.cpu().numpy(), ref.iterates[0].reshape(-1, order="F")) <= TOL_ITER
    u, info = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0, precision="fp32")
    assert info["precision"] == "fp32" and info["iterations"] == K
    uK = ref.iterates[K].reshape(-1, order="F")
    path = sum(np.linalg.norm(ref.iterates[k + 1] - ref.iterates[k]) for k in range(K))
    err = np.linalg.norm(u.cpu().numpy() - uK)
    _say("   mixed-precision |u_K - u_K(FP64 oracle)| / |u_K| = %.3e (path %.3e)" %
         (err / np.linalg.norm(uK), path / np.linalg.norm(uK)))
    assert err <= 2e-3 * path + 1e-12 * np.linalg.norm(uK)
    # the residual history follows the FP64 one to the same relative accuracy
    for k in range(K + 1):
        assert abs(info["res_hist"][k] - ref.res_hist[k]) <= 2e-3 * ref.res_hist[k] + 1e-12 * ref.bnorm, k


def test_mixed_precision_falls_back_on_ill_conditioned_meshes(torch_dev):
    """Where FP32 transforms would not be accurate (6e-8 * prod cond(V_j) > 1e-3 on some mesh) the
    plan keeps FP64 and says so; the result is the FP64 one."""
    from paper_2303_01163_amd.asdsm import Plan
    P = make_problem("sinbump3d", 6, seed=0, alpha=[0.1, 0.5, 0.8], beta=[4.5, 1.0, -1.0])
    pl = Plan(3, P.alpha, P.beta, 6, 3, seed=5)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u64, i64 = pl.solve(s, g, max_iter=3, rtol=0, stag_window=0)
    u32, i32 = pl.solve(s, g, max_iter=3, rtol=0, stag_window=0, precision="fp32")
    assert i32["precision"] == "fp64" and i64["precision"] == "fp64"
    assert np.array_equal(u64.cpu().numpy(), u32.cpu().numpy())


def test_mixed_precision_full_solve(torch_dev):
    """A complete solve with FP32 error guesses on a 127^3 FP32-eligible draw reaches the same
    stopping status and residual level as the FP64 solve (within 1%)."""
    from paper_2303_01163_amd.asdsm import Plan
    P = make_problem("sinbump3d", 7, seed=1)
    pl = Plan(3, P.alpha, P.beta, 7, 0, seed=1)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u64, i64 = pl.solve(s, g, max_iter=50)
    u32, i32 = pl.solve(s, g, max_iter=50, precision="fp32")
    assert i32["precision"] == "fp32"
    _say("   fp64: %s after %d, rel res %.4e; fp32: %s after %d, rel res %.4e; |u32-u64|/|u64| %.3e" % (
        i64["status_name"], i64["iterations"], i64["rnorm"] / i64["bnorm"], i32["status_name"],
        i32["iterations"], i32["rnorm"] / i32["bnorm"], _rel(u32.cpu().numpy(), u64.cpu().numpy())))
    assert i32["status"] == i64["status"]
    assert abs(i32["rnorm"] - i64["rnorm"]) <= 1e-2 * i64["rnorm"]


# ---- batches: independent problems advanced together by one graph
BATCH_MEMBERS = [  # (family, level, coarse_level, d, seed, alpha, beta)
    ("sinprod2d", 6, 0, None, 0, None, None),
    ("sinbump3d", 5, 0, None, 2, None, None),
    ("sinbump3d", 6, 3, None, 4, None, None),
    ("sinprod", 5, 3, 3, 1, None, None),
    ("sinbump3d", 6, 3, None, 0, [0.1, 0.5, 0.8], [4.5, 1.0, -1.0]),  # needs refinement sweeps
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_individual_solves(torch_dev, precision):
    """Every member of a batch ends bitwise where asdsm_solve on its own plan ends (same kernels,
    fixed-order reductions), including members that stop earlier than others."""
    from paper_2303_01163_amd.asdsm import Batch, Plan
    plans, ss, gs = [], [], []
    for fam, L, Lc, d, seed, al, be in BATCH_MEMBERS:
        P = make_problem(fam, L, seed=seed, d=d, alpha=al, beta=be)
        plans.append(Plan(P.d, P.alpha, P.beta, L, Lc, seed=seed + 3))
        ss.append(_t(torch_dev, P.s_flat()))
        gs.append(_t(torch_dev, P.g_flat()))
    ref = [pl.solve(s, g, max_iter=40, precision=precision) for pl, s, g in zip(plans, ss, gs)]
    iters = sorted({info["iterations"] for _, info in ref})
    _say("   individual iteration counts", [info["iterations"] for _, info in ref])
    assert len(iters) > 1  # members stop at different steps
    batch = Batch(plans)
    for rep in range(2):  # the second call replays the captured graph
        us, infos = batch.solve(ss, gs, max_iter=40, precision=precision)
        for (u_ref, i_ref), u, info in zip(ref, us, infos):
            assert info["iterations"] == i_ref["iterations"] and info["status"] == i_ref["status"]
            assert info["precision"] == i_ref["precision"]
            assert np.array_equal(u.cpu().numpy(), u_ref.cpu().numpy())
            assert info["rnorm"] == i_ref["rnorm"]


def test_batch_skeleton_sparse_matches_individual_solves(torch_dev):
    """With skeleton-sparse refinement requested, the d = 3 members of a batch run it and the others
    the fine-mesh loop; every member ends bitwise where its own asdsm_solve with the same request
    ends, although members stop at different steps and the graph is captured again without them."""
    from paper_2303_01163_amd.asdsm import Batch, Plan
    plans, ss, gs = [], [], []
    for fam, L, Lc, d, seed, al, be in BATCH_MEMBERS:
        P = make_problem(fam, L, seed=seed, d=d, alpha=al, beta=be)
        plans.append(Plan(P.d, P.alpha, P.beta, L, Lc, seed=seed + 3))
        ss.append(_t(torch_dev, P.s_flat()))
        gs.append(_t(torch_dev, P.g_flat()))
    ref = [pl.solve(s, g, max_iter=40, skeleton=(pl.d == 3)) for pl, s, g in zip(plans, ss, gs)]
    assert len({info["iterations"] for _, info in ref}) > 1
    assert any(pl.d == 3 for pl in plans) and any(pl.d != 3 for pl in plans)
    batch = Batch(plans)
    for rep in range(2):
        us, infos = batch.solve(ss, gs, max_iter=40, skeleton=True)
        for (u_ref, i_ref), u, info in zip(ref, us, infos):
            assert info["iterations"] == i_ref["iterations"] and info["status"] == i_ref["status"]
            assert np.array_equal(u.cpu().numpy(), u_ref.cpu().numpy())
            assert info["rnorm"] == i_ref["rnorm"]


def test_probes_measure_plausible_ceilings(torch_dev):
    """The measured ceilings the bench reports next to the datasheet peaks (78.6 TFLOP/s FP64
    matrix, 8 TB/s HBM): positive and below them, and argument errors rejected."""
    from paper_2303_01163_amd import asdsm
    tf = asdsm.probe_mfma_f64(iters=2000)
    tb = asdsm.probe_copy(nbytes=1 << 28, reps=3)
    _say("   probes: FP64 MFMA %.1f TFLOP/s, copy %.2f TB/s" % (tf, tb))
    assert 5.0 < tf < 80.0
    assert 0.5 < tb < 8.5
    lib = asdsm.load_library()
    import ctypes
    out = ctypes.c_double()
    assert lib.asdsm_probe_mfma_f64(None, 10, None, ctypes.byref(out)) == -1
    assert lib.asdsm_probe_copy(None, None, 1024, 1, None, ctypes.byref(out)) == -1


def test_autotuned_plan_keeps_parity(torch_dev):
    """After the autotuner has picked a transform tile shape, the iterates still match the oracle."""
    P = make_problem("sinbump3d", 6, seed=4)
    o = Oracle(P.d, P.alpha, P.beta, 6, 3, seed=21)
    ref = o.solve(P.s, P.g, max_iter=3, rtol=0, stag_window=0, keep_iterates=True)
    pl = _plan(P, 6, 3, seed=21)
    tuned = pl.autotune(repeats=3)
    _say("   autotune:", tuned)
    assert tuned["tile"] in ("32x32 k32", "64x32 k32", "32x64 k32", "64x64 k16", "plane panels 16")
    assert tuned["ms_per_aniso_solve"] > 0
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    for K in (0, 3):
        u, info = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0)
        assert _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F")) <= TOL_ITER, K


ANISO_TILES = ("32x32", "64x32", "32x64", "64x64", "plane")


@pytest.mark.parametrize("L,Lc,seed", [(5, 2, 3), (6, 3, 4)])
def test_every_transform_tile_matches_the_oracle(torch_dev, L, Lc, seed):
    """asdsm_set_tile: the anisotropic solves with every transform tile shape (four batched-GEMM
    tilings, one launch per fine axis, and the plane kernel, both fine axes of a coarse slab in one
    launch) against the oracle's banded LU, and the iterates of a short solve."""
    P = make_problem("sinbump3d", L, seed=seed)
    o = Oracle(3, P.alpha, P.beta, L, Lc, seed=seed + 1)
    ref = o.solve(P.s, P.g, max_iter=2, rtol=0, stag_window=0, keep_iterates=True)
    pl = _plan(P, L, Lc, seed=seed + 1)
    rng = np.random.default_rng(200 + seed)
    rhs = [rng.standard_normal(o.grid.mesh_dims((k,))) for k in range(3)]
    x_or = [o.solve_mesh((k,), rhs[k]) for k in range(3)]
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    line = any(ax >= 0 for ax, _ in pl.line_axes().values())
    for tile in ANISO_TILES:
        if tile == "plane" and line:
            continue  # the plane kernel transforms both fine axes; line-axis plans refuse it
        _say("tile", tile, L, Lc, seed)
        pl.set_tile(tile)
        for k in range(3):
            x = pl.mesh_solve(1 << k, _t(torch_dev, _canon(3, (k,), rhs[k]))).cpu().numpy()
            assert _rel(_uncanon(o.grid, (k,), x), x_or[k]) <= TOL_OP, (tile, k)
        u, _ = pl.solve(s, g, max_iter=2, rtol=0, stag_window=0)
        assert _rel(u.cpu().numpy(), ref.iterates[2].reshape(-1, order="F")) <= TOL_ITER, tile


def test_every_transform_tile_at_full_size(torch_dev):
    """127^3 (the benchmark's plan: line axes on its ill-conditioned fine axis): every tile shape's
    anisotropic solves satisfy their equations, and the complete solves agree."""
    P = make_problem("sinbump3d", 7, seed=0)
    o = Oracle(3, P.alpha, P.beta, 7)
    pl = _plan(P, 7, 0, seed=0)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    rng = np.random.default_rng(9)
    rhs = [rng.standard_normal(o.grid.mesh_dims((k,))) for k in range(3)]
    sols = {}
    line = any(ax >= 0 for ax, _ in pl.line_axes().values())
    for tile in ANISO_TILES:
        if tile == "plane" and line:
            continue  # the plane kernel transforms both fine axes; line-axis plans refuse it
        _say("tile 127^3", tile)
        pl.set_tile(tile)
        for k in range(3):
            x = _uncanon(o.grid, (k,), pl.mesh_solve(1 << k, _t(torch_dev, _canon(3, (k,), rhs[k]))).cpu().numpy())
            res = apply_operator(x, mesh_coeffs(o.grid, P.alpha, P.beta, (k,))) - rhs[k]
            assert np.linalg.norm(res) <= 1e-9 * np.linalg.norm(rhs[k]), (tile, k)
        u, info = pl.solve(s, g, max_iter=50, rtol=1e-10, stag_window=3)
        sols[tile] = (u.cpu().numpy(), info["iterations"])
    u0, it0 = sols[ANISO_TILES[0]]
    for tile, (u1, it1) in sols.items():
        assert it1 == it0, tile
        assert _rel(u1, u0) <= TOL_ITER, tile


def test_set_tile_errors(torch_dev):
    from paper_2303_01163_amd.asdsm import AsdsmError
    P = make_problem("sinprod2d", 5, seed=0)
    pl = _plan(P, 5, 2)
    with pytest.raises(AsdsmError) as ei:
        pl.set_tile("plane")
    assert ei.value.code == -6
    with pytest.raises(AsdsmError) as ei:
        pl.set_tile(9)
    assert ei.value.code == -1
    pl.set_tile("64x64")
    assert pl.tile_name() == "64x64 k16"
    pl.set_tile("auto")
    assert pl.tile_name() == "auto"
    P3 = make_problem("sinbump3d", 5, seed=4)
    pl3 = _plan(P3, 5, 2)
    assert all(ax < 0 for ax, _ in pl3.line_axes().values())
    assert pl3.tile_name() == "plane panels 16"    # picked by size at N_f <= 127
    pl3.set_tile("32x32")
    assert pl3.tile_name() == "32x32 k32"
    # a plan whose anisotropic meshes use line axes refuses the plane kernel
    P4 = make_problem("sinbump3d", 5, seed=0)
    pl4 = _plan(P4, 5, 2)
    assert any(ax >= 0 for ax, _ in pl4.line_axes().values())
    with pytest.raises(AsdsmError) as ei:
        pl4.set_tile("plane")
    assert ei.value.code == -6


SPARSE_CASES = [  # d = 3: (family, level, coarse_level, seed)
    ("sinbump3d", 5, 1, 3),   # 31^3, one coarse plane per axis, holes of 15^3 (MFMA filler)
    ("sinbump3d", 6, 2, 5),   # 63^3, 3 coarse planes per axis, holes of 15^3
    ("sinbump3d", 6, 3, 4),   # 63^3, 7 planes, holes of 7^3 (generic filler)
    ("sinprod", 5, 3, 1),     # 31^3, 7 planes, holes of 3^3
    ("sinprod", 4, 3, 2),     # 15^3, 7 planes, holes of one point
]


@pytest.mark.parametrize("fam,L,Lc,seed", SPARSE_CASES)
@pytest.mark.parametrize("eager", [False, True])
def test_skeleton_sparse_iterates(torch_dev, fam, L, Lc, seed, eager):
    """Skeleton-sparse refinement (r, q and the updates on the coarse planes only, holes filled when
    the loop ends) against the oracle's fine-mesh iteration, iterate by iterate, with the same
    tolerances as the fine-mesh GPU loop."""
    d = 3
    _say("skeleton-sparse iterates", fam, L, Lc, seed, "eager" if eager else "graph")
    P = make_problem(fam, L, seed=seed, d=d)
    o = Oracle(3, P.alpha, P.beta, L, Lc, seed=seed + 17)
    ref = o.solve(P.s, P.g, max_iter=5, rtol=0, stag_window=0, keep_iterates=True)
    pl = _plan(P, L, Lc, seed=seed + 17)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    b = o.fine_rhs(P.s, P.g)
    rtol_r = [100 * 2.2e-16 * _rounding_scale_of_residual(o, ref.iterates[k], b) / ref.res_hist[k]
              for k in range(6)]
    for K in (1, 3, 5):
        u, info = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0, skeleton=True, eager=eager)
        assert info["iterations"] == K
        assert _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F")) <= TOL_ITER, K
        for k in range(K + 1):
            assert abs(info["res_hist"][k] - ref.res_hist[k]) <= 1e-9 * ref.res_hist[k] + rtol_r[k] * ref.res_hist[k], k
        for k in range(K):
            assert abs(info["step_hist"][k] - ref.step_hist[k]) <= (1e-8 + rtol_r[k]) * abs(ref.step_hist[k]) + 1e-300, k
        # the returned iterate's own residual is the last one of the history
        _, nrm = pl.residual(u, s, g)
        assert abs(nrm - info["res_hist"][-1]) <= 1e-8 * nrm + rtol_r[K] * nrm


def test_skeleton_sparse_full_solve_matches_fine_loop(torch_dev):
    """127^3 (the benchmark's configuration, stagnation rule on): the skeleton-sparse solve takes the
    same steps as the fine-mesh solve and returns the same iterate."""
    _say("skeleton-sparse full solve 127^3")
    P = make_problem("sinbump3d", 7, seed=0)
    pl = _plan(P, 7, 0, seed=0)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u0, i0 = pl.solve(s, g, max_iter=50, rtol=1e-10, stag_window=3)
    u1, i1 = pl.solve(s, g, max_iter=50, rtol=1e-10, stag_window=3, skeleton=True)
    assert i1["iterations"] == i0["iterations"] and i1["status"] == i0["status"]
    assert _rel(u1.cpu().numpy(), u0.cpu().numpy()) <= TOL_ITER
    for a, c in zip(i0["res_hist"], i1["res_hist"]):
        assert abs(a - c) <= 1e-8 * a


def test_skeleton_sparse_at_255_matches_fine_loop(torch_dev):
    """255^3 (L_c = 4): the transforms contract over K = 255, so the forward transform that carries
    the skeleton update stages its operand chunk by chunk (the double-buffered form of the GEMM)
    rather than all at once; 12 skeleton-sparse steps, eager and replayed, against the fine-mesh
    loop (itself held to the oracle at smaller sizes): same iterates within 1e-10 and the same
    residual history."""
    _say("skeleton-sparse 255^3 against the fine loop")
    P = make_problem("sinbump3d", 8, seed=0)
    pl = _plan(P, 8, 4, seed=0)
    axes = pl.line_axes()
    # every anisotropic mesh with its line axis at canonical position 1 and no sweeps: the
    # configuration whose update rides on the forward transform
    for k in range(3):
        fine = [j for j in range(3) if j != k]
        assert axes[1 << k][0] == fine[1] and axes[1 << k][1] == 0, (k, axes)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u0, i0 = pl.solve(s, g, max_iter=12, rtol=0, stag_window=0)
    for eager in (False, True):
        u1, i1 = pl.solve(s, g, max_iter=12, rtol=0, stag_window=0, skeleton=True, eager=eager)
        assert i1["iterations"] == 12
        assert _rel(u1.cpu().numpy(), u0.cpu().numpy()) <= TOL_ITER, eager
        for a, c in zip(i0["res_hist"], i1["res_hist"]):
            assert abs(a - c) <= 1e-8 * a, eager


def test_line_solves_at_255_satisfy_their_mesh_equations(torch_dev):
    """255^3 (L_c = 4): each anisotropic mesh solves along a fine axis of 255 positions with the
    15 coarse points as its block; one mode's line and level matrices take 72 KiB, so the form that
    stages them in LDS runs with the workgroup LDS of CDNA4 beyond 64 KiB.  The banded-LU oracle is
    out of reach at this size (bandwidth 3825 over 975 k unknowns), so the solutions are checked
    against the oracle's stencil-form mesh operator: f - A x relative to f."""
    from oracle.asdsm_oracle import Grid
    _say("line solves at 255^3: mesh residuals")
    P = make_problem("sinbump3d", 8, seed=0)
    pl = _plan(P, 8, 4, seed=0)
    grid = Grid(3, 8, 4)
    rng = np.random.default_rng(11)
    for k in range(3):
        S = (k,)
        rhs = rng.standard_normal(grid.mesh_dims(S))
        x = _uncanon(grid, S, pl.mesh_solve(1 << k, _t(torch_dev, _canon(3, S, rhs))).cpu().numpy())
        res = rhs - apply_operator(x, mesh_coeffs(grid, P.alpha, P.beta, S))
        rel = float(np.linalg.norm(res) / np.linalg.norm(rhs))
        _say("  M_%d: ||f - A x|| / ||f|| = %.2e" % (k, rel))
        assert rel <= 1e-11, (k, rel)


def test_hole_line_solve_at_255_leaves_no_hole_residual(torch_dev):
    """255^3 (L_c = 4) on a draw whose 15^3 holes have two axes too ill-conditioned for fast
    diagonalisation (cell Peclet 0.64 and 0.98) and whose mesh with both as fine axes diagonalises
    its coarse axis: 4096 holes solved together by the hole line solve.  Every ASDSM iterate has
    zero residual in the holes (Proposition 3.2(2)), so after skeleton-sparse steps and the final
    fill the fine residual of the returned iterate, taken by the stencil pass, must vanish on the
    hole points to rounding while the skeleton still carries the unconverged residual."""
    from paper_2303_01163_amd.asdsm import Plan
    _say("hole line solve at 255^3: hole residual")
    c = make_problem("sinbump_wide", 2, seed=1034, d=3)
    pl = Plan(3, c.alpha, c.beta, 8, 0, seed=1034)
    P = make_problem("sinbump_wide", 8, seed=1034, d=3)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u, info = pl.solve(s, g, max_iter=5, rtol=0, stag_window=0, skeleton=True)
    assert info["iterations"] == 5
    r, _ = pl.residual(u, s, g)
    Nf, n = 255, 16
    r = r.cpu().numpy().reshape((Nf,) * 3, order="F")
    on_plane = (np.arange(Nf) % n) == n - 1
    hole = ~(on_plane[:, None, None] | on_plane[None, :, None] | on_plane[None, None, :])
    rh, rs = np.linalg.norm(r[hole]), np.linalg.norm(r[~hole])
    _say("  ||r|| holes %.3e, skeleton %.3e, ||b|| %.3e" % (rh, rs, info["bnorm"]))
    assert rs > 1e-6 * info["bnorm"]
    assert rh <= 1e-10 * info["bnorm"], (rh, rs)


def test_skeleton_sparse_refused_where_not_built(torch_dev):
    from paper_2303_01163_amd.asdsm import AsdsmError
    P2 = make_problem("sinprod2d", 6, seed=0)
    pl2 = _plan(P2, 6, 2, seed=0)
    with pytest.raises(AsdsmError) as ei:
        pl2.solve(_t(torch_dev, P2.s_flat()), _t(torch_dev, P2.g_flat()), max_iter=2, skeleton=True)
    assert ei.value.code == -6


def test_skeleton_sparse_resume_and_fp32(torch_dev):
    """Resuming a skeleton-sparse solve continues it exactly as one longer solve would (the skeleton
    is rebuilt from the resumed fine iterate), and FP32 error guesses combine with the skeleton loop
    as with the fine-mesh loop."""
    P = make_problem("sinbump3d", 6, seed=5)
    pl = _plan(P, 6, 2, seed=22)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    u5, i5 = pl.solve(s, g, max_iter=5, rtol=0, stag_window=0, skeleton=True)
    u2, _ = pl.solve(s, g, max_iter=2, rtol=0, stag_window=0, skeleton=True)
    u2b, i3 = pl.solve(s, g, u=u2, max_iter=3, rtol=0, stag_window=0, skeleton=True, resume=True, k0=2)
    assert i3["iterations"] == 3
    assert _rel(u2b.cpu().numpy(), u5.cpu().numpy()) <= TOL_ITER
    uf, if_ = pl.solve(s, g, max_iter=5, rtol=0, stag_window=0, precision="fp32")
    us, is_ = pl.solve(s, g, max_iter=5, rtol=0, stag_window=0, precision="fp32", skeleton=True)
    assert if_["precision"] == is_["precision"]
    assert _rel(us.cpu().numpy(), uf.cpu().numpy()) <= TOL_ITER


def test_new_workspace_rebuilds_the_captured_graph(torch_dev):
    """A plan's captured refinement graph points into its workspace: after asdsm_set_workspace the
    next solve (same iterate pointer) must use the new workspace.  The old one is overwritten with
    NaN before that solve; the result must equal a fresh plan's bit for bit, for a single plan and
    for a member of a batch."""
    import torch
    from paper_2303_01163_amd import asdsm
    P = make_problem("sinbump3d", 5, seed=4)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    kw = dict(max_iter=6, rtol=0, stag_window=0)
    fresh = _plan(P, 5, 2, seed=4)
    want, _ = fresh.solve(s, g, **kw)
    pl = _plan(P, 5, 2, seed=4)
    u = torch.empty_like(want)
    pl.solve(s, g, u=u, **kw)                     # captures the graph
    old = pl.attach_workspace()
    old.fill_(255)                                # all-ones bytes: NaN doubles
    pl.solve(s, g, u=u, **kw)
    assert torch.equal(u, want)
    # batch member: the batch graph is rebuilt when a member's workspace changes
    P2 = make_problem("sinbump3d", 5, seed=6)
    s2, g2 = _t(torch_dev, P2.s_flat()), _t(torch_dev, P2.g_flat())
    want2, _ = _plan(P2, 5, 2, seed=6).solve(s2, g2, **kw)
    pl2 = _plan(P2, 5, 2, seed=6)
    u2 = torch.empty_like(want2)
    batch = asdsm.Batch([pl, pl2])
    batch.solve([s, s2], [g, g2], us=[u, u2], **kw)
    old2 = pl2.attach_workspace()
    old2.fill_(255)
    batch.solve([s, s2], [g, g2], us=[u, u2], **kw)
    batch.close()
    assert torch.equal(u, want) and torch.equal(u2, want2)


def test_skeleton_sparse_resume_from_any_iterate(torch_dev):
    """Resuming the skeleton-sparse loop from an iterate that did not come from ASDSM: its holes are
    re-filled from its skeleton first (Algorithm 3), so the loop's assumption of a zero hole
    residual (Proposition 3.2(2)) holds; the returned iterate has a zero hole residual and the
    reported residual norm is that of the returned iterate."""
    P = make_problem("sinbump3d", 5, seed=5)
    pl = _plan(P, 5, 2, seed=3)
    o = Oracle(3, P.alpha, P.beta, 5, 2)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    rng = np.random.default_rng(1)
    u0 = _t(torch_dev, (P.u_exact + 0.01 * rng.standard_normal(P.u_exact.shape)).reshape(-1, order="F"))
    u, info = pl.solve(s, g, u=u0.clone(), max_iter=4, rtol=0, stag_window=0, skeleton=True, resume=True, k0=0)
    r, nrm = pl.residual(u, s, g)
    assert abs(info["rnorm"] - nrm) <= 1e-12 * nrm
    rr = r.cpu().numpy().reshape((31,) * 3, order="F")
    holes = o.grid.hole_mask()
    assert np.max(np.abs(rr[holes])) <= 1e-11 * info["bnorm"]
    h = info["res_hist"]
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(len(h) - 1))
