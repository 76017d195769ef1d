"""GPU parity of submeshes solved with a line axis (block cyclic reduction along one fine axis, the
other fine axes diagonalised) against the FP64 CPU oracle, whose banded LU with partial pivoting
handles every cell Peclet number.

Draws of the advection-dominated family (alpha log-uniform in [0.01, 1], beta uniform in [-10, 10])
with one axis whose spectrum is complex (|P| >= 1, up to 7.6) or whose eigenvector matrix is too
ill-conditioned for fast diagonalisation, and the 127^3 benchmark draw at lower levels, where line
axes replace the refinement sweeps.  Tolerances as in the other parity tests: submesh solves and
residuals <= 1e-11 relative L2, iterates <= 1e-10.
"""
import itertools
import sys

import numpy as np
import pytest

from oracle.asdsm_oracle import Oracle
from paper_2303_01163_amd.workloads import make_problem

pytestmark = pytest.mark.gpu

TOL_OP = 1e-11
TOL_ITER = 1e-10

# (family, level, coarse level, d, seed, cell Peclet numbers of the fine axes for the record)
LINE_CASES = [
    ("sinbump_wide", 5, 0, 3, 2),    # P = (3.82, 0.79, 0.17): complex axis 0, hard axis 1
    ("sinbump_wide", 5, 0, 3, 6),    # P = (0.33, 3.13, 0.76)
    ("sinbump_wide", 6, 0, 3, 2),    # 63^3: P = (1.91, 0.40, 0.08)
    ("sinbump_wide", 6, 0, 3, 8),    # 63^3: P = (1.00, 0.06, 0.39)
    ("sinbump_wide", 6, 4, 3, 9),    # 63^3, 15 coarse planes: P = (0.08, 0.90, 0.40)
    ("sinbump_wide", 5, 0, 2, 0),    # 31^2: P = (0.76, 4.36)
    ("sinbump_wide", 6, 0, 2, 3),    # 63^2: P = (3.17, 0.43)
    ("sinbump_wide", 4, 2, 4, 5),    # 15^4: P = (0.68, 0.18, 0.53, 7.62)
    ("sinbump_wide", 4, 2, 4, 4),    # 15^4, 3 coarse planes per axis: P = (0.09, 0.73, 0.21, 14.0)
    ("sinbump3d", 5, 0, 3, 0),       # the benchmark draw at 31^3: line axes instead of a sweep
]


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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(fam, L, d, seed):
    return make_problem(fam, L, seed=seed, d=d)


@pytest.mark.parametrize("fam,L,Lc,d,seed", LINE_CASES)
def test_line_axis_mesh_solves(torch_dev, fam, L, Lc, d, seed):
    """Every submesh / intersection / coarse system against the oracle's banded LU."""
    from paper_2303_01163_amd.asdsm import Plan
    P = _problem(fam, L, d, seed)
    o = Oracle(P.d, P.alpha, P.beta, L, Lc or None)
    pl = Plan(P.d, P.alpha, P.beta, L, Lc, seed=seed)
    rng = np.random.default_rng(200 + seed)
    for r_ in range(1, P.d + 1):
        for S in itertools.combinations(range(P.d), r_):
            _say("line mesh", fam, L, Lc, d, seed, S)
            mask = sum(1 << j for j in S)
            rhs = rng.standard_normal(o.grid.mesh_dims(S))
            x_or = o.solve_mesh(S, rhs)
            x = pl.mesh_solve(mask, _t(torch_dev, _canon(P.d, S, rhs))).cpu().numpy()
            rel = _rel(_uncanon(o.grid, S, x), x_or)
            assert rel <= TOL_OP, (S, rel)
    pl.close()


@pytest.mark.parametrize("fam,L,Lc,d,seed", LINE_CASES)
def test_line_axis_iterates(torch_dev, fam, L, Lc, d, seed):
    """u^(0) (Algorithm 1) and u^(1..4) (Algorithm 4): graph replay and eager launches, and the
    skeleton-sparse loop for d = 3."""
    from paper_2303_01163_amd.asdsm import Plan
    P = _problem(fam, L, d, seed)
    _say("line iterates", fam, L, Lc, d, seed)
    o = Oracle(P.d, P.alpha, P.beta, L, Lc or None, seed=seed + 31)
    ref = o.solve(P.s, P.g, max_iter=4, rtol=0, stag_window=0, keep_iterates=True)
    pl = Plan(P.d, P.alpha, P.beta, L, Lc, seed=seed + 31)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    for K in (0, 1, 4):
        u, info = pl.solve(s, g, max_iter=K, rtol=0, stag_window=0)
        assert info["iterations"] == K
        rel = _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F"))
        assert rel <= TOL_ITER, (K, rel)
    ue, _ = pl.solve(s, g, max_iter=4, rtol=0, stag_window=0, eager=True)
    assert _rel(ue.cpu().numpy(), ref.iterates[4].reshape(-1, order="F")) <= TOL_ITER
    if d == 3:
        us, info = pl.solve(s, g, max_iter=4, rtol=0, stag_window=0, skeleton=True)
        assert _rel(us.cpu().numpy(), ref.iterates[4].reshape(-1, order="F")) <= TOL_ITER
    pl.close()


def test_bench_draw_uses_line_axes_without_sweeps(torch_dev):
    """The 127^3 benchmark draw (one fine axis with cond(V) = 1.2e8): the anisotropic meshes are
    solved with line axes, so no refinement sweep is needed; the mesh solves satisfy their systems."""
    from paper_2303_01163_amd.asdsm import Plan
    P = make_problem("sinbump3d", 7, seed=0)
    o = Oracle(3, P.alpha, P.beta, 7, None)
    pl = Plan(3, P.alpha, P.beta, 7, 0, seed=0)
    info = pl.line_axes()
    for k in range(3):
        assert info[1 << k][0] >= 0 and info[1 << k][1] == 0, (k, info[1 << k])
    rng = np.random.default_rng(3)
    for S in ((0,), (1,), (2,)):
        mask = sum(1 << j for j in S)
        rhs = rng.standard_normal(o.grid.mesh_dims(S))
        x_or = o.solve_mesh(S, rhs)
        x = _uncanon(o.grid, S, pl.mesh_solve(mask, _t(torch_dev, _canon(3, S, rhs))).cpu().numpy())
        assert _rel(x, x_or) <= TOL_OP, S
    pl.close()
