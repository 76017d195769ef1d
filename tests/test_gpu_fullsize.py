"""GPU checks at the benchmark's full sizes, against the FP64 CPU oracle.

* The timed path of the benchmark (127^3, seed 0: skeleton-sparse refinement replayed from the
  captured graph, autotuned transform tile, no stagnation cut-off) against the oracle's iterates
  after 5, 15 and 30 refinement steps (relative L2 <= 1e-10, the iterate bar of the FP64 path).
* The benchmark's complete solve (relative residual 1e-10) against the oracle's fine solution u_ff
  (preconditioned GMRES to the rounding floor): relative L2 error <= 1e-8, the metric's target.
* The fine residual r = b - A u at 255^3 and 63^4 against the oracle's stencil form of the operator
  (relative L2 <= 1e-11).
"""
import sys

import numpy as np
import pytest

from oracle.asdsm_oracle import (Grid, Oracle, apply_operator, fine_reference_solve, mesh_coeffs,
                                 rhs_on_mesh)
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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bench_problem():
    return make_problem("sinbump3d", 7, seed=0)


@pytest.fixture(scope="module")
def bench_plan(torch_dev, bench_problem):
    from paper_2303_01163_amd.asdsm import Plan
    P = bench_problem
    pl = Plan(3, P.alpha, P.beta, 7, 0, seed=0)
    pl.autotune(repeats=3)
    return pl


def test_bench_path_iterates_at_full_size(torch_dev, bench_problem, bench_plan):
    """The benchmark's refinement path at 127^3 (skeleton-sparse, graph replay, the autotuned tile)
    against the oracle's Algorithm 4 iterates u^(5), u^(15), u^(30), same seed."""
    P = bench_problem
    _say("oracle 127^3, 30 steps")
    ref = Oracle(3, P.alpha, P.beta, 7, None, seed=0).solve(P.s, P.g, max_iter=30, rtol=0.0,
                                                            stag_window=0, keep_iterates=True)
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    for K in (5, 15, 30):
        _say("gpu 127^3 skeleton-sparse K =", K, bench_plan.tile_name())
        u, info = bench_plan.solve(s, g, max_iter=K, rtol=0.0, stag_window=0, skeleton=True)
        assert info["iterations"] == K
        rel = _rel(u.cpu().numpy(), ref.iterates[K].reshape(-1, order="F"))
        _say("  rel L2 vs oracle", rel)
        assert rel <= TOL_ITER, (K, rel)


def test_bench_solve_meets_the_error_target(torch_dev, bench_problem, bench_plan):
    """The benchmark's complete solve (relative residual <= 1e-10, no stagnation cut-off, at most
    4000 steps) returns an iterate within 1e-8 (relative L2) of the oracle's fine solution u_ff."""
    P = bench_problem
    s, g = _t(torch_dev, P.s_flat()), _t(torch_dev, P.g_flat())
    _say("gpu 127^3 complete solve")
    u, info = bench_plan.solve(s, g, max_iter=4000, rtol=1e-10, stag_window=0, skeleton=True)
    assert info["status_name"] == "ok"
    assert info["rnorm"] <= 1e-10 * info["bnorm"]
    _say("  steps", info["iterations"], "oracle u_ff")
    uff, rr = fine_reference_solve(3, P.alpha, P.beta, 7, P.s, P.g, precond="line")
    assert rr <= 1e-13
    err = _rel(u.cpu().numpy(), uff.reshape(-1, order="F"))
    _say("  rel L2 error vs u_ff", err)
    assert err <= 1e-8


@pytest.mark.parametrize("fam,L,d,seed", [("sinbump3d", 8, 3, 2), ("sinprod", 6, 4, 3)])
def test_residual_parity_beyond_the_cache(torch_dev, fam, L, d, seed):
    """r = b - A u at 255^3 and 63^4 (working sets beyond the 256 MB Infinity Cache) against the
    oracle's right-hand side assembly and stencil-form operator."""
    from paper_2303_01163_amd.asdsm import Plan
    _say("residual", fam, L, d, seed)
    P = make_problem(fam, L, seed=seed, d=d)
    grid = Grid(d, L, None)
    rng = np.random.default_rng(seed)
    u = P.u_exact + 0.1 * rng.standard_normal(P.u_exact.shape)
    b = rhs_on_mesh(grid, (), P.s, P.g, P.alpha, P.beta)
    r_or = (b - apply_operator(u, mesh_coeffs(grid, P.alpha, P.beta, ()))).reshape(-1, order="F")
    del b
    pl = Plan(d, P.alpha, P.beta, L, 0, seed=seed)
    r, nrm = pl.residual(_t(torch_dev, u.reshape(-1, order="F")), _t(torch_dev, P.s_flat()),
                         _t(torch_dev, P.g_flat()))
    assert _rel(r.cpu().numpy(), r_or) <= TOL_OP
    assert abs(nrm - np.linalg.norm(r_or)) <= 1e-12 * np.linalg.norm(r_or)
    pl.close()
