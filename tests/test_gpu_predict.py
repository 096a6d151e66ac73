"""The predicted last check of a compact solve to a tolerance.

The check of round t is fused into sweep t+1, so a solve ends with a sweep
whose messages are never used.  When the residuals seen so far predict that
round t-1 meets the tolerance, launch t is the residual-only check of round
t-1 instead, and sweep t, without repeating that check, follows only if the
check fails.  GABP_FLAG_PREDICT_ALL takes that form at every checked launch
from round 2 on, so both outcomes run all the time: every result must be the
same bits as a handle without the flag.  The inner solves of the FP32
refinement are the exception: without the flag they skip the checks of rounds
far above their predicted stop, so there the two handles must each reach the
tolerance, with corrections that agree to the inner tolerance.
"""
import numpy as np
import pytest
import torch

import _golden
import paper_0811_2518_amd as g
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda"


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def e1():
    E1 = _golden.load("e1_tree.txt")
    return workloads.from_dense(_golden.as_float(_golden.matrix(E1)), _golden.as_float(_golden.vector(E1, "b")))


CASES = {
    "er_3001": lambda: workloads.er_problem(3001, 8, 77, ratio=1.1),      # XCD row order
    "powerlaw": lambda: workloads.powerlaw_problem(8000, 8, 90, beta=2.1),  # rows swept in chunks
    "grid3d_10": lambda: workloads.grid3d_problem(10, 79),
    "e1_toy": e1,
}


def pair(p, **kw):
    plain = g.Solver(p.row_ptr, p.col, p.val, device=DEV, layout="compact", multi_launch=True,
                     reuse_precision=False, **kw)
    every = g.Solver(p.row_ptr, p.col, p.val, device=DEV, layout="compact", predict_all=True,
                     reuse_precision=False, **kw)
    return plain, every


def same(a, b, bvec, **kw):
    xa, ia = a.solve(bvec, check=False, **kw)
    xb, ib = b.solve(bvec, check=False, **kw)
    assert ia["status"] >= 0, ia
    assert torch.equal(xa, xb), kw
    for key in ("sweeps", "outer_iters", "converged", "status", "rel_residual"):
        assert ia[key] == ib[key], (key, ia, ib)
    return ia


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("check_every", [1, 3])
def test_fp64_solves(name, check_every):
    p = CASES[name]()
    a, b = pair(p, check_every=check_every)
    bv = dev(p.b)
    info = same(a, b, bv, tol=1e-10, max_iter=3000)
    assert info["converged"] == 1
    same(a, b, bv, tol=1e-14, max_iter=7)   # every predicted check fails
    same(a, b, bv, tol=1e-10, max_iter=1)
    same(a, b, dev(np.random.default_rng(4).standard_normal(p.n)), tol=1e-8, max_iter=3000)


@pytest.mark.parametrize("name", ["er_3001", "powerlaw", "grid3d_10"])
def test_fp32_refinement(name):
    p = CASES[name]()
    a, b = pair(p, precision="fp32")
    bv = dev(p.b)
    xa, ia = a.solve(bv, check=False, tol=1e-10, max_iter=20000)
    xb, ib = b.solve(bv, check=False, tol=1e-10, max_iter=20000)
    for info in (ia, ib):
        assert info["status"] == 0 and info["converged"] == 1 and info["outer_iters"] >= 1, info
        assert info["rel_residual"] <= 1e-10, info
    # both are within tol of the solution, so within about kappa * tol of each other
    assert float(torch.linalg.norm(xa - xb) / torch.linalg.norm(xb)) <= 1e-8
