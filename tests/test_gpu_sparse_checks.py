"""Sparse checks in the inner solves of the FP32 refinement.

An inner solve checks rounds 0-2, at least every fourth round, and the rounds
from one before the round its residuals predict to meet the inner tolerance,
so it may stop a few rounds after the first round that meets it.  The outer
step's FP64 residual (the correction equation of Ch. 5 Sec. 5.3) sets the
accuracy, so whatever the schedule the refinement must reach the outer
tolerance and the solution of a direct FP64 solve.  The cases include a tree,
on which GaBP is exact after as many rounds as the tree is deep (its residual
falls to rounding at once, far below any prediction from the decay so far),
slowly converging graphs whose inner solves run many rounds, and inner solves
capped at three sweeps.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import paper_0811_2518_amd as g
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda"


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


CASES = {
    "tree": lambda: workloads.random_tree(4000, 81, ratio=1.05),
    "er": lambda: workloads.er_problem(20000, 8, 82, ratio=1.05),
    "grid3d": lambda: workloads.grid3d_problem(16, 83),
    "powerlaw": lambda: workloads.powerlaw_problem(8000, 8, 84, beta=2.1),
}


@pytest.mark.parametrize("inner_max", [10000, 3])
@pytest.mark.parametrize("name", sorted(CASES))
def test_fp32_refinement_reaches_tolerance(name, inner_max):
    p = CASES[name]()
    s = g.Solver(p.row_ptr, p.col, p.val, device=DEV, precision="fp32", layout="compact",
                 reuse_precision=False, inner_max_iter=inner_max, max_outer=5000)
    x, info = s.solve(dev(p.b), tol=1e-10, max_iter=1000000)
    assert info["status"] == 0 and info["converged"] == 1, info
    A = p.scipy()
    xh = x.cpu().numpy()
    assert np.linalg.norm(p.b - A @ xh) / np.linalg.norm(p.b) <= 1.05e-10
    # reference: conjugate gradients in FP64 to a relative residual of 1e-14
    # (A is symmetric and diagonally dominant with a positive diagonal; a
    # direct sparse solve of the random graphs fills in far too much)
    ref, cg_info = spla.cg(A, p.b, rtol=1e-14, atol=0.0, maxiter=20000)
    assert cg_info == 0
    # the residual bounds the error through the condition number, at most
    # (r + 1) / (r - 1) = 41 for the smallest dominance ratio here, r = 1.05
    assert np.linalg.norm(xh - ref) / np.linalg.norm(ref) <= 1e-8
    s.close()
