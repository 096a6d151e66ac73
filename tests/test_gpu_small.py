"""One-workgroup solve of small systems against the multi-launch compact path and the oracle.

Plain FP64 solves of a compact-layout handle with n <= 1024 rows, and at most
4096 directed slots or at most 6 slots per row, run the whole iteration in one
launch: a lane per row when the rows are that short, else a lane per slot.  Both paths perform
the same operations, so x, the variances, the messages, the sweep counts and
the frozen state left for later solves must agree bit for bit; the reported
residual is summed in another order (relative 1e-12).  Each small-path result
is also held to the FP64 oracle (Alg. 2) at the parity bar of the other tests.
"""
import numpy as np
import pytest
import torch

import _golden
import oracle
import paper_0811_2518_amd as g
import workloads
from paper_0811_2518_amd import binding

pytestmark = pytest.mark.gpu
DEV = "cuda"


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def e1():
    E1 = _golden.load("e1_tree.txt")
    return workloads.from_dense(_golden.as_float(_golden.matrix(E1)), _golden.as_float(_golden.vector(E1, "b")))


CASES = {
    "grid32": workloads.config1,                                    # n = 1024, E = 3968 (largest size class)
    "poisson10": lambda: workloads.poisson2d(10),
    "grid3d_8": lambda: workloads.grid3d_problem(8, 5),
    "grid3d_10": lambda: workloads.grid3d_problem(10, 6),           # 5400 slots, rows of at most 6
    "tree": lambda: workloads.random_tree(777, 80),
    "star_long_row": lambda: workloads.star_problem(600, 81),       # one row of 600 slots
    "er_isolated": lambda: workloads.er_problem(1000, 3, 82, ratio=1.3),
    "e1_toy": e1,
    "single_node": lambda: workloads.from_dense(np.array([[2.5]]), np.array([1.5])),
}


def pair(p, **kw):
    one = g.Solver(p.row_ptr, p.col, p.val, device=DEV, layout="compact", **kw)
    multi = g.Solver(p.row_ptr, p.col, p.val, device=DEV, layout="compact", multi_launch=True, **kw)
    return one, multi


def same(a, b):
    return torch.equal(a, b)


@pytest.mark.parametrize("name", sorted(CASES))
def test_fixed_rounds_bitwise_and_oracle(name):
    p = CASES[name]()
    max_deg = int(np.max(np.diff(p.row_ptr))) - 1
    assert p.n <= 1024 and (p.num_offdiag <= 4096 or max_deg <= 6)
    one, multi = pair(p)
    b = dev(p.b)
    for T in (0, 1, 2, 3, 7, 25):
        x1, i1, v1 = one.solve(b, tol=0, max_iter=T, var=True)
        x2, i2, v2 = multi.solve(b, tol=0, max_iter=T, var=True)
        assert same(x1, x2) and same(v1, v2), (name, T)
        assert i1["sweeps"] == i2["sweeps"] == T and i1["status"] == i2["status"] == binding.OK
        assert i1["rel_residual"] == pytest.approx(i2["rel_residual"], rel=1e-12, abs=1e-300)
        P1, h1 = one.messages()
        P2, h2 = multi.messages()
        assert same(P1, P2) and same(h1, h2), (name, T)
        ref = oracle.broadcast_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=T, return_messages=True)
        xr = x1.cpu().numpy()
        assert np.linalg.norm(xr - ref["x"]) <= 1e-13 * max(np.linalg.norm(ref["x"]), 1e-300), (name, T)
        np.testing.assert_allclose(P1.cpu().numpy(), ref["P"], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("check_every", [1, 3])
def test_converged_bitwise_and_oracle(name, check_every):
    p = CASES[name]()
    one, multi = pair(p, check_every=check_every, reuse_precision=False)
    b = dev(p.b)
    x1, i1, v1 = one.solve(b, tol=1e-10, max_iter=2000, var=True)
    x2, i2, v2 = multi.solve(b, tol=1e-10, max_iter=2000, var=True)
    assert i1["sweeps"] == i2["sweeps"] and i1["status"] == i2["status"] == binding.OK
    assert same(x1, x2) and same(v1, v2)
    assert i1["rel_residual"] == pytest.approx(i2["rel_residual"], rel=1e-12, abs=1e-300)
    ref = oracle.broadcast_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=1e-10, max_sweeps=2000,
                                check_every=check_every)
    assert i1["sweeps"] == ref["sweeps"]
    xr = x1.cpu().numpy()
    assert np.linalg.norm(xr - ref["x"]) <= 1e-10 * np.linalg.norm(ref["x"])


def test_reuse_and_adjoint_follow_the_same_state():
    """The frozen precisions left by the one-launch solve drive the later mean-only solves and
    the adjoint exactly as those left by the multi-launch path."""
    p = workloads.config1()
    one, multi = pair(p)
    b = dev(p.b)
    rng = np.random.default_rng(3)
    b2 = dev(rng.standard_normal(p.n))
    for s in (one, multi):
        s.solve(b, tol=1e-10, max_iter=2000)
    xa, ia = one.solve(b2, tol=1e-10, max_iter=2000)
    xb, ib = multi.solve(b2, tol=1e-10, max_iter=2000)
    assert ia["sweeps"] == ib["sweeps"] and same(xa, xb)
    gx = dev(rng.standard_normal(p.n))
    ga, gva, _ = one.backward(xa, gx, tol=1e-12)
    gb, gvb, _ = multi.backward(xb, gx, tol=1e-12)
    assert same(ga, gb) and same(gva, gvb)


@pytest.mark.parametrize("name", ["grid32", "grid3d_10"])  # rows of at most 4 and of 6 slots
@pytest.mark.parametrize("check_every", [1, 3])
def test_caps_and_statuses_match(name, check_every):
    """max_iter caps, M = 0 with a tolerance, and an unreachable tolerance: the
    one-launch loop must end after sweep M and the check of round M."""
    p = CASES[name]()
    one, multi = pair(p, reuse_precision=False, check_every=check_every)
    b = dev(p.b)
    for tol, M in ((1e-10, 0), (1e-10, 1), (1e-10, 10), (1e-300, 40), (1e-300, 41), (0.5, 5)):
        x1, i1 = one.solve(b, tol=tol, max_iter=M, check=False)
        x2, i2 = multi.solve(b, tol=tol, max_iter=M, check=False)
        assert (i1["status"], i1["sweeps"], i1["converged"]) == (i2["status"], i2["sweeps"], i2["converged"]), (tol, M)
        assert same(x1, x2), (tol, M)


def test_breakdown_is_reported_alike():
    """A singular 2 x 2 system: the first aggregates vanish, so the means of round 1 are not
    finite.  Both paths must end with the same error."""
    A = np.array([[1.0, 1.0], [1.0, 1.0]])
    p = workloads.from_dense(A, np.array([1.0, 2.0]))
    one, multi = pair(p, reuse_precision=False)
    _, i1 = one.solve(dev(p.b), tol=1e-10, max_iter=50, check=False)
    _, i2 = multi.solve(dev(p.b), tol=1e-10, max_iter=50, check=False)
    assert i1["status"] == i2["status"]
    assert i1["status"] < 0
