"""Pins of the oracle's serial schedule (Ch. 2 Sec. 2.3) and its colouring.

CPU only.  Each test holds an oracle function to something other than itself:
- a closed form;
- exact rational arithmetic against Gaussian elimination;
- the definition of the colouring checked by brute force;
- the one-node-at-a-time Alg. 1 form against the vectorised Alg. 2 form;
- the paper's claim that serial scheduling needs fewer rounds than parallel
  scheduling.
"""
from fractions import Fraction

import numpy as np
import pytest

import _golden
import oracle
import workloads


def _exact_solve(A, b):
    """Gauss-Jordan elimination over the rationals (plain definition of A^-1 b)."""
    n = len(A)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [M[r][k] - f * M[c][k] for k in range(n + 1)]
    return [M[i][n] / M[i][i] for i in range(n)]


def _neighbours(p):
    rows = np.repeat(np.arange(p.n), np.diff(p.row_ptr))
    off = rows != p.col
    return rows[off], p.col[off]


# ---------------------------------------------------------------------------
# colouring
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["er", "grid", "tree", "star"])
def test_greedy_colouring_is_first_fit(name):
    p = {"er": workloads.er_problem(300, 6, 11),
         "grid": workloads.grid2d_problem(9, 7, 3),
         "tree": workloads.random_tree(200, 5),
         "star": workloads.star_problem(40, 2)}[name]
    col = oracle.greedy_colouring(p.n, p.row_ptr, p.col)
    r, c = _neighbours(p)
    assert np.all(col[r] != col[c])                       # proper
    for i in range(p.n):                                   # first fit in row order
        lower = {int(col[j]) for j in c[r == i] if j < i}
        assert int(col[i]) == min(set(range(len(lower) + 1)) - lower)


def test_greedy_colouring_known_counts():
    # natural-order grids and trees are 2-coloured by first fit in row order
    # (a tree: each node's parent has a smaller index in these generators)
    for p in (workloads.grid2d_problem(6, 5, 1), workloads.grid3d_problem(4, 1)):
        assert oracle.greedy_colouring(p.n, p.row_ptr, p.col).max() == 1
    # the complete graph K_m needs m colours, assigned 0..m-1 in row order
    m = 6
    A = np.full((m, m), -0.1) + np.eye(m) * 2.0
    p = workloads.from_dense(A, np.ones(m))
    assert list(oracle.greedy_colouring(p.n, p.row_ptr, p.col)) == list(range(m))
    # no edges: one colour
    p = workloads.from_dense(np.eye(4) * 3.0, np.ones(4))
    assert list(oracle.greedy_colouring(p.n, p.row_ptr, p.col)) == [0, 0, 0, 0]


# ---------------------------------------------------------------------------
# closed forms and exactness
# ---------------------------------------------------------------------------

def test_serial_two_nodes_closed_form():
    # Sweep 1 visits node 0 with no messages yet, so its mean is b0 / a.
    # Node 1 then receives the exact message from its only neighbour, so it
    # holds the Schur-complement solution at once.  Sweep 2 makes node 0 exact too.
    a, c, d, b0, b1 = 3.0, -1.25, 2.5, 0.7, -1.9
    A = np.array([[a, c], [c, d]])
    b = np.array([b0, b1])
    p = workloads.from_dense(A, b)
    xs = np.linalg.solve(A, b)
    r1 = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=1)
    assert r1["colours"] == 2
    assert r1["x"][0] == pytest.approx(b0 / a, rel=1e-15)
    assert r1["x"][1] == pytest.approx((b1 - c * b0 / a) / (d - c * c / a), rel=1e-14)
    assert r1["x"][1] == pytest.approx(xs[1], rel=1e-14)
    r2 = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=2)
    assert np.allclose(r2["x"], xs, rtol=1e-14, atol=0)
    # marginal precisions after sweep 2: the exact 1 / (A^-1)_ii
    assert np.allclose(r2["prec"], oracle.dense_marginal_precisions(A), rtol=1e-14)


def test_serial_exact_on_trees_rationals():
    # GaBP is exact on trees (Ch. 2 Sec. 2.5) under any schedule, so once the
    # messages have crossed the tree the serial means equal A^-1 b exactly.
    E1 = _golden.load("e1_tree.txt")
    A = _golden.matrix(E1)
    b = _golden.vector(E1, "b")
    exact = _exact_solve(A, b)
    hist = oracle.naive_serial_gabp(A, b, [0, 1, 2], 3)
    assert hist[3] == exact
    rng = np.random.default_rng(4)
    n = 9
    parent = [int(rng.integers(0, i)) for i in range(1, n)]
    A = [[Fraction(0)] * n for _ in range(n)]
    for i, q in enumerate(parent, start=1):
        v = Fraction(int(rng.integers(-9, 10)) or 1, int(rng.integers(1, 7)))
        A[i][q] = A[q][i] = v
    for i in range(n):
        A[i][i] = sum(abs(v) for v in A[i]) + Fraction(1, 3)
    b = [Fraction(int(rng.integers(-5, 6)), 2) for _ in range(n)]
    exact = _exact_solve(A, b)
    hist = oracle.naive_serial_gabp(A, b, list(range(n)), n)
    assert hist[n] == exact
    # and stays exact
    assert oracle.naive_serial_gabp(A, b, list(range(n)), n + 2)[-1] == exact


def test_serial_vectorised_matches_one_node_at_a_time():
    # Alg. 2 form over colour classes against Alg. 1 visiting single nodes in
    # colour order: nodes of one class are not neighbours, so both give the
    # same iterates (up to rounding: the parameterisations differ)
    p = workloads.er_problem(40, 5, 9, ratio=1.15)
    A = oracle.dense_from_csr(p.n, p.row_ptr, p.col, p.val)
    colour = oracle.greedy_colouring(p.n, p.row_ptr, p.col)
    assert colour.max() >= 2
    order = [int(i) for i in np.argsort(colour, kind="stable")]
    hist = oracle.naive_serial_gabp(A.tolist(), list(p.b), order, 6)
    for t in range(1, 7):
        r = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=t)
        np.testing.assert_allclose(r["x"], hist[t], rtol=1e-12, atol=1e-14)


def test_serial_differs_from_parallel():
    # a sweep of serial scheduling is not a round of parallel scheduling
    p = workloads.config1()
    s = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=3)
    q = oracle.broadcast_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=3)
    assert np.max(np.abs(s["x"] - q["x"])) > 1e-3


# ---------------------------------------------------------------------------
# convergence: same fixed point, fewer sweeps (Ch. 4 tables: serial GaBP takes
# fewer rounds than parallel GaBP on every example)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["grid32", "er", "grid3d"])
def test_serial_converges_to_solution_in_fewer_sweeps(name):
    p = {"grid32": workloads.config1(),
         "er": workloads.er_problem(4096, 8, 21),
         "grid3d": workloads.grid3d_problem(12, 3)}[name]
    s = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=1e-12, return_messages=True)
    q = oracle.broadcast_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=1e-12)
    assert s["converged"] and q["converged"]
    A = oracle.dense_from_csr(p.n, p.row_ptr, p.col, p.val)
    xs = oracle.dense_solve(A, p.b)
    assert np.linalg.norm(s["x"] - xs) <= 1e-9 * np.linalg.norm(xs)
    # the converged messages are a fixed point of the message update
    assert oracle.fixpoint_violation(s["graph"], s["P"], s["mu"], p.b) < 1e-9
    assert s["sweeps"] <= 0.75 * q["sweeps"], (s["sweeps"], q["sweeps"])


def test_serial_stop_rule_and_history():
    p = workloads.config1()
    r = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=1e-10, history=True, check_every=3)
    ts = [t for t, _ in r["history"]]
    assert ts == list(range(3, r["sweeps"] + 1, 3))
    assert r["converged"] and r["history"][-1][1] <= 1e-10 < r["history"][-2][1]
    _, rel = oracle.residual(p.n, p.row_ptr, p.col, p.val, r["x"], p.b)
    assert rel == pytest.approx(r["rel_residual"], rel=1e-12)


def test_serial_prior_round_checked_only_without_sweeps():
    d = np.array([2.0, 4.0, 5.0])
    p = workloads.from_dense(np.diag(d), np.array([1.0, 2.0, 3.0]))
    r = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=1e-10, max_sweeps=0)
    assert r["converged"] and r["sweeps"] == 0
    np.testing.assert_array_equal(r["x"], p.b / d)
    r = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=1e-10, max_sweeps=5, history=True)
    assert r["converged"] and r["sweeps"] == 1 and r["history"][0][0] == 1
