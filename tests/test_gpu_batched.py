"""Batched solves (one persistent-kernel graph launch) against per-system references."""
import numpy as np
import pytest
import torch

import oracle
import paper_0811_2518_amd as g
import workloads
from paper_0811_2518_amd import binding

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = 1e-10


@pytest.fixture(scope="module")
def small_batch():
    # uneven sizes, all three topologies, 1..12 right-hand sides (several work
    # items for k > 8)
    return workloads.config3(num_sys=24, nmin=64, nmax=2500, kmax=12, seed=4242)


def _solve(bt, **kw):
    s = g.BatchedSolver(bt.sys_row_off, bt.row_ptr, bt.col, bt.val, device=DEV, **kw)
    B = torch.from_numpy(bt.B).to(DEV)
    X, infos, st = s.solve(bt.nrhs, bt.rhs_off, B, tol=TOL, max_iter=20000)
    return s, B, X, infos, st


def test_batched_matches_per_system_references(small_batch):
    bt = small_batch
    assert max(bt.nrhs) > 8 and min(bt.nrhs) >= 1
    assert set(bt.kinds) == {"grid2d", "grid3d", "er"}
    s, B, X, infos, st = _solve(bt)
    assert st == binding.OK
    Xh = X.cpu().numpy()
    for q in range(bt.num_sys):
        p = bt.system(q)
        info = infos[q]
        assert info["converged"] == 1 and info["rel_residual"] <= TOL, (q, info)
        k = p.b.shape[1]
        xs = Xh[bt.rhs_off[q]:bt.rhs_off[q + 1]].reshape(p.n, k)
        A = p.dense()
        for j in range(k):
            _, rr = oracle.residual(p.n, p.row_ptr, p.col, p.val, xs[:, j], p.b[:, j])
            assert rr <= 1.05 * TOL, (q, j, rr)
            ref = oracle.dense_solve(A, p.b[:, j])
            err = np.linalg.norm(xs[:, j] - ref) / np.linalg.norm(ref)
            assert err <= 1e-8, (q, j, err)


def test_batched_graph_replay_is_deterministic(small_batch):
    bt = small_batch
    s, B, X, infos, st = _solve(bt)
    x1 = X.cpu().numpy().copy()
    X2, infos2, st2 = s.solve(bt.nrhs, bt.rhs_off, B, tol=TOL, max_iter=20000, X=X)
    np.testing.assert_array_equal(X2.cpu().numpy(), x1)
    assert [i["sweeps"] for i in infos2] == [i["sweeps"] for i in infos]


def test_batched_single_system_equals_fp32_solver_accuracy():
    p = workloads.er_problem(3000, 8, 99, ratio=1.1)
    bt_off = np.array([0, p.n], np.int32)
    B = np.random.default_rng(1).standard_normal((p.n, 3))
    s = g.BatchedSolver(bt_off, p.row_ptr, p.col, p.val, device=DEV)
    X, infos, st = s.solve([3], [0, p.n * 3], B.ravel(), tol=TOL, max_iter=20000)
    xs = X.cpu().numpy().reshape(p.n, 3)
    A = p.dense()
    for j in range(3):
        ref = np.linalg.solve(A, B[:, j])
        assert np.linalg.norm(xs[:, j] - ref) / np.linalg.norm(ref) <= 1e-8


def test_batched_rejects_cross_system_entries():
    a = workloads.grid2d_problem(4, 4, 1)
    # two copies of the same 16-node system; then couple row 0 to row 16
    rp = np.concatenate([a.row_ptr, a.row_ptr[1:] + a.row_ptr[-1]]).astype(np.int32)
    col = np.concatenate([a.col, a.col + 16]).astype(np.int32)
    val = np.concatenate([a.val, a.val])
    ok = g.BatchedSolver([0, 16, 32], rp, col, val, device=DEV)
    ok.close()
    col_bad = col.copy()
    assert list(col[:3]) == [0, 1, 4]
    col_bad[2] = 17  # row 0 references a column of the second system (row stays sorted)
    with pytest.raises(binding.GabpError) as e:
        g.BatchedSolver([0, 16, 32], rp, col_bad, val, device=DEV)
    assert e.value.status == binding.E_ARG


def test_batched_rejects_bad_rhs_layout(small_batch):
    bt = small_batch
    s = g.BatchedSolver(bt.sys_row_off, bt.row_ptr, bt.col, bt.val, device=DEV)
    B = torch.from_numpy(bt.B).to(DEV)
    bad = bt.rhs_off.copy()
    bad[1] += 1
    X, infos, st = s.solve(bt.nrhs, bad, B, tol=TOL, check=False)
    assert st == binding.E_ARG


def test_batched_groups_not_dividing_the_workgroup():
    # many small systems with k in {3, 5, 6, 7} right-hand sides: each system's
    # right-hand sides are split into groups of 4, 2 and 1 (a wave's 64 lanes
    # take 64 / kg rows of kg right-hand sides), so every system has items of
    # several group sizes that must cover its right-hand sides exactly once
    rng = np.random.default_rng(11)
    probs, ks = [], []
    for q in range(3000):
        px, py = int(rng.integers(8, 13)), int(rng.integers(8, 13))
        # one dominance ratio for all: equal work weights, so group = k
        probs.append(workloads.grid2d_problem(px, py, 5000 + q, ratio=1.3))
        ks.append(int(rng.choice([3, 5, 6, 7])))
    bt = workloads.batch_of(probs, ks, seed=12)
    s, B, X, infos, st = _solve(bt)
    assert st == binding.OK
    prof = s.profile()
    # groups are powers of two: at least the binary decomposition of each k,
    # at most one item per right-hand side; the precision phase once per system
    popcount = sum(bin(int(k)).count("1") for k in ks)
    assert popcount <= prof["num_items"] <= sum(ks)
    assert prof["precision_items"] == bt.num_sys
    Xh = X.cpu().numpy()
    for q in range(0, bt.num_sys, 7):
        p = bt.system(q)
        k = p.b.shape[1]
        xs = Xh[bt.rhs_off[q]:bt.rhs_off[q + 1]].reshape(p.n, k)
        ref = np.linalg.solve(p.dense(), p.b)
        assert np.linalg.norm(xs - ref) / np.linalg.norm(ref) <= 1e-8, q
    # each outer step's FP32 inner sweeps (to a relative change of 2e-6) gain
    # about five digits
    assert max(i["outer_iters"] for i in infos) <= 6
    assert all(i["converged"] == 1 for i in infos)


# ---------------------------------------------------------------------------
# colour-serial schedule inside each work item (serial scheduling, Ch. 2
# Sec. 2.3): same solutions, fewer sweeps
# ---------------------------------------------------------------------------

def _check_against_dense(bt, X, infos, every=1):
    Xh = X.cpu().numpy()
    for q in range(0, bt.num_sys, every):
        p = bt.system(q)
        info = infos[q]
        assert info["converged"] == 1 and info["rel_residual"] <= TOL, (q, info)
        k = p.b.shape[1]
        xs = Xh[bt.rhs_off[q]:bt.rhs_off[q + 1]].reshape(p.n, k)
        for j in range(k):
            _, rr = oracle.residual(p.n, p.row_ptr, p.col, p.val, xs[:, j], p.b[:, j])
            assert rr <= 1.05 * TOL, (q, j, rr)
        ref = oracle.dense_solve(p.dense(), p.b)
        assert np.linalg.norm(xs - ref) / np.linalg.norm(ref) <= 1e-8, q


def test_batched_serial_matches_per_system_references_in_fewer_sweeps(small_batch):
    bt = small_batch
    s, B, X, infos, st = _solve(bt, layout="serial")
    assert st == binding.OK
    _check_against_dense(bt, X, infos)
    ps = s.profile()
    s0, B0, X0, infos0, st0 = _solve(bt)
    p0 = s0.profile()
    assert ps["inner_sweeps"] < 0.8 * p0["inner_sweeps"], (ps["inner_sweeps"], p0["inner_sweeps"])
    assert ps["precision_sweeps"] < p0["precision_sweeps"]


def test_batched_serial_colours_are_the_oracles(small_batch):
    bt = small_batch
    s = g.BatchedSolver(bt.sys_row_off, bt.row_ptr, bt.col, bt.val, device=DEV, layout="serial")
    col, k = s.colours()
    ref = oracle.greedy_colouring(int(bt.sys_row_off[-1]), bt.row_ptr, bt.col)
    np.testing.assert_array_equal(col, ref)
    assert k == int(ref.max()) + 1


def test_batched_serial_odd_systems_and_replay():
    # long rows (a star larger than a tile's chunk), a tree, isolated nodes,
    # a one-node system and an uneven grid, with 1..9 right-hand sides
    probs = [workloads.star_problem(3000, 1), workloads.random_tree(500, 2),
             workloads.er_problem(700, 2, 3, ratio=1.3), workloads.from_dense(np.array([[3.0]]), np.ones(1)),
             workloads.grid2d_problem(13, 7, 4), workloads.er_problem(2000, 10, 5, ratio=1.05)]
    bt = workloads.batch_of(probs, [3, 9, 1, 2, 5, 8], seed=21)
    s, B, X, infos, st = _solve(bt, layout="serial")
    assert st == binding.OK
    _check_against_dense(bt, X, infos)
    x1 = X.cpu().numpy().copy()
    X2, infos2, st2 = s.solve(bt.nrhs, bt.rhs_off, B, tol=TOL, max_iter=20000, X=X)
    np.testing.assert_array_equal(X2.cpu().numpy(), x1)
    assert [i["sweeps"] for i in infos2] == [i["sweeps"] for i in infos]


@pytest.mark.parametrize("layout", ["auto", "serial"])
def test_batched_powerlaw_systems(layout):
    # heavy-tailed degrees: hub rows longer than a tile's chunk, isolated
    # nodes, and (serial) two to three dozen colour classes per system
    probs = [workloads.powerlaw_problem(n, 8, 300 + i, beta=2.1)
             for i, n in enumerate([3000, 1200, 2500, 400, 1800])]
    bt = workloads.batch_of(probs, [4, 1, 11, 2, 7], seed=31)
    s, B, X, infos, st = _solve(bt, layout=layout)
    assert st == binding.OK
    _check_against_dense(bt, X, infos)
    if layout == "serial":
        col, k = s.colours()
        ref = oracle.greedy_colouring(int(bt.sys_row_off[-1]), bt.row_ptr, bt.col)
        np.testing.assert_array_equal(col, ref)
        assert k >= 20


def test_batched_serial_groups_not_dividing_the_workgroup():
    rng = np.random.default_rng(13)
    probs, ks = [], []
    for q in range(400):
        probs.append(workloads.grid2d_problem(int(rng.integers(8, 13)), int(rng.integers(8, 13)), 7000 + q,
                                              ratio=1.3))
        ks.append(int(rng.choice([3, 5, 6, 7])))
    bt = workloads.batch_of(probs, ks, seed=14)
    s, B, X, infos, st = _solve(bt, layout="serial")
    assert st == binding.OK
    _check_against_dense(bt, X, infos, every=9)


@pytest.mark.parametrize("layout", ["auto", "serial"])
def test_batched_precision_phase_once_per_system(small_batch, layout):
    # the precision update has no b term (Alg. 2): one precision phase per
    # system, whatever the number of right-hand sides and items
    bt = small_batch
    s, B, X, infos, st = _solve(bt, layout=layout)
    assert st == binding.OK
    prof = s.profile()
    assert prof["precision_items"] == bt.num_sys
    assert prof["num_items"] >= bt.num_sys
    assert 3 * bt.num_sys <= prof["precision_sweeps"] <= 10000 * bt.num_sys
    assert prof["precision_ms"] <= prof["makespan_ms"]
    # a second solve reruns the phase from zero messages: identical counts
    X2, infos2, st2 = s.solve(bt.nrhs, bt.rhs_off, B, tol=TOL, max_iter=20000, X=X)
    assert s.profile()["precision_sweeps"] == prof["precision_sweeps"]


def test_batched_rejects_other_layouts(small_batch):
    bt = small_batch
    with pytest.raises(binding.GabpError):
        g.BatchedSolver(bt.sys_row_off, bt.row_ptr, bt.col, bt.val, device=DEV, layout="compact")


@pytest.mark.parametrize("layout", ["auto", "serial"])
def test_batched_degenerate_systems(layout):
    # empty systems, one- and two-node systems and an all-zero right-hand side,
    # between ordinary ones: the empty ones converge at once, a zero right-hand
    # side returns x = 0 exactly, everything else meets the parity bar
    empty = workloads.Problem(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(0))
    probs = [workloads.grid2d_problem(9, 7, 41), empty, workloads.from_dense(np.array([[2.0]]), np.ones(1)),
             workloads.from_dense(np.array([[2.0, -1.0], [-1.0, 3.0]]), np.ones(2)),
             workloads.er_problem(300, 6, 42, ratio=1.2), empty,
             workloads.from_dense(np.array([[0.5]]), np.ones(1))]
    ks = [3, 2, 1, 4, 8, 1, 2]
    bt = workloads.batch_of(probs, ks, seed=43)
    n0 = probs[0].n
    B0 = bt.B[bt.rhs_off[0]:bt.rhs_off[1]].reshape(n0, ks[0])
    B0[:, 1] = 0.0  # one right-hand side of zeros (a view into the batch's B)
    s, B, X, infos, st = _solve(bt, layout=layout)
    assert st == binding.OK
    assert all(i["converged"] == 1 and i["status"] == binding.OK for i in infos)
    Xh = X.cpu().numpy()
    x0 = Xh[bt.rhs_off[0]:bt.rhs_off[1]].reshape(n0, ks[0])
    assert np.all(x0[:, 1] == 0.0)
    for q in range(bt.num_sys):
        p = bt.system(q)
        if p.n == 0:
            continue
        k = p.b.shape[1]
        xs = Xh[bt.rhs_off[q]:bt.rhs_off[q + 1]].reshape(p.n, k)
        ref = oracle.dense_solve(p.dense(), p.b)
        assert np.linalg.norm(xs - ref) <= 1e-8 * max(np.linalg.norm(ref), 1e-300), q


def test_batched_unreachable_tolerance_ends_at_max_iter():
    # every work item stops at the sweep cap and reports it; the launch ends
    bt = workloads.config3(num_sys=16, nmin=64, nmax=1500, kmax=12, seed=4343)
    s = g.BatchedSolver(bt.sys_row_off, bt.row_ptr, bt.col, bt.val, device=DEV)
    B = torch.from_numpy(bt.B).to(DEV)
    X, infos, st = s.solve(bt.nrhs, bt.rhs_off, B, tol=1e-300, max_iter=40, check=False)
    assert st == binding.NOT_CONVERGED
    for i in infos:
        assert i["converged"] == 0 and i["status"] == binding.NOT_CONVERGED
        assert 1 <= i["sweeps"] <= 40, i
    assert torch.isfinite(X).all()
