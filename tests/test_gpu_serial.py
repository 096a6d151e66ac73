"""GPU parity of the colour-serial layout (serial scheduling, Ch. 2 Sec. 2.3).

What is checked against the oracle's serial schedule:
- colouring: bit-exact against the oracle's first-fit colouring;
- means (and variances) after a fixed number of sweeps: relative 2-norm
  error <= 1e-12;
- converged solves: the same sweep count and x within 1e-10.

At the full 2^20-node size:
- the colouring is checked through its defining property;
- the first sweeps are checked against the oracle;
- the converged solution is checked through an independently computed
  residual.
"""
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

CASES = {
    "grid32": workloads.config1,
    "er_ragged": lambda: workloads.er_problem(3001, 8, 77, ratio=1.1),
    "er_sparse_isolated": lambda: workloads.er_problem(4099, 2, 78, ratio=1.3),
    "grid3d_10": lambda: workloads.grid3d_problem(10, 79),
    "tree": lambda: workloads.random_tree(777, 80),
    "star_long_row": lambda: workloads.star_problem(5000, 81),
    # heavy-tailed degrees: rows longer than a workgroup's slot budget (up to
    # 2113 slots) scattered through the row order, and isolated nodes
    "powerlaw": lambda: workloads.powerlaw_problem(8000, 8, 90, beta=2.1),
}


def rel(a, b):
    a = a.detach().cpu().numpy() if torch.is_tensor(a) else np.asarray(a)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def serial(p, **kw):
    return g.Solver(p.row_ptr, p.col, p.val, device=DEV, layout="serial", **kw)


def oracle_serial(p, T, b=None):
    return oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b if b is None else b, tol=0, max_sweeps=T)


def first_fit_property(n, row_ptr, col, colour):
    """No neighbours share a colour, and every colour below colour[i] is
    held by some neighbour j < i (first fit in row order), checked in bulk."""
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    off = rows != col
    r, c = rows[off], np.asarray(col)[off]
    if np.any(colour[r] == colour[c]):
        return False
    low = (c < r) & (colour[c] < colour[r])
    pairs = np.unique(r[low].astype(np.int64) * (int(colour.max()) + 1) + colour[c[low]])
    held = np.bincount((pairs // (int(colour.max()) + 1)).astype(np.int64), minlength=n)
    return bool(np.all(held == colour))


# ---------------------------------------------------------------------------
# colouring and per-sweep parity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", sorted(CASES))
def test_colouring_is_the_oracles_first_fit(name):
    p = CASES[name]()
    s = serial(p)
    col, k = s.colours()
    ref = oracle.greedy_colouring(p.n, p.row_ptr, p.col)
    np.testing.assert_array_equal(col, ref)
    assert k == int(ref.max()) + 1
    assert s.props()["layout"] == 4


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("epb", [512, 2048])
def test_serial_sweep_parity_fixed_sweeps(name, epb):
    p = CASES[name]()
    s = serial(p, edges_per_block=epb)
    for T in (0, 1, 2, 7, 25):
        ref = oracle_serial(p, T)
        x, info, var = s.solve(dev(p.b), tol=0, max_iter=T, var=True)
        assert rel(x, ref["x"]) <= 1e-12, (name, T, rel(x, ref["x"]))
        assert rel(1.0 / var.cpu().numpy(), ref["prec"]) <= 1e-12, (name, T)
        assert info["sweeps"] == T


@pytest.mark.parametrize("name", sorted(CASES))
def test_serial_converged_solve_matches_oracle(name):
    p = CASES[name]()
    s = serial(p)
    ref = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=TOL, max_sweeps=2000)
    x, info = s.solve(dev(p.b), tol=TOL, max_iter=2000)
    assert info["converged"] == 1 and info["status"] == binding.OK
    assert info["sweeps"] == ref["sweeps"]
    assert rel(x, ref["x"]) <= TOL
    assert info["rel_residual"] == pytest.approx(ref["rel_residual"], rel=1e-3)
    if p.n <= 5000:
        assert rel(x, oracle.dense_solve(p.dense(), p.b)) <= 1e-8


def test_serial_check_every_and_fewer_sweeps_than_synchronous():
    p = workloads.config1()
    s = serial(p, check_every=4)
    ref = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=TOL, max_sweeps=2000, check_every=4)
    x, info = s.solve(dev(p.b), tol=TOL, max_iter=2000)
    assert info["sweeps"] == ref["sweeps"] and info["sweeps"] % 4 == 0
    assert rel(x, ref["x"]) <= TOL
    sync = g.Solver(p.row_ptr, p.col, p.val, device=DEV, layout="compact")
    _, si = sync.solve(dev(p.b), tol=TOL, max_iter=2000)
    _, se = serial(p).solve(dev(p.b), tol=TOL, max_iter=2000)
    assert se["sweeps"] < 0.7 * si["sweeps"]


def test_serial_block_size_invariance_and_determinism():
    p = workloads.er_problem(20000, 8, 90)
    xs = []
    for epb in (512, 1024, 2048, 512):
        s = serial(p, edges_per_block=epb)
        x, info = s.solve(dev(p.b), tol=1e-12, max_iter=500)
        xs.append((x.cpu().numpy(), info["sweeps"]))
        s.close()
    for x, sw in xs[1:]:
        assert sw == xs[0][1]
        np.testing.assert_array_equal(x, xs[0][0])


def test_serial_tree_variances_exact():
    p = workloads.random_tree(300, 5)
    x, info, var = serial(p).solve(dev(p.b), tol=1e-14, max_iter=1000, var=True)
    A = p.dense()
    np.testing.assert_allclose(var.cpu().numpy(), np.diag(np.linalg.inv(A)), rtol=1e-11)
    assert rel(x, np.linalg.solve(A, p.b)) <= 1e-11


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_serial_trivial_systems():
    # one class of isolated nodes: sweep 1 is exact and checked by sweep 2
    d = np.array([1.0, -2.0, 4.0, 0.5, 3.0])
    p = workloads.from_dense(np.diag(d), np.arange(5.0))
    s = serial(p)
    assert s.colours()[1] == 1
    x, info = s.solve(dev(p.b), tol=TOL, max_iter=10)
    np.testing.assert_array_equal(x.cpu().numpy(), np.arange(5.0) / d)
    assert info["converged"] == 1 and info["sweeps"] == 1
    # max_iter = 0: the prior, checked as the last allowed sweep
    x, info = s.solve(dev(p.b), tol=TOL, max_iter=0)
    np.testing.assert_array_equal(x.cpu().numpy(), np.arange(5.0) / d)
    assert info["converged"] == 1 and info["sweeps"] == 0
    p = workloads.from_dense(np.array([[4.0]]), np.array([2.0]))
    x, info = serial(p).solve(dev(p.b), tol=TOL, max_iter=10)
    assert x.item() == 0.5 and info["converged"] == 1


def test_serial_empty_system():
    s = g.Solver(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), device=DEV, layout="serial")
    x, info = s.solve(torch.zeros(0, dtype=torch.float64, device=DEV), tol=TOL, max_iter=5)
    assert info["converged"] == 1 and x.numel() == 0
    assert s.colours()[1] == 0


def test_serial_zero_rhs_converges_at_sweep_one():
    p = workloads.config1()
    z = np.zeros(p.n)
    ref = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, z, tol=TOL, max_sweeps=10)
    x, info = serial(p).solve(dev(z), tol=TOL, max_iter=10)
    assert info["converged"] == 1 and info["sweeps"] == ref["sweeps"] == 1
    assert float(x.abs().max()) == 0.0


def test_serial_nan_rhs_is_nonfinite_and_cap_not_converged():
    p = workloads.config1()
    s = serial(p)
    b = p.b.copy()
    b[17] = np.nan
    x, info = s.solve(dev(b), tol=TOL, max_iter=50, check=False)
    assert info["status"] == binding.E_NONFINITE
    x, info = s.solve(dev(p.b), tol=TOL, max_iter=5, check=False)
    assert info["status"] == binding.NOT_CONVERGED and info["sweeps"] == 5
    assert rel(x, oracle_serial(p, 5)["x"]) <= 1e-12


def test_serial_rejections():
    p = workloads.config1()
    st, _ = g.try_create(p.row_ptr, p.col, p.val, device=DEV, layout="serial", single_loop=True, gamma=0.2)
    assert st == binding.E_ARG
    s = serial(p)
    s.solve(dev(p.b), tol=0, max_iter=3)
    with pytest.raises(binding.GabpError):
        s.messages()
    with pytest.raises(binding.GabpError):
        g.Solver(p.row_ptr, p.col, p.val, device=DEV, layout="compact").colours()


# ---------------------------------------------------------------------------
# FP32 messages with FP64 refinement, and the adjoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["grid32", "er_ragged", "grid3d_10", "star_long_row", "powerlaw"])
def test_serial_fp32_refine_reaches_fp64_accuracy(name):
    p = CASES[name]()
    s = serial(p, precision="fp32")
    x, info = s.solve(dev(p.b), tol=TOL, max_iter=5000)
    assert info["converged"] == 1 and info["rel_residual"] <= TOL
    assert info["outer_iters"] >= 1
    _, relr = oracle.residual(p.n, p.row_ptr, p.col, p.val, x.cpu().numpy(), p.b)
    assert relr <= 1.05 * TOL
    xs = (oracle.dense_solve(p.dense(), p.b) if p.n <= 5000 else
          oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=1e-14, max_sweeps=5000)["x"])
    assert rel(x, xs) <= 1e-8


def test_serial_diagonal_loading_double_loop():
    # plain GaBP diverges here; the loaded inner solves run serial sweeps
    p = workloads.config5(n=3000, rows=6000)
    lo, hi = oracle.walk_rho(p.n, p.row_ptr, p.col, p.val, rtol=1e-8, iters=20000)
    gam = oracle.walk_loading(hi, 0.05)
    xd = np.linalg.solve(p.dense(), p.b)
    for prec in ("fp64", "fp32"):
        s = serial(p, precision=prec, gamma=gam, inner_tol=1e-3)
        x, info = s.solve(dev(p.b), tol=1e-9, max_iter=200000)
        assert info["converged"] == 1, info
        assert rel(x, xd) <= 1e-7, (prec, rel(x, xd))


def test_serial_backward_matches_dense_gradient():
    p = workloads.config4(p=8)
    t = p.extra["target"]
    s = serial(p)
    x, info = s.solve(dev(p.b), tol=1e-13, max_iter=5000)
    gb, gv, binfo = s.backward(x, x - dev(t), tol=1e-13, max_iter=5000)
    xr, lam, gvals = oracle.adjoint_gradient(p.dense(), p.b, t, p.row_ptr, p.col)
    assert rel(x, xr) <= TOL
    assert rel(gb, lam) <= TOL
    assert rel(gv, gvals) <= TOL


# ---------------------------------------------------------------------------
# full size: 2^20 nodes, 4n random edges
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def er_full():
    return workloads.config2()


def test_full_er_serial_colouring_and_first_sweeps(er_full):
    p = er_full
    s = serial(p)
    col, k = s.colours()
    assert first_fit_property(p.n, p.row_ptr, p.col, col.astype(np.int64))
    assert k == int(col.max()) + 1
    ref_col = oracle.greedy_colouring(p.n, p.row_ptr, p.col)
    np.testing.assert_array_equal(col, ref_col)
    for T in (1, 3):
        ref = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, colour=ref_col, tol=0, max_sweeps=T)
        x, info = s.solve(dev(p.b), tol=0, max_iter=T)
        assert rel(x, ref["x"]) <= 1e-12, (T, rel(x, ref["x"]))


def test_full_er_serial_converges_with_independent_residual(er_full):
    p = er_full
    A = p.scipy()
    for prec in ("fp64", "fp32"):
        s = serial(p, precision=prec)
        x, info = s.solve(dev(p.b), tol=TOL, max_iter=2000)
        assert info["converged"] == 1
        r = p.b - A @ x.cpu().numpy()
        assert np.linalg.norm(r) / np.linalg.norm(p.b) <= 1.05 * TOL
        s.close()


def test_serial_xcd_parts_change_no_result():
    # the rows of every colour class split by XCD part: same colouring, same
    # iteration, bit for bit
    p = workloads.er_problem(20000, 8, 96)
    s = serial(p, edges_per_block=512)
    s0 = serial(p, edges_per_block=512, natural_order=True)
    assert s.props()["xcd_parts"] == 8 and s0.props()["xcd_parts"] == 0
    np.testing.assert_array_equal(s.colours()[0], s0.colours()[0])
    for T in (0, 1, 2, 9):
        x, _, v = s.solve(dev(p.b), tol=0, max_iter=T, var=True)
        x0, _, v0 = s0.solve(dev(p.b), tol=0, max_iter=T, var=True)
        np.testing.assert_array_equal(x.cpu().numpy(), x0.cpu().numpy())
        np.testing.assert_array_equal(v.cpu().numpy(), v0.cpu().numpy())
    x, i = s.solve(dev(p.b), tol=TOL, max_iter=2000)
    x0, i0 = s0.solve(dev(p.b), tol=TOL, max_iter=2000)
    assert i["sweeps"] == i0["sweeps"]
    np.testing.assert_array_equal(x.cpu().numpy(), x0.cpu().numpy())
    ref = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=TOL, max_sweeps=2000)
    assert i["sweeps"] == ref["sweeps"] and rel(x, ref["x"]) <= TOL


@pytest.mark.parametrize("epb", [512, 1024])
def test_serial_long_rows_report_the_residual_of_x(epb):
    # hub rows swept in chunks: the lag-one residual assembled from the
    # chunks' partial sums is the residual of the returned means, at every
    # stopping sweep, and repeated solves agree bit for bit
    p = CASES["powerlaw"]()
    s = serial(p, edges_per_block=epb)
    b = dev(p.b)
    first = None
    for tol in (1e-6, 1e-8, 1e-10):
        for rep in range(2):
            x, info = s.solve(b, tol=tol, max_iter=2000)
            _, rr = oracle.residual(p.n, p.row_ptr, p.col, p.val, x.cpu().numpy(), p.b)
            assert info["rel_residual"] == pytest.approx(rr, rel=1e-6), (tol, rep, info["rel_residual"], rr)
            if rep == 0:
                first = (x.cpu().numpy().copy(), info["rel_residual"], info["sweeps"])
            else:
                np.testing.assert_array_equal(x.cpu().numpy(), first[0])
                assert (info["rel_residual"], info["sweeps"]) == first[1:]
