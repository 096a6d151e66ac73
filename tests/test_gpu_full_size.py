"""Full-size workloads in the benchmark's launch configuration (autotuned
handles, default options): checked on properties that hold at any size --
residuals computed independently on the host -- and on sampled outputs the
FP64 oracle can compute one by one."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle
import paper_0811_2518_amd as g
import workloads
from paper_0811_2518_amd import binding

pytestmark = pytest.mark.gpu
DEV = "cuda"


def relres(A, x, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(b - A @ x) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def batch_full():
    return workloads.config3()


def test_full_batch_every_system_converges_and_samples_match_dense(batch_full):
    bt = batch_full
    print(f"batch: {bt.num_sys} systems, {bt.sys_row_off[-1]} rows, {bt.rhs_off[-1]} rhs entries", flush=True)
    s = g.BatchedSolver(bt.sys_row_off, bt.row_ptr, bt.col, bt.val, device=DEV)
    B = torch.from_numpy(bt.B).to(DEV)
    X, infos, st = s.solve(bt.nrhs, bt.rhs_off, B, tol=1e-10, max_iter=100000)
    assert st == binding.OK
    assert all(i["converged"] == 1 and i["rel_residual"] <= 1e-10 for i in infos)
    Xh = X.cpu().numpy()
    del X, B
    s.close()
    # independent FP64 residual of every right-hand side of every system
    worst = 0.0
    for q in range(bt.num_sys):
        p = bt.system(q)
        k = p.b.shape[1]
        A = p.scipy()
        xs = Xh[bt.rhs_off[q]:bt.rhs_off[q + 1]].reshape(p.n, k)
        r = np.linalg.norm(p.b - A @ xs, axis=0) / np.linalg.norm(p.b, axis=0)
        worst = max(worst, float(r.max()))
    assert worst <= 1.05e-10, worst
    # sampled systems small enough for a dense reference
    rng = np.random.default_rng(3)
    small = [q for q in range(bt.num_sys) if bt.sys_row_off[q + 1] - bt.sys_row_off[q] <= 1500]
    for q in rng.choice(small, size=12, replace=False):
        p = bt.system(int(q))
        k = p.b.shape[1]
        xs = Xh[bt.rhs_off[q]:bt.rhs_off[q + 1]].reshape(p.n, k)
        ref = oracle.dense_solve(p.dense(), p.b)
        assert np.linalg.norm(xs - ref) / np.linalg.norm(ref) <= 1e-8, q


def test_full_batch_serial_schedule_converges_with_independent_residuals(batch_full):
    bt = batch_full
    s = g.BatchedSolver(bt.sys_row_off, bt.row_ptr, bt.col, bt.val, device=DEV, layout="serial")
    B = torch.from_numpy(bt.B).to(DEV)
    X, infos, st = s.solve(bt.nrhs, bt.rhs_off, B, tol=1e-10, max_iter=100000)
    assert st == binding.OK
    assert all(i["converged"] == 1 and i["rel_residual"] <= 1e-10 for i in infos)
    Xh = X.cpu().numpy()
    del X, B
    s.close()
    worst = 0.0
    for q in range(bt.num_sys):
        p = bt.system(q)
        k = p.b.shape[1]
        xs = Xh[bt.rhs_off[q]:bt.rhs_off[q + 1]].reshape(p.n, k)
        r = np.linalg.norm(p.b - p.scipy() @ xs, axis=0) / np.linalg.norm(p.b, axis=0)
        worst = max(worst, float(r.max()))
    assert worst <= 1.05e-10, worst


def test_full_grid3d_adjoint_residuals_and_sampled_gradient():
    p = workloads.config4()
    t = p.extra["target"]
    s = g.Solver(p.row_ptr, p.col, p.val, device=DEV)
    x, info = s.solve(torch.from_numpy(p.b).to(DEV), tol=1e-12, max_iter=20000)
    assert info["converged"] == 1
    A = p.scipy()
    xh = x.cpu().numpy()
    assert relres(A, xh, p.b) <= 1.05e-12
    gx = xh - t
    gb, gv, binfo = s.backward(x, x - torch.from_numpy(t).to(DEV), tol=1e-12, max_iter=20000)
    assert binfo["converged"] == 1
    lam = gb.cpu().numpy()
    assert relres(A, lam, gx) <= 1.05e-12
    # the gradient on the pattern: -(lambda_i x_j + lambda_j x_i) off the
    # diagonal, -lambda_i x_i on it, from independently solved x and lambda
    xr, i1 = spla.cg(A, p.b, rtol=1e-14, maxiter=5000)
    lr, i2 = spla.cg(A, xr - t, rtol=1e-14, maxiter=5000)
    assert i1 == 0 and i2 == 0
    rows = np.repeat(np.arange(p.n), np.diff(p.row_ptr))
    ref = np.where(rows == p.col, -lr[rows] * xr[p.col], -(lr[rows] * xr[p.col] + lr[p.col] * xr[rows]))
    gvh = gv.cpu().numpy()
    idx = np.random.default_rng(4).choice(len(p.col), 5000, replace=False)
    np.testing.assert_allclose(gvh[idx], ref[idx], rtol=1e-8, atol=1e-10 * np.abs(ref).max())


@pytest.fixture(scope="module")
def btb_full():
    return workloads.config5()


@pytest.mark.parametrize("mode", ["double_loop_fp32_inner", "single_loop_fp64", "single_loop_fp32_inner"])
def test_full_btb_convergence_fix(btb_full, mode):
    p = btb_full
    if mode == "single_loop_fp64":
        s = g.Solver(p.row_ptr, p.col, p.val, gamma=-1.0, single_loop=True, device=DEV)
    elif mode == "single_loop_fp32_inner":
        s = g.Solver(p.row_ptr, p.col, p.val, precision="fp32", gamma=-1.0, single_loop=True,
                     inner_tol=1e-4, inner_max_iter=20000, device=DEV)
    else:
        s = g.Solver(p.row_ptr, p.col, p.val, precision="fp32", gamma=-1.0, inner_tol=1e-2,
                     inner_max_iter=2000, max_outer=5000, device=DEV)
    pr = s.props()
    assert pr["rho_hi"] > 1.0 and pr["gamma"] > 0.0  # not walk-summable: loading chosen
    x, info = s.solve(torch.from_numpy(p.b).to(DEV), tol=1e-9, max_iter=1000000)
    assert info["converged"] == 1
    assert relres(p.scipy(), x.cpu().numpy(), p.b) <= 1.05e-9


def test_full_btb_through_the_augmented_matrix():
    # the same B^T B + 0.1 I system, posed as [[0.1 I, B^T], [B, -I]] {x, z} = {b, 0}
    # (Ch. 5 Sec. 5.4); both residuals are formed from B on the host, never from B^T B
    import scipy.sparse as sp
    q = workloads.augmented_config()
    print(f"augmented: m {q.m}, n {q.n}, nnz(B) {len(q.val)}", flush=True)
    s = g.AugmentedSolver(q.m, q.n, q.row_ptr, q.col, q.val, q.d, q.gamma, precision="fp32", inner_tol=1e-2,
                          inner_max_iter=2000, max_outer=5000, device=DEV)
    pr = s.props()
    assert pr["n"] == q.n + q.m and pr["num_offdiag"] == 2 * len(q.val)
    assert pr["rho_hi"] > 1.0 and pr["gamma"] > 0.0
    x, info, z = s.solve_blocks(b=torch.from_numpy(q.b).to(DEV), tol=1e-9, max_iter=1000000, z=True)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-9
    B = sp.csr_matrix((q.val, q.col, q.row_ptr), shape=(q.m, q.n))
    xh, zh = x.cpu().numpy(), z.cpu().numpy()
    # the K residual, recomputed: {b - D x - B^T z, -B x + gamma z}
    r1 = q.b - q.d * xh - B.T @ zh
    r2 = -(B @ xh) + q.gamma * zh
    rk = np.sqrt(r1 @ r1 + r2 @ r2) / np.linalg.norm(q.b)
    assert rk <= 1.05e-9
    # the eliminated system (B^T B + 0.1 I) x = b: its residual is r1 - B^T r2 (gamma = 1),
    # so it is at most (1 + ||B||_2) times K's, with ||B||_2 <= sqrt(||B||_1 ||B||_inf)
    r = q.b - B.T @ (B @ xh) - q.d * xh
    aB = abs(B)
    nB = float(np.sqrt(aB.sum(axis=0).max() * aB.sum(axis=1).max()))
    assert np.linalg.norm(r) / np.linalg.norm(q.b) <= (1.0 + nB) * rk * (1 + 1e-9)


@pytest.fixture(scope="module")
def powerlaw_full():
    return workloads.powerlaw_config()


def _rel(x, ref):
    return np.linalg.norm(x - ref) / np.linalg.norm(ref)


def test_full_powerlaw_first_rounds_and_converged_solves(powerlaw_full):
    # the heavy-tailed workload of the bench suite (hub rows up to 140,734
    # slots, swept in chunks), autotuned handles as the bench creates them
    p = powerlaw_full
    A = p.scipy()
    s = g.Solver(p.row_ptr, p.col, p.val, device=DEV, reuse_precision=False)
    print(f"power-law: props {s.props()}", flush=True)
    for T in (1, 3):
        ref = oracle.broadcast_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=T)
        x, info = s.solve(torch.from_numpy(p.b).to(DEV), tol=0, max_iter=T)
        assert _rel(x.cpu().numpy(), ref["x"]) <= 1e-12, T
    for prec in ("fp64", "fp32"):
        s = g.Solver(p.row_ptr, p.col, p.val, precision=prec, device=DEV, reuse_precision=False)
        x, info = s.solve(torch.from_numpy(p.b).to(DEV), tol=1e-10, max_iter=2000)
        assert info["converged"] == 1
        r = relres(A, x.cpu().numpy(), p.b)
        assert r <= 1.05e-10, (prec, r)
        if prec == "fp64":  # the fused check reports the residual of the returned means
            assert info["rel_residual"] == pytest.approx(r, rel=1e-6)
        s.close()


def test_full_powerlaw_serial_first_sweeps_and_converged_solve(powerlaw_full):
    p = powerlaw_full
    s = g.Solver(p.row_ptr, p.col, p.val, device=DEV, layout="serial")
    col, k = s.colours()
    ref_col = oracle.greedy_colouring(p.n, p.row_ptr, p.col)
    np.testing.assert_array_equal(col, ref_col)
    print(f"power-law serial: {k} colour classes", flush=True)
    for T in (1, 2):
        ref = oracle.serial_gabp(p.n, p.row_ptr, p.col, p.val, p.b, colour=ref_col, tol=0, max_sweeps=T)
        x, info = s.solve(torch.from_numpy(p.b).to(DEV), tol=0, max_iter=T)
        assert _rel(x.cpu().numpy(), ref["x"]) <= 1e-12, T
    x, info = s.solve(torch.from_numpy(p.b).to(DEV), tol=1e-10, max_iter=2000)
    assert info["converged"] == 1
    r = relres(p.scipy(), x.cpu().numpy(), p.b)
    assert r <= 1.05e-10
    assert info["rel_residual"] == pytest.approx(r, rel=1e-6)
