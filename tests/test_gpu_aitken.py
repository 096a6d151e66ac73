"""GPU parity of Aitken's extrapolation of the means (Ch. 3 Sec. 3.2) against the oracle.

The sweeps are those of Alg. 2; after sweep t the solver returns, node by
node, y_t = x_{t-2} - (x_{t-1} - x_{t-2})^2 / (x_t - 2 x_{t-1} + x_{t-2}).

Bar: status codes bit-exact; y node by node within the perturbation bound of
the step.  The means of the HIP sweeps differ from the oracle's by rounding
(held to the 1e-10 bar of the plain solve, and measured here per node as e_i
on a plain handle of the same configuration, which runs the same sweeps).
With d1 = x_{t-1} - x_{t-2} and den = x_t - 2 x_{t-1} + x_{t-2} from the
oracle, |d(d1)| <= 2e and |d(den)| <= 4e, so while 4e < |den|
  |dy| <= e + (4e|d1| + 4e^2) / (|den| - 4e) + 4e d1^2 / (|den| (|den| - 4e)),
plus the rounding of the step on each side; nodes with 4e >= |den| (the step
is undecidable there) are left out.  The sweep count of a converged solve is
a decision on the residual of y: it must equal the oracle's unless the
oracle's residual lies within the slack || |A| bound ||_2 / ||b||_2 of tol on
the rounds in between.
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
U = np.finfo(float).eps / 2


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).to(DEV)


def solver(p, **kw):
    return g.Solver(p.row_ptr, p.col, p.val, device=DEV, aitken=True, **kw)


def oracle_means(p, t):
    return [oracle.broadcast_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=k)["x"]
            for k in (t - 2, t - 1, t)]


class Means:
    """The oracle's means of rounds t-2, t-1, t and their per-node deviation on the GPU."""

    def __init__(self, p, t, plain):
        self.xs = oracle_means(p, t)
        gx = [plain.solve(dev(p.b), tol=0, max_iter=k)[0].cpu().numpy() for k in (t - 2, t - 1, t)]
        self.gx = gx  # the GPU's own means of the three rounds
        scale = max(float(np.max(np.abs(np.concatenate(self.xs)))), 1e-300)
        dev_max = max(float(np.max(np.abs(a - b))) for a, b in zip(gx, self.xs))
        assert dev_max <= 1e-10 * scale, dev_max / scale   # the plain solve's bar
        self.e = np.max([np.abs(a - b) for a, b in zip(gx, self.xs)], axis=0)

    def bound(self):
        x0, x1, x2 = self.xs
        e = self.e
        ref = oracle.aitken_extrapolate(x0, x1, x2)
        d1 = np.abs(x1 - x0)
        den = np.abs(x2 - 2.0 * x1 + x0)
        gap = den - 4.0 * e
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            corr = d1 * d1 / den
            b = e + (4 * e * d1 + 4 * e * e) / gap + 4 * e * d1 * d1 / (den * gap)
            # rounding of the step itself, on both sides
            b = b + 16 * U * (np.abs(x0) + 2 * np.abs(x1) + np.abs(x2) + corr * (1 + 8 * d1 / np.maximum(gap, 0)))
        b = np.where((gap > 0) & np.isfinite(b) & np.isfinite(ref), b, np.inf)
        # a mean that no longer moves on either side (an isolated node, or one
        # converged to the last bit): both keep it
        still = (d1 == 0) & (den == 0) & (e == 0)
        b[still] = 0.0
        return ref, b


def check_y(y, m):
    """y (device) against the oracle's Aitken step, within the bound of Means m, on the nodes
    whose bound is finite; on every node, y must be the step applied to the GPU's own means
    of the same rounds (the plain twin runs the same sweeps bit for bit), which also covers
    the nodes whose second difference is too close to rounding for the oracle comparison."""
    y = y.cpu().numpy()
    ref, bound = m.bound()
    fin = np.isfinite(bound)
    print(f"decidable nodes: {fin.mean():.4f}")
    assert fin.mean() >= 0.5, fin.mean()   # the cases below keep most nodes decidable
    err = np.abs(y[fin] - ref[fin])
    assert np.all(err <= bound[fin]), (float(np.max(err - bound[fin])), int(np.argmax(err - bound[fin])))
    assert np.all(np.isfinite(y))
    own = oracle.aitken_extrapolate(*m.gx)
    scale = np.abs(own) + np.abs(m.gx[2])
    assert np.all(np.abs(y - own) <= 4 * U * scale), float(np.max(np.abs(y - own) / np.maximum(scale, 1e-300)))


def oracle_rel_and_slack(p, m):
    """Relative residual of the oracle's y_t and the most the HIP path's may differ from it:
    | ||b - A y'|| - ||b - A y|| | <= || |A| |y' - y| || <= || |A| bound ||."""
    ref, bound = m.bound()
    _, rel = oracle.residual(p.n, p.row_ptr, p.col, p.val, ref, p.b)
    rows = np.repeat(np.arange(p.n), np.diff(p.row_ptr))
    with np.errstate(invalid="ignore"):
        ab = np.bincount(rows, weights=np.abs(p.val) * bound[p.col], minlength=p.n)
    return rel, float(np.linalg.norm(ab) / np.linalg.norm(p.b))


def plain_twin(p, **kw):
    """A plain handle that runs the same sweeps as the Aitken handle solver(p, **kw)."""
    return g.Solver(p.row_ptr, p.col, p.val, device=DEV, layout="compact", reuse_precision=False,
                    **{k: v for k, v in kw.items() if k != "check_every"})


CASES = {
    "grid": lambda: workloads.grid2d_problem(40, 37, seed=11),
    "er": lambda: workloads.er_problem(6000, 8, 12),
    "poisson": lambda: workloads.poisson2d(30),
    "powerlaw": lambda: workloads.powerlaw_problem(8000, 8, 90, beta=2.1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_fixed_rounds_match_oracle(case):
    p = CASES[case]()
    s = solver(p, edges_per_block=512)
    plain = plain_twin(p, edges_per_block=512)
    assert s.props()["layout"] == binding.LAYOUTS["compact"]
    for M in (2, 3, 9, 16):
        y, info = s.solve(dev(p.b), tol=0, max_iter=M)
        assert info["sweeps"] == M and info["status"] == binding.OK
        check_y(y, Means(p, M, plain))
        r = oracle.aitken_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=M)
        assert np.isfinite(r["y"]).all()


@pytest.mark.parametrize("case,tol,check_every", [
    ("poisson10", 1e-10, 1), ("poisson10", 1e-6, 1), ("poisson32", 1e-6, 1), ("grid", 1e-10, 1),
    ("grid", 1e-10, 4), ("er", 1e-10, 1), ("powerlaw", 1e-10, 1)])
def test_converged_sweeps_and_estimate_match_oracle(case, tol, check_every):
    p = {"poisson10": lambda: workloads.poisson2d(10), "poisson32": lambda: workloads.poisson2d(32),
         **CASES}[case]()
    s = solver(p, edges_per_block=512, check_every=check_every)
    plain = plain_twin(p, edges_per_block=512)
    y, info = s.solve(dev(p.b), tol=tol, max_iter=20000)
    ref = oracle.aitken_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=tol, max_sweeps=20000,
                             check_every=check_every)
    assert ref["converged"]
    assert info["converged"] == 1 and info["status"] == binding.OK
    tg, to = info["sweeps"], ref["sweeps"]
    assert tg % check_every == 0
    # the stop is a floating-point decision on y, whose rounding the step
    # amplifies: where the counts differ, the oracle's residual on the rounds
    # between them must lie within the rounding slack of tol
    if tg > to:
        for t in range(to, tg, check_every):
            rel_o, slack = oracle_rel_and_slack(p, Means(p, t, plain))
            assert rel_o >= tol - slack, (tg, to, t, rel_o, slack)
    elif tg < to:
        rel_o, slack = oracle_rel_and_slack(p, Means(p, tg, plain))
        assert rel_o <= tol + slack, (tg, to, rel_o, slack)
    # the HIP path's own decision: its estimates of the earlier checked rounds
    # (recomputed by fixed-sweep solves) missed tol
    for t in range(max(2, min(tg, to) - check_every), tg, check_every):
        yt, _ = s.solve(dev(p.b), tol=0, max_iter=t)
        _, rt = oracle.residual(p.n, p.row_ptr, p.col, p.val, yt.cpu().numpy(), p.b)
        assert rt > tol * (1 - 1e-9), (t, rt)
    check_y(y, Means(p, tg, plain))
    # the reported residual is that of the returned estimate (the oracle's own
    # residual is not compared directly: the step amplifies the rounding of
    # the means by up to (1 + 2|r|)^2, which check_y already bounds node by node)
    _, rr = oracle.residual(p.n, p.row_ptr, p.col, p.val, y.cpu().numpy(), p.b)
    assert info["rel_residual"] == pytest.approx(rr, rel=1e-6)
    assert rr <= tol


def test_poisson_needs_fewer_sweeps_than_plain():
    # Ch. 4 Sec. 4.3: the extrapolated estimate reaches the tolerance in a
    # fraction of the plain rounds on the 2-D Poisson example
    p = workloads.poisson2d(10)
    _, ia = solver(p).solve(dev(p.b), tol=1e-10, max_iter=5000)
    _, ip = g.Solver(p.row_ptr, p.col, p.val, device=DEV).solve(dev(p.b), tol=1e-10, max_iter=5000)
    assert 2 * ia["sweeps"] <= ip["sweeps"]


def test_not_converged_returns_last_estimate():
    p = workloads.poisson2d(32)
    s = solver(p)
    y, info = s.solve(dev(p.b), tol=1e-14, max_iter=40)
    assert info["status"] == binding.NOT_CONVERGED and info["converged"] == 0 and info["sweeps"] == 40
    check_y(y, Means(p, 40, plain_twin(p)))
    _, rr = oracle.residual(p.n, p.row_ptr, p.col, p.val, y.cpu().numpy(), p.b)
    assert info["rel_residual"] == pytest.approx(rr, rel=1e-6)


def test_variances_are_those_of_the_last_sweep():
    p = workloads.grid2d_problem(20, 20, seed=3)
    s = solver(p)
    y, info, v = s.solve(dev(p.b), tol=1e-10, max_iter=2000, var=True)
    t = info["sweeps"]
    r = oracle.broadcast_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=t)
    np.testing.assert_allclose(v.cpu().numpy(), 1.0 / r["prec"], rtol=1e-12)


def test_xcd_order_changes_no_result():
    p = workloads.er_problem(20000, 8, 93)
    s = solver(p, edges_per_block=512)
    s0 = solver(p, edges_per_block=512, natural_order=True)
    assert s.props()["xcd_parts"] == 8 and s0.props()["xcd_parts"] == 0
    for M in (2, 7):
        y, _ = s.solve(dev(p.b), tol=0, max_iter=M)
        y0, _ = s0.solve(dev(p.b), tol=0, max_iter=M)
        np.testing.assert_array_equal(y.cpu().numpy(), y0.cpu().numpy())
    y, i = s.solve(dev(p.b), tol=1e-10, max_iter=2000)
    y0, i0 = s0.solve(dev(p.b), tol=1e-10, max_iter=2000)
    assert i["sweeps"] == i0["sweeps"]
    np.testing.assert_array_equal(y.cpu().numpy(), y0.cpu().numpy())


def test_adjoint_matches_dense_gradient():
    p = workloads.grid2d_problem(16, 15, seed=21)
    A = p.dense()
    s = solver(p)
    y, info = s.solve(dev(p.b), tol=1e-12, max_iter=5000)
    assert info["converged"] == 1
    t = np.random.default_rng(4).normal(size=p.n)
    gx = y.cpu().numpy() - t
    gb, gv, bi = s.backward(y, dev(gx), tol=1e-12)
    assert bi["converged"] == 1
    lam = np.linalg.solve(A, gx)
    np.testing.assert_allclose(gb.cpu().numpy(), lam, rtol=0, atol=1e-9 * np.abs(lam).max())


def test_repeated_solves_agree_bit_for_bit():
    p = CASES["er"]()
    s = solver(p)
    b = dev(p.b)
    y1, i1 = s.solve(b, tol=1e-10, max_iter=2000)
    y1 = y1.cpu().numpy().copy()
    y2, i2 = s.solve(b, tol=1e-10, max_iter=2000)
    np.testing.assert_array_equal(y2.cpu().numpy(), y1)
    assert (i1["sweeps"], i1["rel_residual"]) == (i2["sweeps"], i2["rel_residual"])


@pytest.mark.parametrize("kw", [dict(precision="fp32"), dict(layout="serial"), dict(layout="edge"),
                                dict(gamma=0.5), dict(single_loop=True, gamma=0.5)])
def test_unsupported_combinations_are_rejected(kw):
    p = workloads.grid2d_problem(8, 8, seed=1)
    st, s = binding.try_create(p.row_ptr, p.col, p.val, device=DEV, aitken=True, **kw)
    assert st == binding.E_ARG and s is None
    assert "Aitken" in binding.last_create_error()


def test_fewer_than_three_rounds_is_an_argument_error():
    p = workloads.grid2d_problem(8, 8, seed=1)
    s = solver(p)
    for M in (0, 1):
        _, info = s.solve(dev(p.b), tol=0, max_iter=M, check=False)
        assert info["status"] == binding.E_ARG


def test_sweep_timing_covers_every_sweep():
    p = workloads.grid2d_problem(30, 30, seed=2)
    s = solver(p, time_sweeps=True)
    _, info = s.solve(dev(p.b), tol=1e-10, max_iter=2000)
    # every queued sweep is timed, including those that return at once past convergence
    assert info["timed_sweeps"] >= info["sweeps"] and info["sweep_ms"] > 0


@pytest.mark.parametrize("variant", ["aitken", "single_loop"])
def test_autotune_cache_keeps_the_compact_layout(tmp_path, monkeypatch, variant):
    # a plain handle tunes over every layout and caches its choice; handles that
    # need the compact layout are keyed by that request and never take another
    monkeypatch.setenv("GABP_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    p = workloads.er_problem(65536, 8, 31)
    assert p.num_offdiag >= 200000                  # large enough to be timed at create
    g.Solver(p.row_ptr, p.col, p.val, device=DEV).close()
    kw = dict(aitken=True) if variant == "aitken" else dict(single_loop=True, gamma=-1.0)
    for _ in range(2):                               # timed, then from the cache
        s = g.Solver(p.row_ptr, p.col, p.val, device=DEV, **kw)
        assert s.props()["layout"] == binding.LAYOUTS["compact"]
        _, info = s.solve(dev(p.b), tol=1e-10, max_iter=2000)
        assert info["status"] == binding.OK
        s.close()
    assert "L3" in (tmp_path / "tune.txt").read_text()
