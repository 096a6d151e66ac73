"""Steffensen's iterations (Ch. 3 Sec. 3.2) on the compact path against the oracle.

The GPU restart writes the extrapolated means into the aggregate records as
{P~_i, P~_i y_i}; the oracle keeps {P~_i, y_i} and forms the same product in
its message update, so the two agree to rounding in each cycle.  Aitken's
step divides by a second difference that can be far smaller than the means,
and under restarts the amplified rounding feeds back: the oracle's own
trajectory moves by up to O(1) after ten cycles when b is perturbed by one
part in 1e15 (measured below, per case and cycle count).  Parity bars:
  * fixed cycle counts: relative 2-norm deviation <= max(1e-10, 100 s), where
    s is the oracle's spread under three perturbations of b at 1e-15; cycle
    counts whose spread exceeds 1e-8 are chaotic and carry no parity claim;
  * converged solves: residual <= tol recomputed independently, x within
    1e-8 of the dense solution and of the oracle's converged x.  The stop
    round itself depends on rounding noise (the oracle's perturbed runs stop
    at other rounds), so it is not compared.
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


def rel(a, b):
    a = a.detach().cpu().numpy() if torch.is_tensor(a) else np.asarray(a)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def cdma(name):
    d = _golden.load(name)
    A = _golden.as_float(_golden.matrix(d))
    return workloads.from_dense(A, np.ones(len(A)))


CASES = {
    "grid32": workloads.config1,
    "poisson10": lambda: workloads.poisson2d(10),
    "er_3001": lambda: workloads.er_problem(3001, 8, 77, ratio=1.1),
    "grid3d_10": lambda: workloads.grid3d_problem(10, 79),
    "cdma_r4": lambda: cdma("cdma_r4.txt"),
    # rows longer than a workgroup (chunked row sums) and isolated nodes
    "powerlaw": lambda: workloads.powerlaw_problem(8000, 8, 90, beta=2.1),
}


def solver(p, **kw):
    return g.Solver(p.row_ptr, p.col, p.val, device=DEV, steffensen=True, **kw)


def spread(p, M, seeds=3):
    """The oracle's own sensitivity: largest relative change of x_M when b moves by 1e-15."""
    ref = oracle.steffensen_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=M)["x"]
    rng = np.random.default_rng(M)
    out = 0.0
    for _ in range(seeds):
        bp = p.b * (1.0 + 1e-15 * rng.standard_normal(p.n))
        x = oracle.steffensen_gabp(p.n, p.row_ptr, p.col, p.val, bp, tol=0, max_sweeps=M)["x"]
        out = max(out, rel(x, ref))
    return ref, out


@pytest.mark.parametrize("name", sorted(CASES))
def test_fixed_cycles_match_oracle(name):
    p = CASES[name]()
    s = solver(p)
    checked = 0
    for M in (2, 3, 4, 6, 10):
        x, info = s.solve(dev(p.b), tol=0, max_iter=M)
        assert info["sweeps"] == M - (M % 2)
        ref, sp = spread(p, M)
        e = rel(x, ref)
        print(f"{name} M={M}: deviation {e:.2e}, oracle spread {sp:.2e}")
        if sp > 1e-8:
            continue
        assert e <= max(1e-10, 100 * sp), (name, M, e, sp)
        checked += 1
    assert checked >= 2  # at least the first two cycles are well conditioned everywhere


@pytest.mark.parametrize("name", ["grid32", "poisson10", "er_3001", "cdma_r4", "powerlaw"])
@pytest.mark.parametrize("check_every", [1, 4])
def test_converged_solve_matches_oracle(name, check_every):
    p = CASES[name]()
    s = solver(p, check_every=check_every)
    ref = oracle.steffensen_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=1e-10, max_sweeps=20000,
                                 check_every=check_every)
    assert ref["converged"]
    x, info = s.solve(dev(p.b), tol=1e-10, max_iter=20000)
    assert info["status"] == binding.OK and info["converged"] == 1
    assert info["sweeps"] % 2 == 0 and info["sweeps"] <= 2 * ref["sweeps"]
    print(f"{name} check_every={check_every}: sweeps {info['sweeps']} (oracle {ref['sweeps']})")
    # the residual reported is that of the returned means, recomputed here in FP64
    _, r = oracle.residual(p.n, p.row_ptr, p.col, p.val, x.cpu().numpy(), p.b)
    assert r <= 1e-10 * (1 + 1e-6)
    assert info["rel_residual"] == pytest.approx(r, rel=1e-6)
    assert rel(x, ref["x"]) <= 1e-8
    if p.n <= 5000:
        xd = oracle.dense_solve(p.dense(), p.b)
        assert rel(x, xd) <= 1e-8


def test_divergence_is_reported_as_in_the_oracle():
    # the non-PSD example of Ch. 4 Sec. 4.2: the plain iteration converges, these cycles do not
    d = _golden.load("nonpsd3.txt")
    p = workloads.from_dense(_golden.as_float(_golden.matrix(d)), _golden.as_float(_golden.vector(d, "b")))
    ref = oracle.steffensen_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=1e-6, max_sweeps=400)
    assert not ref["converged"]
    s = solver(p)
    _, info = s.solve(dev(p.b), tol=1e-6, max_iter=400, check=False)
    assert info["status"] in (binding.E_DIVERGED, binding.NOT_CONVERGED, binding.E_NONFINITE)
    assert info["converged"] == 0


def test_adjoint_through_the_cycles():
    p = workloads.config1()
    s = solver(p)
    x, info = s.solve(dev(p.b), tol=1e-12, max_iter=20000)
    assert info["converged"] == 1
    t = np.random.default_rng(4).standard_normal(p.n)
    gb, gv, binfo = s.backward(x, x - dev(t), tol=1e-12)
    _, lam, gvals = oracle.adjoint_gradient(p.dense(), p.b, t, p.row_ptr, p.col)
    assert binfo["sweeps"] % 2 == 0
    assert rel(gb, lam) <= 1e-9 and rel(gv, gvals) <= 1e-9


def test_options_are_checked():
    p = workloads.config1()
    for kw in ({"aitken": True}, {"precision": "fp32"}, {"layout": "node"}, {"layout": "serial"}):
        st, _ = binding.try_create(p.row_ptr, p.col, p.val, device=DEV, steffensen=True, **kw)
        assert st == binding.E_ARG, kw
    s = solver(p)
    _, info = s.solve(dev(p.b), tol=1e-10, max_iter=1, check=False)
    assert info["status"] == binding.E_ARG
