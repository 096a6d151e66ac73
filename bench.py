"""Benchmark: synchronous broadcast GaBP on one MI355X.

Workload: a G(n, 4n) random graph, n = 2^20 (8,388,608 directed message
slots), off-diagonals N(0,1), A_ii = 1.1 sum_j |A_ij|, b ~ N(0,1), solved to a
relative residual of 1e-10.  A step is one full solve from zero messages (all
sweeps, the fused residual checks, the output).  ``value`` is FP64 edge
updates per second (E x sweeps / time); the same line reports the FP32 +
FP64-refinement solve, the roofline of the dominant kernel and the CPU oracle.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import os

# the CPU baseline is the single-threaded oracle: pin BLAS/OpenMP pools first
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import argparse  # noqa: E402
import hashlib  # noqa: E402
import json  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TOL = 1e-10


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sweep_bytes(n, E, elt, check=True, honly=False):
    """Algorithmic HBM bytes of one sweep launch (each array element touched once).

    Joint sweep, per slot: rev 4 + A_ij elt + the gathered reverse message
    record (P, h, sender mean x) 3 elt + the written record 3 elt.  Per node:
    row pointer 4 + A_ii elt + b_i elt + x_i written elt, and with the fused
    check the node's own x of the checked round, elt (the neighbours' x come
    inside the gathered records).  h-only sweep: records (h, x) of 2 elt, the
    frozen coefficient instead of A_ij (plus A_ij when checking) and 1/P~_i.
    """
    if honly:
        slot = 4 + elt + 2 * elt + 2 * elt + (elt if check else 0)
        node = 4 + elt + elt + elt + (2 * elt if check else 0)
    else:
        slot = 4 + elt + 3 * elt + 3 * elt
        node = 4 + elt + elt + elt + (elt if check else 0)
    return slot * E + node * n


def source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_0811_2518_amd", "csrc", "sweep.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_tag):
    """HBM bytes per launch from committed rocprofv3 counter runs, if current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(kernel_tag)
    if not ent or ent.get("sweep_hip_sha") != source_hash():
        return None
    return ent.get("bytes_per_launch")


def run_solves(torch, g, p, b, precision, steps, warmup):
    s = g.Solver(p.row_ptr, p.col, p.val, precision=precision, reuse_precision=False)
    x = torch.empty(p.n, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        s.solve(b, tol=TOL, max_iter=2000, x=x)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    infos = []
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        _, info = s.solve(b, tol=TOL, max_iter=2000, x=x)
        infos.append(info)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    props = s.props()
    xs = x.detach().cpu().numpy()
    s.close()
    return {"wall_s": wall, "event_ms": ev_ms, "infos": infos, "props": props, "x": xs}


def sweep_period(torch, g, p, b, n1=8, n2=40, reps=3):
    """Per-sweep time of the checked FP64 joint sweep: slope between two
    fixed-length runs (tolerance below reach, so every sweep carries the fused
    check and nothing stops early), each timed with events around the whole
    call.  Includes the one-workgroup finish kernel and the dispatch gaps."""
    s = g.Solver(p.row_ptr, p.col, p.val, precision="fp64", reuse_precision=False)
    x = torch.empty(p.n, dtype=torch.float64, device="cuda")
    s.solve(b, tol=1e-300, max_iter=n1, x=x)
    best = {}
    for n_sw in (n1, n2):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.solve(b, tol=1e-300, max_iter=n_sw, x=x)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        best[n_sw] = min(ts)
    s.close()
    return (best[n2] - best[n1]) / (n2 - n1)


def cpu_baseline(p, sweeps):
    import oracle
    g = oracle.edge_graph(p.n, p.row_ptr, p.col, p.val)
    t0 = time.perf_counter()
    oracle.broadcast_gabp(p.n, p.row_ptr, p.col, p.val, p.b, tol=0, max_sweeps=sweeps, graph=g)
    dt = time.perf_counter() - t0
    return p.num_offdiag * sweeps / dt, dt


def probe(torch, g, workloads, args):
    """Launches for rocprofv3 counter runs: a plain copy of known size, then solves."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: 3 x {src.numel() * 8} bytes read and written")
    p = workloads.config2(args.n)
    b = torch.from_numpy(p.b).to("cuda")
    for prec in ("fp64", "fp32"):
        s = g.Solver(p.row_ptr, p.col, p.val, precision=prec, reuse_precision=False)
        for _ in range(args.steps):
            _, info = s.solve(b, tol=TOL, max_iter=2000)
        log(f"{prec}: {info}")
        s.close()
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--cpu-sweeps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", action="store_true",
                    help="profiling probe: a 1 GiB device copy (counter calibration) and a few solves")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of the sweep is a design note, not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_0811_2518_amd as g
    import workloads

    if args.probe:
        probe(torch, g, workloads, args)
        return

    log("generating the G(n,4n) workload")
    p = workloads.config2(args.n)
    n, E = p.n, p.num_offdiag
    b = torch.from_numpy(p.b).to("cuda")

    log("FP64 solves")
    r64 = run_solves(torch, g, p, b, "fp64", args.steps, args.warmup)
    log("FP32 + FP64 refinement solves")
    r32 = run_solves(torch, g, p, b, "fp32", args.steps, args.warmup)
    log("sweep period (fixed-length runs)")
    per_launch_ms = sweep_period(torch, g, p, b)

    i64 = r64["infos"][-1]
    sweeps64 = i64["sweeps"]
    ms_step = r64["event_ms"] / args.steps
    value = E * sweeps64 / (ms_step * 1e-3)
    i32 = r32["infos"][-1]
    ms_step32 = r32["event_ms"] / args.steps

    # roofline of the dominant kernel: the FP64 joint sweep with the fused check
    alg = sweep_bytes(n, E, 8, check=True)
    achieved = alg / (per_launch_ms * 1e-3) / 1e9
    traffic = measured_traffic("k_sweep_fp64_joint_check")

    # errors against the FP64 reference x (the FP64 GPU solve is itself checked
    # against the oracle in the tests; here the two precisions are compared)
    nr = np.linalg.norm(r64["x"])
    err32 = float(np.linalg.norm(r32["x"] - r64["x"]) / nr)
    res64 = float(np.linalg.norm(p.b - p.scipy() @ r64["x"]) / np.linalg.norm(p.b))
    res32 = float(np.linalg.norm(p.b - p.scipy() @ r32["x"]) / np.linalg.norm(p.b))

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline ({args.cpu_sweeps} sweeps)")
        rate, dt = cpu_baseline(p, args.cpu_sweeps)
        cpu = {"value": rate, "unit": "edge-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"{args.cpu_sweeps} sweeps of the FP64 NumPy broadcast oracle on the same "
                         f"n={n} workload ({dt:.1f} s, single thread)"}

    out = {
        "metric": "GaBP edge-updates/s + time-to-1e-10 residual (FP64 vs FP32+refine), % HBM peak",
        "value": value,
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"G(n,4n) random graph, n={n}, E={E} directed slots, "
                               f"A_ii=1.1*sum|A_ij|, b~N(0,1), solve to rel. residual 1e-10",
                   "n": n, "num_offdiag": E, "tol": TOL,
                   "edges_per_block": r64["props"]["edges_per_block"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sweep<double,K,joint> with fused residual check",
                     "alg_bytes_per_launch": alg, "avg_launch_ms": per_launch_ms,
                     "timing": "slope of fixed-length checked runs; includes the finish kernel "
                               "and dispatch gaps of each sweep"},
        "cpu_baseline": cpu,
        "fp64": {"time_to_tol_ms": ms_step, "sweeps": sweeps64, "rel_residual": res64,
                 "wall_ms_per_step": 1e3 * r64["wall_s"] / args.steps},
        "fp32_refine": {"time_to_tol_ms": ms_step32, "inner_sweeps": i32["sweeps"],
                        "outer_iters": i32["outer_iters"], "rel_residual": res32,
                        "rel_err_vs_fp64": err32,
                        "edge_updates_per_s": E * i32["sweeps"] / (ms_step32 * 1e-3),
                        "speedup_vs_fp64": ms_step / ms_step32},
        "kernel_hash": source_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
