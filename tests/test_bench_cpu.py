"""Host logic of the benchmark (CPU only): the byte models and roofline
arithmetic, and the aggregation of rocprofv3 counter runs into per-kernel
traffic figures, on synthetic counter files."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_byte_models(bench):
    n, E = 1 << 20, 8 << 20
    # 48 B per slot and 52 B per node in FP64, 28 and 28 in FP32
    assert bench.alg_sweep_bytes(n, E, 8) == 48 * E + 52 * n
    assert bench.alg_sweep_bytes(n, E, 4) == 28 * E + 28 * n
    assert bench.spmv_bytes(n, E) == 20 * E + 36 * n
    r = bench.tol_roofline(2.0, 10, n, E, 8)
    assert r["floor_ms"] == pytest.approx(10 * (48 * E + 52 * n) / 8e12 * 1e3)
    assert r["frac"] == pytest.approx(r["floor_ms"] / 2.0)
    r = bench.tol_roofline(2.0, 10, n, E, 4, spmvs=2)
    assert r["floor_ms"] == pytest.approx((10 * (28 * E + 28 * n) + 2 * (20 * E + 36 * n)) / 8e12 * 1e3)


def _counter_file(d, name, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size",
                                           "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 0
        for kname, value, grid, dur_us in rows:
            w.writerow({"Kernel_Name": kname, "Counter_Name": name, "Counter_Value": value, "Grid_Size": grid,
                        "Start_Timestamp": t, "End_Timestamp": t + int(dur_us * 1000)})
            t += int(dur_us * 1000) + 1000


def test_traffic_aggregation(bench, tmp_path):
    # the 1 GiB copy reads as half its size and writes its size: fetch counts
    # are scaled by 2, write counts by 1; launches under 20 us are left out;
    # the serial sweep is one period of its class launches, summed
    copy = [("__amd_rocclr_copyBuffer", 524288.0, 512, 400.0)] * 3
    cnode = [("void gabp::k_cnode<double, 2, 0>(gabp::CnodeArgs<double>)", v, 4313088, 160.0)
             for v in (480000.0, 482000.0, 481000.0)] + \
            [("void gabp::k_cnode<double, 2, 0>(gabp::CnodeArgs<double>)", 10.0, 4313088, 3.0)]
    serial = [("void gabp::k_serial<double, 2, false>(gabp::SerialArgs<double>)", v, g, 30.0)
              for _ in range(3) for v, g in ((300000.0, 1000), (100000.0, 500))]
    fetch = copy + cnode + serial
    write = [(k, w, g, d) for (k, _, g, d), w in zip(fetch, [1048576.0] * 3 + [158000.0] * 4 + [80000.0, 40000.0] * 3)]
    _counter_file(tmp_path / "f", "FETCH_SIZE", fetch)
    _counter_file(tmp_path / "w", "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    bench.traffic_from(str(tmp_path / "f"), str(tmp_path / "w"), 1 << 20, out_path=str(out))
    d = json.loads(out.read_text())
    c = d["k_cnode_fp64_joint_k2"]
    assert c["units"] == 3 and c["fetch_scale"] == pytest.approx(2.0) and c["write_scale"] == pytest.approx(1.0)
    assert c["fetch_kib"] == pytest.approx(481000.0) and c["write_kib"] == pytest.approx(158000.0)
    assert c["bytes_per_launch"] == pytest.approx((481000.0 * 2 + 158000.0) * 1024)
    sr = d["k_serial_fp64_k2"]
    assert sr["units"] == 3 and sr["unit"].startswith("sweep (2 class launches)")
    assert sr["bytes_per_launch"] == pytest.approx((400000.0 * 2 + 120000.0) * 1024)
    # an entry is used only while its kernel source is unchanged
    assert c["source_sha"] == bench.source_hash("compact.hip")
