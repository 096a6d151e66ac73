"""CPU-side checks of the C ABI library: it loads and exports every declared symbol.

No compute call is made here (no GPU in this environment).
"""
import os
import re

import paper_0811_2518_amd as pkg
from paper_0811_2518_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "gabp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gabp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_bound_entry_points():
    assert _declared() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = pkg.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_opts_match_header_documentation():
    o = pkg.default_opts()
    assert o.precision == binding.FP64 and o.check_every == 1 and o.edges_per_block == 0
    assert o.inner_tol == 1e-5 and o.inner_max_iter == 10000 and o.max_outer == 1000
    assert o.flags == binding.FLAG_REUSE_PRECISION and o.gamma == 0.0 and o.damping == 0.5


def test_struct_layouts():
    import ctypes
    # gabp_opts: 8 int32 then 4 doubles; gabp_info: 4 int32, 3 doubles, 2 int32
    assert ctypes.sizeof(binding.Opts) == 8 * 4 + 4 * 8
    assert ctypes.sizeof(binding.Info) == 4 * 4 + 3 * 8 + 2 * 4
    assert ctypes.sizeof(binding.Props) == 8 + 8 + 6 * 4 + 8 + 3 * 8
    assert ctypes.sizeof(binding.BatchProfile) == 2 * 4 + 3 * 8 + 2 * 8 + 4 * 4 + 8 + 2 * 4 + 8


def test_probe_library_loads_and_exports_its_entry_point():
    # the benchmark's gather-cost probe is a library of its own, outside the ABI above
    import ctypes
    from paper_0811_2518_amd import build
    lib = ctypes.CDLL(build.PROBE_LIB)
    assert hasattr(lib, "gabp_probe_gather16")
    assert hasattr(lib, "gabp_probe_gather16_policy")
