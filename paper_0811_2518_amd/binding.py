"""ctypes binding of libgabp (include/gabp.h): argument marshalling only.

Device memory and streams come from PyTorch; every step of the solve runs in
the library's HIP kernels.  The binding raises if the library is missing or
not built for this machine -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgabp.so")

c_i32, c_i64, c_f64, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p

# gabp_status
OK, NOT_CONVERGED = 0, 1
E_ARG, E_NOT_SYMMETRIC, E_ZERO_DIAG, E_NONFINITE, E_DIVERGED, E_HIP, E_OOM = -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "E_ARG", -2: "E_NOT_SYMMETRIC", -3: "E_ZERO_DIAG",
                -4: "E_NONFINITE", -5: "E_DIVERGED", -6: "E_HIP", -7: "E_OOM"}
FP64, FP32_REFINE = 0, 1
FLAG_REUSE_PRECISION = 1
FLAG_TIME_SWEEPS = 2
FLAG_SINGLE_LOOP = 4
FLAG_NATURAL_ORDER = 8
FLAG_AITKEN = 16
FLAG_MULTI_LAUNCH = 32
FLAG_STEFFENSEN = 64
FLAG_POISON_STALE = 128
FLAG_PREDICT_ALL = 256
LAYOUTS = {"auto": 0, "edge": 1, "node": 2, "compact": 3, "serial": 4}

# every entry point declared in include/gabp.h
EXPORTS = ("gabp_default_opts", "gabp_create", "gabp_solve", "gabp_messages", "gabp_backward",
           "gabp_create_augmented", "gabp_solve_augmented", "gabp_create_batched", "gabp_solve_batched", "gabp_get_batch_profile", "gabp_get_colours",
           "gabp_plan_rows", "gabp_plan_augmented", "gabp_get_props", "gabp_solve_noalloc",
           "gabp_destroy", "gabp_last_error")


class Opts(ctypes.Structure):
    _fields_ = [("precision", c_i32), ("check_every", c_i32), ("edges_per_block", c_i32),
                ("inner_max_iter", c_i32), ("max_outer", c_i32), ("flags", c_i32),
                ("layout", c_i32), ("reserved", c_i32),
                ("gamma", c_f64), ("loading_delta", c_f64), ("inner_tol", c_f64), ("damping", c_f64)]


class Info(ctypes.Structure):
    _fields_ = [("sweeps", c_i32), ("outer_iters", c_i32), ("converged", c_i32), ("status", c_i32),
                ("rel_residual", c_f64), ("gamma", c_f64), ("sweep_ms", c_f64),
                ("timed_sweeps", c_i32), ("sweep_mode", c_i32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Props(ctypes.Structure):
    _fields_ = [("n", c_i64), ("num_offdiag", c_i64), ("edges_per_block", c_i32), ("layout", c_i32),
                ("xcd_parts", c_i32), ("num_blocks", c_i32), ("max_degree", c_i32), ("precision", c_i32),
                ("device_bytes", c_i64), ("rho_lo", c_f64), ("rho_hi", c_f64), ("gamma", c_f64)]


class BatchProfile(ctypes.Structure):
    _fields_ = [("num_items", c_i32), ("workgroups", c_i32), ("makespan_ms", c_f64), ("busy_ms", c_f64),
                ("longest_item_ms", c_f64), ("precision_sweeps", c_i64), ("inner_sweeps", c_i64),
                ("longest_sys", c_i32), ("longest_nrhs", c_i32), ("longest_sweeps", c_i32),
                ("longest_psweeps", c_i32), ("longest_start_ms", c_f64), ("precision_items", c_i32),
                ("pad", c_i32), ("precision_ms", c_f64)]


class GabpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libgabp.so and declare its signatures (raises if not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_0811_2518_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.gabp_default_opts.argtypes = [P(Opts)]
    L.gabp_default_opts.restype = None
    L.gabp_create.argtypes = [c_i32, c_void_p, c_void_p, c_void_p, P(Opts), c_void_p, P(c_void_p)]
    L.gabp_create.restype = c_i32
    L.gabp_solve.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_f64, c_i32, P(Info)]
    L.gabp_solve.restype = c_i32
    L.gabp_messages.argtypes = [c_void_p, c_void_p, c_void_p]
    L.gabp_messages.restype = c_i32
    L.gabp_backward.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_f64, c_i32, P(Info)]
    L.gabp_backward.restype = c_i32
    L.gabp_create_augmented.argtypes = [c_i32, c_i32, c_void_p, c_void_p, c_void_p, c_void_p, c_f64, P(Opts),
                                        c_void_p, P(c_void_p)]
    L.gabp_create_augmented.restype = c_i32
    L.gabp_solve_augmented.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_f64, c_i32, P(Info)]
    L.gabp_solve_augmented.restype = c_i32
    L.gabp_create_batched.argtypes = [c_i32, c_void_p, c_void_p, c_void_p, c_void_p, P(Opts), c_void_p,
                                      P(c_void_p)]
    L.gabp_create_batched.restype = c_i32
    L.gabp_solve_batched.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_f64, c_i32,
                                     c_void_p]
    L.gabp_solve_batched.restype = c_i32
    L.gabp_get_batch_profile.argtypes = [c_void_p, P(BatchProfile)]
    L.gabp_get_batch_profile.restype = c_i32
    L.gabp_get_colours.argtypes = [c_void_p, c_void_p, P(c_i32)]
    L.gabp_get_colours.restype = c_i32
    L.gabp_plan_rows.argtypes = [c_i32, c_void_p, c_void_p, P(Opts), c_void_p, c_void_p, c_void_p, c_i32, c_void_p,
                                 P(Plan)]
    L.gabp_plan_rows.restype = c_i32
    L.gabp_plan_augmented.argtypes = [c_i32, c_i32, c_void_p, c_void_p, c_void_p, c_void_p, c_f64, c_void_p,
                                      c_void_p, c_void_p, c_i64, P(c_i64)]
    L.gabp_plan_augmented.restype = c_i32
    L.gabp_get_props.argtypes = [c_void_p, P(Props)]
    L.gabp_get_props.restype = c_i32
    L.gabp_solve_noalloc.argtypes = [c_i32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_f64, c_i32,
                                     c_void_p, P(Info)]
    L.gabp_solve_noalloc.restype = c_i32
    L.gabp_destroy.argtypes = [c_void_p]
    L.gabp_destroy.restype = None
    L.gabp_last_error.argtypes = [c_void_p]
    L.gabp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


class Plan(ctypes.Structure):
    _fields_ = [("num_colours", c_i32), ("xcd_parts", c_i32), ("num_blocks", c_i32), ("num_chunks", c_i32)]


def plan_rows(row_ptr, col, *, layout="auto", natural_order=False, edges_per_block=0):
    """The row plan gabp_create would make, computed on the host (no GPU):
    dict with perm, colour, blk_row (NumPy int32) and the plan's counts."""
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int32))
    cl = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
    n = len(rp) - 1
    opts = default_opts(layout=LAYOUTS[layout], edges_per_block=edges_per_block,
                        flags=FLAG_REUSE_PRECISION | (FLAG_NATURAL_ORDER if natural_order else 0))
    perm = np.zeros(max(n, 1), np.int32)
    colour = np.zeros(max(n, 1), np.int32)
    cap = 8 * n + 16  # padding at most multiplies the workgroups of a group by 8
    blk = np.zeros(cap, np.int32)
    cls = np.zeros(n + 2, np.int32)
    pl = Plan()
    st = lib().gabp_plan_rows(n, rp.ctypes.data_as(c_void_p), cl.ctypes.data_as(c_void_p), ctypes.byref(opts),
                              perm.ctypes.data_as(c_void_p), colour.ctypes.data_as(c_void_p),
                              blk.ctypes.data_as(c_void_p), cap, cls.ctypes.data_as(c_void_p), ctypes.byref(pl))
    if st != OK:
        raise _err(None, st, "gabp_plan_rows")
    return {"perm": perm[:n], "colour": colour[:n], "blk_row": blk[:pl.num_blocks + 1],
            "class_blk": cls[:pl.num_colours + 1] if pl.num_colours else cls[:0],
            "num_colours": pl.num_colours, "xcd_parts": pl.xcd_parts, "num_blocks": pl.num_blocks,
            "num_chunks": pl.num_chunks}


def plan_augmented(m, n, row_ptr, col, val, d, gamma):
    """The augmented matrix gabp_create_augmented would build, assembled on the host (no GPU):
    (row_ptr, col, val) NumPy arrays of K = [[D, B^T], [B, -gamma I]]."""
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int32))
    cl = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
    vl = np.ascontiguousarray(np.asarray(val, dtype=np.float64))
    dd = np.ascontiguousarray(np.asarray(d, dtype=np.float64))
    nnz = c_i64(0)
    st = lib().gabp_plan_augmented(int(m), int(n), rp.ctypes.data_as(c_void_p), cl.ctypes.data_as(c_void_p),
                                   vl.ctypes.data_as(c_void_p), dd.ctypes.data_as(c_void_p), float(gamma), None,
                                   None, None, 0, ctypes.byref(nnz))
    if st != OK:
        raise _err(None, st, "gabp_plan_augmented")
    Krp = np.zeros(int(m) + int(n) + 1, np.int32)
    Kcl = np.zeros(max(nnz.value, 1), np.int32)
    Kvl = np.zeros(max(nnz.value, 1), np.float64)
    st = lib().gabp_plan_augmented(int(m), int(n), rp.ctypes.data_as(c_void_p), cl.ctypes.data_as(c_void_p),
                                   vl.ctypes.data_as(c_void_p), dd.ctypes.data_as(c_void_p), float(gamma),
                                   Krp.ctypes.data_as(c_void_p), Kcl.ctypes.data_as(c_void_p),
                                   Kvl.ctypes.data_as(c_void_p), int(nnz.value), ctypes.byref(nnz))
    if st != OK:
        raise _err(None, st, "gabp_plan_augmented")
    return Krp, Kcl[:nnz.value], Kvl[:nnz.value]


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().gabp_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _err(handle, status, what):
    msg = lib().gabp_last_error(handle)
    return GabpError(status, f"{what}: {msg.decode() if msg else ''}")


def _torch():
    import torch
    return torch


def _dev(t, dtype, device):
    """Device tensor of the given dtype (copies host arrays; keeps device tensors)."""
    torch = _torch()
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    t = t.to(device=device, dtype=dtype)
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s, ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One symmetric sparse system A (full CSR, diagonal stored) on the GPU."""

    def __init__(self, row_ptr, col, val, *, precision="fp64", check_every=1, edges_per_block=0,
                 gamma=0.0, loading_delta=0.05, inner_tol=1e-5, inner_max_iter=10000, max_outer=1000,
                 reuse_precision=True, time_sweeps=False, layout="auto", single_loop=False, damping=0.5,
                 natural_order=False, aitken=False, steffensen=False, multi_launch=False, poison_stale=False,
                 predict_all=False,
                 device="cuda", stream=None):
        torch = _torch()
        self.device = torch.device(device)
        self.stream, sh = _stream_handle(stream)
        self.row_ptr = _dev(row_ptr, torch.int32, self.device)
        self.col = _dev(col, torch.int32, self.device)
        self.val = _dev(val, torch.float64, self.device)
        self.n = int(self.row_ptr.numel()) - 1
        self.opts = default_opts(
            precision={"fp64": FP64, "fp32": FP32_REFINE, "fp32_refine": FP32_REFINE}[precision],
            check_every=check_every, edges_per_block=edges_per_block, gamma=gamma,
            loading_delta=loading_delta, inner_tol=inner_tol, inner_max_iter=inner_max_iter,
            max_outer=max_outer, layout=LAYOUTS[layout],
            damping=damping,
            flags=(FLAG_REUSE_PRECISION if reuse_precision else 0) | (FLAG_TIME_SWEEPS if time_sweeps else 0)
            | (FLAG_SINGLE_LOOP if single_loop else 0) | (FLAG_NATURAL_ORDER if natural_order else 0)
            | (FLAG_AITKEN if aitken else 0) | (FLAG_STEFFENSEN if steffensen else 0)
            | (FLAG_MULTI_LAUNCH if multi_launch else 0) | (FLAG_POISON_STALE if poison_stale else 0)
            | (FLAG_PREDICT_ALL if predict_all else 0))
        h = ctypes.c_void_p()
        st = lib().gabp_create(self.n, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val),
                               ctypes.byref(self.opts), sh, ctypes.byref(h))
        if st != OK:
            raise _err(None, st, "gabp_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def props(self) -> dict:
        p = Props()
        st = lib().gabp_get_props(self._h, ctypes.byref(p))
        if st != OK:
            raise _err(self._h, st, "gabp_get_props")
        return {f: getattr(p, f) for f, _ in p._fields_}

    def solve(self, b, tol=1e-10, max_iter=2000, *, x=None, var=False, check=True):
        """x = A^-1 b.  Returns (x, info dict[, var])."""
        torch = _torch()
        b = _dev(b, torch.float64, self.device)
        x = torch.empty(self.n, dtype=torch.float64, device=self.device) if x is None else x
        v = torch.empty(self.n, dtype=torch.float64, device=self.device) if var else None
        info = Info()
        st = lib().gabp_solve(self._h, _ptr(b), _ptr(x), _ptr(v), float(tol), int(max_iter),
                              ctypes.byref(info))
        if check and st < 0:
            raise _err(self._h, st, "gabp_solve")
        d = info.as_dict()
        d["status"] = st
        return (x, d, v) if var else (x, d)

    def colours(self):
        """(colour of each row as a NumPy int32 array, number of classes); layout "serial" only."""
        import numpy as np
        col = np.zeros(max(self.n, 1), dtype=np.int32)
        k = c_i32(0)
        st = lib().gabp_get_colours(self._h, col.ctypes.data_as(c_void_p), ctypes.byref(k))
        if st != OK:
            raise _err(self._h, st, "gabp_get_colours")
        return col[: self.n], int(k.value)

    def messages(self):
        """(P, h) of the last fixed-sweep FP64 solve, slot order of the off-diagonal CSR."""
        torch = _torch()
        E = self.props()["num_offdiag"]
        P = torch.empty(E, dtype=torch.float64, device=self.device)
        hm = torch.empty(E, dtype=torch.float64, device=self.device)
        st = lib().gabp_messages(self._h, _ptr(P), _ptr(hm))
        if st != OK:
            raise _err(self._h, st, "gabp_messages")
        return P, hm

    def backward(self, x, grad_x, tol=1e-12, max_iter=5000, grad_vals=True, check=True):
        torch = _torch()
        x = _dev(x, torch.float64, self.device)
        gx = _dev(grad_x, torch.float64, self.device)
        gb = torch.empty(self.n, dtype=torch.float64, device=self.device)
        gv = torch.empty(self.val.numel(), dtype=torch.float64, device=self.device) if grad_vals else None
        info = Info()
        st = lib().gabp_backward(self._h, _ptr(x), _ptr(gx), _ptr(gb), _ptr(gv), float(tol), int(max_iter),
                                 ctypes.byref(info))
        if check and st < 0:
            raise _err(self._h, st, "gabp_backward")
        d = info.as_dict()
        d["status"] = st
        return gb, gv, d

    def close(self):
        if getattr(self, "_h", None):
            lib().gabp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AugmentedSolver(Solver):
    """A rectangular B (m x n) through the symmetric matrix [[D, B^T], [B, -gamma I]] (Ch. 5 Sec. 5.4).

    ``solve`` and ``backward`` of the base class act on the whole system of
    n + m unknowns; ``solve_blocks`` takes the right-hand side {b, h} in its
    two blocks and returns x (and z).  ``loading`` is the diagonal loading of
    the double loop (< 0: picked from rho(|R|)); the system is indefinite, so
    the plain iteration (loading 0) does not converge on it.
    """

    def __init__(self, m, n, row_ptr, col, val, d, gamma, *, loading=-1.0, precision="fp64", check_every=1,
                 edges_per_block=0, loading_delta=0.05, inner_tol=1e-5, inner_max_iter=10000, max_outer=1000,
                 layout="auto", single_loop=False, damping=0.5, natural_order=False, device="cuda",
                 stream=None):
        torch = _torch()
        self.device = torch.device(device)
        self.stream, sh = _stream_handle(stream)
        self.m_rows, self.n_cols = int(m), int(n)
        B_rp = _dev(row_ptr, torch.int32, self.device)
        B_col = _dev(col, torch.int32, self.device)
        B_val = _dev(val, torch.float64, self.device)
        dd = _dev(d, torch.float64, self.device)
        self.opts = default_opts(
            precision={"fp64": FP64, "fp32": FP32_REFINE, "fp32_refine": FP32_REFINE}[precision],
            check_every=check_every, edges_per_block=edges_per_block, gamma=loading,
            loading_delta=loading_delta, inner_tol=inner_tol, inner_max_iter=inner_max_iter,
            max_outer=max_outer, layout=LAYOUTS[layout], damping=damping,
            flags=(FLAG_SINGLE_LOOP if single_loop else 0) | (FLAG_NATURAL_ORDER if natural_order else 0))
        h = ctypes.c_void_p()
        st = lib().gabp_create_augmented(self.m_rows, self.n_cols, _ptr(B_rp), _ptr(B_col), _ptr(B_val), _ptr(dd),
                                         float(gamma), ctypes.byref(self.opts), sh, ctypes.byref(h))
        if st != OK:
            raise _err(None, st, "gabp_create_augmented")
        self._h = h
        self.n = self.n_cols + self.m_rows

    def backward(self, x, grad_x, tol=1e-12, max_iter=5000, grad_vals=False, check=True):
        """Adjoint solve on the whole system; the gradient on K's entries is not offered (K is internal)."""
        if grad_vals:
            raise ValueError("grad_vals needs the caller's CSR; an augmented handle assembles its own")
        return super().backward(x, grad_x, tol, max_iter, grad_vals=False, check=check)

    def solve_blocks(self, b=None, h=None, tol=1e-9, max_iter=100000, *, x=None, z=False, check=True):
        """x (and z) of [[D, B^T], [B, -gamma I]] {x, z} = {b, h}.  Returns (x, info[, z])."""
        torch = _torch()
        bb = None if b is None else _dev(b, torch.float64, self.device)
        hh = None if h is None else _dev(h, torch.float64, self.device)
        x = torch.empty(self.n_cols, dtype=torch.float64, device=self.device) if x is None else x
        zz = torch.empty(self.m_rows, dtype=torch.float64, device=self.device) if z else None
        info = Info()
        st = lib().gabp_solve_augmented(self._h, _ptr(bb), _ptr(hh), _ptr(x), _ptr(zz), float(tol), int(max_iter),
                                        ctypes.byref(info))
        if check and st < 0:
            raise _err(self._h, st, "gabp_solve_augmented")
        d = info.as_dict()
        d["status"] = st
        return (x, d, zz) if z else (x, d)


def solve_noalloc(row_ptr, col, val, b, tol=1e-10, max_iter=2000, *, x=None, var=False, device="cuda",
                  stream=None, check=True):
    """gabp_solve_noalloc: one plain FP64 solve of a small system (n <= 1024, at most 4096
    off-diagonal entries) that allocates nothing on the device.  Returns (x, info[, var])."""
    torch = _torch()
    dv = torch.device(device)
    _, sh = _stream_handle(stream)
    rp = _dev(row_ptr, torch.int32, dv)
    cl = _dev(col, torch.int32, dv)
    vl = _dev(val, torch.float64, dv)
    bb = _dev(b, torch.float64, dv)
    n = int(rp.numel()) - 1
    x = torch.empty(n, dtype=torch.float64, device=dv) if x is None else x
    v = torch.empty(n, dtype=torch.float64, device=dv) if var else None
    info = Info()
    st = lib().gabp_solve_noalloc(n, _ptr(rp), _ptr(cl), _ptr(vl), _ptr(bb), _ptr(x), _ptr(v), float(tol),
                                  int(max_iter), sh, ctypes.byref(info))
    if check and st < 0:
        raise _err(None, st, "gabp_solve_noalloc")
    d = info.as_dict()
    d["status"] = st
    return (x, d, v) if var else (x, d)


def last_create_error() -> str:
    m = lib().gabp_last_error(None)
    return m.decode() if m else ""


def try_create(row_ptr, col, val, **kw):
    """Create and return (status, Solver or None) without raising on a gabp error."""
    try:
        return OK, Solver(row_ptr, col, val, **kw)
    except GabpError as e:
        return e.status, None


class BatchedSolver:
    """Many independent systems (block-diagonal CSR with global columns)."""

    # inner_tol: an outer step's FP32 sweeps stop once the largest change of
    # the correction is at most inner_tol times its largest magnitude
    def __init__(self, sys_row_off, row_ptr, col, val, *, inner_tol=2e-6, check_every=1,
                 inner_max_iter=10000, max_outer=1000, layout="auto", device="cuda", stream=None):
        torch = _torch()
        self.device = torch.device(device)
        self.stream, sh = _stream_handle(stream)
        self.sys_row_off = np.ascontiguousarray(np.asarray(sys_row_off, dtype=np.int32))
        self.row_ptr = _dev(row_ptr, torch.int32, self.device)
        self.col = _dev(col, torch.int32, self.device)
        self.val = _dev(val, torch.float64, self.device)
        self.num_sys = len(self.sys_row_off) - 1
        self.opts = default_opts(precision=FP32_REFINE, inner_tol=inner_tol, check_every=check_every,
                                 inner_max_iter=inner_max_iter, max_outer=max_outer, layout=LAYOUTS[layout])
        h = ctypes.c_void_p()
        st = lib().gabp_create_batched(self.num_sys, self.sys_row_off.ctypes.data_as(c_void_p),
                                       _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val),
                                       ctypes.byref(self.opts), sh, ctypes.byref(h))
        if st != OK:
            raise _err(None, st, "gabp_create_batched")
        self._h = h

    def colours(self):
        """(colour of each global row, number of classes of the largest system); layout "serial" only."""
        n = int(self.sys_row_off[-1])
        col = np.zeros(max(n, 1), dtype=np.int32)
        k = c_i32(0)
        st = lib().gabp_get_colours(self._h, col.ctypes.data_as(c_void_p), ctypes.byref(k))
        if st != OK:
            raise _err(self._h, st, "gabp_get_colours")
        return col[:n], int(k.value)

    def solve(self, nrhs, rhs_off, B, tol=1e-10, max_iter=100000, X=None, check=True):
        torch = _torch()
        nrhs = np.ascontiguousarray(np.asarray(nrhs, dtype=np.int32))
        rhs_off = np.ascontiguousarray(np.asarray(rhs_off, dtype=np.int64))
        B = _dev(B, torch.float64, self.device)
        X = torch.empty_like(B) if X is None else X
        infos = (Info * self.num_sys)()
        st = lib().gabp_solve_batched(self._h, nrhs.ctypes.data_as(c_void_p), rhs_off.ctypes.data_as(c_void_p),
                                      _ptr(B), _ptr(X), float(tol), int(max_iter),
                                      ctypes.cast(infos, c_void_p))
        if check and st < 0:
            raise _err(self._h, st, "gabp_solve_batched")
        return X, [i.as_dict() for i in infos], st

    def profile(self) -> dict:
        pf = BatchProfile()
        st = lib().gabp_get_batch_profile(self._h, ctypes.byref(pf))
        if st != OK:
            raise _err(self._h, st, "gabp_get_batch_profile")
        return {f: getattr(pf, f) for f, _ in pf._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().gabp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
