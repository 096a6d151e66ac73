"""Seeded synthetic inputs for the GaBP solver and for its CPU oracle.

This module builds problem instances only: symmetric sparse matrices in CSR
form (int32 row pointers and columns, float64 values, diagonal included),
right-hand sides and targets.  It contains none of the solver's arithmetic, so
both the HIP path and the oracle can draw their inputs from it.

Shapes follow the workloads the thesis studies (Bickson, "Gaussian Belief
Propagation: Theory and Application"): 2-D grids such as the Poisson example
(Ch. 4, Sec. "2-D Poisson's Equation"), sparse random graphs of about a
million nodes and ten million edges standing in for the rating graphs of
Ch. 6, and normal-equation matrices B^T B like the least-squares setting of
Ch. 5 (Sec. "Extension to General Linear Systems").  None of the paper's data
sets is reproduced; every input here is drawn from a seeded generator.

Recipe shared by every generator:
  * undirected edges are the sorted pairs (u < v) in lexicographic order, the
    off-diagonal value of each pair is drawn in that order and mirrored;
  * the diagonal is ``ratio * sum_j |A_ij|`` (1.0 for a node with no edge);
  * right-hand sides are drawn after the matrix.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np
import scipy.sparse as sp

SEED_BASE = 2518


@dataclasses.dataclass
class Problem:
    """One symmetric system A x = b in full CSR form (diagonal included)."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 [nnz]
    b: np.ndarray        # float64 [n] (or [n, k] row-major for several RHS)
    name: str = ""
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def num_offdiag(self) -> int:
        return self.nnz - self.n

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.scipy().toarray()


@dataclasses.dataclass
class Batch:
    """Block-diagonal concatenation of independent systems, several RHS each.

    ``row_ptr``/``col``/``val`` describe the whole block-diagonal matrix with
    global column indices; system ``s`` owns rows ``sys_row_off[s]:sys_row_off[s+1]``.
    Its right-hand sides are the row-major block ``B[rhs_off[s]:rhs_off[s+1]]``
    viewed as ``[n_s, nrhs[s]]``.
    """

    sys_row_off: np.ndarray  # int32 [S+1]
    row_ptr: np.ndarray      # int32 [N+1]
    col: np.ndarray          # int32 [nnz]
    val: np.ndarray          # float64 [nnz]
    nrhs: np.ndarray         # int32 [S]
    rhs_off: np.ndarray      # int64 [S+1]
    B: np.ndarray            # float64 [sum n_s * k_s]
    kinds: list
    ratios: np.ndarray

    @property
    def num_sys(self) -> int:
        return len(self.nrhs)

    def system(self, s: int) -> Problem:
        r0, r1 = int(self.sys_row_off[s]), int(self.sys_row_off[s + 1])
        p0, p1 = int(self.row_ptr[r0]), int(self.row_ptr[r1])
        rp = (self.row_ptr[r0:r1 + 1] - p0).astype(np.int32)
        col = (self.col[p0:p1] - r0).astype(np.int32)
        k = int(self.nrhs[s])
        B = self.B[self.rhs_off[s]:self.rhs_off[s + 1]].reshape(r1 - r0, k)
        return Problem(r1 - r0, rp, col, self.val[p0:p1].copy(), B.copy(),
                       name=f"batch[{s}]:{self.kinds[s]}")


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def sym_csr_from_pairs(n, u, v, w, ratio, isolated_diag=1.0):
    """Full symmetric CSR from undirected pairs (u<v) with values w.

    The diagonal is ``ratio * sum_j |A_ij|``; nodes without an edge get
    ``isolated_diag``.  ``ratio`` may be a scalar or a per-node array.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    absum = np.bincount(u, weights=np.abs(w), minlength=n) + \
        np.bincount(v, weights=np.abs(w), minlength=n)
    diag = np.asarray(ratio, dtype=np.float64) * absum
    diag = np.where(absum == 0.0, isolated_diag, diag)
    return csr_from_triplets(n, np.concatenate([u, v]), np.concatenate([v, u]),
                             np.concatenate([w, w]), diag)


def csr_from_triplets(n, rows, cols, vals, diag):
    ar = np.arange(n, dtype=np.int64)
    m = sp.coo_matrix((np.concatenate([vals, diag]),
                       (np.concatenate([rows, ar]), np.concatenate([cols, ar]))),
                      shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return (m.indptr.astype(np.int32), m.indices.astype(np.int32),
            m.data.astype(np.float64))


def grid2d_pairs(px, py):
    """4-neighbour grid, natural order k = py_index * px + px_index, no wrap."""
    idx = np.arange(px * py, dtype=np.int64).reshape(py, px)
    right = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], 1)
    up = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], 1)
    return _sorted_pairs(np.concatenate([right, up]))


def grid3d_pairs(p):
    """6-neighbour (7-point stencil) cube grid of side p, natural order."""
    idx = np.arange(p ** 3, dtype=np.int64).reshape(p, p, p)
    a = np.stack([idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel()], 1)
    b = np.stack([idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel()], 1)
    c = np.stack([idx[:-1, :, :].ravel(), idx[1:, :, :].ravel()], 1)
    return _sorted_pairs(np.concatenate([a, b, c]))


def er_pairs(n, m, rng):
    """m distinct undirected pairs drawn uniformly (G(n, M)); u == v rejected."""
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges for G(n, M)")
    keys = np.empty(0, dtype=np.int64)
    while len(keys) < m:
        draw = int((m - len(keys)) * 1.1) + 16
        u = rng.integers(0, n, draw, dtype=np.int64)
        v = rng.integers(0, n, draw, dtype=np.int64)
        ok = u != v
        k = np.minimum(u, v)[ok] * n + np.maximum(u, v)[ok]
        allk = np.concatenate([keys, k])
        _, first = np.unique(allk, return_index=True)
        first.sort()  # keep first occurrences, in draw order
        keys = allk[first][:m]
    keys = np.sort(keys)
    return np.stack([keys // n, keys % n], 1)


def _sorted_pairs(pairs):
    pairs = np.sort(pairs, axis=1)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    return pairs[order]


def from_dense(A, b, name=""):
    """CSR of the nonzeros of a small dense symmetric matrix (diagonal kept)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    mask = (A != 0) | np.eye(n, dtype=bool)
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return Problem(n, rp, cols.astype(np.int32), A[rows, cols].copy(),
                   np.asarray(b, dtype=np.float64), name=name)


# ---------------------------------------------------------------------------
# the five benchmark workloads
# ---------------------------------------------------------------------------

def grid2d_problem(px, py, seed, ratio=1.2, lo=-1.0, hi=0.0, name="grid2d"):
    rng = np.random.default_rng(seed)
    pairs = grid2d_pairs(px, py)
    w = rng.uniform(lo, hi, len(pairs))
    rp, col, val = sym_csr_from_pairs(px * py, pairs[:, 0], pairs[:, 1], w, ratio)
    b = rng.standard_normal(px * py)
    return Problem(px * py, rp, col, val, b, name=name)


def config1():
    """32x32 5-point grid, off-diagonals U(-1,0), A_ii = 1.2 sum|A_ij|, b ~ N(0,1)."""
    return grid2d_problem(32, 32, SEED_BASE + 1, ratio=1.2, name="grid2d-32x32")


def er_problem(n, avg_degree, seed, ratio=1.1, name="er"):
    rng = np.random.default_rng(seed)
    m = (avg_degree * n) // 2
    pairs = er_pairs(n, m, rng)
    w = rng.standard_normal(len(pairs))
    rp, col, val = sym_csr_from_pairs(n, pairs[:, 0], pairs[:, 1], w, ratio)
    b = rng.standard_normal(n)
    return Problem(n, rp, col, val, b, name=name)


def config2(n=1 << 20):
    """Erdos-Renyi G(n, 4n): average degree 8, N(0,1) off-diagonals, A_ii = 1.1 sum|A_ij|."""
    return er_problem(n, 8, SEED_BASE + 2, ratio=1.1, name=f"er-n{n}-deg8")


def grid3d_problem(p, seed, ratio=1.1, lo=-1.0, hi=-0.1, with_target=True, name="grid3d"):
    rng = np.random.default_rng(seed)
    pairs = grid3d_pairs(p)
    w = rng.uniform(lo, hi, len(pairs))
    rp, col, val = sym_csr_from_pairs(p ** 3, pairs[:, 0], pairs[:, 1], w, ratio)
    b = rng.standard_normal(p ** 3)
    extra = {}
    if with_target:
        extra["target"] = rng.standard_normal(p ** 3)
    return Problem(p ** 3, rp, col, val, b, name=name, extra=extra)


def config4(p=64):
    """p^3 7-point grid, off-diagonals U(-1,-0.1), A_ii = 1.1 sum|A_ij|; b, target ~ N(0,1)."""
    return grid3d_problem(p, SEED_BASE + 4, name=f"grid3d-{p}^3")


def rect_rows(rng, rows, n, per_row):
    """B (rows x n, SciPy CSR) with per_row distinct uniform columns per row and N(0,1) values."""
    cols = rng.integers(0, n, (rows, per_row), dtype=np.int64)
    while True:  # redraw rows holding a repeated column
        s = np.sort(cols, axis=1)
        bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
        if len(bad) == 0:
            break
        cols[bad] = rng.integers(0, n, (len(bad), per_row), dtype=np.int64)
    vals = rng.standard_normal((rows, per_row))
    return sp.csr_matrix((vals.ravel(), cols.ravel(),
                          np.arange(0, rows * per_row + 1, per_row)), shape=(rows, n))


class RectProblem:
    """[[D, B^T], [B, -gamma I]] {x, z} = {b, h}: B (m x n) as CSR with sorted columns."""

    def __init__(self, m, n, row_ptr, col, val, d, gamma, b, h, name=""):
        self.m, self.n = m, n
        self.row_ptr, self.col, self.val = row_ptr, col, val
        self.d, self.gamma, self.b, self.h = d, gamma, b, h
        self.name = name


def augmented_config(n=1 << 20, rows=None, per_row=4, shift=0.1):
    """The B^T B + shift I system of config5, posed without forming B^T B.

    Same seed and draws as config5 (B, then b): D = shift I, gamma = 1, h = 0,
    so the x-part of the augmented solution is (B^T B + shift I)^-1 b.
    """
    rows = 2 * n if rows is None else rows
    rng = np.random.default_rng(SEED_BASE + 5)
    Bm = rect_rows(rng, rows, n, per_row)
    b = rng.standard_normal(n)
    Bm.sort_indices()
    return RectProblem(rows, n, Bm.indptr.astype(np.int32), Bm.indices.astype(np.int32),
                       Bm.data.astype(np.float64), np.full(n, shift), 1.0, b, np.zeros(rows),
                       name=f"augmented-B{rows}x{n}+{shift}I")


def ridge_problem(m, n, per_row, gamma, seed):
    """The section's own form: D = I, b = 0, h ~ N(0,1): x = (B^T B + gamma I)^-1 B^T h."""
    rng = np.random.default_rng(seed)
    Bm = rect_rows(rng, m, n, per_row)
    h = rng.standard_normal(m)
    Bm.sort_indices()
    return RectProblem(m, n, Bm.indptr.astype(np.int32), Bm.indices.astype(np.int32),
                       Bm.data.astype(np.float64), np.ones(n), float(gamma), np.zeros(n), h,
                       name=f"ridge-B{m}x{n}-g{gamma}")


def config5(n=1 << 20, rows=None, per_row=4, shift=0.1):
    """A = B^T B + shift*I with B (rows x n) having per_row distinct N(0,1) entries per row."""
    rows = 2 * n if rows is None else rows
    rng = np.random.default_rng(SEED_BASE + 5)
    Bm = rect_rows(rng, rows, n, per_row)
    A = (Bm.T @ Bm).tocsr()
    A = ((A + A.T) * 0.5).tocsr()          # exact symmetry of the stored values
    A = (A + shift * sp.identity(n, format="csr")).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    b = rng.standard_normal(n)
    return Problem(n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                   A.data.astype(np.float64), b, name=f"BtB+{shift}I-{rows}x{n}")


BATCH_KINDS = ("grid2d", "grid3d", "er")


def _batch_system(seq, nmin, nmax, kmax):
    """One system of the uneven batch, drawn from its own child seed."""
    rng = np.random.default_rng(seq)
    kind = BATCH_KINDS[int(rng.integers(0, 3))]
    nt = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    ratio = float(rng.uniform(1.05, 1.5))
    k = int(rng.integers(1, kmax + 1))
    if kind == "grid2d":
        side = max(2, int(round(math.sqrt(nt))))
        n = side * side
        pairs = grid2d_pairs(side, side)
        w = rng.uniform(-1.0, 0.0, len(pairs))
    elif kind == "grid3d":
        side = max(2, int(round(nt ** (1.0 / 3.0))))
        n = side ** 3
        pairs = grid3d_pairs(side)
        w = rng.uniform(-1.0, 0.0, len(pairs))
    else:
        n = nt
        d = int(rng.integers(4, 13))
        pairs = er_pairs(n, (d * n) // 2, rng)
        w = rng.standard_normal(len(pairs))
    rp, col, val = sym_csr_from_pairs(n, pairs[:, 0], pairs[:, 1], w, ratio)
    B = rng.standard_normal((n, k))
    return rp, col, val, B.ravel(), n, k, kind, ratio


def _batch_chunk(args):
    seqs, nmin, nmax, kmax = args
    return [_batch_system(q, nmin, nmax, kmax) for q in seqs]


def config3(num_sys=4096, nmin=64, nmax=65536, kmax=32, seed=SEED_BASE + 3, workers=None):
    """Uneven batch: 2-D / 3-D grids and G(n, dn/2) graphs, n log-uniform, 1..kmax RHS.

    Per system (own child seed of SeedSequence(seed)): kind uniform over
    BATCH_KINDS, n_t = round(exp U(ln nmin, ln nmax)), dominance ratio
    U(1.05, 1.5), RHS count uniform in 1..kmax, then the matrix and B ~ N(0,1).
    Grids use U(-1,0) off-diagonals with side round(sqrt n_t) or round(cbrt
    n_t); random graphs use N(0,1) with degree d uniform in 4..12.  Systems are
    drawn in parallel worker processes when ``workers`` > 1; the result does not
    depend on the number of workers.
    """
    seqs = np.random.SeedSequence(seed).spawn(num_sys)
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if num_sys >= 256 else 1
    if workers > 1:
        import concurrent.futures
        step = max(1, num_sys // (workers * 4))
        chunks = [(seqs[i:i + step], nmin, nmax, kmax) for i in range(0, num_sys, step)]
        with concurrent.futures.ProcessPoolExecutor(max_workers=workers) as ex:
            systems = [sy for part in ex.map(_batch_chunk, chunks) for sy in part]
    else:
        systems = _batch_chunk((seqs, nmin, nmax, kmax))
    return _assemble(systems)


def batch_of(problems, nrhs, seed):
    """Batch of the given systems with ``nrhs[s]`` right-hand sides each,
    B ~ N(0,1) drawn in system order from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    systems = []
    for p, k in zip(problems, nrhs):
        B = rng.standard_normal((p.n, int(k)))
        systems.append((p.row_ptr, p.col, p.val, B.ravel(), p.n, int(k), p.name, 0.0))
    return _assemble(systems)


def _assemble(systems):
    rps, cols, Bs, sizes, nrhs, kinds, ratios = [], [], [], [], [], [], []
    vals = []
    row0 = 0
    nnz0 = 0
    for rp, col, val, B, n, k, kind, ratio in systems:
        rps.append(rp[1:].astype(np.int64) + nnz0)
        cols.append(col.astype(np.int64) + row0)
        vals.append(val)
        Bs.append(B)
        sizes.append(n)
        nrhs.append(k)
        kinds.append(kind)
        ratios.append(ratio)
        row0 += n
        nnz0 += int(rp[-1])
    if nnz0 >= 2 ** 31 or row0 >= 2 ** 31:
        raise ValueError("batch exceeds int32 CSR indexing")
    row_ptr = np.concatenate([[0], np.concatenate(rps)]).astype(np.int32)
    sys_row_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    nrhs = np.asarray(nrhs, dtype=np.int32)
    rhs_off = np.concatenate([[0], np.cumsum(np.asarray(sizes, np.int64) * nrhs)]).astype(np.int64)
    return Batch(sys_row_off, row_ptr, np.concatenate(cols).astype(np.int32),
                 np.concatenate(vals), nrhs, rhs_off, np.concatenate(Bs),
                 kinds, np.asarray(ratios))


# ---------------------------------------------------------------------------
# small structured cases used by the edge-case tests
# ---------------------------------------------------------------------------

def powerlaw_pairs(n, m, rng, beta=2.2):
    """m distinct undirected pairs with a power-law degree distribution.

    Chung-Lu style: both ends of a pair are drawn with probability proportional
    to the node weight (i + 1)^(-1 / (beta - 1)), u == v and repeated pairs are
    rejected, and the node labels are shuffled afterwards so that the heavy
    rows land anywhere in the row order (as in a crawled web graph).
    """
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (beta - 1.0))
    cdf = np.cumsum(w / w.sum())
    keys = np.empty(0, dtype=np.int64)
    while len(keys) < m:
        draw = int((m - len(keys)) * 1.3) + 16
        u = np.minimum(np.searchsorted(cdf, rng.random(draw)), n - 1)
        v = np.minimum(np.searchsorted(cdf, rng.random(draw)), n - 1)
        ok = u != v
        k = np.minimum(u, v)[ok] * n + np.maximum(u, v)[ok]
        allk = np.concatenate([keys, k])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        keys = allk[first][:m]
    label = rng.permutation(n).astype(np.int64)
    return _sorted_pairs(np.stack([label[keys // n], label[keys % n]], 1))


def powerlaw_problem(n, avg_degree, seed, beta=2.2, ratio=1.1, name="powerlaw"):
    """Power-law random graph (degree exponent ``beta``), N(0,1) off-diagonals,
    A_ii = ratio * sum|A_ij|, b ~ N(0,1): the heavy-tailed shape of the web and
    social graphs the thesis runs on."""
    rng = np.random.default_rng(seed)
    pairs = powerlaw_pairs(n, (avg_degree * n) // 2, rng, beta)
    w = rng.standard_normal(len(pairs))
    rp, col, val = sym_csr_from_pairs(n, pairs[:, 0], pairs[:, 1], w, ratio)
    b = rng.standard_normal(n)
    return Problem(n, rp, col, val, b, name=name)


def powerlaw_config(n=1 << 20):
    """Power-law graph at the headline size: n nodes, 4n edges, degree exponent
    2.1, N(0,1) off-diagonals, A_ii = 1.1 sum|A_ij|."""
    return powerlaw_problem(n, 8, SEED_BASE + 6, beta=2.1, name=f"powerlaw-n{n}-deg8")


def random_tree(n, seed, ratio=None, name="tree"):
    """Random recursive tree (node i attaches to a uniform earlier node).

    With ``ratio`` None the diagonal is N(0,1)-perturbed away from dominance
    (any nonzero values are allowed on a tree); otherwise ratio*sum|A_ij|.
    """
    rng = np.random.default_rng(seed)
    parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    child = np.arange(1, n, dtype=np.int64)
    pairs = _sorted_pairs(np.stack([parent, child], 1))
    w = rng.standard_normal(len(pairs))
    rp, col, val = sym_csr_from_pairs(n, pairs[:, 0], pairs[:, 1], w,
                                      1.3 if ratio is None else ratio)
    b = rng.standard_normal(n)
    return Problem(n, rp, col, val, b, name=name)


def star_problem(n_leaves, seed, ratio=1.2, name="star"):
    """One hub joined to every leaf: a single row of very high degree."""
    rng = np.random.default_rng(seed)
    pairs = np.stack([np.zeros(n_leaves, np.int64), np.arange(1, n_leaves + 1)], 1)
    w = rng.uniform(-1.0, 1.0, n_leaves)
    rp, col, val = sym_csr_from_pairs(n_leaves + 1, pairs[:, 0], pairs[:, 1], w, ratio)
    b = rng.standard_normal(n_leaves + 1)
    return Problem(n_leaves + 1, rp, col, val, b, name=name)


def poisson2d(p, f=-1.0):
    """Dirichlet 5-point Poisson matrix on a p x p interior grid, b = -f h^2."""
    pairs = grid2d_pairs(p, p)
    w = -np.ones(len(pairs))
    n = p * p
    rp, col, val = csr_from_triplets(n, np.concatenate([pairs[:, 0], pairs[:, 1]]),
                                     np.concatenate([pairs[:, 1], pairs[:, 0]]),
                                     np.concatenate([w, w]), np.full(n, 4.0))
    h = 1.0 / (p + 1)
    return Problem(n, rp, col, val, np.full(n, -f * h * h), name=f"poisson-{p}")
