"""FP64 reference implementation of synchronous Gaussian BP (test infrastructure).

TEST INFRASTRUCTURE ONLY -- imported by tests, the smoke check and the
benchmark's CPU baseline; never by the solver.  Plain NumPy, FP64, written
from Bickson, "Gaussian Belief Propagation: Theory and Application".

Notation follows the paper: node i has the prior P_ii = A_ii and mu_ii =
b_i / A_ii (the prior of Alg. 1, from the self potential of Ch. 2 Sec. 2.3); every
directed edge i -> j (A_ij != 0, i != j) carries a precision P_ij and a mean
mu_ij.  A sweep is synchronous: every message of round t is computed from the
messages of round t-1 only (parallel scheduling, Ch. 2 Sec. 2.3).  Round 0 has
all messages zero, so the round-0 means are b_i / A_ii; the tentative means of
round t use the messages of round t (Ch. 4 toy example tables).

``serial_gabp`` is the serial scheduling of the same section: one set of
messages updated in place, the nodes visited colour class by colour class of
a first-fit colouring in row order (``greedy_colouring``).

Stop rule (a reading: the algorithm states its stop condition only as the
messages having converged to within a tolerance): the relative residual ||b - A x_t||_2 / ||b||_2 <= tol, evaluated on rounds t with
t % check_every == 0 and on the last allowed round.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

__all__ = [
    "EdgeGraph", "edge_graph", "dense_from_csr", "dense_solve",
    "dense_marginal_precisions", "residual", "naive_gabp", "broadcast_gabp",
    "fixpoint_violation", "is_strictly_dd", "walk_rho", "walk_rho_dense",
    "rate_bound", "dd_loading", "walk_loading", "convfix_dense",
    "convfix_gabp", "convfix_single_loop", "adjoint_gradient", "fd_gradient", "loss",
    "greedy_colouring", "serial_gabp", "naive_serial_gabp",
    "aitken_extrapolate", "aitken_gabp", "steffensen_gabp", "augmented_csr", "augmented_solution",
]


# ---------------------------------------------------------------------------
# graph of the linear system (Ch. 2 Sec. 2.1: one node per variable, one
# undirected edge per nonzero A_ij, i != j; each carries two directed messages)
# ---------------------------------------------------------------------------

class EdgeGraph:
    def __init__(self, n, src, dst, a, rev, diag):
        self.n = n          # number of nodes
        self.src = src      # edge e is the message src[e] -> dst[e]
        self.dst = dst
        self.a = a          # A_{src,dst}
        self.rev = rev      # index of the edge dst[e] -> src[e]
        self.diag = diag    # A_ii

    @property
    def num_edges(self):
        return len(self.src)


def _rows_of(row_ptr):
    n = len(row_ptr) - 1
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(row_ptr, dtype=np.int64)))


def edge_graph(n, row_ptr, col, val):
    """Directed edge list of a symmetric CSR matrix (stored off-diagonal nonzeros)."""
    rows = _rows_of(row_ptr)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    diag = np.zeros(n)
    on_diag = rows == col
    diag[rows[on_diag]] = val[on_diag]
    keep = (~on_diag) & (val != 0.0)
    src, dst, a = rows[keep], col[keep], val[keep]
    key = src * n + dst
    order = np.argsort(key, kind="stable")
    rkey = dst * n + src
    pos = np.searchsorted(key[order], rkey)
    if len(key) and (np.any(pos >= len(key)) or np.any(key[order][np.minimum(pos, len(key) - 1)] != rkey)):
        raise ValueError("matrix pattern is not symmetric")
    rev = order[pos] if len(key) else np.zeros(0, dtype=np.int64)
    return EdgeGraph(n, src, dst, a, rev, diag)


def dense_from_csr(n, row_ptr, col, val):
    A = np.zeros((n, n))
    A[_rows_of(row_ptr), np.asarray(col, dtype=np.int64)] = val
    return A


def residual(n, row_ptr, col, val, x, b):
    """r = b - A x and ||r||_2 / ||b||_2 (||r||_2 when b = 0)."""
    rows = _rows_of(row_ptr)
    Ax = np.bincount(rows, weights=np.asarray(val) * x[np.asarray(col, dtype=np.int64)], minlength=n)
    r = b - Ax
    nb = np.linalg.norm(b)
    return r, (np.linalg.norm(r) / nb if nb > 0 else np.linalg.norm(r))


# ---------------------------------------------------------------------------
# the plain definition: x* = A^-1 b, P_i^-1 = (A^-1)_ii  (Prop. 2.1)
# ---------------------------------------------------------------------------

def dense_solve(A, b):
    """x = A^-1 b by Cholesky (A SPD) or, for indefinite A, LU with pivoting."""
    A = np.asarray(A, dtype=np.float64)
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return np.linalg.solve(A, b)
    y = scipy.linalg.solve_triangular(L, b, lower=True)
    return scipy.linalg.solve_triangular(L.T, y, lower=False)


def dense_marginal_precisions(A):
    """P_i = 1 / (A^-1)_ii, the exact marginal precisions."""
    return 1.0 / np.diag(np.linalg.inv(np.asarray(A, dtype=np.float64)))


# ---------------------------------------------------------------------------
# Alg. 1 -- naive GaBP, scalar loops (exact with Fraction inputs)
# ---------------------------------------------------------------------------

def naive_gabp(A, b, sweeps):
    """Synchronous Alg. 1 for ``sweeps`` rounds on a small dense matrix.

    ``A`` is a list of rows and ``b`` a list; entries may be floats or
    ``fractions.Fraction``.  Returns one record per round t = 0..sweeps with
    the messages ``P[(i, j)]``, ``mu[(i, j)]`` (message i -> j), the tentative
    means ``mean[i]`` and the marginal precisions ``prec[i]`` (the marginals of Alg. 1).
    """
    n = len(A)
    zero = b[0] * 0
    nbr = [[k for k in range(n) if k != i and A[k][i] != 0] for i in range(n)]
    Pii = [A[i][i] for i in range(n)]
    muii = [b[i] / A[i][i] for i in range(n)]
    P = {(k, i): zero for i in range(n) for k in nbr[i]}
    mu = {(k, i): zero for i in range(n) for k in nbr[i]}

    def infer(P, mu):
        prec, mean = [], []
        for i in range(n):
            num = Pii[i] * muii[i] + sum((P[(k, i)] * mu[(k, i)] for k in nbr[i]), zero)
            den = Pii[i] + sum((P[(k, i)] for k in nbr[i]), zero)
            prec.append(den)
            mean.append(num / den)
        return prec, mean

    out = []
    prec, mean = infer(P, mu)
    out.append({"P": dict(P), "mu": dict(mu), "mean": mean, "prec": prec})
    for _ in range(sweeps):
        newP, newmu = {}, {}
        for i in range(n):
            for j in nbr[i]:
                # exclusion sums over N(i) \ j, from the previous round only
                den = Pii[i] + sum((P[(k, i)] for k in nbr[i] if k != j), zero)
                num = Pii[i] * muii[i] + sum((P[(k, i)] * mu[(k, i)] for k in nbr[i] if k != j), zero)
                newP[(i, j)] = -A[i][j] * A[i][j] / den
                newmu[(i, j)] = num / A[i][j]
        P, mu = newP, newmu
        prec, mean = infer(P, mu)
        out.append({"P": dict(P), "mu": dict(mu), "mean": mean, "prec": prec})
    return out


# ---------------------------------------------------------------------------
# Alg. 2 -- broadcast GaBP, vectorised over directed edges
# ---------------------------------------------------------------------------

def _broadcast(g, Pii, muii, P, mu):
    """Node aggregates of Alg. 2: every node i forms P~_i and mu~_i from all k -> i."""
    Pt = Pii + np.bincount(g.dst, weights=P, minlength=g.n)
    mut = (Pii * muii + np.bincount(g.dst, weights=P * mu, minlength=g.n)) / Pt
    return Pt, mut


def _internal_scalars(g, Pt, mut, P, mu):
    """Message update of Alg. 2: message i -> j from node i's broadcast minus j -> i."""
    Pji = P[g.rev]
    muji = mu[g.rev]
    Pi = Pt[g.src]
    Pnew = -g.a * g.a / (Pi - Pji)
    munew = (Pi * mut[g.src] - Pji * muji) / g.a
    return Pnew, munew


def broadcast_gabp(n, row_ptr, col, val, b, tol=1e-10, max_sweeps=2000,
                   check_every=1, history=False, return_messages=False, graph=None):
    """Synchronous broadcast GaBP (Alg. 2) on a symmetric CSR system.

    Runs rounds t = 0, 1, ... until the stop rule of the module docstring
    holds or t == max_sweeps; ``tol <= 0`` runs exactly ``max_sweeps`` rounds.
    Returns a dict with ``x`` (means of the last round), ``prec`` (P~),
    ``sweeps`` (that round's index), ``converged``, ``rel_residual`` and,
    on request, the residual history and the final messages.
    """
    b = np.asarray(b, dtype=np.float64)
    g = graph if graph is not None else edge_graph(n, row_ptr, col, val)
    Pii = g.diag
    muii = b / g.diag
    P = np.zeros(g.num_edges)
    mu = np.zeros(g.num_edges)
    hist = []
    t = 0
    rel = float("nan")
    converged = False
    while True:
        Pt, mut = _broadcast(g, Pii, muii, P, mu)
        if tol > 0 and (t % check_every == 0 or t == max_sweeps):
            _, rel = residual(n, row_ptr, col, val, mut, b)
            hist.append((t, rel))
            if rel <= tol:
                converged = True
                break
            if not np.isfinite(rel):
                break
        if t >= max_sweeps:
            break
        P, mu = _internal_scalars(g, Pt, mut, P, mu)
        t += 1
    if tol <= 0:
        _, rel = residual(n, row_ptr, col, val, mut, b)
    out = {"x": mut, "prec": Pt, "sweeps": t, "converged": converged, "rel_residual": rel}
    if history:
        out["history"] = hist
    if return_messages:
        out.update(graph=g, P=P, mu=mu)
    return out


# ---------------------------------------------------------------------------
# Aitken's extrapolation of the means (Ch. 3 Sec. 3.2, convergence
# acceleration): node-local, from three successive rounds; the iteration
# itself is left unchanged
# ---------------------------------------------------------------------------

def aitken_extrapolate(x0, x1, x2):
    """Aitken's delta-squared step applied node by node to three successive means.

    y = x0 - (x1 - x0)^2 / (x2 - 2 x1 + x0) for rounds n, n+1, n+2 (Ch. 3
    Sec. 3.2).  Reading: where the second difference is zero or the
    correction is not finite (the formula is undefined there, e.g. a mean
    that has stopped moving), y is the newest mean x2.
    """
    x0 = np.asarray(x0, dtype=np.float64)
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    d1 = x1 - x0
    den = x2 - 2.0 * x1 + x0
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        corr = d1 * d1 / den
    ok = (den != 0.0) & np.isfinite(corr)
    return np.where(ok, x0 - corr, x2)


def aitken_gabp(n, row_ptr, col, val, b, tol=1e-10, max_sweeps=2000, check_every=1, history=False):
    """Synchronous Alg. 2 whose output is Aitken's extrapolation of its means.

    The messages follow Alg. 2 exactly as in ``broadcast_gabp``; after round
    t >= 2 the estimate y_t = aitken_extrapolate(x_{t-2}, x_{t-1}, x_t) is
    formed (Ch. 3 Sec. 3.2: every node uses its own history only).  Stop rule
    as in the module docstring, applied to y_t on rounds t >= 2 with
    t % check_every == 0 or t == max_sweeps; tol <= 0 runs exactly
    ``max_sweeps`` (>= 2) rounds and returns y_{max_sweeps}.  A non-finite
    relative residual of y_t ends the run unconverged.  Returns a dict with
    ``y``, ``x`` (the means of the same round), ``sweeps``, ``converged``,
    ``rel_residual`` and, on request, the (round, residual) history.
    """
    if max_sweeps < 2:
        raise ValueError("Aitken's step needs three rounds (max_sweeps >= 2)")
    b = np.asarray(b, dtype=np.float64)
    g = edge_graph(n, row_ptr, col, val)
    Pii = g.diag
    muii = b / g.diag
    P = np.zeros(g.num_edges)
    mu = np.zeros(g.num_edges)
    means = []                        # x_{t-2}, x_{t-1}, x_t
    hist = []
    t = 0
    y = None
    rel = float("nan")
    converged = False
    while True:
        Pt, x = _broadcast(g, Pii, muii, P, mu)
        means = (means + [x])[-3:]
        if t >= 2:
            last = t == max_sweeps
            if tol <= 0:
                if last:
                    y = aitken_extrapolate(*means)
            elif t % check_every == 0 or last:
                y = aitken_extrapolate(*means)
                _, rel = residual(n, row_ptr, col, val, y, b)
                hist.append((t, rel))
                if rel <= tol:
                    converged = True
                    break
                if not np.isfinite(rel):
                    break
        if t >= max_sweeps:
            break
        P, mu = _internal_scalars(g, Pt, x, P, mu)
        t += 1
    if tol <= 0:
        _, rel = residual(n, row_ptr, col, val, y, b)
    out = {"y": y, "x": means[-1], "sweeps": t, "converged": converged, "rel_residual": rel}
    if history:
        out["history"] = hist
    return out


def steffensen_gabp(n, row_ptr, col, val, b, tol=1e-10, max_sweeps=2000, check_every=1, history=False):
    """Steffensen's iterations on the GaBP means (Ch. 3 Sec. 3.2).

    The iteration runs in cycles of two synchronous Alg. 2 rounds.  A cycle
    starts from an estimate s (the round-0 means b_i / A_ii for the first
    cycle), runs two rounds to get the means x1 and x2, and forms Aitken's
    y = aitken_extrapolate(s, x1, x2).  Then y replaces the newest means: the
    next messages are formed from node i's broadcast with its mean set to y_i
    and its precision P~_i unchanged (reading: GaBP "executed again" from y
    means the messages leave every node with y as its current mean), and y
    starts the next cycle.

    Stop rule as in the module docstring, applied to y at the ends of cycles,
    rounds t (even) with t % check_every == 0 and at the last cycle, which ends
    at round 2 * floor(max_sweeps / 2).  tol <= 0 runs every cycle and
    returns the last y.  Needs max_sweeps >= 2.  Returns a dict with ``x``
    (= y), ``prec``, ``sweeps``, ``converged``, ``rel_residual`` and, on
    request, the (round, residual) history.
    """
    if max_sweeps < 2:
        raise ValueError("a Steffensen cycle needs two rounds (max_sweeps >= 2)")
    b = np.asarray(b, dtype=np.float64)
    g = edge_graph(n, row_ptr, col, val)
    Pii = g.diag
    muii = b / g.diag
    P = np.zeros(g.num_edges)
    mu = np.zeros(g.num_edges)
    Pt, mut = _broadcast(g, Pii, muii, P, mu)   # round 0
    start = mut
    hist = []
    t = 0
    rel = float("nan")
    converged = False
    while t + 2 <= max_sweeps:
        P, mu = _internal_scalars(g, Pt, mut, P, mu)
        Pt, x1 = _broadcast(g, Pii, muii, P, mu)
        P, mu = _internal_scalars(g, Pt, x1, P, mu)
        Pt, x2 = _broadcast(g, Pii, muii, P, mu)
        t += 2
        y = aitken_extrapolate(start, x1, x2)
        mut = y          # the broadcast of round t carries y
        start = y
        if tol > 0 and (t % check_every == 0 or t + 2 > max_sweeps):
            _, rel = residual(n, row_ptr, col, val, y, b)
            hist.append((t, rel))
            if rel <= tol:
                converged = True
                break
            if not np.isfinite(rel):
                break
    if tol <= 0:
        _, rel = residual(n, row_ptr, col, val, mut, b)
    out = {"x": mut, "prec": Pt, "sweeps": t, "converged": converged, "rel_residual": rel}
    if history:
        out["history"] = hist
    return out


def fixpoint_violation(g, P, mu, b):
    """Violation of Alg. 2's message equations by (P, mu), relative in the max norm."""
    Pii = g.diag
    muii = np.asarray(b, dtype=np.float64) / g.diag
    Pt, mut = _broadcast(g, Pii, muii, P, mu)
    Pn, mun = _internal_scalars(g, Pt, mut, P, mu)
    if g.num_edges == 0:
        return 0.0
    # infinity-norm relative violation of each message family
    eP = np.max(np.abs(Pn - P)) / max(np.max(np.abs(P)), 1e-300)
    emu = np.max(np.abs(mun - mu)) / max(np.max(np.abs(mu)), 1e-300)
    return max(eP, emu)


# ---------------------------------------------------------------------------
# serial scheduling (Ch. 2 Sec. 2.3): one set of messages, updated in place,
# the nodes visited colour class by colour class
# ---------------------------------------------------------------------------

def greedy_colouring(n, row_ptr, col):
    """First-fit colouring in row order of the stored off-diagonal pattern.

    Node i, visited in increasing i, takes the smallest colour that none of
    its already coloured neighbours (stored columns j < i) holds.  Returns an
    int64 array of colours; no two neighbours share one.
    """
    rp = [int(v) for v in row_ptr]
    cl = [int(v) for v in col]
    colour = [-1] * n
    stamp = [-1] * (max((rp[i + 1] - rp[i] for i in range(n)), default=0) + 2)
    for i in range(n):
        for s in range(rp[i], rp[i + 1]):
            j = cl[s]
            if j < i:
                stamp[colour[j]] = i
        c = 0
        while stamp[c] == i:
            c += 1
        colour[i] = c
    return np.asarray(colour, dtype=np.int64)


def serial_gabp(n, row_ptr, col, val, b, colour=None, tol=1e-10, max_sweeps=2000,
                check_every=1, history=False, return_messages=False):
    """Serially scheduled broadcast GaBP (Ch. 2 Sec. 2.3 with the Alg. 2 updates).

    There is a single set of messages, initially zero, and every update
    overwrites it.  A sweep visits the colour classes of ``colour`` (default:
    ``greedy_colouring``) in increasing order.  No two nodes of a class are
    neighbours, so a class can be updated at once and the order inside it is
    immaterial.  Updating node i:
      - forms P~_i and mu~_i from its current incoming messages (the Alg. 2
        aggregate);
      - takes mu~_i as its mean of this sweep;
      - replaces every outgoing message i -> j by the Alg. 2 update, which
        subtracts the current j -> i.
    x^(t) collects the means of sweep t; round 0 is the prior b_i / A_ii.

    Stop rule (reading): the relative residual of x^(t) is <= tol, checked
    from sweep 1 on at t % check_every == 0 and at the last allowed sweep.
    The prior round is checked only when ``max_sweeps`` is 0.  ``tol <= 0`` runs exactly
    ``max_sweeps`` sweeps.  Returns the same fields as ``broadcast_gabp``,
    plus ``colours``.
    """
    b = np.asarray(b, dtype=np.float64)
    g = edge_graph(n, row_ptr, col, val)
    if colour is None:
        colour = greedy_colouring(n, row_ptr, col)
    colour = np.asarray(colour, dtype=np.int64)
    ncol = int(colour.max()) + 1 if n else 0
    Pii = g.diag
    hii = b                               # P_ii mu_ii
    P = np.zeros(g.num_edges)             # message src -> dst
    h = np.zeros(g.num_edges)             # P * mu of that message
    x = b / Pii
    prec = Pii.copy()
    nodes = [np.nonzero(colour == k)[0] for k in range(ncol)]
    into = [np.nonzero(colour[g.dst] == k)[0] for k in range(ncol)]   # edges k_node <- *
    out_of = [np.nonzero(colour[g.src] == k)[0] for k in range(ncol)]  # edges k_node -> *
    hist = []
    t = 0
    rel = float("nan")
    converged = False
    while t < max_sweeps:
        t += 1
        for k in range(ncol):
            v, ein, eout = nodes[k], into[k], out_of[k]
            # aggregates of class k from the current incoming messages
            Pt = Pii[v] + np.bincount(g.dst[ein], weights=P[ein], minlength=n)[v]
            ht = hii[v] + np.bincount(g.dst[ein], weights=h[ein], minlength=n)[v]
            prec[v] = Pt
            x[v] = ht / Pt
            # outgoing messages: node i's broadcast minus the current j -> i
            Ptn = np.zeros(n)
            htn = np.zeros(n)
            Ptn[v] = Pt
            htn[v] = ht
            src = g.src[eout]
            D = Ptn[src] - P[g.rev[eout]]
            newP = -g.a[eout] * g.a[eout] / D
            newh = -g.a[eout] * (htn[src] - h[g.rev[eout]]) / D
            P[eout] = newP
            h[eout] = newh
        if tol > 0 and (t % check_every == 0 or t == max_sweeps):
            _, rel = residual(n, row_ptr, col, val, x, b)
            hist.append((t, rel))
            if rel <= tol:
                converged = True
                break
            if not np.isfinite(rel):
                break
    if tol <= 0 or t == 0:
        _, rel = residual(n, row_ptr, col, val, x, b)
        if tol > 0:  # no sweep allowed: the prior is the last allowed round
            hist.append((0, rel))
            converged = bool(rel <= tol)
    out = {"x": x.copy(), "prec": prec.copy(), "sweeps": t, "converged": converged,
           "rel_residual": rel, "colours": ncol}
    if history:
        out["history"] = hist
    if return_messages:
        with np.errstate(divide="ignore", invalid="ignore"):
            mu = np.where(P != 0.0, h / np.where(P != 0.0, P, 1.0), 0.0)
        out.update(graph=g, P=P.copy(), mu=mu)
    return out


def naive_serial_gabp(A, b, order, sweeps):
    """Alg. 1 with serial scheduling on a small dense matrix, one node at a time.

    ``order`` lists the nodes in visiting order.  Visiting node i replaces
    each outgoing message i -> j by the Alg. 1 formulas with exclusion sums
    over N(i) \\ j of the CURRENT incoming messages (one data structure), and
    records the mean of i from the same messages.  Entries may be floats or
    ``fractions.Fraction``.  Returns the means after each sweep, sweeps 0
    (the prior) to ``sweeps``.
    """
    n = len(A)
    zero = b[0] * 0
    nbr = [[k for k in range(n) if k != i and A[k][i] != 0] for i in range(n)]
    Pii = [A[i][i] for i in range(n)]
    muii = [b[i] / A[i][i] for i in range(n)]
    P = {(k, i): zero for i in range(n) for k in nbr[i]}
    mu = {(k, i): zero for i in range(n) for k in nbr[i]}
    mean = list(muii)
    out = [list(mean)]
    for _ in range(sweeps):
        for i in order:
            num = Pii[i] * muii[i] + sum((P[(k, i)] * mu[(k, i)] for k in nbr[i]), zero)
            den = Pii[i] + sum((P[(k, i)] for k in nbr[i]), zero)
            mean[i] = num / den
            for j in nbr[i]:
                d = Pii[i] + sum((P[(k, i)] for k in nbr[i] if k != j), zero)
                m = Pii[i] * muii[i] + sum((P[(k, i)] * mu[(k, i)] for k in nbr[i] if k != j), zero)
                P[(i, j)] = -A[i][j] * A[i][j] / d
                mu[(i, j)] = m / A[i][j]
        out.append(list(mean))
    return out


# ---------------------------------------------------------------------------
# convergence conditions and the rate bound
# ---------------------------------------------------------------------------

def is_strictly_dd(A):
    A = np.asarray(A)
    off = np.sum(np.abs(A), axis=1) - np.abs(np.diag(A))
    return bool(np.all(np.abs(np.diag(A)) > off))


def walk_rho_dense(A):
    """rho(|R|) with R = I - D^-1/2 A D^-1/2, D = |diag A| (walk-summability)."""
    A = np.asarray(A, dtype=np.float64)
    s = 1.0 / np.sqrt(np.abs(np.diag(A)))
    R = np.eye(len(A)) - s[:, None] * A * s[None, :]
    return float(np.max(np.abs(np.linalg.eigvals(np.abs(R)))))


def walk_rho(n, row_ptr, col, val, iters=2000, rtol=1e-6):
    """rho(|R|) for sparse A by power iteration on M = |R| + I.

    A is symmetric, so M is symmetric and nonnegative: the Rayleigh quotient
    v^T M v / v^T v is a lower bound on rho(M) and, for v > 0, max_i (Mv)_i / v_i
    is an upper bound (Collatz-Wielandt).  The shift by I keeps the Perron root
    strictly dominant.  Returns (lower, upper) bounds on rho(|R|).
    """
    rows = _rows_of(row_ptr)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    diag = np.zeros(n)
    on = rows == col
    diag[rows[on]] = val[on]
    s = 1.0 / np.sqrt(np.abs(diag))
    w = np.where(on, 0.0, np.abs(val) * s[rows] * s[col])
    v = np.ones(n)
    lo, hi = 0.0, float("inf")
    for _ in range(iters):
        Mv = v + np.bincount(rows, weights=w * v[col], minlength=n)
        lo = float(v @ Mv / (v @ v)) - 1.0
        pos = v > 0
        hi = float(np.max(Mv[pos] / v[pos])) - 1.0
        v = Mv / np.max(Mv)
        if hi - lo <= rtol * max(1.0, hi):
            break
    return lo, hi


def rate_bound(A, eps):
    """Rounds to accuracy eps*||b||_inf from the rate bound of Ch. 3 Sec. 3.1.

    eps_i = |a_ii| - sum_{j in N(i)} |a_ij| (must be > 0), gamma = max over
    i and j in N(i) of 1 / (1 + eps_i / (|a_ij| |N(i)|)), t = ceil(log eps / log gamma).
    """
    A = np.asarray(A, dtype=np.float64)
    n = len(A)
    gamma = 0.0
    for i in range(n):
        nbr = [j for j in range(n) if j != i and A[i, j] != 0]
        if not nbr:
            continue
        gap = abs(A[i, i]) - sum(abs(A[i, j]) for j in nbr)
        if gap <= 0:
            raise ValueError("rate bound needs strict diagonal dominance")
        for j in nbr:
            gamma = max(gamma, 1.0 / (1.0 + gap / (abs(A[i, j]) * len(nbr))))
    if gamma == 0.0:
        return 0, gamma
    return int(math.ceil(math.log(eps) / math.log(gamma))), gamma


# ---------------------------------------------------------------------------
# Ch. 5 -- diagonal loading and the iterative correction (double loop)
# ---------------------------------------------------------------------------

def dd_loading(A, delta=0.05):
    """Gamma_ii making A + Gamma strictly diagonally dominant (Ch. 5 Sec. 5.2).

    Reading of the garbled threshold: Gamma_ii = max(0, (1+delta) sum_{j!=i}
    |A_ij| - A_ii).
    """
    A = np.asarray(A, dtype=np.float64)
    off = np.sum(np.abs(A), axis=1) - np.abs(np.diag(A))
    return np.maximum(0.0, (1.0 + delta) * off - np.diag(A))


def walk_loading(rho, delta=0.05):
    """Normalised loading gamma with (1+gamma) > rho(|R|) (Lemma of Sec. 5.2).

    gamma = (1+delta) rho - 1 when rho >= 1, else 0; applied as Gamma = gamma * diag(A).
    """
    return max(0.0, (1.0 + delta) * rho - 1.0)


def convfix_dense(A, b, Gamma, x0, steps):
    """Iterates x^{t+1} = (A + Gamma)^-1 (b + Gamma x^t) with exact inner solves."""
    A = np.asarray(A, dtype=np.float64)
    G = np.diag(Gamma)
    xs = [np.asarray(x0, dtype=np.float64)]
    for _ in range(steps):
        xs.append(np.linalg.solve(A + G, b + Gamma * xs[-1]))
    return xs


def convfix_gabp(n, row_ptr, col, val, b, Gamma, tol=1e-9, max_outer=1000,
                 inner_tol=1e-12, inner_max=100000):
    """Double loop of Ch. 5: inner Alg. 2 on A + Gamma, outer h^{t+1} = b + Gamma x^t.

    Stops when the relative residual of the original system is <= tol.
    """
    b = np.asarray(b, dtype=np.float64)
    rows = _rows_of(row_ptr)
    loaded = np.asarray(val, dtype=np.float64).copy()
    on = rows == np.asarray(col)
    loaded[on] += Gamma[rows[on]]
    g = edge_graph(n, row_ptr, col, loaded)
    x = np.zeros(n)
    inner_total = 0
    for k in range(max_outer + 1):
        _, rel = residual(n, row_ptr, col, val, x, b)
        if rel <= tol or k == max_outer:
            break
        res = broadcast_gabp(n, row_ptr, col, loaded, b + Gamma * x, tol=inner_tol,
                             max_sweeps=inner_max, graph=g)
        inner_total += res["sweeps"]
        x = res["x"]
    return {"x": x, "outer": k, "inner_sweeps": inner_total, "rel_residual": rel,
            "converged": rel <= tol}


def convfix_single_loop(n, row_ptr, col, val, b, Gamma, s=0.5, tol=1e-9, max_sweeps=100000,
                        check_every=1, history=False):
    """Single-loop form of the correction method of Ch. 5 Sec. 5.3.

    One synchronous Alg. 2 round per outer step on the loaded matrix
    J' = A + Gamma, whose prior potentials follow the damped feedback
    h^(t+1) = b + Gamma ((1 - s) x^(t-1) + s x^(t)), with h^(0) = b and
    x^(-1) = 0 (reading: of the section's two forms of the damped update, the
    explicit two-point one).  Round t's node aggregates use h^(t); the messages
    of round t+1 are formed from round t's aggregates as in Alg. 2.  Stops when
    the relative residual of the ORIGINAL system A x = b is <= tol (checked on
    rounds t % check_every == 0 and the last); tol <= 0 runs exactly
    ``max_sweeps`` rounds.  Gamma = 0 is plain Alg. 2.
    """
    b = np.asarray(b, dtype=np.float64)
    Gamma = np.asarray(Gamma, dtype=np.float64)
    rows = _rows_of(row_ptr)
    loaded = np.asarray(val, dtype=np.float64).copy()
    on = rows == np.asarray(col)
    loaded[on] += Gamma[rows[on]]
    g = edge_graph(n, row_ptr, col, loaded)
    Pii = g.diag
    h = b.copy()                      # prior potentials of the current round
    x_prev = np.zeros(n)              # x^(t-1)
    P = np.zeros(g.num_edges)
    mu = np.zeros(g.num_edges)
    hist = []
    t = 0
    rel = float("nan")
    converged = False
    while True:
        Pt, x = _broadcast(g, Pii, h / Pii, P, mu)      # round t, prior h^(t)
        if tol > 0 and (t % check_every == 0 or t == max_sweeps):
            _, rel = residual(n, row_ptr, col, val, x, b)
            hist.append((t, rel))
            if rel <= tol:
                converged = True
                break
            if not np.isfinite(rel):
                break
        if t >= max_sweeps:
            break
        P, mu = _internal_scalars(g, Pt, x, P, mu)       # messages of round t+1
        h = b + Gamma * ((1.0 - s) * x_prev + s * x)     # h^(t+1)
        x_prev = x
        t += 1
    if tol <= 0:
        _, rel = residual(n, row_ptr, col, val, x, b)
    out = {"x": x, "prec": Pt, "sweeps": t, "converged": converged, "rel_residual": rel}
    if history:
        out["history"] = hist
    return out


# ---------------------------------------------------------------------------
# general (rectangular) systems through the symmetric augmented matrix of
# Ch. 5 Sec. 5.4
# ---------------------------------------------------------------------------

def augmented_csr(m, n, row_ptr, col, val, d, gamma):
    """CSR of the symmetric block matrix [[D, B^T], [B, -gamma I]] for B of m x n.

    B is given as CSR (rows of length n); D = diag(d), d_i != 0; gamma > 0.
    Unknowns 0..n-1 are x, unknowns n..n+m-1 the auxiliary vector z of Ch. 5
    Sec. 5.4; the section's own matrix is D = I with right-hand side {0, h}.
    Returns (N, row_ptr, col, val) with sorted columns and the diagonal stored.
    """
    import scipy.sparse as sp
    B = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)),
                      shape=(m, n))
    K = sp.bmat([[sp.diags(np.asarray(d, dtype=np.float64)), B.T],
                 [B, -float(gamma) * sp.identity(m)]], format="csr")
    K.sort_indices()
    return (n + m, K.indptr.astype(np.int32), K.indices.astype(np.int32),
            K.data.astype(np.float64))


def augmented_solution(m, n, row_ptr, col, val, d, gamma, b=None, h=None):
    """x-part of the solution of [[D, B^T], [B, -gamma I]] {x, z} = {b, h}, by elimination of z.

    The second block row gives z = (B x - h) / gamma; the first then reads
    (B^T B / gamma + D) x = b + B^T h / gamma.  With D = I and b = 0 this is
    the regularised pseudo-inverse solution (B^T B + gamma I)^-1 B^T h of Ch. 5
    Sec. 5.4, and with h = 0, gamma = 1 it is (B^T B + D)^-1 b.  Dense; small
    systems only.
    """
    B = np.zeros((m, n))
    rows = _rows_of(row_ptr)
    np.add.at(B, (rows, np.asarray(col)), np.asarray(val, dtype=np.float64))
    b = np.zeros(n) if b is None else np.asarray(b, dtype=np.float64)
    h = np.zeros(m) if h is None else np.asarray(h, dtype=np.float64)
    S = B.T @ B / gamma + np.diag(np.asarray(d, dtype=np.float64))
    return dense_solve(S, b + B.T @ h / gamma)


# ---------------------------------------------------------------------------
# gradients of L = 0.5 ||x - target||^2 with x = A^-1 b
# ---------------------------------------------------------------------------

def loss(A, b, target):
    x = np.linalg.solve(A, b)
    return 0.5 * float(np.sum((x - target) ** 2))


def adjoint_gradient(A, b, target, row_ptr, col):
    """Dense adjoint: lambda = A^-T (x - t); dL/db = lambda; dL/dA = -lambda x^T.

    A symmetric CSR value array ties A_ij and A_ji: the stored entry (i, j),
    i != j, gets G_ij + G_ji = -(lambda_i x_j + lambda_j x_i), the derivative
    when both mirror entries move together; a diagonal entry gets G_ii.
    """
    A = np.asarray(A, dtype=np.float64)
    x = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, x - target)
    G = -np.outer(lam, x)
    rows = _rows_of(row_ptr)
    col = np.asarray(col, dtype=np.int64)
    gv = np.where(rows == col, G[rows, col], G[rows, col] + G[col, rows])
    return x, lam, gv


def fd_gradient(A, b, target, row_ptr, col, rel_step=1e-6):
    """Central finite differences of L over b_i and over mirror pairs of A."""
    A = np.asarray(A, dtype=np.float64)
    rows = _rows_of(row_ptr)
    col = np.asarray(col, dtype=np.int64)
    gv = np.zeros(len(col))
    for e in range(len(col)):
        i, j = rows[e], col[e]
        h = rel_step * max(abs(A[i, j]), 1.0)
        Ap = A.copy()
        Am = A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        if i != j:
            Ap[j, i] += h
            Am[j, i] -= h
        gv[e] = (loss(Ap, b, target) - loss(Am, b, target)) / (2 * h)
    gb = np.zeros(len(b))
    for i in range(len(b)):
        h = rel_step * max(abs(b[i]), 1.0)
        bp = b.copy()
        bm = b.copy()
        bp[i] += h
        bm[i] -= h
        gb[i] = (loss(A, bp, target) - loss(A, bm, target)) / (2 * h)
    return gv, gb
