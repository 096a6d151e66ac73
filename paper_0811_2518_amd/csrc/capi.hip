// extern "C" entry points of libgabp (declared in include/gabp.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gabp_internal.h"

namespace gabp {

static thread_local std::string tl_error;

gabp_status fail(Ctx* c, gabp_status s, const std::string& msg) {
  if (c) c->err = msg;
  else tl_error = msg;
  return s;
}

gabp_status hip_fail(Ctx* c, hipError_t e, const char* what) {
  const std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? GABP_E_OOM : GABP_E_HIP, msg);
}

}  // namespace gabp

using namespace gabp;

namespace {

#define TRY(x)                       \
  do {                               \
    gabp_status s_ = (x);            \
    if (s_ != GABP_OK) return s_;    \
  } while (0)

gabp_status check_opts(Ctx* c, const gabp_opts& o) {
  if (o.precision != GABP_FP64 && o.precision != GABP_FP32_REFINE) return fail(c, GABP_E_ARG, "precision");
  if (o.check_every < 1) return fail(c, GABP_E_ARG, "check_every must be >= 1");
  if (o.edges_per_block != 0 && o.edges_per_block != 512 && o.edges_per_block != 1024 &&
      o.edges_per_block != 2048)
    return fail(c, GABP_E_ARG, "edges_per_block must be 0, 512, 1024 or 2048");
  if (o.inner_max_iter < 0 || o.max_outer < 0) return fail(c, GABP_E_ARG, "negative iteration cap");
  if (o.layout < 0 || o.layout > kLayoutSerial || o.reserved != 0) return fail(c, GABP_E_ARG, "layout");
  if (!(o.inner_tol > 0.0) || !std::isfinite(o.gamma) || !std::isfinite(o.loading_delta))
    return fail(c, GABP_E_ARG, "inner_tol, gamma and loading_delta must be finite (inner_tol > 0)");
  if (!(o.damping > 0.0 && o.damping <= 1.0)) return fail(c, GABP_E_ARG, "damping must lie in (0, 1]");
  if ((o.flags & GABP_FLAG_SINGLE_LOOP) && o.layout != 0 && o.layout != kLayoutCompact)
    return fail(c, GABP_E_ARG, "the single loop needs the compact layout");
  if (o.flags & GABP_FLAG_AITKEN) {
    if (o.layout != 0 && o.layout != kLayoutCompact)
      return fail(c, GABP_E_ARG, "Aitken's extrapolation needs the compact layout");
    if (o.precision != GABP_FP64 || o.gamma != 0.0 || (o.flags & GABP_FLAG_SINGLE_LOOP))
      return fail(c, GABP_E_ARG, "Aitken's extrapolation applies to the plain FP64 iteration");
  }
  if (o.flags & GABP_FLAG_STEFFENSEN) {
    if (o.layout != 0 && o.layout != kLayoutCompact)
      return fail(c, GABP_E_ARG, "Steffensen's iterations need the compact layout");
    if (o.precision != GABP_FP64 || o.gamma != 0.0 || (o.flags & (GABP_FLAG_SINGLE_LOOP | GABP_FLAG_AITKEN)))
      return fail(c, GABP_E_ARG, "Steffensen's iterations apply to the plain FP64 iteration, without Aitken's step");
  }
  return GABP_OK;
}

gabp_status common_setup(Ctx* c) {
  GABP_HIP(c, hipHostMalloc((void**)&c->st_h, 4 * sizeof(DevStatus), hipHostMallocDefault));
  GABP_HIP(c, hipHostMalloc((void**)&c->st_small_h, sizeof(DevStatus), hipHostMallocMapped | hipHostMallocCoherent));
  GABP_HIP(c, hipHostGetDevicePointer((void**)&c->st_small_d, c->st_small_h, 0));
  GABP_HIP(c, hipHostMalloc((void**)&c->st_mir_h, 3 * sizeof(DevStatus), hipHostMallocMapped | hipHostMallocCoherent));
  GABP_HIP(c, hipHostGetDevicePointer((void**)&c->st_mir_d, c->st_mir_h, 0));
  for (auto& e : c->ev) GABP_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  TRY(dev_alloc(c, (void**)&c->st_d, 2 * sizeof(DevStatus)));
  TRY(dev_alloc(c, (void**)&c->norms_d, 4 * sizeof(double)));
  GABP_HIP(c, launch_reset_status(c->st_d, 2, c->stream));
  if (c->opts.flags & GABP_FLAG_TIME_SWEEPS) {
    c->tev.resize(2 * 2048, nullptr);
    for (auto& e : c->tev) GABP_HIP(c, hipEventCreate(&e));
  }
  return GABP_OK;
}

// Buffers of the solve loops, sized for the handle's precision, for every
// layout the autotuner may pick (the unused layout's are released after it).
gabp_status alloc_solver(Ctx* c) {
  const int64_t n = c->n, E = c->E;
  const bool fp32 = c->opts.precision == GABP_FP32_REFINE;
  const size_t elt = fp32 ? sizeof(float) : sizeof(double);
  const bool serial = c->opts.layout == kLayoutSerial;
  const bool edge = !serial && !node_family(c->opts.layout);
  const bool node = !serial && c->opts.layout != kLayoutEdge;
  if (node)
    for (int i = 0; i < 3; ++i) TRY(dev_alloc(c, &c->agg_d[i], 2 * elt * n));
  if (serial) {  // one set of aggregates and of messages, updated in place
    TRY(dev_alloc(c, &c->agg_d[0], 2 * elt * n));
    TRY(dev_alloc(c, &c->bstate_d, 2 * elt * E));
    TRY(dev_alloc(c, (void**)&c->lsum_d, sizeof(double) * n));
  }
  if (c->perm_d) {  // rows renumbered: b, x and the variances in internal order
    TRY(dev_alloc(c, (void**)&c->bperm_d, sizeof(double) * n));
    TRY(dev_alloc(c, (void**)&c->xperm_d, sizeof(double) * n));
    TRY(dev_alloc(c, (void**)&c->vperm_d, sizeof(double) * n));
  }
  for (int i = 0; i < 2; ++i) {
    if (edge) {
      TRY(dev_alloc(c, &c->msg_d[i], msg_bytes((int)elt, true) * E));
      c->hmsg_d[i] = c->msg_d[i];  // h-only sweeps reuse the message buffers
    }
    TRY(dev_alloc(c, (void**)&c->x64_d[i], sizeof(double) * n));
    TRY(dev_alloc(c, (void**)&c->pt64_d[i], sizeof(double) * n));
    TRY(dev_alloc(c, (void**)&c->xo_d[i], sizeof(double) * n));
    if (fp32) TRY(dev_alloc(c, (void**)&c->x32_d[i], sizeof(float) * n));
  }
  if (node) TRY(dev_alloc(c, &c->bstate_d, bcast_state_bytes((int)elt) * E));
  if (!serial) {  // frozen precisions
    TRY(dev_alloc(c, &c->gcoef_d, std::max(bcast_coef_bytes((int)elt), elt) * E));
    TRY(dev_alloc(c, &c->inv_pt_d, elt * n));
  }
  if (fp32) TRY(dev_alloc(c, (void**)&c->rin32_d, sizeof(float) * n));
  TRY(dev_alloc(c, (void**)&c->rin64_d, sizeof(double) * n));
  TRY(dev_alloc(c, (void**)&c->din32_d, sizeof(float) * n));
  // diagonal of the inner matrix A + gamma diag(A)
  double gamma = c->opts.gamma;
  if (gamma < 0.0) {
    // automatic loading: gamma = (1 + delta) rho(|R|) - 1 from an upper bound on rho
    TRY(estimate_walk_rho(c, &c->rho_lo, &c->rho_hi, 4000, 1e-4));
    gamma = c->rho_hi >= 1.0 ? (1.0 + c->opts.loading_delta) * c->rho_hi - 1.0 : 0.0;
  }
  c->gamma_used = gamma;
  if (gamma > 0.0) {
    TRY(dev_alloc(c, (void**)&c->din64_d, sizeof(double) * n));
    GABP_HIP(c, launch_scale_diag(c->d64_d, 1.0 + gamma, c->din64_d, c->din32_d, c->n, c->stream));
    if (fp32 && (c->opts.flags & GABP_FLAG_SINGLE_LOOP)) {
      TRY(dev_alloc(c, (void**)&c->d32_d, sizeof(float) * n));
      GABP_HIP(c, launch_scale_diag(c->d64_d, 1.0, nullptr, c->d32_d, c->n, c->stream));
    }
  } else {
    c->din64_d = c->d64_d;
    GABP_HIP(c, launch_scale_diag(c->d64_d, 1.0, nullptr, c->din32_d, c->n, c->stream));
  }
  return GABP_OK;
}

void release_unused_layout(Ctx* c) {
  if (c->layout == kLayoutSerial) return;  // allocated for that layout alone
  if (node_family(c->layout)) {
    for (int i = 0; i < 2; ++i) {
      dev_free(c, c->msg_d[i]);
      c->msg_d[i] = c->hmsg_d[i] = nullptr;
    }
    if (c->layout == kLayoutNode) {  // two aggregate generations suffice
      dev_free(c, c->agg_d[2]);
      c->agg_d[2] = nullptr;
    }
  } else {
    dev_free(c, c->bstate_d);
    c->bstate_d = nullptr;
    for (int i = 0; i < 3; ++i) {
      dev_free(c, c->agg_d[i]);
      c->agg_d[i] = nullptr;
    }
  }
}

bool plain_mode(const Ctx* c) { return c->opts.precision == GABP_FP64 && c->gamma_used == 0.0 && c->opts.gamma == 0.0; }
bool single_loop_mode(const Ctx* c) { return !plain_mode(c) && (c->opts.flags & GABP_FLAG_SINGLE_LOOP); }

// The symmetric augmented matrix of Ch. 5 Sec. 5.4, [[D, B^T], [B, -gamma I]],
// assembled on the host from a validated B (m x n CSR with sorted columns).
// Rows 0..n-1 hold D_ii, then the entries of B^T in increasing row of B
// (columns n + r); rows n..n+m-1 hold row r of B, then -gamma on the diagonal,
// so every row's columns increase.
struct HostCsr {
  std::vector<int32_t> row_ptr, col;
  std::vector<double> val;
};

std::string check_rect(int32_t m, int32_t n, const std::vector<int32_t>& bp, const std::vector<int32_t>& bc,
                       const std::vector<double>& bv, const std::vector<double>& d, double gamma) {
  if (!(gamma > 0.0) || !std::isfinite(gamma)) return "gamma must be finite and > 0";
  for (int32_t i = 0; i < n; ++i)
    if (!(d[i] != 0.0) || !std::isfinite(d[i])) return "d must be finite and nonzero";
  if (bp[0] != 0) return "row_ptr[0] must be 0";
  for (int32_t r = 0; r < m; ++r)  // first, so that every row lies inside the nnz entries copied
    if (bp[r + 1] < bp[r]) return "row_ptr decreases";
  for (int32_t r = 0; r < m; ++r) {
    for (int32_t e = bp[r]; e < bp[r + 1]; ++e) {
      if (bc[e] < 0 || bc[e] >= n) return "column index out of [0, n)";
      if (e > bp[r] && bc[e] <= bc[e - 1]) return "columns of a row must increase strictly";
      if (!std::isfinite(bv[e])) return "non-finite value in B";
    }
  }
  return "";
}

HostCsr assemble_augmented(int32_t m, int32_t n, const std::vector<int32_t>& bp, const std::vector<int32_t>& bc,
                           const std::vector<double>& bv, const std::vector<double>& d, double gamma) {
  const int32_t N = n + m;
  const int64_t nnzB = bp[m];
  std::vector<int64_t> cnt(n, 0);  // entries per column of B = per row of B^T
  for (int64_t e = 0; e < nnzB; ++e) ++cnt[bc[e]];
  HostCsr K;
  K.row_ptr.assign(N + 1, 0);
  for (int32_t i = 0; i < n; ++i) K.row_ptr[i + 1] = K.row_ptr[i] + 1 + (int32_t)cnt[i];
  for (int32_t r = 0; r < m; ++r) K.row_ptr[n + r + 1] = K.row_ptr[n + r] + (bp[r + 1] - bp[r]) + 1;
  K.col.resize(K.row_ptr[N]);
  K.val.resize(K.row_ptr[N]);
  std::vector<int32_t> next(n);
  for (int32_t i = 0; i < n; ++i) {
    K.col[K.row_ptr[i]] = i;
    K.val[K.row_ptr[i]] = d[i];
    next[i] = K.row_ptr[i] + 1;
  }
  for (int32_t r = 0; r < m; ++r) {
    int32_t q = K.row_ptr[n + r];
    for (int32_t e = bp[r]; e < bp[r + 1]; ++e, ++q) {
      const int32_t c = bc[e];
      K.col[next[c]] = n + r;  // B^T entry (c, n + r)
      K.val[next[c]++] = bv[e];
      K.col[q] = c;            // B entry (n + r, c)
      K.val[q] = bv[e];
    }
    K.col[q] = n + r;
    K.val[q] = -gamma;
  }
  return K;
}

}  // namespace

extern "C" {

void gabp_default_opts(gabp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = GABP_FP64;
  o->check_every = 1;
  o->edges_per_block = 0;
  o->inner_max_iter = 10000;
  o->max_outer = 1000;
  o->flags = GABP_FLAG_REUSE_PRECISION;
  o->gamma = 0.0;
  o->loading_delta = 0.05;
  o->inner_tol = 1e-5;
  o->damping = 0.5;
}

gabp_status gabp_create(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* vals,
                        const gabp_opts* opts, hipStream_t stream, gabp_handle* out) {
  if (!out) return fail(nullptr, GABP_E_ARG, "out is NULL");
  *out = nullptr;
  if (n < 0) return fail(nullptr, GABP_E_ARG, "n < 0");
  if (n > 0 && (!row_ptr || !col_idx || !vals)) return fail(nullptr, GABP_E_ARG, "NULL CSR array");
  gabp_ctx* c = new gabp_ctx();
  c->n = n;
  c->stream = stream;
  if (opts) c->opts = *opts;
  else gabp_default_opts(&c->opts);
  gabp_status r = check_opts(c, c->opts);
  if (r == GABP_OK) r = common_setup(c);
  if (r == GABP_OK && n > 0) r = ingest(c, row_ptr, col_idx, vals, nullptr, 0);
  if (r == GABP_OK && n > 0 && c->opts.layout == kLayoutSerial) r = apply_colour_order(c, nullptr, 0);
  else if (r == GABP_OK && n > 0 && !(c->opts.flags & GABP_FLAG_NATURAL_ORDER)) r = apply_xcd_order(c);
  if (r == GABP_OK && n > 0) r = alloc_solver(c);
  if (r == GABP_OK && n > 0) r = autotune(c);
  if (r == GABP_OK && n > 0) release_unused_layout(c);
  if (r == GABP_OK) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) r = hip_fail(c, e, "hipStreamSynchronize");
  }
  if (r != GABP_OK) {
    tl_error = c->err;
    gabp_destroy(c);
    return r;
  }
  *out = c;
  return GABP_OK;
}

gabp_status gabp_solve(gabp_handle h, const double* b, double* x, double* var, double tol, int32_t max_iter,
                       gabp_info* info) {
  if (!h) return fail(nullptr, GABP_E_ARG, "NULL handle");
  Ctx* c = h;
  if (info) std::memset(info, 0, sizeof(*info));
  if (c->batched) return fail(c, GABP_E_ARG, "batched handle: use gabp_solve_batched");
  if (max_iter < 0) return fail(c, GABP_E_ARG, "max_iter < 0");
  if (std::isnan(tol)) return fail(c, GABP_E_ARG, "tol is NaN");
  if (c->n == 0) {
    if (info) info->converged = 1;
    return GABP_OK;
  }
  if (!b || !x) return fail(c, GABP_E_ARG, "NULL b or x");
  if (var && !plain_mode(c)) return fail(c, GABP_E_ARG, "variances are only available in plain FP64 mode");
  if (!plain_mode(c) && !(single_loop_mode(c) && c->opts.precision == GABP_FP64) && !(tol > 0.0))
    return fail(c, GABP_E_ARG, "the correction loop needs tol > 0");
  // renumbered handles solve in their internal numbering
  const bool perm = c->perm_d != nullptr;
  if (perm && !(c->bperm_d && c->xperm_d && c->vperm_d))
    return fail(c, GABP_E_ARG, "internal order buffers missing");
  if (perm) GABP_HIP(c, launch_gather(b, c->inv_d, c->bperm_d, c->n, c->stream));
  const double* bi = perm ? c->bperm_d : b;
  double* xi = perm ? c->xperm_d : x;
  double* vi = (perm && var) ? c->vperm_d : var;
  gabp_status r;
  if (plain_mode(c)) r = solve_plain(c, bi, xi, vi, tol, max_iter, info, true);
  else if (single_loop_mode(c) && c->opts.precision == GABP_FP64) r = solve_single_loop(c, bi, xi, tol, max_iter, info);
  else r = solve_outer(c, bi, xi, tol, max_iter, info);
  if (perm && r >= 0) {
    GABP_HIP(c, launch_gather(xi, c->perm_d, x, c->n, c->stream));
    if (var) GABP_HIP(c, launch_gather(vi, c->perm_d, var, c->n, c->stream));
    GABP_HIP(c, hipStreamSynchronize(c->stream));
  }
  return r;
}

gabp_status gabp_messages(gabp_handle h, double* P, double* hm) {
  if (!h) return fail(nullptr, GABP_E_ARG, "NULL handle");
  Ctx* c = h;
  if (c->layout == kLayoutSerial)
    return fail(c, GABP_E_ARG, "messages are exported by the synchronous layouts only");
  if (c->last_msg_round < 0 || c->opts.precision != GABP_FP64)
    return fail(c, GABP_E_ARG, "no FP64 messages from a fixed-sweep solve (tol <= 0) are held");
  if (c->E == 0) return GABP_OK;
  if (!P || !hm) return fail(c, GABP_E_ARG, "NULL output");
  double* Pc = P;  // caller's outputs
  double* hc = hm;
  if (c->slot_of_d) {  // rows renumbered: messages in internal slot order first
    if (!c->msg_tmp_d) TRY(dev_alloc(c, (void**)&c->msg_tmp_d, 2 * sizeof(double) * (size_t)c->E));
    P = c->msg_tmp_d;
    hm = c->msg_tmp_d + c->E;
  }
  if (c->last_msg_round == 0) {  // round 0: every message is zero (initial state of Alg. 2)
    GABP_HIP(c, launch_fill(P, c->E, 0.0, c->stream));
    GABP_HIP(c, launch_fill(hm, c->E, 0.0, c->stream));
  } else if (c->layout == kLayoutCompact) {
    // out^(T) recomputed from in^(T-1) and the aggregates of round T-1
    const int T = c->last_msg_round;
    const void* in_prev = (char*)c->bstate_d + ((T - 1) & 1) * 2 * sizeof(double) * (size_t)c->E;
    GABP_HIP(c, launch_cnode_out(c->n, c->off_ptr_d, c->a64_d, in_prev, c->agg_d[(T - 1) % 3], T == 1, P, hm,
                                 c->stream));
  } else if (c->layout == kLayoutNode) {
    GABP_HIP(c, launch_split_out(c->bstate_d, P, hm, c->E, c->stream));
  } else {
    GABP_HIP(c, launch_split_pairs(c->msg_d[c->last_msg_round & 1], P, hm, c->E, c->stream));
  }
  if (c->slot_of_d) {
    GABP_HIP(c, launch_scatter_slots(P, c->slot_of_d, Pc, c->E, c->stream));
    GABP_HIP(c, launch_scatter_slots(hm, c->slot_of_d, hc, c->E, c->stream));
  }
  GABP_HIP(c, hipStreamSynchronize(c->stream));
  return GABP_OK;
}

gabp_status gabp_backward(gabp_handle h, const double* x, const double* grad_x, double* grad_b,
                          double* grad_vals, double tol, int32_t max_iter, gabp_info* info) {
  if (!h) return fail(nullptr, GABP_E_ARG, "NULL handle");
  Ctx* c = h;
  if (info) std::memset(info, 0, sizeof(*info));
  if (c->batched) return fail(c, GABP_E_ARG, "batched handle");
  if (max_iter < 0 || !(tol > 0.0)) return fail(c, GABP_E_ARG, "backward needs tol > 0 and max_iter >= 0");
  if (c->n == 0) return GABP_OK;
  if (!x || !grad_x || !grad_b) return fail(c, GABP_E_ARG, "NULL x, grad_x or grad_b");
  // A is symmetric: the adjoint system A^T lambda = dL/dx is a second GaBP solve against A
  const bool perm = c->perm_d != nullptr;
  if (perm && !(c->bperm_d && c->xperm_d)) return fail(c, GABP_E_ARG, "internal order buffers missing");
  if (perm) GABP_HIP(c, launch_gather(grad_x, c->inv_d, c->bperm_d, c->n, c->stream));
  const double* gi = perm ? c->bperm_d : grad_x;
  double* li = perm ? c->xperm_d : grad_b;
  gabp_status r = plain_mode(c)         ? solve_plain(c, gi, li, nullptr, tol, max_iter, info, true)
                  : single_loop_mode(c) && c->opts.precision == GABP_FP64
                        ? solve_single_loop(c, gi, li, tol, max_iter, info)
                                        : solve_outer(c, gi, li, tol, max_iter, info);
  if (r < 0) return r;
  if (perm) {
    GABP_HIP(c, launch_gather(li, c->perm_d, grad_b, c->n, c->stream));
    if (!grad_vals) GABP_HIP(c, hipStreamSynchronize(c->stream));
  }
  if (grad_vals) {
    GABP_HIP(c, launch_grad_vals(c->row_ptr_d, c->col_d, grad_b, x, grad_vals, c->n, c->stream));
    GABP_HIP(c, hipStreamSynchronize(c->stream));
  }
  return r;
}

gabp_status gabp_plan_augmented(int32_t m, int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                const double* vals, const double* d, double gamma, int32_t* K_row_ptr,
                                int32_t* K_col, double* K_val, int64_t cap, int64_t* nnz_out) {
  if (nnz_out) *nnz_out = 0;
  if (m < 1 || n < 1 || (int64_t)n + m >= INT32_MAX) return fail(nullptr, GABP_E_ARG, "m >= 1 and n >= 1");
  if (!row_ptr || !col_idx || !vals || !d) return fail(nullptr, GABP_E_ARG, "NULL B or d");
  std::vector<int32_t> bp(row_ptr, row_ptr + m + 1);
  const int64_t nnzB = bp[m];
  if (bp[0] != 0 || nnzB < 0 || (int64_t)n + m + 2 * nnzB >= INT32_MAX)
    return fail(nullptr, GABP_E_ARG, "row_ptr[0] must be 0 and the augmented matrix must fit int32 indices");
  for (int32_t r = 0; r < m; ++r)
    if (bp[r + 1] < bp[r]) return fail(nullptr, GABP_E_ARG, "row_ptr decreases");
  std::vector<int32_t> bc(col_idx, col_idx + nnzB);
  std::vector<double> bv(vals, vals + nnzB);
  std::vector<double> dh(d, d + n);
  const std::string bad = check_rect(m, n, bp, bc, bv, dh, gamma);
  if (!bad.empty()) return fail(nullptr, GABP_E_ARG, bad);
  const HostCsr K = assemble_augmented(m, n, bp, bc, bv, dh, gamma);
  const int64_t nnzK = (int64_t)K.col.size();
  if (nnz_out) *nnz_out = nnzK;
  if (K_row_ptr) std::copy(K.row_ptr.begin(), K.row_ptr.end(), K_row_ptr);
  if (K_col || K_val) {
    if (cap < nnzK) return fail(nullptr, GABP_E_ARG, "cap below the number of stored entries of K");
    if (K_col) std::copy(K.col.begin(), K.col.end(), K_col);
    if (K_val) std::copy(K.val.begin(), K.val.end(), K_val);
  }
  return GABP_OK;
}

gabp_status gabp_create_augmented(int32_t m, int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                  const double* vals, const double* d, double gamma, const gabp_opts* opts,
                                  hipStream_t stream, gabp_handle* out) {
  if (!out) return fail(nullptr, GABP_E_ARG, "out is NULL");
  *out = nullptr;
  if (m < 1 || n < 1 || (int64_t)n + m >= INT32_MAX) return fail(nullptr, GABP_E_ARG, "m >= 1 and n >= 1");
  if (!row_ptr || !col_idx || !vals || !d) return fail(nullptr, GABP_E_ARG, "NULL B or d");
  // B and D to the host
  std::vector<int32_t> bp(m + 1);
  std::vector<double> dh(n);
  hipError_t e = hipMemcpyAsync(bp.data(), row_ptr, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dh.data(), d, sizeof(double) * n, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "copy of B");
  const int64_t nnzB = bp[m];
  if (bp[0] != 0 || nnzB < 0 || (int64_t)n + m + 2 * nnzB >= INT32_MAX)
    return fail(nullptr, GABP_E_ARG, "row_ptr[0] must be 0 and the augmented matrix must fit int32 indices");
  std::vector<int32_t> bc(nnzB);
  std::vector<double> bv(nnzB);
  if (nnzB > 0) {
    e = hipMemcpyAsync(bc.data(), col_idx, sizeof(int32_t) * nnzB, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(bv.data(), vals, sizeof(double) * nnzB, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "copy of B");
  }
  const std::string bad = check_rect(m, n, bp, bc, bv, dh, gamma);
  if (!bad.empty()) return fail(nullptr, GABP_E_ARG, bad);
  const HostCsr K = assemble_augmented(m, n, bp, bc, bv, dh, gamma);
  gabp_opts o;
  if (opts) o = *opts;
  else {
    gabp_default_opts(&o);
    o.gamma = -1.0;
  }
  // ingest as any symmetric system (the library copies what it keeps)
  const int32_t N = n + m;
  const size_t nnzK = K.col.size();
  void *rp_d = nullptr, *cl_d = nullptr, *vl_d = nullptr;
  e = hipMalloc(&rp_d, sizeof(int32_t) * (N + 1));
  if (e == hipSuccess) e = hipMalloc(&cl_d, sizeof(int32_t) * nnzK);
  if (e == hipSuccess) e = hipMalloc(&vl_d, sizeof(double) * nnzK);
  if (e == hipSuccess)
    e = hipMemcpyAsync(rp_d, K.row_ptr.data(), sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(cl_d, K.col.data(), sizeof(int32_t) * nnzK, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(vl_d, K.val.data(), sizeof(double) * nnzK, hipMemcpyHostToDevice, stream);
  gabp_status r = GABP_OK;
  if (e != hipSuccess) r = hip_fail(nullptr, e, "upload of the augmented matrix");
  gabp_handle h = nullptr;
  if (r == GABP_OK) r = gabp_create(N, (const int32_t*)rp_d, (const int32_t*)cl_d, (const double*)vl_d, &o, stream, &h);
  (void)hipStreamSynchronize(stream);
  (void)hipFree(rp_d);
  (void)hipFree(cl_d);
  (void)hipFree(vl_d);
  if (r != GABP_OK) return r;
  Ctx* c = h;
  c->aug_n = n;
  c->aug_m = m;
  r = dev_alloc(c, (void**)&c->aug_rhs_d, sizeof(double) * N);
  if (r == GABP_OK) r = dev_alloc(c, (void**)&c->aug_x_d, sizeof(double) * N);
  if (r != GABP_OK) {
    tl_error = c->err;
    gabp_destroy(h);
    return r;
  }
  *out = h;
  return GABP_OK;
}

gabp_status gabp_solve_augmented(gabp_handle hdl, const double* b, const double* h, double* x, double* z,
                                 double tol, int32_t max_iter, gabp_info* info) {
  if (!hdl) return fail(nullptr, GABP_E_ARG, "NULL handle");
  Ctx* c = hdl;
  if (info) std::memset(info, 0, sizeof(*info));
  if (c->aug_n < 0) return fail(c, GABP_E_ARG, "not a handle of gabp_create_augmented");
  if (!x) return fail(c, GABP_E_ARG, "NULL x");
  const int32_t n = c->aug_n, m = c->aug_m;
  hipStream_t s = c->stream;
  if (b) GABP_HIP(c, hipMemcpyAsync(c->aug_rhs_d, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  else GABP_HIP(c, launch_fill(c->aug_rhs_d, n, 0.0, s));
  if (h) GABP_HIP(c, hipMemcpyAsync(c->aug_rhs_d + n, h, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
  else GABP_HIP(c, launch_fill(c->aug_rhs_d + n, m, 0.0, s));
  const gabp_status r = gabp_solve(hdl, c->aug_rhs_d, c->aug_x_d, nullptr, tol, max_iter, info);
  if (r < 0) return r;
  GABP_HIP(c, hipMemcpyAsync(x, c->aug_x_d, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  if (z) GABP_HIP(c, hipMemcpyAsync(z, c->aug_x_d + n, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
  GABP_HIP(c, hipStreamSynchronize(s));
  return r;
}

gabp_status gabp_create_batched(int32_t num_sys, const int32_t* sys_row_off, const int32_t* row_ptr,
                                const int32_t* col_idx, const double* vals, const gabp_opts* opts,
                                hipStream_t stream, gabp_handle* out) {
  if (!out) return fail(nullptr, GABP_E_ARG, "out is NULL");
  *out = nullptr;
  if (num_sys < 1 || !sys_row_off || sys_row_off[0] != 0) return fail(nullptr, GABP_E_ARG, "num_sys / sys_row_off");
  for (int32_t s = 0; s < num_sys; ++s)
    if (sys_row_off[s + 1] < sys_row_off[s]) return fail(nullptr, GABP_E_ARG, "sys_row_off decreases");
  const int32_t n = sys_row_off[num_sys];
  if (n > 0 && (!row_ptr || !col_idx || !vals)) return fail(nullptr, GABP_E_ARG, "NULL CSR array");
  gabp_ctx* c = new gabp_ctx();
  c->n = n;
  c->stream = stream;
  c->batched = true;
  if (opts) c->opts = *opts;
  else {
    gabp_default_opts(&c->opts);
    c->opts.precision = GABP_FP32_REFINE;
  }
  gabp_status r = check_opts(c, c->opts);
  if (r == GABP_OK && c->opts.precision != GABP_FP32_REFINE)
    r = fail(c, GABP_E_ARG, "batched solves run FP32 messages with FP64 refinement");
  if (r == GABP_OK && c->opts.layout != 0 && c->opts.layout != kLayoutSerial)
    r = fail(c, GABP_E_ARG, "batched solves take layout 0 (synchronous) or 4 (colour-serial)");
  if (r == GABP_OK) r = common_setup(c);
  int32_t* sys_d = nullptr;
  if (r == GABP_OK) r = dev_alloc(c, (void**)&sys_d, sizeof(int32_t) * (num_sys + 1));
  if (r == GABP_OK) {
    hipError_t e = hipMemcpyAsync(sys_d, sys_row_off, sizeof(int32_t) * (num_sys + 1), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) r = hip_fail(c, e, "hipMemcpyAsync");
  }
  if (r == GABP_OK && n > 0) r = ingest(c, row_ptr, col_idx, vals, sys_d, num_sys);
  if (r == GABP_OK && n > 0 && c->opts.layout == kLayoutSerial) r = apply_colour_order(c, sys_row_off, num_sys);
  if (r == GABP_OK) r = batched_create(c, num_sys, sys_row_off);
  if (r == GABP_OK) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) r = hip_fail(c, e, "hipStreamSynchronize");
  }
  if (r != GABP_OK) {
    tl_error = c->err;
    gabp_destroy(c);
    return r;
  }
  *out = c;
  return GABP_OK;
}

gabp_status gabp_solve_batched(gabp_handle h, const int32_t* nrhs, const int64_t* rhs_off, const double* B,
                               double* X, double tol, int32_t max_iter, gabp_info* infos) {
  if (!h) return fail(nullptr, GABP_E_ARG, "NULL handle");
  Ctx* c = h;
  if (!c->batched) return fail(c, GABP_E_ARG, "not a batched handle");
  if (!nrhs || !rhs_off || !(tol > 0.0) || max_iter < 0) return fail(c, GABP_E_ARG, "arguments");
  return batched_solve(c, nrhs, rhs_off, B, X, tol, max_iter, infos);
}

gabp_status gabp_get_batch_profile(gabp_handle h, gabp_batch_profile* out) {
  if (!h || !out) return fail(h, GABP_E_ARG, "NULL argument");
  Ctx* c = h;
  if (!c->batched) return fail(c, GABP_E_ARG, "not a batched handle");
  return batched_profile(c, out);
}

gabp_status gabp_get_colours(gabp_handle h, int32_t* colour, int32_t* num_colours) {
  if (!h) return fail(nullptr, GABP_E_ARG, "NULL handle");
  Ctx* c = h;
  if (c->opts.layout != kLayoutSerial) return fail(c, GABP_E_ARG, "not a colour-serial handle (layout 4)");
  if (num_colours) *num_colours = c->ncol;
  if (colour && c->n > 0) std::memcpy(colour, c->colour_h.data(), sizeof(int32_t) * c->n);
  return GABP_OK;
}

gabp_status gabp_plan_rows(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const gabp_opts* opts,
                           int32_t* perm, int32_t* colour, int32_t* blk_row, int32_t blk_cap, int32_t* class_blk,
                           gabp_plan* plan) {
  if (n < 0 || (n > 0 && (!row_ptr || !col_idx))) return fail(nullptr, GABP_E_ARG, "n < 0 or NULL CSR array");
  gabp_ctx c;
  c.n = n;
  if (opts) c.opts = *opts;
  else gabp_default_opts(&c.opts);
  if (check_opts(&c, c.opts) != GABP_OK) return fail(nullptr, GABP_E_ARG, c.err);
  // the off-diagonal pattern, checked as gabp_create checks it
  if (n > 0 && (row_ptr[0] != 0 || row_ptr[n] < n)) return fail(nullptr, GABP_E_ARG, "row_ptr");
  c.off_ptr_h.assign((size_t)n + 1, 0);
  std::vector<int32_t> col;
  for (int32_t r = 0; r < n; ++r) {
    if (row_ptr[r + 1] < row_ptr[r]) return fail(nullptr, GABP_E_ARG, "row pointers decrease");
    int32_t prev = -1, ndiag = 0;
    for (int32_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      const int32_t j = col_idx[e];
      if (j < 0 || j >= n || j <= prev) return fail(nullptr, GABP_E_ARG, "columns unsorted, duplicated or out of range");
      prev = j;
      if (j == r) ++ndiag;
      else col.push_back(j);
    }
    if (ndiag != 1) return fail(nullptr, GABP_E_ZERO_DIAG, "a diagonal entry is missing");
    c.off_ptr_h[r + 1] = (int32_t)col.size();
    c.max_degree = std::max(c.max_degree, c.off_ptr_h[r + 1] - c.off_ptr_h[r]);
  }
  c.E = (int64_t)col.size();
  std::vector<int32_t> perm_inv;
  bool renumbered = false;
  if (n > 0 && c.opts.layout == kLayoutSerial) {
    plan_colour_order(&c, col, nullptr, 0, perm_inv);
    renumbered = true;
  } else if (n > 0 && !(c.opts.flags & GABP_FLAG_NATURAL_ORDER)) {
    renumbered = plan_xcd_order(&c, col, perm_inv);
  }
  if (renumbered) c.off_ptr_h = permuted_ptr(c.off_ptr_h, perm_inv, n);
  std::vector<int32_t> br, group_blk;
  if (n > 0) build_blocks(&c, c.opts.edges_per_block ? c.opts.edges_per_block / kBlock : 2, br, group_blk);
  const int32_t nb = n > 0 ? (int32_t)br.size() - 1 : 0;
  if (blk_row && blk_cap < nb + 1) return fail(nullptr, GABP_E_ARG, "blk_cap below num_blocks + 1");
  for (int32_t i = 0; i < n; ++i) {
    if (perm) perm[i] = renumbered ? perm_inv[i] : i;
    if (colour) colour[i] = c.colour_h.empty() ? 0 : c.colour_h[i];
  }
  if (blk_row) {
    if (n > 0) std::copy(br.begin(), br.end(), blk_row);
    else blk_row[0] = 0;
  }
  if (class_blk && c.ncol > 0) {
    const std::vector<int32_t> cb = class_blocks(&c, br, group_blk);
    std::copy(cb.begin(), cb.end(), class_blk);
  }
  if (plan) {
    plan->num_colours = c.ncol;
    plan->xcd_parts = c.nparts;
    plan->num_blocks = nb;
    plan->num_chunks = 0;
    if (n > 0) {
      std::vector<LongRow> lr;
      std::vector<ChunkRef> xc;
      std::vector<int32_t> xb;
      plan_long_rows(c.off_ptr_h, br, nb, c.opts.edges_per_block ? c.opts.edges_per_block / kBlock : 2, lr, xc, xb);
      plan->num_chunks = (int32_t)xc.size();
    }
  }
  return GABP_OK;
}

gabp_status gabp_get_props(gabp_handle h, gabp_props* p) {
  if (!h || !p) return fail(h, GABP_E_ARG, "NULL argument");
  Ctx* c = h;
  p->n = c->n;
  p->num_offdiag = c->E;
  p->edges_per_block = c->K * kBlock;
  p->num_blocks = c->nblk;
  p->layout = c->layout;
  p->xcd_parts = c->nparts;
  p->rho_lo = c->rho_lo;
  p->rho_hi = c->rho_hi;
  p->gamma = c->gamma_used;
  p->max_degree = c->max_degree;
  p->precision = c->opts.precision;
  p->device_bytes = c->device_bytes;
  return GABP_OK;
}

void gabp_destroy(gabp_handle h) {
  if (!h) return;
  gabp_ctx* c = h;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  batched_destroy(c);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->st_h) (void)hipHostFree(c->st_h);
  if (c->st_small_h) (void)hipHostFree(c->st_small_h);
  if (c->st_mir_h) (void)hipHostFree(c->st_mir_h);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->tev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

const char* gabp_last_error(gabp_handle h) {
  if (!h) return tl_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
