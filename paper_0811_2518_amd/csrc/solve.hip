// Host drivers: the synchronous sweep loop, the outer correction loop
// (iterative refinement / diagonal loading of Ch. 5), the adjoint solve and
// the block-size autotuner.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

#include "gabp_internal.h"

namespace gabp {

namespace {

struct RunCfg {
  bool honly = false;           // frozen precisions, h-only sweeps
  const void* rhs = nullptr;    // T [n]
  const void* diag = nullptr;   // T [n]
  const double* rhs_norm = nullptr;
  double tol = 0.0;             // <= 0: exactly max_iter sweeps
  int max_iter = 0;
  int check_every = 1;
  void* x2[2] = {nullptr, nullptr};   // T [n] x by round parity
  void* pt2[2] = {nullptr, nullptr};  // T [n] P~ by round parity (nullable)
  DevStatus* st = nullptr;
  // single-loop correction (compact layout): damped feedback of the means
  // into the prior potentials, residual checked against chk_diag
  bool feedback = false;
  double damp = 0.5;
  const void* chk_diag = nullptr;     // T [n]
  // Aitken's extrapolation (compact layout, FP64): every round's means are
  // written, the fused check is off, and after the sweep of round t the
  // estimate y_t is formed and its residual checked in its place
  double* ait_y = nullptr;            // [n] nullable: plain checks
  double* ait_hist = nullptr;         // [n]
  // Steffensen's iterations (compact layout, FP64): cycles of two sweeps;
  // after each, the extrapolated means replace those of the cycle's last
  // round and start the next cycle; only cycle ends are checked
  double* stf_start = nullptr;        // [n] nullable: no restarts
  // compact layout with a tolerance: the sweeps write no means; the caller
  // forms x of the returned round from that round's aggregate record, which
  // the three rotating buffers still hold when the run ends
  bool x_at_end = false;
  // the caller freezes the precisions of the last computed round after the
  // run, so the run must end with the sweep that checks the returned round
  bool keep_held = false;
  // an inner solve of the refinement (compact layout): once the residuals
  // give a decay rate, checks of rounds it places well above the tolerance
  // are left out, so the run stops at the first checked round that meets it
  bool sparse_checks = false;
};

template <typename T>
const T* coef_array(const Ctx* c) {
  if constexpr (sizeof(T) == 8) return (const T*)c->a64_d;
  else return (const T*)c->a32_d;
}

// Host-side polling of the device status: after each chunk of sweeps the
// status reaches pinned memory, either written there by the chunk's finish
// kernels (mirrored) or by a copy; the host waits for the previous chunk
// while the current one runs.  Returns true once the device reported
// convergence or failure.
struct Poller {
  int pending = -1, slot = 0;
  bool from_mirror[2] = {false, false};
  gabp_status err = GABP_OK;
  DevStatus seen{};  // the last status observed on the host
  bool have = false;
  // where the finish kernels of the current chunk write the status
  DevStatus* mirror(const Ctx* c) const { return c->st_mir_d + slot; }
  bool read(Ctx* c, int q) {
    hipError_t e = hipEventSynchronize(c->ev[q]);
    if (e != hipSuccess) {
      err = hip_fail(c, e, "status poll");
      return true;
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    seen = from_mirror[q] ? c->st_mir_h[q] : c->st_h[q];
    have = true;
    return seen.done != 0;
  }
  // mirrored: the chunk's last finish kernel wrote the status to mirror(c)
  bool step(Ctx* c, const DevStatus* st, bool mirrored = false) {
    hipError_t e = hipSuccess;
    if (!mirrored) e = hipMemcpyAsync(&c->st_h[slot], st, sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream);
    from_mirror[slot] = mirrored;
    if (e == hipSuccess) e = hipEventRecord(c->ev[slot], c->stream);
    if (e != hipSuccess) {
      err = hip_fail(c, e, "status poll");
      return true;
    }
    const bool done = pending >= 0 && read(c, pending);
    pending = slot;
    slot ^= 1;
    return done || err != GABP_OK;
  }
  // wait for the chunk just polled as well
  bool drain(Ctx* c) { return pending >= 0 && read(c, pending); }
};

// A sweep loop has ended: keep the status its poller observed.  Once done is
// set, every later sweep and finish kernel returns at once, so that status is
// final and the caller need not read it again.
gabp_status finish_run(Ctx* c, const Poller& p) {
  c->run_seen = p.seen;
  c->run_seen_final = p.err == GABP_OK && p.have && p.seen.done != 0;
  return p.err;
}

// Size of the next chunk of sweeps.  The first chunk reaches the sweep that
// checks the second checked round; the second has the same size; without a
// usable history the chunks then double up to 16.  Once two checked rounds have been observed (the device
// status carries the last two), the relative residual's decay rate predicts
// the round that reaches tol, and the chunk only covers the sweeps up to the
// one that checks that round (a zero chunk just polls the sweeps already
// queued), so few early-return sweeps are queued past convergence.
struct ChunkPlan {
  int chunk = 2;
  double rel0 = -1.0, rel1 = -1.0;
  int round0 = -1, round1 = -1;
  int idle = 0;
  // the round predicted to meet the tolerance with a margin of 10% in the
  // residual (checking every round), else -1; near convergence the residual
  // of GaBP falls by a steady factor per round (on G(n, 4n), 0.377 with
  // extrapolations over eight rounds within 1%)
  int pass_round = -1;
  // the round predicted to meet the tolerance (no margin), else -1
  int need_round = -1;
  int first(int lag, int check_every) {
    chunk = std::min(16, 2 * std::max(1, check_every) + lag);
    return chunk;
  }
  int next(const Poller& p, int queued_through, int lag, int check_every, double tol) {
    // no status seen yet: keep the first size (a short solve, such as an inner
    // solve of a few sweeps, then queues few sweeps past its end)
    int c = p.have ? std::min(chunk * 2, 16) : chunk;
    if (p.have && p.seen.last_round > round1) {
      if (p.seen.prev_round >= 0) {
        rel0 = p.seen.prev_rel;
        round0 = p.seen.prev_round;
      } else {
        rel0 = rel1;
        round0 = round1;
      }
      rel1 = p.seen.last_rel;
      round1 = p.seen.last_round;
    }
    pass_round = -1;
    need_round = -1;
    if (tol > 0.0 && round0 >= 0 && round1 > round0 && rel0 > 0.0 && rel1 > tol && rel1 < rel0) {
      const double rate = std::pow(rel1 / rel0, 1.0 / (round1 - round0));
      if (rate < 1.0) {
        const double m = std::ceil(std::log(tol / rel1) / std::log(rate));
        if (m < 1e6) {
          const int ce = std::max(1, check_every);
          int need = round1 + std::max(1, (int)m);
          need = ((need + ce - 1) / ce) * ce;  // the next checked round at or after it
          need_round = need;
          c = std::max(0, std::min(16, need + lag - queued_through));
          if (ce == 1 && rel1 * std::pow(rate, (double)(need - round1)) <= 0.9 * tol) pass_round = need;
        }
      }
    }
    if (c == 0 && ++idle > 1) c = 1;  // never poll twice without queueing work
    if (c > 0) idle = 0;
    chunk = std::max(c, 1);
    return c;
  }
};

template <typename T>
void start_timed(Ctx* c, bool timed, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (timed && c->tev_used + 2 <= (int)c->tev.size()) {
    *e0 = c->tev[c->tev_used];
    *e1 = c->tev[c->tev_used + 1];
    c->tev_used += 2;
  }
}

// Reverse-index layout.  Sweep t produces the messages of round t and the
// means x of round t-1, and checks x of round t-2 (its neighbours' means
// arrive inside the gathered records); rounds 1..M, then the aggregates of
// round M and a residual-only launch for round M.
template <typename T>
gabp_status run_edge(Ctx* c, const RunCfg& cfg) {
  hipStream_t s = c->stream;
  const bool exact = cfg.tol <= 0.0;
  const int M = cfg.max_iter;
  const int ce = std::max(1, cfg.check_every);
  auto in_set = [&](int j) { return j == M || (j % ce) == 0; };

  SweepArgs<T> a{};
  a.blk_row = c->blk_row_d;
  a.off_ptr = c->off_ptr_d;
  a.off_col = c->off_col_d;
  a.rev = c->rev_d;
  a.a = coef_array<T>(c);
  a.diag = (const T*)cfg.diag;
  a.rhs = (const T*)cfg.rhs;
  a.gcoef = (const T*)c->gcoef_d;
  a.inv_pt = (const T*)c->inv_pt_d;
  a.partials = c->partials_d;
  a.st = cfg.st;
  a.rhs_norm = cfg.rhs_norm;
  a.nblk = c->nblk;
  a.tol = exact ? -1.0 : cfg.tol;
  GABP_HIP(c, launch_reset_status(cfg.st, 1, s));

  const int main_mode = cfg.honly ? kHOnly : kJoint;
  const int last = M + 2;
  Poller poll;
  ChunkPlan plan;
  int t = 1, chunk = plan.first(2, ce);
  bool stop = false;
  while (t <= last && !stop) {
    const int tend = std::min(last, t + chunk - 1);
    for (; t <= tend; ++t) {
      int mode;
      if (t <= M) mode = main_mode;
      else if (t == M + 1) mode = cfg.honly ? kHOnly : kAgg;
      else mode = kResid;
      const int j = t - 1;
      SweepArgs<T> k = a;
      k.zero_in = (t == 1);
      k.min = c->msg_d[(t - 1) & 1];
      k.mout = c->msg_d[t & 1];
      const bool wx = (mode != kResid) && (exact ? (t == M + 1) : in_set(j));
      k.xout = wx ? (T*)cfg.x2[j & 1] : nullptr;
      k.ptout = (wx && cfg.pt2[0]) ? (T*)cfg.pt2[j & 1] : nullptr;
      const bool ck = (t >= 2) && (exact ? (t == M + 2) : in_set(t - 2));
      k.check = ck ? 1 : 0;
      k.xchk = (const T*)cfg.x2[(t - 2) & 1];
      k.round_checked = t - 2;
      if (mode == kResid && !ck) continue;
      hipEvent_t e0, e1;
      start_timed<T>(c, (c->opts.flags & GABP_FLAG_TIME_SWEEPS) && mode == main_mode && ck, &e0, &e1);
      if (e0) c->timed_mode = cfg.honly ? 1 : 0;
      GABP_HIP(c, launch_sweep<T>(mode, c->K, k, s, e0, e1));
      if (ck)
        GABP_HIP(c, launch_check_finish(c->partials_d, c->nblk, cfg.st, cfg.rhs_norm, k.tol, t - 2, nullptr,
                                        true, s));
    }
    stop = poll.step(c, cfg.st);
    chunk = plan.next(poll, t - 1, 2, ce, exact ? -1.0 : cfg.tol);
  }
  return finish_run(c, poll);
}

// Node-broadcast layout.  Sweep t publishes the aggregates of round t (and
// the means x of round t) and checks round t-1, whose neighbour means come
// with the gathered aggregates; rounds 1..M, then a residual-only launch for
// round M.
template <typename T>
gabp_status run_node(Ctx* c, const RunCfg& cfg) {
  hipStream_t s = c->stream;
  const bool exact = cfg.tol <= 0.0;
  const int M = cfg.max_iter;
  const int ce = std::max(1, cfg.check_every);
  auto in_set = [&](int j) { return j == M || (j % ce) == 0; };

  BcastArgs<T> a{};
  a.blk_row = c->blk_row_d;
  a.off_ptr = c->off_ptr_d;
  a.col = c->off_col_d;
  a.a = coef_array<T>(c);
  a.diag = (const T*)cfg.diag;
  a.rhs = (const T*)cfg.rhs;
  a.state = c->bstate_d;
  a.coef = c->gcoef_d;
  a.inv_pt = (const T*)c->inv_pt_d;
  a.partials = c->partials_d;
  a.st = cfg.st;
  a.nblk = c->nblk;
  a.honly_nodes = cfg.honly ? 1 : 0;
  const double tol = exact ? -1.0 : cfg.tol;
  GABP_HIP(c, launch_reset_status(cfg.st, 1, s));

  const int main_mode = cfg.honly ? kHOnly : kJoint;
  const int last = M + 1;
  Poller poll;
  ChunkPlan plan;
  int t = 1, chunk = plan.first(1, ce);
  bool stop = false;
  while (t <= last && !stop) {
    const int tend = std::min(last, t + chunk - 1);
    for (; t <= tend; ++t) {
      const int mode = (t <= M) ? main_mode : kResid;
      BcastArgs<T> k = a;
      k.zero_in = (t == 1);
      k.aold = c->agg_d[(t - 1) & 1];
      k.anew = c->agg_d[t & 1];
      k.xold = (const T*)cfg.x2[(t - 1) & 1];
      if (mode != kResid) {
        const bool wx = exact ? t == M : in_set(t);
        k.xout = wx ? (T*)cfg.x2[t & 1] : nullptr;
        k.ptout = (wx && cfg.pt2[0]) ? (T*)cfg.pt2[t & 1] : nullptr;
      }
      if (t == 1 && (exact ? M == 0 : in_set(0))) {
        k.xout_prev = (T*)cfg.x2[0];
        k.ptout_prev = cfg.pt2[0] ? (T*)cfg.pt2[0] : nullptr;
      }
      const bool ck = exact ? (t == M + 1) : in_set(t - 1);
      k.check = ck ? 1 : 0;
      if (mode == kResid && !ck) continue;
      hipEvent_t e0, e1;
      start_timed<T>(c, (c->opts.flags & GABP_FLAG_TIME_SWEEPS) && mode == main_mode && ck, &e0, &e1);
      if (e0) c->timed_mode = cfg.honly ? 1 : 0;
      GABP_HIP(c, launch_bcast<T>(mode, c->K, k, s, e0, e1));
      if (ck)
        GABP_HIP(c, launch_check_finish(c->partials_d, c->nblk, cfg.st, cfg.rhs_norm, tol, t - 1, nullptr,
                                        true, s));
    }
    stop = poll.step(c, cfg.st);
    chunk = plan.next(poll, t - 1, 1, ce, exact ? -1.0 : cfg.tol);
  }
  return finish_run(c, poll);
}

// Compact layout: the incoming messages of even and odd rounds live in the
// two halves of the slot-state buffer (in^(t) overwrites in^(t-2) in place);
// the aggregates rotate through three buffers by round mod 3.
template <typename T>
void* cin_buf(const Ctx* c, int parity) {
  return (char*)c->bstate_d + (parity & 1) * 2 * sizeof(T) * (size_t)c->E;
}

// The partition's long rows and their chunk workgroups.
template <typename T>
void set_long_rows(const Ctx* c, CnodeArgs<T>& k) {
  k.longs = c->longs_d;
  k.xch = c->xch_d;
  k.lpart = c->lpart_d;
  k.nlong = c->nlong;
  k.nxch = c->nxch;
}

// Compact node layout: like run_node, sweep t publishes round t and checks
// round t-1; rounds 1..M, then a residual-only launch for round M.
template <typename T>
gabp_status run_cnode(Ctx* c, const RunCfg& cfg) {
  hipStream_t s = c->stream;
  const bool exact = cfg.tol <= 0.0;
  const int M = cfg.max_iter;
  const int ce = std::max(1, cfg.check_every);
  auto in_set = [&](int j) { return j == M || (j % ce) == 0; };
  const bool ait = cfg.ait_y != nullptr;
  const bool stf = cfg.stf_start != nullptr;
  if ((ait || stf) && sizeof(T) != 8) return fail(c, GABP_E_ARG, "Aitken's and Steffensen's steps run in FP64");
  if (stf && (M < 2 || (M & 1))) return fail(c, GABP_E_ARG, "internal: Steffensen cycles need an even max_iter >= 2");
  // Steffensen: only the ends of cycles (even rounds >= 2) are checked
  auto checked = [&](int j) { return !stf || (j >= 2 && (j & 1) == 0); };
  const int lag = ait ? 0 : 1;  // sweep t checks round t (Aitken) or t-1 (fused)
  OuterArgs ra{};               // residual of the Aitken estimate
  ra.blk_row = c->blk_row_d;
  ra.off_ptr = c->off_ptr_d;
  ra.off_col = c->off_col_d;
  ra.a = c->a64_d;
  ra.diag = c->d64_d;
  ra.b = (const double*)cfg.rhs;
  ra.xnew = cfg.ait_y;
  ra.partials = c->partials_d;
  ra.nblk = c->nblk;
  ra.n = c->n;
  ra.gate = cfg.st;  // no residual of y once the solve has ended

  CnodeArgs<T> a{};
  a.blk_row = c->blk_row_d;
  a.blk_e0 = c->blk_e0_d;
  a.off_ptr = c->off_ptr_d;
  a.col = c->off_col_d;
  a.a = coef_array<T>(c);
  a.diag = (const T*)cfg.diag;
  a.rhs = (const T*)cfg.rhs;
  a.coef = c->gcoef_d;
  a.inv_pt = (const T*)c->inv_pt_d;
  a.partials = c->partials_d;
  a.st = cfg.st;
  a.nblk = c->nblk;
  set_long_rows<T>(c, a);
  a.honly_nodes = cfg.honly ? 1 : 0;
  a.feedback = cfg.feedback ? 1 : 0;
  a.damp = (T)cfg.damp;
  a.chk_diag = (const T*)cfg.chk_diag;
  const double tol = exact ? -1.0 : cfg.tol;

  // round 0: the prior as aggregate record, (A_ii, b_i) or (1 / P~_i, b_i);
  // the same launch resets the run's status
  GABP_HIP(c, launch_cnode_prior<T>(c->n, cfg.honly ? (const T*)c->inv_pt_d : (const T*)cfg.diag,
                                    (const T*)cfg.rhs, c->agg_d[0], s, cfg.st));
  const int main_mode = cfg.honly ? kHOnly : kJoint;
  // test aid: stale buffers filled with NaN around every sweep
  const bool poison = (c->opts.flags & GABP_FLAG_POISON_STALE) && c->E > 0;
  const size_t half = 2 * sizeof(T) * (size_t)c->E;
  if (poison && !c->poison_save_d) {
    const gabp_status r = dev_alloc(c, &c->poison_save_d, 2 * sizeof(double) * (size_t)c->E);
    if (r != GABP_OK) return r;
  }
  const int last = M + 1;
  Poller poll;
  ChunkPlan plan;
  int t = 1, chunk = plan.first(lag, ce);
  bool stop = false;
  // Predicted last check: when the planner expects round t-1 to meet the
  // tolerance with a margin, launch t is the residual-only mode (the
  // neighbour gathers and 12 B per slot instead of a full sweep) and the
  // chunk ends there; only if that check fails does sweep t follow, without
  // repeating the check.  Same rounds, same checks, same results.
  const bool can_predict = !exact && !ait && !stf && !poison && !cfg.feedback && !cfg.keep_held && lag == 1;
  const bool predict_all = (c->opts.flags & GABP_FLAG_PREDICT_ALL) != 0;  // test aid
  int checked_ahead = -1;  // position whose check a residual-only launch has already made
  // Sparse checks (inner solves of the refinement): rounds 0-2 are checked
  // for the decay rate, later rounds only from one before the predicted one
  // on, and at least every fourth round.  The stop then falls on the first
  // checked round that meets the tolerance; the test aid above checks all.
  const bool sparse = cfg.sparse_checks && !exact && !ait && !stf && !cfg.feedback && !cfg.keep_held && ce == 1 &&
                      !predict_all;
  int last_ck = -1;  // last round whose check has been queued
  // the finish kernels of a chunk leave the status in pinned memory (not with
  // Aitken's extra finish, which checks y with its own limit)
  const bool mirror_ok = !ait;
  while (t <= last && !stop) {
    const int tend = std::min(last, t + chunk - 1);
    bool predicted_end = false;
    bool mirrored = false;  // the last launch of the chunk is a mirrored finish
    DevStatus* mir = mirror_ok ? poll.mirror(c) : nullptr;
    for (; t <= tend; ++t) {
      const int mode = (t <= M) ? main_mode : kResid;
      if (ait && mode == kResid) continue;
      if (can_predict && mode == main_mode && t >= 2 && (t - 1 == plan.pass_round || predict_all) &&
          checked_ahead != t && in_set(t - 1)) {
        CnodeArgs<T> k = a;
        k.second = (t == 2);
        k.cin = cin_buf<T>(c, t);
        k.agg1 = c->agg_d[(t - 1) % 3];
        k.agg2 = c->agg_d[(t + 1) % 3];
        k.anew = c->agg_d[t % 3];
        k.check = 1;
        GABP_HIP(c, launch_cnode<T>(kResid, c->K, k, s, nullptr, nullptr));
        GABP_HIP(c, launch_check_finish(c->partials_d, c->nblk, cfg.st, cfg.rhs_norm, tol, t - 1, nullptr,
                                        true, s, kDivergeLimit, mir));
        mirrored = mir != nullptr;
        checked_ahead = t;
        last_ck = t - 1;
        predicted_end = true;
        break;  // t stays: sweep t runs only if the check fails
      }
      CnodeArgs<T> k = a;
      k.first = (t == 1);
      k.second = (t == 2);
      k.cin = cin_buf<T>(c, t);
      k.agg1 = c->agg_d[(t - 1) % 3];
      k.agg2 = c->agg_d[(t + 1) % 3];  // round t-2
      k.anew = c->agg_d[t % 3];
      if (mode != kResid) {
        const bool wx = ait || stf || (exact ? t == M : (in_set(t) && !cfg.x_at_end));
        k.xout = wx ? (T*)cfg.x2[t & 1] : nullptr;
        k.ptout = (wx && cfg.pt2[0]) ? (T*)cfg.pt2[t & 1] : nullptr;
      }
      if (t == 1 && (ait || stf || (exact ? M == 0 : (in_set(0) && !cfg.x_at_end)))) {
        k.xout_prev = stf ? (T*)cfg.stf_start : (T*)cfg.x2[0];  // Steffensen: round 0 starts cycle 1
        k.ptout_prev = cfg.pt2[0] ? (T*)cfg.pt2[0] : nullptr;
      }
      bool ck = !ait && (exact ? (t == M + 1) : (in_set(t - 1) && checked(t - 1))) && checked_ahead != t;
      if (ck && sparse && mode == main_mode) {
        const int j = t - 1;
        ck = j <= 2 || plan.need_round < 0 || j >= plan.need_round - 1 || j - last_ck >= 4;
      }
      if (ck) last_ck = t - 1;
      k.check = ck ? 1 : 0;
      if (mode == kResid && !ck) continue;
      void* other = poison ? cin_buf<T>(c, t + 1) : nullptr;  // in^(t-1): not sweep t's to touch
      if (poison) {
        GABP_HIP(c, hipMemcpyAsync(c->poison_save_d, other, half, hipMemcpyDeviceToDevice, s));
        GABP_HIP(c, launch_poison(other, half, cfg.st, s));
        GABP_HIP(c, launch_poison(k.anew, 2 * sizeof(T) * (size_t)c->n, cfg.st, s));  // round t-3
      }
      hipEvent_t e0, e1;
      start_timed<T>(c, (c->opts.flags & GABP_FLAG_TIME_SWEEPS) && mode == main_mode && (ck || ait), &e0, &e1);
      if (e0) c->timed_mode = cfg.honly ? 1 : 0;
      GABP_HIP(c, launch_cnode<T>(mode, c->K, k, s, e0, e1));
      mirrored = false;
      if (poison) GABP_HIP(c, hipMemcpyAsync(other, c->poison_save_d, half, hipMemcpyDeviceToDevice, s));
      if (ck) {
        GABP_HIP(c, launch_check_finish(c->partials_d, c->nblk, cfg.st, cfg.rhs_norm, tol, t - 1, nullptr,
                                        true, s, kDivergeLimit, mir));
        mirrored = mir != nullptr;
      }
      if (stf && mode != kResid && t >= 2 && (t & 1) == 0)  // end of a cycle: y replaces x_t
        GABP_HIP(c, launch_steffensen((const double*)cfg.x2[(t - 1) & 1], (double*)cfg.x2[t & 1], cfg.stf_start,
                                      c->agg_d[t % 3], cfg.st, c->n, s));
      if (ait) {
        // means of rounds t-2 (history), t-1 and t; y_t on the checked rounds
        const bool wy = t >= 2 && (exact ? t == M : in_set(t));
        GABP_HIP(c, launch_aitken((const double*)cfg.x2[(t - 1) & 1], (const double*)cfg.x2[t & 1],
                                  cfg.ait_hist, cfg.ait_y, cfg.st, wy ? 1 : 0, c->n, s));
        if (wy && !exact) {
          GABP_HIP(c, launch_outer_only(c->K, ra, s));
          GABP_HIP(c, launch_check_finish(c->partials_d, c->nblk, cfg.st, cfg.rhs_norm, tol, t, nullptr, true,
                                          s, INFINITY));
        }
      }
    }
    stop = poll.step(c, cfg.st, mirrored);
    if (predicted_end && !stop) stop = poll.drain(c);  // wait for the predicted check itself
    chunk = plan.next(poll, t - 1, lag, ce, exact ? -1.0 : cfg.tol);
  }
  return finish_run(c, poll);
}

// Colour-serial layout: sweep t updates the colour classes in turn (one
// launch each) and checks the means of sweep t-1; sweeps 1..M, then a
// residual-only launch for sweep M.  Sweep 0 (the prior) is checked only
// when it is the last allowed sweep.
template <typename T>
gabp_status run_serial(Ctx* c, const RunCfg& cfg) {
  hipStream_t s = c->stream;
  const bool exact = cfg.tol <= 0.0;
  const int M = cfg.max_iter;
  const int ce = std::max(1, cfg.check_every);
  auto in_set = [&](int j) { return j == M || (j % ce) == 0; };
  const double tol = exact ? -1.0 : cfg.tol;
  // the class launches must tile the workgroup partition exactly
  bool tiled = (int)c->colour_blk.size() == c->ncol + 1 && (int)c->colour_start.size() == c->ncol + 1 &&
               c->ncol > 0 && c->colour_blk[0] == 0 && c->colour_blk[c->ncol] == c->nblk;
  for (int q = 0; tiled && q < c->ncol; ++q) tiled = c->colour_blk[q] <= c->colour_blk[q + 1];
  // and the classes' chunk workgroups the chunk list
  tiled = tiled && (int)c->long_xch0.size() == c->ncol + 1 && c->long_xch0[0] == 0 &&
          c->long_xch0[c->ncol] == c->nxch;
  for (int q = 0; tiled && q < c->ncol; ++q) tiled = c->long_xch0[q] <= c->long_xch0[q + 1];
  if (!tiled) return fail(c, GABP_E_ARG, "colour classes do not tile the workgroup partition");

  SerialArgs<T> a{};
  a.blk_row = c->blk_row_d;
  a.blk_e0 = c->blk_e0_d;
  a.off_ptr = c->off_ptr_d;
  a.col = c->off_col_d;
  a.a = coef_array<T>(c);
  a.diag = (const T*)cfg.diag;
  a.rhs = (const T*)cfg.rhs;
  a.out = c->bstate_d;
  a.agg = c->agg_d[0];
  a.lsum = c->lsum_d;
  a.partials = c->partials_d;
  a.st = cfg.st;
  a.longs = c->longs_d;
  a.xch = c->xch_d;
  a.lpart = c->lpart_d;
  GABP_HIP(c, launch_reset_status(cfg.st, 1, s));

  if (M == 0) {  // the prior means b_i / P_ii
    GABP_HIP(c, launch_serial_prior_x<T>(c->n, a.diag, a.rhs, (T*)cfg.x2[0], cfg.pt2[0] ? (T*)cfg.pt2[0] : nullptr,
                                         s));
    if (!exact) {
      GABP_HIP(c, launch_cnode_prior<T>(c->n, a.diag, a.rhs, a.agg, s));
      SerialArgs<T> k = a;
      k.blk0 = 0;
      k.nblk = c->nblk;
      k.xch0 = 0;
      k.nxch = c->nxch;
      k.check = 1;
      GABP_HIP(c, launch_serial<T>(k, c->K, true, s));
      GABP_HIP(c, launch_check_finish(c->partials_d, c->nblk, cfg.st, cfg.rhs_norm, tol, 0, nullptr, true, s));
    }
    return GABP_OK;
  }

  const int last = M + 1;
  Poller poll;
  ChunkPlan plan;
  int t = 1, chunk = plan.first(1, ce);
  bool stop = false;
  while (t <= last && !stop) {
    const int tend = std::min(last, t + chunk - 1);
    for (; t <= tend; ++t) {
      const bool ck = exact ? (t == M + 1) : (t >= 2 && in_set(t - 1));
      if (t == M + 1) {  // residual of sweep M, every node at sweep M
        if (!ck) continue;
        SerialArgs<T> k = a;
        k.blk0 = 0;
        k.nblk = c->nblk;
        k.xch0 = 0;
        k.nxch = c->nxch;
        k.check = 1;
        GABP_HIP(c, launch_serial<T>(k, c->K, true, s));
      } else {
        const bool wx = exact ? t == M : in_set(t);
        hipEvent_t e0, e1;
        start_timed<T>(c, (c->opts.flags & GABP_FLAG_TIME_SWEEPS) && ck, &e0, &e1);
        if (e0) {
          c->timed_mode = 0;
          GABP_HIP(c, hipEventRecord(e0, s));
        }
        for (int q = 0; q < c->ncol; ++q) {
          SerialArgs<T> k = a;
          k.blk0 = c->colour_blk[q];
          k.nblk = c->colour_blk[q + 1] - c->colour_blk[q];
          k.xch0 = c->long_xch0[q];
          k.nxch = c->long_xch0[q + 1] - c->long_xch0[q];
          k.lo = c->colour_start[q];
          k.hi = c->colour_start[q + 1];
          k.first = (t == 1);
          k.check = ck ? 1 : 0;
          k.wl = (!exact && t < M && in_set(t)) ? 1 : 0;
          k.xout = wx ? (T*)cfg.x2[t & 1] : nullptr;
          k.ptout = (wx && cfg.pt2[0]) ? (T*)cfg.pt2[t & 1] : nullptr;
          GABP_HIP(c, launch_serial<T>(k, c->K, false, s));
        }
        if (e1) GABP_HIP(c, hipEventRecord(e1, s));
      }
      if (ck)
        GABP_HIP(c, launch_check_finish(c->partials_d, c->nblk, cfg.st, cfg.rhs_norm, tol, t - 1, nullptr, true, s));
    }
    stop = poll.step(c, cfg.st);
    chunk = plan.next(poll, t - 1, 1, ce, exact ? -1.0 : cfg.tol);
  }
  return finish_run(c, poll);
}

// The whole plain FP64 iteration in one launch (small.hip), leaving the
// state of the multi-launch compact path: the means (and P~) of the returned
// round by parity, the incoming messages of the last two rounds and the
// aggregates of the last three, and the status the finish kernels would leave.
gabp_status run_small(Ctx* c, const RunCfg& cfg, double* x, double* var) {
  SmallArgs a{};
  a.n = c->n;
  a.E = (int32_t)c->E;
  a.off_ptr = c->off_ptr_d;
  a.col = c->off_col_d;
  a.a = c->a64_d;
  a.diag = (const double*)cfg.diag;
  a.rhs = (const double*)cfg.rhs;
  a.rhs_norm = nullptr;  // ||b|| formed in the kernel
  a.max_deg = c->max_degree;
  a.x_direct = x;
  a.var_direct = var;
  a.tol = cfg.tol;
  a.max_iter = cfg.max_iter;
  a.check_every = cfg.check_every;
  a.st = c->st_small_d;  // the status goes straight to pinned host memory (no copy launch)
  DevStatus blank{};     // as the status reset leaves it, should the kernel not write
  blank.conv_round = blank.last_round = blank.prev_round = -1;
  blank.last_rel = blank.prev_rel = -1.0;
  *c->st_small_h = blank;
  // the messages and aggregates are left in the handle only where something
  // reads them later: the frozen-precision pass of the reuse flag, and
  // gabp_messages after a fixed-sweep solve (x and the variances go straight
  // to the caller)
  if (cfg.tol <= 0.0 || (c->opts.flags & GABP_FLAG_REUSE_PRECISION)) {
    a.cin_out = c->bstate_d;
    for (int q = 0; q < 3; ++q) a.agg_out[q] = c->agg_d[q];
  }
  c->run_seen_final = false;
  GABP_HIP(c, launch_small(a, c->stream));
  return GABP_OK;
}

// Plain FP64 solves of small compact-layout handles take the one-launch path.
bool use_small(const Ctx* c, const RunCfg& cfg) {
  return c->layout == kLayoutCompact && !cfg.honly && !cfg.feedback && !cfg.ait_y && !cfg.stf_start &&
         !(c->opts.flags &
           (GABP_FLAG_MULTI_LAUNCH | GABP_FLAG_TIME_SWEEPS | GABP_FLAG_POISON_STALE | GABP_FLAG_PREDICT_ALL)) &&
         (small_fits(c->n, c->E) || small_rows_fit(c->n, c->max_degree));
}

template <typename T>
gabp_status run_sweeps(Ctx* c, const RunCfg& cfg) {
  c->run_seen_final = false;
  if (c->layout == kLayoutSerial) return run_serial<T>(c, cfg);
  if (c->layout == kLayoutCompact) return run_cnode<T>(c, cfg);
  return c->layout == kLayoutNode ? run_node<T>(c, cfg) : run_edge<T>(c, cfg);
}

// Latest round whose messages are held after a solve stopped at round
// `conv` (or ran out at max_iter): sweeps past convergence return at once, so
// the edge layout (lagged by two) holds round conv+2, the node layouts conv+1.
int held_round(const Ctx* c, int conv, int M) {
  if (conv < 0) return M;
  return std::min(conv + (node_family(c->layout) ? 1 : 2), M);
}

// Sum the durations of the timed sweeps (after the stream has been synchronised).
gabp_status collect_timing(Ctx* c) {
  for (int i = 0; i + 1 < c->tev_used; i += 2) {
    float ms = 0.f;
    GABP_HIP(c, hipEventElapsedTime(&ms, c->tev[i], c->tev[i + 1]));
    c->sweep_ms += ms;
    c->timed_sweeps += 1;
  }
  c->tev_used = 0;
  return GABP_OK;
}

void reset_timing(Ctx* c) {
  c->tev_used = 0;
  c->sweep_ms = 0.0;
  c->timed_sweeps = 0;
}

void report_timing(const Ctx* c, gabp_info* info) {
  info->sweep_ms = c->sweep_ms;
  info->timed_sweeps = c->timed_sweeps;
  info->sweep_mode = c->timed_mode;
}

gabp_status read_status(Ctx* c, const DevStatus* st_d, DevStatus* out) {
  GABP_HIP(c, hipMemcpyAsync(&c->st_h[2], st_d, sizeof(DevStatus), hipMemcpyDeviceToHost, c->stream));
  GABP_HIP(c, hipStreamSynchronize(c->stream));
  *out = c->st_h[2];
  return collect_timing(c);
}

// The status a finish kernel left in pinned memory slot q, once the stream
// has drained (no copy launch).
gabp_status read_mirror(Ctx* c, int q, DevStatus* out) {
  GABP_HIP(c, hipStreamSynchronize(c->stream));
  std::atomic_thread_fence(std::memory_order_acquire);
  *out = c->st_mir_h[q];
  return collect_timing(c);
}

// The final status of a sweep run: the one its poller already saw when that
// was final, else a read of the device status.
gabp_status read_run_status(Ctx* c, const DevStatus* st_d, DevStatus* out) {
  if (!c->run_seen_final) return read_status(c, st_d, out);
  GABP_HIP(c, hipStreamSynchronize(c->stream));
  *out = c->run_seen;
  return collect_timing(c);
}

// Freeze the precisions of the messages of round `round`: the h update
// coefficient -A_ij / (P~_i - P_ji) of every message and 1 / P~_i of every
// node, so that later sweeps update the h messages only (the P update has no
// b term).
template <typename T>
gabp_status freeze(Ctx* c, int round, const void* diag, const void* rhs, int prec) {
  if (c->layout == kLayoutSerial) return GABP_OK;  // the serial sweeps always update P and h
  DevStatus* st = c->st_d + 1;  // fresh status: the freeze must not be skipped
  GABP_HIP(c, launch_reset_status(st, 1, c->stream));
  if (c->layout == kLayoutCompact) {
    CnodeArgs<T> k{};
    k.blk_row = c->blk_row_d;
    k.blk_e0 = c->blk_e0_d;
    k.off_ptr = c->off_ptr_d;
    k.col = c->off_col_d;
    k.a = coef_array<T>(c);
    k.diag = (const T*)diag;
    k.rhs = (const T*)rhs;
    k.cin = cin_buf<T>(c, round);
    k.cin_old = cin_buf<T>(c, round + 1);  // round - 1
    k.agg1 = c->agg_d[round % 3];
    k.agg2 = c->agg_d[(round + 2) % 3];  // round - 1
    k.first = (round == 0);
    k.second = (round == 1);
    k.coef_out = c->gcoef_d;
    k.inv_pt_out = (T*)c->inv_pt_d;
    k.partials = c->partials_d;
    k.st = st;
    k.nblk = c->nblk;
    set_long_rows<T>(c, k);
    GABP_HIP(c, launch_cnode<T>(kFreeze, c->K, k, c->stream));
  } else if (c->layout == kLayoutNode) {
    BcastArgs<T> k{};
    k.blk_row = c->blk_row_d;
    k.off_ptr = c->off_ptr_d;
    k.col = c->off_col_d;
    k.a = coef_array<T>(c);
    k.diag = (const T*)diag;
    k.rhs = (const T*)rhs;
    k.state = c->bstate_d;
    k.aold = c->agg_d[round & 1];
    k.zero_in = (round == 0);
    k.coef_out = c->gcoef_d;
    k.inv_pt_out = (T*)c->inv_pt_d;
    k.partials = c->partials_d;
    k.st = st;
    k.nblk = c->nblk;
    GABP_HIP(c, launch_bcast<T>(kFreeze, c->K, k, c->stream));
  } else {
    SweepArgs<T> k{};
    k.blk_row = c->blk_row_d;
    k.off_ptr = c->off_ptr_d;
    k.off_col = c->off_col_d;
    k.rev = c->rev_d;
    k.a = coef_array<T>(c);
    k.diag = (const T*)diag;
    k.rhs = (const T*)rhs;
    k.min = c->msg_d[round & 1];
    k.zero_in = (round == 0);
    k.gcoef_out = (T*)c->gcoef_d;
    k.inv_pt_out = (T*)c->inv_pt_d;
    k.partials = c->partials_d;
    k.st = st;
    k.nblk = c->nblk;
    GABP_HIP(c, launch_sweep<T>(kFreeze, c->K, k, c->stream));
  }
  c->frozen_valid = true;
  c->frozen_prec = prec;
  return GABP_OK;
}

gabp_status map_status(Ctx* c, const DevStatus& st, bool exact) {
  if (st.error & kErrNonfinite) return fail(c, GABP_E_NONFINITE, "non-finite message (P~_i = P_ji or overflow)");
  if (!exact && (st.error & kErrDiverged)) return fail(c, GABP_E_DIVERGED, "residual diverged");
  if (exact || st.conv_round >= 0) return GABP_OK;
  return GABP_NOT_CONVERGED;
}

}  // namespace

gabp_status solve_plain(Ctx* c, const double* b, double* x, double* var, double tol, int32_t max_iter,
                        gabp_info* info, bool allow_reuse) {
  hipStream_t s = c->stream;
  const bool exact = tol <= 0.0;
  const bool ait = (c->opts.flags & GABP_FLAG_AITKEN) != 0;
  const bool stf = (c->opts.flags & GABP_FLAG_STEFFENSEN) != 0;
  const bool honly = allow_reuse && (c->opts.flags & GABP_FLAG_REUSE_PRECISION) && c->frozen_valid &&
                     c->frozen_prec == GABP_FP64 && !exact && !ait && !stf;
  if (stf) {
    if (c->layout != kLayoutCompact) return fail(c, GABP_E_ARG, "Steffensen's iterations need the compact layout");
    if (max_iter < 2) return fail(c, GABP_E_ARG, "Steffensen's iterations need max_iter >= 2");
    max_iter &= ~1;  // whole cycles of two sweeps
    if (!c->ait_hist_d) {
      gabp_status e = dev_alloc(c, (void**)&c->ait_hist_d, sizeof(double) * c->n);
      if (e != GABP_OK) return e;
    }
  }
  if (ait) {
    if (c->layout != kLayoutCompact) return fail(c, GABP_E_ARG, "Aitken's extrapolation needs the compact layout");
    if (max_iter < 2) return fail(c, GABP_E_ARG, "Aitken's extrapolation needs max_iter >= 2");
    for (double** p : {&c->ait_y_d, &c->ait_hist_d})
      if (!*p) {
        gabp_status e = dev_alloc(c, (void**)p, sizeof(double) * c->n);
        if (e != GABP_OK) return e;
      }
  }
  reset_timing(c);
  RunCfg cfg;
  cfg.honly = honly;
  cfg.rhs = b;
  cfg.diag = c->din64_d;
  cfg.rhs_norm = c->norms_d;
  cfg.tol = tol;
  cfg.max_iter = max_iter;
  cfg.check_every = c->opts.check_every;
  cfg.x2[0] = c->x64_d[0];
  cfg.x2[1] = c->x64_d[1];
  if (var && !honly) {
    cfg.pt2[0] = c->pt64_d[0];
    cfg.pt2[1] = c->pt64_d[1];
  }
  cfg.st = c->st_d;
  if (ait) {
    cfg.ait_y = c->ait_y_d;
    cfg.ait_hist = c->ait_hist_d;
  }
  if (stf) cfg.stf_start = c->ait_hist_d;
  // the one-launch path forms ||b|| itself and writes x and the variances of
  // the returned round directly
  const bool small = use_small(c, cfg);
  // compact sweeps to a tolerance leave x to the end (8 B per node and sweep
  // fewer), unless the variances of every round are kept too
  cfg.x_at_end = !small && c->layout == kLayoutCompact && !exact && !ait && !stf && !cfg.pt2[0];
  cfg.keep_held = (c->opts.flags & GABP_FLAG_REUSE_PRECISION) != 0;  // the freeze below takes the held round
  if (!small) GABP_HIP(c, launch_norm(b, c->n, c->partials_d, std::max(1, c->nblk), c->norms_d, nullptr, s));
  gabp_status rs = small ? run_small(c, cfg, x, var) : run_sweeps<double>(c, cfg);
  if (rs != GABP_OK) return rs;
  const double* xs[2] = {c->x64_d[0], c->x64_d[1]};
  const double* ps[2] = {c->pt64_d[0], c->pt64_d[1]};
  if (cfg.x_at_end)
    GABP_HIP(c, launch_x_from_agg(c->agg_d, honly, c->st_d, max_iter, x, c->n, s));
  else if (!small)
    GABP_HIP(c, launch_copy_round(xs, ps, c->st_d, max_iter, x, honly ? nullptr : var, c->n, s));
  if (ait) GABP_HIP(c, hipMemcpyAsync(x, c->ait_y_d, sizeof(double) * c->n, hipMemcpyDeviceToDevice, s));
  if (var && honly) GABP_HIP(c, hipMemcpyAsync(var, c->inv_pt_d, sizeof(double) * c->n, hipMemcpyDeviceToDevice, s));
  DevStatus st;
  gabp_status r = GABP_OK;
  if (small) {
    GABP_HIP(c, hipStreamSynchronize(s));
    st = *c->st_small_h;
  } else {
    r = read_run_status(c, c->st_d, &st);
  }
  if (r != GABP_OK) return r;
  r = map_status(c, st, exact);
  const int sweeps = st.conv_round >= 0 ? st.conv_round : max_iter;
  if (info) {
    info->sweeps = sweeps;
    info->outer_iters = 0;
    info->converged = (st.conv_round >= 0) ? 1 : 0;
    info->status = r;
    info->rel_residual = st.last_rel;
    info->gamma = 0.0;
    report_timing(c, info);
  }
  c->last_msg_round = (exact && !honly && r == GABP_OK) ? max_iter : -1;
  if (r == GABP_OK && !exact && !honly && !ait && !stf && (c->opts.flags & GABP_FLAG_REUSE_PRECISION) &&
      c->layout != kLayoutSerial) {
    const int last = held_round(c, st.conv_round, max_iter);
    gabp_status fr = freeze<double>(c, last, c->din64_d, b, GABP_FP64);
    if (fr != GABP_OK) return fr;
    GABP_HIP(c, hipStreamSynchronize(s));
  }
  return r;
}

// Single-loop form of the correction method (Ch. 5 Sec. 5.3): FP64 sweeps of
// Alg. 2 on A + Gamma whose prior potentials follow the damped feedback
// h^(t) = b + Gamma ((1 - s) x^(t-2) + s x^(t-1)); the residual of A x = b
// itself is checked, so the stop rule is that of the plain solve.
gabp_status solve_single_loop(Ctx* c, const double* b, double* x, double tol, int32_t max_iter,
                              gabp_info* info) {
  hipStream_t s = c->stream;
  if (c->layout != kLayoutCompact) return fail(c, GABP_E_ARG, "the single loop needs the compact layout");
  reset_timing(c);
  c->frozen_valid = false;
  GABP_HIP(c, launch_norm(b, c->n, c->partials_d, std::max(1, c->nblk), c->norms_d, nullptr, s));
  RunCfg cfg;
  cfg.rhs = b;
  cfg.diag = c->din64_d;
  cfg.chk_diag = c->d64_d;
  cfg.feedback = true;
  cfg.damp = c->opts.damping;
  cfg.rhs_norm = c->norms_d;
  cfg.tol = tol;
  cfg.max_iter = max_iter;
  cfg.check_every = c->opts.check_every;
  cfg.x2[0] = c->x64_d[0];
  cfg.x2[1] = c->x64_d[1];
  cfg.st = c->st_d;
  gabp_status rs = run_sweeps<double>(c, cfg);
  if (rs != GABP_OK) return rs;
  const double* xs[2] = {c->x64_d[0], c->x64_d[1]};
  const double* ps[2] = {c->pt64_d[0], c->pt64_d[1]};
  GABP_HIP(c, launch_copy_round(xs, ps, c->st_d, max_iter, x, nullptr, c->n, s));
  DevStatus st;
  gabp_status r = read_status(c, c->st_d, &st);
  if (r != GABP_OK) return r;
  const bool exact = tol <= 0.0;
  r = map_status(c, st, exact);
  if (info) {
    info->sweeps = st.conv_round >= 0 ? st.conv_round : max_iter;
    info->outer_iters = info->sweeps;  // one outer step per sweep
    info->converged = (st.conv_round >= 0) ? 1 : 0;
    info->status = r;
    info->rel_residual = st.last_rel;
    info->gamma = c->gamma_used;
    report_timing(c, info);
  }
  c->last_msg_round = -1;
  return r;
}

gabp_status solve_outer(Ctx* c, const double* b, double* x, double tol, int32_t max_iter, gabp_info* info) {
  hipStream_t s = c->stream;
  const bool fp32 = c->opts.precision == GABP_FP32_REFINE;
  // single-loop inner solves (loading present): no frozen precisions, the
  // feedback needs the joint sweeps
  const bool single = (c->opts.flags & GABP_FLAG_SINGLE_LOOP) && c->gamma_used > 0.0;
  if (single && c->layout != kLayoutCompact) return fail(c, GABP_E_ARG, "the single loop needs the compact layout");
  const int prec = c->opts.precision;
  reset_timing(c);
  // frozen precisions of an earlier call are used only when asked for
  if (!(c->opts.flags & GABP_FLAG_REUSE_PRECISION)) c->frozen_valid = false;
  // ||b|| comes from the first outer step's check of r = b (no separate norm)
  if (c->nblk <= 0) GABP_HIP(c, launch_norm(b, c->n, c->partials_d, 1, c->norms_d, nullptr, s));
  DevStatus* st_out = c->st_d + 1;
  DevStatus* st_in = c->st_d;

  OuterArgs o{};
  o.blk_row = c->blk_row_d;
  o.off_ptr = c->off_ptr_d;
  o.off_col = c->off_col_d;
  o.a = c->a64_d;
  o.diag = c->d64_d;
  o.b = b;
  o.xold = nullptr;
  o.xnew = c->xo_d[0];
  o.d32[0] = c->x32_d[0];
  o.d32[1] = c->x32_d[1];
  o.d64[0] = fp32 ? nullptr : c->x64_d[0];
  o.d64[1] = fp32 ? nullptr : c->x64_d[1];
  o.st_in = st_in;
  o.use_d = 0;
  o.rin32 = fp32 ? c->rin32_d : nullptr;
  o.rin64 = fp32 ? nullptr : c->rin64_d;
  o.partials = c->partials_d;
  o.st = st_out;
  o.b_norm = c->norms_d;
  o.r_norm = c->norms_d + 1;
  o.tol = tol;
  o.nblk = c->nblk;
  o.n = c->n;
  o.reset_st = 1;  // each outer launch resets the outer status first
  o.mirror = c->nblk > 0 ? c->st_mir_d + 2 : nullptr;  // and its finish leaves it in pinned memory
  auto read_outer = [&](DevStatus* out) { return o.mirror ? read_mirror(c, 2, out) : read_status(c, st_out, out); };
  // step 0 (x = 0, r = b): its check measures ||r|| = ||b|| and keeps it as ||b||
  if (c->nblk > 0) {
    o.b_norm = nullptr;
    o.r_norm = c->norms_d;
  }
  GABP_HIP(c, launch_outer(c->K, o, s));
  o.b_norm = c->norms_d;
  o.r_norm = c->norms_d + 1;
  DevStatus so, si;
  gabp_status r = read_outer(&so);
  if (r != GABP_OK) return r;

  int cur = 0, k = 0, total = 0;
  gabp_status result = GABP_NOT_CONVERGED;
  for (;;) {
    if (so.error & (kErrDiverged | kErrNonfinite)) {
      result = fail(c, GABP_E_DIVERGED, "outer residual diverged");
      break;
    }
    if (so.conv_round >= 0) {
      result = GABP_OK;
      break;
    }
    if (k >= c->opts.max_outer || total >= max_iter) break;
    const int budget = std::max(0, std::min(c->opts.inner_max_iter, max_iter - total));
    RunCfg cfg;
    cfg.honly = !single && c->frozen_valid && c->frozen_prec == prec;
    cfg.rhs = fp32 ? (const void*)c->rin32_d : (const void*)c->rin64_d;
    cfg.diag = fp32 ? (const void*)c->din32_d : (const void*)c->din64_d;
    if (single) {  // inner solves by the single loop on A + Gamma, checked against A
      cfg.feedback = true;
      cfg.damp = c->opts.damping;
      cfg.chk_diag = fp32 ? (const void*)c->d32_d : (const void*)c->d64_d;
    }
    cfg.rhs_norm = k == 0 ? c->norms_d : c->norms_d + 1;  // ||r|| (= ||b|| before the first step)
    cfg.tol = c->opts.inner_tol;
    cfg.max_iter = budget;
    cfg.check_every = c->opts.check_every;
    cfg.x2[0] = fp32 ? (void*)c->x32_d[0] : (void*)c->x64_d[0];
    cfg.x2[1] = fp32 ? (void*)c->x32_d[1] : (void*)c->x64_d[1];
    cfg.st = st_in;
    // compact inner solves write no means; the outer step forms d from the
    // returned round's aggregate record (the single loop keeps them)
    cfg.x_at_end = !single && c->layout == kLayoutCompact;
    cfg.keep_held = (c->opts.flags & GABP_FLAG_REUSE_PRECISION) || c->gamma_used > 0.0;  // a freeze may follow
    cfg.sparse_checks = true;  // the outer step, not the inner stop round, sets the accuracy
    r = fp32 ? run_sweeps<float>(c, cfg) : run_sweeps<double>(c, cfg);
    if (r != GABP_OK) return r;
    if (c->run_seen_final && c->tev_used == 0) {  // the poller already waited for the final status
      si = c->run_seen;
    } else {
      r = read_status(c, st_in, &si);
    }
    if (r != GABP_OK) return r;
    if (si.error & kErrNonfinite) return fail(c, GABP_E_NONFINITE, "non-finite inner message");
    if (si.error & kErrDiverged) {
      result = fail(c, GABP_E_DIVERGED,
                    "inner GaBP diverged (the inner matrix is not walk-summable: use diagonal loading)");
      break;
    }
    const int used = si.conv_round >= 0 ? si.conv_round : budget;
    total += used;
    // Frozen precisions pay where later inner solves use them: the loading
    // loops take many outer steps, and with the reuse flag later calls start
    // from them.  Refinement on A itself takes about log(tol) / log(inner_tol)
    // = 2 steps, and an h-only sweep moves as many bytes as a joint one, so
    // there the freeze pass is left out and every inner solve runs joint
    // sweeps (measured on the bench workload: 3.09 against 3.31 ms).
    const bool want_freeze = (c->opts.flags & GABP_FLAG_REUSE_PRECISION) || c->gamma_used > 0.0;
    if (!single && !cfg.honly && si.conv_round >= 0 && c->layout != kLayoutSerial && want_freeze) {
      const int last = held_round(c, si.conv_round, budget);
      r = fp32 ? freeze<float>(c, last, cfg.diag, cfg.rhs, prec) : freeze<double>(c, last, cfg.diag, cfg.rhs, prec);
      if (r != GABP_OK) return r;
    }
    o.xold = c->xo_d[cur];
    o.xnew = c->xo_d[cur ^ 1];
    o.use_d = 1;
    o.in_fallback = budget;
    for (int q = 0; q < 3; ++q) o.dagg[q] = c->agg_d[q];
    o.dagg_elt = cfg.x_at_end ? (fp32 ? 4 : 8) : 0;
    o.dagg_honly = cfg.honly ? 1 : 0;
    GABP_HIP(c, launch_outer(c->K, o, s));
    cur ^= 1;
    ++k;
    r = read_outer(&so);
    if (r != GABP_OK) return r;
  }
  GABP_HIP(c, hipMemcpyAsync(x, c->xo_d[cur], sizeof(double) * c->n, hipMemcpyDeviceToDevice, s));
  GABP_HIP(c, hipStreamSynchronize(s));
  if (info) {
    info->sweeps = total;
    info->outer_iters = k;
    info->converged = so.conv_round >= 0 ? 1 : 0;
    info->status = result;
    info->rel_residual = so.last_rel;
    info->gamma = c->gamma_used;
    report_timing(c, info);
  }
  c->last_msg_round = -1;
  return result;
}

// ---------------------------------------------------------------------------
// autotuner: message layout and slots per workgroup
// ---------------------------------------------------------------------------

namespace {

// Layout asked for at create: the caller's, else the compact layout for the
// single loop and Aitken's extrapolation (both live in its sweep), else 0.
int layout_request(const Ctx* c) {
  if (c->opts.layout) return c->opts.layout;
  return (c->opts.flags & (GABP_FLAG_SINGLE_LOOP | GABP_FLAG_AITKEN | GABP_FLAG_STEFFENSEN)) ? kLayoutCompact : 0;
}

std::string tune_key(const Ctx* c) {
  int nb = 0;
  while ((1LL << (nb + 1)) <= (long long)std::max(1, c->n)) ++nb;
  const double avg = c->n ? (double)c->E / c->n : 0.0;
  char buf[160];
  std::snprintf(buf, sizeof(buf), "fp%d-n2^%d-deg%d-max%d-L%d-epb%d-x%d",
                c->opts.precision == GABP_FP32_REFINE ? 32 : 64, nb, (int)std::lround(avg),
                c->max_degree > 2048 ? 9999 : (c->max_degree > 256 ? 2048 : 256), layout_request(c),
                c->opts.edges_per_block, c->nparts);
  return buf;
}

bool cache_lookup(const std::string& path, const std::string& key, int* layout, int* K) {
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
    const auto pk = line.find("\"K\": ");
    const auto pl = line.find("\"layout\": ");
    if (pk == std::string::npos || pl == std::string::npos) continue;
    const int k = std::atoi(line.c_str() + pk + 5), l = std::atoi(line.c_str() + pl + 10);
    if ((k == 2 || k == 4 || k == 8) && (l == kLayoutEdge || node_family(l) || l == kLayoutSerial)) {
      *K = k;
      *layout = l;
      found = true;
    }
  }
  return found;
}

void cache_store(const std::string& path, const std::string& key, int layout, int K, const std::string& detail) {
  std::ofstream f(path, std::ios::app);
  if (!f) return;
  f << "{\"key\": \"" << key << "\", \"layout\": " << layout << ", \"K\": " << K << ", \"ms_per_sweep\": {"
    << detail << "}}\n";
}

// Time a few checking sweeps of the handle's main precision, from zero
// messages, with events around the whole run: the fastest of three runs, so
// that block sizes a percent apart are told apart from run to run.
template <typename T>
gabp_status time_candidate(Ctx* c, int layout, int K, const void* rhs, const void* diag, float* ms_out) {
  c->layout = layout;
  gabp_status r = set_partition(c, K);
  if (r != GABP_OK) return r;
  RunCfg cfg;
  cfg.rhs = rhs;
  cfg.diag = diag;
  cfg.rhs_norm = c->norms_d;
  cfg.tol = 1e-300;  // never reached: every sweep carries the check
  cfg.max_iter = 8;
  cfg.x2[0] = sizeof(T) == 8 ? (void*)c->x64_d[0] : (void*)c->x32_d[0];
  cfg.x2[1] = sizeof(T) == 8 ? (void*)c->x64_d[1] : (void*)c->x32_d[1];
  cfg.st = c->st_d;
  hipEvent_t e0, e1;
  GABP_HIP(c, hipEventCreate(&e0));
  GABP_HIP(c, hipEventCreate(&e1));
  r = run_sweeps<T>(c, cfg);  // warm-up
  float best = 1e30f;
  for (int rep = 0; rep < 3 && r == GABP_OK; ++rep) {
    GABP_HIP(c, hipEventRecord(e0, c->stream));
    r = run_sweeps<T>(c, cfg);
    GABP_HIP(c, hipEventRecord(e1, c->stream));
    GABP_HIP(c, hipEventSynchronize(e1));
    float ms = 0.f;
    GABP_HIP(c, hipEventElapsedTime(&ms, e0, e1));
    best = std::min(best, ms);
  }
  *ms_out = best / cfg.max_iter;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return r;
}

}  // namespace

gabp_status autotune(Ctx* c) {
  const int epb = c->opts.edges_per_block;
  std::vector<int> layouts, Ks;
  const int req = layout_request(c);
  if (req) layouts.push_back(req);
  else layouts = {kLayoutEdge, kLayoutNode, kLayoutCompact};
  if (epb) Ks.push_back(epb / kBlock);
  else Ks = {2, 4, 8};
  int best_l = req ? req : layouts.back(), best_k = epb ? epb / kBlock : 4;
  if (c->E >= 200000 && layouts.size() * Ks.size() > 1) {
    const std::string key = tune_key(c);
    const char* path = std::getenv("GABP_AUTOTUNE_CACHE");
    if (path && *path && cache_lookup(path, key, &best_l, &best_k)) {
      c->layout = best_l;
      return set_partition(c, best_k);
    }
    const bool fp32 = c->opts.precision == GABP_FP32_REFINE;
    // right-hand side: the diagonal itself (any finite vector will do)
    const void* rhs = fp32 ? (const void*)c->din32_d : (const void*)c->din64_d;
    GABP_HIP(c, launch_fill(c->norms_d, 1, 1.0, c->stream));
    float best_ms = 1e30f;
    std::string detail;
    for (int l : layouts)
      for (int K : Ks) {
        float t = 0.f;
        gabp_status r = fp32 ? time_candidate<float>(c, l, K, rhs, rhs, &t)
                             : time_candidate<double>(c, l, K, rhs, rhs, &t);
        if (r != GABP_OK) return r;
        char buf[64];
        std::snprintf(buf, sizeof(buf), "%s\"L%d-K%d\": %.4f", detail.empty() ? "" : ", ", l, K, t);
        detail += buf;
        if (t < best_ms) {
          best_ms = t;
          best_l = l;
          best_k = K;
        }
      }
    if (path && *path) cache_store(path, key, best_l, best_k, detail);
  }
  c->layout = best_l;
  return set_partition(c, best_k);
}

}  // namespace gabp
