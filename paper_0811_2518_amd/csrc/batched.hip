// Batched solves: many independent systems, several right-hand sides each, in
// one persistent-kernel launch captured in a HIP graph.
//
// Work items are (system, group of up to kMaxGroup right-hand sides), handed
// out largest-first through an atomic queue; one 512-lane workgroup solves an
// item from start to finish, so every barrier is a workgroup barrier and no
// workgroup ever waits for another.  Per item:
//   1. precision phase (FP32): synchronous P-only sweeps of Alg. 2 -- the P
//      update has no b term, so the precisions are shared by all right-hand
//      sides of the item -- until the node precisions P~_i stop changing; then
//      freeze g_s = -A_ij / (P~_i - P_ji) and 1 / P~_i;
//   2. FP64 iterative refinement: r = b - A x in FP64; the correction A d = r
//      by h-only FP32 sweeps on all right-hand sides of the group at once
//      (messages stored [slot][rhs], so the reverse-message gather reads
//      kg contiguous words), x += d in FP64; until every right-hand side
//      reaches the relative residual tolerance.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "gabp_internal.h"

namespace gabp {

namespace {

constexpr int kBT = 512;       // lanes per batched workgroup
constexpr int kMaxGroup = 8;   // right-hand sides per work item
constexpr float kPrecTol = 4e-7f;

struct Item {
  int32_t sys, j0, kg, k;  // right-hand sides j0 .. j0+kg-1 of k
  int32_t r0, r1;          // global rows of the system
  int64_t s0, s1;          // global off-diagonal slots of the system
  int64_t off_e;           // item scratch: per-slot arrays (3 E floats)
  int64_t off_n;           // per-node arrays (2 n floats)
  int64_t off_he;          // h messages (2 E kg floats)
  int64_t off_nk;          // d and r (2 n kg floats)
  int64_t rhs_off;         // B / X offset of the system
};

struct ItemInfo {
  int32_t sweeps, outer, converged, status;
  double rel;
  int32_t psweeps, pad;
  uint64_t t0, t1;  // device wall clock at the item's start and end
};

struct BatchArgs {
  const int32_t* off_ptr;
  const int32_t* off_col;
  const int32_t* rev;
  const float* a32;
  const double* a64;
  const float* d32;
  const double* d64;
  const Item* items;
  ItemInfo* infos;
  int32_t num_items;
  uint32_t* queue;
  float* ebuf;
  float* nbuf;
  float* hbuf;
  float* kbuf;
  const double* B;
  double* X;
  double tol;
  float inner_tol;
  int32_t inner_max;
  int32_t max_outer;
  int32_t max_iter;
};

__device__ __forceinline__ void lds_max(unsigned* slot, float v) {
  // nonnegative floats order like their bit patterns; NaN maps above +inf
  atomicMax(slot, isnan(v) ? 0x7f800001u : __float_as_uint(v));
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per right-hand-side sums: lane t < Tq always owns column t % kg, so the
// partial sums of one column are combined in a fixed order.
__device__ void column_sums(double v, int kg, int Tq, double* s_part, double* out) {
  const int tid = threadIdx.x;
  s_part[tid] = (tid < Tq) ? v : 0.0;
  __syncthreads();
  if (tid < kg) {
    double acc = 0.0;
    for (int t = tid; t < Tq; t += kg) acc += s_part[t];
    out[tid] = acc;
  }
  __syncthreads();
}

__device__ void solve_item(const BatchArgs& A, const Item& I, int it, unsigned* s_max, double* s_part,
                           double* s_col, double* s_bn, int* s_flag) {
  const int tid = threadIdx.x;
  const int n = I.r1 - I.r0;
  const int64_t E = I.s1 - I.s0;
  const int kg = I.kg, k = I.k;
  const int Tq = (kBT / kg) * kg;  // lanes used for (row, rhs) items
  float* P0 = A.ebuf + 3 * I.off_e;
  float* P1 = P0 + E;
  float* g = P1 + E;
  float* Ptprev = A.nbuf + 2 * I.off_n;
  float* invPt = Ptprev + n;
  float* h0 = A.hbuf + 2 * I.off_he;
  float* h1 = h0 + E * kg;
  float* d = A.kbuf + 2 * I.off_nk;
  float* r32 = d + (int64_t)n * kg;
  const double* B = A.B + I.rhs_off;
  double* X = A.X + I.rhs_off;
  int status = 0;
  const uint64_t t_start = wall_clock64();

  // ---- 1. precision phase --------------------------------------------------
  int tp = 1;
  for (;; ++tp) {
    const float* Pold = (tp & 1) ? P0 : P1;
    float* Pnew = (tp & 1) ? P1 : P0;
    if (tid == 0) s_max[0] = 0u;
    __syncthreads();
    float lmax = 0.f;
    for (int i = tid; i < n; i += kBT) {
      const int R = I.r0 + i;
      const int lo = A.off_ptr[R], hi = A.off_ptr[R + 1];
      float Pt = A.d32[R];
      if (tp > 1)
        for (int s = lo; s < hi; ++s) Pt += Pold[A.rev[s] - I.s0];
      if (tp > 1) lmax = fmaxf(lmax, fabsf(Pt - Ptprev[i]) / fabsf(Pt));
      Ptprev[i] = Pt;
      for (int s = lo; s < hi; ++s) {
        const float pin = (tp > 1) ? Pold[A.rev[s] - I.s0] : 0.f;
        const float av = A.a32[s];
        Pnew[s - I.s0] = -av * av / (Pt - pin);
      }
    }
    lds_max(&s_max[0], lmax);
    __syncthreads();
    const float ch = __uint_as_float(s_max[0]);
    __syncthreads();
    if (tp >= 3 && ch <= kPrecTol) break;
    if (tp >= A.inner_max || !(ch <= 1e30f)) break;
  }
  // freeze from the last round's precisions
  {
    const float* Pf = (tp & 1) ? P1 : P0;
    for (int i = tid; i < n; i += kBT) {
      const int R = I.r0 + i;
      const int lo = A.off_ptr[R], hi = A.off_ptr[R + 1];
      float Pt = A.d32[R];
      for (int s = lo; s < hi; ++s) Pt += Pf[A.rev[s] - I.s0];
      invPt[i] = 1.f / Pt;
      for (int s = lo; s < hi; ++s) g[s - I.s0] = -A.a32[s] / (Pt - Pf[A.rev[s] - I.s0]);
      if (!isfinite(1.f / Pt)) *s_flag = 1;
    }
    __syncthreads();
  }

  // ---- 2. refinement -------------------------------------------------------
  const int jj = tid % kg;
  double bpart = 0.0;
  if (tid < Tq)
    for (int q = tid; q < n * kg; q += Tq) {
      const int i = q / kg;
      const double bv = B[(int64_t)i * k + I.j0 + jj];
      X[(int64_t)i * k + I.j0 + jj] = 0.0;
      r32[q] = (float)bv;
      bpart += bv * bv;
    }
  column_sums(bpart, kg, Tq, s_part, s_bn);
  if (tid < kg) s_bn[tid] = sqrt(s_bn[tid]);
  __syncthreads();

  int outer = 0, total = 0, converged = 0;
  double relmax = 1.0;
  for (;;) {
    // inner: h-only sweeps on the correction system A d = r
    int t = 1;
    for (;; ++t) {
      const float* hold = (t & 1) ? h0 : h1;
      float* hnew = (t & 1) ? h1 : h0;
      if (tid < 2 * kMaxGroup) s_max[tid] = 0u;
      __syncthreads();
      float dmax = 0.f, xmax = 0.f;
      if (tid < Tq)
        for (int q = tid; q < n * kg; q += Tq) {
          const int i = q / kg;
          const int R = I.r0 + i;
          const int lo = A.off_ptr[R], hi = A.off_ptr[R + 1];
          float ht = r32[q];
          if (t > 1)
            for (int s = lo; s < hi; ++s) ht += hold[(int64_t)(A.rev[s] - I.s0) * kg + jj];
          const float dn = ht * invPt[i];
          const float dold = (t > 1) ? d[q] : 0.f;
          d[q] = dn;
          dmax = fmaxf(dmax, fabsf(dn - dold));
          xmax = fmaxf(xmax, fabsf(dn));
          for (int s = lo; s < hi; ++s) {
            const float hin = (t > 1) ? hold[(int64_t)(A.rev[s] - I.s0) * kg + jj] : 0.f;
            hnew[(int64_t)(s - I.s0) * kg + jj] = g[s - I.s0] * (ht - hin);
          }
        }
      if (tid < Tq) {
        lds_max(&s_max[jj], dmax);
        lds_max(&s_max[kMaxGroup + jj], xmax);
      }
      __syncthreads();
      bool done = t >= 2;
      for (int j = 0; j < kg; ++j) {
        const float dm = __uint_as_float(s_max[j]), xm = __uint_as_float(s_max[kMaxGroup + j]);
        if (!(dm <= A.inner_tol * xm)) done = false;
        if (!(dm <= 1e30f)) status = GABP_E_NONFINITE;
      }
      __syncthreads();
      if (done || status || total + t >= A.max_iter || t >= A.inner_max) break;
    }
    total += t;
    // x += d (FP64), then r = b - A x
    if (tid < Tq)
      for (int q = tid; q < n * kg; q += Tq) X[(int64_t)(q / kg) * k + I.j0 + jj] += (double)d[q];
    __syncthreads();
    double rpart = 0.0;
    if (tid < Tq)
      for (int q = tid; q < n * kg; q += Tq) {
        const int i = q / kg;
        const int R = I.r0 + i;
        double r = B[(int64_t)i * k + I.j0 + jj] - A.d64[R] * X[(int64_t)i * k + I.j0 + jj];
        for (int s = A.off_ptr[R]; s < A.off_ptr[R + 1]; ++s)
          r -= A.a64[s] * X[(int64_t)(A.off_col[s] - I.r0) * k + I.j0 + jj];
        r32[q] = (float)r;
        rpart += r * r;
      }
    column_sums(rpart, kg, Tq, s_part, s_col);
    ++outer;
    relmax = 0.0;
    for (int j = 0; j < kg; ++j) {
      const double nr = sqrt(s_col[j]);
      const double rel = s_bn[j] > 0.0 ? nr / s_bn[j] : nr;
      relmax = (rel > relmax || rel != rel) ? rel : relmax;
    }
    if (relmax <= A.tol) {
      converged = 1;
      break;
    }
    if (!(relmax <= kDivergeLimit)) {
      status = GABP_E_DIVERGED;
      break;
    }
    if (status || outer >= A.max_outer || total >= A.max_iter) break;
  }
  if (*s_flag) status = GABP_E_NONFINITE;
  if (tid == 0) {
    ItemInfo inf;
    inf.sweeps = total;
    inf.outer = outer;
    inf.converged = converged;
    inf.status = status ? status : (converged ? GABP_OK : GABP_NOT_CONVERGED);
    inf.rel = relmax;
    inf.psweeps = tp;
    inf.t0 = t_start;
    inf.t1 = wall_clock64();
    inf.pad = 0;
    A.infos[it] = inf;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBT) void k_batched(BatchArgs A) {
  __shared__ int s_item;
  __shared__ int s_flag;
  __shared__ unsigned s_max[2 * kMaxGroup];
  __shared__ double s_part[kBT];
  __shared__ double s_col[kMaxGroup];
  __shared__ double s_bn[kMaxGroup];
  for (;;) {
    if (threadIdx.x == 0) {
      s_item = (int)atomicAdd(A.queue, 1u);
      s_flag = 0;
    }
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= A.num_items) return;  // every workgroup leaves once the queue is empty
    solve_item(A, A.items[it], it, s_max, s_part, s_col, s_bn, &s_flag);
  }
}

__global__ void k_reset_queue(uint32_t* q) {
  if (threadIdx.x == 0) *q = 0u;
}

struct BatchState {
  int32_t num_sys = 0;
  std::vector<int32_t> sys_row_off;
  std::vector<int64_t> sys_slot_off;
  // per-solve work list and scratch (grown on demand)
  std::vector<Item> items;
  Item* items_d = nullptr;
  ItemInfo* infos_d = nullptr;
  size_t items_cap = 0;
  uint32_t* queue_d = nullptr;
  float* ebuf = nullptr;
  float* nbuf = nullptr;
  float* hbuf = nullptr;
  float* kbuf = nullptr;
  int64_t ecap = 0, ncap = 0, hcap = 0, kcap = 0;
  int grid = 0;
  int launched_grid = 0;
  hipStream_t gs = nullptr;
  double clock_khz = 0.0;
  gabp_batch_profile prof{};
  // cached graph of the last solve
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<int32_t> key_nrhs;
  std::vector<int64_t> key_off;
  const double* key_B = nullptr;
  double* key_X = nullptr;
  double key_tol = -1.0;
  int32_t key_iter = -1;
};

void free_raw(void* p) {
  if (p) (void)hipFree(p);
}

gabp_status grow(Ctx* c, float** p, int64_t* cap, int64_t need) {
  if (need <= *cap) return GABP_OK;
  free_raw(*p);
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc((void**)p, sizeof(float) * std::max<int64_t>(need, 16));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(c, GABP_E_OOM, "batched scratch allocation failed");
  }
  *cap = need;
  return GABP_OK;
}

}  // namespace

gabp_status batched_create(Ctx* c, int32_t num_sys, const int32_t* sys_row_off) {
  auto* bs = new BatchState();
  c->batch = bs;
  bs->num_sys = num_sys;
  bs->sys_row_off.assign(sys_row_off, sys_row_off + num_sys + 1);
  bs->sys_slot_off.resize(num_sys + 1);
  for (int s = 0; s <= num_sys; ++s)
    bs->sys_slot_off[s] = c->n > 0 ? c->off_ptr_h[sys_row_off[s]] : 0;
  GABP_HIP(c, hipMalloc((void**)&bs->queue_d, sizeof(uint32_t)));
  // the persistent grid: as many workgroups as can be resident at once
  int dev = 0, ncu = 0, per_cu = 0;
  GABP_HIP(c, hipGetDevice(&dev));
  GABP_HIP(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  GABP_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched, kBT, 0));
  bs->grid = std::max(1, ncu * std::max(1, per_cu));
  int khz = 0;
  GABP_HIP(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  bs->clock_khz = khz;
  // the graph is captured and replayed on a stream of the handle's own, ordered
  // after the caller's stream by synchronisation (capture needs a non-null stream)
  GABP_HIP(c, hipStreamCreateWithFlags(&bs->gs, hipStreamNonBlocking));
  // FP32 copies of the diagonal (no loading for batched solves)
  {
    void* p = nullptr;
    gabp_status r = dev_alloc(c, &p, sizeof(float) * std::max<int64_t>(1, c->n));
    if (r != GABP_OK) return r;
    c->din32_d = (float*)p;
    GABP_HIP(c, launch_scale_diag(c->d64_d, 1.0, nullptr, c->din32_d, c->n, c->stream));
  }
  return GABP_OK;
}

gabp_status batched_solve(Ctx* c, const int32_t* nrhs, const int64_t* rhs_off, const double* B, double* X,
                          double tol, int32_t max_iter, gabp_info* infos) {
  auto* bs = (BatchState*)c->batch;
  const int S = bs->num_sys;
  // validate the right-hand-side layout
  if (rhs_off[0] != 0) return fail(c, GABP_E_ARG, "rhs_off[0] must be 0");
  for (int s = 0; s < S; ++s) {
    const int64_t ns = bs->sys_row_off[s + 1] - bs->sys_row_off[s];
    if (nrhs[s] < 1) return fail(c, GABP_E_ARG, "nrhs must be >= 1");
    if (rhs_off[s + 1] - rhs_off[s] != ns * nrhs[s]) return fail(c, GABP_E_ARG, "rhs_off does not match n_s * k_s");
  }
  if (rhs_off[S] > 0 && (!B || !X)) return fail(c, GABP_E_ARG, "NULL B or X");
  const bool same = bs->exec && bs->key_B == B && bs->key_X == X && bs->key_tol == tol &&
                    bs->key_iter == max_iter &&
                    bs->key_nrhs == std::vector<int32_t>(nrhs, nrhs + S) &&
                    bs->key_off == std::vector<int64_t>(rhs_off, rhs_off + S + 1);
  if (!same) {
    // Work items, largest first.  The work of a right-hand side per sweep is
    // taken as E_s + n_s; a system's right-hand sides are grouped so that no
    // item exceeds half of an even share of the whole batch per workgroup,
    // which keeps the longest item below the average workgroup load.
    double total = 0.0;
    for (int s = 0; s < S; ++s)
      total += (double)(bs->sys_slot_off[s + 1] - bs->sys_slot_off[s] + bs->sys_row_off[s + 1] -
                        bs->sys_row_off[s]) * nrhs[s];
    const double cap = std::max(1.0, total / (2.0 * std::max(1, bs->grid)));
    std::vector<Item> items;
    int64_t oe = 0, on = 0, ohe = 0, onk = 0;
    for (int s = 0; s < S; ++s) {
      const int32_t r0 = bs->sys_row_off[s], r1 = bs->sys_row_off[s + 1];
      if (r1 == r0) continue;
      const int64_t E = bs->sys_slot_off[s + 1] - bs->sys_slot_off[s];
      const int32_t k = nrhs[s];
      const int32_t group = (int32_t)std::max(1.0, std::min((double)kMaxGroup, std::floor(cap / (double)(E + r1 - r0))));
      for (int32_t j0 = 0; j0 < k; j0 += group) {
        Item it{};
        it.sys = s;
        it.j0 = j0;
        it.kg = std::min(group, k - j0);
        it.k = k;
        it.r0 = r0;
        it.r1 = r1;
        it.s0 = bs->sys_slot_off[s];
        it.s1 = bs->sys_slot_off[s + 1];
        it.off_e = oe;
        it.off_n = on;
        it.off_he = ohe;
        it.off_nk = onk;
        it.rhs_off = rhs_off[s];
        oe += E;
        on += (r1 - r0);
        ohe += E * it.kg;
        onk += (int64_t)(r1 - r0) * it.kg;
        items.push_back(it);
      }
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
      const int64_t wa = ((a.s1 - a.s0) + (a.r1 - a.r0)) * a.kg, wb = ((b.s1 - b.s0) + (b.r1 - b.r0)) * b.kg;
      return wa > wb;
    });
    bs->items = items;
    gabp_status r = grow(c, &bs->ebuf, &bs->ecap, 3 * oe);
    if (r == GABP_OK) r = grow(c, &bs->nbuf, &bs->ncap, 2 * on);
    if (r == GABP_OK) r = grow(c, &bs->hbuf, &bs->hcap, 2 * ohe);
    if (r == GABP_OK) r = grow(c, &bs->kbuf, &bs->kcap, 2 * onk);
    if (r != GABP_OK) return r;
    if (items.size() > bs->items_cap) {
      free_raw(bs->items_d);
      free_raw(bs->infos_d);
      bs->items_d = nullptr;
      bs->infos_d = nullptr;
      bs->items_cap = 0;
      GABP_HIP(c, hipMalloc((void**)&bs->items_d, sizeof(Item) * std::max<size_t>(1, items.size())));
      GABP_HIP(c, hipMalloc((void**)&bs->infos_d, sizeof(ItemInfo) * std::max<size_t>(1, items.size())));
      bs->items_cap = items.size();
    }
    if (!items.empty())
      GABP_HIP(c, hipMemcpyAsync(bs->items_d, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice,
                                 c->stream));
    BatchArgs a{};
    a.off_ptr = c->off_ptr_d;
    a.off_col = c->off_col_d;
    a.rev = c->rev_d;
    a.a32 = c->a32_d;
    a.a64 = c->a64_d;
    a.d32 = c->din32_d;
    a.d64 = c->d64_d;
    a.items = bs->items_d;
    a.infos = bs->infos_d;
    a.num_items = (int32_t)items.size();
    a.queue = bs->queue_d;
    a.ebuf = bs->ebuf;
    a.nbuf = bs->nbuf;
    a.hbuf = bs->hbuf;
    a.kbuf = bs->kbuf;
    a.B = B;
    a.X = X;
    a.tol = tol;
    a.inner_tol = (float)c->opts.inner_tol;
    a.inner_max = std::max(1, c->opts.inner_max_iter);
    a.max_outer = std::max(1, c->opts.max_outer);
    a.max_iter = std::max(1, max_iter);
    if (bs->exec) {
      (void)hipGraphExecDestroy(bs->exec);
      bs->exec = nullptr;
    }
    if (bs->graph) {
      (void)hipGraphDestroy(bs->graph);
      bs->graph = nullptr;
    }
    // capture: queue reset (a kernel, not a memset node) + the persistent kernel
    GABP_HIP(c, hipStreamSynchronize(c->stream));
    GABP_HIP(c, hipStreamBeginCapture(bs->gs, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, bs->gs, bs->queue_d);
    const int grid = std::max(1, std::min<int>(bs->grid, (int)items.size()));
    bs->launched_grid = grid;
    hipLaunchKernelGGL(k_batched, dim3(grid), dim3(kBT), 0, bs->gs, a);
    hipError_t e = hipStreamEndCapture(bs->gs, &bs->graph);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    GABP_HIP(c, hipGraphInstantiate(&bs->exec, bs->graph, nullptr, nullptr, 0));
    bs->key_B = B;
    bs->key_X = X;
    bs->key_tol = tol;
    bs->key_iter = max_iter;
    bs->key_nrhs.assign(nrhs, nrhs + S);
    bs->key_off.assign(rhs_off, rhs_off + S + 1);
  }
  if (bs->items.empty()) return GABP_OK;
  GABP_HIP(c, hipStreamSynchronize(c->stream));  // B written by the caller's stream
  GABP_HIP(c, hipGraphLaunch(bs->exec, bs->gs));
  std::vector<ItemInfo> ii(bs->items.size());
  GABP_HIP(c, hipMemcpyAsync(ii.data(), bs->infos_d, sizeof(ItemInfo) * ii.size(), hipMemcpyDeviceToHost,
                             bs->gs));
  GABP_HIP(c, hipStreamSynchronize(bs->gs));
  // load-balance profile of the launch
  {
    gabp_batch_profile& pf = bs->prof;
    pf = gabp_batch_profile{};
    pf.num_items = (int32_t)ii.size();
    pf.workgroups = bs->launched_grid;
    uint64_t lo = ~0ull, hi = 0;
    double busy = 0.0, longest = 0.0;
    for (const ItemInfo& q : ii) {
      lo = std::min(lo, q.t0);
      hi = std::max(hi, q.t1);
      const double ms = (double)(q.t1 - q.t0) / bs->clock_khz;
      busy += ms;
      longest = std::max(longest, ms);
      pf.precision_sweeps += q.psweeps;
      pf.inner_sweeps += q.sweeps;
    }
    pf.makespan_ms = ii.empty() ? 0.0 : (double)(hi - lo) / bs->clock_khz;
    pf.busy_ms = busy;
    pf.longest_item_ms = longest;
  }
  // per-system info: worst over the system's items
  std::vector<gabp_info> out(S);
  for (int s = 0; s < S; ++s) {
    out[s] = gabp_info{};
    out[s].converged = 1;
    out[s].status = GABP_OK;
  }
  gabp_status worst = GABP_OK;
  for (size_t q = 0; q < ii.size(); ++q) {
    const Item& it = bs->items[q];
    gabp_info& o = out[it.sys];
    o.sweeps = std::max(o.sweeps, ii[q].sweeps);
    o.outer_iters = std::max(o.outer_iters, ii[q].outer);
    o.converged = o.converged && ii[q].converged;
    o.rel_residual = std::max(o.rel_residual, ii[q].rel);
    if (ii[q].status < 0 || (o.status >= 0 && ii[q].status > o.status)) o.status = (gabp_status)ii[q].status;
  }
  for (int s = 0; s < S; ++s) {
    if (out[s].status < 0 && (worst >= 0 || out[s].status < worst)) worst = (gabp_status)out[s].status;
    else if (worst >= 0 && out[s].status > worst) worst = (gabp_status)out[s].status;
  }
  if (infos)
    for (int s = 0; s < S; ++s) infos[s] = out[s];
  if (worst < 0) fail(c, worst, "a batched system failed (see per-system infos)");
  return worst;
}

gabp_status batched_profile(Ctx* c, gabp_batch_profile* out) {
  auto* bs = (BatchState*)c->batch;
  if (!bs) return fail(c, GABP_E_ARG, "not a batched handle");
  *out = bs->prof;
  return GABP_OK;
}

void batched_destroy(Ctx* c) {
  auto* bs = (BatchState*)c->batch;
  if (!bs) return;
  if (bs->exec) (void)hipGraphExecDestroy(bs->exec);
  if (bs->graph) (void)hipGraphDestroy(bs->graph);
  free_raw(bs->items_d);
  free_raw(bs->infos_d);
  free_raw(bs->queue_d);
  free_raw(bs->ebuf);
  free_raw(bs->nbuf);
  free_raw(bs->hbuf);
  free_raw(bs->kbuf);
  if (bs->gs) (void)hipStreamDestroy(bs->gs);
  delete bs;
  c->batch = nullptr;
}

}  // namespace gabp
