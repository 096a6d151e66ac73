// Synchronous broadcast GaBP sweep kernels for gfx950 (wave64).
//
// One launch = one round of Alg. 2 (Ch. 3 Sec. 3.3) over the whole graph.
// Messages live in "outgoing" slot order: slot s = (i, j) of the off-diagonal
// CSR holds the message i -> j, in information form (P_ij, h_ij = P_ij mu_ij).
// A workgroup owns a contiguous group of rows i and, for every slot of those
// rows,
//   1. gathers the reverse message j -> i = msg[rev[s]] (the only irregular
//      access), coalesced reads of rev[] and a[] in slot order,
//   2. forms the node aggregates of Alg. 2, P~_i = A_ii + sum_k P_ki and
//      h~_i = b_i + sum_k h_ki, with one lane per row over the row segment
//      staged in LDS; x_i = h~_i / P~_i is the tentative mean of the round,
//   3. writes the new outgoing messages, subtracting the reverse message
//      (broadcast form): D = P~_i - P_ji, P_ij = -A_ij^2 / D,
//      h_ij = -A_ij (h~_i - h_ji) / D  (the mean rule of Alg. 2 multiplied by
//      P_ij), coalesced in slot order.
// Steps 2 and 3 of the paper's round are thus fused: the aggregate of node i is
// formed once, in registers/LDS, and never written to HBM.  Optionally the same
// launch checks the residual b - A x of an earlier round (fused convergence
// check: wave64 reductions into one partial per workgroup, added in a fixed
// order by a one-workgroup finish kernel).
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>

#include "gabp_internal.h"

namespace gabp {

// Message records.  A joint message i -> j carries (P_ij, h_ij) and, beside
// them, the sender's tentative mean x_i of the round its aggregate was formed
// in; with frozen precisions only (h_ij, x_i) remain.  The residual check of
// row j needs x_i of every neighbour: it arrives in the same cache line as the
// gathered reverse message instead of costing a second random access.
template <typename T>
struct MsgJ {
  T P, h, x;
};
template <typename T>
struct MsgH {
  T h, x;
};

// Workgroups are dealt round-robin over the 8 XCDs of the chip.  Give each
// XCD a contiguous range of logical row groups so that rows that exchange
// messages (neighbours in a banded or grid ordering) share one L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, rem = nb % kXcd;
  const int x = b % kXcd, j = b / kXcd;
  return x * q + min(x, rem) + j;
}

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic sum over the 256 lanes of a workgroup (fixed reduction tree).
template <typename V>
__device__ __forceinline__ V block_sum(V v, V* s_red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// Residual bookkeeping shared by the sweep and outer kernels: every workgroup
// stores its partial sum of r_i^2 with a plain store; k_check_finish, launched
// right after, adds the partials in index order and updates the status.  No
// fence or device-scope atomic is needed inside the sweep: the kernel boundary
// makes the partials visible.
__device__ __forceinline__ void store_partial(double res2, double* s_red, double* partials, int b) {
  const double bs = block_sum(res2, s_red);
  if (threadIdx.x == 0) partials[b] = bs;
}

constexpr int kFinishBlock = 1024;

__global__ __launch_bounds__(kFinishBlock) void k_check_finish(const double* __restrict__ partials, int nblk,
                                                               DevStatus* st, const double* rhs_norm,
                                                               double tol, int round, double* norm_out,
                                                               int gate_on_done, double diverge_limit,
                                                               DevStatus* mirror) {
  __shared__ double s_red[kFinishBlock / 64];
  // the status, the norm of b and the partials are all requested before the
  // gate on a finished solve is taken, so that one round trip covers them
  DevStatus cur{};
  double nbv = 0.0;
  if (threadIdx.x == 0) {
    cur = *st;
    if (rhs_norm) nbv = *rhs_norm;
  }
  const int gated = gate_on_done ? st->done : 0;
  // thread t adds partials t + j * kFinishBlock: even j into v0, odd j into
  // v1, each in increasing j.  Thirty-two loads are issued before their
  // additions, so up to 32768 partials (16,384 workgroups at 512 slots on
  // the 2^20-node graphs) cost one round trip to memory; a missing element
  // counts as +0.0, which leaves a sum of squares bit for bit unchanged.
  constexpr int kAhead = 32;
  double v0 = 0.0, v1 = 0.0;
  for (int j0 = 0; j0 * kFinishBlock < nblk; j0 += kAhead) {
    double p[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const int i = threadIdx.x + (j0 + u) * kFinishBlock;
      p[u] = i < nblk ? partials[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kAhead; u += 2) {
      v0 += p[u];
      v1 += p[u + 1];
    }
  }
  if (gated) {
    if (mirror && threadIdx.x == 0) *mirror = cur;  // the host reads the final status there
    return;
  }
  double v = wave_sum(v0 + v1);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < kFinishBlock / 64; ++w) tot += s_red[w];
    const double rn = sqrt(tot);
    const double nb = rhs_norm ? nbv : rn;  // without one: relative to itself
    const double rel = nb > 0.0 ? rn / nb : rn;
    if (norm_out) *norm_out = rn;
    cur.prev_rel = cur.last_rel;
    cur.prev_round = cur.last_round;
    cur.last_rel = rel;
    cur.last_round = round;
    if (rel <= tol) {
      cur.conv_round = round;
      cur.done = 1;
    } else if (!(rel <= diverge_limit)) {
      cur.error |= kErrDiverged;
      cur.done = 1;
    }
    *st = cur;
    if (mirror) *mirror = cur;
  }
}

hipError_t launch_check_finish(const double* partials, int nblk, DevStatus* st, const double* rhs_norm,
                               double tol, int round, double* norm_out, bool gate_on_done, hipStream_t s,
                               double diverge_limit, DevStatus* mirror) {
  hipLaunchKernelGGL(k_check_finish, dim3(1), dim3(kFinishBlock), 0, s, partials, nblk, st, rhs_norm, tol,
                     round, norm_out, gate_on_done ? 1 : 0, diverge_limit, mirror);
  return hipGetLastError();
}

size_t msg_bytes(int elt, bool joint) { return (size_t)elt * (joint ? 3 : 2); }

// LDS layout of the sweep kernel (bytes): row aggregates and means, staged
// incoming messages, staged a_ij x_j products, row pointers, local row of
// each slot.
__host__ __device__ constexpr size_t lds_layout(int K, int elt, bool joint) {
  return (size_t)elt * (3 * kMaxRowsPerBlock + (size_t)kBlock * K * (joint ? 3 : 2)) +
         sizeof(int32_t) * (kMaxRowsPerBlock + 4) + (size_t)kBlock * K;
}

size_t sweep_lds_bytes(int K, int elt, bool joint) { return lds_layout(K, elt, joint); }

// Gather of the reverse message (and the sender's mean) of slot s.
template <typename T, int MODE>
__device__ __forceinline__ void gather(const SweepArgs<T>& A, int s, T& pin, T& hin, T& xin) {
  const int rv = A.rev[s];
  if (MODE == kHOnly) {
    const MsgH<T> m = ((const MsgH<T>*)A.min)[rv];
    hin = m.h;
    xin = m.x;
  } else {
    const MsgJ<T> m = ((const MsgJ<T>*)A.min)[rv];
    pin = m.P;
    hin = m.h;
    xin = m.x;
  }
}

// A row longer than the workgroup's slot capacity: block-wide reductions,
// then a second pass over the row for the outgoing messages.
template <typename T, int MODE>
__device__ double long_row(const SweepArgs<T>& A, int r, int e0, int ne, T* s_redT, double* s_red,
                           T* s_bc) {
  constexpr bool kJointLike = (MODE == kJoint || MODE == kAgg || MODE == kFreeze);
  const int tid = threadIdx.x;
  T pP = 0, ph = 0;
  double pax = 0.0;
  for (int i = tid; i < ne; i += kBlock) {
    const int s = e0 + i;
    T pin = 0, hin = 0, xin = 0;
    if (MODE != kResid && !A.zero_in) gather<T, MODE>(A, s, pin, hin, xin);
    pP += pin;
    ph += hin;
    if (A.check) {
      const T xc = (MODE == kResid) ? A.xchk[A.off_col[s]] : xin;
      pax += (double)(A.a[s] * xc);
    }
  }
  pP = block_sum(pP, s_redT);
  ph = block_sum(ph, s_redT);
  pax = block_sum(pax, s_red);
  double res2 = 0.0;
  if (tid == 0) {
    const T Pt = kJointLike ? A.diag[r] + pP : T(0);
    const T ht = A.rhs[r] + ph;
    T xr = 0;
    if (MODE != kResid) {
      xr = (MODE == kHOnly) ? ht * A.inv_pt[r] : ht / Pt;
      if (A.xout) A.xout[r] = xr;
      if (A.ptout && kJointLike) A.ptout[r] = Pt;
      if (MODE == kFreeze) A.inv_pt_out[r] = T(1) / Pt;
    }
    if (A.check) {
      const double acc = (double)A.rhs[r] - (double)A.diag[r] * (double)A.xchk[r] - pax;
      res2 = acc * acc;
    }
    s_bc[0] = Pt;
    s_bc[1] = ht;
    s_bc[2] = xr;
  }
  __syncthreads();
  if (MODE == kJoint || MODE == kHOnly || MODE == kFreeze) {
    const T Pt = s_bc[0], ht = s_bc[1], xr = s_bc[2];
    bool bad = false;
    for (int i = tid; i < ne; i += kBlock) {
      const int s = e0 + i;
      T pin = 0, hin = 0, xin = 0;
      if (!A.zero_in) gather<T, MODE>(A, s, pin, hin, xin);
      if (MODE == kHOnly) {
        MsgH<T> m;
        m.h = A.gcoef[s] * (ht - hin);
        m.x = xr;
        ((MsgH<T>*)A.mout)[s] = m;
        bad |= !isfinite(m.h);
      } else {
        const T av = A.a[s];
        const T inv = T(1) / (Pt - pin);
        if (MODE == kFreeze) {
          A.gcoef_out[s] = -av * inv;
          bad |= !isfinite(inv);
        } else {
          MsgJ<T> m;
          m.P = -av * av * inv;
          m.h = -av * (ht - hin) * inv;
          m.x = xr;
          ((MsgJ<T>*)A.mout)[s] = m;
          bad |= !(isfinite(m.P) && isfinite(m.h));
        }
      }
    }
    if (bad) {
      atomicOr(&A.st->error, kErrNonfinite);
      atomicExch(&A.st->done, 1);
    }
  }
  return res2;
}

template <typename T, int K, int MODE>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs<T> A) {
  constexpr bool kJointLike = (MODE == kJoint || MODE == kAgg || MODE == kFreeze);
  constexpr int S = kBlock * K;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[kBlock / 64];
  __shared__ T s_redT[kBlock / 64];
  __shared__ T s_bc[3];

  const int tid = threadIdx.x;
  // written by an earlier kernel: visible after the kernel boundary
  if (A.st->done) return;

  const int b = xcd_remap(blockIdx.x, A.nblk);
  const int r0 = A.blk_row[b], r1 = A.blk_row[b + 1];
  const int nrow = r1 - r0;
  const int e0 = A.off_ptr[r0];
  const int ne = A.off_ptr[r1] - e0;
  double res2 = 0.0;

  if (ne > S) {
    res2 = long_row<T, MODE>(A, r0, e0, ne, s_redT, s_red, s_bc);
  } else {
    T* s_Pt = (T*)smem;
    T* s_ht = s_Pt + kMaxRowsPerBlock;
    T* s_x = s_ht + kMaxRowsPerBlock;
    T* s_h = s_x + kMaxRowsPerBlock;
    T* s_ax = s_h + S;
    T* s_P = s_ax + S;  // joint-like modes only
    int32_t* s_ptr = (int32_t*)(s_P + (kJointLike ? S : 0));
    uint8_t* s_row = (uint8_t*)(s_ptr + kMaxRowsPerBlock + 4);

    for (int i = tid; i <= nrow; i += kBlock) s_ptr[i] = A.off_ptr[r0 + i] - e0;

    // 1. slot phase: coalesced rev/a, gather of the reverse message
    T pin[K], hin[K], coef[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      pin[k] = 0;
      hin[k] = 0;
      coef[k] = 0;
      if (i < ne) {
        const int s = e0 + i;
        T xin = 0;
        if (MODE != kResid) {
          if (MODE == kHOnly) coef[k] = A.gcoef[s];
          else if (MODE != kAgg) coef[k] = A.a[s];
          if (!A.zero_in) gather<T, MODE>(A, s, pin[k], hin[k], xin);
          if (kJointLike) s_P[i] = pin[k];
          s_h[i] = hin[k];
        }
        if (A.check) {
          const T av = (MODE == kJoint || MODE == kFreeze) ? coef[k] : A.a[s];
          const T xc = (MODE == kResid) ? A.xchk[A.off_col[s]] : xin;
          s_ax[i] = av * xc;
        }
      }
    }
    __syncthreads();

    // 2. row phase: node aggregates of Alg. 2, tentative mean, residual
    if (tid < nrow) {
      const int r = r0 + tid;
      const int lo = s_ptr[tid], hi = s_ptr[tid + 1];
      if (MODE != kResid) {
        T Pt = kJointLike ? A.diag[r] : T(0);
        T ht = A.rhs[r];
        fill_row_ids(s_row, lo, hi, tid);
        if (kJointLike) Pt = lds_row_sum(Pt, s_P, lo, hi);
        ht = lds_row_sum(ht, s_h, lo, hi);
        const T xr = (MODE == kHOnly) ? ht * A.inv_pt[r] : ht / Pt;
        s_ht[tid] = ht;
        s_Pt[tid] = Pt;
        s_x[tid] = xr;
        if (A.xout) A.xout[r] = xr;
        if (A.ptout && kJointLike) A.ptout[r] = Pt;
        if (MODE == kFreeze) A.inv_pt_out[r] = T(1) / Pt;
      }
      if (A.check) {
        double acc = (double)A.rhs[r] - (double)A.diag[r] * (double)A.xchk[r];
        acc = lds_row_sub(acc, s_ax, lo, hi);
        res2 = acc * acc;
      }
    }
    __syncthreads();

    // 3. edge phase: new outgoing messages, reverse message subtracted
    if (MODE == kJoint || MODE == kHOnly || MODE == kFreeze) {
      bool bad = false;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = tid + k * kBlock;
        if (i < ne) {
          const int s = e0 + i;
          const int lr = s_row[i];
          if (MODE == kHOnly) {
            MsgH<T> m;
            m.h = coef[k] * (s_ht[lr] - hin[k]);
            m.x = s_x[lr];
            ((MsgH<T>*)A.mout)[s] = m;
            bad |= !isfinite(m.h);
          } else {
            const T inv = T(1) / (s_Pt[lr] - pin[k]);
            const T av = coef[k];
            if (MODE == kFreeze) {
              A.gcoef_out[s] = -av * inv;
              bad |= !isfinite(inv);
            } else {
              MsgJ<T> m;
              m.P = -av * av * inv;
              m.h = -av * (s_ht[lr] - hin[k]) * inv;
              m.x = s_x[lr];
              ((MsgJ<T>*)A.mout)[s] = m;
              bad |= !(isfinite(m.P) && isfinite(m.h));
            }
          }
        }
      }
      if (bad) {
        atomicOr(&A.st->error, kErrNonfinite);
        atomicExch(&A.st->done, 1);
      }
    }
  }

  if (A.check) store_partial(res2, s_red, A.partials, b);
}

// ev0/ev1 (nullable): events attached to the dispatch itself, so that their
// interval is the kernel's own execution time.
template <typename T, int K>
static hipError_t launch_k(int mode, const SweepArgs<T>& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const bool joint = (mode == kJoint || mode == kAgg || mode == kFreeze);
  const uint32_t lds = (uint32_t)lds_layout(K, sizeof(T), joint);
  const dim3 grid(a.nblk), block(kBlock);
  switch (mode) {
    case kJoint: hipExtLaunchKernelGGL((k_sweep<T, K, kJoint>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kHOnly: hipExtLaunchKernelGGL((k_sweep<T, K, kHOnly>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kAgg: hipExtLaunchKernelGGL((k_sweep<T, K, kAgg>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kFreeze: hipExtLaunchKernelGGL((k_sweep<T, K, kFreeze>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kResid: hipExtLaunchKernelGGL((k_sweep<T, K, kResid>), grid, block, lds, s, ev0, ev1, 0, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(int mode, int K, const SweepArgs<T>& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.nblk <= 0) return hipSuccess;
  switch (K) {
    case 2: return launch_k<T, 2>(mode, a, s, ev0, ev1);
    case 4: return launch_k<T, 4>(mode, a, s, ev0, ev1);
    case 8: return launch_k<T, 8>(mode, a, s, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_sweep<double>(int, int, const SweepArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_sweep<float>(int, int, const SweepArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);

// ---------------------------------------------------------------------------
// outer correction step (FP64): x_new = x_old + d, r = b - A x_new
// ---------------------------------------------------------------------------

// x_new = x_old + d, the correction d taken from the inner solve's round that
// met the inner tolerance (chosen on the device by the inner status).
__global__ void k_update(OuterArgs A) {
  if (A.reset_st && blockIdx.x == 0 && threadIdx.x == 0) reset_status_dev(A.st);
  const DevStatus* si = A.st_in;
  const int round = (si && si->conv_round >= 0) ? si->conv_round : A.in_fallback;
  const float* d32 = A.d32[round & 1];
  const double* d64 = A.d64[round & 1];
  const void* agg = A.dagg[round % 3];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += gridDim.x * blockDim.x) {
    double v = A.xold ? A.xold[i] : 0.0;
    if (A.use_d) {
      if (A.dagg_elt == 4) {
        const float2 g = ((const float2*)agg)[i];
        v += (double)(A.dagg_honly ? g.y * g.x : g.y / g.x);
      } else if (A.dagg_elt == 8) {
        const double2 g = ((const double2*)agg)[i];
        v += A.dagg_honly ? g.y * g.x : g.y / g.x;
      } else {
        v += d64 ? d64[i] : (double)d32[i];
      }
    }
    A.xnew[i] = v;
  }
}

// r = b - A x_new in FP64 (one gather of x per slot), the inner right-hand
// side in the inner precision, and the partial sums of r^2.
template <int K>
__global__ __launch_bounds__(kBlock) void k_outer(OuterArgs A) {
  constexpr int S = kBlock * K;
  __shared__ double s_ax[S];
  __shared__ int32_t s_ptr[kMaxRowsPerBlock + 4];
  __shared__ double s_red[kBlock / 64];
  if (A.gate && A.gate->done) return;  // a residual queued past the end of a solve
  const int tid = threadIdx.x;
  const int b = xcd_remap(blockIdx.x, A.nblk);
  const int r0 = A.blk_row[b], r1 = A.blk_row[b + 1];
  const int nrow = r1 - r0;
  const int e0 = A.off_ptr[r0];
  const int ne = A.off_ptr[r1] - e0;
  const double* x = A.xnew;
  double res2 = 0.0;
  if (ne > S) {  // one long row
    double p = 0.0;
    for (int i = tid; i < ne; i += kBlock) p += A.a[e0 + i] * x[A.off_col[e0 + i]];
    p = block_sum(p, s_red);
    if (tid == 0) {
      const double res = A.b[r0] - A.diag[r0] * x[r0] - p;
      if (A.rin32) A.rin32[r0] = (float)res;
      if (A.rin64) A.rin64[r0] = res;
      res2 = res * res;
    }
  } else {
    // every independent load first (the slots' columns and coefficients,
    // streamed once, then the rows' own data), the x gathers next, so that
    // their latencies overlap
    int c[K];
    double av[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      if (i < ne) {
        c[k] = __builtin_nontemporal_load(A.off_col + e0 + i);
        av[k] = __builtin_nontemporal_load(A.a + e0 + i);
      }
    }
    for (int i = tid; i <= nrow; i += kBlock) s_ptr[i] = A.off_ptr[r0 + i] - e0;
    double br = 0.0, dr = 0.0, xr = 0.0;
    if (tid < nrow) {
      br = A.b[r0 + tid];
      dr = A.diag[r0 + tid];
      xr = x[r0 + tid];
    }
    double xg[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      if (i < ne) xg[k] = x[c[k]];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      if (i < ne) s_ax[i] = av[k] * xg[k];
    }
    __syncthreads();
    if (tid < nrow) {
      const int r = r0 + tid;
      double res = br - dr * xr;
      res = lds_row_sub(res, s_ax, s_ptr[tid], s_ptr[tid + 1]);
      if (A.rin32) A.rin32[r] = (float)res;
      if (A.rin64) A.rin64[r] = res;
      res2 = res * res;
    }
  }
  store_partial(res2, s_red, A.partials, b);
}

// The first outer step from x = 0: x_new = 0 and r = b, so no gather is
// needed. Same row partition and per-workgroup partial sums as k_outer, so
// the residual norm is that of k_outer bit for bit.
__global__ __launch_bounds__(kBlock) void k_outer_zero(OuterArgs A) {
  __shared__ double s_red[kBlock / 64];
  if (A.reset_st && blockIdx.x == 0 && threadIdx.x == 0) reset_status_dev(A.st);
  const int b = xcd_remap(blockIdx.x, A.nblk);
  const int r0 = A.blk_row[b], r1 = A.blk_row[b + 1];
  double res2 = 0.0;
  if ((int)threadIdx.x < r1 - r0) {
    const int r = r0 + threadIdx.x;
    const double res = A.b[r];
    A.xnew[r] = 0.0;
    if (A.rin32) A.rin32[r] = (float)res;
    if (A.rin64) A.rin64[r] = res;
    res2 = res * res;
  }
  store_partial(res2, s_red, A.partials, b);
}

hipError_t launch_outer(int K, const OuterArgs& a, hipStream_t s) {
  if (a.nblk <= 0) return a.reset_st ? launch_reset_status(a.st, 1, s) : hipSuccess;
  hipError_t e;
  if (!a.xold && !a.use_d) {
    hipLaunchKernelGGL(k_outer_zero, dim3(a.nblk), dim3(kBlock), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_check_finish(a.partials, a.nblk, a.st, a.b_norm, a.tol, 0, a.r_norm, false, s, kDivergeLimit,
                               a.mirror);
  }
  hipLaunchKernelGGL(k_update, dim3(std::min((a.n + 255) / 256, 4096)), dim3(256), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_outer_only(K, a, s);
  if (e != hipSuccess) return e;
  return launch_check_finish(a.partials, a.nblk, a.st, a.b_norm, a.tol, 0, a.r_norm, false, s, kDivergeLimit,
                             a.mirror);
}

hipError_t launch_outer_only(int K, const OuterArgs& a, hipStream_t s) {
  const dim3 grid(a.nblk), block(kBlock);
  switch (K) {
    case 2: hipLaunchKernelGGL(k_outer<2>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_outer<4>, grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_outer<8>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

__global__ void k_reset_status(DevStatus* st, int count) {
  const int i = threadIdx.x;
  if (i < count) reset_status_dev(st + i);
}

hipError_t launch_reset_status(DevStatus* st, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, st, count);
  return hipGetLastError();
}

__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void k_poison(uint32_t* p, int64_t n, const DevStatus* st) {
  if (st && st->done) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0xffffffffu;
}

hipError_t launch_poison(void* p, size_t bytes, const DevStatus* st, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_poison, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, n, st);
  return hipGetLastError();
}

// ||v||_2 in two deterministic stages: per-workgroup partial sums, then one
// workgroup adding them in index order.
__global__ __launch_bounds__(kBlock) void k_sumsq_partial(const double* v, int64_t n, double* partials) {
  __shared__ double s_red[kBlock / 64];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    acc += v[i] * v[i];
  acc = block_sum(acc, s_red);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void k_sumsq_final(const double* partials, int nparts, double* out) {
  __shared__ double s_red[kBlock / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) acc += partials[i];
  acc = block_sum(acc, s_red);
  if (threadIdx.x == 0) *out = sqrt(acc);
}

hipError_t launch_norm(const double* v, int64_t n, double* partials, int nparts, double* out,
                       DevStatus*, hipStream_t s) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, nparts));
  hipLaunchKernelGGL(k_sumsq_partial, dim3(blocks), dim3(kBlock), 0, s, v, n, partials);
  hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(kBlock), 0, s, partials, blocks, out);
  return hipGetLastError();
}

// Final copy of the converged round (chosen on the device, no host sync):
// x = x_round, var = 1 / P~_round.
__global__ void k_copy_round(const double* x0, const double* x1, const double* p0, const double* p1,
                             const DevStatus* st, int32_t fallback, double* x, double* var, int32_t n) {
  const int round = st->conv_round >= 0 ? st->conv_round : fallback;
  const double* xs = (round & 1) ? x1 : x0;
  const double* ps = (round & 1) ? p1 : p0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    x[i] = xs[i];
    if (var) var[i] = 1.0 / ps[i];
  }
}

hipError_t launch_copy_round(const double* const* x2, const double* const* pt2, const DevStatus* st,
                             int32_t fallback_round, double* x, double* var, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_copy_round, dim3(blocks), dim3(256), 0, s, x2[0], x2[1], pt2 ? pt2[0] : nullptr,
                     pt2 ? pt2[1] : nullptr, st, fallback_round, x, var, n);
  return hipGetLastError();
}

__global__ void k_x_from_agg(const double2* a0, const double2* a1, const double2* a2, int32_t honly,
                             const DevStatus* st, int32_t fallback, double* x, int32_t n) {
  const int round = st->conv_round >= 0 ? st->conv_round : fallback;
  const double2* a = (round % 3 == 0) ? a0 : (round % 3 == 1) ? a1 : a2;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double2 v = a[i];
    x[i] = honly ? v.y * v.x : v.y / v.x;
  }
}

hipError_t launch_x_from_agg(void* const* agg, bool honly, const DevStatus* st, int32_t fallback_round, double* x,
                             int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_x_from_agg, dim3(blocks), dim3(256), 0, s, (const double2*)agg[0], (const double2*)agg[1],
                     (const double2*)agg[2], honly ? 1 : 0, st, fallback_round, x, n);
  return hipGetLastError();
}

// Aitken's delta-squared step on each node's last three means (Ch. 3
// Sec. 3.2).  hist holds round t-2 and is advanced to round t-1 by the same
// thread, so one vector of history suffices.  The second difference is formed
// as (x2 - 2 x1) + x0; 2 x1 is exact, so a fused multiply-add leaves it
// unchanged.
__global__ void k_aitken(const double* __restrict__ x1, const double* __restrict__ x2, double* hist,
                         double* __restrict__ y, const DevStatus* st, int make_y, int32_t n) {
  if (st->done) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double a = hist[i], b = x1[i];
    if (make_y) {
      const double c = x2[i];
      const double d1 = b - a;
      const double den = (c - 2.0 * b) + a;
      const double corr = d1 * d1 / den;
      y[i] = (den != 0.0 && isfinite(corr)) ? a - corr : c;
    }
    hist[i] = b;
  }
}

// Steffensen's restart (Ch. 3 Sec. 3.2): the extrapolated means replace the
// newest ones, so the next sweep's messages are formed from {P~_i, P~_i y_i}.
__global__ void k_steffensen(const double* __restrict__ x1, double* x2, double* start, double2* agg,
                             const DevStatus* st, int32_t n) {
  if (st->done) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double a = start[i], b = x1[i], c = x2[i];
    const double d1 = b - a;
    const double den = (c - 2.0 * b) + a;
    const double corr = d1 * d1 / den;
    const double y = (den != 0.0 && isfinite(corr)) ? a - corr : c;
    start[i] = y;
    x2[i] = y;
    double2 g = agg[i];
    g.y = g.x * y;
    agg[i] = g;
  }
}

hipError_t launch_steffensen(const double* x1, double* x2, double* start, void* agg, const DevStatus* st,
                             int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_steffensen, dim3(blocks), dim3(256), 0, s, x1, x2, start, (double2*)agg, st, n);
  return hipGetLastError();
}

hipError_t launch_aitken(const double* x1, const double* x2, double* hist, double* y, const DevStatus* st,
                         int make_y, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_aitken, dim3(blocks), dim3(256), 0, s, x1, x2, hist, y, st, make_y, n);
  return hipGetLastError();
}

// dL/dA on the stored pattern of the caller's CSR (tied mirror entries).
__global__ void k_grad_vals(const int32_t* row_ptr, const int32_t* col, const double* lam, const double* x,
                            double* gv, int32_t n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double lr = lam[r], xr = x[r];
  for (int32_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
    const int32_t c = col[e];
    gv[e] = (c == r) ? -lr * xr : -(lr * x[c] + lam[c] * xr);
  }
}

hipError_t launch_grad_vals(const int32_t* row_ptr, const int32_t* col, const double* lam, const double* x,
                            double* gv, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_vals, dim3((n + 255) / 256), dim3(256), 0, s, row_ptr, col, lam, x, gv, n);
  return hipGetLastError();
}

__global__ void k_scale_diag(const double* d, double f, double* out64, float* out32, int32_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double v = d[i] * f;
    if (out64) out64[i] = v;
    if (out32) out32[i] = (float)v;
  }
}

hipError_t launch_scale_diag(const double* d, double f, double* out64, float* out32, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_diag, dim3(std::min((n + 255) / 256, 4096)), dim3(256), 0, s, d, f, out64, out32, n);
  return hipGetLastError();
}

// Copy P and h out of the FP64 joint message records.
__global__ void k_split_msgs(const MsgJ<double>* m, double* P, double* h, int64_t E) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
    const MsgJ<double> v = m[i];
    P[i] = v.P;
    h[i] = v.h;
  }
}

hipError_t launch_split_pairs(const void* m, double* P, double* h, int64_t E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((E + 255) / 256, 4096);
  hipLaunchKernelGGL(k_split_msgs, dim3(blocks), dim3(256), 0, s, (const MsgJ<double>*)m, P, h, E);
  return hipGetLastError();
}

}  // namespace gabp
