// Compact node-broadcast sweep kernels: the broadcast variant of Alg. 2
// (Ch. 3 Sec. 3.3) with ONE message per slot.
//
// Slot (j, i) of row j keeps only the incoming message i -> j.  The outgoing
// message j -> i of the previous round is a function of data that row j owns,
//     out^(t-1) = F(A_j^(t-2), in^(t-2)),
// so it is recomputed instead of stored, and the new incoming message is
//     in^(t)    = F(A_i^(t-1), out^(t-1)),
// with F(A, m) = (-a^2 / (A.P - m.P), -a (A.h - m.h) / (A.P - m.P)) the
// message update of Alg. 2 in information form (P~, h~ the node aggregates).
// in^(t) depends on in^(t-2) alone, so the even and the odd rounds each update
// one slot buffer in place, and the node aggregates rotate through three
// buffers (rounds t-2, t-1, t).  Per slot a sweep streams the column, A_ij and
// one message pair, and gathers the neighbour's aggregate of round t-1, which
// also yields the neighbour's mean for the residual check of round t-1.
//
// Frozen precisions (h-only sweeps):
//     h_out = g_out (h~_j^(t-2) - h_in^(t-2)),   h_in = g_in (h~_i^(t-1) - h_out),
// and the aggregate record of a node is {1/P~, h~}.  The iteration is the same
// as that of the two-message node layout, operation for operation.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>

#include "gabp_internal.h"

// Keep every product and sum separately rounded, as in the two-message layout
// (a fused multiply-add across the recomputed outgoing message would change
// the rounding of the iteration).
#pragma clang fp contract(off)

namespace gabp {

namespace {

template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));

template <typename T>
struct Msg {  // one message in information form
  T P, h;
};

__device__ __forceinline__ int xcd_remap_c(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, rem = nb % kXcd;
  const int x = b % kXcd, j = b / kXcd;
  return x * q + min(x, rem) + j;
}

template <typename V>
__device__ __forceinline__ V wsum_c(V v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename V>
__device__ __forceinline__ V bsum_c(V v, V* s_red) {
  v = wsum_c(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// Streamed per-slot data is touched once per sweep: non-temporal accesses keep
// it from displacing the gathered aggregates in L2.
template <typename T>
__device__ __forceinline__ T lds_(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ Msg<T> ld_msg(const void* base, int s) {
  const vec2<T> v = __builtin_nontemporal_load((const vec2<T>*)base + s);
  return Msg<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st_msg(void* base, int s, T P, T h) {
  vec2<T> v;
  v.x = P;
  v.y = h;
  __builtin_nontemporal_store(v, (vec2<T>*)base + s);
}
template <typename T>
__device__ __forceinline__ Msg<T> ld_agg(const void* base, int q) {
  const vec2<T> v = ((const vec2<T>*)base)[q];
  return Msg<T>{v.x, v.y};
}

// Dynamic LDS of one workgroup: s_Pn, s_hn, s_ax [S]; the rows' own
// aggregates of round t-2 [rows] x 2, and of round t-1 [rows] x 2 for the
// freeze only (the other modes use those in the row lane's registers alone);
// s_ptr [rows+4]; s_row [S].  Leaving out the unused pair lets one more FP64
// workgroup reside per CU.
__host__ __device__ constexpr size_t cn_lds(int K, int elt, bool freeze) {
  return (size_t)elt * (3 * (size_t)kBlock * K + (freeze ? 4 : 2) * kMaxRowsPerBlock) +
         sizeof(int32_t) * (kMaxRowsPerBlock + 4) + (size_t)kBlock * K;
}

// Mean of a node from its aggregate record.
template <typename T, int MODE>
__device__ __forceinline__ T mean_of(const CnodeArgs<T>& A, Msg<T> g) {
  if (MODE == kHOnly || (MODE == kResid && A.honly_nodes)) return g.h * g.P;
  return g.h / g.P;
}

// Streamed inputs of one slot, loaded before anything that depends on the
// row structure so that their latency overlaps the rest of the prologue.
template <typename T>
struct SlotIn {
  int c;       // neighbour i of slot (j, i)
  T av;        // A_ji (0 when not needed)
  Msg<T> m;    // joint: in^(t-2); freeze: in^(T)
  T mold;      // h-only: h_in^(t-2); freeze: P_in^(T-1)
  vec2<T> cf;  // h-only: frozen {g_in, g_out}
};

template <typename T, int MODE>
__device__ __forceinline__ void load_slot(const CnodeArgs<T>& A, int s, SlotIn<T>& in) {
  in.c = lds_(A.col + s);
  // with frozen precisions A_ji enters only the residual check
  in.av = (MODE != kHOnly || A.check) ? lds_(A.a + s) : T(0);
  in.m = Msg<T>{0, 0};
  in.mold = 0;
  if (MODE == kJoint) {
    if (!A.first && !A.second) in.m = ld_msg<T>(A.cin, s);
  } else if (MODE == kHOnly) {
    in.cf = __builtin_nontemporal_load((const vec2<T>*)A.coef + s);
    if (!A.first && !A.second) in.mold = lds_((const T*)A.cin + s);
  } else if (MODE == kFreeze) {
    if (!A.first) {
      in.m = ld_msg<T>(A.cin, s);
      if (!A.second) in.mold = ld_msg<T>(A.cin_old, s).P;
    }
  }
}

// Per-slot arithmetic.  g: the neighbour's aggregate of round t-1 (T for the
// freeze); o1 / o2: the row's own aggregates of rounds t-1 and t-2 (T and
// T-1).  Returns the new incoming message (Pn, hn) and the a_ji x_i term of
// the residual check.
template <typename T, int MODE>
__device__ __forceinline__ void compute_slot(const CnodeArgs<T>& A, int s, const SlotIn<T>& in, Msg<T> g, Msg<T> o1,
                                             Msg<T> o2, T& Pn, T& hn, T& ax) {
  const T av = in.av;
  Pn = 0;
  hn = 0;
  ax = 0;
  if (MODE == kJoint) {
    T Pout = 0, hout = 0;
    if (!A.first) {  // out^(t-1) = F(A_j^(t-2), in^(t-2))
      const T inv_out = T(1) / (o2.P - in.m.P);
      Pout = -av * av * inv_out;
      hout = -av * (o2.h - in.m.h) * inv_out;
    }
    const T inv_in = T(1) / (g.P - Pout);  // in^(t) = F(A_i^(t-1), out^(t-1))
    Pn = -av * av * inv_in;
    hn = -av * (g.h - hout) * inv_in;
    st_msg<T>(A.cin, s, Pn, hn);
    if (A.check) ax = av * (g.h / g.P);
  } else if (MODE == kHOnly) {
    T hout = 0;
    if (!A.first) hout = in.cf.y * (o2.h - in.mold);
    hn = in.cf.x * (g.h - hout);
    __builtin_nontemporal_store(hn, (T*)A.cin + s);
    if (A.check) ax = av * (g.h * g.P);
  } else if (MODE == kFreeze) {
    // messages of round T: in^(T) from the slot, out^(T) recomputed
    T Pout = 0;
    if (!A.first) {
      const T inv_o = T(1) / (o2.P - in.mold);
      Pout = -av * av * inv_o;
    }
    const T inv_in = T(1) / (g.P - Pout);
    const T inv_out = T(1) / (o1.P - in.m.P);
    vec2<T> cf;
    cf.x = -av * inv_in;
    cf.y = -av * inv_out;
    ((vec2<T>*)A.coef_out)[s] = cf;
    Pn = inv_in;  // only checked for finiteness
    hn = inv_out;
  } else {  // kResid: means of the neighbours in round t-1
    ax = av * mean_of<T, MODE>(A, g);
  }
}

// Prior potential of round t: b, or with the single-loop feedback
// b + Gamma ((1 - s) x^(t-2) + s x^(t-1)), Gamma = diag - chk_diag.
template <typename T, int MODE>
__device__ __forceinline__ T cn_prior_h(const CnodeArgs<T>& A, int r, T br, Msg<T> o1, Msg<T> o2) {
  if (MODE != kJoint || !A.feedback) return br;
  const T x1 = o1.h / o1.P;
  const T x2 = A.first ? T(0) : o2.h / o2.P;
  return br + (A.diag[r] - A.chk_diag[r]) * ((T(1) - A.damp) * x2 + A.damp * x1);
}

// Diagonal of the checked system.
template <typename T>
__device__ __forceinline__ T cn_chk_d(const CnodeArgs<T>& A, int r, T dr) {
  return A.chk_diag ? A.chk_diag[r] : dr;
}

// Row epilogue: publish the aggregates (P, h) of round t, the means and, on
// the first sweep, the round-0 means.
template <typename T, int MODE>
__device__ __forceinline__ void cn_publish(const CnodeArgs<T>& A, int r, Msg<T> o1, T P, T h) {
  if (MODE == kJoint) {
    vec2<T> v;
    v.x = P;
    v.y = h;
    ((vec2<T>*)A.anew)[r] = v;
    if (A.xout) A.xout[r] = h / P;
    if (A.ptout) A.ptout[r] = P;
  } else if (MODE == kHOnly) {
    const T ip = A.inv_pt[r];
    vec2<T> v;
    v.x = ip;
    v.y = h;
    ((vec2<T>*)A.anew)[r] = v;
    if (A.xout) A.xout[r] = h * ip;
  } else if (MODE == kFreeze) {
    A.inv_pt_out[r] = T(1) / o1.P;
  }
  if (A.first && A.xout_prev) A.xout_prev[r] = mean_of<T, MODE>(A, o1);
  if (A.first && A.ptout_prev) A.ptout_prev[r] = o1.P;
}

// One chunk (at most 256 K slots) of a long row: the slots' new messages, and
// the chunk's partial sums of P, h and the residual terms in lpart.
template <typename T, int K, int MODE>
__device__ __forceinline__ void cnode_chunk(const CnodeArgs<T>& A, const LongRow& L, int ci, double* s_red,
                                            T* s_redT) {
  constexpr int S = kBlock * K;
  const int tid = threadIdx.x;
  const int r = L.row;
  const int e0 = L.e0 + ci * S;
  const int ne = min(S, L.ne - ci * S);
  const bool need_o2 = (MODE == kJoint || MODE == kHOnly || MODE == kFreeze) && !A.first;
  SlotIn<T> in[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * kBlock;
    if (i < ne) load_slot<T, MODE>(A, e0 + i, in[k]);
  }
  const Msg<T> o1 = ld_agg<T>(A.agg1, r);
  const Msg<T> o2 = need_o2 ? ld_agg<T>(A.agg2, r) : Msg<T>{0, 0};
  Msg<T> g[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * kBlock;
    if (i < ne) g[k] = ld_agg<T>(A.agg1, in[k].c);
  }
  T pP = 0, ph = 0;
  double pax = 0.0;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * kBlock;
    if (i < ne) {
      T Pn, hn, ax;
      compute_slot<T, MODE>(A, e0 + i, in[k], g[k], o1, o2, Pn, hn, ax);
      pP += Pn;
      ph += hn;
      pax += (double)ax;
      if (MODE != kResid) bad |= !(isfinite(Pn) && isfinite(hn));
    }
  }
  if (bad) {
    atomicOr(&A.st->error, kErrNonfinite);
    atomicExch(&A.st->done, 1);
  }
  pP = bsum_c(pP, s_redT);
  ph = bsum_c(ph, s_redT);
  pax = bsum_c(pax, s_red);
  if (tid == 0) {
    double* q = A.lpart + 4 * (size_t)(L.cbase + ci);
    q[0] = (double)pP;
    q[1] = (double)ph;
    q[2] = pax;
  }
}

template <typename T, int K, int MODE>
__global__ __launch_bounds__(kBlock) void k_cnode(CnodeArgs<T> A) {
  constexpr int S = kBlock * K;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[kBlock / 64];
  __shared__ T s_redT[kBlock / 64];
  if (A.st->done) return;
  if ((int)blockIdx.x >= A.nblk) {  // a chunk of a long row
    const ChunkRef x = A.xch[blockIdx.x - A.nblk];
    cnode_chunk<T, K, MODE>(A, A.longs[x.li], x.c, s_red, s_redT);
    return;
  }

  const int tid = threadIdx.x;
  const int b = xcd_remap_c(blockIdx.x, A.nblk);
  const int r0 = A.blk_row[b], r1 = A.blk_row[b + 1];
  const int e0 = A.blk_e0[b], ne = A.blk_e0[b + 1] - e0;
  const int nrow = r1 - r0;
  // a long row is swept by its chunk workgroups and finished by k_cnode_long
  if (ne > S) return;
  // own-aggregate records: o1 = round t-1 (T), o2 = round t-2 (T-1)
  const bool need_o2 = (MODE == kJoint || MODE == kHOnly || MODE == kFreeze) && !A.first;
  double res2 = 0.0;
  bool bad = false;

  {
    T* s_Pn = (T*)smem;
    T* s_hn = s_Pn + S;
    T* s_ax = s_hn + S;
    constexpr int kO1 = MODE == kFreeze ? kMaxRowsPerBlock : 0;  // round t-1 pair: freeze only
    T* s_o2P = s_ax + S;
    T* s_o2h = s_o2P + kMaxRowsPerBlock;
    T* s_o1P = s_o2h + kMaxRowsPerBlock;
    T* s_o1h = s_o1P + kO1;
    int32_t* s_ptr = (int32_t*)(s_o1h + kO1);
    uint8_t* s_row = (uint8_t*)(s_ptr + kMaxRowsPerBlock + 4);

    // 1. every independent load at once: the slots' streamed data, then the
    //    rows' pointers, own aggregates and diagonal / right-hand side
    SlotIn<T> in[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      if (i < ne) load_slot<T, MODE>(A, e0 + i, in[k]);
    }
    const int r = r0 + tid;
    int rp = 0;
    Msg<T> o1{0, 0}, o2{0, 0};
    T dr = 0, br = 0;
    if (tid < nrow) {
      rp = A.off_ptr[r] - e0;
      o1 = ld_agg<T>(A.agg1, r);
      if (need_o2) o2 = ld_agg<T>(A.agg2, r);
      dr = A.diag[r];
      br = A.rhs[r];
    }
    // 2. the neighbours' aggregates (the only irregular reads)
    Msg<T> g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      if (i < ne) g[k] = ld_agg<T>(A.agg1, in[k].c);
    }
    // 3. row structure and own aggregates into LDS
    if (tid < nrow) {
      s_ptr[tid] = rp;
      if (kO1) {
        s_o1P[tid] = o1.P;
        s_o1h[tid] = o1.h;
      }
      s_o2P[tid] = o2.P;
      s_o2h[tid] = o2.h;
    }
    if (tid == 0) s_ptr[nrow] = ne;
    __syncthreads();
    if (tid < nrow) fill_row_ids(s_row, s_ptr[tid], s_ptr[tid + 1], tid);
    __syncthreads();

    // 4. slot arithmetic
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      if (i < ne) {
        const int lr = s_row[i];
        const Msg<T> q1 = kO1 ? Msg<T>{s_o1P[lr], s_o1h[lr]} : Msg<T>{0, 0};
        const Msg<T> q2{s_o2P[lr], s_o2h[lr]};
        T Pn, hn, ax;
        compute_slot<T, MODE>(A, e0 + i, in[k], g[k], q1, q2, Pn, hn, ax);
        s_Pn[i] = Pn;
        s_hn[i] = hn;
        s_ax[i] = ax;
        if (MODE != kResid) bad |= !(isfinite(Pn) && isfinite(hn));
      }
    }
    __syncthreads();

    // 5. row sums: diagonal first, then the slots in CSR order
    if (tid < nrow) {
      const int lo = s_ptr[tid], hi = s_ptr[tid + 1];
      T P = dr, h = cn_prior_h<T, MODE>(A, r, br, o1, o2);
      if (MODE == kJoint) P = lds_row_sum(P, s_Pn, lo, hi);
      if (MODE == kJoint || MODE == kHOnly) h = lds_row_sum(h, s_hn, lo, hi);
      cn_publish<T, MODE>(A, r, o1, P, h);
      if (A.check) {
        double acc = (double)br - (double)cn_chk_d(A, r, dr) * (double)mean_of<T, MODE>(A, o1);
        acc = lds_row_sub(acc, s_ax, lo, hi);
        res2 = acc * acc;
      }
    }
  }
  if (bad) {
    atomicOr(&A.st->error, kErrNonfinite);
    atomicExch(&A.st->done, 1);
  }
  if (A.check) {
    const double bs = bsum_c(res2, s_red);
    if (tid == 0) A.partials[b] = bs;
  }
}

// Finish of the long rows, one wave each: the chunks' partial sums are added
// in a fixed order (lane-strided, then a butterfly), and the row epilogue of
// the sweep follows, including the row's squared residual in the partial of
// the partition workgroup that holds the row.
template <typename T, int MODE>
__global__ __launch_bounds__(64) void k_cnode_long(CnodeArgs<T> A) {
  if (A.st->done) return;
  const LongRow L = A.longs[blockIdx.x];
  const int lane = threadIdx.x;
  T sP = 0, sh = 0;
  double sax = 0.0;
  for (int j = lane; j < L.nch; j += 64) {
    const double* q = A.lpart + 4 * (size_t)(L.cbase + j);
    sP += (T)q[0];
    sh += (T)q[1];
    sax += q[2];
  }
  sP = wsum_c(sP);
  sh = wsum_c(sh);
  sax = wsum_c(sax);
  if (lane == 0) {
    const int r = L.row;
    const bool need_o2 = (MODE == kJoint || MODE == kHOnly || MODE == kFreeze) && !A.first;
    const Msg<T> o1 = ld_agg<T>(A.agg1, r);
    const Msg<T> o2 = need_o2 ? ld_agg<T>(A.agg2, r) : Msg<T>{0, 0};
    const T dr = A.diag[r], br = A.rhs[r];
    cn_publish<T, MODE>(A, r, o1, dr + sP, cn_prior_h<T, MODE>(A, r, br, o1, o2) + sh);
    if (A.check) {
      const double acc = (double)br - (double)cn_chk_d(A, r, dr) * (double)mean_of<T, MODE>(A, o1) - sax;
      A.partials[L.blk] = acc * acc;
    }
  }
}

template <typename T, int K>
hipError_t launch_ck(int mode, const CnodeArgs<T>& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const uint32_t lds = (uint32_t)cn_lds(K, sizeof(T), mode == kFreeze);
  const dim3 grid(a.nblk + a.nxch), block(kBlock);
  switch (mode) {
    case kJoint: hipExtLaunchKernelGGL((k_cnode<T, K, kJoint>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kHOnly: hipExtLaunchKernelGGL((k_cnode<T, K, kHOnly>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kFreeze: hipExtLaunchKernelGGL((k_cnode<T, K, kFreeze>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kResid: hipExtLaunchKernelGGL((k_cnode<T, K, kResid>), grid, block, lds, s, ev0, ev1, 0, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.nlong == 0) return e;
  const dim3 lg(a.nlong), lb(64);
  switch (mode) {
    case kJoint: hipLaunchKernelGGL((k_cnode_long<T, kJoint>), lg, lb, 0, s, a); break;
    case kHOnly: hipLaunchKernelGGL((k_cnode_long<T, kHOnly>), lg, lb, 0, s, a); break;
    case kFreeze: hipLaunchKernelGGL((k_cnode_long<T, kFreeze>), lg, lb, 0, s, a); break;
    case kResid: hipLaunchKernelGGL((k_cnode_long<T, kResid>), lg, lb, 0, s, a); break;
  }
  return hipGetLastError();
}

// Outgoing messages of round T (slot (j, i) holds the message j -> i), FP64
// joint state: out^(T) = F(A_j^(T-1), in^(T-1)), one lane per row.  With
// zero_in the incoming messages of round T-1 are all zero (T = 1).
__global__ void k_cnode_out(int32_t n, const int32_t* __restrict__ off_ptr, const double* __restrict__ a,
                            const vec2<double>* __restrict__ in_prev, const vec2<double>* __restrict__ agg_prev,
                            int32_t zero_in, double* P, double* h) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const double AP = agg_prev[r].x, Ah = agg_prev[r].y;
    for (int s = off_ptr[r]; s < off_ptr[r + 1]; ++s) {
      double mP = 0.0, mh = 0.0;
      if (!zero_in) {
        mP = in_prev[s].x;
        mh = in_prev[s].y;
      }
      const double av = a[s];
      const double inv = 1.0 / (AP - mP);
      P[s] = -av * av * inv;
      h[s] = -av * (Ah - mh) * inv;
    }
  }
}

// The prior of every node as the aggregate record of round 0: (A_ii, b_i), or
// (1 / P~_i, b_i) with frozen precisions.  Gathered like any later round.
// With rst, the run's status is reset here too (one launch fewer).
template <typename T>
__global__ void k_cnode_prior(int32_t n, const T* __restrict__ first, const T* __restrict__ rhs,
                              vec2<T>* __restrict__ out, DevStatus* rst) {
  if (rst && blockIdx.x == 0 && threadIdx.x == 0) reset_status_dev(rst);
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    vec2<T> v;
    v.x = first[r];
    v.y = rhs[r];
    out[r] = v;
  }
}

}  // namespace

size_t cnode_lds_bytes(int K, int elt) { return cn_lds(K, elt, true); }

template <typename T>
hipError_t launch_cnode_prior(int32_t n, const T* first, const T* rhs, void* out, hipStream_t s, DevStatus* reset) {
  if (n <= 0) return reset ? launch_reset_status(reset, 1, s) : hipSuccess;
  const int blocks = std::min((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_cnode_prior<T>, dim3(blocks), dim3(256), 0, s, n, first, rhs, (vec2<T>*)out, reset);
  return hipGetLastError();
}
template hipError_t launch_cnode_prior<double>(int32_t, const double*, const double*, void*, hipStream_t,
                                               DevStatus*);
template hipError_t launch_cnode_prior<float>(int32_t, const float*, const float*, void*, hipStream_t, DevStatus*);

template <typename T>
hipError_t launch_cnode(int mode, int K, const CnodeArgs<T>& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.nblk <= 0) return hipSuccess;
  switch (K) {
    case 2: return launch_ck<T, 2>(mode, a, s, ev0, ev1);
    case 4: return launch_ck<T, 4>(mode, a, s, ev0, ev1);
    case 8: return launch_ck<T, 8>(mode, a, s, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_cnode<double>(int, int, const CnodeArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_cnode<float>(int, int, const CnodeArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);

hipError_t launch_cnode_out(int32_t n, const int32_t* off_ptr, const double* a, const void* in_prev,
                            const void* agg_prev, bool zero_in, double* P, double* h, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_cnode_out, dim3(blocks), dim3(256), 0, s, n, off_ptr, a, (const vec2<double>*)in_prev,
                     (const vec2<double>*)agg_prev, zero_in ? 1 : 0, P, h);
  return hipGetLastError();
}

}  // namespace gabp
