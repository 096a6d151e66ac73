// Node-broadcast sweep kernels: the broadcast variant of Alg. 2 (Ch. 3
// Sec. 3.3) taken literally.  Node i publishes only its aggregate
// (P~_i, h~_i); the receiving node j forms the incoming message i -> j itself,
// subtracting the message j -> i that it sent in the previous round:
//     P_ij = -A_ij^2 / (P~_i - P_ji),  h_ij = -A_ij (h~_i - h_ji) / (P~_i - P_ji).
// Every slot (j, i) of row j therefore keeps the pair of messages on its edge
// (in = i -> j, out = j -> i) in place; a sweep reads and rewrites that pair
// with coalesced accesses and gathers only the neighbour's aggregate from an
// n-sized array, which stays largely resident in L2 and the Infinity Cache.
// No reverse-slot index is needed.
//
// Sweep t (t >= 1) reads the aggregates A^(t-1) and the slot pairs of round
// t-1 and writes
//   in^(t)  = F(A_i^(t-1), out^(t-1)),   out^(t) = F(A_j^(t-1), in^(t-1)),
//   A_j^(t) = (A_jj + sum_i P_in^(t), b_j + sum_i h_in^(t)),  x_j^(t) = h~/P~,
// and optionally checks the residual of round t-1, whose means come with the
// gathered aggregates.  With frozen precisions only the h parts move:
//   h_in = g_in (h~_i - h_out),  h_out = g_out (h~_j - h_in).
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>

#include "gabp_internal.h"

namespace gabp {

namespace {

template <typename T>
struct PairJ {  // joint slot state: message in (i -> j) and out (j -> i)
  T Pin, hin, Pout, hout;
};
template <typename T>
struct PairH {  // h-only slot state
  T hin, hout;
};
template <typename T>
struct Agg {  // published node aggregate
  T P, h;
};
template <typename T>
struct Coef {  // frozen h-update coefficients of a slot, and 1 / P~ of its neighbour
  T gin, gout, ipn;
};

__device__ __forceinline__ int xcd_remap_b(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, rem = nb % kXcd;
  const int x = b % kXcd, j = b / kXcd;
  return x * q + min(x, rem) + j;
}

template <typename V>
__device__ __forceinline__ V wsum(V v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename V>
__device__ __forceinline__ V bsum(V v, V* s_red) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// Streamed data (slot pairs, coefficients, columns, A_ij) is read and written
// once per sweep: non-temporal accesses keep it from displacing the gathered
// neighbour aggregates in L2.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ PairJ<T> ld_pairj(const void* base, int s) {
  const vec2<T>* q = (const vec2<T>*)base + 2 * (size_t)s;
  const vec2<T> a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + 1);
  return PairJ<T>{a.x, a.y, b.x, b.y};
}
template <typename T>
__device__ __forceinline__ void st_pairj(void* base, int s, const PairJ<T>& v) {
  vec2<T>* q = (vec2<T>*)base + 2 * (size_t)s;
  vec2<T> a, b;
  a.x = v.Pin;
  a.y = v.hin;
  b.x = v.Pout;
  b.y = v.hout;
  __builtin_nontemporal_store(a, q);
  __builtin_nontemporal_store(b, q + 1);
}
template <typename T>
__device__ __forceinline__ PairH<T> ld_pairh(const void* base, int s) {
  const vec2<T> a = __builtin_nontemporal_load((const vec2<T>*)base + s);
  return PairH<T>{a.x, a.y};
}
template <typename T>
__device__ __forceinline__ void st_pairh(void* base, int s, const PairH<T>& v) {
  vec2<T> a;
  a.x = v.hin;
  a.y = v.hout;
  __builtin_nontemporal_store(a, (vec2<T>*)base + s);
}
template <typename T>
__device__ __forceinline__ Coef<T> ld_coef(const void* base, int s) {
  const T* q = (const T*)base + 3 * (size_t)s;
  return Coef<T>{__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1), __builtin_nontemporal_load(q + 2)};
}

__host__ __device__ constexpr size_t bc_lds(int K, int elt) {
  // s_Pn, s_hn, s_ax [S]; s_AoP, s_Aoh [rows]; s_ptr [rows+4]; s_row [S]
  return (size_t)elt * (3 * (size_t)kBlock * K + 2 * kMaxRowsPerBlock) + sizeof(int32_t) * (kMaxRowsPerBlock + 4) +
         (size_t)kBlock * K;
}

// Per-slot work shared by the multi-row and long-row paths.  Returns the
// incoming message of round t (P, h) and the a_ij x_i term of the check.
template <typename T, int MODE>
__device__ __forceinline__ void slot_update(const BcastArgs<T>& A, int s, T AoP, T Aoh, T& Pn, T& hn, T& ax) {
  const int c = ld_stream(A.col + s);
  const T av = ld_stream(A.a + s);
  Pn = 0;
  hn = 0;
  ax = 0;
  if (MODE == kJoint || MODE == kFreeze) {
    PairJ<T> st{0, 0, 0, 0};
    T Pi, hi;
    if (A.zero_in) {
      Pi = A.diag[c];
      hi = A.rhs[c];
    } else {
      st = ld_pairj<T>(A.state, s);
      const Agg<T> ag = ((const Agg<T>*)A.aold)[c];
      Pi = ag.P;
      hi = ag.h;
    }
    const T inv_in = T(1) / (Pi - st.Pout);
    const T inv_out = T(1) / (AoP - st.Pin);
    if (MODE == kFreeze) {
      Coef<T> cf;
      cf.gin = -av * inv_in;
      cf.gout = -av * inv_out;
      cf.ipn = T(1) / Pi;
      ((Coef<T>*)A.coef_out)[s] = cf;
      Pn = inv_in;  // only checked for finiteness
      hn = inv_out;
    } else {
      PairJ<T> ns;
      ns.Pin = -av * av * inv_in;
      ns.hin = -av * (hi - st.hout) * inv_in;
      ns.Pout = -av * av * inv_out;
      ns.hout = -av * (Aoh - st.hin) * inv_out;
      st_pairj<T>(A.state, s, ns);
      Pn = ns.Pin;
      hn = ns.hin;
    }
    if (A.check) ax = av * (hi / Pi);
  } else if (MODE == kHOnly) {
    const Coef<T> cf = ld_coef<T>(A.coef, s);
    PairH<T> st{0, 0};
    T hi;
    if (A.zero_in) {
      hi = A.rhs[c];
    } else {
      st = ld_pairh<T>(A.state, s);
      hi = ((const T*)A.aold)[c];
    }
    PairH<T> ns;
    ns.hin = cf.gin * (hi - st.hout);
    ns.hout = cf.gout * (Aoh - st.hin);
    st_pairh<T>(A.state, s, ns);
    hn = ns.hin;
    // the neighbour's mean from its published h~ and its frozen 1/P~
    if (A.check) ax = av * (hi * cf.ipn);
  } else {  // kResid: neighbours' means of the published round
    T xc;
    if (A.zero_in) xc = A.honly_nodes ? A.rhs[c] * A.inv_pt[c] : A.rhs[c] / A.diag[c];
    else if (A.honly_nodes) xc = A.xold[c];
    else {
      const Agg<T> ag = ((const Agg<T>*)A.aold)[c];
      xc = ag.h / ag.P;
    }
    ax = av * xc;
  }
}

template <typename T, int K, int MODE>
__global__ __launch_bounds__(kBlock) void k_bcast(BcastArgs<T> A) {
  constexpr int S = kBlock * K;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[kBlock / 64];
  __shared__ T s_redT[kBlock / 64];
  if (A.st->done) return;

  const int tid = threadIdx.x;
  const int b = xcd_remap_b(blockIdx.x, A.nblk);
  const int r0 = A.blk_row[b], r1 = A.blk_row[b + 1];
  const int nrow = r1 - r0;
  const int e0 = A.off_ptr[r0];
  const int ne = A.off_ptr[r1] - e0;
  constexpr bool kJoint_ = (MODE == kJoint || MODE == kFreeze);
  double res2 = 0.0;
  bool bad = false;

  // own aggregate of round t-1 (published by the previous sweep)
  const bool joint_nodes = kJoint_ || (MODE == kResid && !A.honly_nodes);
  auto own = [&](int r, T& P, T& h) {
    if (A.zero_in) {
      P = joint_nodes ? A.diag[r] : T(0);
      h = A.rhs[r];
    } else if (joint_nodes) {
      const Agg<T> ag = ((const Agg<T>*)A.aold)[r];
      P = ag.P;
      h = ag.h;
    } else {
      P = 0;
      h = ((const T*)A.aold)[r];
    }
  };
  auto own_x = [&](int r, T P, T h) -> T {
    if (MODE == kHOnly) return h * A.inv_pt[r];
    if (!joint_nodes) return A.zero_in ? A.rhs[r] * A.inv_pt[r] : A.xold[r];
    return h / P;
  };

  if (ne > S) {  // one long row: per-lane partial sums, block reductions
    T AoP, Aoh;
    own(r0, AoP, Aoh);
    T pP = 0, ph = 0;
    double pax = 0.0;
    for (int i = tid; i < ne; i += kBlock) {
      T Pn, hn, ax;
      slot_update<T, MODE>(A, e0 + i, AoP, Aoh, Pn, hn, ax);
      pP += Pn;
      ph += hn;
      pax += (double)ax;
      if (MODE != kResid) bad |= !(isfinite(Pn) && isfinite(hn));
    }
    pP = bsum(pP, s_redT);
    ph = bsum(ph, s_redT);
    pax = bsum(pax, s_red);
    if (tid == 0) {
      const int r = r0;
      if (MODE == kJoint) {
        Agg<T> an;
        an.P = A.diag[r] + pP;
        an.h = A.rhs[r] + ph;
        ((Agg<T>*)A.anew)[r] = an;
        if (A.xout) A.xout[r] = an.h / an.P;
        if (A.ptout) A.ptout[r] = an.P;
      } else if (MODE == kHOnly) {
        const T ht = A.rhs[r] + ph;
        ((T*)A.anew)[r] = ht;
        if (A.xout) A.xout[r] = ht * A.inv_pt[r];
      } else if (MODE == kFreeze) {
        A.inv_pt_out[r] = T(1) / AoP;
      }
      if (A.zero_in && A.xout_prev) A.xout_prev[r] = own_x(r, AoP, Aoh);
      if (A.zero_in && A.ptout_prev) A.ptout_prev[r] = AoP;
      if (A.check) {
        const double acc = (double)A.rhs[r] - (double)A.diag[r] * (double)own_x(r, AoP, Aoh) - pax;
        res2 = acc * acc;
      }
    }
  } else {
    T* s_Pn = (T*)smem;
    T* s_hn = s_Pn + S;
    T* s_ax = s_hn + S;
    T* s_AoP = s_ax + S;
    T* s_Aoh = s_AoP + kMaxRowsPerBlock;
    int32_t* s_ptr = (int32_t*)(s_Aoh + kMaxRowsPerBlock);
    uint8_t* s_row = (uint8_t*)(s_ptr + kMaxRowsPerBlock + 4);

    for (int i = tid; i <= nrow; i += kBlock) s_ptr[i] = A.off_ptr[r0 + i] - e0;
    __syncthreads();
    if (tid < nrow) {
      T P, h;
      own(r0 + tid, P, h);
      s_AoP[tid] = P;
      s_Aoh[tid] = h;
      fill_row_ids(s_row, s_ptr[tid], s_ptr[tid + 1], tid);
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      if (i < ne) {
        const int lr = s_row[i];
        T Pn, hn, ax;
        slot_update<T, MODE>(A, e0 + i, s_AoP[lr], s_Aoh[lr], Pn, hn, ax);
        s_Pn[i] = Pn;
        s_hn[i] = hn;
        s_ax[i] = ax;
        if (MODE != kResid) bad |= !(isfinite(Pn) && isfinite(hn));
      }
    }
    __syncthreads();

    if (tid < nrow) {
      const int r = r0 + tid;
      const int lo = s_ptr[tid], hi = s_ptr[tid + 1];
      if (MODE == kJoint) {
        Agg<T> an;
        an.P = A.diag[r];
        an.h = A.rhs[r];
        an.P = lds_row_sum(an.P, s_Pn, lo, hi);
        an.h = lds_row_sum(an.h, s_hn, lo, hi);
        ((Agg<T>*)A.anew)[r] = an;
        if (A.xout) A.xout[r] = an.h / an.P;
        if (A.ptout) A.ptout[r] = an.P;
      } else if (MODE == kHOnly) {
        T ht = A.rhs[r];
        ht = lds_row_sum(ht, s_hn, lo, hi);
        ((T*)A.anew)[r] = ht;
        if (A.xout) A.xout[r] = ht * A.inv_pt[r];
      } else if (MODE == kFreeze) {
        A.inv_pt_out[r] = T(1) / s_AoP[tid];
      }
      if (A.zero_in && A.xout_prev) A.xout_prev[r] = own_x(r, s_AoP[tid], s_Aoh[tid]);
      if (A.zero_in && A.ptout_prev) A.ptout_prev[r] = s_AoP[tid];
      if (A.check) {
        double acc = (double)A.rhs[r] - (double)A.diag[r] * (double)own_x(r, s_AoP[tid], s_Aoh[tid]);
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
    const double bs = bsum(res2, s_red);
    if (tid == 0) A.partials[b] = bs;
  }
}

template <typename T, int K>
hipError_t launch_bk(int mode, const BcastArgs<T>& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const uint32_t lds = (uint32_t)bc_lds(K, sizeof(T));
  const dim3 grid(a.nblk), block(kBlock);
  switch (mode) {
    case kJoint: hipExtLaunchKernelGGL((k_bcast<T, K, kJoint>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kHOnly: hipExtLaunchKernelGGL((k_bcast<T, K, kHOnly>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kFreeze: hipExtLaunchKernelGGL((k_bcast<T, K, kFreeze>), grid, block, lds, s, ev0, ev1, 0, a); break;
    case kResid: hipExtLaunchKernelGGL((k_bcast<T, K, kResid>), grid, block, lds, s, ev0, ev1, 0, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Copy P and h of the outgoing messages (j -> i in slot (j, i)) out of the
// FP64 joint slot states.
__global__ void k_split_out(const PairJ<double>* st, double* P, double* h, int64_t E) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
    const PairJ<double> v = st[i];
    P[i] = v.Pout;
    h[i] = v.hout;
  }
}

}  // namespace

size_t bcast_state_bytes(int elt) { return 4 * (size_t)elt; }
size_t bcast_coef_bytes(int elt) { return 3 * (size_t)elt; }
size_t bcast_lds_bytes(int K, int elt) { return bc_lds(K, elt); }

template <typename T>
hipError_t launch_bcast(int mode, int K, const BcastArgs<T>& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.nblk <= 0) return hipSuccess;
  switch (K) {
    case 2: return launch_bk<T, 2>(mode, a, s, ev0, ev1);
    case 4: return launch_bk<T, 4>(mode, a, s, ev0, ev1);
    case 8: return launch_bk<T, 8>(mode, a, s, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_bcast<double>(int, int, const BcastArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_bcast<float>(int, int, const BcastArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);

hipError_t launch_split_out(const void* state, double* P, double* h, int64_t E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((E + 255) / 256, 4096);
  hipLaunchKernelGGL(k_split_out, dim3(blocks), dim3(256), 0, s, (const PairJ<double>*)state, P, h, E);
  return hipGetLastError();
}

}  // namespace gabp
