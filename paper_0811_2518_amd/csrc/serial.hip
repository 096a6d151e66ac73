// Colour-serial sweeps: the serial scheduling of Ch. 2 Sec. 2.3 applied to
// the broadcast updates of Alg. 2 (Ch. 3 Sec. 3.3), with all nodes of one
// colour class updated by one launch.
//
// The handle stores the system in colour order: class k is the row range
// [lo, hi), and no two rows of a class are neighbours.  Messages and
// aggregates form a single set, overwritten in place:
//   * slot (j, i) of row j holds out_{j->i}, the message node j sent to i at
//     its last update;
//   * agg[i] = {P~_i, h~_i} is the aggregate node i formed at its last update.
//
// Updating node j:
//   1. Pull each incoming message from the sender's aggregate,
//          in_{i->j} = F(agg_i, out_{j->i}),
//          F(A, m) = (-a^2 / (A.P - m.P), -a (A.h - m.h) / (A.P - m.P)).
//      This is exactly the message i sent.  i's update subtracted
//      out_{j->i}, and j has not been updated since, because a sweep
//      updates every node once.  In the first sweep a neighbour of a later
//      class has sent nothing yet, so it contributes the zero message of
//      the initial state.
//   2. Form P~_j = A_jj + sum P_in and h~_j = b_j + sum h_in.
//   3. Publish them with the mean h~_j / P~_j.
//   4. Store out_{j->i} = F(agg_j, in_{i->j}).
//
// Residual of the previous sweep's means, checked one sweep late.  With x_j
// taken from j's aggregate before its update,
//     r_j = b_j - A_jj x_j - L_j - U_j,
// where U_j is the part from neighbours of later classes (not yet updated
// in this sweep, so still at the previous one).  L_j is the part from
// earlier classes; j's own update stored it in the previous sweep, right
// after those classes had been updated.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "gabp_internal.h"

// Every product and sum is rounded separately.  The pulled message must
// equal, bit for bit, the one its sender subtracted.
#pragma clang fp contract(off)

namespace gabp {

namespace {

template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));

template <typename T>
struct Msg {
  T P, h;
};

__device__ __forceinline__ int xcd_remap_s(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, rem = nb % kXcd;
  const int x = b % kXcd, j = b / kXcd;
  return x * q + min(x, rem) + j;
}

template <typename V>
__device__ __forceinline__ V bsum_s(V v, V* s_red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

template <typename T>
__device__ __forceinline__ Msg<T> ld_pair(const void* base, int q) {
  const vec2<T> v = ((const vec2<T>*)base)[q];
  return Msg<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ Msg<T> ld_pair_nt(const void* base, int s) {
  const vec2<T> v = __builtin_nontemporal_load((const vec2<T>*)base + s);
  return Msg<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st_pair(void* base, int q, T P, T h) {
  vec2<T> v;
  v.x = P;
  v.y = h;
  ((vec2<T>*)base)[q] = v;
}
template <typename T>
__device__ __forceinline__ void st_pair_nt(void* base, int s, T P, T h) {
  vec2<T> v;
  v.x = P;
  v.y = h;
  __builtin_nontemporal_store(v, (vec2<T>*)base + s);
}

// F(A, m): the message a node with aggregate A sends back along a slot whose
// opposite message is m.
template <typename T>
__device__ __forceinline__ Msg<T> pass(T av, Msg<T> A, Msg<T> m) {
  const T inv = T(1) / (A.P - m.P);
  return Msg<T>{-av * av * inv, -av * (A.h - m.h) * inv};
}

__host__ __device__ constexpr size_t sr_lds(int K, int elt) {
  // s_Pn, s_hn [S] (T); s_ax [S] (double); new aggregates [rows] x 2 (T);
  // s_ptr [rows + 4]; s_row, s_low [S] (bytes)
  return (size_t)kBlock * K * (2 * (size_t)elt + sizeof(double) + 2) + 2 * (size_t)elt * kMaxRowsPerBlock +
         sizeof(int32_t) * (kMaxRowsPerBlock + 4);
}

// Pass 1 over one chunk (at most 256 K slots) of a long row: the pulled
// messages, kept in their slots until pass 2, and the chunk's partial sums of
// P, h and the two residual parts (earlier and later classes) in lpart.
template <typename T, int K, bool RESID>
__device__ __forceinline__ void serial_chunk(const SerialArgs<T>& A, const LongRow& L, int ci, double* s_red,
                                             T* s_redT) {
  constexpr int S = kBlock * K;
  const int tid = threadIdx.x;
  const int e0 = L.e0 + ci * S;
  const int ne = min(S, L.ne - ci * S);
  const bool check = RESID || A.check;
  int c[K];
  T av[K];
  Msg<T> m[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * kBlock;
    c[k] = 0;
    av[k] = 0;
    m[k] = Msg<T>{0, 0};
    if (i < ne) {
      c[k] = __builtin_nontemporal_load(A.col + e0 + i);
      av[k] = __builtin_nontemporal_load(A.a + e0 + i);
      if (!RESID && !A.first) m[k] = ld_pair_nt<T>(A.out, e0 + i);
    }
  }
  Msg<T> g[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * kBlock;
    if (i < ne) g[k] = ld_pair<T>(A.agg, c[k]);
  }
  T pP = 0, ph = 0;
  double pl = 0.0, pu = 0.0;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * kBlock;
    if (i < ne) {
      const bool lower = c[k] < A.lo;
      if (!RESID) {
        Msg<T> in{0, 0};
        if (!A.first || lower) in = pass<T>(av[k], g[k], m[k]);
        st_pair_nt<T>(A.out, e0 + i, in.P, in.h);
        pP += in.P;
        ph += in.h;
        bad |= !(isfinite(in.P) && isfinite(in.h));
      }
      if (lower ? (!RESID && A.wl) : check) {
        const double ax = (double)(av[k] * (g[k].h / g[k].P));
        if (lower) pl += ax;
        else pu += ax;
      }
    }
  }
  if (bad) {
    atomicOr(&A.st->error, kErrNonfinite);
    atomicExch(&A.st->done, 1);
  }
  pP = bsum_s(pP, s_redT);
  ph = bsum_s(ph, s_redT);
  pl = bsum_s(pl, s_red);
  pu = bsum_s(pu, s_red);
  if (tid == 0) {
    double* q = A.lpart + 4 * (size_t)(L.cbase + ci);
    q[0] = (double)pP;
    q[1] = (double)ph;
    q[2] = pl;
    q[3] = pu;
  }
}

// Finish and pass 2 of the long rows, one workgroup per chunk.  Every
// workgroup of a row adds the row's chunk sums in the same fixed order
// (lane-strided, then a butterfly), so all hold the same new aggregate.  The
// chunk-0 workgroup publishes it and the residual term of the previous sweep;
// every workgroup then replaces the pulled messages of its chunk by the
// outgoing ones, out_{j->i} = F(agg_j, in_{i->j}).
template <typename T, int K, bool RESID>
__global__ __launch_bounds__(kBlock) void k_serial_long(SerialArgs<T> A) {
  constexpr int S = kBlock * K;
  __shared__ double s_tot[4];
  if (A.st->done) return;
  const int tid = threadIdx.x;
  const ChunkRef x = A.xch[A.xch0 + blockIdx.x];
  const LongRow L = A.longs[x.li];
  const int r = L.row;
  const bool check = RESID || A.check;
  // the row's aggregate and earlier-class residual part of the previous sweep,
  // loaded before the barrier below, so that they have arrived before this
  // workgroup overwrites them
  Msg<T> o{1, 0};
  double lold = 0.0;
  if (x.c == 0 && tid == 0) {
    if (check) o = ld_pair<T>(A.agg, r);
    if (!RESID && A.check) lold = A.lsum[r];
  }
  if (tid < 64) {
    T sP = 0, sh = 0;
    double sl = 0.0, su = 0.0;
    for (int j = tid; j < L.nch; j += 64) {
      const double* q = A.lpart + 4 * (size_t)(L.cbase + j);
      sP += (T)q[0];
      sh += (T)q[1];
      sl += q[2];
      su += q[3];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      sP += __shfl_xor(sP, off, 64);
      sh += __shfl_xor(sh, off, 64);
      sl += __shfl_xor(sl, off, 64);
      su += __shfl_xor(su, off, 64);
    }
    if (tid == 0) {
      s_tot[0] = (double)sP;
      s_tot[1] = (double)sh;
      s_tot[2] = sl;
      s_tot[3] = su;
    }
  }
  __syncthreads();
  const T dr = A.diag[r], br = A.rhs[r];
  const Msg<T> an{dr + (T)s_tot[0], br + (T)s_tot[1]};
  if (x.c == 0 && tid == 0) {
    if (!RESID) {
      st_pair<T>(A.agg, r, an.P, an.h);
      if (A.xout) A.xout[r] = an.h / an.P;
      if (A.ptout) A.ptout[r] = an.P;
      if (A.wl) A.lsum[r] = s_tot[2];
    }
    if (check) {
      const double acc = (double)br - (double)dr * (double)(o.h / o.P) - lold - s_tot[3];
      A.partials[L.blk] = acc * acc;
    }
  }
  if (RESID) return;
  const int e0 = L.e0 + x.c * S;
  const int ne = min(S, L.ne - x.c * S);
  bool bad = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * kBlock;
    if (i < ne) {
      const Msg<T> in = ld_pair_nt<T>(A.out, e0 + i);
      const Msg<T> out = pass<T>(__builtin_nontemporal_load(A.a + e0 + i), an, in);
      st_pair_nt<T>(A.out, e0 + i, out.P, out.h);
      bad |= !(isfinite(out.P) && isfinite(out.h));
    }
  }
  if (bad) {
    atomicOr(&A.st->error, kErrNonfinite);
    atomicExch(&A.st->done, 1);
  }
}

// RESID: residual of the current means only (every node at the same sweep),
// all workgroups, no update.
template <typename T, int K, bool RESID>
__global__ __launch_bounds__(kBlock) void k_serial(SerialArgs<T> A) {
  constexpr int S = kBlock * K;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[kBlock / 64];
  __shared__ T s_redT[kBlock / 64];
  if (A.st->done) return;
  if ((int)blockIdx.x >= A.nblk) {  // a chunk of a long row
    const ChunkRef x = A.xch[A.xch0 + blockIdx.x - A.nblk];
    serial_chunk<T, K, RESID>(A, A.longs[x.li], x.c, s_red, s_redT);
    return;
  }

  const int tid = threadIdx.x;
  const int b = A.blk0 + xcd_remap_s(blockIdx.x, A.nblk);
  const int r0 = A.blk_row[b], r1 = A.blk_row[b + 1];
  const int e0 = A.blk_e0[b], ne = A.blk_e0[b + 1] - e0;
  const int nrow = r1 - r0;
  const bool check = RESID || A.check;
  double res2 = 0.0;
  bool bad = false;

  // a long row is swept by its chunk workgroups and finished by k_serial_long
  if (ne > S) return;
  {
    T* s_Pn = (T*)smem;
    T* s_hn = s_Pn + S;
    double* s_ax = (double*)(s_hn + S);
    T* s_aP = (T*)(s_ax + S);
    T* s_ah = s_aP + kMaxRowsPerBlock;
    int32_t* s_ptr = (int32_t*)(s_ah + kMaxRowsPerBlock);
    uint8_t* s_row = (uint8_t*)(s_ptr + kMaxRowsPerBlock + 4);
    uint8_t* s_low = s_row + S;

    // 1. independent loads: the slots' streamed data, then the rows'
    int c[K];
    T av[K];
    Msg<T> m[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      c[k] = 0;
      av[k] = 0;
      m[k] = Msg<T>{0, 0};
      if (i < ne) {
        c[k] = __builtin_nontemporal_load(A.col + e0 + i);
        av[k] = __builtin_nontemporal_load(A.a + e0 + i);
        if (!RESID && !A.first) m[k] = ld_pair_nt<T>(A.out, e0 + i);
      }
    }
    const int r = r0 + tid;
    int rp = 0;
    Msg<T> o{1, 0};
    T dr = 0, br = 0;
    double lold = 0.0;
    if (tid < nrow) {
      rp = A.off_ptr[r] - e0;
      if (check) o = ld_pair<T>(A.agg, r);
      dr = A.diag[r];
      br = A.rhs[r];
      if (!RESID && A.check) lold = A.lsum[r];
    }
    // 2. the neighbours' aggregates (the only irregular reads)
    Msg<T> g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      if (i < ne) g[k] = ld_pair<T>(A.agg, c[k]);
    }
    // 3. row structure into LDS
    if (tid < nrow) s_ptr[tid] = rp;
    if (tid == 0) s_ptr[nrow] = ne;
    __syncthreads();
    if (tid < nrow) fill_row_ids(s_row, s_ptr[tid], s_ptr[tid + 1], tid);

    // 4. pulled messages and residual terms
    Msg<T> in[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kBlock;
      in[k] = Msg<T>{0, 0};
      if (i < ne) {
        const bool lower = c[k] < A.lo;
        if (!RESID && (!A.first || lower)) in[k] = pass<T>(av[k], g[k], m[k]);
        double ax = 0.0;
        if (lower ? (!RESID && A.wl) : check) ax = (double)(av[k] * (g[k].h / g[k].P));
        s_Pn[i] = in[k].P;
        s_hn[i] = in[k].h;
        s_ax[i] = ax;
        s_low[i] = lower ? 1 : 0;
        if (!RESID) bad |= !(isfinite(in[k].P) && isfinite(in[k].h));
      }
    }
    __syncthreads();

    // 5. row sums: diagonal first, then the slots in CSR order
    if (tid < nrow) {
      const int lo = s_ptr[tid], hi = s_ptr[tid + 1];
      // the earlier and the later classes' terms, each added in slot order,
      // eight slots loaded ahead
      double L = 0.0, U = 0.0;
      int j = lo;
      for (; j + 8 <= hi; j += 8) {
        double v[8];
        uint8_t w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          v[u] = s_ax[j + u];
          w[u] = s_low[j + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (w[u]) L += v[u];
          else U += v[u];
        }
      }
      for (; j < hi; ++j) {
        if (s_low[j]) L += s_ax[j];
        else U += s_ax[j];
      }
      if (!RESID) {
        T P = lds_row_sum(dr, s_Pn, lo, hi);
        T h = lds_row_sum(br, s_hn, lo, hi);
        st_pair<T>(A.agg, r, P, h);
        if (A.xout) A.xout[r] = h / P;
        if (A.ptout) A.ptout[r] = P;
        if (A.wl) A.lsum[r] = L;
        s_aP[tid] = P;
        s_ah[tid] = h;
      }
      if (check) {
        const double acc = (double)br - (double)dr * (double)(o.h / o.P) - lold - U;
        res2 = acc * acc;
      }
    }

    // 6. the new outgoing messages
    if (!RESID) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = tid + k * kBlock;
        if (i < ne) {
          const int lr = s_row[i];
          const Msg<T> out = pass<T>(av[k], Msg<T>{s_aP[lr], s_ah[lr]}, in[k]);
          st_pair_nt<T>(A.out, e0 + i, out.P, out.h);
          bad |= !(isfinite(out.P) && isfinite(out.h));
        }
      }
    }
  }
  if (bad) {
    atomicOr(&A.st->error, kErrNonfinite);
    atomicExch(&A.st->done, 1);
  }
  if (check) {
    const double bs = bsum_s(res2, s_red);
    if (tid == 0) A.partials[b] = bs;
  }
}

template <typename T>
__global__ void k_serial_prior_x(int32_t n, const T* diag, const T* rhs, T* x, T* pt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    x[i] = rhs[i] / diag[i];
    if (pt) pt[i] = diag[i];
  }
}

__global__ void k_gather(const double* __restrict__ src, const int32_t* __restrict__ idx, double* __restrict__ dst,
                         int32_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[idx[i]];
}

__global__ void k_scatter_slots(const double* __restrict__ src, const int32_t* __restrict__ idx,
                                double* __restrict__ dst, int64_t E) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x)
    dst[idx[i]] = src[i];
}

template <typename T, int K>
hipError_t launch_sk(const SerialArgs<T>& a, bool resid, hipStream_t s) {
  const uint32_t lds = (uint32_t)sr_lds(K, sizeof(T));
  const dim3 grid(a.nblk + a.nxch);
  if (resid) hipLaunchKernelGGL((k_serial<T, K, true>), grid, dim3(kBlock), lds, s, a);
  else hipLaunchKernelGGL((k_serial<T, K, false>), grid, dim3(kBlock), lds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.nxch == 0) return e;
  if (resid) hipLaunchKernelGGL((k_serial_long<T, K, true>), dim3(a.nxch), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_serial_long<T, K, false>), dim3(a.nxch), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace

size_t serial_lds_bytes(int K, int elt) { return sr_lds(K, elt); }

template <typename T>
hipError_t launch_serial(const SerialArgs<T>& a, int K, bool resid, hipStream_t s) {
  if (a.nblk <= 0) return hipSuccess;
  switch (K) {
    case 2: return launch_sk<T, 2>(a, resid, s);
    case 4: return launch_sk<T, 4>(a, resid, s);
    case 8: return launch_sk<T, 8>(a, resid, s);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_serial<double>(const SerialArgs<double>&, int, bool, hipStream_t);
template hipError_t launch_serial<float>(const SerialArgs<float>&, int, bool, hipStream_t);

template <typename T>
hipError_t launch_serial_prior_x(int32_t n, const T* diag, const T* rhs, T* x, T* pt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serial_prior_x<T>, dim3(std::min((n + 255) / 256, 4096)), dim3(256), 0, s, n, diag, rhs, x,
                     pt);
  return hipGetLastError();
}
template hipError_t launch_serial_prior_x<double>(int32_t, const double*, const double*, double*, double*,
                                                  hipStream_t);
template hipError_t launch_serial_prior_x<float>(int32_t, const float*, const float*, float*, float*, hipStream_t);

hipError_t launch_scatter_slots(const double* src, const int32_t* idx, double* dst, int64_t E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_slots, dim3((unsigned)std::min<int64_t>((E + 255) / 256, 8192)), dim3(256), 0, s, src,
                     idx, dst, E);
  return hipGetLastError();
}

hipError_t launch_gather(const double* src, const int32_t* idx, double* dst, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3(std::min((n + 255) / 256, 4096)), dim3(256), 0, s, src, idx, dst, n);
  return hipGetLastError();
}

}  // namespace gabp
