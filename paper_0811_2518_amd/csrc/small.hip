// One-workgroup solve of a small system: every sweep of the synchronous
// iteration of Alg. 2 (Ch. 3 Sec. 3.3), the fused residual checks and the stop
// rule run inside a single launch of 1024 lanes.
//
// A small system (n <= 1024 rows, E <= 4096 directed slots) spends more time
// in kernel launches and host polling than in arithmetic when every sweep is a
// launch of its own.  Here the whole state stays on chip:
//   * lane l owns the slots l, l + 1024, ... of the off-diagonal CSR and keeps
//     the incoming messages of its slots of the last two rounds in registers
//     (the compact recurrence: in^(t) depends on in^(t-2) of the same slot
//     only, so messages are never exchanged between lanes);
//   * the node aggregates {P~, h~} of the last three rounds live in LDS, where
//     the slot lanes gather them;
//   * each round's new messages are staged in LDS and summed per row, in CSR
//     order after the diagonal term, by one lane per row.
// The arithmetic is that of the compact sweep kernel operation for operation
// (products and sums separately rounded), so x, the variances and the messages
// equal those of the multi-launch compact path bit for bit; only the residual
// norm is summed in another order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "gabp_internal.h"

#pragma clang fp contract(off)

namespace gabp {

namespace {

constexpr int kSB = kSmallLanes;  // lanes of the one workgroup

__host__ __device__ constexpr size_t small_lds(int n, int K) {
  // aggregates [3][n] {P, h}; means of the last round [n]; staged P, h and
  // a x terms [S]; residual partials of two sweeps
  return sizeof(double) * (7 * (size_t)n + 3 * (size_t)kSB * K) + sizeof(double) * (2 * kSB / 64);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic sum over the 1024 lanes: wave sums, then the 16 wave sums in
// order, by every lane.  Every lane gets the total.  The caller passes one of
// two buffers by sweep parity, so no barrier is needed before the wave sums are
// stored (a lane cannot be a whole sweep ahead of another); the barrier after
// them also orders everything the lanes did before the call.
__device__ __forceinline__ double small_sum(double v, double* s_red) {
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < kSB / 64; ++w) tot += s_red[w];
  return tot;
}

template <int K>
__global__ __launch_bounds__(kSB) void k_small(SmallArgs A) {
  extern __shared__ __align__(16) double sm[];
  const int tid = threadIdx.x;
  if (A.gate && *A.gate) return;  // the inputs failed validation
  const int n = A.n, E = A.E_dev ? *A.E_dev : A.E;
  if (E < 0 || E > kSB * K || n < 1 || n > kSB) return;  // never run past the lanes' slots
  double* aggP = sm;              // [3][n]
  double* aggH = sm + 3 * n;      // [3][n]
  double* xm = sm + 6 * n;        // [n] means h~ / P~ of the last round, for the next check
  double* sP = sm + 7 * n;        // [S]
  double* sH = sP + kSB * K;      // [S]
  double* sX = sH + kSB * K;      // [S]
  double* s_red = sX + kSB * K;   // [2][16]

  // ---- set-up: the lane's slots and row, the prior as round 0 --------------
  int sc[K], srow[K];
  double sa[K];
  // incoming messages of the even and of the odd rounds (named registers: an
  // array indexed by the round's parity would live in scratch memory)
  double mP0[K], mH0[K], mP1[K], mH1[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int s = tid + k * kSB;
    sc[k] = 0;
    srow[k] = 0;
    sa[k] = 0.0;
    mP0[k] = mH0[k] = mP1[k] = mH1[k] = 0.0;
    if (s < E) {
      sc[k] = A.col[s];
      sa[k] = A.a[s];
    }
  }
  const bool own_row = tid < n;
  int rlo = 0, rhi = 0;
  double dr = 0.0, br = 0.0;
  if (own_row) {
    rlo = A.off_ptr[tid];
    rhi = A.off_ptr[tid + 1];
    dr = A.diag[tid];
    br = A.rhs[tid];
    aggP[tid] = dr;  // round 0: the prior {A_ii, b_i}
    aggH[tid] = br;
    xm[tid] = br / dr;
    // the row of each slot, through the staging area
    for (int s = rlo; s < rhi; ++s) ((int*)sX)[s] = tid;
  }
  // ||b||_2 (the norm kernel's value when given)
  double bnorm;
  if (A.rhs_norm) {
    bnorm = *A.rhs_norm;
  } else {
    bnorm = sqrt(small_sum(own_row ? br * br : 0.0, s_red + kSB / 64));
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int s = tid + k * kSB;
    if (s < E) srow[k] = ((const int*)sX)[s];
  }

  const bool exact = !(A.tol > 0.0);
  const int M = A.max_iter;
  const int ce = max(1, A.check_every);
  auto in_set = [&](int j) { return j == M || (j % ce) == 0; };
  double last_rel = -1.0, prev_rel = -1.0;
  int last_round = -1, prev_round = -1, conv = -1, err = 0;
  int t = 1;
  bool synced = true;  // the set-up ended with a barrier
  // sweeps 1..M update the messages; sweep M+1 only checks round M
  for (; t <= M + 1; ++t) {
    const bool upd = t <= M;
    const bool ck = exact ? (t == M + 1) : in_set(t - 1);
    if (!upd && !ck) break;
    const bool ck_next = upd && (exact ? (t == M) : in_set(t));  // sweep t+1 checks round t
    const int q1 = (t - 1) % 3, q2 = (t + 1) % 3, qn = t % 3;  // rounds t-1, t-2, t
    const bool first = t == 1;
    const bool odd = (t & 1) != 0;
    bool bad = false;
    // 1. slot updates: in^(t) = F(A_i^(t-1), out^(t-1)), out^(t-1) = F(A_j^(t-2), in^(t-2))
    if (!synced) __syncthreads();  // the last row phase's aggregates and means are in place
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int s = tid + k * kSB;
      if (s < E) {
        const int c = sc[k], j = srow[k];
        const double av = sa[k];
        const double gP = aggP[q1 * n + c], gh = aggH[q1 * n + c];
        double ax = 0.0;
        if (ck) ax = av * xm[c];  // x_c of round t-1 = gh / gP, formed once by c's row lane
        if (upd) {
          double Pout = 0.0, hout = 0.0;
          if (!first) {  // in^(t-2): the same parity as round t
            const double o2P = aggP[q2 * n + j], o2h = aggH[q2 * n + j];
            const double inv_out = 1.0 / (o2P - (odd ? mP1[k] : mP0[k]));
            Pout = -av * av * inv_out;
            hout = -av * (o2h - (odd ? mH1[k] : mH0[k])) * inv_out;
          }
          const double inv_in = 1.0 / (gP - Pout);
          const double Pn = -av * av * inv_in;
          const double hn = -av * (gh - hout) * inv_in;
          if (odd) {
            mP1[k] = Pn;
            mH1[k] = hn;
          } else {
            mP0[k] = Pn;
            mH0[k] = hn;
          }
          sP[s] = Pn;
          sH[s] = hn;
          bad |= !(isfinite(Pn) && isfinite(hn));
        }
        sX[s] = ax;
      }
    }
    if (__syncthreads_or(bad ? 1 : 0)) {  // as the multi-launch path: the error ends the solve
      err |= kErrNonfinite;
      ++t;
      break;
    }
    // 2. row sums: round t's aggregates; the residual of round t-1
    double res2 = 0.0;
    if (own_row) {
      double xi = 0.0;
      if (ck) xi = xm[tid];  // read before it is replaced by round t's mean below
      if (upd) {
        const double P = lds_row_sum(dr, sP, rlo, rhi);
        const double h = lds_row_sum(br, sH, rlo, rhi);
        aggP[qn * n + tid] = P;
        aggH[qn * n + tid] = h;
        if (ck_next) xm[tid] = h / P;
      }
      if (ck) {
        double acc = br - dr * xi;
        acc = lds_row_sub(acc, sX, rlo, rhi);
        res2 = acc * acc;
      }
    }
    synced = false;
    if (ck) {
      const double rn = sqrt(small_sum(res2, s_red + (t & 1) * (kSB / 64)));
      synced = true;
      const double rel = bnorm > 0.0 ? rn / bnorm : rn;
      prev_rel = last_rel;
      prev_round = last_round;
      last_rel = rel;
      last_round = t - 1;
      if (rel <= A.tol) conv = t - 1;
      else if (!(rel <= kDivergeLimit)) err |= kErrDiverged;
    }
    if (conv >= 0 || err) {
      ++t;
      break;
    }
  }
  __syncthreads();

  // ---- results: the returned round and the state it leaves -----------------
  const int ret = conv >= 0 ? conv : M;  // round whose means are returned
  if (own_row) {
    const int qr = ret % 3;
    const double P = aggP[qr * n + tid], h = aggH[qr * n + tid];
    if (A.xout[ret & 1]) A.xout[ret & 1][tid] = h / P;
    if (A.ptout[ret & 1]) A.ptout[ret & 1][tid] = P;
    if (A.x_direct) A.x_direct[tid] = h / P;
    if (A.var_direct) A.var_direct[tid] = 1.0 / P;
    for (int q = 0; q < 3; ++q)
      if (A.agg_out[q]) {
        double2 v;
        v.x = aggP[q * n + tid];
        v.y = aggH[q * n + tid];
        ((double2*)A.agg_out[q])[tid] = v;
      }
  }
  if (A.cin_out) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int s = tid + k * kSB;
      if (s < E) {
        double2 v0, v1;
        v0.x = mP0[k];
        v0.y = mH0[k];
        v1.x = mP1[k];
        v1.y = mH1[k];
        ((double2*)A.cin_out)[s] = v0;
        ((double2*)A.cin_out)[(size_t)E + s] = v1;
      }
    }
  }
  if (tid == 0) {
    DevStatus st{};
    st.done = 1;
    st.conv_round = conv;
    st.error = err;
    st.last_rel = last_rel;
    st.last_round = last_round;
    st.prev_rel = prev_rel;
    st.prev_round = prev_round;
    *A.st = st;
  }
}

}  // namespace

// Rows of at most KR slots: lane i owns row i.  The messages of the row's
// slots and the row's own aggregates of the last three rounds stay in
// registers; only the aggregates the neighbours gather live in LDS, two rounds
// by parity.  The lane sums its row as it updates the slots, in CSR order
// after the diagonal (the order of the slot-per-lane kernel above and of the
// multi-launch path), so the results are the same bit for bit.  A sweep needs
// one barrier: the lanes publish round t and their residual partials, then
// wait for each other, and only then read round t or overwrite round t-1.
// Workgroup barrier ordering LDS only (the sweeps touch no global memory).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A value every lane of the workgroup holds alike, kept in scalar registers
// (the lane-per-row kernel runs at the VGPR limit of a 1024-lane workgroup).
__device__ __forceinline__ double uni_d(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int KR>
__global__ __launch_bounds__(kSB) void k_small_rows(SmallArgs A) {
  extern __shared__ __align__(16) double sm[];
  // non-finite message flags by sweep mod 3: sweep t sets [t % 3] and clears
  // [(t + 1) % 3], which no lane reads or sets until sweep t + 1
  __shared__ int s_bad[3];
  const int tid = threadIdx.x;
  if (A.gate && *A.gate) return;
  const int n = A.n;
  if (n < 1 || n > kSB) return;
  double* gP = sm;               // [2][n] P~ by round parity
  double* gH = sm + 2 * n;       // [2][n] h~ by round parity
  double* gX = sm + 4 * n;       // [2][n] means h~ / P~ by round parity, for the next check
  double* s_red = sm + 6 * n;    // [2][16] residual partials by sweep parity
  const bool own = tid < n;
  int rlo = 0, deg = 0;
  double dr = 1.0, br = 0.0;
  if (own) {
    rlo = A.off_ptr[tid];
    deg = A.off_ptr[tid + 1] - rlo;
    dr = A.diag[tid];
    br = A.rhs[tid];
  }
  if (deg > KR) deg = KR;  // the host sends only rows of at most KR slots
  int cc[KR];
  double aa[KR], mP0[KR], mH0[KR], mP1[KR], mH1[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    cc[k] = 0;
    aa[k] = 0.0;
    mP0[k] = mH0[k] = mP1[k] = mH1[k] = 0.0;
    if (k < deg) {
      cc[k] = A.col[rlo + k];
      aa[k] = A.a[rlo + k];
    }
  }
  // own aggregates of rounds t-1, t-2, t-3 (round 0: the prior {A_ii, b_i})
  double o1P = dr, o1h = br, o2P = 0.0, o2h = 0.0, o3P = 0.0, o3h = 0.0;
  if (own) {
    gP[tid] = dr;
    gH[tid] = br;
    gX[tid] = br / dr;
  }
  if (tid < 3) s_bad[tid] = 0;
  double bnorm;
  if (A.rhs_norm) {
    bnorm = *A.rhs_norm;
  } else {
    bnorm = sqrt(small_sum(own ? br * br : 0.0, s_red + kSB / 64));
  }
  bnorm = uni_d(bnorm);
  __syncthreads();

  const bool exact = !(A.tol > 0.0);
  const int M = A.max_iter;
  const int ce = max(1, A.check_every);
  auto in_set = [&](int j) { return j == M || (j % ce) == 0; };
  // relative residual of a checked round from its sum of squares, formed as
  // the multi-launch finish forms it
  auto rel_of = [&](double tot) {
    const double rn = sqrt(tot);
    return bnorm > 0.0 ? rn / bnorm : rn;
  };
  // the stop test needs that relative residual only near a threshold: a sum
  // of squares clearly above (tol |b|)^2 cannot pass, one clearly below
  // (1e8 |b|)^2 cannot diverge (margins far above the rounding of sqrt and
  // the division); the decisions are the exact ones
  const double scale = bnorm > 0.0 ? bnorm : 1.0;
  double conv_pre = A.tol >= 0.0 ? (A.tol * scale) * (A.tol * scale) * (1.0 + 1e-6) : -1.0;
  if (A.tol > 0.0 && !(conv_pre > 1e-280 && conv_pre < 1e280)) conv_pre = INFINITY;  // out of range: always exact
  conv_pre = uni_d(conv_pre);
  const double div_pre = uni_d((kDivergeLimit * scale) * (kDivergeLimit * scale) * (1.0 - 1e-6));
  double last_tot = 0.0, prev_tot = 0.0;
  int last_round = -1, prev_round = -1, conv = -1, err = 0;
  int T = 0;  // the last round whose aggregates were formed
  // One sweep.  Rows of at most 4 slots take the parity of t as a
  // compile-time constant (std::true_type / std::false_type), so the message
  // registers of the two parities need no selects or moves; rows of up to 6
  // slots take it at run time, which keeps the code within the register
  // budget.  Returns true when the solve ends.
  auto sweep = [&](auto odd_c, const int t) -> bool {
    const bool ODD = odd_c;
    if (t > M + 1) return true;  // sweeps 1..M, then the check of round M
    const bool upd = t <= M;
    const bool ck = exact ? (t == M + 1) : in_set(t - 1);
    if (!upd && !ck) return true;
    const bool ck_next = upd && (exact ? (t == M) : in_set(t));  // sweep t+1 checks round t
    const int p1 = ODD ? 0 : 1, pn = ODD ? 1 : 0;  // parities of rounds t-1 (read) and t (written)
    const bool first = ODD && t == 1;
    bool bad = false;
    double P = dr, h = br, acc = 0.0;
    if (ck) acc = br - dr * gX[p1 * n + tid];  // the row's residual in round t-1
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      if (k < deg) {
        const int c = cc[k];
        const double av = aa[k];
        const double gPc = gP[p1 * n + c], gHc = gH[p1 * n + c];
        if (ck) acc -= av * gX[p1 * n + c];  // x_c = h~_c / P~_c, formed once by c's lane
        if (upd) {
          // in^(t) = F(A_c^(t-1), out^(t-1)), out^(t-1) = F(A_own^(t-2), in^(t-2))
          double Pout = 0.0, hout = 0.0;
          if (!first) {  // in^(t-2) has the parity of t
            const double inv_out = 1.0 / (o2P - (ODD ? mP1[k] : mP0[k]));
            Pout = -av * av * inv_out;
            hout = -av * (o2h - (ODD ? mH1[k] : mH0[k])) * inv_out;
          }
          const double inv_in = 1.0 / (gPc - Pout);
          const double Pn = -av * av * inv_in;
          const double hn = -av * (gHc - hout) * inv_in;
          if (ODD) {
            mP1[k] = Pn;
            mH1[k] = hn;
          } else {
            mP0[k] = Pn;
            mH0[k] = hn;
          }
          P += Pn;
          h += hn;
          bad |= !(isfinite(Pn) && isfinite(hn));
        }
      }
    }
    if (upd && own) {
      gP[pn * n + tid] = P;
      gH[pn * n + tid] = h;
      if (ck_next) gX[pn * n + tid] = h / P;
    }
    double* red = s_red + pn * (kSB / 64);
    if (ck) {
      const double v = wsum(own ? acc * acc : 0.0);
      if ((tid & 63) == 0) red[tid >> 6] = v;
    }
    if (tid == 0) s_bad[(t + 1) % 3] = 0;
    if (bad) s_bad[t % 3] = 1;
    lds_barrier();
    const bool any_bad = s_bad[t % 3] != 0;
    if (upd) {
      o3P = o2P;
      o3h = o2h;
      o2P = o1P;
      o2h = o1h;
      o1P = P;
      o1h = h;
      T = t;
    }
    if (any_bad) {  // as the multi-launch path: the error ends the solve
      err |= kErrNonfinite;
      return true;
    }
    if (ck) {
      double tot = 0.0;
      for (int w = 0; w < kSB / 64; ++w) tot += red[w];
      tot = uni_d(tot);
      prev_tot = last_tot;
      prev_round = last_round;
      last_tot = tot;
      last_round = t - 1;
      if (tot <= conv_pre && rel_of(tot) <= A.tol) conv = t - 1;
      else if (!(tot < div_pre) && !(rel_of(tot) <= kDivergeLimit)) err |= kErrDiverged;
    }
    return conv >= 0 || err != 0;
  };
  if constexpr (KR <= 4) {
    for (int t = 1;; t += 2) {
      if (sweep(std::true_type{}, t)) break;
      if (sweep(std::false_type{}, t + 1)) break;
    }
  } else {
    for (int t = 1;; ++t)
      if (sweep((t & 1) != 0, t)) break;
  }
  const double last_rel = last_round >= 0 ? rel_of(last_tot) : -1.0;
  const double prev_rel = prev_round >= 0 ? rel_of(prev_tot) : -1.0;

  // ---- results: the returned round and the state it leaves -----------------
  const int ret = conv >= 0 ? conv : M;
  double rP = o1P, rh = o1h;
  if (ret == T - 1) {
    rP = o2P;
    rh = o2h;
  } else if (ret == T - 2) {
    rP = o3P;
    rh = o3h;
  }
  if (own) {
    if (A.xout[ret & 1]) A.xout[ret & 1][tid] = rh / rP;
    if (A.ptout[ret & 1]) A.ptout[ret & 1][tid] = rP;
    if (A.x_direct) A.x_direct[tid] = rh / rP;
    if (A.var_direct) A.var_direct[tid] = 1.0 / rP;
    // the aggregates of rounds T, T-1 and T-2 by round mod 3
    const double P3[3] = {o1P, o2P, o3P}, H3[3] = {o1h, o2h, o3h};
    for (int j = 0; j < 3 && j <= T; ++j) {
      void* dst = A.agg_out[(T - j) % 3];
      if (dst) {
        double2 v;
        v.x = P3[j];
        v.y = H3[j];
        ((double2*)dst)[tid] = v;
      }
    }
  }
  if (A.cin_out && own) {
    const int E = A.E;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      if (k < deg) {
        double2 v0, v1;
        v0.x = mP0[k];
        v0.y = mH0[k];
        v1.x = mP1[k];
        v1.y = mH1[k];
        ((double2*)A.cin_out)[rlo + k] = v0;
        ((double2*)A.cin_out)[(size_t)E + rlo + k] = v1;
      }
    }
  }
  if (tid == 0) {
    DevStatus st{};
    st.done = 1;
    st.conv_round = conv;
    st.error = err;
    st.last_rel = last_rel;
    st.last_round = last_round;
    st.prev_rel = prev_rel;
    st.prev_round = prev_round;
    *A.st = st;
  }
}

size_t small_lds_bytes(int n, int K) { return small_lds(n, K); }

bool small_fits(int64_t n, int64_t E) { return n >= 1 && n <= kSmallLanes && E <= (int64_t)kSmallLanes * 4; }

bool small_rows_fit(int64_t n, int32_t max_deg) { return n >= 1 && n <= kSmallLanes && max_deg >= 1 && max_deg <= 6; }

hipError_t launch_small(const SmallArgs& a, hipStream_t s) {
  if (a.E_dev == nullptr && small_rows_fit(a.n, a.max_deg)) {  // a lane per row
    const uint32_t lds = (uint32_t)(sizeof(double) * (6 * (size_t)a.n + 2 * kSB / 64));
    if (a.max_deg <= 4) hipLaunchKernelGGL(k_small_rows<4>, dim3(1), dim3(kSB), lds, s, a);
    else hipLaunchKernelGGL(k_small_rows<6>, dim3(1), dim3(kSB), lds, s, a);
    return hipGetLastError();
  }
  if (!small_fits(a.n, a.E)) return hipErrorInvalidValue;
  const int K = a.E <= kSB ? 1 : (a.E <= 2 * kSB ? 2 : 4);
  const uint32_t lds = (uint32_t)small_lds(a.n, K);
  switch (K) {
    case 1:
      (void)hipFuncSetAttribute((const void*)k_small<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(k_small<1>, dim3(1), dim3(kSB), lds, s, a);
      break;
    case 2:
      (void)hipFuncSetAttribute((const void*)k_small<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(k_small<2>, dim3(1), dim3(kSB), lds, s, a);
      break;
    default:
      (void)hipFuncSetAttribute((const void*)k_small<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(k_small<4>, dim3(1), dim3(kSB), lds, s, a);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_small_k4(const SmallArgs& a, hipStream_t s) {
  if (a.n < 1 || a.n > kSB) return hipErrorInvalidValue;
  const uint32_t lds = (uint32_t)small_lds(a.n, 4);
  (void)hipFuncSetAttribute((const void*)k_small<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_small<4>, dim3(1), dim3(kSB), lds, s, a);
  return hipGetLastError();
}

}  // namespace gabp
