// Batched solves: many independent systems, several right-hand sides each, in
// one HIP graph of two persistent kernels.
//
//  1. k_bprec -- the precision phase, once per system: synchronous P-only
//     sweeps of Alg. 2 (the precision update has no b term, so the precisions
//     are shared by every right-hand side of the system) until the node
//     precisions P~_i settle, then the frozen h-update coefficients
//     g_in = -A_ij / (P~_i - P_ji), g_out and 1 / P~_i of the system.
//  2. k_brhs -- FP64 iterative refinement of every (system, group of 1, 2, 4
//     or 8 right-hand sides): r = b - A x in FP64; the correction A d = r by
//     h-only FP32 sweeps with the system's frozen coefficients on all
//     right-hand sides of the group at once; x += d; until every right-hand
//     side of the group reaches the relative residual tolerance.
// Work items are handed out costliest first through atomic queues; one
// 512-lane workgroup runs an item from start to finish, so every barrier is a
// workgroup barrier and no workgroup waits for another.  The second kernel
// starts when the first has finished (graph order), so the frozen
// coefficients are complete and visible.
//
// Layout.  At create, each system's rows are renumbered: inside each segment
// (the whole system; with the colour-serial schedule, each colour class) the
// rows are sorted by decreasing degree within windows of 512, and every 64
// consecutive rows form a slice.  A slice stores its slots column-major
// (SELL-64): the q-th slot of each of its rows lies at base + 64 q + row, so
// the lanes of a wave that take one row each read slot q of 64 rows in one
// coalesced access, and a row's slots are visited in their CSR order.  A
// wave takes a slice (one right-hand side per lane) or a part of it (kg
// right-hand sides: 64 / kg rows, kg lanes per row, whose h messages and
// aggregates are stored [slot][rhs] and [node][rhs], so a neighbour gather
// reads kg contiguous words).  Each lane sums its own row in registers: no
// LDS staging, no barrier inside a sweep.  Messages follow the compact
// one-message-per-slot recursion of the single-system path:
//     out^(t-1) = F(A_j^(t-2), in^(t-2)),   in^(t) = F(A_i^(t-1), out^(t-1)),
// the node aggregates rotating through three buffers (round mod 3).  The
// colour-serial schedule instead updates one colour class at a time, in
// place, with a workgroup barrier between classes (serial scheduling, Ch. 2
// Sec. 2.3).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "gabp_internal.h"

namespace gabp {

namespace {

constexpr int kBT = 512;                // lanes per batched workgroup
constexpr int kWave = 64;
constexpr int kWaves = kBT / kWave;
constexpr int kSlice = 64;              // rows per slice
constexpr int kSortWindow = 512;        // rows sorted by degree together
constexpr int kQSlots = 4;              // slots of a row loaded together (FP32 passes)
constexpr int kMaxGroup = 8;            // right-hand sides per work item (1, 2, 4 or 8)
constexpr float kPrecTol = 4e-7f;       // precision phase: relative change of P~ to stop at
constexpr float kPrecStall = 2e-5f;     // ... or below this, once it stops halving (FP32 rounding floor)
constexpr int kPrecStallSweeps = 8;

enum PassKind : int {
  kKP = 0,       // precision-only message sweep
  kKFreeze = 1,  // frozen h-update coefficients from the precisions of a round
  kKH = 2,       // h-only message sweep, all right-hand sides of the item
  kKSpmv = 3     // FP64 residual r = b - A x
};

struct Slice {
  int64_t base;    // first SELL slot (global)
  int32_t row0;    // first row (system-local internal numbering)
  int32_t nrows;   // rows (<= 64)
  int32_t L;       // slots per row stored (the largest degree of its rows)
  int32_t pad;
};

struct SysRec {
  int32_t r0, n;      // global rows r0 .. r0 + n - 1 (the same range in the caller's and the internal numbering)
  int32_t sl0, nsl;   // slices
  int64_t ss0, S;     // SELL slots
  int64_t off_ps;     // precision scratch: P [2][S], coef [S] (slot units)
  int64_t off_pn;     // Pagg [3][n], invPt [n] (node units)
  int32_t cls0, ncls; // colour-serial: the system's class slice starts cls_sl[cls0 .. cls0 + ncls]
};

struct BItem {
  int32_t sys, j0, kg, k;  // right-hand sides j0 .. j0 + kg - 1 of the system's k
  int64_t off_h;           // h messages [2][S kg] (float units)
  int64_t off_nk;          // h~ [3][n kg] and the correction's right-hand side [n kg] (float units)
  int64_t off_x;           // x [n kg] in internal row order (double units)
  int64_t rhs_off;         // B / X offset of the system
};

struct ItemInfo {
  int32_t sweeps, outer, converged, status;
  double rel;
  int32_t psweeps, pad;
  uint64_t t0, t1;  // device wall clock at the item's start and end
};

struct BatchArgs {
  const SysRec* sys;
  const Slice* slices;
  const int32_t* cls_sl;
  const int32_t* deg;     // [N] degree of each internal row
  const float* d32;       // [N]
  const double* d64;      // [N]
  const int32_t* umap;    // [N] internal row -> caller row (global)
  const int32_t* col;     // [Stot] system-local internal column
  const float* a32;       // [Stot]
  const double* a64;      // [Stot]
  // precision phase
  const int32_t* porder;  // systems, costliest first
  int32_t num_sys;
  float* pP;
  float2* pcoef;
  float* pagg;
  float* pinv;
  ItemInfo* pinfos;       // [num_sys]
  // right-hand-side phase
  const BItem* items;
  int32_t num_items;
  ItemInfo* infos;
  float* hbuf;
  float* nkbuf;
  double* xbuf;
  uint32_t* queue;        // [2]: precision, right-hand sides
  const double* B;
  double* X;
  double tol;
  float inner_tol;
  int32_t inner_max;
  int32_t max_outer;
  int32_t max_iter;
};

__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Reciprocal for the FP32 inner passes (about 1 ulp; the FP64 outer loop
// corrects whatever the inner solves leave).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// The uniform view of a system and, in the second phase, of a work item.
struct View {
  int r0, n, sl0, nsl;
  int64_t ss0, S;
  float* P0;       // [2][S] precisions by round parity (colour-serial: [S] outgoing, in place)
  float2* coef;    // [S]
  float* Pagg0;    // [3][n] P~ by round mod 3 (colour-serial: [n] in place)
  float* invPt;    // [n]
  int kg, lgk, k, j0;
  float* H0;       // [2][S kg] (colour-serial: [S kg] outgoing, in place)
  float* hagg0;    // [3][n kg] (colour-serial: [n kg] in place)
  float* r32;      // [n kg]
  double* xint;    // [n kg]
  const double* B;  // the system's [n][k] block, caller row order
  double* X;
  __device__ float* P(int t) const { return P0 + (t & 1) * S; }
  __device__ float* Pagg(int t) const { return Pagg0 + (t % 3) * (int64_t)n; }
  __device__ float* H(int t) const { return H0 + (t & 1) * S * kg; }
  __device__ float* hagg(int t) const { return hagg0 + (t % 3) * (int64_t)n * kg; }
};

__device__ View sys_view(const BatchArgs& A, int s) {
  const SysRec R = A.sys[s];
  View V{};
  V.r0 = uni(R.r0);
  V.n = uni(R.n);
  V.sl0 = uni(R.sl0);
  V.nsl = uni(R.nsl);
  V.ss0 = uni(R.ss0);
  V.S = uni(R.S);
  const int64_t ops = uni(R.off_ps), opn = uni(R.off_pn);
  V.P0 = A.pP + 2 * ops;
  V.coef = A.pcoef + ops;
  V.Pagg0 = A.pagg + 3 * opn;
  V.invPt = A.pinv + opn;
  V.kg = 1;
  V.lgk = 0;
  return V;
}

// Per-lane results of a pass.
struct Red {
  float dmax, xmax;  // h pass: change of d and size of d; P pass: relative change of P~
  double r2;         // residual pass: sum of squares
  int bad;           // a non-finite frozen coefficient
};

// One pass of the given kind over the slices [slo, shi) of a system.  rhi is
// the end of the rows being updated (colour-serial: of the current class, so
// that a neighbour at or beyond it belongs to a later class).  Each wave walks
// its own units (slice, part of the right-hand sides); the caller
// synchronises the workgroup after the pass.
template <int KIND, bool SER>
__device__ void pass(const BatchArgs& A, const View& V, int t, int slo, int shi, int rhi, Red& rd) {
  constexpr bool MULTI = KIND == kKH || KIND == kKSpmv;
  constexpr int kQ = KIND == kKSpmv ? 4 : kQSlots;  // FP64 slots hold twice the registers
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uni((int32_t)(threadIdx.x / kWave));
  const int lgk = MULTI ? V.lgk : 0;
  const int kgE = 1 << lgk;
  const int R = kWave >> lgk;  // rows per unit
  const int lr = lane >> lgk, jj = lane & (kgE - 1);
  const int kg = V.kg;
  const bool first = t == 1, second = t == 2;
  const int units = (shi - slo) << lgk;
  const int32_t* colp = A.col + V.ss0;
  const float* a32p = A.a32 + V.ss0;
  const double* a64p = A.a64 + V.ss0;
  const int32_t* degp = A.deg + V.r0;
  const float* d32p = A.d32 + V.r0;
  const double* d64p = A.d64 + V.r0;
  // the buffers of this round
  float* Pt_ = SER ? V.P0 : V.P(t);
  const float* Pold_ = V.P(t + 1);                                             // freeze: in^(T-1)
  const float* Pg_ = SER ? V.Pagg0 : V.Pagg(KIND == kKFreeze ? t : t + 2);    // gathered P~ (round t-1; freeze T)
  float* Pn_ = SER ? V.Pagg0 : V.Pagg(t);
  float* Ht_ = SER ? V.H0 : V.H(t);
  const float* hg_ = SER ? V.hagg0 : V.hagg(t + 2);
  float* hn_ = SER ? V.hagg0 : V.hagg(t);
  for (int u = wave; u < units; u += kWaves) {
    const Slice sl = A.slices[slo + (u >> lgk)];
    const int64_t base = uni(sl.base) - V.ss0;
    const int row0 = uni(sl.row0), nrows = uni(sl.nrows), L = uni(sl.L);
    const int lrow = (u & (kgE - 1)) * R + lr;
    const bool valid = lrow < nrows;
    const int i = row0 + lrow;  // the lane's row
    const int deg = valid ? degp[i] : 0;
    // system-local slot q of the row: sbase + 64 q (a system's slots and
    // [slot][rhs] words fit 32-bit offsets from the uniform bases)
    const int sbase = (int)base + lrow;
    const int qi = i * kg + jj;
    // own values
    float er = 0.f, ip = 0.f, o1 = 0.f, o2 = 0.f;
    double xo = 0.0, bo = 0.0;
    if (valid) {
      if (KIND == kKP) {
        if (SER) {
          o1 = first ? d32p[i] : V.Pagg0[i];
        } else {
          o1 = first ? d32p[i] : V.Pagg(t + 2)[i];                         // round t-1
          o2 = second ? d32p[i] : (first ? 0.f : V.Pagg(t + 1)[i]);         // round t-2
        }
      } else if (KIND == kKFreeze) {
        if (SER) {
          o1 = V.Pagg0[i];
        } else {
          o1 = V.Pagg(t)[i];                                                // round T
          o2 = t >= 2 ? V.Pagg(t + 2)[i] : d32p[i];                         // round T-1
        }
      } else if (KIND == kKH) {
        er = V.r32[qi];
        ip = V.invPt[i];
        if (SER) {
          o1 = first ? 0.f : V.hagg0[qi];
        } else {
          o1 = first ? er : V.hagg(t + 2)[qi];
          o2 = second ? er : (first ? 0.f : V.hagg(t + 1)[qi]);
        }
      } else {
        xo = V.xint[qi];
        bo = V.B[(int64_t)(A.umap[V.r0 + i] - V.r0) * V.k + V.j0 + jj];
      }
    }
    float accf = 0.f;
    double accd = 0.0;
    for (int q0 = 0; q0 < L; q0 += kQ) {
      int c[kQ];
      float va[kQ], vm[kQ], vg[kQ], vx[kQ];
      float2 vc[kQ];
      double vad[kQ], vxd[kQ];
      // streamed loads of up to kQ slots, then the neighbour gathers
#pragma unroll
      for (int u8 = 0; u8 < kQ; ++u8) {
        const int q = q0 + u8;
        c[u8] = i;
        va[u8] = vm[u8] = vx[u8] = 0.f;
        vc[u8] = float2{0.f, 0.f};
        vad[u8] = 0.0;
        if (q < deg) {
          const int s = sbase + q * kSlice;
          c[u8] = colp[s];
          if (KIND == kKP || KIND == kKFreeze) {
            va[u8] = a32p[s];
            if (SER) {
              if (!first || KIND == kKFreeze) vm[u8] = Pt_[s];           // out_{j->i} of j's last update
            } else if (KIND == kKP) {
              if (!first && !second) vm[u8] = Pt_[s];                      // in^(t-2)
            } else {
              vm[u8] = Pt_[s];                                             // in^(T)
              if (t >= 2) vx[u8] = Pold_[s];                               // in^(T-1)
            }
          } else if (KIND == kKH) {
            vc[u8] = V.coef[s];
            if (SER) vm[u8] = first ? 0.f : Ht_[s * kg + jj];              // h_out of j's last update
            else vm[u8] = (!first && !second) ? Ht_[s * kg + jj] : 0.f;    // h_in^(t-2)
          } else {
            vad[u8] = a64p[s];
          }
        }
      }
#pragma unroll
      for (int u8 = 0; u8 < kQ; ++u8) {
        const int q = q0 + u8;
        vg[u8] = 0.f;
        vxd[u8] = 0.0;
        if (q < deg) {
          const int cn = c[u8];
          const bool silent = SER && first && cn >= rhi;  // a later class has sent nothing yet
          if (KIND == kKP || KIND == kKFreeze) vg[u8] = silent ? 0.f : ((first && !SER && KIND == kKP) ? d32p[cn] : Pg_[cn]);
          else if (KIND == kKH) vg[u8] = silent ? 0.f : ((first && !SER) ? V.r32 : hg_)[cn * kg + jj];
          else vxd[u8] = V.xint[cn * kg + jj];
        }
      }
      // the slot arithmetic, in the row's slot order
#pragma unroll
      for (int u8 = 0; u8 < kQ; ++u8) {
        const int q = q0 + u8;
        if (q < deg) {
          const int s = sbase + q * kSlice;
          const bool silent = SER && first && c[u8] >= rhi;
          if (KIND == kKP) {
            const float av2 = -va[u8] * va[u8];
            float Pin;
            if (SER) {
              Pin = silent ? 0.f : av2 * rcp(vg[u8] - vm[u8]);  // pulled in_{i->j} = F(P~_i, out_{j->i})
            } else {
              float Pout = 0.f;
              if (!first) Pout = av2 * rcp(o2 - vm[u8]);        // out^(t-1)
              Pin = av2 * rcp(vg[u8] - Pout);                    // in^(t)
            }
            Pt_[s] = Pin;  // colour-serial: kept in the slot until the row's new aggregate is known
            accf += Pin;
          } else if (KIND == kKFreeze) {
            const float av = va[u8];
            float2 cf;
            if (SER) {
              const float r_in = rcp(vg[u8] - vm[u8]);
              const float Pin = -av * av * r_in;
              cf.x = -av * r_in;                    // g_in  = -a / (P~_i - P_{j->i})
              cf.y = -av * rcp(o1 - Pin);           // g_out = -a / (P~_j - P_{i->j})
            } else {
              const float Pout = -av * av * rcp(o2 - vx[u8]);  // out^(T) = F(A_j^(T-1), in^(T-1))
              cf.x = -av * rcp(vg[u8] - Pout);
              cf.y = -av * rcp(o1 - vm[u8]);
            }
            V.coef[s] = cf;
            if (!(isfinite(cf.x) && isfinite(cf.y))) rd.bad = 1;
          } else if (KIND == kKH) {
            float hin;
            if (SER) {
              hin = silent ? 0.f : vc[u8].x * (vg[u8] - vm[u8]);
            } else {
              float hout = 0.f;
              if (!first) hout = vc[u8].y * (o2 - vm[u8]);      // h_out^(t-1)
              hin = vc[u8].x * (vg[u8] - hout);                  // h_in^(t)
            }
            Ht_[s * kg + jj] = hin;
            accf += hin;
          } else {
            accd += vad[u8] * vxd[u8];
          }
        }
      }
    }
    if (!valid) continue;
    // row epilogue
    if (KIND == kKP) {
      const float Pt = d32p[i] + accf;
      Pn_[i] = Pt;
      rd.dmax = fmaxf(rd.dmax, fabsf(Pt - o1) / fabsf(Pt));
      if (SER)  // the new outgoing messages out_{j->i} = F(P~_j, in_{i->j})
        for (int q = 0; q < deg; ++q) {
          const int s = sbase + q * kSlice;
          const float av = a32p[s];
          Pt_[s] = -av * av * rcp(Pt - Pt_[s]);
        }
    } else if (KIND == kKFreeze) {
      const float ipt = rcp(o1);
      V.invPt[i] = ipt;
      if (!isfinite(ipt)) rd.bad = 1;
    } else if (KIND == kKH) {
      const float ht = er + accf;
      hn_[qi] = ht;
      const float dn = ht * ip;
      const float dold = first ? 0.f : o1 * ip;
      rd.dmax = fmaxf(rd.dmax, fabsf(dn - dold));
      rd.xmax = fmaxf(rd.xmax, fabsf(dn));
      if (SER)
        for (int q = 0; q < deg; ++q) {
          const int s = sbase + q * kSlice;
          const float gout = V.coef[s].y;
          Ht_[s * kg + jj] = gout * (ht - Ht_[s * kg + jj]);
        }
    } else {
      const double r = bo - d64p[i] * xo - accd;
      V.r32[qi] = (float)r;
      rd.r2 += r * r;
    }
  }
}

// Nonnegative floats order like their bit patterns; NaN maps above +inf.
__device__ __forceinline__ unsigned fkey(float v) { return isnan(v) ? 0x7f800001u : __float_as_uint(v); }

// Per right-hand-side reductions over the workgroup: lanes with the same
// right-hand side (lane mod kg) are combined in a fixed tree, then the waves
// in order, so sums are reproducible.
struct Shared {
  unsigned mx[kWaves][2 * kMaxGroup];
  double sm[kWaves][kMaxGroup];
  double tot[kMaxGroup];
  double bn[kMaxGroup];
  unsigned fmx[2 * kMaxGroup];
  int item;
  int bad;
};

__device__ void reduce_max2(Shared& sh, float a, float b, int kg) {
  unsigned ka = fkey(a), kb = fkey(b);
  for (int off = kWave / 2; off >= kg; off >>= 1) {
    ka = max(ka, (unsigned)__shfl_xor((int)ka, off, kWave));
    kb = max(kb, (unsigned)__shfl_xor((int)kb, off, kWave));
  }
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane < kg) {
    sh.mx[w][lane] = ka;
    sh.mx[w][kMaxGroup + lane] = kb;
  }
  __syncthreads();
  if ((int)threadIdx.x < kg) {
    unsigned ra = 0u, rb = 0u;
    for (int v = 0; v < kWaves; ++v) {
      ra = max(ra, sh.mx[v][threadIdx.x]);
      rb = max(rb, sh.mx[v][kMaxGroup + threadIdx.x]);
    }
    sh.fmx[threadIdx.x] = ra;
    sh.fmx[kMaxGroup + threadIdx.x] = rb;
  }
  __syncthreads();
}

__device__ void reduce_sum(Shared& sh, double v, int kg) {
  for (int off = kWave / 2; off >= kg; off >>= 1) v += __shfl_xor(v, off, kWave);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane < kg) sh.sm[w][lane] = v;
  __syncthreads();
  if ((int)threadIdx.x < kg) {
    double acc = 0.0;
    for (int q = 0; q < kWaves; ++q) acc += sh.sm[q][threadIdx.x];
    sh.tot[threadIdx.x] = acc;
  }
  __syncthreads();
}

// The class slice range and row end of class q of a colour-serial system.
__device__ __forceinline__ void class_range(const BatchArgs& A, int cls0, int q, const View& V, int& slo, int& shi,
                                            int& rhi) {
  slo = uni(A.cls_sl[cls0 + q]);
  shi = uni(A.cls_sl[cls0 + q + 1]);
  rhi = shi >= V.sl0 + V.nsl ? V.n : uni(A.slices[shi].row0);
}

// ---- phase 1: the precision phase of one system -----------------------------
template <bool SER>
__device__ void precision_item(const BatchArgs& A, int s, Shared& sh) {
  const View V = sys_view(A, s);
  const SysRec R = A.sys[s];
  const int cls0 = uni(R.cls0), ncls = uni(R.ncls);
  const uint64_t t_start = wall_clock64();
  // P-only sweeps until P~ settles.  The FP32 change of P~ settles at a
  // rounding floor that can lie above kPrecTol on weakly dominant systems;
  // the phase also ends once the change is small and has stopped halving
  // (the FP64 refinement absorbs the rest).
  int tp = 1;
  float best = INFINITY;
  int tbest = 0;
  for (;; ++tp) {
    Red rd{0.f, 0.f, 0.0, 0};
    if (SER) {
      for (int q = 0; q < ncls; ++q) {
        int slo, shi, rhi;
        class_range(A, cls0, q, V, slo, shi, rhi);
        pass<kKP, true>(A, V, tp, slo, shi, rhi, rd);
        __syncthreads();
      }
    } else {
      pass<kKP, false>(A, V, tp, V.sl0, V.sl0 + V.nsl, V.n, rd);
    }
    reduce_max2(sh, rd.dmax, 0.f, 1);  // also orders this round's aggregates before the next pass
    const float ch = __uint_as_float(sh.fmx[0]);
    if (ch < 0.5f * best) {
      best = ch;
      tbest = tp;
    }
    if (tp >= 3 && ch <= kPrecTol) break;
    if (tp - tbest >= kPrecStallSweeps && best <= kPrecStall) break;
    if (tp >= A.inner_max || !(ch <= 1e30f)) break;
  }
  // freeze the h-update coefficients from the precisions of round tp
  Red rd{0.f, 0.f, 0.0, 0};
  pass<kKFreeze, SER>(A, V, tp, V.sl0, V.sl0 + V.nsl, V.n, rd);
  if (threadIdx.x == 0) sh.bad = 0;
  __syncthreads();
  if (rd.bad) sh.bad = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    ItemInfo inf{};
    inf.psweeps = tp;
    inf.status = sh.bad ? GABP_E_NONFINITE : GABP_OK;
    inf.t0 = t_start;
    inf.t1 = wall_clock64();
    A.pinfos[s] = inf;
  }
  __syncthreads();
}

// ---- phase 2: FP64 refinement of one item ----------------------------------
template <bool SER>
__device__ void rhs_item(const BatchArgs& A, const BItem& I, int it, Shared& sh) {
  const int tid = threadIdx.x;
  View V = sys_view(A, I.sys);
  const SysRec R = A.sys[I.sys];
  const int cls0 = uni(R.cls0), ncls = uni(R.ncls);
  V.kg = I.kg;
  V.lgk = I.kg == 8 ? 3 : (I.kg == 4 ? 2 : (I.kg == 2 ? 1 : 0));
  V.k = I.k;
  V.j0 = I.j0;
  V.H0 = A.hbuf + I.off_h;
  const int64_t nk = (int64_t)V.n * V.kg;
  V.hagg0 = A.nkbuf + I.off_nk;
  V.r32 = V.hagg0 + 3 * nk;
  V.xint = A.xbuf + I.off_x;
  V.B = A.B + I.rhs_off;
  V.X = A.X + I.rhs_off;
  const int kg = V.kg;
  const int jj = tid & (kg - 1);
  const uint64_t t_start = wall_clock64();
  const int pstatus = A.pinfos[I.sys].status;

  // x = 0, the correction's right-hand side r = b, and ||b|| per right-hand side
  double bpart = 0.0;
  for (int64_t q = tid; q < nk; q += kBT) {
    const int i = (int)(q >> V.lgk);
    const double bv = V.B[(int64_t)(A.umap[V.r0 + i] - V.r0) * V.k + V.j0 + jj];
    V.xint[q] = 0.0;
    V.r32[q] = (float)bv;
    bpart += bv * bv;
  }
  reduce_sum(sh, bpart, kg);
  if (tid < kg) sh.bn[tid] = sqrt(sh.tot[tid]);
  __syncthreads();

  int status = pstatus, outer = 0, total = 0, converged = 0;
  double relmax = 1.0;
  while (status == GABP_OK) {
    // inner: h-only sweeps on the correction system A d = r
    int t = 1;
    for (;; ++t) {
      Red rd{0.f, 0.f, 0.0, 0};
      if (SER) {
        for (int q = 0; q < ncls; ++q) {
          int slo, shi, rhi;
          class_range(A, cls0, q, V, slo, shi, rhi);
          pass<kKH, true>(A, V, t, slo, shi, rhi, rd);
          __syncthreads();
        }
      } else {
        pass<kKH, false>(A, V, t, V.sl0, V.sl0 + V.nsl, V.n, rd);
      }
      reduce_max2(sh, rd.dmax, rd.xmax, kg);
      bool done = t >= 2;
      for (int j = 0; j < kg; ++j) {
        const float dm = __uint_as_float(sh.fmx[j]), xm = __uint_as_float(sh.fmx[kMaxGroup + j]);
        if (!(dm <= A.inner_tol * xm)) done = false;
        if (!(dm <= 1e30f)) status = GABP_E_NONFINITE;
      }
      if (done || status != GABP_OK || total + t >= A.max_iter || t >= A.inner_max) break;
    }
    total += t;
    // x += d (FP64) with d = h~ / P~ of the last inner round, then r = b - A x
    {
      const float* hT = SER ? V.hagg0 : V.hagg(t);
      for (int64_t q = tid; q < nk; q += kBT) V.xint[q] += (double)(hT[q] * V.invPt[q >> V.lgk]);
      __syncthreads();
    }
    Red rd{0.f, 0.f, 0.0, 0};
    pass<kKSpmv, false>(A, V, 0, V.sl0, V.sl0 + V.nsl, V.n, rd);
    reduce_sum(sh, rd.r2, kg);
    ++outer;
    relmax = 0.0;
    for (int j = 0; j < kg; ++j) {
      const double nr = sqrt(sh.tot[j]);
      const double rel = sh.bn[j] > 0.0 ? nr / sh.bn[j] : nr;
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
    if (outer >= A.max_outer || total >= A.max_iter) break;
  }
  // X in the caller's row order
  for (int64_t q = tid; q < nk; q += kBT) {
    const int i = (int)(q >> V.lgk);
    V.X[(int64_t)(A.umap[V.r0 + i] - V.r0) * V.k + V.j0 + jj] = V.xint[q];
  }
  if (tid == 0) {
    ItemInfo inf{};
    inf.sweeps = total;
    inf.outer = outer;
    inf.converged = converged;
    inf.status = status != GABP_OK ? status : (converged ? GABP_OK : GABP_NOT_CONVERGED);
    inf.rel = relmax;
    inf.psweeps = A.pinfos[I.sys].psweeps;
    inf.t0 = t_start;
    inf.t1 = wall_clock64();
    A.infos[it] = inf;
  }
  __syncthreads();
}

__device__ __forceinline__ BItem uniform_item(const BItem& x) {
  BItem u;
  u.sys = uni(x.sys);
  u.j0 = uni(x.j0);
  u.kg = uni(x.kg);
  u.k = uni(x.k);
  u.off_h = uni(x.off_h);
  u.off_nk = uni(x.off_nk);
  u.off_x = uni(x.off_x);
  u.rhs_off = uni(x.rhs_off);
  return u;
}

// Persistent kernels: every workgroup takes items until its queue is empty.
// At most 64 VGPRs, so that four 512-lane workgroups reside per CU: measured
// on the 4096-system batch, 97 VGPRs (two workgroups per CU) took 1.27 s
// (colour-serial 0.82 s), 80 (three) 1.04 s (0.73 s) and 64 (four) 1.05 s
// (0.69 s); 256-lane workgroups with five per CU took 1.34 s (0.83 s).  With
// four per CU the chip runs near its memory bandwidth, so the few spilled
// registers cost nothing measurable.
template <bool SER>
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(8))) void k_bprec(BatchArgs A) {
  __shared__ Shared sh;
  for (;;) {
    if (threadIdx.x == 0) sh.item = (int)atomicAdd(&A.queue[0], 1u);
    __syncthreads();
    const int q = __builtin_amdgcn_readfirstlane(sh.item);
    __syncthreads();
    if (q >= A.num_sys) return;
    precision_item<SER>(A, __builtin_amdgcn_readfirstlane(A.porder[q]), sh);
  }
}

template <bool SER>
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(8))) void k_brhs(BatchArgs A) {
  __shared__ Shared sh;
  for (;;) {
    if (threadIdx.x == 0) sh.item = (int)atomicAdd(&A.queue[1], 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(sh.item);
    __syncthreads();
    if (it >= A.num_items) return;
    rhs_item<SER>(A, uniform_item(A.items[it]), it, sh);
  }
}

__global__ void k_reset_queues(uint32_t* q) {
  if (threadIdx.x < 2) q[threadIdx.x] = 0u;
}

// The SELL arrays of every slice: one thread per (slice, lane).  new2cur maps
// a row of the new internal order to the row of the ingested (possibly
// colour-ordered) off-diagonal CSR, cur2new back; slots beyond a row's degree
// are padding and are never read.
__global__ void k_build_sell(int32_t nslices, const Slice* __restrict__ slices, const int32_t* __restrict__ slice_sys,
                             const SysRec* __restrict__ sys, const int32_t* __restrict__ new2cur,
                             const int32_t* __restrict__ cur2new, const int32_t* __restrict__ cur2caller,
                             const int32_t* __restrict__ off_ptr, const int32_t* __restrict__ off_col,
                             const float* __restrict__ a32, const double* __restrict__ a64,
                             const float* __restrict__ dcur32, const double* __restrict__ dcur64, int32_t* col_s,
                             float* a32_s, double* a64_s, int32_t* deg, float* d32, double* d64, int32_t* umap) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nslices * kSlice) return;
  const int sl_i = (int)(gid / kSlice), lane = (int)(gid % kSlice);
  const Slice sl = slices[sl_i];
  const SysRec R = sys[slice_sys[sl_i]];
  const bool valid = lane < sl.nrows;
  const int row = sl.row0 + lane;  // system-local, new order
  int d = 0, cur = 0, e0 = 0;
  if (valid) {
    const int grow = R.r0 + row;
    cur = new2cur[grow];
    e0 = off_ptr[cur];
    d = off_ptr[cur + 1] - e0;
    deg[grow] = d;
    d32[grow] = dcur32[cur];
    d64[grow] = dcur64[cur];
    umap[grow] = cur2caller ? cur2caller[cur] : cur;
  }
  for (int q = 0; q < sl.L; ++q) {
    const int64_t s = sl.base + (int64_t)q * kSlice + lane;
    if (q < d) {
      col_s[s] = cur2new[off_col[e0 + q]] - R.r0;
      a32_s[s] = a32[e0 + q];
      a64_s[s] = a64[e0 + q];
    } else {
      col_s[s] = valid ? row : 0;
      a32_s[s] = 0.f;
      a64_s[s] = 0.0;
    }
  }
}

// Spectral radius of R = D^-1/2 (D - A) D^-1/2 (the signed off-diagonal part,
// D = diag A) of every system, for the work estimate: kRhoIters steps of the
// power iteration from a scrambled start, one workgroup per system, on the
// similar matrix D^-1 (D - A) (same spectrum, no square roots), the estimate
// being the growth of the 2-norm in the last step (it approaches rho).
// Attractive systems (all A_ij < 0, the grids) have rho(R) = rho(|R|) =
// 1 / (dominance ratio); mixed signs give much less, and GaBP's sweep count
// follows rho(R), not the dominance ratio.
constexpr int kRhoIters = 30;

__global__ __launch_bounds__(256) void k_sys_rho(int num_sys, const int32_t* __restrict__ sys_row_off,
                                                 const int32_t* __restrict__ off_ptr,
                                                 const int32_t* __restrict__ off_col,
                                                 const double* __restrict__ a, const double* __restrict__ d,
                                                 double* xa, double* xb, float* __restrict__ out) {
  __shared__ double s_red[4];
  for (int s = blockIdx.x; s < num_sys; s += gridDim.x) {
    const int r0 = sys_row_off[s], r1 = sys_row_off[s + 1];
    for (int r = r0 + (int)threadIdx.x; r < r1; r += 256) {
      const uint32_t h = (uint32_t)r * 2654435761u;
      xa[r] = (double)(h >> 8) * (1.0 / 16777216.0) - 0.5;
    }
    __syncthreads();
    double* x = xa;
    double* y = xb;
    double grow = 0.0;
    for (int it = 0; it < kRhoIters; ++it) {
      double nx = 0.0, ny = 0.0;
      for (int r = r0 + (int)threadIdx.x; r < r1; r += 256) {
        double acc = 0.0;
        for (int q = off_ptr[r]; q < off_ptr[r + 1]; ++q) acc -= a[q] * x[off_col[q]];
        acc /= d[r];
        y[r] = acc;
        nx += x[r] * x[r];
        ny += acc * acc;
      }
      // block sums of ||x||^2 and ||y||^2
      double v[2] = {nx, ny};
      for (int k = 0; k < 2; ++k) {
        double w = v[k];
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = w;
        __syncthreads();
        v[k] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
      }
      grow = v[0] > 0.0 ? sqrt(v[1] / v[0]) : 0.0;
      const double sc = v[1] > 0.0 ? 1.0 / sqrt(v[1]) : 0.0;
      for (int r = r0 + (int)threadIdx.x; r < r1; r += 256) y[r] *= sc;
      __syncthreads();
      double* t = x;
      x = y;
      y = t;
    }
    if (threadIdx.x == 0) out[s] = (float)grow;
    __syncthreads();
  }
}

// Relative sweep count of a system for the work estimate: GaBP's error
// contracts by about rho(R) per sweep, so the sweeps to a fixed reduction
// scale as -1 / ln(rho(R)) (bounded both ways).
double sweep_weight(float rho) {
  if (!(rho < 1.0f)) return 100.0;
  if (!(rho > 0.0f)) return 0.1;
  return std::min(100.0, std::max(0.1, -1.0 / std::log((double)rho)));
}

struct BatchState {
  int32_t num_sys = 0;
  std::vector<int32_t> sys_row_off;
  std::vector<SysRec> sys_h;
  std::vector<double> sys_weight;  // relative sweeps per system (work estimate)
  int64_t Stot = 0;
  int32_t nslices = 0;
  // device structure
  SysRec* sys_d = nullptr;
  Slice* slices_d = nullptr;
  int32_t* cls_sl_d = nullptr;
  int32_t* deg_d = nullptr;
  float* d32_d = nullptr;
  double* d64_d = nullptr;
  int32_t* umap_d = nullptr;
  int32_t* col_d = nullptr;
  float* a32_d = nullptr;
  double* a64_d = nullptr;
  // precision phase: per-system state and outputs
  int32_t* porder_d = nullptr;
  float* pP_d = nullptr;
  float2* pcoef_d = nullptr;
  float* pagg_d = nullptr;
  float* pinv_d = nullptr;
  ItemInfo* pinfo_d = nullptr;
  // per-solve work list and scratch (grown on demand)
  std::vector<BItem> items;
  BItem* items_d = nullptr;
  ItemInfo* infos_d = nullptr;
  size_t items_cap = 0;
  uint32_t* queue_d = nullptr;
  float* hbuf = nullptr;
  float* nkbuf = nullptr;
  double* xbuf = nullptr;
  int64_t hcap = 0, nkcap = 0, xcap = 0;
  int grid_p = 0, grid_r = 0;
  int launched_grid = 0;
  bool serial = false;
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

template <typename T>
gabp_status raw_alloc(Ctx* c, T** p, int64_t count) {
  hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)std::max<int64_t>(count, 16));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(c, GABP_E_OOM, "batched allocation failed");
  }
  return GABP_OK;
}

template <typename T>
gabp_status grow(Ctx* c, T** p, int64_t* cap, int64_t need) {
  if (need <= *cap) return GABP_OK;
  free_raw(*p);
  *p = nullptr;
  *cap = 0;
  gabp_status r = raw_alloc(c, p, need);
  if (r != GABP_OK) return r;
  *cap = need;
  return GABP_OK;
}

#define BTRY(x)                    \
  do {                             \
    gabp_status s_ = (x);          \
    if (s_ != GABP_OK) return s_;  \
  } while (0)

}  // namespace

gabp_status batched_create(Ctx* c, int32_t num_sys, const int32_t* sys_row_off) {
  auto* bs = new BatchState();
  c->batch = bs;
  bs->num_sys = num_sys;
  bs->sys_row_off.assign(sys_row_off, sys_row_off + num_sys + 1);
  bs->serial = c->opts.layout == kLayoutSerial;
  hipStream_t st = c->stream;
  const int32_t N = c->n;
  if (bs->serial) {
    c->layout = kLayoutSerial;
    if (c->cls_row.empty()) {  // no rows: one empty class list per system
      c->cls_row.assign(num_sys, 0);
      c->cls_base.resize(num_sys + 1);
      for (int s = 0; s <= num_sys; ++s) c->cls_base[s] = s;
    }
    // every system's class list runs from its first row to its end, in order
    bool ok = (int32_t)c->cls_base.size() == num_sys + 1;
    for (int s = 0; ok && s < num_sys; ++s) {
      const int32_t b0 = c->cls_base[s], b1 = c->cls_base[s + 1];
      ok = b1 > b0 && b1 <= (int32_t)c->cls_row.size() && c->cls_row[b0] == sys_row_off[s] &&
           c->cls_row[b1 - 1] == sys_row_off[s + 1];
      for (int32_t k = b0; ok && k + 1 < b1; ++k) ok = c->cls_row[k] <= c->cls_row[k + 1];
    }
    if (!ok) return fail(c, GABP_E_ARG, "internal: invalid colour class lists");
  }
  GABP_HIP(c, hipMalloc((void**)&bs->queue_d, 2 * sizeof(uint32_t)));

  // ---- the new row order and the slices, on the host ----------------------
  const std::vector<int32_t>& op = c->off_ptr_h;
  std::vector<int32_t> new2cur(std::max(N, 1)), cur2new(std::max(N, 1));
  std::vector<Slice> slices;
  std::vector<int32_t> slice_sys;
  std::vector<int32_t> cls_sl;
  bs->sys_h.resize(num_sys);
  int64_t ss = 0, offps = 0, offpn = 0;
  for (int s = 0; s < num_sys; ++s) {
    SysRec& R = bs->sys_h[s];
    R.r0 = sys_row_off[s];
    R.n = sys_row_off[s + 1] - sys_row_off[s];
    R.sl0 = (int32_t)slices.size();
    R.ss0 = ss;
    // segments: the whole system, or its colour classes
    std::vector<int32_t> seg;
    if (bs->serial) {
      for (int32_t k = c->cls_base[s]; k < c->cls_base[s + 1]; ++k) seg.push_back(c->cls_row[k]);
    } else {
      seg = {R.r0, R.r0 + R.n};
    }
    R.cls0 = (int32_t)cls_sl.size();
    R.ncls = (int32_t)seg.size() - 1;
    for (size_t g = 0; g + 1 < seg.size(); ++g) {
      cls_sl.push_back((int32_t)slices.size());
      // decreasing degree inside windows of kSortWindow rows (stable: the
      // caller's order among equal degrees)
      for (int32_t w0 = seg[g]; w0 < seg[g + 1]; w0 += kSortWindow) {
        const int32_t w1 = std::min(seg[g + 1], w0 + kSortWindow);
        std::vector<int32_t> rows(w1 - w0);
        std::iota(rows.begin(), rows.end(), w0);
        std::stable_sort(rows.begin(), rows.end(), [&](int32_t a, int32_t b) {
          return op[a + 1] - op[a] > op[b + 1] - op[b];
        });
        for (int32_t k = 0; k < w1 - w0; ++k) {
          new2cur[w0 + k] = rows[k];
          cur2new[rows[k]] = w0 + k;
        }
      }
      for (int32_t r = seg[g]; r < seg[g + 1]; r += kSlice) {
        Slice sl{};
        sl.base = ss;
        sl.row0 = r - R.r0;
        sl.nrows = std::min(kSlice, seg[g + 1] - r);
        int L = 0;
        for (int32_t k = 0; k < sl.nrows; ++k) {
          const int32_t cur = new2cur[r + k];
          L = std::max(L, op[cur + 1] - op[cur]);
        }
        sl.L = L;
        ss += (int64_t)kSlice * L;
        slices.push_back(sl);
        slice_sys.push_back(s);
      }
    }
    cls_sl.push_back((int32_t)slices.size());
    R.nsl = (int32_t)slices.size() - R.sl0;
    R.S = ss - R.ss0;
    R.off_ps = offps;
    R.off_pn = offpn;
    offps += R.S;
    offpn += R.n;
  }
  bs->Stot = ss;
  bs->nslices = (int32_t)slices.size();

  // ---- device structure ----------------------------------------------------
  // FP32 copy of the diagonal in the ingested order
  {
    void* p = nullptr;
    gabp_status r = dev_alloc(c, &p, sizeof(float) * std::max<int64_t>(1, N));
    if (r != GABP_OK) return r;
    c->din32_d = (float*)p;
    if (N > 0) GABP_HIP(c, launch_scale_diag(c->d64_d, 1.0, nullptr, c->din32_d, N, st));
  }
  BTRY(raw_alloc(c, &bs->sys_d, num_sys));
  BTRY(raw_alloc(c, &bs->slices_d, bs->nslices));
  BTRY(raw_alloc(c, &bs->cls_sl_d, (int64_t)cls_sl.size()));
  BTRY(raw_alloc(c, &bs->deg_d, N));
  BTRY(raw_alloc(c, &bs->d32_d, N));
  BTRY(raw_alloc(c, &bs->d64_d, N));
  BTRY(raw_alloc(c, &bs->umap_d, N));
  BTRY(raw_alloc(c, &bs->col_d, bs->Stot));
  BTRY(raw_alloc(c, &bs->a32_d, bs->Stot));
  BTRY(raw_alloc(c, &bs->a64_d, bs->Stot));
  BTRY(raw_alloc(c, &bs->porder_d, num_sys));
  BTRY(raw_alloc(c, &bs->pP_d, 2 * bs->Stot));
  BTRY(raw_alloc(c, &bs->pcoef_d, bs->Stot));
  BTRY(raw_alloc(c, &bs->pagg_d, 3 * (int64_t)N));
  BTRY(raw_alloc(c, &bs->pinv_d, N));
  BTRY(raw_alloc(c, &bs->pinfo_d, num_sys));
  GABP_HIP(c, hipMemcpyAsync(bs->sys_d, bs->sys_h.data(), sizeof(SysRec) * num_sys, hipMemcpyHostToDevice, st));
  if (bs->nslices > 0) {
    GABP_HIP(c, hipMemcpyAsync(bs->slices_d, slices.data(), sizeof(Slice) * slices.size(), hipMemcpyHostToDevice, st));
  }
  GABP_HIP(c, hipMemcpyAsync(bs->cls_sl_d, cls_sl.data(), sizeof(int32_t) * cls_sl.size(), hipMemcpyHostToDevice, st));
  if (N > 0 && bs->nslices > 0) {
    int32_t *n2c = nullptr, *c2n = nullptr, *ssys = nullptr;
    BTRY(raw_alloc(c, &n2c, N));
    BTRY(raw_alloc(c, &c2n, N));
    BTRY(raw_alloc(c, &ssys, bs->nslices));
    hipError_t e = hipMemcpyAsync(n2c, new2cur.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(c2n, cur2new.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ssys, slice_sys.data(), sizeof(int32_t) * bs->nslices, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      const int64_t threads = (int64_t)bs->nslices * kSlice;
      hipLaunchKernelGGL(k_build_sell, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, bs->nslices,
                         bs->slices_d, ssys, bs->sys_d, n2c, c2n, bs->serial ? c->inv_d : nullptr, c->off_ptr_d,
                         c->off_col_d, c->a32_d, c->a64_d, c->din32_d, c->d64_d, bs->col_d, bs->a32_d, bs->a64_d,
                         bs->deg_d, bs->d32_d, bs->d64_d, bs->umap_d);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    free_raw(n2c);
    free_raw(c2n);
    free_raw(ssys);
    if (e != hipSuccess) return hip_fail(c, e, "batched layout");
  }
  // persistent grids: as many workgroups as can be resident at once
  int dev = 0, ncu = 0, per_p = 0, per_r = 0;
  GABP_HIP(c, hipGetDevice(&dev));
  GABP_HIP(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  if (bs->serial) {
    GABP_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_p, k_bprec<true>, kBT, 0));
    GABP_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_r, k_brhs<true>, kBT, 0));
  } else {
    GABP_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_p, k_bprec<false>, kBT, 0));
    GABP_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_r, k_brhs<false>, kBT, 0));
  }
  bs->grid_p = std::max(1, ncu * std::max(1, per_p));
  bs->grid_r = std::max(1, ncu * std::max(1, per_r));
  int khz = 0;
  GABP_HIP(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  bs->clock_khz = khz;
  // the graph is captured and replayed on a stream of the handle's own, ordered
  // after the caller's stream by synchronisation (capture needs a non-null stream)
  GABP_HIP(c, hipStreamCreateWithFlags(&bs->gs, hipStreamNonBlocking));
  // per-system spectral radius of R for the work estimate
  bs->sys_weight.assign(num_sys, 1.0);
  if (c->E > 0) {
    int32_t* so_d = nullptr;
    float* rho_d = nullptr;
    double *xa = nullptr, *xb = nullptr;
    std::vector<float> rho(num_sys);
    hipError_t e = hipMalloc((void**)&so_d, sizeof(int32_t) * (num_sys + 1));
    if (e == hipSuccess) e = hipMalloc((void**)&rho_d, sizeof(float) * num_sys);
    if (e == hipSuccess) e = hipMalloc((void**)&xa, sizeof(double) * std::max(1, N));
    if (e == hipSuccess) e = hipMalloc((void**)&xb, sizeof(double) * std::max(1, N));
    if (e == hipSuccess)
      e = hipMemcpyAsync(so_d, sys_row_off, sizeof(int32_t) * (num_sys + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_sys_rho, dim3(std::min(num_sys, 8192)), dim3(256), 0, st, num_sys, so_d, c->off_ptr_d,
                         c->off_col_d, c->a64_d, c->d64_d, xa, xb, rho_d);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(rho.data(), rho_d, sizeof(float) * num_sys, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) (void)hipGetLastError();
    free_raw(so_d);
    free_raw(rho_d);
    free_raw(xa);
    free_raw(xb);
    if (e != hipSuccess) return hip_fail(c, e, "batched work estimate");
    for (int s = 0; s < num_sys; ++s) bs->sys_weight[s] = sweep_weight(rho[s]);
  }
  // the precision phase's order: largest systems first
  {
    std::vector<int32_t> order(num_sys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return (double)(bs->sys_h[a].S + bs->sys_h[a].n) > (double)(bs->sys_h[b].S + bs->sys_h[b].n);
    });
    GABP_HIP(c, hipMemcpyAsync(bs->porder_d, order.data(), sizeof(int32_t) * num_sys, hipMemcpyHostToDevice, st));
    GABP_HIP(c, hipStreamSynchronize(st));
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
    // Work items, costliest first.  The work of one right-hand side of a
    // system is taken as (slots + rows) per sweep times the system's relative
    // sweep count.  A system's right-hand sides are grouped in 8, 4, 2 or 1,
    // the largest group whose item stays within a third of an even share of
    // the whole batch per workgroup, so that no item is long next to the
    // makespan.
    auto unit = [&](int s) { return (double)(bs->sys_h[s].S + bs->sys_h[s].n) * bs->sys_weight[s]; };
    double total = 0.0;
    for (int s = 0; s < S; ++s) total += unit(s) * nrhs[s];
    const double cap = std::max(1.0, total / (3.0 * std::max(1, bs->grid_r)));
    std::vector<BItem> items;
    int64_t oh = 0, onk = 0, ox = 0;
    for (int s = 0; s < S; ++s) {
      const SysRec& R = bs->sys_h[s];
      if (R.n == 0) continue;
      const int32_t k = nrhs[s];
      int32_t gmax = kMaxGroup;
      while (gmax > 1 && unit(s) * gmax > cap) gmax >>= 1;
      for (int32_t j0 = 0; j0 < k;) {
        int32_t kg = gmax;
        while (kg > k - j0) kg >>= 1;
        BItem it{};
        it.sys = s;
        it.j0 = j0;
        it.kg = kg;
        it.k = k;
        it.off_h = oh;
        it.off_nk = onk;
        it.off_x = ox;
        it.rhs_off = rhs_off[s];
        oh += 2 * R.S * kg;
        onk += 4 * (int64_t)R.n * kg;
        ox += (int64_t)R.n * kg;
        items.push_back(it);
        j0 += kg;
      }
    }
    std::stable_sort(items.begin(), items.end(), [&](const BItem& a, const BItem& b) {
      return unit(a.sys) * a.kg > unit(b.sys) * b.kg;
    });
    bs->items = items;
    BTRY(grow(c, &bs->hbuf, &bs->hcap, oh));
    BTRY(grow(c, &bs->nkbuf, &bs->nkcap, onk));
    BTRY(grow(c, &bs->xbuf, &bs->xcap, ox));
    if (items.size() > bs->items_cap) {
      free_raw(bs->items_d);
      free_raw(bs->infos_d);
      bs->items_d = nullptr;
      bs->infos_d = nullptr;
      bs->items_cap = 0;
      BTRY(raw_alloc(c, &bs->items_d, (int64_t)items.size()));
      BTRY(raw_alloc(c, &bs->infos_d, (int64_t)items.size()));
      bs->items_cap = items.size();
    }
    if (!items.empty())
      GABP_HIP(c, hipMemcpyAsync(bs->items_d, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice,
                                 c->stream));
    BatchArgs a{};
    a.sys = bs->sys_d;
    a.slices = bs->slices_d;
    a.cls_sl = bs->cls_sl_d;
    a.deg = bs->deg_d;
    a.d32 = bs->d32_d;
    a.d64 = bs->d64_d;
    a.umap = bs->umap_d;
    a.col = bs->col_d;
    a.a32 = bs->a32_d;
    a.a64 = bs->a64_d;
    a.porder = bs->porder_d;
    a.num_sys = S;
    a.pP = bs->pP_d;
    a.pcoef = bs->pcoef_d;
    a.pagg = bs->pagg_d;
    a.pinv = bs->pinv_d;
    a.pinfos = bs->pinfo_d;
    a.items = bs->items_d;
    a.num_items = (int32_t)items.size();
    a.infos = bs->infos_d;
    a.hbuf = bs->hbuf;
    a.nkbuf = bs->nkbuf;
    a.xbuf = bs->xbuf;
    a.queue = bs->queue_d;
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
    // capture: queue reset (a kernel, not a memset node), the precision phase,
    // then the right-hand sides
    GABP_HIP(c, hipStreamSynchronize(c->stream));
    GABP_HIP(c, hipStreamBeginCapture(bs->gs, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, bs->gs, bs->queue_d);
    const int gp = std::max(1, std::min(bs->grid_p, S));
    const int gr = std::max(1, std::min<int>(bs->grid_r, (int)items.size()));
    bs->launched_grid = gr;
    if (bs->serial) {
      hipLaunchKernelGGL(k_bprec<true>, dim3(gp), dim3(kBT), 0, bs->gs, a);
      if (!items.empty()) hipLaunchKernelGGL(k_brhs<true>, dim3(gr), dim3(kBT), 0, bs->gs, a);
    } else {
      hipLaunchKernelGGL(k_bprec<false>, dim3(gp), dim3(kBT), 0, bs->gs, a);
      if (!items.empty()) hipLaunchKernelGGL(k_brhs<false>, dim3(gr), dim3(kBT), 0, bs->gs, a);
    }
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
  std::vector<ItemInfo> ii(bs->items.size()), pi(S);
  GABP_HIP(c, hipMemcpyAsync(ii.data(), bs->infos_d, sizeof(ItemInfo) * ii.size(), hipMemcpyDeviceToHost, bs->gs));
  GABP_HIP(c, hipMemcpyAsync(pi.data(), bs->pinfo_d, sizeof(ItemInfo) * S, hipMemcpyDeviceToHost, bs->gs));
  GABP_HIP(c, hipStreamSynchronize(bs->gs));
  // load-balance profile of the launch
  {
    gabp_batch_profile& pf = bs->prof;
    pf = gabp_batch_profile{};
    pf.num_items = (int32_t)ii.size();
    pf.workgroups = bs->launched_grid;
    uint64_t lo = ~0ull, hi = 0, plo = ~0ull, phi = 0;
    double busy = 0.0, longest = -1.0;
    size_t arg = 0;
    for (int s = 0; s < S; ++s) {
      if (bs->sys_h[s].n == 0) continue;
      plo = std::min(plo, pi[s].t0);
      phi = std::max(phi, pi[s].t1);
      busy += (double)(pi[s].t1 - pi[s].t0) / bs->clock_khz;
      pf.precision_sweeps += pi[s].psweeps;
    }
    for (size_t q = 0; q < ii.size(); ++q) {
      lo = std::min(lo, ii[q].t0);
      hi = std::max(hi, ii[q].t1);
      const double ms = (double)(ii[q].t1 - ii[q].t0) / bs->clock_khz;
      busy += ms;
      if (ms > longest) {
        longest = ms;
        arg = q;
      }
      pf.inner_sweeps += ii[q].sweeps;
    }
    const uint64_t first = std::min(lo, plo);
    pf.makespan_ms = ii.empty() ? 0.0 : (double)(hi - first) / bs->clock_khz;
    pf.busy_ms = busy;
    pf.longest_item_ms = std::max(0.0, longest);
    pf.precision_items = S;
    pf.precision_ms = plo <= phi ? (double)(phi - plo) / bs->clock_khz : 0.0;
    if (!ii.empty()) {
      pf.longest_sys = bs->items[arg].sys;
      pf.longest_nrhs = bs->items[arg].kg;
      pf.longest_sweeps = ii[arg].sweeps;
      pf.longest_psweeps = ii[arg].psweeps;
      pf.longest_start_ms = (double)(ii[arg].t0 - first) / bs->clock_khz;
    }
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
    const BItem& it = bs->items[q];
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
  for (void* p : {(void*)bs->items_d, (void*)bs->infos_d, (void*)bs->queue_d, (void*)bs->sys_d,
                  (void*)bs->slices_d, (void*)bs->cls_sl_d, (void*)bs->deg_d, (void*)bs->d32_d, (void*)bs->d64_d,
                  (void*)bs->umap_d, (void*)bs->col_d, (void*)bs->a32_d, (void*)bs->a64_d, (void*)bs->porder_d,
                  (void*)bs->pP_d, (void*)bs->pcoef_d, (void*)bs->pagg_d, (void*)bs->pinv_d, (void*)bs->pinfo_d,
                  (void*)bs->hbuf, (void*)bs->nkbuf, (void*)bs->xbuf})
    free_raw(p);
  if (bs->gs) (void)hipStreamDestroy(bs->gs);
  delete bs;
  c->batch = nullptr;
}

}  // namespace gabp
