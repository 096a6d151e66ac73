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
//      freeze g_in = -A_ij / (P~_i - P_ji), g_out and 1 / P~_i;
//   2. FP64 iterative refinement: r = b - A x in FP64; the correction A d = r
//      by h-only FP32 sweeps on all right-hand sides of the group at once
//      (messages and aggregates stored [slot][rhs] / [node][rhs], so a
//      neighbour gather reads kg contiguous words), x += d in FP64; until
//      every right-hand side reaches the relative residual tolerance.
// Every sweep walks the item's rows in tiles with slot-parallel tasks (see
// tile_pass); messages follow the compact one-message-per-slot form.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "gabp_internal.h"

namespace gabp {

namespace {

constexpr int kBT = 512;                // lanes per batched workgroup
constexpr int kKT = 4;                  // tasks per lane per chunk (FP32 passes)
constexpr int kMaxGroup = 8;            // right-hand sides per work item
constexpr float kPrecTol = 4e-7f;    // precision phase: relative change of P~ to stop at
constexpr float kPrecStall = 2e-5f;  // ... or below this, once it stops halving (FP32 rounding floor)
constexpr int kPrecStallSweeps = 8;

// Sweep kinds of the tile loop.
enum TileKind : int {
  kTP = 0,      // precision-only message sweep
  kTFreeze = 1, // frozen h-update coefficients from the precisions of a round
  kTH = 2,      // h-only message sweep, all right-hand sides of the item
  kTSpmv = 3    // FP64 residual r = b - A x
};

struct Item {
  int32_t sys, j0, kg, k;  // right-hand sides j0 .. j0+kg-1 of k
  int32_t r0, r1;          // global rows of the system
  int64_t s0, s1;          // global off-diagonal slots of the system
  int64_t off_e;           // item scratch: per-slot arrays (4 E floats)
  int64_t off_n;           // per-node arrays (4 n floats)
  int64_t off_he;          // h messages (2 E kg floats)
  int64_t off_nk;          // h aggregates and inner right-hand side (4 n kg floats)
  int64_t rhs_off;         // B / X offset of the system
  int32_t cls0, ncls;      // colour-serial: the system's class starts in cls_row, number of classes
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
  // colour-serial schedule: rows renumbered by colour class inside each system
  const int32_t* cls_row;  // global first row of each class (see Item::cls0)
  const int32_t* umap;     // [n] internal row -> caller row (B and X stay in caller order)
  int32_t serial;
};

using f2 = float __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void lds_max(unsigned* slot, float v) {
  // nonnegative floats order like their bit patterns; NaN maps above +inf
  atomicMax(slot, isnan(v) ? 0x7f800001u : __float_as_uint(v));
}

// Views of one item's scratch.  The message recursion is the compact form of
// Alg. 2: slot (j, i) keeps the incoming message i -> j of the even and of the
// odd rounds; the outgoing message j -> i of the previous round is recomputed
// from row j's own aggregate two rounds back,
//     out^(t-1) = F(A_j^(t-2), in^(t-2)),   in^(t) = F(A_i^(t-1), out^(t-1)),
// and the node aggregates rotate through three buffers (round mod 3).
struct ItemView {
  int n, kg, k, j0, r0;
  int64_t s0, E;
  f2* coef;        // [E] frozen {g_in, g_out}
  float* P0;       // [2][E] incoming precisions by round parity
  float* Pagg0;    // [3][n] P~ by round mod 3
  float* invPt;    // [n] frozen 1 / P~
  float* H0;       // [2][E kg] incoming h messages by round parity, [slot][rhs]
  float* hagg0;    // [3][n kg] h~ by round mod 3, [node][rhs]
  float* r32;      // [n kg] right-hand side of the correction system
  const double* B; // [n][k] of the system, caller's row order
  double* X;       // [n][k] of the system, caller's row order
  const int32_t* umap;  // colour-serial: item-local internal row -> global caller row (else null)
  // row of B and X (item-local) that holds internal row i
  __device__ int urow(int i) const { return umap ? umap[i] - r0 : i; }
  // buffers of a round (pointer arithmetic keeps the view in registers)
  __device__ float* P(int t) const { return P0 + (t & 1) * E; }
  __device__ float* Pagg(int t) const { return Pagg0 + (t % 3) * (int64_t)n; }
  __device__ float* H(int t) const { return H0 + (t & 1) * E * kg; }
  __device__ float* hagg(int t) const { return hagg0 + (t % 3) * (int64_t)n * kg; }
};

constexpr int kWave = 64;
constexpr int kWaves = kBT / kWave;
constexpr int kWChunk = kWave * kKT;  // tasks per wave chunk (FP32 passes)

// LDS of one wave (every wave walks its own tiles).
struct WaveShared {
  unsigned char* stage;  // kWChunk results (float; double for the residual, half as many)
  uint16_t* row;         // tile-local row of each slot of the chunk
  int32_t* ptr;          // tile-local slot offsets of the rows [kWave + 1]
  float* own;            // [kWave] own values per (row, rhs): round t-2 (freeze: T-1)
  float* own1;           // [kWave] own values per (row, rhs): round t-1 (freeze: T)
};

// Per-(row, right-hand side) results handed back by a tile sweep.
struct RowOut {
  float dmax, xmax;  // h sweep: change of d and size of d; P sweep: relative change of P~
  double r2;         // residual: sum of squares of this lane's rows
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One pass of the given kind over all rows of an item.  The rows are cut into
// tiles of R = 64 / kgE consecutive rows, and each wave of the workgroup
// walks its own tiles (tile w, w + 8, ...) with wave-level synchronisation
// only, so the waves' memory latencies overlap.  A tile's (slot, rhs) tasks
// are processed in chunks of up to kWChunk, up to kKT per lane with every load
// issued before the first is used; per-task results are staged in the wave's
// LDS and summed per (row, rhs) in slot order by the lane that owns the pair.
// The caller synchronises the workgroup after the pass.
// Reciprocal for the FP32 inner passes (about 1 ulp; the FP64 outer loop
// corrects whatever the inner solves leave).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <int KIND, bool SER>
__device__ void tile_pass(const BatchArgs& A, const ItemView& V, int t, const WaveShared& sh, RowOut& ro, int rlo,
                          int rhi) {
  const int lane = threadIdx.x & (kWave - 1);
  // uniform within the wave: the tile loop runs on scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int kgE = (KIND == kTH || KIND == kTSpmv) ? V.kg : 1;
  const int R = kWave / kgE;    // rows per tile; also slots per k-step of a chunk
  constexpr int KT = (KIND == kTSpmv) ? kKT / 2 : kKT;  // FP64 tasks hold twice the registers
  const int CHS = R * KT;       // slots per chunk
  // sweeps (synchronous freeze: T == 0, T == 1); the serial freeze has no first sweep
  const bool first = (t == 1) && !(SER && KIND == kTFreeze), second = (t == 2);
  // lane -> (slot offset, right-hand side); lanes R * kgE .. 63 idle when kgE
  // does not divide 64
  const bool tl = lane < R * kgE;
  const int ls = lane / kgE, jj = lane % kgE;
  const int kg = V.kg;
  // item-local bases (uniform), so that every per-task address is a 32-bit
  // offset from a scalar base
  const int* off_ptr = A.off_ptr + V.r0;
  const int* colp = A.off_col + V.s0;
  const float* a32p = A.a32 + V.s0;
  const double* a64p = A.a64 + V.s0;
  const float* d32p = A.d32 + V.r0;
  // synchronous: in^(t-2) -> in^(t) (freeze: in^(T)); serial: one set of
  // outgoing messages, updated in place
  float* Pt_ = SER ? V.P0 : V.P(t);
  const float* Pold_ = V.P(t + 1);                                       // freeze: in^(T-1)
  const float* Pg_ = SER ? V.Pagg0 : V.Pagg(KIND == kTFreeze ? t : t + 2);  // gathered P~ of round t-1 (T)
  float* Ht_ = SER ? V.H0 : V.H(t);
  const float* hg_ = SER ? V.hagg0 : V.hagg(t + 2);                      // gathered h~ of round t-1
  const float* r32_ = V.r32;
  const double* Xs = V.X + V.j0;
  float* stagef = (float*)sh.stage;
  double* staged = (double*)sh.stage;
  const int ntiles = (rhi - rlo + R - 1) / R;

  for (int tile = wave; tile < ntiles; tile += kWaves) {
    const int tr0 = rlo + tile * R;
    const int nr = min(R, rhi - tr0);
    const int e0 = off_ptr[tr0] - (int)V.s0;  // item-local slot of the tile's first row
    const int ne = off_ptr[tr0 + nr] - (int)V.s0 - e0;
    const bool rl = tl && ls < nr;  // lane owns the (row ls, rhs jj) pair
    const int i = tr0 + ls;         // item-local row of that pair

    // per-task registers of one chunk
    int tc[KT];
    float ta[KT], tm[KT], tg[KT];
    f2 tcf[KT];
    double tad[KT], txd[KT];
    auto load_chunk = [&](int cs0) {
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const int sl = cs0 + ls + k * R;  // tile-local slot
        if (tl && sl < ne) {
          const int e = e0 + sl;
          const int c = colp[e] - V.r0;
          tc[k] = c;
          if (KIND == kTP || KIND == kTFreeze) {
            ta[k] = a32p[e];
            tm[k] = 0.f;
            tcf[k] = f2{0.f, 0.f};
            if (SER) {
              if (!first) tm[k] = Pt_[e];                          // out_{j->i} of j's last update
            } else {
              if (KIND == kTP && !first && !second) tm[k] = Pt_[e];  // in^(t-2)
              if (KIND == kTFreeze && !first) {
                tm[k] = Pt_[e];                                      // in^(T)
                if (!second) tcf[k].x = Pold_[e];                    // in^(T-1)
              }
            }
          } else if (KIND == kTH) {
            tcf[k] = V.coef[e];
            if (SER) tm[k] = first ? 0.f : Ht_[e * kg + jj];             // h_out of j's last update
            else tm[k] = (!first && !second) ? Ht_[e * kg + jj] : 0.f;  // h_in^(t-2)
          } else {
            tad[k] = a64p[e];
          }
        }
      }
      // the gathers: neighbour aggregates of round t-1 (freeze: T), or x
      // (serial: the neighbour's last update; nothing from a later class in
      // the first sweep)
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const int sl = cs0 + ls + k * R;
        if (tl && sl < ne) {
          const int c = tc[k];
          const bool silent = SER && first && c >= rhi;
          if (KIND == kTP || KIND == kTFreeze) tg[k] = silent ? 0.f : ((first && !SER) ? d32p[c] : Pg_[c]);
          else if (KIND == kTH) tg[k] = silent ? 0.f : ((first && !SER) ? r32_ : hg_)[c * kg + jj];
          else txd[k] = Xs[(int64_t)V.urow(c) * V.k + jj];
        }
      }
    };
    load_chunk(0);

    // row side: slot offsets and own values of round t-2 (freeze: T-1) and
    // t-1 (T); what the epilogue needs besides is loaded here as well
    // (serial: the row's own aggregate of its last update)
    int rp = 0;
    float er = 0.f, eip = 0.f;  // epilogue: prior / inner right-hand side, 1 / P~
    if (rl) {
      rp = off_ptr[i] - (int)V.s0 - e0;
      float o1 = 0.f, o2 = 0.f;
      if (KIND == kTP) {
        if (SER) {
          o1 = first ? d32p[i] : V.Pagg0[i];
        } else {
          o1 = first ? d32p[i] : V.Pagg(t + 2)[i];
          o2 = second ? d32p[i] : (first ? 0.f : V.Pagg(t + 1)[i]);
        }
        er = d32p[i];
      } else if (KIND == kTFreeze) {
        if (SER) {
          o1 = V.Pagg0[i];
        } else {
          o1 = first ? d32p[i] : V.Pagg(t)[i];
          o2 = second ? d32p[i] : (first ? 0.f : V.Pagg(t + 2)[i]);
        }
      } else if (KIND == kTH) {
        const int q = i * kg + jj;
        er = r32_[q];
        eip = V.invPt[i];
        if (SER) {
          o1 = first ? 0.f : V.hagg0[q];
        } else {
          o1 = first ? er : V.hagg(t + 2)[q];
          o2 = second ? er : (first ? 0.f : V.hagg(t + 1)[q]);
        }
      }
      sh.own[lane] = o2;
      sh.own1[lane] = o1;
    }
    if (rl && jj == 0) sh.ptr[ls] = rp;
    if (lane == 0) sh.ptr[nr] = ne;
    wave_sync();
    const int lo = rl ? sh.ptr[ls] : 0, hi = rl ? sh.ptr[ls + 1] : 0;

    float accf = 0.f;
    double accd = 0.0;
    for (int cs0 = 0; cs0 < ne; cs0 += CHS) {
      if (cs0 > 0) load_chunk(cs0);
      const int cs1 = min(ne, cs0 + CHS);  // slots of this chunk
      if (rl && jj == 0)
        for (int e = max(lo, cs0); e < min(hi, cs1); ++e) sh.row[e - cs0] = (uint16_t)ls;
      wave_sync();
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const int sl = cs0 + ls + k * R;
        if (tl && sl < ne) {
          const int e = e0 + sl;
          const int st = (sl - cs0) * kgE + jj;  // stage slot of the task
          const int lr = sh.row[sl - cs0];
          if (SER && KIND == kTP) {
            // pulled in_{i->j} = F(P~_i, out_{j->i}), kept in the slot until pass 2
            const float Pin = (first && tc[k] >= rhi) ? 0.f : -ta[k] * ta[k] * rcp(tg[k] - tm[k]);
            Pt_[e] = Pin;
            stagef[st] = Pin;
          } else if (SER && KIND == kTFreeze) {
            const float av = ta[k];
            const float r_in = rcp(tg[k] - tm[k]);
            const float Pin = -av * av * r_in;
            f2 cf;
            cf.x = -av * r_in;                       // g_in  = -a / (P~_i - P_{j->i})
            cf.y = -av * rcp(sh.own1[lr] - Pin);     // g_out = -a / (P~_j - P_{i->j})
            V.coef[e] = cf;
            stagef[st] = cf.x + cf.y;  // finiteness only
          } else if (SER && KIND == kTH) {
            const float hin = (first && tc[k] >= rhi) ? 0.f : tcf[k].x * (tg[k] - tm[k]);
            Ht_[e * kg + jj] = hin;
            stagef[st] = hin;
          } else if (KIND == kTP) {
            const float av2 = -ta[k] * ta[k];
            float Pout = 0.f;
            if (!first) Pout = av2 * rcp(sh.own[lr] - tm[k]);  // out^(t-1)
            const float Pin = av2 * rcp(tg[k] - Pout);         // in^(t)
            Pt_[e] = Pin;
            stagef[st] = Pin;
          } else if (KIND == kTFreeze) {
            const float av = ta[k];
            float Pout = 0.f;
            if (!first) Pout = -av * av * rcp(sh.own[lr] - tcf[k].x);  // out^(T)
            f2 cf;
            cf.x = -av * rcp(tg[k] - Pout);          // g_in  = -a / (P~_i - P_ji)
            cf.y = -av * rcp(sh.own1[lr] - tm[k]);   // g_out = -a / (P~_j - P_ij)
            V.coef[e] = cf;
            stagef[st] = cf.x + cf.y;  // finiteness only
          } else if (KIND == kTH) {
            float hout = 0.f;
            if (!first) hout = tcf[k].y * (sh.own[lr * kgE + jj] - tm[k]);  // h_out^(t-1)
            const float hin = tcf[k].x * (tg[k] - hout);                     // h_in^(t)
            Ht_[e * kg + jj] = hin;
            stagef[st] = hin;
          } else {
            staged[st] = tad[k] * txd[k];
          }
        }
      }
      wave_sync();
      if (rl)
        for (int e = max(lo, cs0); e < min(hi, cs1); ++e) {
          const int st = (e - cs0) * kgE + jj;
          if (KIND == kTSpmv) accd += staged[st];
          else accf += stagef[st];
        }
      wave_sync();
    }

    // row epilogue
    if (rl) {
      const float o1 = sh.own1[lane];
      if (KIND == kTP) {
        const float Pt = er + accf;
        (SER ? V.Pagg0 : V.Pagg(t))[i] = Pt;
        ro.dmax = fmaxf(ro.dmax, fabsf(Pt - o1) / fabsf(Pt));
        if (SER) sh.own1[lane] = Pt;
      } else if (KIND == kTFreeze) {
        const float ip = rcp(o1);
        V.invPt[i] = ip;
        if (!isfinite(accf) || !isfinite(ip)) ro.dmax = __int_as_float(0x7fc00000);
      } else if (KIND == kTH) {
        const float ht = er + accf;
        (SER ? V.hagg0 : V.hagg(t))[i * kg + jj] = ht;
        const float dn = ht * eip;
        const float dold = first ? 0.f : o1 * eip;
        ro.dmax = fmaxf(ro.dmax, fabsf(dn - dold));
        ro.xmax = fmaxf(ro.xmax, fabsf(dn));
        if (SER) sh.own1[lane] = ht;
      } else {
        const int q = V.urow(i) * V.k + V.j0 + jj;
        const double r = V.B[q] - A.d64[V.r0 + i] * V.X[q] - accd;
        V.r32[i * kg + jj] = (float)r;
        ro.r2 += r * r;
      }
    }
    // serial pass 2: the new outgoing messages out_{j->i} = F(agg_j, in_{i->j}),
    // from the row's new aggregate and the pulled message kept in the slot
    if (SER && (KIND == kTP || KIND == kTH)) {
      wave_sync();
      for (int cs0 = 0; cs0 < ne; cs0 += CHS) {
        const int cs1 = min(ne, cs0 + CHS);
        if (rl && jj == 0)
          for (int e = max(lo, cs0); e < min(hi, cs1); ++e) sh.row[e - cs0] = (uint16_t)ls;
        wave_sync();
#pragma unroll
        for (int k = 0; k < KT; ++k) {
          const int sl = cs0 + ls + k * R;
          if (tl && sl < ne) {
            const int e = e0 + sl;
            const int lr = sh.row[sl - cs0];
            if (KIND == kTP) {
              const float av = a32p[e];
              const float Pin = Pt_[e];
              Pt_[e] = -av * av * rcp(sh.own1[lr] - Pin);
            } else {
              const float gout = V.coef[e].y;
              const float hin = Ht_[e * kg + jj];
              Ht_[e * kg + jj] = gout * (sh.own1[lr * kgE + jj] - hin);
            }
          }
        }
        wave_sync();
      }
    }
    wave_sync();  // the next tile rewrites the wave's LDS row structure
  }
}

// Column of the (row, rhs) pairs a thread owns in the tile passes (threads
// that own none contribute zeros under any column).
__device__ __forceinline__ int tile_col(int kg) { return (threadIdx.x & (kWave - 1)) % kg; }

// Per right-hand-side sums of one value per thread, column `col`, combined in
// thread order (deterministic).
__device__ void col_sums(double v, int col, int kg, double* s_part, int* s_cidx, double* out) {
  const int tid = threadIdx.x;
  s_part[tid] = v;
  s_cidx[tid] = col;
  __syncthreads();
  if (tid < kg) {
    double acc = 0.0;
    for (int t = 0; t < kBT; ++t)
      if (s_cidx[t] == tid) acc += s_part[t];
    out[tid] = acc;
  }
  __syncthreads();
}

// The item record read by every lane, made provably uniform (the compiler
// cannot use scalar loads for it), so that everything derived from it stays in
// scalar registers.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <bool SER>
__device__ void solve_item(const BatchArgs& A, const Item& I, int it, const WaveShared& sh, unsigned* s_max,
                           double* s_part, int* s_cidx, double* s_col, double* s_bn, int* s_flag) {
  const int tid = threadIdx.x;
  ItemView V;
  V.n = I.r1 - I.r0;
  V.kg = I.kg;
  V.k = I.k;
  V.j0 = I.j0;
  V.r0 = I.r0;
  V.s0 = I.s0;
  V.E = I.s1 - I.s0;
  float* eb = A.ebuf + 4 * I.off_e;
  V.coef = (f2*)eb;
  V.P0 = eb + 2 * V.E;
  float* nb = A.nbuf + 4 * I.off_n;
  V.Pagg0 = nb;
  V.invPt = nb + 3 * (int64_t)V.n;
  V.H0 = A.hbuf + 2 * I.off_he;
  float* kb = A.kbuf + 4 * I.off_nk;
  const int64_t nk = (int64_t)V.n * V.kg;
  V.hagg0 = kb;
  V.r32 = kb + 3 * nk;
  V.B = A.B + I.rhs_off;
  V.X = A.X + I.rhs_off;
  V.umap = SER ? A.umap + I.r0 : nullptr;
  const int kg = V.kg;
  const int Tq = (kBT / kg) * kg;  // lanes that own (row, rhs) pairs
  int status = 0;
  const uint64_t t_start = wall_clock64();

  // ---- 1. precision phase: P-only sweeps until P~ settles ------------------
  // The FP32 change of P~ settles at a rounding floor that can lie above
  // kPrecTol on weakly dominant systems; the phase also ends once the change
  // is small and has stopped halving (the FP64 refinement absorbs the rest).
  int tp = 1;
  float best = INFINITY;
  int tbest = 0;
  for (;; ++tp) {
    if (tid == 0) s_max[0] = 0u;
    __syncthreads();
    RowOut ro{0.f, 0.f, 0.0};
    if (SER) {
      for (int q = 0; q < I.ncls; ++q) {  // the colour classes in turn
        const int rlo = uni(A.cls_row[I.cls0 + q]) - I.r0, rhi = uni(A.cls_row[I.cls0 + q + 1]) - I.r0;
        tile_pass<kTP, true>(A, V, tp, sh, ro, rlo, rhi);
        __syncthreads();
      }
    } else {
      tile_pass<kTP, false>(A, V, tp, sh, ro, 0, V.n);
    }
    lds_max(&s_max[0], ro.dmax);
    __syncthreads();  // also orders this round's aggregates before the next pass
    const float ch = __uint_as_float(s_max[0]);
    __syncthreads();
    if (ch < 0.5f * best) {
      best = ch;
      tbest = tp;
    }
    if (tp >= 3 && ch <= kPrecTol) break;
    if (tp - tbest >= kPrecStallSweeps && best <= kPrecStall) break;
    if (tp >= A.inner_max || !(ch <= 1e30f)) break;
  }
  // freeze the h-update coefficients from the precisions of round tp
  {
    if (tid == 0) s_max[0] = 0u;
    __syncthreads();
    RowOut ro{0.f, 0.f, 0.0};
    tile_pass<kTFreeze, SER>(A, V, tp, sh, ro, 0, V.n);
    if (!(ro.dmax == 0.f)) *s_flag = 1;
    __syncthreads();
  }

  // ---- 2. FP64 refinement --------------------------------------------------
  const int jj = tid % kg;
  double bpart = 0.0;
  if (tid < Tq)
    for (int q = tid; q < V.n * kg; q += Tq) {
      const int i = q / kg;
      const int64_t qb = (int64_t)V.urow(i) * V.k + V.j0 + jj;
      const double bv = V.B[qb];
      V.X[qb] = 0.0;
      V.r32[q] = (float)bv;
      bpart += bv * bv;
    }
  col_sums(bpart, tid % kg, kg, s_part, s_cidx, s_bn);
  if (tid < kg) s_bn[tid] = sqrt(s_bn[tid]);
  __syncthreads();

  int outer = 0, total = 0, converged = 0;
  double relmax = 1.0;
  for (;;) {
    // inner: h-only sweeps on the correction system A d = r
    int t = 1;
    for (;; ++t) {
      if (tid < 2 * kMaxGroup) s_max[tid] = 0u;
      __syncthreads();
      RowOut ro{0.f, 0.f, 0.0};
      if (SER) {
        for (int q = 0; q < I.ncls; ++q) {
          const int rlo = uni(A.cls_row[I.cls0 + q]) - I.r0, rhi = uni(A.cls_row[I.cls0 + q + 1]) - I.r0;
          tile_pass<kTH, true>(A, V, t, sh, ro, rlo, rhi);
          __syncthreads();
        }
      } else {
        tile_pass<kTH, false>(A, V, t, sh, ro, 0, V.n);
      }
      lds_max(&s_max[tile_col(kg)], ro.dmax);
      lds_max(&s_max[kMaxGroup + tile_col(kg)], ro.xmax);
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
    // x += d (FP64) with d = h~ / P~ of the last inner round, then r = b - A x
    {
      const float* hT = SER ? V.hagg0 : V.hagg(t);
      if (tid < Tq)
        for (int q = tid; q < V.n * kg; q += Tq)
          V.X[(int64_t)V.urow(q / kg) * V.k + V.j0 + jj] += (double)(hT[q] * V.invPt[q / kg]);
      __syncthreads();
    }
    RowOut ro{0.f, 0.f, 0.0};
    __syncthreads();
    tile_pass<kTSpmv, SER>(A, V, 0, sh, ro, 0, V.n);
    col_sums(ro.r2, tile_col(kg), kg, s_part, s_cidx, s_col);
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

__device__ __forceinline__ Item uniform_item(const Item& x) {
  Item u;
  u.sys = uni(x.sys);
  u.j0 = uni(x.j0);
  u.kg = uni(x.kg);
  u.k = uni(x.k);
  u.r0 = uni(x.r0);
  u.r1 = uni(x.r1);
  u.s0 = uni(x.s0);
  u.s1 = uni(x.s1);
  u.off_e = uni(x.off_e);
  u.off_n = uni(x.off_n);
  u.off_he = uni(x.off_he);
  u.off_nk = uni(x.off_nk);
  u.rhs_off = uni(x.rhs_off);
  u.cls0 = uni(x.cls0);
  u.ncls = uni(x.ncls);
  return u;
}

// Register budget of 6 waves per SIMD (80 VGPRs): three 512-lane workgroups
// per CU.  A few registers spill, which costs less than the extra resident
// workgroups gain (two per CU without the cap, four with a tighter one are
// both slower on the 4096-system batch).
// SER: the colour-serial schedule (a separate kernel, so that the synchronous
// one keeps its own register allocation).
template <bool SER>
__global__ __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(6))) void k_batched(BatchArgs A) {
  __shared__ int s_item;
  __shared__ int s_flag;
  __shared__ unsigned s_max[2 * kMaxGroup];
  __shared__ double s_part[kBT];
  __shared__ int s_cidx[kBT];
  __shared__ double s_col[kMaxGroup];
  __shared__ double s_bn[kMaxGroup];
  // per-wave tile scratch
  __shared__ __align__(16) unsigned char s_stage[kWaves][kWChunk * sizeof(float)];
  __shared__ uint16_t s_row[kWaves][kWChunk];
  __shared__ int32_t s_ptr[kWaves][kWave + 4];
  __shared__ float s_own[kBT];
  __shared__ float s_own1[kBT];
  const int w = threadIdx.x / kWave;
  const WaveShared sh{s_stage[w], s_row[w], s_ptr[w], s_own + w * kWave, s_own1 + w * kWave};
  for (;;) {
    if (threadIdx.x == 0) {
      s_item = (int)atomicAdd(A.queue, 1u);
      s_flag = 0;
    }
    __syncthreads();
    // uniform across the workgroup: keeps the item's fields in scalar registers
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= A.num_items) return;  // every workgroup leaves once the queue is empty
    solve_item<SER>(A, uniform_item(A.items[it]), it, sh, s_max, s_part, s_cidx, s_col, s_bn, &s_flag);
  }
}

__global__ void k_reset_queue(uint32_t* q) {
  if (threadIdx.x == 0) *q = 0u;
}

// Smallest diagonal-dominance ratio |A_ii| / sum_j |A_ij| over the rows of
// each system (+inf for a system without off-diagonal entries).
__global__ __launch_bounds__(256) void k_sys_ratio(int num_sys, const int32_t* __restrict__ sys_row_off,
                                                   const int32_t* __restrict__ off_ptr,
                                                   const double* __restrict__ a, const double* __restrict__ d,
                                                   float* __restrict__ out) {
  __shared__ float s_min[256];
  for (int s = blockIdx.x; s < num_sys; s += gridDim.x) {
    float m = INFINITY;
    for (int r = sys_row_off[s] + (int)threadIdx.x; r < sys_row_off[s + 1]; r += 256) {
      double sum = 0.0;
      for (int q = off_ptr[r]; q < off_ptr[r + 1]; ++q) sum += fabs(a[q]);
      if (sum > 0.0) m = fminf(m, (float)(fabs(d[r]) / sum));
    }
    s_min[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) s_min[threadIdx.x] = fminf(s_min[threadIdx.x], s_min[threadIdx.x + off]);
      __syncthreads();
    }
    if (threadIdx.x == 0) out[s] = s_min[0];
    __syncthreads();
  }
}

// Relative sweep count of a system for the work estimate: Jacobi-like
// contraction by about 1 / rho per sweep for dominance ratio rho, so the
// sweeps to a fixed reduction scale as 1 / ln(rho) (bounded both ways).
double sweep_weight(float ratio) {
  if (!(ratio > 1.0f)) return 100.0;
  return std::min(100.0, std::max(0.1, 1.0 / std::log((double)ratio)));
}

struct BatchState {
  int32_t num_sys = 0;
  std::vector<int32_t> sys_row_off;
  std::vector<int64_t> sys_slot_off;
  std::vector<double> sys_weight;  // relative sweeps per system (work estimate)
  // per-solve work list and scratch (grown on demand)
  std::vector<Item> items;
  Item* items_d = nullptr;
  ItemInfo* infos_d = nullptr;
  size_t items_cap = 0;
  uint32_t* queue_d = nullptr;
  int32_t* cls_row_d = nullptr;  // colour-serial: class starts of every system
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
  if (c->opts.layout == kLayoutSerial) {
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
    GABP_HIP(c, hipMalloc((void**)&bs->cls_row_d, sizeof(int32_t) * c->cls_row.size()));
    GABP_HIP(c, hipMemcpyAsync(bs->cls_row_d, c->cls_row.data(), sizeof(int32_t) * c->cls_row.size(),
                               hipMemcpyHostToDevice, c->stream));
  }
  // the persistent grid: as many workgroups as can be resident at once
  int dev = 0, ncu = 0, per_cu = 0;
  GABP_HIP(c, hipGetDevice(&dev));
  GABP_HIP(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  GABP_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched<false>, kBT, 0));
  bs->grid = std::max(1, ncu * std::max(1, per_cu));
  int khz = 0;
  GABP_HIP(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  bs->clock_khz = khz;
  // the graph is captured and replayed on a stream of the handle's own, ordered
  // after the caller's stream by synchronisation (capture needs a non-null stream)
  GABP_HIP(c, hipStreamCreateWithFlags(&bs->gs, hipStreamNonBlocking));
  // per-system dominance ratios for the work estimate
  bs->sys_weight.assign(num_sys, 1.0);
  if (c->E > 0) {
    int32_t* so_d = nullptr;
    float* ratio_d = nullptr;
    std::vector<float> ratio(num_sys);
    hipError_t e = hipMalloc((void**)&so_d, sizeof(int32_t) * (num_sys + 1));
    if (e == hipSuccess) e = hipMalloc((void**)&ratio_d, sizeof(float) * num_sys);
    if (e == hipSuccess)
      e = hipMemcpyAsync(so_d, sys_row_off, sizeof(int32_t) * (num_sys + 1), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_sys_ratio, dim3(std::min(num_sys, 4096)), dim3(256), 0, c->stream, num_sys, so_d,
                         c->off_ptr_d, c->a64_d, c->d64_d, ratio_d);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(ratio.data(), ratio_d, sizeof(float) * num_sys, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    free_raw(so_d);
    free_raw(ratio_d);
    if (e != hipSuccess) return hip_fail(c, e, "batched work estimate");
    for (int s = 0; s < num_sys; ++s) bs->sys_weight[s] = sweep_weight(ratio[s]);
  }
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
    // Work items, costliest first.  The work of one right-hand side is taken
    // as (E_s + n_s) per sweep times the system's relative sweep count; a
    // system's right-hand sides are grouped so that no item exceeds half of
    // an even share of the whole batch per workgroup, which keeps the longest
    // item below the average workgroup load.
    auto unit = [&](int s) {
      return (double)(bs->sys_slot_off[s + 1] - bs->sys_slot_off[s] + bs->sys_row_off[s + 1] - bs->sys_row_off[s]) *
             bs->sys_weight[s];
    };
    double total = 0.0;
    for (int s = 0; s < S; ++s) total += unit(s) * nrhs[s];
    const double cap = std::max(1.0, total / (2.0 * std::max(1, bs->grid)));
    std::vector<Item> items;
    int64_t oe = 0, on = 0, ohe = 0, onk = 0;
    for (int s = 0; s < S; ++s) {
      const int32_t r0 = bs->sys_row_off[s], r1 = bs->sys_row_off[s + 1];
      if (r1 == r0) continue;
      const int64_t E = bs->sys_slot_off[s + 1] - bs->sys_slot_off[s];
      const int32_t k = nrhs[s];
      const int32_t group = (int32_t)std::max(1.0, std::min((double)kMaxGroup, std::floor(cap / std::max(1e-30, unit(s)))));
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
        if (bs->cls_row_d) {
          it.cls0 = c->cls_base[s];
          it.ncls = c->cls_base[s + 1] - c->cls_base[s] - 1;
        }
        oe += E;
        on += (r1 - r0);
        ohe += E * it.kg;
        onk += (int64_t)(r1 - r0) * it.kg;
        items.push_back(it);
      }
    }
    std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) {
      return unit(a.sys) * a.kg > unit(b.sys) * b.kg;
    });
    bs->items = items;
    gabp_status r = grow(c, &bs->ebuf, &bs->ecap, 4 * oe);
    if (r == GABP_OK) r = grow(c, &bs->nbuf, &bs->ncap, 4 * on);
    if (r == GABP_OK) r = grow(c, &bs->hbuf, &bs->hcap, 2 * ohe);
    if (r == GABP_OK) r = grow(c, &bs->kbuf, &bs->kcap, 4 * onk);
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
    a.serial = bs->cls_row_d ? 1 : 0;
    a.cls_row = bs->cls_row_d;
    a.umap = bs->cls_row_d ? c->inv_d : nullptr;
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
    if (a.serial) hipLaunchKernelGGL(k_batched<true>, dim3(grid), dim3(kBT), 0, bs->gs, a);
    else hipLaunchKernelGGL(k_batched<false>, dim3(grid), dim3(kBT), 0, bs->gs, a);
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
    double busy = 0.0, longest = -1.0;
    size_t arg = 0;
    for (size_t q = 0; q < ii.size(); ++q) {
      lo = std::min(lo, ii[q].t0);
      hi = std::max(hi, ii[q].t1);
      const double ms = (double)(ii[q].t1 - ii[q].t0) / bs->clock_khz;
      busy += ms;
      if (ms > longest) {
        longest = ms;
        arg = q;
      }
      pf.precision_sweeps += ii[q].psweeps;
      pf.inner_sweeps += ii[q].sweeps;
    }
    pf.makespan_ms = ii.empty() ? 0.0 : (double)(hi - lo) / bs->clock_khz;
    pf.busy_ms = busy;
    pf.longest_item_ms = std::max(0.0, longest);
    if (!ii.empty()) {
      pf.longest_sys = bs->items[arg].sys;
      pf.longest_nrhs = bs->items[arg].kg;
      pf.longest_sweeps = ii[arg].sweeps;
      pf.longest_psweeps = ii[arg].psweeps;
      pf.longest_start_ms = (double)(ii[arg].t0 - lo) / bs->clock_khz;
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
  free_raw(bs->cls_row_d);
  free_raw(bs->ebuf);
  free_raw(bs->nbuf);
  free_raw(bs->hbuf);
  free_raw(bs->kbuf);
  if (bs->gs) (void)hipStreamDestroy(bs->gs);
  delete bs;
  c->batch = nullptr;
}

}  // namespace gabp
