// Internal declarations shared by the HIP translation units of libgabp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gabp.h"

namespace gabp {

constexpr int kBlock = 256;            // lanes per workgroup in the sweep kernels
constexpr int kMaxRowsPerBlock = 256;  // one aggregate lane per row
constexpr double kDivergeLimit = 1e8;  // relative residual treated as divergence

// Device-side solver status.  Written only by the last-arriving workgroup of a
// checking sweep (or by any workgroup for the error bits); read at the start
// of every sweep so that sweeps enqueued after convergence return at once.
struct DevStatus {
  int32_t done;        // nonzero: converged or failed, later sweeps are no-ops
  int32_t conv_round;  // round whose x met the tolerance (-1: none)
  int32_t error;       // kErr* bits
  uint32_t ticket;     // arrival counter of the checking workgroups
  double last_rel;     // last relative residual computed
  int32_t last_round;  // round of last_rel (-1: none)
  int32_t pad;
  double prev_rel;     // the relative residual checked before last_rel
  int32_t prev_round;  // round of prev_rel (-1: none)
  int32_t pad2;
};
// The status of a solve that has not begun: no round checked, nothing done.
__device__ __forceinline__ void reset_status_dev(DevStatus* st) {
  st->done = 0;
  st->conv_round = -1;
  st->error = 0;
  st->ticket = 0;
  st->last_rel = -1.0;
  st->last_round = -1;
  st->pad = 0;
  st->prev_rel = -1.0;
  st->prev_round = -1;
  st->pad2 = 0;
}
constexpr int32_t kErrNonfinite = 1;
constexpr int32_t kErrDiverged = 2;

enum SweepMode : int {
  kJoint = 0,   // P and h messages (Alg. 2 message update)
  kHOnly = 1,   // h messages with frozen precisions (coefficient per slot)
  kAgg = 2,     // node aggregates only: x (and P~) of the current messages
  kFreeze = 3,  // aggregates + freeze: g_s = -a_s / (P~_i - P_ji), 1 / P~_i
  kResid = 4    // residual check only
};

// Arguments of one sweep launch.  T is the message precision.
template <typename T>
struct SweepArgs {
  const int32_t* blk_row;  // [nblk+1] first row of each workgroup
  const int32_t* off_ptr;  // [n+1] off-diagonal CSR row pointers
  const int32_t* off_col;  // [E]
  const int32_t* rev;      // [E] slot of the reverse edge
  const T* a;              // [E] A_ij of slot s = (i, j)
  const T* diag;           // [n] P_ii (possibly loaded)
  const T* rhs;            // [n] right-hand side
  const void* min;         // messages of the previous round (pair or h only)
  void* mout;              // messages of this round
  const T* gcoef;          // [E] frozen coefficient (kHOnly)
  const T* inv_pt;         // [n] frozen 1 / P~ (kHOnly)
  T* gcoef_out;            // kFreeze outputs
  T* inv_pt_out;
  T* xout;                 // [n] x of round t-1 (nullable)
  T* ptout;                // [n] P~ of round t-1 (nullable)
  const T* xchk;           // [n] x of round t-2 (checked)
  double* partials;        // [nblk] per-workgroup sums of squared residuals
  DevStatus* st;
  const double* rhs_norm;  // device scalar ||rhs||_2
  double tol;
  int32_t nblk;
  int32_t round_checked;   // round index of xchk
  int32_t zero_in;         // previous messages are all zero (first sweep)
  int32_t check;           // compute the residual of xchk
};

// Arguments of one node-broadcast sweep launch (bcast.hip).
template <typename T>
struct BcastArgs {
  const int32_t* blk_row;
  const int32_t* off_ptr;
  const int32_t* col;      // [E] neighbour of each slot
  const T* a;              // [E] A_ji of slot (j, i)
  const T* diag;           // [n] P_ii (possibly loaded)
  const T* rhs;            // [n]
  void* state;             // [E] per-slot message pairs, updated in place
  const void* aold;        // [n] aggregates of round t-1 ({P~, h~}, or h~ with frozen precisions)
  void* anew;              // [n] aggregates of round t
  const T* xold;           // [n] means of round t-1 (frozen precisions / residual-only launches)
  const void* coef;        // [E] frozen {g_in, g_out}
  void* coef_out;          // freeze output
  const T* inv_pt;         // [n] frozen 1 / P~
  T* inv_pt_out;           // freeze output
  T* xout;                 // [n] means of round t
  T* xout_prev;            // [n] first sweep only: means of round 0
  T* ptout;                // [n] P~ of round t (nullable)
  T* ptout_prev;           // [n] first sweep only: P~ of round 0 (nullable)
  double* partials;
  DevStatus* st;
  int32_t nblk;
  int32_t zero_in;
  int32_t check;
  int32_t honly_nodes;     // residual-only launch after frozen-precision sweeps
};

// The local row index of each of a row's slots, s_row[lo .. hi) = row.  The
// bounds are passed in registers: read from LDS inside the loop, they would be
// reloaded after every byte store (the stores might alias them).
__device__ __forceinline__ void fill_row_ids(uint8_t* s_row, int lo, int hi, int row) {
  for (int j = lo; j < hi; ++j) s_row[j] = (uint8_t)row;
}

// Row sums over a lane's slots in LDS, added in slot order (the rounding of
// the plain loop) with the loads of eight slots issued ahead of their
// additions: a lane summing a row of hundreds of slots otherwise waits out
// one LDS round trip per slot.
template <typename Acc, typename V>
__device__ __forceinline__ Acc lds_row_sum(Acc acc, const V* s, int lo, int hi) {
  int j = lo;
  for (; j + 8 <= hi; j += 8) {
    V v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = s[j + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (Acc)v[u];
  }
  for (; j < hi; ++j) acc += (Acc)s[j];
  return acc;
}
// The same for acc - s[lo] - s[lo + 1] - ...
template <typename Acc, typename V>
__device__ __forceinline__ Acc lds_row_sub(Acc acc, const V* s, int lo, int hi) {
  int j = lo;
  for (; j + 8 <= hi; j += 8) {
    V v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = s[j + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc -= (Acc)v[u];
  }
  for (; j < hi; ++j) acc -= (Acc)s[j];
  return acc;
}

// A row with more slots than one workgroup takes (256 K) is swept in chunks
// of 256 K slots, one workgroup each, launched after the partition's
// workgroups; a finish kernel then adds the chunks' partial row sums in a
// fixed order.  The partition's own workgroup of such a row does nothing.
struct LongRow {
  int32_t row, blk;    // the row, and the partition workgroup that holds it
  int32_t e0, ne;      // its slots
  int32_t cbase, nch;  // its chunks: partial-sum records cbase .. cbase + nch - 1
};
struct ChunkRef {
  int32_t li, c;       // long row, chunk of it
};

// Arguments of one compact node-broadcast sweep launch (compact.hip).
template <typename T>
struct CnodeArgs {
  const int32_t* blk_row;
  const int32_t* blk_e0;   // [nblk+1] first slot of each workgroup
  const int32_t* off_ptr;
  const int32_t* col;      // [E] neighbour of each slot
  const T* a;              // [E] A_ji of slot (j, i)
  const T* diag;           // [n] P_ii (possibly loaded)
  const T* rhs;            // [n]
  void* cin;               // [E] incoming messages: round t-2 on entry, round t on exit (freeze: round T)
  const void* cin_old;     // [E] freeze only: incoming messages of round T-1
  const void* agg2;        // [n] aggregates of round t-2 (freeze: T-1)
  const void* agg1;        // [n] aggregates of round t-1 (freeze: T)
  void* anew;              // [n] aggregates of round t
  const void* coef;        // [E] frozen {g_in, g_out}
  void* coef_out;          // freeze output
  const T* inv_pt;         // [n] frozen 1 / P~
  T* inv_pt_out;           // freeze output
  T* xout;                 // [n] means of round t
  T* xout_prev;            // [n] first sweep only: means of round 0
  T* ptout;                // [n] P~ of round t (nullable)
  T* ptout_prev;           // [n] first sweep only: P~ of round 0 (nullable)
  const T* chk_diag;       // [n] diagonal of the checked system (nullptr: diag)
  T damp;                  // feedback step s
  int32_t feedback;        // single-loop correction: prior h^(t) = rhs + (diag - chk_diag)
                           //   ((1 - s) x^(t-2) + s x^(t-1)), joint sweeps only
  double* partials;
  DevStatus* st;
  const LongRow* longs;    // [nlong] rows swept in chunks (nullable)
  const ChunkRef* xch;     // [nxch] chunk workgroups, launched after the nblk partition workgroups
  double* lpart;           // [chunks][4] partial row sums of the chunks
  int32_t nlong, nxch;
  int32_t nblk;
  int32_t first;           // t == 1 (freeze: T == 0): no outgoing message yet
  int32_t second;          // t == 2 (freeze: T == 1): the incoming messages of round t-2 are zero
                           // (round 0's aggregate record is the prior, written before sweep 1)
  int32_t check;
  int32_t honly_nodes;     // residual-only launch after frozen-precision sweeps
};

// Arguments of one colour-serial launch (serial.hip): the rows of one colour
// class, updated in place.
template <typename T>
struct SerialArgs {
  const int32_t* blk_row;
  const int32_t* blk_e0;
  const int32_t* off_ptr;
  const int32_t* col;      // [E] neighbour of each slot (colour-ordered numbering)
  const T* a;              // [E] A_ji of slot (j, i)
  const T* diag;           // [n] P_ii (possibly loaded)
  const T* rhs;            // [n]
  void* out;               // [E] {P, h} of the message j -> i sent at j's last update
  void* agg;               // [n] {P~, h~} of each node's last update
  double* lsum;            // [n] residual part of the earlier classes (read: check, written: wl)
  T* xout;                 // [n] means of this sweep (nullable)
  T* ptout;                // [n] P~ of this sweep (nullable)
  double* partials;        // [all workgroups] squared residual sums
  DevStatus* st;
  const LongRow* longs;    // rows swept in chunks (nullable)
  const ChunkRef* xch;     // chunk workgroups of all classes
  double* lpart;           // [chunks][4] partial sums of the chunks
  int32_t xch0, nxch;      // this launch's chunk workgroups: xch[xch0 .. xch0 + nxch)
  int32_t blk0;            // first workgroup of the class
  int32_t nblk;            // workgroups of the class
  int32_t lo, hi;          // rows of the class
  int32_t first;           // sweep 1: later classes have sent nothing yet
  int32_t check;           // residual of the previous sweep's means
  int32_t wl;              // store the earlier classes' residual part for the next sweep
};

// One-workgroup solve of a small system (small.hip): the whole synchronous
// iteration in one launch of kSmallLanes lanes, for n <= kSmallLanes rows and
// at most 4 kSmallLanes directed slots.
constexpr int kSmallLanes = 1024;
struct SmallArgs {
  int32_t n;
  int32_t E;
  const int32_t* off_ptr;   // [n+1] off-diagonal CSR
  const int32_t* col;       // [E]
  const double* a;          // [E]
  const double* diag;       // [n]
  const double* rhs;        // [n]
  const double* rhs_norm;   // device scalar ||rhs||_2 (nullable: formed in the kernel)
  double tol;               // <= 0: exactly max_iter sweeps
  int32_t max_iter;
  int32_t check_every;
  DevStatus* st;            // written once, at the end (as the finish kernels leave it)
  double* xout[2];          // nullable: x of the returned round into [round & 1]
  double* ptout[2];         // nullable: P~ of the returned round into [round & 1]
  double* x_direct;         // nullable: x of the returned round
  double* var_direct;       // nullable: 1 / P~ of the returned round
  void* cin_out;            // nullable: [2][E] {P, h} incoming messages by round parity
  void* agg_out[3];         // nullable: [n] {P~, h~} aggregates by round mod 3
  const int32_t* gate;      // nullable: nonzero -> the kernel returns at once
  const int32_t* E_dev;     // nullable: E read on the device (then E is ignored)
  int32_t max_deg;          // largest row of the off-diagonal CSR (0: not known on the host)
};
bool small_fits(int64_t n, int64_t E);
// rows of at most 6 slots: a lane per row, any E
bool small_rows_fit(int64_t n, int32_t max_deg);
hipError_t launch_small(const SmallArgs& a, hipStream_t s);
// the same with K = 4 slots per lane (E <= 4096, also when E lives on the device)
hipError_t launch_small_k4(const SmallArgs& a, hipStream_t s);

constexpr int kLayoutEdge = 1;     // outgoing message records + reverse-slot index
constexpr int kLayoutNode = 2;     // node broadcast: aggregates published, edge pairs kept in place
constexpr int kLayoutCompact = 3;  // node broadcast, one incoming message per slot, outgoing recomputed
constexpr int kLayoutSerial = 4;   // serial scheduling over colour classes, rows stored in colour order
inline bool node_family(int layout) { return layout == kLayoutNode || layout == kLayoutCompact; }

// Everything a handle owns.  Device arrays are suffixed _d.
struct Ctx {
  int32_t n = 0;
  int64_t E = 0;
  int32_t nnz = 0;
  hipStream_t stream = nullptr;
  gabp_opts opts{};
  int32_t max_degree = 0;
  int64_t device_bytes = 0;
  std::vector<void*> allocs;
  std::vector<int64_t> alloc_sizes;

  // caller's full CSR (kept for the gradient assembly)
  int32_t* row_ptr_d = nullptr;
  int32_t* col_d = nullptr;
  // off-diagonal CSR
  int32_t* off_ptr_d = nullptr;
  int32_t* off_col_d = nullptr;
  int32_t* rev_d = nullptr;
  double* a64_d = nullptr;
  double* d64_d = nullptr;     // A_ii
  float* a32_d = nullptr;
  float* din32_d = nullptr;    // inner diagonal in FP32 (loaded)
  float* d32_d = nullptr;      // A_ii in FP32 (single-loop inner solves with loading)
  double* din64_d = nullptr;   // inner diagonal in FP64 (loaded; == d64 when gamma = 0)
  double gamma_used = 0.0;
  double rho_lo = 0.0, rho_hi = 0.0;  // bounds on rho(|R|) when loading was chosen automatically

  // workgroup partition of the rows
  int32_t K = 0;               // slots per lane
  int32_t nblk = 0;
  int32_t* blk_row_d = nullptr;
  int32_t* blk_e0_d = nullptr;  // first slot of each workgroup (same allocation as blk_row_d)
  int32_t nblk_capacity = 0;
  int32_t partials_capacity = 0;
  // rows longer than one workgroup's slots, swept in chunks (compact and
  // colour-serial layouts)
  std::vector<LongRow> longs_h;
  std::vector<int32_t> long_xch0;  // colour-serial: first chunk workgroup of each class ([ncol + 1])
  LongRow* longs_d = nullptr;
  ChunkRef* xch_d = nullptr;
  double* lpart_d = nullptr;
  int32_t nlong = 0, nxch = 0;
  int32_t longs_capacity = 0, xch_capacity = 0;
  std::vector<int32_t> off_ptr_h;

  // message buffers (double-buffered), frozen precisions
  void* msg_d[2] = {nullptr, nullptr};  // message records [E] (P, h, x) or (h, x)
  void* hmsg_d[2] = {nullptr, nullptr}; // h only [E]
  void* gcoef_d = nullptr;              // [E]
  void* inv_pt_d = nullptr;             // [n]
  bool frozen_valid = false;
  int32_t frozen_prec = -1;
  int last_msg_round = -1;              // round held by msg_d[last_msg_round & 1] (tol <= 0 solves)
  int layout = kLayoutEdge;
  void* bstate_d = nullptr;             // node layout: per-slot message pairs [E]
  void* poison_save_d = nullptr;        // GABP_FLAG_POISON_STALE: one saved slot-state half
                                        // (compact layout: the two incoming-message buffers)
  void* agg_d[3] = {nullptr, nullptr, nullptr};  // published aggregates [n]: by round parity (node
                                                 // layout), by round mod 3 (compact layout)

  // node vectors
  double* x64_d[2] = {nullptr, nullptr};  // x of rounds (plain) / inner FP64 iterates
  double* xo_d[2] = {nullptr, nullptr};   // outer iterates
  double* pt64_d[2] = {nullptr, nullptr};
  float* x32_d[2] = {nullptr, nullptr};
  float* rin32_d = nullptr;               // inner right-hand side (FP32)
  double* rin64_d = nullptr;              // inner right-hand side (FP64 inner)
  double* partials_d = nullptr;
  double* norms_d = nullptr;              // [4]: ||b||, ||r_outer||, spare
  DevStatus* st_d = nullptr;              // [2]: inner / outer
  DevStatus* st_h = nullptr;              // pinned host mirror [4]
  DevStatus* st_small_h = nullptr;        // pinned, coherent: written by the one-launch solve itself
  DevStatus* st_small_d = nullptr;        // ... its device address
  // pinned, coherent: copies of the device status written by finish kernels
  // (two slots for the chunks of a compact run, one for the outer step), so
  // the host reads them without a copy launch
  DevStatus* st_mir_h = nullptr;
  DevStatus* st_mir_d = nullptr;          // ... their device address
  DevStatus run_seen{};                   // status the last sweep loop's poller observed
  bool run_seen_final = false;            // ... and it was final (done set, nothing runs after)
  hipEvent_t ev[2] = {nullptr, nullptr};
  // GABP_FLAG_TIME_SWEEPS: event pairs attached to main-mode checking sweeps
  std::vector<hipEvent_t> tev;
  int tev_used = 0;
  double sweep_ms = 0.0;
  int timed_sweeps = 0;
  int timed_mode = 0;

  // colour-serial layout: rows renumbered so that each colour class is a
  // contiguous range; the caller's order is restored at the C ABI
  int32_t ncol = 0;
  std::vector<int32_t> colour_start;  // [ncol+1] first row of each class
  std::vector<int32_t> cls_row;       // per system: first row of each class, then the system's end
  std::vector<int32_t> cls_base;      // [systems + 1] start of each system's list in cls_row
  std::vector<int32_t> colour_blk;    // [ncol+1] first workgroup of each class
  std::vector<int32_t> colour_h;      // [n] colour of each caller row
  int32_t* slot_of_d = nullptr;       // [E] caller slot of each internal slot (XCD order only)
  double* msg_tmp_d = nullptr;        // [2E] exported messages in internal slot order (XCD order only)
  int32_t aug_n = -1, aug_m = 0;      // augmented handle: x and z block sizes (-1: not one)
  double* aug_rhs_d = nullptr;        // [n] right-hand side {b, h} of an augmented solve
  double* aug_x_d = nullptr;          // [n] its solution {x, z}
  double* ait_y_d = nullptr;          // [n] Aitken estimate (GABP_FLAG_AITKEN)
  double* ait_hist_d = nullptr;       // [n] x_{t-2} for the next Aitken step
  int32_t nparts = 0;                 // XCD order: parts per group (8), else 0
  std::vector<int32_t> part_start;    // XCD order: first row of every part of every group, then n
                                      // (one group; colour-serial: one group per colour class)
  int32_t* perm_d = nullptr;          // [n] caller row -> internal row, then [n] internal -> caller
  int32_t* inv_d = nullptr;
  double* bperm_d = nullptr;          // right-hand side, x and variances in internal order
  double* xperm_d = nullptr;
  double* vperm_d = nullptr;
  double* lsum_d = nullptr;           // [n] residual part of the earlier classes

  // batched
  bool batched = false;
  void* batch = nullptr;

  std::string err;
};

// ---- helpers ---------------------------------------------------------------
gabp_status fail(Ctx* c, gabp_status s, const std::string& msg);
gabp_status hip_fail(Ctx* c, hipError_t e, const char* what);
#define GABP_HIP(ctx, call)                                   \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return gabp::hip_fail((ctx), e_, #call); \
  } while (0)

gabp_status dev_alloc(Ctx* c, void** p, size_t bytes);

// ---- ingest (ingest.hip) ---------------------------------------------------
gabp_status ingest(Ctx* c, const int32_t* row_ptr, const int32_t* col, const double* vals,
                   const int32_t* sys_row_off_d, int32_t num_sys);
gabp_status build_partition(const Ctx* c, int K, std::vector<int32_t>& blk_row);
gabp_status set_long_rows(Ctx* c, int K, const std::vector<int32_t>& br);
void plan_long_rows(const std::vector<int32_t>& op, const std::vector<int32_t>& br, int32_t nb, int K,
                    std::vector<LongRow>& lr, std::vector<ChunkRef>& xc, std::vector<int32_t>& xch_of_blk);
gabp_status set_partition(Ctx* c, int K);
// host part of set_partition: workgroup starts (then n) and, with XCD parts,
// the first workgroup of every group of parts (then the count)
void build_blocks(const Ctx* c, int K, std::vector<int32_t>& blk_row, std::vector<int32_t>& group_blk);
// first workgroup of every colour class, then the count (colour-serial)
std::vector<int32_t> class_blocks(const Ctx* c, const std::vector<int32_t>& blk_row,
                                  const std::vector<int32_t>& group_blk);
// colour.hip: first-fit colouring in row order and the colour-ordered
// renumbering of the off-diagonal CSR (colour-serial layout)
gabp_status apply_colour_order(Ctx* c, const int32_t* sys_row_off, int32_t num_sys);  // host offsets, nullable
// host part: colours, class (and XCD part) ranges and perm_inv from the
// caller's off-diagonal pattern (c->off_ptr_h, col)
void plan_colour_order(Ctx* c, const std::vector<int32_t>& col, const int32_t* sys_row_off, int32_t num_sys,
                       std::vector<int32_t>& perm_inv);
std::vector<int32_t> permuted_ptr(const std::vector<int32_t>& op, const std::vector<int32_t>& perm_inv, int32_t n);
// renumber the rows of the off-diagonal CSR: perm_inv = [perm | inv] (caller row
// -> internal row, internal -> caller); keep_slots keeps the caller slot of every
// internal slot and the reverse-slot index
gabp_status permute_rows(Ctx* c, const std::vector<int32_t>& perm_inv, bool keep_slots);
// partition.hip: XCD-aware row order (8 slot-balanced parts, part x on XCD x).
// xcd_parts fills part[caller row] and says whether the parts pay off.
bool xcd_parts(const Ctx* c, const std::vector<int32_t>& col, std::vector<int32_t>& part);
// time_slabs cuts every part into kTimeSlabs slabs of equal work (slab[caller row]).
constexpr int kTimeSlabs = 8;
std::vector<int32_t> time_slabs(const Ctx* c, const std::vector<int32_t>& col, const std::vector<int32_t>& part);
bool plan_xcd_order(Ctx* c, const std::vector<int32_t>& col, std::vector<int32_t>& perm_inv);
gabp_status apply_xcd_order(Ctx* c);

// ---- kernels (sweep.hip) ---------------------------------------------------
template <typename T>
hipError_t launch_sweep(int mode, int K, const SweepArgs<T>& a, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
size_t sweep_lds_bytes(int K, int elt, bool joint);
size_t msg_bytes(int elt, bool joint);  // bytes of one message record
hipError_t launch_reset_status(DevStatus* st, int count, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
// All-ones words over [p, p + bytes) unless st->done is set (bytes a multiple of 4).
hipError_t launch_poison(void* p, size_t bytes, const DevStatus* st, hipStream_t s);
hipError_t launch_norm(const double* v, int64_t n, double* partials, int nparts, double* out,
                       DevStatus* st, hipStream_t s);
hipError_t launch_copy_round(const double* const* x2, const double* const* pt2, const DevStatus* st,
                             int32_t fallback_round, double* x, double* var, int32_t n,
                             hipStream_t s);
// x of the returned round (the converged one, else fallback_round) of a
// compact run from its aggregate record, as the sweep forms it: h~ / P~, or
// h~ * (1 / P~) with frozen precisions.  agg: the three rotating FP64
// aggregate buffers, [n] {P~ or 1 / P~, h~} each.
hipError_t launch_x_from_agg(void* const* agg, bool honly, const DevStatus* st, int32_t fallback_round, double* x,
                             int32_t n, hipStream_t s);
// outer correction step: x_new = x_old + d (d from the inner solve, FP32 or FP64
// selected on the device by the inner status), r = b - A x_new in FP64, r_in =
// r in the inner precision, ||r|| and the check against tol.
struct OuterArgs {
  const int32_t* blk_row;
  const int32_t* off_ptr;
  const int32_t* off_col;
  const double* a;
  const double* diag;
  const double* b;
  const double* xold;     // nullable (x = 0)
  double* xnew;
  const float* d32[2];    // inner iterates (FP32) by round parity
  const double* d64[2];   // inner iterates (FP64) by round parity
  // or, when dagg_elt is 4 (FP32) or 8 (FP64): the inner compact run's
  // aggregate records by round mod 3, {P~, h~} (d = h~ / P~) or with frozen
  // precisions {1 / P~, h~} (d = h~ * (1 / P~)), as the sweep forms means
  const void* dagg[3];
  int32_t dagg_elt;
  int32_t dagg_honly;
  const DevStatus* st_in; // selects the inner round
  int32_t in_fallback;    // inner round when the inner solve did not converge
  int32_t use_d;          // 0: no correction (x_new = x_old)
  float* rin32;
  double* rin64;
  double* partials;
  DevStatus* st;          // outer status
  const double* b_norm;
  double* r_norm;         // output ||r||
  double tol;
  int32_t nblk;
  int32_t n;
  const DevStatus* gate;  // nullable: the launch returns at once once gate->done is set
  int32_t reset_st;       // launch_outer: the first kernel resets *st before the step's finish
  DevStatus* mirror;      // nullable: the step's finish also writes *st there (host memory)
};
hipError_t launch_outer(int K, const OuterArgs& a, hipStream_t s);
hipError_t launch_outer_only(int K, const OuterArgs& a, hipStream_t s);
hipError_t launch_check_finish(const double* partials, int nblk, DevStatus* st, const double* rhs_norm,
                               double tol, int round, double* norm_out, bool gate_on_done, hipStream_t s,
                               double diverge_limit = kDivergeLimit, DevStatus* mirror = nullptr);
// Aitken step after the sweep of round t (Ch. 3 Sec. 3.2): with make_y,
// y = hist - (x1 - hist)^2 / (x2 - 2 x1 + hist), or x2 where undefined; then
// hist = x1.  x1 and x2 are the means of rounds t-1 and t, hist those of
// round t-2.  Returns at once once the status is done.
hipError_t launch_aitken(const double* x1, const double* x2, double* hist, double* y, const DevStatus* st,
                         int make_y, int32_t n, hipStream_t s);
// Steffensen step at the end of a cycle (round t even, Ch. 3 Sec. 3.2): y =
// aitken(start, x1, x2) with the same formula and fallback as launch_aitken;
// then start = y, x2 = y and the round-t aggregate record {P~, h~} becomes
// {P~, P~ y}.  Returns at once once the status is done.
hipError_t launch_steffensen(const double* x1, double* x2, double* start, void* agg, const DevStatus* st,
                             int32_t n, hipStream_t s);
hipError_t launch_grad_vals(const int32_t* row_ptr, const int32_t* col, const double* lam,
                            const double* x, double* gv, int32_t n, hipStream_t s);
hipError_t launch_scale_diag(const double* d, double f, double* out64, float* out32, int32_t n,
                             hipStream_t s);
hipError_t launch_split_pairs(const void* m, double* P, double* h, int64_t E, hipStream_t s);
template <typename T>
hipError_t launch_bcast(int mode, int K, const BcastArgs<T>& a, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
hipError_t launch_split_out(const void* state, double* P, double* h, int64_t E, hipStream_t s);
template <typename T>
hipError_t launch_cnode(int mode, int K, const CnodeArgs<T>& a, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
hipError_t launch_cnode_out(int32_t n, const int32_t* off_ptr, const double* a, const void* in_prev,
                            const void* agg_prev, bool zero_in, double* P, double* h, hipStream_t s);
size_t cnode_lds_bytes(int K, int elt);
template <typename T>
hipError_t launch_cnode_prior(int32_t n, const T* first, const T* rhs, void* out, hipStream_t s,
                              DevStatus* reset = nullptr);
template <typename T>
hipError_t launch_serial(const SerialArgs<T>& a, int K, bool resid, hipStream_t s);
template <typename T>
hipError_t launch_serial_prior_x(int32_t n, const T* diag, const T* rhs, T* x, T* pt, hipStream_t s);
size_t serial_lds_bytes(int K, int elt);
hipError_t launch_gather(const double* src, const int32_t* idx, double* dst, int32_t n, hipStream_t s);
hipError_t launch_scatter_slots(const double* src, const int32_t* idx, double* dst, int64_t E, hipStream_t s);
size_t bcast_state_bytes(int elt);
size_t bcast_coef_bytes(int elt);
size_t bcast_lds_bytes(int K, int elt);
void dev_free(Ctx* c, void* p);

// ---- drivers (solve.hip) ---------------------------------------------------
gabp_status solve_plain(Ctx* c, const double* b, double* x, double* var, double tol,
                        int32_t max_iter, gabp_info* info, bool allow_reuse);
gabp_status solve_outer(Ctx* c, const double* b, double* x, double tol, int32_t max_iter,
                        gabp_info* info);
gabp_status solve_single_loop(Ctx* c, const double* b, double* x, double tol, int32_t max_iter,
                              gabp_info* info);
gabp_status autotune(Ctx* c);
gabp_status estimate_walk_rho(Ctx* c, double* lo, double* hi, int max_iter, double rtol);

// ---- batched (batched.hip) -------------------------------------------------
gabp_status batched_create(Ctx* c, int32_t num_sys, const int32_t* sys_row_off);
gabp_status batched_solve(Ctx* c, const int32_t* nrhs, const int64_t* rhs_off, const double* B,
                          double* X, double tol, int32_t max_iter, gabp_info* infos);
void batched_destroy(Ctx* c);
gabp_status batched_profile(Ctx* c, gabp_batch_profile* out);

}  // namespace gabp

// The opaque handle type of the C ABI.
struct gabp_ctx : public gabp::Ctx {};
