// CSR ingest: validation, diagonal split, reverse-slot index, workgroup partition.
//
// Alg. 2 starts from the neighbourhood N(i) (the nonzeros of row i, diagonal
// excluded) and the priors P_ii = A_ii.  Here that becomes an off-diagonal CSR
// whose slot s = (i, j) holds the message i -> j, plus rev[s] = the slot of
// (j, i), which the broadcast update subtracts (Alg. 2, P_ij = -A_ij^2 /
// (P~_i - P_ji)).
#include <algorithm>
#include <cmath>

#include "gabp_internal.h"

namespace gabp {

namespace {

constexpr int kFlagArg = 1;
constexpr int kFlagZeroDiag = 2;
constexpr int kFlagAsym = 4;
constexpr int kFlagNonfinite = 8;

struct IngestScratch {
  int32_t flags;
  int32_t max_degree;
  unsigned long long maxabs_bits;  // |A| max as IEEE bits (nonnegative doubles order as integers)
};

// One lane per row: structure checks, diagonal, off-diagonal row pointers.
__global__ void k_validate_rows(int32_t n, int32_t nnz, const int32_t* __restrict__ row_ptr,
                                const int32_t* __restrict__ col, const double* __restrict__ vals,
                                const int32_t* __restrict__ row_lo,  // nullable: first col allowed
                                const int32_t* __restrict__ row_hi,  // nullable: one past last col
                                double* __restrict__ diag, int32_t* __restrict__ off_ptr,
                                IngestScratch* sc) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int32_t lo = row_ptr[r], hi = row_ptr[r + 1];
  int flags = 0;
  if (lo < 0 || hi > nnz || hi < lo) {  // never read outside col/vals
    flags |= kFlagArg;
    lo = hi = 0;
  }
  const int32_t cmin = row_lo ? row_lo[r] : 0;
  const int32_t cmax = row_hi ? row_hi[r] : n;
  int32_t prev = -1;
  int ndiag = 0;
  double dv = 0.0, maxabs = 0.0;
  for (int32_t e = lo; e < hi; ++e) {
    const int32_t c = col[e];
    const double v = vals[e];
    if (c < cmin || c >= cmax || c <= prev) flags |= kFlagArg;
    prev = c;
    if (!isfinite(v)) flags |= kFlagNonfinite;
    if (c == r) {
      ++ndiag;
      dv = v;
    }
    maxabs = fmax(maxabs, fabs(v));
  }
  if (ndiag != 1 || dv == 0.0) flags |= kFlagZeroDiag;
  diag[r] = dv;
  off_ptr[r] = lo - r;
  if (r == n - 1) off_ptr[n] = hi - n;
  if (flags) atomicOr(&sc->flags, flags);
  if (isfinite(maxabs)) atomicMax(&sc->maxabs_bits, (unsigned long long)__double_as_longlong(maxabs));
  atomicMax(&sc->max_degree, hi - lo - ndiag);
}

__global__ void k_split(int32_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                        const double* __restrict__ vals, const int32_t* __restrict__ off_ptr,
                        int32_t* __restrict__ off_col, double* __restrict__ a64, float* __restrict__ a32) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int32_t k = off_ptr[r];
  for (int32_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
    const int32_t c = col[e];
    if (c == r) continue;
    off_col[k] = c;
    a64[k] = vals[e];
    a32[k] = (float)vals[e];
    ++k;
  }
}

// rev[s] for every slot of row r: binary search for column r in row col[s].
__global__ void k_reverse(int32_t n, const int32_t* __restrict__ off_ptr,
                          const int32_t* __restrict__ off_col, const double* __restrict__ a64,
                          int32_t* __restrict__ rev, IngestScratch* sc) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double tolv = 1e-12 * __longlong_as_double((long long)sc->maxabs_bits);
  int flags = 0;
  for (int32_t s = off_ptr[r]; s < off_ptr[r + 1]; ++s) {
    const int32_t c = off_col[s];
    int32_t lo = off_ptr[c], hi = off_ptr[c + 1] - 1, found = -1;
    while (lo <= hi) {
      const int32_t mid = (lo + hi) >> 1;
      const int32_t v = off_col[mid];
      if (v == r) {
        found = mid;
        break;
      }
      if (v < r) lo = mid + 1;
      else hi = mid - 1;
    }
    if (found < 0) {
      flags |= kFlagAsym;
      rev[s] = s;  // keeps every later gather in bounds
      continue;
    }
    rev[s] = found;
    if (fabs(a64[s] - a64[found]) > tolv) flags |= kFlagAsym;
  }
  if (flags) atomicOr(&sc->flags, flags);
}

__global__ void k_fill_rows_of_system(int32_t num_sys, const int32_t* __restrict__ sys_row_off,
                                      int32_t* __restrict__ row_lo, int32_t* __restrict__ row_hi) {
  const int32_t s = blockIdx.x;
  if (s >= num_sys) return;
  const int32_t lo = sys_row_off[s], hi = sys_row_off[s + 1];
  for (int32_t r = lo + threadIdx.x; r < hi; r += blockDim.x) {
    row_lo[r] = lo;
    row_hi[r] = hi;
  }
}

}  // namespace

gabp_status dev_alloc(Ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(c, GABP_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  c->allocs.push_back(*p);
  c->alloc_sizes.push_back((int64_t)bytes);
  c->device_bytes += (int64_t)bytes;
  return GABP_OK;
}

void dev_free(Ctx* c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c->allocs.size(); ++i)
    if (c->allocs[i] == p) {
      (void)hipFree(p);
      c->device_bytes -= c->alloc_sizes[i];
      c->allocs.erase(c->allocs.begin() + i);
      c->alloc_sizes.erase(c->alloc_sizes.begin() + i);
      return;
    }
}

#define GABP_TRY(x)                   \
  do {                                \
    gabp_status s_ = (x);             \
    if (s_ != GABP_OK) return s_;     \
  } while (0)

gabp_status ingest(Ctx* c, const int32_t* row_ptr, const int32_t* col, const double* vals,
                   const int32_t* sys_row_off_d, int32_t num_sys) {
  hipStream_t s = c->stream;
  const int32_t n = c->n;
  int32_t bounds[2] = {0, 0};
  GABP_HIP(c, hipMemcpyAsync(&bounds[0], row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GABP_HIP(c, hipMemcpyAsync(&bounds[1], row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GABP_HIP(c, hipStreamSynchronize(s));
  if (bounds[0] != 0 || bounds[1] < n)
    return fail(c, GABP_E_ARG, "row_ptr[0] must be 0 and row_ptr[n] >= n (diagonal stored)");
  c->nnz = bounds[1];
  c->E = (int64_t)c->nnz - n;

  GABP_TRY(dev_alloc(c, (void**)&c->row_ptr_d, sizeof(int32_t) * (n + 1)));
  GABP_TRY(dev_alloc(c, (void**)&c->col_d, sizeof(int32_t) * c->nnz));
  GABP_HIP(c, hipMemcpyAsync(c->row_ptr_d, row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
  GABP_HIP(c, hipMemcpyAsync(c->col_d, col, sizeof(int32_t) * c->nnz, hipMemcpyDeviceToDevice, s));

  GABP_TRY(dev_alloc(c, (void**)&c->off_ptr_d, sizeof(int32_t) * (n + 1)));
  GABP_TRY(dev_alloc(c, (void**)&c->d64_d, sizeof(double) * n));
  GABP_TRY(dev_alloc(c, (void**)&c->off_col_d, sizeof(int32_t) * c->E));
  GABP_TRY(dev_alloc(c, (void**)&c->rev_d, sizeof(int32_t) * c->E));
  GABP_TRY(dev_alloc(c, (void**)&c->a64_d, sizeof(double) * c->E));
  GABP_TRY(dev_alloc(c, (void**)&c->a32_d, sizeof(float) * c->E));

  IngestScratch* sc = nullptr;
  GABP_TRY(dev_alloc(c, (void**)&sc, sizeof(IngestScratch)));
  GABP_HIP(c, hipMemsetAsync(sc, 0, sizeof(IngestScratch), s));

  int32_t* row_lo = nullptr;
  int32_t* row_hi = nullptr;
  const int threads = 256;
  const int blocks = (n + threads - 1) / threads;
  if (sys_row_off_d != nullptr && num_sys > 0) {
    // rows of system s may only reference columns of system s
    GABP_TRY(dev_alloc(c, (void**)&row_lo, sizeof(int32_t) * n));
    GABP_TRY(dev_alloc(c, (void**)&row_hi, sizeof(int32_t) * n));
    hipLaunchKernelGGL(k_fill_rows_of_system, dim3(num_sys), dim3(256), 0, s, num_sys, sys_row_off_d,
                       row_lo, row_hi);
    GABP_HIP(c, hipGetLastError());
  }
  hipLaunchKernelGGL(k_validate_rows, dim3(blocks), dim3(threads), 0, s, n, c->nnz, row_ptr, col, vals,
                     row_lo, row_hi, c->d64_d, c->off_ptr_d, sc);
  GABP_HIP(c, hipGetLastError());
  IngestScratch h{};
  GABP_HIP(c, hipMemcpyAsync(&h, sc, sizeof(h), hipMemcpyDeviceToHost, s));
  GABP_HIP(c, hipStreamSynchronize(s));
  if (h.flags & kFlagArg)
    return fail(c, GABP_E_ARG, "CSR structure: row pointers decrease, columns unsorted/duplicated or out of range");
  if (h.flags & kFlagNonfinite) return fail(c, GABP_E_NONFINITE, "non-finite matrix value");
  if (h.flags & kFlagZeroDiag) return fail(c, GABP_E_ZERO_DIAG, "a diagonal entry is missing or zero");
  c->max_degree = h.max_degree;

  if (c->E > 0) {
    hipLaunchKernelGGL(k_split, dim3(blocks), dim3(threads), 0, s, n, row_ptr, col, vals,
                       c->off_ptr_d, c->off_col_d, c->a64_d, c->a32_d);
    GABP_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(k_reverse, dim3(blocks), dim3(threads), 0, s, n, c->off_ptr_d, c->off_col_d,
                       c->a64_d, c->rev_d, sc);
    GABP_HIP(c, hipGetLastError());
    GABP_HIP(c, hipMemcpyAsync(&h, sc, sizeof(h), hipMemcpyDeviceToHost, s));
    GABP_HIP(c, hipStreamSynchronize(s));
    if (h.flags & kFlagAsym) return fail(c, GABP_E_NOT_SYMMETRIC, "pattern or values of A are not symmetric");
  }

  c->off_ptr_h.resize(n + 1);
  GABP_HIP(c, hipMemcpyAsync(c->off_ptr_h.data(), c->off_ptr_d, sizeof(int32_t) * (n + 1),
                             hipMemcpyDeviceToHost, s));
  GABP_HIP(c, hipStreamSynchronize(s));
  return GABP_OK;
}

// Greedy packing of whole rows into workgroups of at most 256*K slots and 256
// rows; a row longer than 256*K gets a workgroup of its own (the edge and node
// sweeps loop over it; the compact and colour-serial sweeps split it into the
// chunk workgroups of set_long_rows).  With colour classes or XCD parts, no
// workgroup spans two of them.
gabp_status build_partition(const Ctx* c, int K, std::vector<int32_t>& blk_row) {
  const int64_t cap = (int64_t)kBlock * K;
  blk_row.clear();
  blk_row.push_back(0);
  int64_t slots = 0;
  int32_t rows = 0;
  const auto& op = c->off_ptr_h;
  const std::vector<int32_t>& breaks = c->nparts > 0 ? c->part_start : c->colour_start;
  size_t next_class = 1;  // index into breaks of the next boundary
  for (int32_t r = 0; r < c->n; ++r) {
    const int64_t d = op[r + 1] - op[r];
    bool boundary = false;
    while (next_class < breaks.size() && breaks[next_class] <= r) {
      boundary = boundary || breaks[next_class] == r;
      ++next_class;
    }
    if (rows > 0 && (boundary || slots + d > cap || rows == kMaxRowsPerBlock)) {
      blk_row.push_back(r);
      slots = 0;
      rows = 0;
    }
    slots += d;
    ++rows;
    if (d > cap) {  // close a long row's workgroup at once
      blk_row.push_back(r + 1);
      slots = 0;
      rows = 0;
    }
  }
  if (blk_row.back() != c->n) blk_row.push_back(c->n);
  return GABP_OK;
}

void build_blocks(const Ctx* c, int K, std::vector<int32_t>& br, std::vector<int32_t>& group_blk) {
  build_partition(c, K, br);
  group_blk.clear();
  if (c->nparts > 0) {
    // XCD parts: inside a group (the whole matrix, or one colour class), every
    // part gets the same number of workgroups, the short ones padded with
    // empty workgroups at the part's end, so that the XCD-aware workgroup map
    // of a launch over the group sends part x to XCD x
    const size_t nsub = c->part_start.size() - 1;
    const int np = c->nparts;
    std::vector<int32_t> cnt(nsub, 0);
    for (size_t i = 0; i + 1 < br.size(); ++i) {
      const size_t p = (size_t)(std::upper_bound(c->part_start.begin(), c->part_start.end(), br[i]) -
                                c->part_start.begin()) - 1;
      ++cnt[p];
    }
    std::vector<int32_t> padded;
    size_t i = 0;
    for (size_t g = 0; g * np < nsub; ++g) {
      group_blk.push_back((int32_t)padded.size());
      const int32_t q = *std::max_element(cnt.begin() + g * np, cnt.begin() + (g + 1) * np);
      for (size_t p = g * np; p < (g + 1) * np; ++p) {
        for (int32_t k = 0; k < cnt[p]; ++k) padded.push_back(br[i++]);
        for (int32_t k = cnt[p]; k < q; ++k) padded.push_back(c->part_start[p + 1]);
      }
    }
    group_blk.push_back((int32_t)padded.size());
    padded.push_back(c->n);
    br.swap(padded);
  }
}

std::vector<int32_t> class_blocks(const Ctx* c, const std::vector<int32_t>& br, const std::vector<int32_t>& group_blk) {
  if (c->ncol <= 0) return {};
  if (c->nparts > 0) return group_blk;  // a colour class is a group of XCD parts
  const int32_t nb = (int32_t)br.size() - 1;
  std::vector<int32_t> out(c->ncol + 1, nb);
  for (int32_t k = c->ncol - 1; k >= 0; --k)
    out[k] = (int32_t)(std::lower_bound(br.begin(), br.begin() + nb + 1, c->colour_start[k]) - br.begin());
  return out;
}

gabp_status set_partition(Ctx* c, int K) {
  std::vector<int32_t> br, group_blk;  // XCD parts: first workgroup of every group of parts
  build_blocks(c, K, br, group_blk);
  const int32_t nb = (int32_t)br.size() - 1;
  // what the sweep kernels assume of every workgroup: rows in order covering
  // 0..n, at most 256 rows, at most 256 K slots unless it is one long row
  bool ok = nb >= 1 && br[0] == 0 && br[nb] == c->n;
  for (int32_t i = 0; ok && i < nb; ++i) {
    const int32_t rows = br[i + 1] - br[i];
    const int64_t slots = (int64_t)c->off_ptr_h[br[i + 1]] - c->off_ptr_h[br[i]];
    ok = rows >= 0 && rows <= kMaxRowsPerBlock && (slots <= (int64_t)kBlock * K || rows == 1);
  }
  if (!ok) return fail(c, GABP_E_ARG, "internal: invalid workgroup partition");
  std::vector<int32_t> cls_blk = class_blocks(c, br, group_blk);  // before br is extended below
  // first rows, then first slots, of the workgroups: [2 (nb + 1)]
  for (int32_t i = 0; i <= nb; ++i) br.push_back(c->off_ptr_h[br[i]]);
  if (c->blk_row_d == nullptr || nb > c->nblk_capacity) {
    void* p = nullptr;
    GABP_TRY(dev_alloc(c, &p, sizeof(int32_t) * 2 * (nb + 1)));
    c->blk_row_d = (int32_t*)p;
    c->nblk_capacity = nb;
  }
  c->blk_e0_d = c->blk_row_d + (nb + 1);
  GABP_HIP(c, hipMemcpyAsync(c->blk_row_d, br.data(), sizeof(int32_t) * 2 * (nb + 1),
                             hipMemcpyHostToDevice, c->stream));
  GABP_HIP(c, hipStreamSynchronize(c->stream));
  c->K = K;
  c->nblk = nb;
  c->colour_blk.swap(cls_blk);
  if (c->partials_d == nullptr || nb > c->partials_capacity) {
    void* p = nullptr;
    GABP_TRY(dev_alloc(c, &p, sizeof(double) * (nb + 1024)));
    c->partials_d = (double*)p;
    c->partials_capacity = nb;
  }
  return set_long_rows(c, K, br);
}

// The long rows of a partition (more than 256 K slots, a workgroup of their
// own) and their chunk workgroups, in workgroup order, so that the chunks of
// one colour class's long rows are a contiguous range.  br: the first rows of
// the nb + 1 workgroups; op: the off-diagonal row pointers in that order.
// xch_of_blk[i]: chunk workgroups before workgroup i.
void plan_long_rows(const std::vector<int32_t>& op, const std::vector<int32_t>& br, int32_t nb, int K,
                    std::vector<LongRow>& lr, std::vector<ChunkRef>& xc, std::vector<int32_t>& xch_of_blk) {
  const int64_t S = (int64_t)kBlock * K;
  lr.clear();
  xc.clear();
  xch_of_blk.assign((size_t)nb + 1, 0);
  int32_t chunks = 0;
  for (int32_t i = 0; i < nb; ++i) {
    xch_of_blk[i] = (int32_t)xc.size();
    const int32_t e0 = op[br[i]], e1 = op[br[i + 1]];
    if (e1 - e0 <= S) continue;
    LongRow L{br[i], i, e0, e1 - e0, chunks, (int32_t)((e1 - e0 + S - 1) / S)};
    for (int32_t k = 0; k < L.nch; ++k) xc.push_back(ChunkRef{(int32_t)lr.size(), k});
    chunks += L.nch;
    lr.push_back(L);
  }
  xch_of_blk[nb] = (int32_t)xc.size();
}

gabp_status set_long_rows(Ctx* c, int K, const std::vector<int32_t>& br) {
  std::vector<LongRow> lr;
  std::vector<ChunkRef> xc;
  std::vector<int32_t> xch_of_blk;
  plan_long_rows(c->off_ptr_h, br, c->nblk, K, lr, xc, xch_of_blk);
  c->long_xch0.clear();
  for (int32_t b : c->colour_blk) c->long_xch0.push_back(xch_of_blk[b]);
  c->nlong = (int32_t)lr.size();
  c->nxch = (int32_t)xc.size();
  if (!lr.empty()) {
    if (c->longs_d == nullptr || c->nlong > c->longs_capacity) {
      void* p = nullptr;
      GABP_TRY(dev_alloc(c, &p, sizeof(LongRow) * lr.size()));
      c->longs_d = (LongRow*)p;
      c->longs_capacity = c->nlong;
    }
    if (c->xch_d == nullptr || c->nxch > c->xch_capacity) {
      void* p = nullptr;
      GABP_TRY(dev_alloc(c, &p, sizeof(ChunkRef) * xc.size()));
      c->xch_d = (ChunkRef*)p;
      GABP_TRY(dev_alloc(c, &p, 4 * sizeof(double) * xc.size()));
      c->lpart_d = (double*)p;
      c->xch_capacity = c->nxch;
    }
    GABP_HIP(c, hipMemcpyAsync(c->longs_d, lr.data(), sizeof(LongRow) * lr.size(), hipMemcpyHostToDevice,
                               c->stream));
    GABP_HIP(c, hipMemcpyAsync(c->xch_d, xc.data(), sizeof(ChunkRef) * xc.size(), hipMemcpyHostToDevice,
                               c->stream));
    GABP_HIP(c, hipStreamSynchronize(c->stream));
  }
  c->longs_h.swap(lr);
  return GABP_OK;
}

}  // namespace gabp
