// Colour classes for serial scheduling (Ch. 2 Sec. 2.3).
//
// Nodes of one class are pairwise non-adjacent, so a class can be updated at
// once, and a sweep over the classes in turn is a serial schedule.  The
// colouring is first fit in row order: node i takes the smallest colour
// that none of its neighbours j < i holds.  That is a sequential O(E) pass on
// the host over the already validated off-diagonal pattern.  The
// off-diagonal CSR is then renumbered on the device so that each class is a
// contiguous row range, rows kept in increasing caller order inside a class
// (for a single system with XCD parts: inside a class's part and time slab).
// For a batch of independent systems, first fit in global row order colours
// every system on its own (no edge crosses a system), and the renumbering
// stays inside each system's row block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "gabp_internal.h"

namespace gabp {

namespace {

#define GABP_TRY_STATUS(x)          \
  do {                              \
    gabp_status s_ = (x);           \
    if (s_ != GABP_OK) return s_;   \
  } while (0)

// One lane per new row p: copy the slots of caller row inv[p], with the
// columns renumbered (the slot order inside the row is kept), and record the
// caller's slot of every new slot (nullable).
__global__ void k_permute_rows(int32_t n, const int32_t* __restrict__ inv, const int32_t* __restrict__ perm,
                               const int32_t* __restrict__ old_ptr, const int32_t* __restrict__ old_col,
                               const double* __restrict__ old_a64, const float* __restrict__ old_a32,
                               const double* __restrict__ old_d64, const int32_t* __restrict__ new_ptr,
                               int32_t* __restrict__ new_col, double* __restrict__ new_a64,
                               float* __restrict__ new_a32, double* __restrict__ new_d64,
                               int32_t* __restrict__ slot_of) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const int32_t r = inv[p];
    int32_t k = new_ptr[p];
    for (int32_t s = old_ptr[r]; s < old_ptr[r + 1]; ++s, ++k) {
      new_col[k] = perm[old_col[s]];
      new_a64[k] = old_a64[s];
      new_a32[k] = old_a32[s];
      if (slot_of) slot_of[k] = s;
    }
    new_d64[p] = old_d64[r];
  }
}

// old2new[slot_of[k]] = k
__global__ void k_invert_slots(int64_t E, const int32_t* __restrict__ slot_of, int32_t* __restrict__ old2new) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < E; k += (int64_t)gridDim.x * blockDim.x)
    old2new[slot_of[k]] = (int32_t)k;
}

// reverse-slot index in the new numbering
__global__ void k_remap_rev(int64_t E, const int32_t* __restrict__ slot_of, const int32_t* __restrict__ old2new,
                            const int32_t* __restrict__ old_rev, int32_t* __restrict__ new_rev) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < E; k += (int64_t)gridDim.x * blockDim.x)
    new_rev[k] = old2new[old_rev[slot_of[k]]];
}

}  // namespace

std::vector<int32_t> permuted_ptr(const std::vector<int32_t>& op, const std::vector<int32_t>& perm_inv, int32_t n) {
  std::vector<int32_t> new_ptr((size_t)n + 1, 0);
  for (int32_t p = 0; p < n; ++p) {
    const int32_t r = perm_inv[n + p];
    new_ptr[p + 1] = new_ptr[p] + (op[r + 1] - op[r]);
  }
  return new_ptr;
}

gabp_status permute_rows(Ctx* c, const std::vector<int32_t>& perm_inv, bool keep_slots) {
  hipStream_t s = c->stream;
  const int32_t n = c->n;
  const int64_t E = c->E;
  std::vector<int32_t> new_ptr = permuted_ptr(c->off_ptr_h, perm_inv, n);
  void* pi = nullptr;
  GABP_TRY_STATUS(dev_alloc(c, &pi, sizeof(int32_t) * 2 * (size_t)n));
  c->perm_d = (int32_t*)pi;
  c->inv_d = c->perm_d + n;
  int32_t* nptr_d = nullptr;
  int32_t* ncol_d = nullptr;
  double* na64_d = nullptr;
  float* na32_d = nullptr;
  double* nd64_d = nullptr;
  GABP_TRY_STATUS(dev_alloc(c, (void**)&nptr_d, sizeof(int32_t) * ((size_t)n + 1)));
  GABP_TRY_STATUS(dev_alloc(c, (void**)&ncol_d, sizeof(int32_t) * (size_t)E));
  GABP_TRY_STATUS(dev_alloc(c, (void**)&na64_d, sizeof(double) * (size_t)E));
  GABP_TRY_STATUS(dev_alloc(c, (void**)&na32_d, sizeof(float) * (size_t)E));
  GABP_TRY_STATUS(dev_alloc(c, (void**)&nd64_d, sizeof(double) * (size_t)n));
  if (keep_slots) GABP_TRY_STATUS(dev_alloc(c, (void**)&c->slot_of_d, sizeof(int32_t) * (size_t)E));
  GABP_HIP(c, hipMemcpyAsync(c->perm_d, perm_inv.data(), sizeof(int32_t) * 2 * (size_t)n, hipMemcpyHostToDevice, s));
  GABP_HIP(c, hipMemcpyAsync(nptr_d, new_ptr.data(), sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s));
  if (n > 0) {
    hipLaunchKernelGGL(k_permute_rows, dim3(std::min((n + 255) / 256, 4096)), dim3(256), 0, s, n, c->inv_d,
                       c->perm_d, c->off_ptr_d, c->off_col_d, c->a64_d, c->a32_d, c->d64_d, nptr_d, ncol_d, na64_d,
                       na32_d, nd64_d, c->slot_of_d);
    GABP_HIP(c, hipGetLastError());
  }
  int32_t* nrev_d = nullptr;
  if (keep_slots && E > 0) {  // the reverse-slot index follows the slots
    int32_t* old2new_d = nullptr;
    GABP_TRY_STATUS(dev_alloc(c, (void**)&old2new_d, sizeof(int32_t) * (size_t)E));
    GABP_TRY_STATUS(dev_alloc(c, (void**)&nrev_d, sizeof(int32_t) * (size_t)E));
    const int blocks = (int)std::min<int64_t>((E + 255) / 256, 8192);
    hipLaunchKernelGGL(k_invert_slots, dim3(blocks), dim3(256), 0, s, E, c->slot_of_d, old2new_d);
    GABP_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(k_remap_rev, dim3(blocks), dim3(256), 0, s, E, c->slot_of_d, old2new_d, c->rev_d, nrev_d);
    GABP_HIP(c, hipGetLastError());
    GABP_HIP(c, hipStreamSynchronize(s));
    dev_free(c, old2new_d);
  }
  GABP_HIP(c, hipStreamSynchronize(s));
  dev_free(c, c->off_ptr_d);
  dev_free(c, c->off_col_d);
  dev_free(c, c->a64_d);
  dev_free(c, c->a32_d);
  dev_free(c, c->d64_d);
  dev_free(c, c->rev_d);
  c->rev_d = nrev_d;
  c->off_ptr_d = nptr_d;
  c->off_col_d = ncol_d;
  c->a64_d = na64_d;
  c->a32_d = na32_d;
  c->d64_d = nd64_d;
  c->off_ptr_h = std::move(new_ptr);
  return GABP_OK;
}

void plan_colour_order(Ctx* c, const std::vector<int32_t>& col, const int32_t* sys_row_off, int32_t num_sys,
                       std::vector<int32_t>& perm_inv) {
  const int32_t n = c->n;
  const std::vector<int32_t>& op = c->off_ptr_h;

  // first fit in row order
  std::vector<int32_t>& colour = c->colour_h;
  colour.assign(n, 0);
  std::vector<int32_t> stamp((size_t)c->max_degree + 2, -1);
  int32_t ncol = n > 0 ? 1 : 0;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t e = op[i]; e < op[i + 1]; ++e) {
      const int32_t j = col[e];
      if (j < i) stamp[colour[j]] = i;
    }
    int32_t k = 0;
    while (stamp[k] == i) ++k;
    colour[i] = k;
    ncol = std::max(ncol, k + 1);
  }

  // a single system may also split every class by XCD part, and each part's
  // rows by time slab (the order inside a class does not change the
  // iteration)
  std::vector<int32_t> part;
  const bool parts = !sys_row_off && !(c->opts.flags & GABP_FLAG_NATURAL_ORDER) && xcd_parts(c, col, part);
  const std::vector<int32_t> slab = parts ? time_slabs(c, col, part) : std::vector<int32_t>();

  // classes as contiguous ranges inside each system, caller order inside a
  // class (inside a class's part and slab with XCD parts); cls_row lists every
  // system's class starts (global rows) followed by its end, cls_base[s]
  // where system s's list begins
  c->ncol = ncol;
  const int32_t S = sys_row_off ? num_sys : 1;
  c->cls_base.assign(S + 1, 0);
  c->cls_row.clear();
  perm_inv.assign(2 * (size_t)n, 0);  // [perm | inv]
  for (int32_t q = 0; q < S; ++q) {
    const int32_t r0 = sys_row_off ? sys_row_off[q] : 0, r1 = sys_row_off ? sys_row_off[q + 1] : n;
    int32_t nc = r1 > r0 ? 1 : 0;
    for (int32_t i = r0; i < r1; ++i) nc = std::max(nc, colour[i] + 1);
    std::vector<int32_t> start(nc + 1, 0);
    for (int32_t i = r0; i < r1; ++i) ++start[colour[i] + 1];
    std::partial_sum(start.begin(), start.end(), start.begin());
    c->cls_base[q] = (int32_t)c->cls_row.size();
    for (int32_t k = 0; k <= nc; ++k) c->cls_row.push_back(r0 + start[k]);
    if (parts) {  // (class, part) sub-ranges, 8 per class
      const int np = 8;
      std::vector<int32_t> sub((size_t)nc * np + 1, 0);
      for (int32_t i = r0; i < r1; ++i) ++sub[(size_t)colour[i] * np + part[i] + 1];
      std::partial_sum(sub.begin(), sub.end(), sub.begin());
      c->nparts = np;
      c->part_start.assign(sub.size(), 0);
      for (size_t k = 0; k < sub.size(); ++k) c->part_start[k] = r0 + sub[k];
      // inside a (class, part) range, the rows slab by slab (time slabs, as
      // in the synchronous XCD order), caller order inside a slab
      const int ns = kTimeSlabs;
      std::vector<int32_t> cell((size_t)nc * np * ns + 1, 0);
      for (int32_t i = r0; i < r1; ++i) ++cell[((size_t)colour[i] * np + part[i]) * ns + slab[i] + 1];
      std::partial_sum(cell.begin(), cell.end(), cell.begin());
      for (int32_t i = r0; i < r1; ++i) {
        const int32_t p = r0 + cell[((size_t)colour[i] * np + part[i]) * ns + slab[i]]++;
        perm_inv[i] = p;
        perm_inv[n + p] = i;
      }
      continue;
    }
    std::vector<int32_t> next(start.begin(), start.end() - 1);
    for (int32_t i = r0; i < r1; ++i) {
      const int32_t p = r0 + next[colour[i]]++;
      perm_inv[i] = p;
      perm_inv[n + p] = i;
    }
  }
  c->cls_base[S] = (int32_t)c->cls_row.size();
  if (!sys_row_off) c->colour_start = c->cls_row;
}

gabp_status apply_colour_order(Ctx* c, const int32_t* sys_row_off, int32_t num_sys) {
  hipStream_t s = c->stream;
  std::vector<int32_t> col((size_t)c->E);
  if (c->E > 0)
    GABP_HIP(c, hipMemcpyAsync(col.data(), c->off_col_d, sizeof(int32_t) * c->E, hipMemcpyDeviceToHost, s));
  GABP_HIP(c, hipStreamSynchronize(s));
  std::vector<int32_t> perm_inv;
  plan_colour_order(c, col, sys_row_off, num_sys, perm_inv);
  return permute_rows(c, perm_inv, false);  // the serial sweeps pull through aggregates only
}

}  // namespace gabp
