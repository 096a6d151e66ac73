// XCD-aware row order.
//
// The chip's eight XCDs each have their own L2.  A sweep gathers neighbour
// aggregates at random.  When the rows one XCD processes have many of their
// neighbours among themselves, those gathers stay in that XCD's L2.  So at
// create time:
//   1. The nodes are split into 8 parts of equal work (slots + rows; a long
//      row, swept in chunks spread over all XCDs, counts as a row).  The
//      parts are grown breadth-first from 8 seeds, then refined by label
//      propagation: a node moves to the part holding most of its neighbours,
//      within a 2% balance margin, until a pass moves fewer than 0.1% of
//      the nodes.
//   2. The rows are renumbered part by part.
//   3. The workgroup partition pads every part to the same number of
//      workgroups, so the XCD-aware workgroup map sends part x to XCD x.
// The iteration is unchanged: every row keeps its slots, in order.  Only the
// numbering differs, and the C ABI restores the caller's order.  The order is
// used only when its parts hold clearly more of the edges (25 points) than 8
// contiguous ranges of the caller's own order do (on a naturally ordered grid
// they hold nearly all).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <vector>

#include "gabp_internal.h"

namespace gabp {

namespace {

constexpr int kParts = 8;          // XCDs
constexpr double kBalance = 0.02;  // allowed deviation of a part's work from the mean
constexpr int kRefine = 8;         // label-propagation passes
constexpr int64_t kMinSlots = 4096;
// required rise of the fraction of edges inside the parts: measured, parts
// holding 43% of G(n, 4n)'s edges (31 points above 8 ranges of the caller's
// order) shorten the sweep by 11%, while the 28-34% a power-law graph reaches
// make it slower than the caller's order
constexpr double kMinGain = 0.25;
constexpr int64_t kLongRow = 2 * kBlock;  // slots of the smallest workgroup budget

double inside_fraction(const std::vector<int32_t>& op, const std::vector<int32_t>& col,
                       const std::vector<int32_t>& part) {
  int64_t in = 0, all = 0;
  const int32_t n = (int32_t)part.size();
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = op[i]; e < op[i + 1]; ++e) {
      in += part[col[e]] == part[i];
      ++all;
    }
  return all ? (double)in / (double)all : 1.0;
}

}  // namespace

bool xcd_parts(const Ctx* c, const std::vector<int32_t>& col, std::vector<int32_t>& part) {
  const int32_t n = c->n;
  const int64_t E = c->E;
  if (E < kMinSlots || n < 4 * kParts) return false;
  const std::vector<int32_t>& op = c->off_ptr_h;

  // work of a row: its slots and itself; a row longer than the smallest
  // workgroup budget is swept by chunk workgroups spread over every XCD, so
  // it weighs as one row in its part
  std::vector<int64_t> w(n);
  int64_t total = 0;
  for (int32_t i = 0; i < n; ++i) {
    const int64_t d = op[i + 1] - op[i];
    total += (w[i] = (d > kLongRow ? 0 : d) + 1);
  }
  const double target = (double)total / kParts;

  // the caller's order cut into 8 ranges of equal work
  std::vector<int32_t> natural(n);
  {
    int64_t acc = 0;
    for (int32_t i = 0; i < n; ++i) {
      natural[i] = std::min(kParts - 1, (int)((double)acc / target));
      acc += w[i];
    }
  }

  // 1. breadth-first growth, the parts taking turns; a part whose frontier
  //    runs dry restarts at the lowest unassigned node
  part.assign(n, -1);
  std::vector<int64_t> load(kParts, 0);
  std::vector<std::deque<int32_t>> front(kParts);
  int32_t scan = 0;
  auto next_free = [&]() -> int32_t {
    while (scan < n && part[scan] >= 0) ++scan;
    return scan < n ? scan : -1;
  };
  for (int p = 0; p < kParts; ++p) {
    const int32_t seed = (int32_t)((int64_t)p * n / kParts);
    if (part[seed] < 0) {
      part[seed] = p;
      load[p] += w[seed];
      front[p].push_back(seed);
    }
  }
  int32_t assigned = 0;
  for (int32_t i = 0; i < n; ++i) assigned += part[i] >= 0;
  bool progress = true;
  while (assigned < n && progress) {
    progress = false;
    for (int p = 0; p < kParts && assigned < n; ++p) {
      if ((double)load[p] >= target) continue;
      if (front[p].empty()) {
        const int32_t v = next_free();
        if (v < 0) break;
        part[v] = p;
        load[p] += w[v];
        ++assigned;
        front[p].push_back(v);
        progress = true;
        continue;
      }
      const int32_t v = front[p].front();
      front[p].pop_front();
      for (int32_t e = op[v]; e < op[v + 1] && (double)load[p] < target; ++e) {
        const int32_t u = col[e];
        if (part[u] >= 0) continue;
        part[u] = p;
        load[p] += w[u];
        ++assigned;
        front[p].push_back(u);
      }
      progress = true;
    }
  }
  for (int32_t i = 0; i < n; ++i)  // whatever is left goes to the lightest part
    if (part[i] < 0) {
      const int p = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      part[i] = p;
      load[p] += w[i];
    }

  // 2. label propagation within the balance margin
  const double hi = (1.0 + kBalance) * target, lo = (1.0 - kBalance) * target;
  for (int it = 0; it < kRefine; ++it) {
    int64_t moved = 0;
    for (int32_t v = 0; v < n; ++v) {
      int cnt[kParts] = {0};
      for (int32_t e = op[v]; e < op[v + 1]; ++e) ++cnt[part[col[e]]];
      const int cur = part[v];
      int best = cur;
      for (int p = 0; p < kParts; ++p)
        if (cnt[p] > cnt[best]) best = p;
      if (best != cur && (double)(load[best] + w[v]) <= hi && (double)(load[cur] - w[v]) >= lo) {
        part[v] = best;
        load[best] += w[v];
        load[cur] -= w[v];
        ++moved;
      }
    }
    if (moved * 1000 < n) break;  // settled: fewer than 0.1% of the nodes moved
  }

  return inside_fraction(op, col, part) >= inside_fraction(op, col, natural) + kMinGain;
}

bool plan_xcd_order(Ctx* c, const std::vector<int32_t>& col, std::vector<int32_t>& perm_inv) {
  const int32_t n = c->n;
  std::vector<int32_t> part;
  if (!xcd_parts(c, col, part)) return false;
  // 3. rows part by part, caller order inside a part
  c->nparts = kParts;
  c->part_start.assign(kParts + 1, 0);
  for (int32_t i = 0; i < n; ++i) ++c->part_start[part[i] + 1];
  for (int p = 0; p < kParts; ++p) c->part_start[p + 1] += c->part_start[p];
  perm_inv.assign(2 * (size_t)n, 0);
  std::vector<int32_t> next(c->part_start.begin(), c->part_start.end() - 1);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t p = next[part[i]]++;
    perm_inv[i] = p;
    perm_inv[n + p] = i;
  }
  return true;
}

gabp_status apply_xcd_order(Ctx* c) {
  if (c->E < kMinSlots || c->n < 4 * kParts) return GABP_OK;
  hipStream_t s = c->stream;
  std::vector<int32_t> col((size_t)c->E);
  GABP_HIP(c, hipMemcpyAsync(col.data(), c->off_col_d, sizeof(int32_t) * c->E, hipMemcpyDeviceToHost, s));
  GABP_HIP(c, hipStreamSynchronize(s));
  std::vector<int32_t> perm_inv;
  if (!plan_xcd_order(c, col, perm_inv)) return GABP_OK;
  return permute_rows(c, perm_inv, true);
}

}  // namespace gabp
