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
//   2. Each part is cut into 8 time slabs of equal work.  Workgroups are
//      dispatched in order, so at any moment every XCD sweeps rows of about
//      the same slab, and the aggregates of that slab (of all parts, an
//      eighth of the array) are what its gathers mostly touch: a gather whose
//      neighbour lies in the current slab is likely to find the line in its
//      XCD's L2, brought there by a recent gather of the same XCD, as is one
//      whose neighbour lies in the XCD's own part.  The slabs are grown
//      breadth-first over the whole graph from 8 seeds, a node joining a slab
//      only while its part's share of that slab has room, then refined by
//      two passes of label propagation on the slab label alone (the part is
//      kept).  On G(n, 4n) the slabs hold 43% of the edges, as the parts do,
//      and two thirds of the edges lie inside a part or a slab.
//   3. The rows are renumbered part by part, slab by slab inside a part.
//   4. The workgroup partition pads every part to the same number of
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
constexpr int kSlabs = kTimeSlabs;  // time slabs per part
constexpr int kSlabRefine = 2;     // label-propagation passes on the slabs
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

// 2. time slabs inside the parts (part[] is kept); returns the slab of every node
std::vector<int32_t> time_slabs(const Ctx* c, const std::vector<int32_t>& col, const std::vector<int32_t>& part) {
  const int32_t n = c->n;
  const std::vector<int32_t>& op = c->off_ptr_h;
  // what the growth reads of a neighbour, in one record: one cache miss per
  // visited slot instead of three
  struct Node {
    int32_t part, w, slab, pad;
  };
  std::vector<Node> nd(n);
  std::vector<int64_t> ptot(kParts, 0);
  for (int32_t i = 0; i < n; ++i) {
    const int64_t d = op[i + 1] - op[i];
    nd[i] = Node{part[i], (int32_t)((d > kLongRow ? 0 : d) + 1), -1, 0};
    ptot[part[i]] += nd[i].w;
  }
  // a slab's share of part p: its work may reach cap[p] while growing, and
  // stays within the balance margin around it under refinement
  std::vector<int64_t> cap(kParts);
  for (int p = 0; p < kParts; ++p) cap[p] = ptot[p] / kSlabs + 1;
  std::vector<int64_t> load((size_t)kParts * kSlabs, 0);
  auto fits = [&](const Node& v, int s) { return load[(size_t)v.part * kSlabs + s] + v.w <= cap[v.part]; };
  // one queue per slab (a vector and its read position); a node enters one queue once
  std::vector<std::vector<int32_t>> fifo(kSlabs);
  int32_t assigned = 0;
  auto take = [&](int32_t v, int s) {
    nd[v].slab = s;
    load[(size_t)nd[v].part * kSlabs + s] += nd[v].w;
    ++assigned;
    fifo[s].push_back(v);
  };
  std::vector<size_t> head(kSlabs, 0);
  // seeds between the parts' seeds of the caller's order
  for (int s = 0; s < kSlabs; ++s) {
    const int32_t v = (int32_t)(((int64_t)2 * s + 1) * n / (2 * kSlabs));
    if (nd[v].slab < 0) take(v, s);
  }
  // restart points: a node that a slab skips here never fits it later, since
  // the loads only grow while the slabs grow
  std::vector<int32_t> scan(kSlabs, 0);
  while (assigned < n) {
    bool grew = false;
    for (int s = 0; s < kSlabs; ++s) {
      if (head[s] == fifo[s].size()) continue;
      const int32_t v = fifo[s][head[s]++];
      grew = true;
      for (int32_t e = op[v]; e < op[v + 1]; ++e) {
        const int32_t u = col[e];
        if (nd[u].slab < 0 && fits(nd[u], s)) take(u, s);
      }
    }
    if (grew) continue;
    // every queue ran dry: restart each slab at the lowest node it can take
    bool seeded = false;
    for (int s = 0; s < kSlabs; ++s) {
      int32_t& v = scan[s];
      while (v < n && (nd[v].slab >= 0 || !fits(nd[v], s))) ++v;
      if (v < n) {
        take(v, s);
        seeded = true;
      }
    }
    if (!seeded) break;
  }
  std::vector<int32_t> slab(n);
  for (int32_t i = 0; i < n; ++i) {
    if (nd[i].slab < 0) {  // whatever is left goes to its part's lightest slab
      const int64_t* L = &load[(size_t)nd[i].part * kSlabs];
      int best = 0;
      for (int s = 1; s < kSlabs; ++s)
        if (L[s] < L[best]) best = s;
      nd[i].slab = best;
      load[(size_t)nd[i].part * kSlabs + best] += nd[i].w;
    }
    slab[i] = nd[i].slab;
  }
  // label propagation on the slab label; two passes take nearly all the gain
  for (int it = 0; it < kSlabRefine; ++it) {
    int64_t moved = 0;
    for (int32_t v = 0; v < n; ++v) {
      int cnt[kSlabs] = {0};
      for (int32_t e = op[v]; e < op[v + 1]; ++e) ++cnt[slab[col[e]]];
      const int cur = slab[v];
      int best = cur;
      for (int s = 0; s < kSlabs; ++s)
        if (cnt[s] > cnt[best]) best = s;
      int64_t* L = &load[(size_t)nd[v].part * kSlabs];
      const double cp = (double)cap[nd[v].part];
      if (best != cur && (double)(L[best] + nd[v].w) <= (1.0 + kBalance) * cp &&
          (double)(L[cur] - nd[v].w) >= (1.0 - kBalance) * cp) {
        slab[v] = best;
        L[best] += nd[v].w;
        L[cur] -= nd[v].w;
        ++moved;
      }
    }
    if (moved * 1000 < n) break;
  }
  return slab;
}

bool plan_xcd_order(Ctx* c, const std::vector<int32_t>& col, std::vector<int32_t>& perm_inv) {
  const int32_t n = c->n;
  std::vector<int32_t> part;
  if (!xcd_parts(c, col, part)) return false;
  const std::vector<int32_t> slab = time_slabs(c, col, part);
  // 3. rows part by part, slab by slab inside a part, caller order inside a slab
  c->nparts = kParts;
  c->part_start.assign(kParts + 1, 0);
  std::vector<int32_t> cell((size_t)kParts * kSlabs + 1, 0);
  for (int32_t i = 0; i < n; ++i) {
    ++c->part_start[part[i] + 1];
    ++cell[(size_t)part[i] * kSlabs + slab[i] + 1];
  }
  for (int p = 0; p < kParts; ++p) c->part_start[p + 1] += c->part_start[p];
  for (size_t k = 0; k + 1 < cell.size(); ++k) cell[k + 1] += cell[k];
  perm_inv.assign(2 * (size_t)n, 0);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t p = cell[(size_t)part[i] * kSlabs + slab[i]]++;
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
