// Drives the library's host-side planning code -- the row plan of
// gabp_plan_rows (first-fit colouring, XCD parts, row order, workgroup
// partition, long-row chunks) and the augmented assembly of
// gabp_plan_augmented -- on valid and malformed inputs, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code.  No GPU
// call is made.  Exits 0 when every status is the expected one; a sanitizer
// report ends the process with its own error.
#include <cstdint>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "gabp.h"

namespace {

struct Csr {
  int32_t n = 0;
  std::vector<int32_t> rp, col;
};

// Full symmetric pattern (diagonal stored) from undirected pairs.
Csr from_pairs(int32_t n, const std::vector<std::pair<int32_t, int32_t>>& pairs) {
  std::vector<std::set<int32_t>> adj(n);
  for (int32_t i = 0; i < n; ++i) adj[i].insert(i);
  for (auto [u, v] : pairs)
    if (u != v) {
      adj[u].insert(v);
      adj[v].insert(u);
    }
  Csr c;
  c.n = n;
  c.rp.push_back(0);
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t j : adj[i]) c.col.push_back(j);
    c.rp.push_back((int32_t)c.col.size());
  }
  return c;
}

Csr grid(int32_t px, int32_t py) {
  std::vector<std::pair<int32_t, int32_t>> p;
  for (int32_t i = 0; i < px; ++i)
    for (int32_t j = 0; j < py; ++j) {
      if (i + 1 < px) p.push_back({i * py + j, (i + 1) * py + j});
      if (j + 1 < py) p.push_back({i * py + j, i * py + j + 1});
    }
  return from_pairs(px * py, p);
}

Csr random_graph(int32_t n, int32_t m, uint32_t seed, bool hubs) {
  std::mt19937 g(seed);
  std::vector<std::pair<int32_t, int32_t>> p;
  std::uniform_int_distribution<int32_t> u(0, n - 1);
  for (int32_t k = 0; k < m; ++k) {
    int32_t a = u(g), b = u(g);
    if (hubs && (k % 3 == 0)) a = (int32_t)(g() % 4);  // a few rows with thousands of slots
    p.push_back({a, b});
  }
  return from_pairs(n, p);
}

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s\n", what);
    ++failures;
  }
}

void plan(const Csr& c, int layout, int flags, int epb, gabp_status want, const char* what) {
  gabp_opts o;
  gabp_default_opts(&o);
  o.layout = layout;
  o.flags = flags;
  o.edges_per_block = epb;
  const int32_t n = c.n;
  std::vector<int32_t> perm(n + 1), colour(n + 1), cls(n + 2);
  const int32_t cap = 8 * n + 16;
  std::vector<int32_t> blk(cap);
  gabp_plan pl{};
  const gabp_status st = gabp_plan_rows(n, c.rp.data(), c.col.data(), &o, perm.data(), colour.data(), blk.data(),
                                        cap, cls.data(), &pl);
  expect(st == want, what);
  if (st == GABP_OK && n > 0) {
    // the plan is a permutation and the workgroups cover the rows in order
    std::vector<int32_t> seen(n, 0);
    for (int32_t i = 0; i < n; ++i) {
      expect(perm[i] >= 0 && perm[i] < n, "perm in range");
      if (perm[i] >= 0 && perm[i] < n) ++seen[perm[i]];
    }
    for (int32_t i = 0; i < n; ++i) expect(seen[i] == 1, "perm is a permutation");
    expect(blk[0] == 0 && blk[pl.num_blocks] == n, "blocks cover the rows");
    for (int32_t b = 0; b < pl.num_blocks; ++b) expect(blk[b] <= blk[b + 1], "blocks in order");
  }
  // too little room for the workgroup table
  if (st == GABP_OK && n > 0) {
    const gabp_status s2 = gabp_plan_rows(n, c.rp.data(), c.col.data(), &o, nullptr, nullptr, blk.data(),
                                          pl.num_blocks, nullptr, nullptr);
    expect(s2 == GABP_E_ARG, "blk_cap below num_blocks + 1");
  }
}

void augmented(uint32_t seed, int32_t m, int32_t n, int per_row) {
  std::mt19937 g(seed);
  std::vector<int32_t> bp{0}, bc;
  std::vector<double> bv;
  for (int32_t r = 0; r < m; ++r) {
    std::set<int32_t> cs;
    while ((int)cs.size() < std::min(per_row, n)) cs.insert((int32_t)(g() % n));
    for (int32_t c : cs) {
      bc.push_back(c);
      bv.push_back(std::normal_distribution<double>(0.0, 1.0)(g));
    }
    bp.push_back((int32_t)bc.size());
  }
  std::vector<double> d(n, 1.0);
  int64_t nnz = 0;
  gabp_status st = gabp_plan_augmented(m, n, bp.data(), bc.data(), bv.data(), d.data(), 0.5, nullptr, nullptr,
                                       nullptr, 0, &nnz);
  expect(st == GABP_OK && nnz == n + m + 2 * (int64_t)bc.size(), "augmented size");
  std::vector<int32_t> Krp(n + m + 1), Kcol(nnz);
  std::vector<double> Kval(nnz);
  st = gabp_plan_augmented(m, n, bp.data(), bc.data(), bv.data(), d.data(), 0.5, Krp.data(), Kcol.data(),
                           Kval.data(), nnz, &nnz);
  expect(st == GABP_OK, "augmented assembly");
  for (int32_t r = 0; r < n + m; ++r)
    for (int32_t e = Krp[r] + 1; e < Krp[r + 1]; ++e) expect(Kcol[e] > Kcol[e - 1], "K columns increase");
  // room for one entry less
  st = gabp_plan_augmented(m, n, bp.data(), bc.data(), bv.data(), d.data(), 0.5, Krp.data(), Kcol.data(),
                           Kval.data(), nnz - 1, nullptr);
  expect(st == GABP_E_ARG, "augmented cap too small");
  // malformed inputs
  if (!bc.empty()) {
    std::vector<int32_t> bad = bc;
    bad[0] = n;  // column out of range
    st = gabp_plan_augmented(m, n, bp.data(), bad.data(), bv.data(), d.data(), 0.5, nullptr, nullptr, nullptr, 0,
                             nullptr);
    expect(st == GABP_E_ARG, "augmented column out of range");
  }
  std::vector<double> d0 = d;
  d0[0] = 0.0;
  st = gabp_plan_augmented(m, n, bp.data(), bc.data(), bv.data(), d0.data(), 0.5, nullptr, nullptr, nullptr, 0,
                           nullptr);
  expect(st == GABP_E_ARG, "augmented zero d");
  st = gabp_plan_augmented(m, n, bp.data(), bc.data(), bv.data(), d.data(), -1.0, nullptr, nullptr, nullptr, 0,
                           nullptr);
  expect(st == GABP_E_ARG, "augmented gamma <= 0");
  std::vector<int32_t> bpd = bp;
  if (m >= 2) {
    bpd[1] = bp[2] + 1;  // decreasing row pointers
    st = gabp_plan_augmented(m, n, bpd.data(), bc.data(), bv.data(), d.data(), 0.5, nullptr, nullptr, nullptr, 0,
                             nullptr);
    expect(st == GABP_E_ARG, "augmented decreasing row_ptr");
  }
}

}  // namespace

int main() {
  const Csr cases[] = {grid(32, 32), grid(1, 1), grid(3, 7), random_graph(5000, 20000, 1, false),
                       random_graph(20000, 80000, 2, true), random_graph(300, 2000, 3, true)};
  for (const Csr& c : cases)
    for (int layout : {0, 1, 2, 3, 4})
      for (int flags : {0, GABP_FLAG_NATURAL_ORDER})
        for (int epb : {0, 512, 2048}) plan(c, layout, flags, epb, GABP_OK, "valid pattern");
  Csr empty;
  empty.rp = {0};
  plan(empty, 0, 0, 0, GABP_OK, "empty pattern");
  // malformed patterns: unsorted columns, a missing diagonal, a column out of
  // range, decreasing row pointers
  Csr g = grid(4, 4);
  Csr bad = g;
  std::swap(bad.col[1], bad.col[2]);
  plan(bad, 0, 0, 0, GABP_E_ARG, "unsorted columns");
  bad = g;
  bad.col[g.rp[3]] = 99;
  plan(bad, 4, 0, 0, GABP_E_ARG, "column out of range");
  Csr nodiag;
  nodiag.n = 2;
  nodiag.rp = {0, 1, 2};
  nodiag.col = {1, 0};
  plan(nodiag, 0, 0, 0, GABP_E_ZERO_DIAG, "missing diagonal");
  bad = g;
  bad.rp[2] = bad.rp[1] - 1;
  plan(bad, 0, 0, 0, GABP_E_ARG, "decreasing row pointers");
  for (uint32_t s = 0; s < 4; ++s) augmented(s, 50 + 37 * s, 20 + 11 * s, 1 + (int)s);
  augmented(9, 1, 1, 1);
  std::printf("%s: %d failure(s)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
