// Host-side run of the library's graph checks, clique-tree builder, counter and
// planner, and of the CPU oracle, built with the address and undefined-
// behaviour sanitizers (see tests/test_sanitizers.py).  Each case checks a
// property that holds by construction (Lemma 5's clique count against the
// oracle's enumeration, the planner's leaf and member totals, the error
// codes of bad input), so a sanitizer report or a failed check fails the run.
// Test infrastructure only.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/kdss.h"

extern "C" {
int kor_count(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, int k, int threads, uint64_t* lo,
              uint64_t* hi);
int kor_validate(uint32_t n, uint64_t nnz, const uint64_t* row_ptr, const uint32_t* col);
typedef struct {
  uint64_t c_k_lo, c_k_hi;
  uint32_t T, size;
  uint64_t dens_num, ub_num_lo, ub_num_hi;
  double enum_seconds, iter_seconds, extract_seconds;
  int threads, streamed;
} kor_result;
int kor_solve(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, int k, uint32_t T, const uint64_t* r0,
              int threads, uint64_t max_store_bytes, uint64_t* r_lo, uint64_t* r_hi, uint32_t* order,
              kor_result* res, void* trace);
int kor_prefix_counts(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, int k, const uint64_t* r,
                      int threads, uint32_t* order, uint32_t* size, uint64_t* dens, uint64_t* K);
int kor_pb_run(uint32_t n, uint64_t npairs, const uint32_t* h, const uint32_t* p, const uint64_t* off,
               const uint32_t* mem, int k, uint32_t T, int synchronous, uint64_t* r, double* seconds);
}

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

struct Graph {
  uint32_t n = 0;
  std::vector<uint64_t> rp;
  std::vector<uint32_t> col;
  kdss_csr csr() const { return kdss_csr{n, rp.empty() ? 0 : rp.back(), rp.data(), col.data()}; }
};

// Simple undirected graph from an edge predicate on pairs u < v.
template <class F>
static Graph make_graph(uint32_t n, F edge) {
  Graph g;
  g.n = n;
  g.rp.assign(n + 1, 0);
  std::vector<std::vector<uint32_t>> adj(n);
  for (uint32_t u = 0; u < n; ++u)
    for (uint32_t v = u + 1; v < n; ++v)
      if (edge(u, v)) {
        adj[u].push_back(v);
        adj[v].push_back(u);
      }
  for (uint32_t u = 0; u < n; ++u) {
    std::sort(adj[u].begin(), adj[u].end());
    g.rp[u + 1] = g.rp[u] + adj[u].size();
    g.col.insert(g.col.end(), adj[u].begin(), adj[u].end());
  }
  return g;
}

static uint64_t mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static void tree_case(const Graph& g, uint32_t k) {
  kdss_csr c = g.csr();
  kdss_sct* t = nullptr;
  CHECK(kdss_sct_build(&c, k, 3, &t) == KDSS_OK);
  kdss_tree_stats st{}, sc{};
  CHECK(kdss_sct_info(t, &st) == KDSS_OK);
  CHECK(kdss_sct_count(&c, k, 2, &sc) == KDSS_OK);
  CHECK(st.leaves == sc.leaves && st.members == sc.members && st.c_k.lo == sc.c_k.lo && st.s_max == sc.s_max);
  uint64_t lo = 0, hi = 0;
  CHECK(kor_count(g.n, g.rp.data(), g.col.data(), (int)k, 2, &lo, &hi) == 0);
  CHECK(st.c_k.lo == lo && st.c_k.hi == hi);
  std::vector<uint32_t> h(st.leaves + 1), p(st.leaves + 1), m(st.members + 1), core(g.n + 1);
  CHECK(kdss_sct_export(t, h.data(), p.data(), m.data(), st.leaves, st.members) == KDSS_OK);
  CHECK(kdss_sct_export(t, h.data(), p.data(), m.data(), st.leaves ? st.leaves - 1 : 0, st.members) ==
        (st.leaves ? KDSS_ERANGE : KDSS_OK));
  CHECK(kdss_sct_core_numbers(t, core.data(), g.n) == KDSS_OK);
  if (g.n > 0) {
    // a single plan, a batch of the tree twice, the workspace query
    kdss_plan* pl = nullptr;
    CHECK(kdss_plan_create(t, 20, 7, nullptr, &pl) == KDSS_OK);
    kdss_plan_stats ps{};
    CHECK(kdss_plan_info(pl, &ps) == KDSS_OK);
    uint64_t L = 0, M = 0;
    for (int q = 0; q < 5; ++q) {
      L += ps.leaves[q];
      M += ps.members[q];
    }
    CHECK(L == st.leaves && M == st.members);
    size_t ws = 0;
    CHECK(kdss_workspace_size(t, 20, 7, nullptr, &ws) == KDSS_OK && ws == ps.workspace_bytes);
    kdss_plan_free(pl);
    const kdss_sct* two[2] = {t, t};
    kdss_plan* b = nullptr;
    kdss_opts o{};
    o.schedule = 2;
    CHECK(kdss_batch_create(two, 2, 10, 0, &o, &b) == KDSS_OK);
    std::vector<uint64_t> off(3);
    CHECK(kdss_batch_offsets(b, off.data(), 2) == KDSS_OK && off[2] == 2ull * g.n);
    kdss_batch_free(b);
    // the one-shot call sizes its buffers without a device
    size_t need = 0;
    kdss_result res{};
    CHECK(kdss_solve(&c, k, 9, nullptr, nullptr, 0, nullptr, 0, &need, nullptr, 0, nullptr, &res, nullptr) ==
          KDSS_EWORKSPACE);
    CHECK(need > 0 && res.n == g.n);
  }
  kdss_sct_free(t);
  // the oracle's run, prefix counts and PBUpdate passes on the same graph
  std::vector<uint64_t> rlo(g.n + 1), rhi(g.n + 1), K(g.n + 1);
  std::vector<uint32_t> order(g.n + 1);
  kor_result r{};
  CHECK(kor_solve(g.n, g.rp.data(), g.col.data(), (int)k, 6, nullptr, 2, 1ull << 30, rlo.data(), rhi.data(),
                  order.data(), &r, nullptr) == 0);
  uint32_t size = 0;
  uint64_t dens = 0;
  CHECK(kor_prefix_counts(g.n, g.rp.data(), g.col.data(), (int)k, rlo.data(), 2, order.data(), &size, &dens,
                          K.data()) == 0);
  CHECK(g.n == 0 || K[g.n - 1] == lo);
  CHECK(size == r.size && dens == r.dens_num);
}

int main() {
  // bad input: the library and the oracle refuse the same graphs
  {
    const uint64_t rp[] = {0, 1, 3, 5, 6};
    const uint32_t bad_cols[][6] = {{1, 2, 0, 1, 3, 2}, {1, 0, 2, 2, 3, 2}, {1, 0, 2, 1, 9, 2}};
    for (const auto& cl : bad_cols) {
      kdss_csr c{4, 6, rp, cl};
      CHECK(kdss_csr_validate(&c) == KDSS_EGRAPH);
      CHECK(kor_validate(4, 6, rp, cl) != 0);
      kdss_sct* t = nullptr;
      CHECK(kdss_sct_build(&c, 3, 1, &t) == KDSS_EGRAPH && t == nullptr);
    }
    const uint32_t good[] = {1, 0, 2, 1, 3, 2};
    kdss_csr c{4, 6, rp, good};
    CHECK(kdss_csr_validate(&c) == KDSS_OK);
    kdss_sct* t = nullptr;
    CHECK(kdss_sct_build(&c, 1, 1, &t) == KDSS_EINVAL);
    CHECK(kdss_sct_build(&c, 32, 1, &t) == KDSS_ERANGE);
    CHECK(kdss_sct_build(nullptr, 3, 1, &t) == KDSS_EINVAL);
    kdss_sct_free(nullptr);
    kdss_plan_free(nullptr);
  }
  // graphs: empty, complete, random with a planted clique, a denser one
  tree_case(make_graph(0, [](uint32_t, uint32_t) { return true; }), 3);
  tree_case(make_graph(7, [](uint32_t, uint32_t) { return false; }), 2);
  for (uint32_t k = 2; k <= 6; ++k) tree_case(make_graph(9, [](uint32_t, uint32_t) { return true; }), k);
  for (uint64_t seed = 0; seed < 6; ++seed) {
    const uint32_t n = 40 + 30 * (uint32_t)seed;
    const double p = 0.08 + 0.04 * (double)(seed % 3);
    Graph g = make_graph(n, [&](uint32_t u, uint32_t v) {
      if (u < 14 && v < 14) return true;   // a planted 14-clique
      return (double)(mix(seed * 1000003ull + (uint64_t)u * n + v) >> 11) * 0x1p-53 < p;
    });
    for (uint32_t k : {3u, 4u, 5u, 7u}) tree_case(g, k);
  }
  // PBUpdate over pairs with h = k and pivots (Lemma 4)
  {
    const uint32_t h[] = {3, 1}, p[] = {2, 3};
    const uint64_t off[] = {0, 5, 9};
    const uint32_t mem[] = {0, 1, 2, 3, 4, 5, 0, 1, 2};
    std::vector<uint64_t> r(6, 0);
    double secs = 0;
    CHECK(kor_pb_run(6, 2, h, p, off, mem, 3, 4, 1, r.data(), &secs) == 0);
    uint64_t tot = 0;
    for (uint64_t x : r) tot += x;
    CHECK(tot == 4 * (1 + 3));
  }
  std::printf("%s (%d failed checks)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
