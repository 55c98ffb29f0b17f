// Host construction of the k-pruned succinct clique tree (SCT).
//
// The paper uses the SCT as an index of all cliques (Sec. 2, "Succinct Clique
// Tree", Lemma 3): every root-to-leaf path is a pair (H, P) of a hold set and
// a pivot set whose union is a clique, the pair encodes the cliques
// H + C' for every subset C' of P, and the pairs partition all cliques of G.
// For a fixed k only pairs with |H| <= k <= |H| + |P| hold k-cliques
// (Lemma 4), each holding C(|P|, k - |H|) of them (Lemma 5).
//
// The tree itself is the pivoting clique enumeration the paper cites for it:
// nodes are visited in degeneracy order; the subtree of a node v searches its
// later neighbours S.  At a tree node with candidates S, a pivot q in S with
// the most neighbours inside S is chosen; one child adds q to P and keeps
// S & N(q); every other candidate w outside N(q) (in a fixed order w_1, w_2,
// ...) gets a child that adds w to H and keeps S & N(w) minus w_1..w_{i-1}.
// A clique avoiding all the w_i lies in {q} + N(q) and is encoded below the
// pivot child; otherwise its first w_i decides the hold child, so every clique
// is encoded exactly once.  Subtrees that cannot reach k nodes are cut, and a
// hold set that reaches k nodes is emitted at once as the leaf (H, {}), since H
// is its only k-clique.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>

#include "kdss_internal.h"

namespace kdss {

u128 binom128(uint64_t a, uint64_t b) {
  if (b > a) return 0;
  if (b > a - b) b = a - b;
  u128 r = 1;
  const u128 kMax = ~(u128)0;
  for (uint64_t i = 1; i <= b; ++i) {
    // r = r * (a - b + i) / i stays an integer at every step
    u128 f = a - b + i;
    if (r > kMax / f) return kMax;
    r = r * f / i;
  }
  return r;
}

int validate_csr(const kdss_csr* g) {
  if (!g || !g->row_ptr || (g->nnz && !g->col)) return fail(KDSS_EINVAL, "null graph array");
  const uint64_t* rp = g->row_ptr;
  const uint32_t n = g->n;
  if (rp[0] != 0 || rp[n] != g->nnz) return fail(KDSS_EGRAPH, "row_ptr[0] != 0 or row_ptr[n] != nnz");
  for (uint32_t u = 0; u < n; ++u)
    if (rp[u + 1] < rp[u]) return fail(KDSS_EGRAPH, "row_ptr decreases at node " + std::to_string(u));
  // rows in contiguous ranges on host threads; each range keeps its first
  // error, and the earliest range's is reported (the error a row-by-row pass
  // meets first)
  struct Err {
    bool set = false;
    std::string msg;
  };
  std::vector<Err> errs(host_threads());
  parallel_ranges(n, 4096, [&](unsigned t, uint64_t b, uint64_t e) {
    for (uint32_t u = (uint32_t)b; u < (uint32_t)e; ++u) {
      for (uint64_t x = rp[u]; x < rp[u + 1]; ++x) {
        const uint32_t v = g->col[x];
        std::string m;
        if (v >= n) m = "neighbour id out of range in row " + std::to_string(u);
        else if (v == u) m = "self-loop at node " + std::to_string(u);
        else if (x > rp[u] && g->col[x - 1] >= v) m = "row " + std::to_string(u) + " not strictly ascending";
        else {
          const uint32_t* bb = g->col + rp[v];
          const uint32_t* en = g->col + rp[v + 1];
          const uint32_t* f = std::lower_bound(bb, en, u);
          if (f == en || *f != u) m = "edge " + std::to_string(u) + "-" + std::to_string(v) + " is not symmetric";
        }
        if (!m.empty()) {
          errs[t] = Err{true, m};
          return;
        }
      }
    }
  });
  for (const Err& e : errs)
    if (e.set) return fail(KDSS_EGRAPH, e.msg);
  return KDSS_OK;
}

// Peeling by minimum degree with bucket queues; linear time.
void degeneracy_order(const kdss_csr* g, Degeneracy* out) {
  const uint32_t n = g->n;
  std::vector<uint32_t> deg(n), pos(n), vert(n);
  uint32_t md = 0;
  for (uint32_t v = 0; v < n; ++v) {
    deg[v] = (uint32_t)(g->row_ptr[v + 1] - g->row_ptr[v]);
    md = std::max(md, deg[v]);
  }
  std::vector<uint32_t> bin(md + 2, 0);
  for (uint32_t v = 0; v < n; ++v) bin[deg[v]]++;
  uint32_t start = 0;
  for (uint32_t d = 0; d <= md; ++d) {
    uint32_t c = bin[d];
    bin[d] = start;
    start += c;
  }
  for (uint32_t v = 0; v < n; ++v) {
    pos[v] = bin[deg[v]];
    vert[pos[v]] = v;
    bin[deg[v]]++;
  }
  for (uint32_t d = md; d >= 1; --d) bin[d] = bin[d - 1];
  bin[0] = 0;
  out->order.resize(n);
  out->rank.resize(n);
  out->core.resize(n);
  uint32_t dg = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t v = vert[i];
    out->order[i] = v;
    out->rank[v] = i;
    out->core[v] = deg[v];
    dg = std::max(dg, deg[v]);
    for (uint64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
      uint32_t u = g->col[e];
      if (deg[u] > deg[v]) {
        uint32_t du = deg[u], pu = pos[u], pw = bin[du], w = vert[pw];
        if (u != w) {
          pos[u] = pw; vert[pu] = w;
          pos[w] = pu; vert[pw] = u;
        }
        bin[du]++;
        deg[u]--;
      }
    }
  }
  out->degeneracy = dg;
}

namespace {

struct LeafBuf {
  std::vector<uint32_t> members;
  std::vector<uint8_t> h;
  std::vector<uint32_t> p;
  u128 c_k = 0;
  uint32_t s_max = 0;
  bool count_only = false;      // keep only the counts below, not the leaves
  bool ck_wrapped = false;      // c_k passed 2^128 - 1
  uint64_t leaves = 0, nmembers = 0;
};

// Per-thread search state for the subtree of one root.
class RootSearch {
 public:
  RootSearch(const kdss_csr* g, const std::vector<uint64_t>& out_rp, const std::vector<uint32_t>& out_col,
             uint32_t k, const std::vector<u128>& binom_row)
      : g_(g), orp_(out_rp), ocol_(out_col), k_(k), binom_(binom_row), loc_(g->n, -1) {}

  void run(uint32_t v, LeafBuf* out) {
    out_ = out;
    const uint64_t b = orp_[v], e = orp_[v + 1];
    d_ = (uint32_t)(e - b);
    if (1 + d_ < k_) return;
    nodes_.assign(ocol_.begin() + b, ocol_.begin() + e);
    W_ = (d_ + 63) / 64;
    adj_.assign((size_t)d_ * W_, 0);
    for (uint32_t i = 0; i < d_; ++i) loc_[nodes_[i]] = (int32_t)i;
    for (uint32_t i = 0; i < d_; ++i) {
      uint32_t a = nodes_[i];
      for (uint64_t x = orp_[a]; x < orp_[a + 1]; ++x) {
        int32_t j = loc_[ocol_[x]];
        if (j >= 0) {
          adj_[(size_t)i * W_ + (j >> 6)] |= 1ull << (j & 63);
          adj_[(size_t)j * W_ + (i >> 6)] |= 1ull << (i & 63);
        }
      }
    }
    for (uint32_t i = 0; i < d_; ++i) loc_[nodes_[i]] = -1;
    // levels of candidate sets: depth <= d_ + 1
    sets_.assign((size_t)(d_ + 2) * 2 * W_, 0);
    uint64_t* S = level(0, 0);
    for (uint32_t i = 0; i < d_; ++i) S[i >> 6] |= 1ull << (i & 63);
    H_.clear();
    P_.clear();
    H_.push_back(v);
    rec(0, d_);
  }

 private:
  uint64_t* level(uint32_t depth, int which) { return sets_.data() + ((size_t)depth * 2 + which) * W_; }
  uint32_t popc(const uint64_t* s) const {
    uint32_t c = 0;
    for (uint32_t w = 0; w < W_; ++w) c += (uint32_t)__builtin_popcountll(s[w]);
    return c;
  }
  uint32_t popc_and(const uint64_t* a, const uint64_t* b) const {
    uint32_t c = 0;
    for (uint32_t w = 0; w < W_; ++w) c += (uint32_t)__builtin_popcountll(a[w] & b[w]);
    return c;
  }

  void emit(bool drop_pivots) {
    const uint32_t h = (uint32_t)H_.size();
    const uint32_t p = drop_pivots ? 0 : (uint32_t)P_.size();
    if (out_->count_only) {
      const u128 before = out_->c_k;
      out_->c_k += binom_[(size_t)p * (k_ + 1) + (k_ - h)];
      if (out_->c_k < before) out_->ck_wrapped = true;
      out_->leaves += 1;
      out_->nmembers += h + p;
      out_->s_max = std::max(out_->s_max, h + p);
      return;
    }
    out_->members.insert(out_->members.end(), H_.begin(), H_.end());
    for (uint32_t i = 0; i < p; ++i) out_->members.push_back(nodes_[P_[i]]);
    out_->h.push_back((uint8_t)h);
    out_->p.push_back(p);
    out_->c_k += binom_[(size_t)p * (k_ + 1) + (k_ - h)];
    out_->s_max = std::max(out_->s_max, h + p);
  }

  // Candidates are level(depth, 0), with `cnt` members.
  void rec(uint32_t depth, uint32_t cnt) {
    const uint64_t* S = level(depth, 0);
    const uint32_t h = (uint32_t)H_.size(), p = (uint32_t)P_.size();
    if (cnt == 0) {
      emit(false);
      return;
    }
    // pivot: candidate with the most neighbours among the candidates
    int32_t q = -1;
    int32_t best = -1, worst = (int32_t)cnt;
    for (uint32_t w = 0; w < W_; ++w) {
      uint64_t bits = S[w];
      while (bits) {
        uint32_t i = (w << 6) + (uint32_t)__builtin_ctzll(bits);
        bits &= bits - 1;
        int32_t c = (int32_t)popc_and(S, &adj_[(size_t)i * W_]);
        if (c > best) { best = c; q = (int32_t)i; }
        if (c < worst) worst = c;
      }
    }
    if (worst == (int32_t)cnt - 1) {
      // the candidates form a clique: the chain of pivot children below this
      // node ends in the single leaf (H, P + S)
      const size_t keep = P_.size();
      for (uint32_t w = 0; w < W_; ++w) {
        uint64_t bits = S[w];
        while (bits) {
          P_.push_back((w << 6) + (uint32_t)__builtin_ctzll(bits));
          bits &= bits - 1;
        }
      }
      emit(false);
      P_.resize(keep);
      return;
    }
    const uint64_t* Nq = &adj_[(size_t)q * W_];
    uint64_t* child = level(depth + 1, 0);
    // pivot child: q joins P, candidates S & N(q)
    if (h + p + 1 + (uint32_t)best >= k_) {
      for (uint32_t w = 0; w < W_; ++w) child[w] = S[w] & Nq[w];
      P_.push_back((uint32_t)q);
      rec(depth + 1, (uint32_t)best);
      P_.pop_back();
    }
    // hold children: each candidate w outside N(q) + {q}, in index order
    uint64_t* rest = level(depth, 1);
    for (uint32_t w = 0; w < W_; ++w) rest[w] = S[w];
    for (uint32_t w = 0; w < W_; ++w) {
      uint64_t bits = S[w] & ~Nq[w];
      if (w == ((uint32_t)q >> 6)) bits &= ~(1ull << (q & 63));
      while (bits) {
        uint32_t i = (w << 6) + (uint32_t)__builtin_ctzll(bits);
        bits &= bits - 1;
        const uint64_t* Ni = &adj_[(size_t)i * W_];
        if (h + 1 == k_) {
          H_.push_back(nodes_[i]);
          emit(true);
          H_.pop_back();
        } else {
          uint32_t c = 0;
          for (uint32_t x = 0; x < W_; ++x) {
            child[x] = rest[x] & Ni[x];
            c += (uint32_t)__builtin_popcountll(child[x]);
          }
          if (h + 1 + p + c >= k_) {
            H_.push_back(nodes_[i]);
            rec(depth + 1, c);
            H_.pop_back();
          }
        }
        rest[i >> 6] &= ~(1ull << (i & 63));
      }
    }
  }

  const kdss_csr* g_;
  const std::vector<uint64_t>& orp_;
  const std::vector<uint32_t>& ocol_;
  uint32_t k_;
  const std::vector<u128>& binom_;
  std::vector<int32_t> loc_;
  std::vector<uint32_t> nodes_;
  std::vector<uint64_t> adj_, sets_;
  std::vector<uint32_t> H_, P_;
  uint32_t d_ = 0, W_ = 0;
  LeafBuf* out_ = nullptr;
};

}  // namespace

int build_sct(const kdss_csr* g, uint32_t k, uint32_t threads, Sct* out) {
  return build_sct_impl(g, k, threads, out, nullptr);
}

int count_sct(const kdss_csr* g, uint32_t k, uint32_t threads, kdss_tree_stats* stats) {
  Sct tmp;
  return build_sct_impl(g, k, threads, &tmp, stats);
}

// With stats != nullptr only the counts are kept (out receives the degeneracy
// order and nothing else).
int build_sct_impl(const kdss_csr* g, uint32_t k, uint32_t threads, Sct* out, kdss_tree_stats* stats) {
  auto t0 = std::chrono::steady_clock::now();
  if (!g || !out) return fail(KDSS_EINVAL, "null argument");
  if (k < 2) return fail(KDSS_EINVAL, "k must be at least 2");
  if (k > kMaxK) return fail(KDSS_ERANGE, "k must be at most 31");
  int st = validate_csr(g);
  if (st) return st;
  const uint32_t n = g->n;
  out->n = n;
  out->k = k;
  degeneracy_order(g, &out->deg);

  // orient every edge from the earlier to the later node of the degeneracy order
  std::vector<uint64_t> orp(n + 1, 0);
  for (uint32_t v = 0; v < n; ++v)
    for (uint64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e)
      if (out->deg.rank[g->col[e]] > out->deg.rank[v]) orp[v + 1]++;
  for (uint32_t v = 0; v < n; ++v) orp[v + 1] += orp[v];
  std::vector<uint32_t> ocol(orp[n]);
  {
    std::vector<uint64_t> fillp(orp.begin(), orp.end() - 1);
    for (uint32_t v = 0; v < n; ++v)
      for (uint64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e)
        if (out->deg.rank[g->col[e]] > out->deg.rank[v]) ocol[fillp[v]++] = g->col[e];
  }
  const uint32_t dmax = out->deg.degeneracy;
  // C(a, b) for a <= dmax + 1, b <= k
  std::vector<u128> binom((size_t)(dmax + 2) * (k + 1));
  for (uint32_t a = 0; a <= dmax + 1; ++a)
    for (uint32_t b = 0; b <= k; ++b) binom[(size_t)a * (k + 1) + b] = binom128(a, b);

  unsigned nt = threads ? threads : host_threads();
  nt = std::min<unsigned>(nt, 256);
  // roots in degeneracy order, in chunks; each chunk's leaves are kept apart and
  // concatenated in chunk order so the output does not depend on scheduling
  const uint32_t chunk = 256;
  const uint32_t nchunks = (n + chunk - 1) / chunk;
  std::vector<LeafBuf> bufs(nchunks);
  for (auto& b : bufs) b.count_only = stats != nullptr;
  std::atomic<uint32_t> next{0};
  std::atomic<bool> oom{false};
  auto worker = [&]() {
    try {
      RootSearch rs(g, orp, ocol, k, binom);
      for (;;) {
        uint32_t c = next.fetch_add(1);
        if (c >= nchunks) break;
        uint32_t lo = c * chunk, hi = std::min(n, lo + chunk);
        for (uint32_t i = lo; i < hi; ++i) rs.run(out->deg.order[i], &bufs[c]);
      }
    } catch (const std::bad_alloc&) {
      oom = true;
    }
  };
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nt; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  if (oom) return fail(KDSS_ENOMEM, "host memory exhausted while building the clique tree");

  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    u128 ck = 0;
    for (auto& b : bufs) {
      const u128 before = ck;
      ck += b.c_k;
      if (b.ck_wrapped || ck < before) return fail(KDSS_EOVERFLOW, "k-clique count exceeds 2^128");
      stats->leaves += b.leaves;
      stats->members += b.nmembers;
      stats->s_max = std::max(stats->s_max, b.s_max);
    }
    stats->k = k;
    stats->n = n;
    stats->degeneracy = out->deg.degeneracy;
    stats->c_k.lo = (uint64_t)ck;
    stats->c_k.hi = (uint64_t)(ck >> 64);
    stats->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return KDSS_OK;
  }

  uint64_t L = 0, M = 0;
  for (auto& b : bufs) { L += b.h.size(); M += b.members.size(); }
  try {
    out->members.resize(M);
    out->off.resize(L + 1);
    out->h.resize(L);
    out->p.resize(L);
  } catch (const std::bad_alloc&) {
    return fail(KDSS_ENOMEM, "host memory exhausted while flattening the clique tree");
  }
  uint64_t li = 0, mi = 0;
  u128 ck = 0;
  uint32_t smax = 0;
  for (auto& b : bufs) {
    if (!b.members.empty())
      std::memcpy(out->members.data() + mi, b.members.data(), b.members.size() * sizeof(uint32_t));
    for (size_t i = 0; i < b.h.size(); ++i) {
      out->off[li] = mi;
      out->h[li] = b.h[i];
      out->p[li] = b.p[i];
      mi += b.h[i] + b.p[i];
      ++li;
    }
    u128 before = ck;
    ck += b.c_k;
    if (ck < before) return fail(KDSS_EOVERFLOW, "k-clique count exceeds 2^128");
    smax = std::max(smax, b.s_max);
    std::vector<uint32_t>().swap(b.members);
  }
  out->off[L] = mi;
  out->c_k = ck;
  out->s_max = smax;
  out->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return KDSS_OK;
}

}  // namespace kdss
