// Host side of the C-ABI: status strings, clique-tree handles and the planner
// that lays a tree out for the GPU.
#include <algorithm>
#include <array>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>

#include "kdss_internal.h"

namespace kdss {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

unsigned host_threads() {
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v > 0) return (unsigned)std::min<long>(v, 256);
  }
  return std::max(1u, std::min(256u, std::thread::hardware_concurrency()));
}

void parallel_ranges(uint64_t count, uint64_t min_per_thread,
                     const std::function<void(unsigned, uint64_t, uint64_t)>& f) {
  const unsigned nt = (unsigned)std::max<uint64_t>(
      1, std::min<uint64_t>(host_threads(), count / std::max<uint64_t>(1, min_per_thread)));
  if (nt == 1) {
    f(0, 0, count);
    return;
  }
  const uint64_t chunk = (count + nt - 1) / nt;
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nt; ++t)
    pool.emplace_back([&f, t, chunk, count]() {
      const uint64_t b = std::min<uint64_t>(count, (uint64_t)t * chunk), e = std::min<uint64_t>(count, b + chunk);
      f(t, b, e);
    });
  for (auto& th : pool) th.join();
}

namespace {

uint32_t bit_length(uint64_t x) {
  uint32_t b = 0;
  while (x) { ++b; x >>= 1; }
  return b;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Reporting bucket of a leaf with s members: 0..3 for s <= 8, 16, 32, 64; 4 above.
int size_bucket(uint32_t s) {
  for (int c = 0; c < kBigClass; ++c)
    if (s <= (8u << c)) return c;
  return kBigClass;
}

// Lane-tile group of a leaf with s <= 64 members: the first bound >= s.
int lane_group(uint32_t s) {
  for (int g = 0; g < kNumLaneGroups; ++g)
    if (s <= kLaneBounds[g]) return g;
  return kNumLaneGroups - 1;
}

}  // namespace
}  // namespace kdss

using namespace kdss;

extern "C" {

const char* kdss_status_string(int status) {
  switch (status) {
    case KDSS_OK: return "ok";
    case KDSS_EINVAL: return "invalid argument";
    case KDSS_EGRAPH: return "not a simple undirected graph";
    case KDSS_ERANGE: return "size out of range";
    case KDSS_EOVERFLOW: return "exact count would overflow";
    case KDSS_EWORKSPACE: return "workspace too small or not uploaded";
    case KDSS_EHIP: return "HIP runtime error";
    case KDSS_ENOMEM: return "out of host memory";
    case KDSS_EUNSUPPORTED: return "unsupported case";
    default: return "unknown status";
  }
}

const char* kdss_last_error(void) { return g_last_error.c_str(); }

int kdss_csr_validate(const kdss_csr* g) { return validate_csr(g); }

int kdss_sct_build(const kdss_csr* g, uint32_t k, uint32_t threads, kdss_sct** out) {
  if (!out) return fail(KDSS_EINVAL, "null output handle");
  *out = nullptr;
  kdss_sct* s = new (std::nothrow) kdss_sct();
  if (!s) return fail(KDSS_ENOMEM, "cannot allocate the tree handle");
  int st;
  try {
    st = build_sct(g, k, threads, &s->s);
  } catch (const std::bad_alloc&) {
    st = fail(KDSS_ENOMEM, "host memory exhausted while building the clique tree");
  }
  if (st) {
    delete s;
    return st;
  }
  *out = s;
  return KDSS_OK;
}

int kdss_sct_count(const kdss_csr* g, uint32_t k, uint32_t threads, kdss_tree_stats* out) {
  if (!out) return fail(KDSS_EINVAL, "null output");
  try {
    return count_sct(g, k, threads, out);
  } catch (const std::bad_alloc&) {
    return fail(KDSS_ENOMEM, "host memory exhausted while counting the clique tree");
  }
}

int kdss_sct_info(const kdss_sct* s, kdss_tree_stats* out) {
  if (!s || !out) return fail(KDSS_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->k = s->s.k;
  out->n = s->s.n;
  out->leaves = s->s.leaves();
  out->members = s->s.members.size();
  out->s_max = s->s.s_max;
  out->degeneracy = s->s.deg.degeneracy;
  out->c_k.lo = (uint64_t)s->s.c_k;
  out->c_k.hi = (uint64_t)(s->s.c_k >> 64);
  out->build_seconds = s->s.build_seconds;
  return KDSS_OK;
}

int kdss_sct_export(const kdss_sct* s, uint32_t* h, uint32_t* p, uint32_t* members, uint64_t leaf_cap,
                    uint64_t member_cap) {
  if (!s || !h || !p || (!members && s->s.members.size())) return fail(KDSS_EINVAL, "null argument");
  if (leaf_cap < s->s.leaves() || member_cap < s->s.members.size())
    return fail(KDSS_ERANGE, "export capacity too small");
  for (uint64_t i = 0; i < s->s.leaves(); ++i) {
    h[i] = s->s.h[i];
    p[i] = s->s.p[i];
  }
  if (!s->s.members.empty()) std::memcpy(members, s->s.members.data(), s->s.members.size() * sizeof(uint32_t));
  return KDSS_OK;
}

int kdss_sct_core_numbers(const kdss_sct* s, uint32_t* core, uint32_t n) {
  if (!s || !core) return fail(KDSS_EINVAL, "null argument");
  if (n != s->s.n) return fail(KDSS_ERANGE, "n does not match the tree");
  if (s->s.deg.core.size() != n) return fail(KDSS_EUNSUPPORTED, "a tree of sampled cliques has no core numbers");
  if (n) std::memcpy(core, s->s.deg.core.data(), sizeof(uint32_t) * n);
  return KDSS_OK;
}

void kdss_sct_free(kdss_sct* s) { delete s; }

}  // extern "C"

namespace kdss {

// Byte offsets of every device buffer inside the caller's workspace.
static void layout_workspace(kdss_plan* P) {
  const size_t n = P->n;
  const size_t nprob = P->node_off.size() - 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + std::max<size_t>(bytes, 1));
    return at;
  };
  P->sort_blocks = (uint32_t)((n + kSortTile - 1) / kSortTile);
  P->scan_blocks = (uint32_t)((n + kScanTile - 1) / kScanTile);
  P->red_blocks = (uint32_t)((n + kRedTile - 1) / kRedTile);
  P->off_members = take(P->members.size() * 4);
  P->off_hdr = take(P->hdr.size() * 4);
  P->off_tiles = take(P->tiles.size() * sizeof(Tile));
  P->off_binom = take(P->binom.size() * 8);
  P->off_delta = take(n * 8);
  P->off_cnt = take(n * 8);
  P->off_kw[0][0] = take(n * 8);
  P->off_kw[1][0] = take(n * 8);
  P->off_kw[0][1] = take(P->width == 128 ? n * 8 : 8);
  P->off_kw[1][1] = take(P->width == 128 ? n * 8 : 8);
  P->off_perm[0] = take(n * 4);
  P->off_perm[1] = take(n * 4);
  P->off_keyp = take(n * 4);
  P->off_hist = take((size_t)256 * P->sort_blocks * 4);
  P->off_dbase = take(256 * 4);
  P->off_bsum = take((size_t)P->scan_blocks * 8);
  P->off_bbest = take((size_t)P->scan_blocks * 16);
  P->off_red = take((size_t)P->red_blocks * 16);   // a (lo, hi) pair per block
  P->off_dres = take(sizeof(DevResult));
  P->off_tb_binom = take(P->tb_binom.size() * 8);
  P->leaf_blocks = (uint32_t)std::min<uint64_t>(kLeafBlocksDefault, std::max<uint64_t>(1, (P->tiles.size() + 3) / 4));
  P->heavy_blocks = kHeavyBlocksDefault;
  P->off_hot = take(P->hot.size() * 4);
  P->off_hot_base = take(P->hot.size() * 4);
  // hot-node credit slots, hot-node-major (kept zero between passes)
  P->off_scratch = take((size_t)kHotSlots * P->hot.size() * 8);
  P->lane_leaves = 0;
  for (const Tile& tl : P->tiles)
    if ((tl.info & 7u) == kTileLane) P->lane_leaves += (tl.info >> 3) & 0x1FFFu;
  // PBUpdate: the lane tiles of at most kPbRegRows rows form a suffix (groups
  // run from the largest to the smallest); the tiles before it are staged in LDS
  P->pb_split = (uint32_t)P->tiles.size();
  while (P->pb_split > 0) {
    const Tile& tl = P->tiles[P->pb_split - 1];
    if ((tl.info & 7u) != kTileLane || (tl.info >> 16) > kPbRegRows) break;
    --P->pb_split;
  }
  // ... and before it, a run of lane tiles of at most kPbMidRows rows
  P->pb_mid = P->pb_split;
  while (P->pb_mid > 0) {
    const Tile& tl = P->tiles[P->pb_mid - 1];
    if ((tl.info & 7u) != kTileLane || (tl.info >> 16) > kPbMidRows) break;
    --P->pb_mid;
  }
  P->pb_rows = 1;
  P->pb_rows_lo = 1;
  for (uint32_t i = 0; i < P->pb_split; ++i) {
    const Tile& tl = P->tiles[i];
    const uint32_t smax = tl.info >> 16;
    uint32_t& rows = i < P->pb_mid ? P->pb_rows : P->pb_rows_lo;
    rows = std::max(rows, (tl.info & 7u) == kTileLane ? smax : (smax + 63) / 64);
  }
  P->off_queue = take(P->lane_leaves * 16);   // 16-byte heavy-leaf entries
  P->off_hotkey = take((size_t)kHotMax * 32);     // hot-node keys of the current pass
  P->off_hotkey_fw = take((size_t)kHotMax * 32);  // hot-node keys at the current loads (64-bit runs)
  P->off_qcount = take(64);
  P->off_qlog = take((size_t)P->T_max * 4);
  // XCD ranges: cut points of equal work (a lane tile costs its 64-member rows,
  // a big tile its members)
  {
    std::vector<uint64_t> cum(P->tiles.size() + 1, 0);
    for (size_t i = 0; i < P->tiles.size(); ++i) {
      const Tile& tl = P->tiles[i];
      const uint64_t rows = tl.info >> 16;
      const uint32_t hd = P->hdr[tl.lbase];
      const uint64_t big = (hd & 31u) + (hd >> 10);
      cum[i + 1] = cum[i] + ((tl.info & 7u) == kTileLane ? 64 * rows : big) + 64;
    }
    for (uint32_t x = 0; x <= kXcds; ++x) {
      const uint64_t want = cum.back() * x / kXcds;
      P->xcd_bounds[x] = (uint32_t)(std::lower_bound(cum.begin(), cum.end(), want) - cum.begin());
    }
    P->xcd_bounds[kXcds] = (uint32_t)P->tiles.size();
  }
  P->off_xcd = take(sizeof(P->xcd_bounds));
  // batch extraction: prefix sums, per-problem results and node offsets
  P->off_prefix = take(n * 8);
  P->off_pres = take(nprob * sizeof(DevResult));
  P->off_nodeoff = take((nprob + 1) * 8);
  P->ws_bytes = o;
}

// Lays out one or more trees (a batch) for the GPU.  Problem q's nodes get the
// ids node_off[q] .. node_off[q + 1] - 1 of one concatenated id space; leaves
// never span problems, and each leaf header carries its own j = k - h.
static int build_plan(const std::vector<const Sct*>& trees, uint32_t T_max, uint64_t r0_max,
                      const kdss_opts* opts, kdss_plan** out) {
  if (T_max == 0) return fail(KDSS_EINVAL, "T_max must be at least 1");
  uint64_t n_total = 0;
  uint32_t kmax = 0, s_max = 0;
  u128 bound_max = 0, ck_total = 0;
  for (const Sct* t : trees) {
    if (t->n == 0) return fail(KDSS_EINVAL, "graph has no nodes");
    if ((t->c_k >> 64) != 0) return fail(KDSS_EOVERFLOW, "k-clique count does not fit 64 bits");
    if (t->s_max > kMaxBigLeaf) return fail(KDSS_EUNSUPPORTED, "a leaf has more than 4096 members");
    n_total += t->n;
    kmax = std::max(kmax, t->k);
    s_max = std::max(s_max, t->s_max);
    ck_total += t->c_k;
    // every load of problem q stays <= r0_max + T_max * c_k(q)
    bound_max = std::max(bound_max, (u128)r0_max + (u128)T_max * t->c_k);
  }
  if (n_total > kHotFlag) return fail(KDSS_EUNSUPPORTED, "more than 2^31 nodes");
  kdss_plan* P = new (std::nothrow) kdss_plan();
  if (!P) return fail(KDSS_ENOMEM, "cannot allocate the plan");
  try {
    P->n = (uint32_t)n_total;
    P->k = trees.size() == 1 ? trees[0]->k : kmax;
    P->k1 = kmax + 1;
    P->T_max = T_max;
    P->r0_max = r0_max;
    P->c_k = trees.size() == 1 ? trees[0]->c_k : ck_total;
    P->s_max = s_max;
    if (opts) P->opts = *opts;
    // packed keys hold problem-local ids: ties are only ever compared inside one leaf
    uint64_t n_max = 1;
    for (const Sct* t : trees) n_max = std::max<uint64_t>(n_max, t->n);
    P->id_bits = std::max<uint32_t>(1, bit_length(n_max - 1));
    P->node_off.assign(1, 0);
    for (const Sct* t : trees) {
      P->node_off.push_back(P->node_off.back() + t->n);
      P->prob_k.push_back(t->k);
      P->prob_ck.push_back(t->c_k);
    }
    const bool fits64 = (bound_max >> 64) == 0;
    if (P->opts.width != 0 && P->opts.width != 64 && P->opts.width != 128) {
      delete P;
      return fail(KDSS_EINVAL, "width must be 0, 64 or 128");
    }
    if (P->opts.gather < 0 || P->opts.gather > 2) {
      delete P;
      return fail(KDSS_EINVAL, "gather must be 0, 1 or 2");
    }
    if (P->opts.update < 0 || P->opts.update > 1) {
      delete P;
      return fail(KDSS_EINVAL, "update must be 0 (Frank-Wolfe) or 1 (PBUpdate)");
    }
    if (P->opts.schedule < 0 || P->opts.schedule > 2) {
      delete P;
      return fail(KDSS_EINVAL, "schedule must be 0, 1 or 2");
    }
    P->sched = P->opts.schedule == 2 ? 2 : 1;
    if (P->opts.heavy < 0 || P->opts.heavy > 3) {
      delete P;
      return fail(KDSS_EINVAL, "heavy must be 0, 1, 2 or 3");
    }
    P->heavy = P->opts.heavy ? P->opts.heavy : 1;
    if (P->opts.update == 1 && (P->opts.width == 128 || !fits64)) {
      delete P;
      return fail(KDSS_EINVAL, "PBUpdate runs with 64-bit loads only");
    }
    if (P->opts.width == 64 && !fits64) {
      delete P;
      return fail(KDSS_EOVERFLOW, "loads may exceed 2^64 - 1 but width 64 was forced");
    }
    P->width = (P->opts.width == 128 || !fits64) ? 128 : 64;
    // packed keys r << id_bits | id need every load below 2^(64 - id_bits) - 1
    const u128 packed_limit = ((u128)1 << (64 - P->id_bits)) - 1;
    P->key_mode = (P->width == 64 && bound_max < packed_limit) ? 0 : 1;
    P->bound_max = bound_max;

    // ---- hot nodes: those occurring in the most leaves (per-thread counts) ----
    std::vector<uint32_t> hot_index(n_total, ~0u);
    {
      std::vector<uint64_t> occ(n_total, 0);
      for (size_t q = 0; q < trees.size(); ++q) {
        const std::vector<uint32_t>& mem = trees[q]->members;
        const uint32_t tn = trees[q]->n;
        const unsigned nt = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(host_threads(), mem.size() >> 20));
        std::vector<std::vector<uint32_t>> local(nt, std::vector<uint32_t>(tn, 0));
        parallel_ranges(mem.size(), (mem.size() + nt - 1) / nt, [&](unsigned t, uint64_t b, uint64_t e) {
          for (uint64_t x = b; x < e; ++x) local[t][mem[x]]++;
        });
        for (const auto& lc : local)
          for (uint32_t u = 0; u < lc.size(); ++u) occ[P->node_off[q] + u] += lc[u];
      }
      std::vector<uint32_t> cand;
      for (uint64_t u = 0; u < n_total; ++u)
        if (occ[u] >= kHotMinOccurrences) cand.push_back((uint32_t)u);
      std::sort(cand.begin(), cand.end(), [&](uint32_t a, uint32_t b) {
        return occ[a] != occ[b] ? occ[a] > occ[b] : a < b;
      });
      if (cand.size() > kHotMax) cand.resize(kHotMax);
      P->hot = cand;
      uint64_t occ_all = 0, occ_hot = 0;
      for (uint64_t u = 0; u < n_total; ++u) occ_all += occ[u];
      for (uint32_t u : cand) occ_hot += occ[u];
      P->hot_share = occ_all ? (double)occ_hot / (double)occ_all : 0.0;
      P->gather = P->opts.gather != 0 ? P->opts.gather : (P->hot_share >= kMaskedGatherShare ? 1 : 2);
      for (uint32_t i = 0; i < P->hot.size(); ++i) {
        hot_index[P->hot[i]] = i;
        const uint64_t q = std::upper_bound(P->node_off.begin(), P->node_off.end(), (uint64_t)P->hot[i]) -
                           P->node_off.begin() - 1;
        P->hot_base.push_back((uint32_t)P->node_off[q]);
      }
    }
    auto encode = [&](uint64_t u) -> uint32_t {
      return hot_index[u] != ~0u ? (kHotFlag | hot_index[u]) : (uint32_t)u;
    };

    // ---- tiles: big leaves first (longest work first), then lane tiles from
    // the largest group to the smallest; a tile holds leaves of one problem.
    // Within a group, leaves keep the tree's (depth-first) order. ----
    // a leaf reference packs (problem << 40 | leaf index)
    auto ref_q = [](uint64_t r) { return (uint32_t)(r >> 40); };
    auto ref_id = [](uint64_t r) { return r & ((1ull << 40) - 1); };
    constexpr int kGroups = kNumLaneGroups + 1;   // the last one holds big leaves
    std::vector<std::vector<uint64_t, NoInitAlloc<uint64_t>>> groups(kGroups);
    uint64_t L = 0, M = 0;
    for (uint32_t q = 0; q < trees.size(); ++q) {
      const Sct& t = *trees[q];
      if (t.leaves() >= (1ull << 40)) {
        delete P;
        return fail(KDSS_ERANGE, "more than 2^40 leaves in one tree");
      }
      L += t.leaves();
      M += t.members.size();
      // count per thread range, then scatter in order
      const unsigned nt = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(host_threads(), t.leaves() >> 18));
      const uint64_t chunk = (t.leaves() + nt - 1) / nt;
      std::vector<std::array<uint64_t, kGroups>> cnt(nt);
      std::vector<std::array<uint64_t, kNumClasses>> cl(nt), cm(nt);
      auto group_of = [&](uint64_t i) {
        const uint32_t s = t.h[i] + t.p[i];
        return s > 64 ? kNumLaneGroups : lane_group(s);
      };
      parallel_ranges(t.leaves(), chunk, [&](unsigned th, uint64_t b, uint64_t e) {
        for (uint64_t i = b; i < e; ++i) {
          const uint32_t s = t.h[i] + t.p[i];
          cnt[th][group_of(i)]++;
          cl[th][size_bucket(s)]++;
          cm[th][size_bucket(s)] += s;
        }
      });
      std::vector<std::array<uint64_t, kGroups>> pos(nt);
      for (int gi = 0; gi < kGroups; ++gi) {
        uint64_t at = groups[gi].size();
        for (unsigned th = 0; th < nt; ++th) {
          pos[th][gi] = at;
          at += cnt[th][gi];
        }
        groups[gi].resize(at);
      }
      for (unsigned th = 0; th < nt; ++th)
        for (int c = 0; c < kNumClasses; ++c) {
          P->class_leaves[c] += cl[th][c];
          P->class_members[c] += cm[th][c];
        }
      parallel_ranges(t.leaves(), chunk, [&](unsigned th, uint64_t b, uint64_t e) {
        auto at = pos[th];
        for (uint64_t i = b; i < e; ++i) {
          const int gi = group_of(i);
          groups[gi][at[gi]++] = ((uint64_t)q << 40) | i;
        }
      });
    }
    auto leaf_size = [&](uint64_t r) {
      const Sct& t = *trees[ref_q(r)];
      return (uint32_t)(t.h[ref_id(r)] + t.p[ref_id(r)]);
    };
    auto header = [&](uint64_t r) {
      const Sct& t = *trees[ref_q(r)];
      return pack_leaf(t.h[ref_id(r)], t.k - t.h[ref_id(r)], t.p[ref_id(r)]);
    };
    // tile shapes (sequential, cheap), then the member fill (parallel over tiles)
    struct TileJob { int gi; uint64_t i0; };
    std::vector<TileJob> jobs;
    uint64_t mtotal = 0;
    P->hdr.reserve(L);
    {
      const auto& refs = groups[kNumLaneGroups];
      for (uint64_t i = 0; i < refs.size(); ++i) {
        Tile tl{};
        tl.mbase = mtotal;
        tl.lbase = (uint32_t)P->hdr.size();
        tl.info = pack_tile_info(kTileBig, 1, 0);
        tl.nbase = (uint32_t)P->node_off[ref_q(refs[i])];
        P->hdr.push_back(header(refs[i]));
        mtotal += leaf_size(refs[i]);
        jobs.push_back({kNumLaneGroups, i});
        P->tiles.push_back(tl);
        P->class_tiles[kBigClass]++;
      }
    }
    for (int gi = kNumLaneGroups - 1; gi >= 0; --gi) {
      const auto& refs = groups[gi];
      uint64_t i0 = 0;
      while (i0 < refs.size()) {
        // up to 64 leaves of the same problem
        uint32_t nl = 0, smax = 0;
        while (nl < 64 && i0 + nl < refs.size() && ref_q(refs[i0 + nl]) == ref_q(refs[i0])) {
          smax = std::max<uint32_t>(smax, leaf_size(refs[i0 + nl]));
          P->hdr.push_back(header(refs[i0 + nl]));
          ++nl;
        }
        Tile tl{};
        tl.mbase = mtotal;
        tl.lbase = (uint32_t)(P->hdr.size() - nl);
        tl.info = pack_tile_info(kTileLane, nl, smax);
        tl.nbase = (uint32_t)P->node_off[ref_q(refs[i0])];
        mtotal += (uint64_t)64 * smax;
        jobs.push_back({gi, i0});
        P->tiles.push_back(tl);
        P->class_tiles[size_bucket(smax)]++;
        i0 += nl;
      }
    }
    // every word of the stream is written below, padding included (node 0)
    P->members.resize(mtotal);
    parallel_ranges(jobs.size(), 256, [&](unsigned, uint64_t b, uint64_t e) {
      for (uint64_t j = b; j < e; ++j) {
        const Tile& tl = P->tiles[j];
        uint32_t* dst = P->members.data() + tl.mbase;
        const auto& refs = groups[jobs[j].gi];
        if ((tl.info & 7u) == kTileBig) {
          const uint64_t r = refs[jobs[j].i0];
          const Sct& t = *trees[ref_q(r)];
          const uint64_t nb = P->node_off[ref_q(r)];
          for (uint64_t x = t.off[ref_id(r)]; x < t.off[ref_id(r) + 1]; ++x) *dst++ = encode(nb + t.members[x]);
          continue;
        }
        // column-major: member x of leaf r at mbase + 64 x + r
        const uint32_t nl = (tl.info >> 3) & 0x1FFFu, smax = tl.info >> 16;
        const uint32_t rows = smax;
        uint64_t moff[64];
        uint32_t msz[64];
        const Sct& t = *trees[ref_q(refs[jobs[j].i0])];
        const uint64_t nb = P->node_off[ref_q(refs[jobs[j].i0])];
        for (uint32_t r = 0; r < 64; ++r) {
          msz[r] = 0;
          if (r < nl) {
            const uint64_t id = ref_id(refs[jobs[j].i0 + r]);
            moff[r] = t.off[id];
            msz[r] = t.h[id] + t.p[id];
          }
        }
        for (uint32_t x = 0; x < rows; ++x)
          for (uint32_t r = 0; r < 64; ++r)
            dst[lane_tile_offset(x, r)] = x < msz[r] ? encode(nb + t.members[moff[r] + x]) : 0u;
      }
    });
    if (P->tiles.size() >= (1ull << 26)) {
      delete P;
      return fail(KDSS_ERANGE, "more than 2^26 tiles");
    }
    // Frank-Wolfe batches list their tiles problem by problem (each problem's
    // in the order above): a contiguous range of tiles then touches the keys
    // of few problems.  (PBUpdate keeps the size-class order its launch split
    // relies on.)
    if (trees.size() > 1 && P->opts.update == 0)
      std::stable_sort(P->tiles.begin(), P->tiles.end(),
                       [](const Tile& a, const Tile& b) { return a.nbase < b.nbase; });
    if (P->hdr.size() > 0xFFFFFFFFull) {
      delete P;
      return fail(KDSS_ERANGE, "more than 2^32 - 1 leaves");
    }
    // binomial table C(a, b), a <= s_max, b <= kmax (saturated entries are never
    // used: every used entry is at most C(p, k - h) <= c_k < 2^64)
    const uint32_t rows = s_max + 1, cols = P->k1;
    P->binom.resize((size_t)rows * cols);
    for (uint32_t a = 0; a < rows; ++a)
      for (uint32_t b = 0; b < cols; ++b) {
        u128 v = binom128(a, b);
        P->binom[(size_t)a * cols + b] = (v >> 64) ? ~0ull : (uint64_t)v;
      }
    // the top-s bound looks at s <= s0 only, s0 the first s with C(s, k) >= c_k:
    // beyond it every candidate is A_s, and A_s / s does not grow
    if (trees.size() == 1 && n_total > 0 && (P->c_k >> 64) == 0) {
      const uint32_t k = P->k;
      u128 c = 0;   // C(s, k)
      P->tb_binom.push_back(0);
      for (uint64_t s = 1; s <= n_total; ++s) {
        if (s == k) c = 1;
        else if (s > k) c = c * s / (s - k);   // c < c_k < 2^64 here, so no overflow
        P->tb_binom.push_back((c >> 64) ? ~0ull : (uint64_t)c);
        if (c >= P->c_k) break;
      }
    }
    layout_workspace(P);
  } catch (const std::bad_alloc&) {
    delete P;
    return fail(KDSS_ENOMEM, "host memory exhausted while planning");
  }
  *out = P;
  return KDSS_OK;
}

}  // namespace kdss

extern "C" {

int kdss_plan_create(const kdss_sct* s, uint32_t T_max, uint64_t r0_max, const kdss_opts* opts,
                     kdss_plan** out) {
  if (!s || !out) return fail(KDSS_EINVAL, "null argument");
  *out = nullptr;
  return build_plan({&s->s}, T_max, r0_max, opts, out);
}

int kdss_batch_create(const kdss_sct* const* trees, uint32_t count, uint32_t T_max, uint64_t r0_max,
                      const kdss_opts* opts, kdss_plan** out) {
  if (!trees || !out || count == 0) return fail(KDSS_EINVAL, "null argument or empty batch");
  *out = nullptr;
  std::vector<const Sct*> v;
  for (uint32_t i = 0; i < count; ++i) {
    if (!trees[i]) return fail(KDSS_EINVAL, "null tree in batch");
    v.push_back(&trees[i]->s);
  }
  return build_plan(v, T_max, r0_max, opts, out);
}

int kdss_workspace_size(const kdss_sct* s, uint32_t T_max, uint64_t r0_max, const kdss_opts* opts,
                        size_t* bytes) {
  if (!s || !bytes) return fail(KDSS_EINVAL, "null argument");
  kdss_plan* P = nullptr;
  int rc = build_plan({&s->s}, T_max, r0_max, opts, &P);
  if (rc) return rc;
  *bytes = P->ws_bytes;
  kdss_plan_free(P);
  return KDSS_OK;
}

int kdss_solve(const kdss_csr* g, uint32_t k, uint32_t T, const kdss_opts* opts, const uint64_t* d_r0,
               uint64_t r0_max, void* d_ws, size_t ws_bytes, size_t* ws_needed, void* d_r, size_t r_words,
               uint32_t* d_order, kdss_result* h_res, void* stream) {
  if (!g || !ws_needed || !h_res) return fail(KDSS_EINVAL, "null argument");
  std::memset(h_res, 0, sizeof(*h_res));
  kdss_sct* tree = nullptr;
  int rc = kdss_sct_build(g, k, 0, &tree);
  if (rc) return rc;
  kdss_plan* P = nullptr;
  rc = build_plan({&tree->s}, T, r0_max, opts, &P);
  if (!rc) {
    *ws_needed = P->ws_bytes;
    h_res->width = P->width;
    h_res->n = P->n;
    const size_t words = (size_t)P->n * (P->width == 128 ? 2 : 1);
    if (!d_ws || ws_bytes < P->ws_bytes)
      rc = fail(KDSS_EWORKSPACE, "workspace smaller than the plan needs (see *ws_needed)");
    else if (r_words < words)
      rc = fail(KDSS_EWORKSPACE, "load buffer smaller than n words (2n for 128-bit loads)");
    else if (!d_r || !d_order)
      rc = fail(KDSS_EINVAL, "null output");
    if (!rc) rc = kdss_plan_upload(P, d_ws, ws_bytes, stream);
    if (!rc) rc = kdss_run(P, d_ws, ws_bytes, T, d_r0, d_r, d_order, nullptr, 0, h_res, stream);
  }
  kdss_plan_free(P);
  kdss_sct_free(tree);
  return rc;
}

int kdss_batch_offsets(const kdss_plan* P, uint64_t* node_off, uint32_t count) {
  if (!P || !node_off) return fail(KDSS_EINVAL, "null argument");
  if (count + 1 != P->node_off.size()) return fail(KDSS_ERANGE, "count does not match the plan");
  std::memcpy(node_off, P->node_off.data(), sizeof(uint64_t) * (count + 1));
  return KDSS_OK;
}

int kdss_plan_info(const kdss_plan* P, kdss_plan_stats* out) {
  if (!P || !out) return fail(KDSS_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->workspace_bytes = P->ws_bytes;
  out->stream_bytes = P->members.size() * 4 + P->hdr.size() * 4 + P->tiles.size() * sizeof(Tile);
  out->width = P->width;
  out->key_mode = P->key_mode;
  out->id_bits = P->id_bits;
  out->T_max = P->T_max;
  out->gather = P->gather;
  out->update = P->opts.update;
  out->schedule = P->sched;
  out->heavy = P->heavy;
  out->hot_nodes = (uint32_t)P->hot.size();
  out->hot_share = P->hot_share;
  for (int c = 0; c < kNumClasses; ++c) {
    out->tiles[c] = P->class_tiles[c];
    out->leaves[c] = P->class_leaves[c];
    out->members[c] = P->class_members[c];
  }
  return KDSS_OK;
}

}  // extern "C"
