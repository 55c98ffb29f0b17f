// Host side of the C-ABI: status strings, clique-tree handles and the planner
// that lays a tree out for the GPU.
#include <algorithm>
#include <cstring>
#include <new>

#include "kdss_internal.h"

struct kdss_sct {
  kdss::Sct s;
};

namespace kdss {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
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
  std::memcpy(core, s->s.deg.core.data(), sizeof(uint32_t) * n);
  return KDSS_OK;
}

void kdss_sct_free(kdss_sct* s) { delete s; }

int kdss_plan_create(const kdss_sct* s, uint32_t T_max, uint64_t r0_max, const kdss_opts* opts,
                     kdss_plan** out) {
  if (!s || !out) return fail(KDSS_EINVAL, "null argument");
  *out = nullptr;
  if (T_max == 0) return fail(KDSS_EINVAL, "T_max must be at least 1");
  const Sct& t = s->s;
  if (t.n == 0) return fail(KDSS_EINVAL, "graph has no nodes");
  if ((t.c_k >> 64) != 0) return fail(KDSS_EOVERFLOW, "k-clique count does not fit 64 bits");
  if (t.s_max > kMaxBigLeaf) return fail(KDSS_EUNSUPPORTED, "a leaf has more than 4096 members");
  if (t.n > kHotFlag) return fail(KDSS_EUNSUPPORTED, "more than 2^31 nodes");
  kdss_plan* P = new (std::nothrow) kdss_plan();
  if (!P) return fail(KDSS_ENOMEM, "cannot allocate the plan");
  try {
    P->n = t.n;
    P->k = t.k;
    P->T_max = T_max;
    P->r0_max = r0_max;
    P->c_k = t.c_k;
    P->s_max = t.s_max;
    if (opts) P->opts = *opts;
    P->id_bits = std::max<uint32_t>(1, bit_length(t.n - 1));
    // every load stays <= r0_max + T_max * c_k
    const u128 bound = (u128)r0_max + (u128)T_max * t.c_k;
    const bool fits64 = (bound >> 64) == 0;
    if (P->opts.width == 64 && !fits64) {
      delete P;
      return fail(KDSS_EOVERFLOW, "loads may exceed 2^64 - 1 but width 64 was forced");
    }
    if (P->opts.width != 0 && P->opts.width != 64 && P->opts.width != 128) {
      delete P;
      return fail(KDSS_EINVAL, "width must be 0, 64 or 128");
    }
    P->width = (P->opts.width == 128 || !fits64) ? 128 : 64;
    // packed keys r << id_bits | id need every load below 2^(64 - id_bits) - 1
    const u128 packed_limit = ((u128)1 << (64 - P->id_bits)) - 1;
    P->key_mode = (P->width == 64 && bound < packed_limit) ? 0 : 1;

    // ---- hot nodes: those occurring in the most leaves (ids must leave the flag bit free) ----
    const uint64_t L = t.leaves();
    std::vector<uint32_t> hot_index;
    {
      std::vector<uint64_t> occ(t.n, 0);
      for (uint32_t u : t.members) occ[u]++;
      std::vector<uint32_t> cand;
      for (uint32_t u = 0; u < t.n; ++u)
        if (occ[u] >= kHotMinOccurrences) cand.push_back(u);
      std::sort(cand.begin(), cand.end(), [&](uint32_t a, uint32_t b) {
        return occ[a] != occ[b] ? occ[a] > occ[b] : a < b;
      });
      if (cand.size() > kHotMax) cand.resize(kHotMax);
      P->hot = cand;
      hot_index.assign(t.n, ~0u);
      for (uint32_t i = 0; i < P->hot.size(); ++i) hot_index[P->hot[i]] = i;
    }
    auto encode = [&](uint32_t u) -> uint32_t {
      return (!hot_index.empty() && hot_index[u] != ~0u) ? (kHotFlag | hot_index[u]) : u;
    };
    auto append_leaf = [&](uint64_t id) {
      const uint64_t b = t.off[id], e = b + t.h[id] + t.p[id];
      for (uint64_t x = b; x < e; ++x) P->members.push_back(encode(t.members[x]));
    };

    // ---- tiles: big leaves first (longest work first), then lane tiles from
    // the largest group to the smallest ----
    std::vector<uint64_t> big;
    std::vector<std::vector<uint64_t>> groups(kNumLaneGroups);
    for (uint64_t i = 0; i < L; ++i) {
      const uint32_t s = t.h[i] + t.p[i];
      const int b = size_bucket(s);
      P->class_leaves[b]++;
      P->class_members[b] += s;
      if (s > 64) big.push_back(i);
      else groups[lane_group(s)].push_back(i);
    }
    P->members.reserve(t.members.size() + t.members.size() / 8);
    P->hdr.reserve(L);
    for (uint64_t id : big) {
      Tile tl;
      tl.mbase = P->members.size();
      tl.lbase = (uint32_t)P->hdr.size();
      const uint32_t h = t.h[id], p = t.p[id];
      tl.info = pack_tile_info(kTileBig, 1, 0);
      P->hdr.push_back(pack_leaf(h, p));
      append_leaf(id);
      P->tiles.push_back(tl);
      P->class_tiles[kBigClass]++;
    }
    for (int gi = kNumLaneGroups - 1; gi >= 0; --gi) {
      const auto& ids = groups[gi];
      for (uint64_t i0 = 0; i0 < ids.size(); i0 += 64) {
        const uint32_t nl = (uint32_t)std::min<uint64_t>(64, ids.size() - i0);
        uint32_t smax = 0;
        for (uint32_t r = 0; r < nl; ++r) smax = std::max<uint32_t>(smax, t.h[ids[i0 + r]] + t.p[ids[i0 + r]]);
        Tile tl;
        tl.mbase = P->members.size();
        tl.lbase = (uint32_t)P->hdr.size();
        tl.info = pack_tile_info(kTileLane, nl, smax);
        // column-major: member x of leaf r at mbase + 64 x + r; padding reads node 0
        P->members.resize(P->members.size() + (size_t)64 * smax, 0u);
        uint32_t* col = P->members.data() + tl.mbase;
        for (uint32_t r = 0; r < nl; ++r) {
          const uint64_t id = ids[i0 + r];
          const uint32_t h = t.h[id], p = t.p[id];
          P->hdr.push_back(pack_leaf(h, p));
          for (uint32_t x = 0; x < h + p; ++x) col[(size_t)64 * x + r] = encode(t.members[t.off[id] + x]);
        }
        P->tiles.push_back(tl);
        P->class_tiles[size_bucket(smax)]++;
      }
    }
    if (P->tiles.size() >= (1ull << 26)) {
      delete P;
      return fail(KDSS_ERANGE, "more than 2^26 tiles");
    }
    if (P->hdr.size() > 0xFFFFFFFFull) {
      delete P;
      return fail(KDSS_ERANGE, "more than 2^32 - 1 leaves");
    }
    // binomial table C(a, b), a <= s_max, b <= k (saturated entries are never used
    // because every used entry is at most C(p, k - h) <= c_k < 2^64)
    const uint32_t rows = t.s_max + 1, cols = t.k + 1;
    P->binom.resize((size_t)rows * cols);
    for (uint32_t a = 0; a < rows; ++a)
      for (uint32_t b = 0; b < cols; ++b) {
        u128 v = binom128(a, b);
        P->binom[(size_t)a * cols + b] = (v >> 64) ? ~0ull : (uint64_t)v;
      }

    // ---- workspace layout ----
    const size_t n = t.n;
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
    P->leaf_blocks = (uint32_t)std::min<uint64_t>(kLeafBlocksMax, std::max<uint64_t>(1, (P->tiles.size() + 3) / 4));
    P->off_hot = take(P->hot.size() * 4);
    P->heavy_blocks = kHeavyBlocks;
    P->off_scratch = take((size_t)(P->leaf_blocks + P->heavy_blocks) * P->hot.size() * 8);
    P->lane_leaves = 0;
    for (const Tile& tl : P->tiles)
      if ((tl.info & 7u) == kTileLane) P->lane_leaves += (tl.info >> 3) & 0x1FFFu;
    P->off_queue = take(P->lane_leaves * 4);
    P->off_qcount = take(64);
    P->ws_bytes = o;
  } catch (const std::bad_alloc&) {
    delete P;
    return fail(KDSS_ENOMEM, "host memory exhausted while planning");
  }
  *out = P;
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
  for (int c = 0; c < kNumClasses; ++c) {
    out->tiles[c] = P->class_tiles[c];
    out->leaves[c] = P->class_leaves[c];
    out->members[c] = P->class_members[c];
  }
  return KDSS_OK;
}

}  // extern "C"
