// Device side of kdss for gfx950 (CDNA4, 64-lane wavefronts): the leaf-credit
// pass, the load update, and the extraction (radix sort, prefix clique counts,
// exact best-prefix search), plus the C-ABI entry points that launch them.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "kdss_internal.h"

using namespace kdss;

namespace {

// ----------------------------------------------------------------------------
// Cross-lane helpers on 64-bit values (two 32-bit lane operations each).
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int lane) {
  uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, lane);
  uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int mask) {
  uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask);
  uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t shfl32(uint32_t v, int lane) { return (uint32_t)__shfl((int)v, lane); }
__device__ __forceinline__ uint32_t shfl_xor32(uint32_t v, int mask) { return (uint32_t)__shfl_xor((int)v, mask); }
__device__ __forceinline__ uint32_t readlane32(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// ----------------------------------------------------------------------------
// Keys.  A leaf orders its members by (load, node id); the minimum of a clique
// is the member with the smallest key.  Every selection between keys goes
// through pick() field by field, so multi-word keys stay in registers.  Four
// encodings:
//   KPacked: load << id_bits | local id in one u64 (built from the gathered
//            load; local id = id - first id of the node's problem);
//   KFull:   (u64 load, id);  KWide: (u128 load, id);
//   KRank:   a unique u32 (the extraction's n - 1 - position).
// ----------------------------------------------------------------------------
struct KeySrc {
  const uint64_t* r;      // loads (u64, or u128 as lo/hi pairs)
  const uint32_t* rank;   // extraction keys
  uint32_t id_bits;       // packed keys: load << id_bits | (id - base)
  uint32_t base;          // first node id of the problem being processed
};

struct KPacked {
  uint64_t v;
  __device__ static KPacked mx() { return {~0ull}; }
  __device__ static KPacked load(const KeySrc& s, uint32_t u) { return {(s.r[u] << s.id_bits) | (u - s.base)}; }
  // the memory read of load alone, and the key made from it
  using Raw = uint64_t;
  __device__ static Raw fetch(const KeySrc& s, uint32_t u) { return s.r[u]; }
  __device__ static KPacked finish(Raw x, const KeySrc& s, uint32_t u) { return {(x << s.id_bits) | (u - s.base)}; }
  __device__ bool lt(const KPacked& o) const { return v < o.v; }
  __device__ bool eq(const KPacked& o) const { return v == o.v; }
  __device__ KPacked sx(int m) const { return {shfl_xor64(v, m)}; }
  __device__ KPacked sl(int l) const { return {shfl64(v, l)}; }
  __device__ KPacked rl(int l) const { return {readlane64(v, l)}; }
  __device__ static KPacked pick(bool c, const KPacked& a, const KPacked& b) { return {c ? a.v : b.v}; }
};

struct KFull {
  uint64_t r;
  uint32_t id;
  __device__ static KFull mx() { return {~0ull, ~0u}; }
  __device__ static KFull load(const KeySrc& s, uint32_t u) { return {s.r[u], u}; }
  using Raw = uint64_t;
  __device__ static Raw fetch(const KeySrc& s, uint32_t u) { return s.r[u]; }
  __device__ static KFull finish(Raw x, const KeySrc&, uint32_t u) { return {x, u}; }
  __device__ bool lt(const KFull& o) const { return r < o.r || (r == o.r && id < o.id); }
  __device__ bool eq(const KFull& o) const { return r == o.r && id == o.id; }
  __device__ KFull sx(int m) const { return {shfl_xor64(r, m), shfl_xor32(id, m)}; }
  __device__ KFull sl(int l) const { return {shfl64(r, l), shfl32(id, l)}; }
  __device__ KFull rl(int l) const { return {readlane64(r, l), readlane32(id, l)}; }
  __device__ static KFull pick(bool c, const KFull& a, const KFull& b) { return {c ? a.r : b.r, c ? a.id : b.id}; }
};

struct KWide {
  uint64_t hi, lo;
  uint32_t id;
  __device__ static KWide mx() { return {~0ull, ~0ull, ~0u}; }
  __device__ static KWide load(const KeySrc& s, uint32_t u) { return {s.r[2ull * u + 1], s.r[2ull * u], u}; }
  struct Raw {
    uint64_t hi, lo;
  };
  __device__ static Raw fetch(const KeySrc& s, uint32_t u) { return {s.r[2ull * u + 1], s.r[2ull * u]}; }
  __device__ static KWide finish(Raw x, const KeySrc&, uint32_t u) { return {x.hi, x.lo, u}; }
  __device__ bool lt(const KWide& o) const {
    return hi < o.hi || (hi == o.hi && (lo < o.lo || (lo == o.lo && id < o.id)));
  }
  __device__ bool eq(const KWide& o) const { return hi == o.hi && lo == o.lo && id == o.id; }
  __device__ KWide sx(int m) const { return {shfl_xor64(hi, m), shfl_xor64(lo, m), shfl_xor32(id, m)}; }
  __device__ KWide sl(int l) const { return {shfl64(hi, l), shfl64(lo, l), shfl32(id, l)}; }
  __device__ KWide rl(int l) const { return {readlane64(hi, l), readlane64(lo, l), readlane32(id, l)}; }
  __device__ static KWide pick(bool c, const KWide& a, const KWide& b) {
    return {c ? a.hi : b.hi, c ? a.lo : b.lo, c ? a.id : b.id};
  }
};

struct KRank {
  uint32_t v;
  __device__ static KRank mx() { return {~0u}; }
  __device__ static KRank load(const KeySrc& s, uint32_t u) { return {s.rank[u]}; }
  using Raw = uint32_t;
  __device__ static Raw fetch(const KeySrc& s, uint32_t u) { return s.rank[u]; }
  __device__ static KRank finish(Raw x, const KeySrc&, uint32_t) { return {x}; }
  __device__ bool lt(const KRank& o) const { return v < o.v; }
  __device__ bool eq(const KRank& o) const { return v == o.v; }
  __device__ KRank sx(int m) const { return {shfl_xor32(v, m)}; }
  __device__ KRank sl(int l) const { return {shfl32(v, l)}; }
  __device__ KRank rl(int l) const { return {readlane32(v, l)}; }
  __device__ static KRank pick(bool c, const KRank& a, const KRank& b) { return {c ? a.v : b.v}; }
};

// Where a lane's credits go.  Hot nodes (member id kHotFlag | index) add into
// the workgroup's LDS counters; other nodes go through one pending
// (node, credit) pair per lane, which absorbs repeated credits to the same node
// (a leaf's root is usually its minimum, and a lane sees leaf after leaf of the
// same root), before a global atomic.
struct Sink {
  unsigned long long* hcnt;
  uint64_t* out;
  uint32_t pu;
  uint64_t pc;
  __device__ __forceinline__ void flush() {
    if (pc) {
      atomicAdd(reinterpret_cast<unsigned long long*>(out + pu), (unsigned long long)pc);
      pc = 0;
    }
  }
  __device__ __forceinline__ void add(uint32_t raw, uint64_t c) {
    if (raw & kHotFlag) {
      atomicAdd(&hcnt[raw & ~kHotFlag], (unsigned long long)c);
    } else if (raw == pu) {
      pc += c;
    } else {
      flush();
      pu = raw;
      pc = c;
    }
  }
};

// A member's key: from the hot table in LDS or from the loads in memory, each
// by its own unconditional load and the key chosen afterwards (a load in each
// arm of a choice becomes one flat load through a chosen pointer, and the
// wait for a flat load drains every load in flight).  A hot member reads the
// problem's first node (in bounds) and drops it.
template <class KT>
__device__ __forceinline__ KT member_key(const KeySrc& src, const KT* hkey, uint32_t raw) {
  const bool hot = (raw & kHotFlag) != 0;
  const KT g = KT::load(src, hot ? src.base : raw);
  const KT hk = hkey[raw & (kHotMax - 1)];
  return KT::pick(hot, hk, g);
}

// Gather modes of the lane-tile pass (every lane gathers a key for every row,
// with no lane mask; only the address of a hot or padding member differs):
// * Masked: it reads the problem's first node, one line shared by the
//   wavefront, so the gather costs the cache almost nothing (the right choice
//   when hot nodes hold most member occurrences).
// * Full: it reads its hot index as a node id (below the hot count, which
//   never exceeds n; padding is node 0).
// ----------------------------------------------------------------------------
// Leaf credit (paper: Algorithm 1's per-clique minimum-load step, batched per
// SCT leaf with the counts of Lemma 5).
//
// A leaf (H, P) with h = |H|, p = |P|, j = k - h holds the k-cliques H + C'
// (the header carries h, j and p, so leaves of problems with different k can
// share a launch; k1 is the row length of the binomial table),
// C' a j-subset of P.  Let m be the hold member with the smallest key.  The
// minimum of H + C' is m unless C' holds a pivot member below m; then it is
// the smallest such member u of C'.  With a(x) = the number of pivot members
// whose key exceeds x's:
//   pivot u below m gets C(a(u), j - 1);   m gets C(a(m), j);   others get 0.
// Pivot members below m are the "low" ones; a(u) = p - 1 - (number of low
// members below u), and a(m) = p - (number of low members).
// ----------------------------------------------------------------------------

// Data-parallel-primitive lane moves (DPP controls of the CDNA ISA).  Lanes
// whose source is outside the row (or outside the wavefront) read 0; rows
// left out by the row mask keep 0.
constexpr int kDppRowShr = 0x110;     // + n: lane l reads lane l - n of its row of 16
constexpr int kDppWaveShl1 = 0x130;   // lane l reads lane l + 1
constexpr int kDppWaveShr1 = 0x138;   // lane l reads lane l - 1
constexpr int kDppRowBcast15 = 0x142; // rows 1 and 3 (row mask 0xA) read lane 15 of the row before
constexpr int kDppRowBcast31 = 0x143; // rows 2 and 3 (row mask 0xC) read lane 31

template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xF, true);
}

// One step of a segmented inclusive scan: (vu, fu) is the partial sum and
// head flag of the lane the step reads (0, 0 where there is none).
template <int kCtrl, int kRowMask = 0xF>
__device__ __forceinline__ void seg_scan_step(uint64_t& v, uint32_t& f) {
  const uint32_t lo = dpp32<kCtrl, kRowMask>((uint32_t)v);
  const uint32_t hi = dpp32<kCtrl, kRowMask>((uint32_t)(v >> 32));
  const uint32_t fu = dpp32<kCtrl, kRowMask>(f);
  if (!f) {
    v += ((uint64_t)hi << 32) | lo;
    f |= fu;
  }
}

// Adds (key, val) of every lane to the sink after combining runs of adjacent
// lanes with the same key (a segmented inclusive scan over the wavefront): only
// the last lane of a run adds the run's total.  Lanes with val == 0 add nothing.
// The scan runs within rows of 16 lanes (shifts by 1, 2, 4, 8), then carries
// each row's open segment into the rows after it (the last lane of row 0 into
// rows 1 and 3, then the last lane of row 1 into rows 2 and 3), all as DPP
// lane moves.  Every lane of the wavefront must be active.
__device__ __forceinline__ void combine_add(Sink& sink, uint32_t key, uint64_t val) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t kp = dpp32<kDppWaveShr1>(key);
  const uint32_t head = (lane == 0 || kp != key) ? 1u : 0u;
  uint32_t f = head;
  uint64_t v = val;
  seg_scan_step<kDppRowShr + 1>(v, f);
  seg_scan_step<kDppRowShr + 2>(v, f);
  seg_scan_step<kDppRowShr + 4>(v, f);
  seg_scan_step<kDppRowShr + 8>(v, f);
  seg_scan_step<kDppRowBcast15, 0xA>(v, f);
  seg_scan_step<kDppRowBcast31, 0xC>(v, f);
  const uint32_t next_head = dpp32<kDppWaveShl1>(head);
  const bool run_end = lane == 63 || next_head;
  if (run_end && v) sink.add(key, v);
}

constexpr uint32_t kLaneBatch = 4;   // rows per lane-tile batch

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wavefront's heavy-leaf queue entries, staged in its LDS slice and copied
// to the global queue with one counter atomic per flush (at the end of the
// wavefront's tiles, or when the slice is full) instead of one per tile.  An
// entry carries what the heavy pass needs without looking the tile up again:
// the word of the leaf's first member (tile member base + lane), the leaf's
// header word and the first node id of its problem.
constexpr uint32_t kQueueBuf = 32;   // a tile with more heavy leaves writes them to the queue directly

struct WaveQueue {
  uint4* buf;      // the wavefront's kQueueBuf LDS entries
  uint32_t n;      // entries staged (wave-uniform)
  __device__ __forceinline__ void flush(uint4* __restrict__ queue, uint32_t* __restrict__ qcount) {
    if (n == 0) return;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(qcount, n);
    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
    wave_lds_sync();
    for (uint32_t i = lane; i < n; i += 64) queue[base + i] = buf[i];
    wave_lds_sync();   // the slice is reused only after every lane has read it
    n = 0;
  }
};

// Lane tile: one leaf per lane; member x of the lane's leaf is the row-x word
// of the column-major tile, so every row load below is one contiguous 256-byte
// row.  A single pass over the rows finds the hold minimum m (hold members come
// first in every leaf) and counts the pivot members below m.  The member words
// of the first low members go to the lane's four LDS slots (lcol[i * 256],
// written only by lanes that find one, so a row costs no register selects);
// lanes with at most four rank them from their keys, looked up again; leaves
// with more go to the heavy-leaf queue, or are taken up in place by the whole
// wavefront.  Keys are gathered for every row (a hot or padding member reads a
// harmless address, see the gather modes); hot keys come from LDS.
constexpr uint32_t kLeafThreads = 256;   // leaf-credit workgroup size (LDS slot stride)

// A tile descriptor's fields (and one padding word, see the leaf-credit loop).
__device__ __forceinline__ Tile load_tile(const Tile* __restrict__ tiles, uint32_t i) {
  const uint4 a = reinterpret_cast<const uint4*>(tiles + i)[0];
  Tile t{};
  t.mbase = ((uint64_t)a.y << 32) | a.x;
  t.lbase = a.z;
  t.info = a.w;
  t.nbase = reinterpret_cast<const uint32_t*>(tiles + i)[4];
  t.pad[0] = reinterpret_cast<const uint32_t*>(tiles + i)[5];
  return t;
}
// The heavy leaves of a lane tile (more than four pivot members below the
// hold minimum; heavy has bit c set for column c), taken by the whole
// wavefront up to four at a time: one member per lane (member x of column c
// is tile word c + 64 x), the hold minimum by a reduction over lanes 0..31
// (hold members come first, h <= 31), and each low member's rank among the
// low members by broadcasting their keys one at a time.  Only the low members
// are credited here; the lane tile credits the hold minimum.
template <class KT>
__device__ __forceinline__ void tile_heavy(uint64_t heavy, uint64_t mbase, uint32_t hd,
                                           const uint32_t* __restrict__ members, const uint64_t* binom, uint32_t k1,
                                           const KeySrc& src, const KT* hkey, Sink& sink) {
  constexpr uint32_t B = sizeof(KT) > 8 ? 2 : 4;   // (load, id) keys: two at a time (registers)
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t xoff = (uint64_t)64 * lane;
  while (heavy) {
    // a slot past the last heavy leaf reads column 0's first word and has
    // no members
    uint32_t hq[B], sq[B], jq[B], ra[B];
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) {
      const uint32_t c = heavy ? (uint32_t)__builtin_ctzll(heavy) : 0u;
      const uint32_t hdq = heavy ? readlane32(hd, (int)c) : 0u;
      heavy &= heavy - 1ull;
      hq[q] = hdq & 31u;
      jq[q] = (hdq >> 5) & 31u;
      sq[q] = hq[q] + (hdq >> 10);
      ra[q] = members[mbase + c + (lane < sq[q] ? xoff : 0ull)];
    }
    KT ka[B], kh[B];
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) ka[q] = member_key<KT>(src, hkey, ra[q]);
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) {
      ka[q] = KT::pick(lane < sq[q], ka[q], KT::mx());
      kh[q] = KT::pick(lane < hq[q], ka[q], KT::mx());
    }
#pragma unroll
    for (int d = 16; d >= 1; d >>= 1) {
#pragma unroll
      for (uint32_t q = 0; q < B; ++q) {
        const KT o = kh[q].sx(d);
        kh[q] = KT::pick(o.lt(kh[q]), o, kh[q]);
      }
    }
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) {
      const KT m = kh[q].rl(0);
      const bool low = lane < sq[q] && lane >= hq[q] && ka[q].lt(m);
      uint32_t below = 0;
      for (uint64_t bm = __ballot(low); bm; bm &= bm - 1ull) {
        const KT kt = ka[q].rl(__builtin_ctzll(bm));
        below += kt.lt(ka[q]) ? 1u : 0u;
      }
      const uint32_t p = sq[q] - hq[q], j = jq[q];
      if (low && j >= 1) {
        const uint64_t c = binom[(size_t)(p - 1 - below) * k1 + (j - 1)];
        if (c) sink.add(ra[q], c);
      }
    }
  }
}

template <class KT, bool kMasked>
__device__ __forceinline__ void tile_lane(const Tile& t, uint32_t tile_idx, const uint32_t* __restrict__ members,
                                          const uint32_t* __restrict__ hdr, const uint64_t* binom, uint32_t k1,
                                          const KeySrc& src, const KT* hkey, Sink& sink, uint4* __restrict__ queue,
                                          uint32_t* __restrict__ qcount, WaveQueue& hq, uint32_t* lcol,
                                          bool in_place) {
  constexpr uint32_t U = kLaneBatch;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t nl = (t.info >> 3) & 0x1FFFu, smax = t.info >> 16;
  const uint32_t* __restrict__ col = members + t.mbase + lane;
  // rows past the tile repeat its last; each batch's rows are requested
  // during the batch before, right after that batch's key gathers, so waiting
  // for those keys leaves the rows in flight.  The first batch's rows go out
  // before the headers, so the two requests overlap.
  uint32_t nxt[U];
#pragma unroll
  for (uint32_t u = 0; u < U; ++u) nxt[u] = col[(size_t)min(u, smax - 1) * 64];
  __builtin_amdgcn_sched_barrier(0);
  const uint32_t hd = lane < nl ? hdr[t.lbase + lane] : 0u;   // a missing leaf reads as empty
  const uint32_t h = hd & 31u, j = (hd >> 5) & 31u, p = hd >> 10, s = h + p;
  KT km = KT::mx();
  uint32_t mraw = 0, nlow = 0;
  for (uint32_t x0 = 0; x0 < smax; x0 += U) {
    uint32_t raw[U];
    KT key[U], hk[U];
    typename KT::Raw g[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) raw[u] = nxt[u];
    // Hot keys first (so every row has arrived before the first gather and no
    // gather waits behind a row), then every lane's gather with no lane mask
    // (so the compiler counts the loads in flight exactly), then the next
    // batch's rows; the keys are made only after that, so waiting for the
    // gathers leaves the rows in flight.  A hot or padding member gathers a
    // line shared by the wavefront (masked mode: the problem's first node) or
    // its hot index read as a node id (full mode), and takes its hot key.
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) hk[u] = hkey[raw[u] & (kHotMax - 1)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      uint32_t at = raw[u] & ~kHotFlag;
      if constexpr (kMasked) at = (x0 + u < s && !(raw[u] & kHotFlag)) ? raw[u] : src.base;
      g[u] = KT::fetch(src, at);
    }
    __builtin_amdgcn_sched_barrier(0);
    // unconditional (the last batch reads the tile's last row again)
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) nxt[u] = col[(size_t)min(x0 + U + u, smax - 1) * 64];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u)
      key[u] = KT::pick((raw[u] & kHotFlag) != 0, hk[u], KT::finish(g[u], src, raw[u] & ~kHotFlag));
    if (__ballot(x0 < h)) {
      // some lane still has hold rows here (hold members precede pivot
      // members, so m is final when a lane compares its first pivot member)
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t x = x0 + u;
        const bool hold = x < h;
        const bool better = hold && key[u].lt(km);
        km = KT::pick(better, key[u], km);
        mraw = better ? raw[u] : mraw;
        const bool take = !hold && x < s && key[u].lt(km);
        if (take) lcol[min(nlow, 3u) * kLeafThreads] = raw[u];
        nlow += take ? 1u : 0u;
      }
    } else {
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const bool take = x0 + u < s && key[u].lt(km);
        if (take) lcol[min(nlow, 3u) * kLeafThreads] = raw[u];
        nlow += take ? 1u : 0u;
      }
    }
  }
  if (nlow && nlow <= 4 && j >= 1) {
    // the low members' keys again (unused slots hold the maximum key), and
    // the rank of each among the low members
    const uint32_t r0 = lcol[0], r1 = lcol[kLeafThreads], r2 = lcol[2 * kLeafThreads], r3 = lcol[3 * kLeafThreads];
    // (all four read together; a slot past nlow holds a valid member word,
    // of this tile or an earlier one, and its key is replaced by the maximum)
    const KT l0 = member_key<KT>(src, hkey, r0);
    const KT l1 = KT::pick(nlow > 1, member_key<KT>(src, hkey, r1), KT::mx());
    const KT l2 = KT::pick(nlow > 2, member_key<KT>(src, hkey, r2), KT::mx());
    const KT l3 = KT::pick(nlow > 3, member_key<KT>(src, hkey, r3), KT::mx());
    const uint32_t b0 = (l1.lt(l0) ? 1u : 0u) + (l2.lt(l0) ? 1u : 0u) + (l3.lt(l0) ? 1u : 0u);
    const uint32_t b1 = (l0.lt(l1) ? 1u : 0u) + (l2.lt(l1) ? 1u : 0u) + (l3.lt(l1) ? 1u : 0u);
    const uint32_t b2 = (l0.lt(l2) ? 1u : 0u) + (l1.lt(l2) ? 1u : 0u) + (l3.lt(l2) ? 1u : 0u);
    const uint32_t b3 = (l0.lt(l3) ? 1u : 0u) + (l1.lt(l3) ? 1u : 0u) + (l2.lt(l3) ? 1u : 0u);
    // the four binomials read together (an unused slot reads row 0)
    const uint64_t* row = binom + (j - 1);
    const uint64_t c0 = row[(size_t)(p - 1 - b0) * k1];
    const uint64_t c1 = row[(size_t)(nlow > 1 ? p - 1 - b1 : 0u) * k1];
    const uint64_t c2 = row[(size_t)(nlow > 2 ? p - 1 - b2 : 0u) * k1];
    const uint64_t c3 = row[(size_t)(nlow > 3 ? p - 1 - b3 : 0u) * k1];
    sink.add(r0, c0);
    if (nlow > 1) sink.add(r1, c1);
    if (nlow > 2) sink.add(r2, c2);
    if (nlow > 3) sink.add(r3, c3);
  }
  // Leaves with more than four low members: in place, the whole wavefront
  // takes them up right away (the tile's rows are still in the caches);
  // otherwise they go to the heavy-leaf queue (through the wavefront's LDS
  // buffer), which the heavy kernel spreads over the grid.
  const uint64_t heavy = __ballot(nlow > 4);
  if (heavy) {
    if (in_place) {
      tile_heavy<KT>(heavy, t.mbase, hd, members, binom, k1, src, hkey, sink);
    } else {
      const uint32_t cnt = (uint32_t)__popcll(heavy);
      const uint32_t below = (uint32_t)__popcll(heavy & ((1ull << lane) - 1ull));
      const uint64_t mw = t.mbase + lane;
      const uint4 entry = make_uint4((uint32_t)mw, (uint32_t)(mw >> 32), hd, t.nbase);
      if (hq.n + cnt > kQueueBuf) hq.flush(queue, qcount);
      if (cnt > kQueueBuf) {
        // more than the slice holds: this tile's entries go to the queue at once
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(qcount, cnt);
        base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
        if (nlow > 4) queue[base + below] = entry;
      } else {
        if (nlow > 4) hq.buf[hq.n + below] = entry;
        hq.n += cnt;
      }
    }
  }
  const uint64_t cm = h ? binom[(size_t)(p - nlow) * k1 + j] : 0ull;
  combine_add(sink, cm ? mraw : 0xFFFFFFFFu, cm);
}

// Big tile: one leaf of more than 64 members per wavefront, in chunks of 64.
template <class KT>
__device__ __forceinline__ void tile_big(const Tile& t, const uint32_t* __restrict__ members,
                                         const uint32_t* __restrict__ hdr, const uint64_t* __restrict__ binom,
                                         uint32_t k1, const KeySrc& src, const KT* hkey, Sink& sink) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t hd = hdr[t.lbase];
  const uint32_t h = hd & 31u, j = (hd >> 5) & 31u, p = hd >> 10, s = h + p;
  const uint32_t* __restrict__ mem = members + t.mbase;
  // the hold members all sit in the first chunk (h <= 31)
  const uint32_t r0 = lane < s ? mem[lane] : 0u;
  const KT k0 = lane < s ? member_key<KT>(src, hkey, r0) : KT::mx();
  KT kh = lane < h ? k0 : KT::mx();
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const KT o = kh.sx(d);
    if (o.lt(kh)) kh = o;
  }
  uint32_t nlow = 0;
  for (uint32_t a0 = 0; a0 < s; a0 += 64) {
    const uint32_t ia = a0 + lane;
    const bool va = ia < s;
    const uint32_t ra = va ? mem[ia] : 0u;
    const KT ka = va ? member_key<KT>(src, hkey, ra) : KT::mx();
    const bool low = va && ia >= h && ka.lt(kh);
    const uint64_t lm = __ballot(low);
    nlow += (uint32_t)__popcll(lm);
    if (!lm) continue;
    uint32_t below = 0;
    for (uint32_t b0 = 0; b0 < s; b0 += 64) {
      const uint32_t ib = b0 + lane;
      const bool vb = ib < s && ib >= h;
      const KT kb = vb ? member_key<KT>(src, hkey, mem[ib]) : KT::mx();
      uint64_t bm = __ballot(vb && kb.lt(kh));   // low members of this chunk
      while (bm) {
        const int tl = __ffsll((unsigned long long)bm) - 1;
        const KT kt = kb.rl(tl);
        below += (low && kt.lt(ka)) ? 1u : 0u;
        bm &= bm - 1;
      }
    }
    if (low && j >= 1) {
      const uint64_t c = binom[(size_t)(p - 1 - below) * k1 + (j - 1)];
      if (c) sink.add(ra, c);
    }
  }
  if (lane < h && k0.eq(kh)) {
    const uint64_t c = binom[(size_t)(p - nlow) * k1 + j];
    if (c) sink.add(r0, c);
  }
}

// Strided grid: wave w of the grid takes tiles w, w + 4 * gridDim.x, ...
// (grids larger than the 2048 workgroups that stay resident shorten each
// wave's walk, and workgroups that start as others finish even out the
// tail).  Each workgroup adds its nonzero hot-node credit totals into one of
// kHotSlots scratch rows (row blockIdx.x % kHotSlots).
// Eight wavefronts per SIMD (<= 64 VGPRs, 18 KB of LDS per workgroup): the
// pass is latency-bound, and occupancy hides more of it than wider row
// batches do.
template <class KT, bool kMasked, bool kLdsBinom>
__global__ __launch_bounds__(256, 8) void leaf_credit_kernel(const Tile* __restrict__ tiles, uint32_t ntiles,
                                                          const uint32_t* __restrict__ members,
                                                          const uint32_t* __restrict__ hdr,
                                                          const uint64_t* __restrict__ binom, uint32_t nbinom,
                                                          uint32_t k1, KeySrc src, uint64_t* __restrict__ out,
                                                          const uint32_t* __restrict__ hot,
                                                          const uint32_t* __restrict__ hot_base, uint32_t nhot,
                                                          uint64_t* __restrict__ scratch, uint4* __restrict__ queue,
                                                          uint32_t* __restrict__ qcount, KT* __restrict__ hotkey,
                                                          bool hot_published, const uint32_t* __restrict__ xcd,
                                                          bool in_place) {
  __shared__ KT hkey[kHotMax];
  __shared__ unsigned long long hcnt[kHotMax];
  __shared__ uint64_t sbinom[kLdsBinom ? kBinomLds : 1];
  __shared__ uint4 qslice[4][kQueueBuf];
  __shared__ uint32_t lowslot[4 * kLeafThreads];   // four low-member slots per lane
  uint32_t* lcol = lowslot + threadIdx.x;
  for (uint32_t i = 0; i < 4; ++i) lcol[i * kLeafThreads] = 0u;   // node 0 until a lane writes its own
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // strided: every wavefront of the grid walks the whole list; XCD ranges
  // (xcd != null, grid of 8 or more workgroups): the workgroups with
  // blockIdx mod 8 = x walk range x = [xcd[x], xcd[x + 1]) in strides of
  // their own wavefront count, so every tile is still taken exactly once
  uint32_t tile = blockIdx.x * 4u + w, stride = gridDim.x * 4u, tend = ntiles;
  if (xcd && gridDim.x >= kXcds) {
    const uint32_t x = blockIdx.x % kXcds;
    tile = xcd[x] + (blockIdx.x / kXcds) * 4u + w;
    stride = ((gridDim.x - x + kXcds - 1) / kXcds) * 4u;
    tend = xcd[x + 1];
  }
  Tile t = tile < tend ? tiles[tile] : Tile{};   // in flight during the LDS set-up
  if (hot_published) {
    // the hot keys at these loads were written by the previous load update
    for (uint32_t i = threadIdx.x; i < nhot; i += blockDim.x) {
      hkey[i] = hotkey[i];
      hcnt[i] = 0;
    }
  } else {
    for (uint32_t i = threadIdx.x; i < nhot; i += blockDim.x) {
      KeySrc hs = src;
      hs.base = hot_base[i];
      hkey[i] = KT::load(hs, hot[i]);
      hcnt[i] = 0;
      if (blockIdx.x == 0) hotkey[i] = hkey[i];   // for the heavy pass
    }
  }
  if (kLdsBinom)
    for (uint32_t i = threadIdx.x; i < nbinom; i += blockDim.x) sbinom[i] = binom[i];
  __syncthreads();
  // the binomial table's memory space fixed at compile time (a pointer chosen
  // at run time would make flat loads, whose waits drain every load in flight)
  const uint64_t* bt = kLdsBinom ? sbinom : binom;
  Sink sink{hcnt, out, 0u, 0ull};
  WaveQueue hq{qslice[w], 0u};
  for (; tile < tend; tile += stride) {
    // the next tile's descriptor, in flight during this tile (scalar loads)
    const Tile tn = load_tile(tiles, min(tile + stride, tend - 1));
    KeySrc ts = src;
    ts.base = t.nbase;
    if ((t.info & 7u) == kTileBig) tile_big<KT>(t, members, hdr, bt, k1, ts, hkey, sink);
    else tile_lane<KT, kMasked>(t, tile, members, hdr, bt, k1, ts, hkey, sink, queue, qcount, hq, lcol, in_place);
    // the descriptor's last loaded word is kept alive to here, so its register
    // is not reused (and the load not waited for) while this tile runs
    asm volatile("" ::"s"(tn.pad[0]));
    t = tn;
  }
  sink.flush();
  // the heavy entries the four wavefronts still stage: one counter atomic for
  // the workgroup (thousands of wavefronts contending for one counter cost
  // more than the barrier)
  __shared__ uint32_t qn[4], qbase;
  if ((threadIdx.x & 63u) == 0) qn[w] = hq.n;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t staged = qn[0] + qn[1] + qn[2] + qn[3];
    qbase = staged ? atomicAdd(qcount, staged) : 0u;
  }
  __syncthreads();
  {
    uint32_t at = qbase;
    for (uint32_t x = 0; x < w; ++x) at += qn[x];
    for (uint32_t i = threadIdx.x & 63u; i < hq.n; i += 64) queue[at + i] = hq.buf[i];
  }
  // hot-node totals into slot blockIdx % kHotSlots of each node (nonzero ones only)
  const uint32_t slot = blockIdx.x % kHotSlots;
  for (uint32_t i = threadIdx.x; i < nhot; i += blockDim.x)
    if (hcnt[i]) atomicAdd(reinterpret_cast<unsigned long long*>(scratch + (size_t)i * kHotSlots + slot), hcnt[i]);
}

// Heavy leaves (more than four pivot members below the hold minimum), queued
// by the leaf-credit kernel as 16-byte entries: one leaf per wavefront, one
// member per lane, four leaves per batch (eight with kEight and 64-bit or
// smaller keys: more leaves in flight per wavefront at five wavefronts per
// SIMD instead of six, faster on queues of millions and slower on short ones,
// where fewer wavefronts then share the work), the batches pipelined.  The hold
// minimum m is recomputed; the low members' keys are compacted into LDS and
// each counts the smaller ones by broadcast reads.  Hot members' keys come
// from the table the leaf pass published; their credits add up in LDS and
// reach the nodes' slot entries (slot blockIdx.x % kHotSlots) once per
// workgroup.  Workgroups past the queue return at once.
template <class KT, bool kLdsBinom, bool kEight>
__global__ __launch_bounds__(256) void heavy_kernel(const uint32_t* __restrict__ members,
                                                    const uint64_t* __restrict__ binom, uint32_t k1, KeySrc src,
                                                    uint64_t* __restrict__ out, uint32_t nhot,
                                                    uint64_t* __restrict__ scratch, const uint4* __restrict__ queue,
                                                    const uint32_t* __restrict__ qcount,
                                                    const KT* __restrict__ hotkey, uint32_t nbinom) {
  constexpr uint32_t B = (kEight && sizeof(KT) <= 8) ? 8 : 4;
  __shared__ KT hkey[kHotMax];
  __shared__ unsigned long long hcnt[kHotMax];
  __shared__ uint64_t sbinom[kLdsBinom ? kHeavyBinomLds : 1];
  __shared__ KT lowk[4][B][64];   // per wavefront and queued leaf: its low members' keys, compacted
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t total = *qcount;
  const uint32_t nw = gridDim.x * 4u;
  if ((blockIdx.x * 4u) * B >= total) return;   // no entries for this workgroup (uniform)
  // member x of the queued leaf: its first word + 64 x
  const uint64_t xoff = (uint64_t)64 * lane;
  const uint32_t stride = nw * B;
  // The batches of a wavefront form a three-stage pipeline: while batch i's
  // keys are gathered and ranked, batch i + 1's member words and batch i + 2's
  // entries are in flight.  Lane q loads entry q of a batch (one vector load
  // per batch) and the fields are broadcast from it; lanes past a leaf read
  // the leaf's first word (in bounds) and drop it.  Batches past the queue
  // read its last entry and are not credited.
  auto entries = [&](uint32_t e0) -> uint4 {
    return queue[min(min(e0, total - 1) + min(lane, B - 1), total - 1)];
  };
  uint32_t hq1[B], sq1[B], jq1[B], nb1[B], wd1[B];
  auto words = [&](const uint4& ent) {
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) {
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)ent.x, q);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)ent.y, q);
      const uint32_t hd = (uint32_t)__builtin_amdgcn_readlane((int)ent.z, q);
      nb1[q] = (uint32_t)__builtin_amdgcn_readlane((int)ent.w, q);
      const uint64_t mw = ((uint64_t)hi << 32) | lo;
      hq1[q] = hd & 31u;
      jq1[q] = (hd >> 5) & 31u;
      sq1[q] = hq1[q] + (hd >> 10);
      wd1[q] = members[mw + (lane < sq1[q] ? xoff : 0ull)];
    }
  };
  const uint32_t first = (blockIdx.x * 4u + w) * B;
  uint4 ent2 = make_uint4(0u, 0u, 0u, 0u);
  if (first < total) {   // in flight during the LDS set-up
    words(entries(first));
    ent2 = entries(first + stride);
  }
  for (uint32_t i = threadIdx.x; i < nhot; i += blockDim.x) {
    hkey[i] = hotkey[i];
    hcnt[i] = 0;
  }
  if (kLdsBinom)
    for (uint32_t i = threadIdx.x; i < nbinom; i += blockDim.x) sbinom[i] = binom[i];
  __syncthreads();
  Sink sink{hcnt, out, 0u, 0ull};
  for (uint32_t e0 = first; e0 < total; e0 += stride) {
    uint32_t hq[B], sq[B], jq[B], ra[B], nb[B];
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) {
      hq[q] = hq1[q];
      sq[q] = sq1[q];
      jq[q] = jq1[q];
      nb[q] = nb1[q];
      ra[q] = lane < sq[q] ? wd1[q] : 0u;
    }
    // every lane gathers (a hot member's hot index and a missing member's 0
    // are node ids too), so the four gathers are in flight together; the LDS
    // key, or the maximum past the leaf, is selected afterwards
    KT ka[B];
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) {
      KeySrc ts = src;
      ts.base = nb[q];
      ka[q] = KT::load(ts, ra[q] & ~kHotFlag);
    }
    // the next batch's member words, and the entries of the one after (also
    // past the queue, unconditionally, so the wait for this batch's keys
    // below leaves them in flight)
    words(ent2);
    ent2 = entries(e0 + 2 * stride);
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) {
      ka[q] = KT::pick((ra[q] & kHotFlag) != 0, hkey[ra[q] & (kHotMax - 1)], ka[q]);
      ka[q] = KT::pick(lane < sq[q], ka[q], KT::mx());
    }
    // the hold minimum m of each leaf: the hold members are its first h <= 31
    // members, so lanes 0..31 hold them all; the B reductions are interleaved
    KT kh[B];
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) kh[q] = KT::pick(lane < hq[q], ka[q], KT::mx());
#pragma unroll
    for (int d = 16; d >= 1; d >>= 1) {
#pragma unroll
      for (uint32_t q = 0; q < B; ++q) {
        const KT o = kh[q].sx(d);
        kh[q] = KT::pick(o.lt(kh[q]), o, kh[q]);
      }
    }
    // the low members (pivot members below m) are compacted into LDS, and each
    // counts the smaller ones with broadcast reads
    bool low[B];
    uint32_t nlow[B];
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) {
      const KT m = kh[q].rl(0);
      low[q] = lane < sq[q] && lane >= hq[q] && ka[q].lt(m);
      const uint64_t bm = __ballot(low[q]);
      nlow[q] = (uint32_t)__popcll(bm);
      if (low[q]) lowk[w][q][__popcll(bm & ((1ull << lane) - 1ull))] = ka[q];
    }
    wave_lds_sync();
#pragma unroll
    for (uint32_t q = 0; q < B; ++q) {
      if (e0 + q >= total) break;
      uint32_t below = 0;
#pragma unroll 4
      for (uint32_t i = 0; i < nlow[q]; ++i) below += lowk[w][q][i].lt(ka[q]) ? 1u : 0u;
      const uint32_t p = sq[q] - hq[q], j = jq[q];
      if (low[q] && j >= 1) {
        // the table from LDS or from memory, chosen at compile time (a
        // pointer chosen at run time would make a flat load, whose wait would
        // also drain the next batches' loads)
        const size_t bi = (size_t)(p - 1 - below) * k1 + (j - 1);
        const uint64_t c = kLdsBinom ? sbinom[bi] : binom[bi];
        if (c) sink.add(ra[q], c);
      }
    }
    wave_lds_sync();   // the slices are rewritten by the next batch
  }
  sink.flush();
  __syncthreads();
  const uint32_t slot = blockIdx.x % kHotSlots;
  for (uint32_t i = threadIdx.x; i < nhot; i += blockDim.x)
    if (hcnt[i]) atomicAdd(reinterpret_cast<unsigned long long*>(scratch + (size_t)i * kHotSlots + slot), hcnt[i]);
}

// ----------------------------------------------------------------------------
// PBUpdate (paper: Algorithm 3), synchronous over the pairs (leaves) of the
// tree: every leaf reads r_{t-1} and its allocation goes into out.
//
// A leaf with h hold and p pivot members holds n_C = C(p, j) k-cliques,
// j = k - h; member x may receive at most cap(x) = n_C (hold) or C(p - 1, j - 1)
// (pivot), the number of the leaf's cliques that contain it.  The algorithm's
// plateau steps raise the lowest loads first, equally, within the caps; they end
// at a level L: every member gets min(cap, max(0, L - r)), and the n_C - S(L)
// cliques left over (fewer than the members still below both L + 1 and their
// caps) go one each to the lowest ids among those.  Here L is found in closed
// form: S(L) = sum over members of min(cap, max(0, L - r)) is piecewise linear
// with breakpoints r(x) and r(x) + cap(x); b0 = the largest breakpoint with
// S(b0) <= n_C; sigma = the members growing just above b0; then
// L = b0 + floor((n_C - S(b0)) / sigma) and the remainder is
// (n_C - S(b0)) mod sigma.
// ----------------------------------------------------------------------------

// S(L) saturated at n_C + 1 (only S <= n_C matters), over members
// x = x0, x0 + dx, .. < s whose loads are lr[x * stride].
__device__ __forceinline__ uint64_t pb_level_sum(const uint64_t* lr, uint32_t stride, uint32_t x0, uint32_t dx,
                                                 uint32_t s, uint32_t h, uint64_t nC, uint64_t cp, uint64_t L) {
  const uint64_t sat = nC + 1;   // n_C < 2^64 - 1: the plan keeps r_0 + T c_k below 2^64
  uint64_t S = 0;
#pragma unroll 4
  for (uint32_t x = x0; x < s; x += dx) {
    const uint64_t rx = lr[(size_t)x * stride];
    const uint64_t cap = x < h ? nC : cp;
    const uint64_t term = L > rx ? min(cap, L - rx) : 0ull;
    S = term > sat - S ? sat : S + term;   // saturating, never wraps (S <= sat)
  }
  return S;
}

// A member's load: from the hot table in LDS or the load array in memory,
// each by its own unconditional load and the value chosen afterwards (a load
// in each arm of a choice becomes one flat load through a chosen pointer,
// whose wait drains every load in flight).  Hot members read r[0] (in bounds)
// and drop it.
__device__ __forceinline__ uint64_t pb_member_load(const uint64_t* __restrict__ r, const uint64_t* hr, uint32_t raw) {
  const bool hot = (raw & kHotFlag) != 0;
  const uint64_t g = r[hot ? 0u : raw];
  const uint64_t hv = hr[raw & (kHotMax - 1)];
  return hot ? hv : g;
}

__device__ __forceinline__ uint32_t pb_node_id(uint32_t raw, const uint32_t* hid) {
  return (raw & kHotFlag) ? hid[raw & (kHotMax - 1)] : raw;
}

// One leaf per lane: lr (LDS) and lm (the tile's member words in memory) hold
// the lane's column (member x at x * 64).
__device__ __forceinline__ void pb_leaf_lane(const uint64_t* lr, const uint32_t* lm, uint32_t h, uint32_t p,
                                             uint64_t nC, uint64_t cp, const uint32_t* hid, Sink& sink) {
  const uint32_t s = h + p;
  if (s == 0 || nC == 0) return;
  uint64_t b0 = ~0ull, top = 0;
  for (uint32_t x = 0; x < s; ++x) {
    b0 = min(b0, lr[(size_t)x * 64]);   // S(min r) = 0
    top = max(top, lr[(size_t)x * 64]);
  }
  if (s <= 16) {
    // small leaves: every breakpoint r(x), r(x) + cap(x) in turn
    for (uint32_t y = 0; y < s; ++y) {
      const uint64_t ry = lr[(size_t)y * 64];
      if (ry > b0 && pb_level_sum(lr, 64, 0, 1, s, h, nC, cp, ry) <= nC) b0 = ry;
      if (y >= h) {
        const uint64_t c = ry + cp;
        if (c > b0 && pb_level_sum(lr, 64, 0, 1, s, h, nC, cp, c) <= nC) b0 = c;
      }
    }
  } else {
    // larger leaves: bisection on the level itself, S(lo) <= n_C < S(hi)
    // (at max r + n_C + 1 every member is at its cap, and the caps sum to
    // k n_C > n_C); the level found is the largest with S <= n_C, so the
    // closing steps below give the same allocation
    uint64_t lo = b0, hi = top + nC + 1;
    while (hi - lo > 1) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if (pb_level_sum(lr, 64, 0, 1, s, h, nC, cp, mid) <= nC) lo = mid;
      else hi = mid;
    }
    b0 = lo;
  }
  uint64_t S0 = 0;
  uint32_t sigma = 0;
  for (uint32_t x = 0; x < s; ++x) {
    const uint64_t rx = lr[(size_t)x * 64], cap = x < h ? nC : cp;
    if (b0 > rx) S0 += min(cap, b0 - rx);
    sigma += (rx <= b0 && b0 - rx < cap) ? 1u : 0u;
  }
  sigma = max(sigma, 1u);   // at least one member grows above b0 whenever n_C > 0
  const uint64_t L = b0 + (nC - S0) / sigma, R = (nC - S0) % sigma;
  for (uint32_t x = 0; x < s; ++x) {
    const uint64_t rx = lr[(size_t)x * 64], cap = x < h ? nC : cp;
    uint64_t inc = L > rx ? min(cap, L - rx) : 0ull;
    if (R && rx <= L && L - rx < cap) {
      // rank of this member's id among the members still growing at L
      const uint32_t id = pb_node_id(lm[(size_t)x * 64], hid);
      uint32_t below = 0;
      for (uint32_t y = 0; y < s; ++y) {
        const uint64_t ry = lr[(size_t)y * 64], cy = y < h ? nC : cp;
        below += (ry <= L && L - ry < cy && pb_node_id(lm[(size_t)y * 64], hid) < id) ? 1u : 0u;
      }
      inc += below < R ? 1u : 0u;
    }
    if (inc) sink.add(lm[(size_t)x * 64], inc);
  }
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v = max(v, shfl_xor64(v, d));
  return v;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v = min(v, shfl_xor64(v, d));
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v += shfl_xor64(v, d);
  return v;
}

// One leaf of more than 64 members per wavefront: lr (LDS) and lm (memory)
// hold its members contiguously (member x at x); lane l owns members l, l + 64, ..
__device__ __forceinline__ void pb_leaf_wave(const uint64_t* lr, const uint32_t* lm, uint32_t h, uint32_t p,
                                             uint64_t nC, uint64_t cp, const uint32_t* hid, Sink& sink) {
  const uint32_t lane = threadIdx.x & 63u, s = h + p;
  if (s == 0 || nC == 0) return;
  uint64_t m = ~0ull;
  for (uint32_t x = lane; x < s; x += 64) m = min(m, lr[x]);
  uint64_t b0 = wave_min_u64(m);
  uint64_t best = b0;
  for (uint32_t y = lane; y < s; y += 64) {
    const uint64_t ry = lr[y];
    if (ry > best && pb_level_sum(lr, 1, 0, 1, s, h, nC, cp, ry) <= nC) best = ry;
    if (y >= h) {
      const uint64_t c = ry + cp;
      if (c > best && pb_level_sum(lr, 1, 0, 1, s, h, nC, cp, c) <= nC) best = c;
    }
  }
  b0 = wave_max_u64(best);
  uint64_t S0 = 0, sg = 0;
  for (uint32_t x = lane; x < s; x += 64) {
    const uint64_t rx = lr[x], cap = x < h ? nC : cp;
    if (b0 > rx) S0 += min(cap, b0 - rx);
    sg += (rx <= b0 && b0 - rx < cap) ? 1u : 0u;
  }
  S0 = wave_sum_u64(S0);
  const uint64_t sigma = max(wave_sum_u64(sg), (uint64_t)1);
  const uint64_t L = b0 + (nC - S0) / sigma, R = (nC - S0) % sigma;
  for (uint32_t x = lane; x < s; x += 64) {
    const uint64_t rx = lr[x], cap = x < h ? nC : cp;
    uint64_t inc = L > rx ? min(cap, L - rx) : 0ull;
    if (R && rx <= L && L - rx < cap) {
      const uint32_t id = pb_node_id(lm[x], hid);
      uint64_t below = 0;
      for (uint32_t y = 0; y < s; ++y) {
        const uint64_t ry = lr[y], cy = y < h ? nC : cp;
        below += (ry <= L && L - ry < cy && pb_node_id(lm[y], hid) < id) ? 1u : 0u;
      }
      inc += below < R ? 1u : 0u;
    }
    if (inc) sink.add(lm[x], inc);
  }
}

// Four wavefronts per workgroup.  The first `nbig` workgroups take one tile
// each of tiles 0 .. nbig - 1 (big leaves and lane tiles of more than
// kPbMidRows rows) on their first wavefront, staged in the whole dynamic LDS;
// the others take tiles nbig .. ntiles - 1, wavefront w of workgroup nbig + b
// taking tiles nbig + 4 b + w, + 4 (gridDim.x - nbig), .., each staged in its
// own region of `rows` rows (one launch, so the large tiles' long searches
// overlap the rest).  A lane tile stages its members' loads (u64) in rows of
// 64 (each lane then reads only its own column), a big leaf its members' loads
// contiguously.  Member words are read from memory (a lane tile's rows are
// contiguous).  Hot loads, ids and credit totals live in static LDS, shared by
// the workgroup; the totals reach the hot nodes' slot entries at the end, as
// in the leaf-credit pass.
__global__ __launch_bounds__(256) void pb_kernel(const Tile* __restrict__ tiles, uint32_t nbig, uint32_t ntiles,
                                                 const uint32_t* __restrict__ members,
                                                 const uint32_t* __restrict__ hdr,
                                                 const uint64_t* __restrict__ binom, uint32_t k1,
                                                 const uint64_t* __restrict__ r, const uint32_t* __restrict__ hot,
                                                 uint32_t nhot, uint64_t* __restrict__ out,
                                                 uint64_t* __restrict__ scratch, uint32_t rows) {
  extern __shared__ uint64_t pb_lds[];
  __shared__ uint64_t hr[kHotMax];
  __shared__ uint32_t hid[kHotMax];
  __shared__ unsigned long long hcnt[kHotMax];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const bool big = blockIdx.x < nbig;
  uint64_t* lr = big ? pb_lds : pb_lds + (size_t)w * rows * 64;
  // this wavefront's tiles: one large tile, or every (4 (gridDim.x - nbig))-th from its start
  uint32_t tile = big ? (w == 0 ? blockIdx.x : ntiles) : nbig + (blockIdx.x - nbig) * 4u + w;
  const uint32_t step = big ? ntiles : (gridDim.x - nbig) * 4u;
  for (uint32_t i = threadIdx.x; i < nhot; i += blockDim.x) {
    hid[i] = hot[i];
    hr[i] = r[hot[i]];
    hcnt[i] = 0;
  }
  __syncthreads();
  Sink sink{hcnt, out, 0u, 0ull};
  for (; tile < ntiles; tile += step) {
    const Tile t = tiles[tile];
    const uint32_t smax = t.info >> 16;
    if ((t.info & 7u) == kTileBig) {
      const uint32_t hd = hdr[t.lbase];
      const uint32_t h = hd & 31u, j = (hd >> 5) & 31u, p = hd >> 10, sz = h + p;
      const uint32_t* lm = members + t.mbase;
      wave_lds_sync();   // the previous tile's reads are done
      for (uint32_t x = lane; x < sz; x += 64) {
        const uint32_t raw = lm[x];
        lr[x] = pb_member_load(r, hr, raw);
      }
      wave_lds_sync();
      const uint64_t nC = binom[(size_t)p * k1 + j], cp = j ? binom[(size_t)(p - 1) * k1 + (j - 1)] : 0ull;
      pb_leaf_wave(lr, lm, h, p, nC, cp, hid, sink);
    } else {
      const uint32_t nl = (t.info >> 3) & 0x1FFFu;
      const uint32_t hd = lane < nl ? hdr[t.lbase + lane] : 0u;   // a missing leaf reads as empty
      const uint32_t h = hd & 31u, j = (hd >> 5) & 31u, p = hd >> 10;
      const uint32_t* col = members + t.mbase + lane;
      wave_lds_sync();
      for (uint32_t x = 0; x < smax; ++x) {
        const uint32_t raw = col[(size_t)x * 64];
        lr[(size_t)x * 64 + lane] = pb_member_load(r, hr, raw);
      }
      const uint64_t nC = hd ? binom[(size_t)p * k1 + j] : 0ull;
      const uint64_t cp = (hd && j) ? binom[(size_t)(p - 1) * k1 + (j - 1)] : 0ull;
      pb_leaf_lane(lr + lane, col, h, p, nC, cp, hid, sink);
    }
  }
  sink.flush();
  __syncthreads();
  const uint32_t slot = blockIdx.x % kHotSlots;
  for (uint32_t i = threadIdx.x; i < nhot; i += blockDim.x)
    if (hcnt[i]) atomicAdd(reinterpret_cast<unsigned long long*>(scratch + (size_t)i * kHotSlots + slot), hcnt[i]);
}

// The same for lane tiles of at most SM rows, the members' loads and words in
// registers (loops unrolled over SM, masked to the leaf's s members).
template <int SM>
__device__ __forceinline__ uint64_t pb_level_sum_reg(const uint64_t (&rv)[SM], uint32_t s, uint32_t h, uint64_t nC,
                                                     uint64_t cp, uint64_t L) {
  const uint64_t sat = nC + 1;
  uint64_t S = 0;
#pragma unroll
  for (int x = 0; x < SM; ++x) {
    const uint64_t cap = (uint32_t)x < h ? nC : cp;
    const uint64_t term = ((uint32_t)x < s && L > rv[x]) ? min(cap, L - rv[x]) : 0ull;
    S = term > sat - S ? sat : S + term;
  }
  return S;
}

template <int SM>
__device__ __forceinline__ void pb_tile_reg(const Tile& t, const uint32_t* __restrict__ members,
                                            const uint32_t* __restrict__ hdr, const uint64_t* __restrict__ binom,
                                            uint32_t k1, const uint64_t* __restrict__ r, const uint64_t* hr,
                                            const uint32_t* hid, Sink& sink) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t nl = (t.info >> 3) & 0x1FFFu, smax = t.info >> 16;
  const uint32_t hd = lane < nl ? hdr[t.lbase + lane] : 0u;
  const uint32_t h = hd & 31u, j = (hd >> 5) & 31u, p = hd >> 10, s = h + p;
  const uint32_t* col = members + t.mbase + lane;
  uint32_t raw[SM];
  uint64_t rv[SM];
#pragma unroll
  for (int x = 0; x < SM; ++x) raw[x] = (uint32_t)x < smax ? col[(size_t)x * 64] : 0u;
#pragma unroll
  for (int x = 0; x < SM; ++x) rv[x] = pb_member_load(r, hr, raw[x]);
  const uint64_t nC = hd ? binom[(size_t)p * k1 + j] : 0ull;
  const uint64_t cp = (hd && j) ? binom[(size_t)(p - 1) * k1 + (j - 1)] : 0ull;
  if (s == 0 || nC == 0) return;
  uint64_t b0 = ~0ull, top = 0;
#pragma unroll
  for (int x = 0; x < SM; ++x)
    if ((uint32_t)x < s) {
      b0 = min(b0, rv[x]);
      top = max(top, rv[x]);
    }
  if (SM <= 16) {
    // breakpoints r(y), r(y) + cap(y) in turn; the candidate is selected out of
    // the register array (a runtime index would put the array in scratch)
#pragma unroll 1
    for (uint32_t y = 0; y < s; ++y) {
      uint64_t ry = 0;
#pragma unroll
      for (int x = 0; x < SM; ++x) ry = (uint32_t)x == y ? rv[x] : ry;
      if (ry > b0 && pb_level_sum_reg<SM>(rv, s, h, nC, cp, ry) <= nC) b0 = ry;
      const uint64_t c = ry + cp;
      if (y >= h && c > b0 && pb_level_sum_reg<SM>(rv, s, h, nC, cp, c) <= nC) b0 = c;
    }
  } else {
    uint64_t lo = b0, hi = top + nC + 1;
    while (hi - lo > 1) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if (pb_level_sum_reg<SM>(rv, s, h, nC, cp, mid) <= nC) lo = mid;
      else hi = mid;
    }
    b0 = lo;
  }
  uint64_t S0 = 0;
  uint32_t sigma = 0;
#pragma unroll
  for (int x = 0; x < SM; ++x) {
    const uint64_t cap = (uint32_t)x < h ? nC : cp;
    if ((uint32_t)x < s) {
      if (b0 > rv[x]) S0 += min(cap, b0 - rv[x]);
      sigma += (rv[x] <= b0 && b0 - rv[x] < cap) ? 1u : 0u;
    }
  }
  sigma = max(sigma, 1u);
  const uint64_t L = b0 + (nC - S0) / sigma, R = (nC - S0) % sigma;
  // members still growing at L, with their node ids (the remainder goes to the lowest)
  uint32_t gid[SM];
#pragma unroll
  for (int x = 0; x < SM; ++x) {
    const uint64_t cap = (uint32_t)x < h ? nC : cp;
    const bool grow = (uint32_t)x < s && rv[x] <= L && L - rv[x] < cap;
    gid[x] = grow ? pb_node_id(raw[x], hid) : ~0u;   // ~0u: not growing (ids stay below it)
  }
#pragma unroll
  for (int x = 0; x < SM; ++x) {
    if ((uint32_t)x >= s) continue;
    const uint64_t cap = (uint32_t)x < h ? nC : cp;
    uint64_t inc = L > rv[x] ? min(cap, L - rv[x]) : 0ull;
    if (R && gid[x] != ~0u) {
      uint32_t below = 0;
#pragma unroll
      for (int y = 0; y < SM; ++y) below += gid[y] < gid[x] ? 1u : 0u;
      inc += below < R ? 1u : 0u;
    }
    if (inc) sink.add(raw[x], inc);
  }
}

// Lane tiles of at most kPbRegRows rows (a suffix of the tile list, which runs from the
// largest size group to the smallest): four wavefronts per workgroup, wavefront
// w takes tiles first + w, first + w + 4 gridDim.x, ..; no staging in LDS.
__global__ __launch_bounds__(256) void pb_reg_kernel(const Tile* __restrict__ tiles, uint32_t first, uint32_t ntiles,
                                                     const uint32_t* __restrict__ members,
                                                     const uint32_t* __restrict__ hdr,
                                                     const uint64_t* __restrict__ binom, uint32_t k1,
                                                     const uint64_t* __restrict__ r, const uint32_t* __restrict__ hot,
                                                     uint32_t nhot, uint64_t* __restrict__ out,
                                                     uint64_t* __restrict__ scratch) {
  __shared__ uint64_t hr[kHotMax];
  __shared__ uint32_t hid[kHotMax];
  __shared__ unsigned long long hcnt[kHotMax];
  for (uint32_t i = threadIdx.x; i < nhot; i += blockDim.x) {
    hid[i] = hot[i];
    hr[i] = r[hot[i]];
    hcnt[i] = 0;
  }
  __syncthreads();
  Sink sink{hcnt, out, 0u, 0ull};
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (uint32_t tile = first + blockIdx.x * 4u + w; tile < ntiles; tile += gridDim.x * 4u) {
    const Tile t = tiles[tile];
    const uint32_t smax = t.info >> 16;
    if (smax <= 8) pb_tile_reg<8>(t, members, hdr, binom, k1, r, hr, hid, sink);
    else pb_tile_reg<16>(t, members, hdr, binom, k1, r, hr, hid, sink);
  }
  sink.flush();
  __syncthreads();
  const uint32_t slot = blockIdx.x % kHotSlots;
  for (uint32_t i = threadIdx.x; i < nhot; i += blockDim.x)
    if (hcnt[i]) atomicAdd(reinterpret_cast<unsigned long long*>(scratch + (size_t)i * kHotSlots + slot), hcnt[i]);
}

// Hot-node totals: out[hot[i]] += the sum of hot node i's kHotSlots slot
// entries (contiguous: slot b of node i is scratch[i * kHotSlots + b]), and the
// entries are cleared for the next pass (each is read exactly once).  One
// wavefront per hot node; block 0 also empties the heavy-leaf queue.
__global__ __launch_bounds__(256) void hot_reduce_kernel(uint64_t* __restrict__ scratch,
                                                         const uint32_t* __restrict__ hot, uint32_t nhot,
                                                         uint64_t* __restrict__ out, uint32_t* __restrict__ qcount,
                                                         uint32_t* __restrict__ qlog) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (qlog) *qlog = *qcount;   // timed runs keep the queue size
    *qcount = 0;                 // heavy queue emptied
  }
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t i = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (i >= nhot) return;
  uint64_t* e = scratch + (size_t)i * kHotSlots;
  uint64_t t = 0;
  for (uint32_t b = lane; b < kHotSlots; b += 64) {
    t += e[b];
    e[b] = 0;
  }
  for (int d = 32; d >= 1; d >>= 1) t += shfl_xor64(t, d);
  if (lane == 0 && t) atomicAdd(reinterpret_cast<unsigned long long*>(out + hot[i]), (unsigned long long)t);
}

// ----------------------------------------------------------------------------
// Load update r_t = r_{t-1} + d_t (Algorithm 1's unit increments summed over
// the iteration), and its start.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fill_u64_kernel(uint64_t* a, uint64_t v, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void reset_result_kernel(DevResult* d) {
  if (threadIdx.x == 0) {
    d->dens_num = 0;
    d->size = 0;
    d->pad0 = 0;
    d->ub_lo = d->ub_hi = 0;
    d->r0max = 0;
    d->pad1[0] = d->pad1[1] = d->pad1[2] = 0;
    d->tb_lo = d->tb_hi = 0;
    d->tb_size = 0;
  }
}

__global__ __launch_bounds__(256) void init_loads_kernel(const uint64_t* __restrict__ r0, uint64_t* __restrict__ r,
                                                         uint64_t* __restrict__ delta, uint32_t n, int wide,
                                                         DevResult* dres) {
  uint64_t mx = 0;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    const uint64_t x = r0 ? r0[u] : 0ull;
    mx = x > mx ? x : mx;
    if (wide) {
      r[2ull * u] = x;
      r[2ull * u + 1] = 0;
    } else {
      r[u] = x;
    }
    delta[u] = 0;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = shfl_xor64(mx, d);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & 63u) == 0 && mx) atomicMax(reinterpret_cast<unsigned long long*>(&dres->r0max), (unsigned long long)mx);
}

__global__ __launch_bounds__(256) void apply64_kernel(uint64_t* __restrict__ r, uint64_t* __restrict__ delta,
                                                      uint32_t n) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    r[u] += delta[u];
    delta[u] = 0;
  }
}

// Key of hot node i (node u of the problem starting at base) at load v into
// the table the next leaf pass reads: packed (key_mode 0) or (load, id).
__device__ __forceinline__ void publish_hot_key(uint64_t* __restrict__ table, uint32_t i, uint64_t v, uint32_t u,
                                                uint32_t base, int key_mode, uint32_t id_bits) {
  if (key_mode == 0) {
    table[i] = (v << id_bits) | (u - base);
  } else {
    KFull* t = reinterpret_cast<KFull*>(table);
    t[i] = KFull{v, u};
  }
}

// The hot-node key table at the start loads of a run (64-bit loads).
__global__ __launch_bounds__(256) void hot_keys_kernel(const uint64_t* __restrict__ r, const uint32_t* __restrict__ hot,
                                                       const uint32_t* __restrict__ hot_base, uint32_t nhot,
                                                       int key_mode, uint32_t id_bits, uint64_t* __restrict__ table) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nhot) publish_hot_key(table, i, r[hot[i]], hot[i], hot_base[i], key_mode, id_bits);
}

// The load update fused with the hot-node reduction (64-bit loads): the first
// ceil(nhot / 4) workgroups give each hot node i a wavefront that sums and
// clears its kHotSlots slot entries, adds the total to r[hot[i]] and writes
// the node's new key into the hot-key table of the next leaf pass; the other
// workgroups apply the credits pairwise, writing only the entries whose credit
// is nonzero.  Hot nodes never have one (their credits live in slot entries),
// so the two parts never touch the same word and r[hot[i]] is written by its
// wavefront alone.  Also empties the heavy-leaf queue, keeping its size in
// *qlog for timed runs.
__global__ __launch_bounds__(256) void apply64_hot_kernel(uint64_t* __restrict__ r, uint64_t* __restrict__ delta,
                                                          uint32_t n, uint64_t* __restrict__ scratch,
                                                          const uint32_t* __restrict__ hot,
                                                          const uint32_t* __restrict__ hot_base, uint32_t nhot,
                                                          uint32_t hot_blocks, uint32_t* __restrict__ qcount,
                                                          uint32_t* __restrict__ qlog, int key_mode, uint32_t id_bits,
                                                          uint64_t* __restrict__ hot_table) {
  const uint32_t lane = threadIdx.x & 63u;
  if (blockIdx.x < hot_blocks) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (qlog) *qlog = *qcount;
      *qcount = 0;
    }
    const uint32_t i = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (i >= nhot) return;
    uint64_t* e = scratch + (size_t)i * kHotSlots;
    uint64_t t = 0;
    for (uint32_t b = lane; b < kHotSlots; b += 64) {
      t += e[b];
      e[b] = 0;
    }
    for (int d = 32; d >= 1; d >>= 1) t += shfl_xor64(t, d);
    if (lane == 0) {
      const uint32_t u = hot[i];
      const uint64_t v = r[u] + t;
      if (t) r[u] = v;
      publish_hot_key(hot_table, i, v, u, hot_base[i], key_mode, id_bits);
    }
    return;
  }
  const uint32_t pairs = n / 2;
  const ulonglong2* d2 = reinterpret_cast<const ulonglong2*>(delta);
  const uint32_t nb = gridDim.x - hot_blocks, b = blockIdx.x - hot_blocks;
  for (uint32_t k = b * blockDim.x + threadIdx.x; k < pairs; k += nb * blockDim.x) {
    const ulonglong2 d = d2[k];
    if (d.x) {
      r[2 * k] += d.x;
      delta[2 * k] = 0;
    }
    if (d.y) {
      r[2 * k + 1] += d.y;
      delta[2 * k + 1] = 0;
    }
  }
  if ((n & 1u) && b == 0 && threadIdx.x == 0 && delta[n - 1]) {
    r[n - 1] += delta[n - 1];
    delta[n - 1] = 0;
  }
}

// The same on 16-byte pairs (r and delta 16-byte aligned): the credits are
// read for every pair, the loads are read and written, and the credits
// cleared, only where a credit arrived.
__global__ __launch_bounds__(256) void apply64_pairs_kernel(uint64_t* __restrict__ r, uint64_t* __restrict__ delta,
                                                            uint32_t n) {
  const uint32_t pairs = n / 2;
  ulonglong2* r2 = reinterpret_cast<ulonglong2*>(r);
  ulonglong2* d2 = reinterpret_cast<ulonglong2*>(delta);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < pairs; i += gridDim.x * blockDim.x) {
    const ulonglong2 d = d2[i];
    if (d.x | d.y) {
      ulonglong2 v = r2[i];
      v.x += d.x;
      v.y += d.y;
      r2[i] = v;
      d2[i] = make_ulonglong2(0ull, 0ull);
    }
  }
  if ((n & 1u) && blockIdx.x == 0 && threadIdx.x == 0) {
    r[n - 1] += delta[n - 1];
    delta[n - 1] = 0;
  }
}

__global__ __launch_bounds__(256) void apply128_kernel(uint64_t* __restrict__ r, uint64_t* __restrict__ delta,
                                                       uint32_t n) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    const uint64_t d = delta[u];
    const uint64_t lo = r[2ull * u] + d;
    r[2ull * u] = lo;
    r[2ull * u + 1] += (lo < d) ? 1ull : 0ull;
    delta[u] = 0;
  }
}

// ----------------------------------------------------------------------------
// Maxima: max_u (r(u) - sub(u)) as a 128-bit value (sub may be null).
// ----------------------------------------------------------------------------
__device__ __forceinline__ bool gt128(uint64_t ah, uint64_t al, uint64_t bh, uint64_t bl) {
  return ah > bh || (ah == bh && al > bl);
}

__global__ __launch_bounds__(256) void max_partial_kernel(const uint64_t* __restrict__ r, const uint64_t* __restrict__ sub,
                                                          uint32_t n, int wide, uint64_t* __restrict__ red) {
  __shared__ uint64_t sh[4], sl[4];
  uint64_t bh = 0, bl = 0;
  const uint32_t base = blockIdx.x * kRedTile;
  for (uint32_t i = threadIdx.x; i < kRedTile; i += blockDim.x) {
    const uint32_t u = base + i;
    if (u >= n) break;
    uint64_t lo = wide ? r[2ull * u] : r[u];
    uint64_t hi = wide ? r[2ull * u + 1] : 0ull;
    if (sub) {
      const uint64_t s = sub[u];
      hi -= (lo < s) ? 1ull : 0ull;
      lo -= s;
    }
    if (gt128(hi, lo, bh, bl)) { bh = hi; bl = lo; }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t oh = shfl_xor64(bh, d), ol = shfl_xor64(bl, d);
    if (gt128(oh, ol, bh, bl)) { bh = oh; bl = ol; }
  }
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0) { sh[w] = bh; sl[w] = bl; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t x = 1; x < blockDim.x / 64; ++x)
      if (gt128(sh[x], sl[x], bh, bl)) { bh = sh[x]; bl = sl[x]; }
    red[2ull * blockIdx.x] = bl;
    red[2ull * blockIdx.x + 1] = bh;
  }
}

__global__ __launch_bounds__(256) void max_final_kernel(const uint64_t* __restrict__ red, uint32_t nb,
                                                        uint64_t* out_lo, uint64_t* out_hi) {
  __shared__ uint64_t sh[4], sl[4];
  uint64_t bh = 0, bl = 0;
  for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x)
    if (gt128(red[2ull * i + 1], red[2ull * i], bh, bl)) { bh = red[2ull * i + 1]; bl = red[2ull * i]; }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t oh = shfl_xor64(bh, d), ol = shfl_xor64(bl, d);
    if (gt128(oh, ol, bh, bl)) { bh = oh; bl = ol; }
  }
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0) { sh[w] = bh; sl[w] = bl; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t x = 1; x < blockDim.x / 64; ++x)
      if (gt128(sh[x], sl[x], bh, bl)) { bh = sh[x]; bl = sl[x]; }
    *out_lo = bl;
    *out_hi = bh;
  }
}

// ----------------------------------------------------------------------------
// Extraction order (Algorithm 2: sort V by r): stable LSD radix sort of
// d(u) = B - r(u) (B >= every load), starting from ascending ids, so the
// result is r non-increasing with ties in ascending id.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sort_init_kernel(const uint64_t* __restrict__ r, uint32_t n, int wide,
                                                        uint64_t b_lo, uint64_t b_hi, uint64_t* __restrict__ kw_lo,
                                                        uint64_t* __restrict__ kw_hi, uint32_t* __restrict__ perm) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    const uint64_t lo = wide ? r[2ull * u] : r[u];
    const uint64_t hi = wide ? r[2ull * u + 1] : 0ull;
    kw_lo[u] = b_lo - lo;
    if (wide) kw_hi[u] = b_hi - hi - ((b_lo < lo) ? 1ull : 0ull);
    perm[u] = u;
  }
}

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint64_t* __restrict__ kw, uint32_t n,
                                                                  uint32_t shift, uint32_t* __restrict__ hist,
                                                                  uint32_t nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kSortTile;
  for (uint32_t j = 0; j < kSortItems; ++j) {
    const uint32_t i = base + j * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(kw[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

template <typename T>
__global__ __launch_bounds__(1024) void scan_exclusive_single_kernel(T* a, uint32_t count) {
  __shared__ T part[1024];
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (count + 1023u) / 1024u;
  const uint32_t b = min(count, tid * per), e = min(count, b + per);
  T s = 0;
  for (uint32_t i = b; i < e; ++i) s += a[i];
  part[tid] = s;
  __syncthreads();
  for (uint32_t off = 1; off < 1024; off <<= 1) {
    const T v = tid >= off ? part[tid - off] : (T)0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  T run = tid ? part[tid - 1] : (T)0;
  for (uint32_t i = b; i < e; ++i) {
    const T x = a[i];
    a[i] = run;
    run += x;
  }
}

// Exclusive scan of a u32 value over a 256-thread block; returns the exclusive
// prefix of this thread and sets *total to the block sum.
__device__ __forceinline__ uint32_t block_exclusive_scan256(uint32_t v, uint32_t* total, uint32_t* sh) {
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = shfl32(inc, (int)lane >= d ? (int)lane - d : (int)lane);
    if ((int)lane >= d) inc += o;
  }
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  uint32_t before = 0, sum = 0;
  for (uint32_t x = 0; x < 4; ++x) {
    if (x < w) before += sh[x];
    sum += sh[x];
  }
  __syncthreads();
  *total = sum;
  return before + inc - v;
}

// Digit offsets, step 1: block d scans row d of the digit-major histogram in
// place (exclusive) and records the row total.
__global__ __launch_bounds__(256) void radix_rowscan_kernel(uint32_t* __restrict__ hist, uint32_t nblocks,
                                                            uint32_t* __restrict__ rowtot) {
  __shared__ uint32_t sh[4];
  uint32_t* row = hist + (size_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nblocks; b0 += 256) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t v = b < nblocks ? row[b] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan256(v, &total, sh);
    if (b < nblocks) row[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = carry;
}

// Digit offsets, step 2: exclusive scan of the 256 row totals (one block).
__global__ __launch_bounds__(256) void radix_digitscan_kernel(uint32_t* __restrict__ rowtot) {
  __shared__ uint32_t sh[4];
  uint32_t total;
  const uint32_t ex = block_exclusive_scan256(rowtot[threadIdx.x], &total, sh);
  rowtot[threadIdx.x] = ex;
}

// Stable scatter of one 8-bit digit: elements of a tile keep their relative order.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint64_t* __restrict__ klo, const uint64_t* __restrict__ khi, const uint32_t* __restrict__ pin,
    uint64_t* __restrict__ olo, uint64_t* __restrict__ ohi, uint32_t* __restrict__ pout, uint32_t n,
    uint32_t shift, int use_hi, int wide, const uint32_t* __restrict__ hist, uint32_t nblocks,
    const uint32_t* __restrict__ dbase) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[4][256];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  base[tid] = dbase[tid] + hist[(size_t)tid * nblocks + blockIdx.x];
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  for (uint32_t j = 0; j < kSortItems; ++j) {
    const uint32_t i = blockIdx.x * kSortTile + j * kSortThreads + tid;
    const bool valid = i < n;
    const uint64_t vlo = valid ? klo[i] : 0ull;
    const uint64_t vhi = (valid && wide) ? khi[i] : 0ull;
    const uint32_t d = (uint32_t)((use_hi ? vhi : vlo) >> shift) & 255u;
    wcnt[0][tid] = 0;
    wcnt[1][tid] = 0;
    wcnt[2][tid] = 0;
    wcnt[3][tid] = 0;
    __syncthreads();
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(valid && bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    const uint32_t c0 = wcnt[0][tid], c1 = wcnt[1][tid], c2 = wcnt[2][tid], c3 = wcnt[3][tid];
    __syncthreads();
    wcnt[0][tid] = 0;
    wcnt[1][tid] = c0;
    wcnt[2][tid] = c0 + c1;
    wcnt[3][tid] = c0 + c1 + c2;
    __syncthreads();
    if (valid) {
      const uint32_t dst = base[d] + wcnt[w][d] + rank;
      olo[dst] = vlo;
      if (wide) ohi[dst] = vhi;
      pout[dst] = pin[i];
    }
    __syncthreads();
    base[tid] += c0 + c1 + c2 + c3;
    __syncthreads();
  }
}

// extraction key n - 1 - position (smallest key = latest position), and zeroed counts
__global__ __launch_bounds__(256) void rank_keys_kernel(const uint32_t* __restrict__ perm, uint32_t n,
                                                        uint32_t* __restrict__ rank, uint64_t* __restrict__ cnt) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    rank[perm[i]] = n - 1 - i;
    cnt[i] = 0;
  }
}

// ----------------------------------------------------------------------------
// Prefix clique counts K_i and the best prefix (Algorithm 2: argmax_i rho_k(V_i)).
// cnt[u] holds the number of cliques whose latest-positioned member is u, so
// K_i = sum of cnt[order[0 .. i)).  Ratios are compared exactly:
// K_a / a > K_b / b  iff  K_a * b > K_b * a (96-bit products); ties -> larger i.
// ----------------------------------------------------------------------------
__device__ __forceinline__ bool better(uint64_t Ka, uint32_t ia, uint64_t Kb, uint32_t ib) {
  if (Ka == 0) return false;
  if (Kb == 0) return true;
  const uint64_t xl = Ka * (uint64_t)ib, xh = __umul64hi(Ka, (uint64_t)ib);
  const uint64_t yl = Kb * (uint64_t)ia, yh = __umul64hi(Kb, (uint64_t)ia);
  if (xh != yh) return xh > yh;
  if (xl != yl) return xl > yl;
  return ia > ib;
}

__global__ __launch_bounds__(kScanThreads) void scan_blocksum_kernel(const uint64_t* __restrict__ cnt,
                                                                     const uint32_t* __restrict__ perm, uint32_t n,
                                                                     uint64_t* __restrict__ bsum) {
  __shared__ uint64_t ws[kScanThreads / 64];
  uint64_t s = 0;
  const uint32_t base = blockIdx.x * kScanTile;
  for (uint32_t j = 0; j < kScanItems; ++j) {
    const uint32_t i = base + j * kScanThreads + threadIdx.x;
    if (i < n) s += cnt[perm[i]];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += shfl_xor64(s, d);
  if ((threadIdx.x & 63u) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (uint32_t x = 0; x < kScanThreads / 64; ++x) t += ws[x];
    bsum[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_argmax_kernel(const uint64_t* __restrict__ cnt,
                                                                   const uint32_t* __restrict__ perm, uint32_t n,
                                                                   const uint64_t* __restrict__ bsum,
                                                                   uint64_t* __restrict__ bbest) {
  __shared__ uint64_t wsum[kScanThreads / 64];
  __shared__ uint64_t bk[kScanThreads / 64];
  __shared__ uint32_t bi[kScanThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  // thread t owns positions base + t*items .. + items - 1 (consecutive)
  const uint32_t first = blockIdx.x * kScanTile + tid * kScanItems;
  uint64_t v[kScanItems];
  uint64_t tsum = 0;
#pragma unroll
  for (uint32_t j = 0; j < kScanItems; ++j) {
    const uint32_t i = first + j;
    v[j] = i < n ? cnt[perm[i]] : 0ull;
    tsum += v[j];
  }
  // inclusive scan of thread sums within the wave
  uint64_t inc = tsum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = shfl64(inc, (int)lane - d < 0 ? (int)lane : (int)lane - d);
    if ((int)lane - d >= 0) inc += o;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint64_t before = bsum[blockIdx.x];
  for (uint32_t x = 0; x < w; ++x) before += wsum[x];
  uint64_t K = before + inc - tsum;
  uint64_t bestK = 0;
  uint32_t besti = 0;
#pragma unroll
  for (uint32_t j = 0; j < kScanItems; ++j) {
    const uint32_t i = first + j;
    K += v[j];
    if (i < n && better(K, i + 1, bestK, besti)) { bestK = K; besti = i + 1; }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t ok = shfl_xor64(bestK, d);
    const uint32_t oi = shfl_xor32(besti, d);
    if (better(ok, oi, bestK, besti)) { bestK = ok; besti = oi; }
  }
  if (lane == 0) { bk[w] = bestK; bi[w] = besti; }
  __syncthreads();
  if (tid == 0) {
    for (uint32_t x = 1; x < kScanThreads / 64; ++x)
      if (better(bk[x], bi[x], bestK, besti)) { bestK = bk[x]; besti = bi[x]; }
    bbest[2ull * blockIdx.x] = bestK;
    bbest[2ull * blockIdx.x + 1] = besti;
  }
}

__global__ __launch_bounds__(256) void argmax_final_kernel(const uint64_t* __restrict__ bbest, uint32_t nb,
                                                           DevResult* dres) {
  __shared__ uint64_t bk[4];
  __shared__ uint32_t bi[4];
  uint64_t bestK = 0;
  uint32_t besti = 0;
  for (uint32_t x = threadIdx.x; x < nb; x += blockDim.x) {
    const uint64_t K = bbest[2ull * x];
    const uint32_t i = (uint32_t)bbest[2ull * x + 1];
    if (better(K, i, bestK, besti)) { bestK = K; besti = i; }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t ok = shfl_xor64(bestK, d);
    const uint32_t oi = shfl_xor32(besti, d);
    if (better(ok, oi, bestK, besti)) { bestK = ok; besti = oi; }
  }
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0) { bk[w] = bestK; bi[w] = besti; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t x = 1; x < blockDim.x / 64; ++x)
      if (better(bk[x], bi[x], bestK, besti)) { bestK = bk[x]; besti = bi[x]; }
    dres->dens_num = bestK;
    dres->size = besti;
  }
}

__global__ __launch_bounds__(256) void copy_u32_kernel(const uint32_t* __restrict__ a, uint32_t* __restrict__ b,
                                                       uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = a[i];
}

// ----------------------------------------------------------------------------
// Batch extraction: problem q owns node ids [off[q], off[q+1]); after the sort
// it also owns order positions [off[q], off[q+1]).
// ----------------------------------------------------------------------------

// Sort keys q << rbits | (B - r(u)): problems stay contiguous, and inside a
// problem the order is r non-increasing with ties in ascending id.
__global__ __launch_bounds__(256) void batch_sort_init_kernel(const uint64_t* __restrict__ r,
                                                              const uint64_t* __restrict__ off, uint32_t rbits,
                                                              uint64_t bound, uint64_t* __restrict__ kw,
                                                              uint32_t* __restrict__ perm) {
  const uint32_t q = blockIdx.x;
  const uint64_t b = off[q], e = off[q + 1];
  const uint64_t hi = (uint64_t)q << rbits;
  for (uint64_t u = b + threadIdx.x; u < e; u += blockDim.x) {
    kw[u] = hi | (bound - r[u]);
    perm[u] = (uint32_t)u;
  }
}

// Inclusive prefix sums P[i] = sum of cnt[order[0 .. i]] (block sums already scanned).
__global__ __launch_bounds__(kScanThreads) void scan_prefix_kernel(const uint64_t* __restrict__ cnt,
                                                                   const uint32_t* __restrict__ perm, uint32_t n,
                                                                   const uint64_t* __restrict__ bsum,
                                                                   uint64_t* __restrict__ prefix) {
  __shared__ uint64_t wsum[kScanThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t first = blockIdx.x * kScanTile + tid * kScanItems;
  uint64_t v[kScanItems];
  uint64_t tsum = 0;
#pragma unroll
  for (uint32_t j = 0; j < kScanItems; ++j) {
    const uint32_t i = first + j;
    v[j] = i < n ? cnt[perm[i]] : 0ull;
    tsum += v[j];
  }
  uint64_t inc = tsum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = shfl64(inc, (int)lane - d < 0 ? (int)lane : (int)lane - d);
    if ((int)lane - d >= 0) inc += o;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint64_t K = bsum[blockIdx.x];
  for (uint32_t x = 0; x < w; ++x) K += wsum[x];
  K += inc - tsum;
#pragma unroll
  for (uint32_t j = 0; j < kScanItems; ++j) {
    const uint32_t i = first + j;
    K += v[j];
    if (i < n) prefix[i] = K;
  }
}

// One workgroup per problem: exact best prefix (largest i on ties), the upper
// bound max (r - r0) over the problem's nodes, and the order in local ids.
__global__ __launch_bounds__(256) void segment_best_kernel(const uint64_t* __restrict__ prefix,
                                                           const uint64_t* __restrict__ off,
                                                           const uint64_t* __restrict__ r,
                                                           const uint64_t* __restrict__ r0,
                                                           const uint32_t* __restrict__ perm,
                                                           uint32_t* __restrict__ order, DevResult* __restrict__ pres) {
  __shared__ uint64_t bk[4], ub[4];
  __shared__ uint32_t bi[4];
  const uint32_t q = blockIdx.x;
  const uint64_t b = off[q], e = off[q + 1];
  const uint64_t base = b ? prefix[b - 1] : 0ull;
  uint64_t bestK = 0, mx = 0;
  uint32_t besti = 0;
  for (uint64_t pos = b + threadIdx.x; pos < e; pos += blockDim.x) {
    const uint64_t K = prefix[pos] - base;
    const uint32_t i = (uint32_t)(pos - b + 1);
    if (better(K, i, bestK, besti)) { bestK = K; besti = i; }
    order[pos] = perm[pos] - (uint32_t)b;
    const uint64_t x = r[pos] - (r0 ? r0[pos] : 0ull);   // node ids of q are the same range
    mx = x > mx ? x : mx;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t ok = shfl_xor64(bestK, d);
    const uint32_t oi = shfl_xor32(besti, d);
    if (better(ok, oi, bestK, besti)) { bestK = ok; besti = oi; }
    const uint64_t om = shfl_xor64(mx, d);
    mx = om > mx ? om : mx;
  }
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0) { bk[w] = bestK; bi[w] = besti; ub[w] = mx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t x = 1; x < blockDim.x / 64; ++x) {
      if (better(bk[x], bi[x], bestK, besti)) { bestK = bk[x]; besti = bi[x]; }
      mx = ub[x] > mx ? ub[x] : mx;
    }
    DevResult d{};
    d.dens_num = bestK;
    d.size = besti;
    d.ub_lo = mx;
    d.ub_hi = 0;
    pres[q] = d;
  }
}

// ----------------------------------------------------------------------------
// Host-side launch helpers.
// ----------------------------------------------------------------------------
int hip_fail(hipError_t e, const char* what) {
#ifdef KDSS_FAULT_INJECTION
  if (e == hipErrorLaunchFailure) return fail(KDSS_EHIP, std::string(what) + ": injected failure");
#endif
  return fail(KDSS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#ifdef KDSS_FAULT_INJECTION
// Test builds only: after kdss_debug_inject_hip_failure(k), the k-th checked
// HIP call from then on reports a failure (the call itself has run), so every
// error path of the run can be driven from the host.
std::atomic<long> g_inject{-1};
hipError_t injected_failure() {
  long v = g_inject.load();
  while (v > 0 && !g_inject.compare_exchange_weak(v, v - 1)) {
  }
  return v == 1 ? hipErrorLaunchFailure : hipSuccess;
}
#else
constexpr hipError_t injected_failure() { return hipSuccess; }
#endif

#define HIP_TRY(call, what)                              \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ == hipSuccess) e_ = injected_failure();       \
    if (e_ != hipSuccess) return hip_fail(e_, what);     \
  } while (0)

uint32_t grid_for(size_t n, uint32_t threads = 256, uint32_t cap = 16384) {
  size_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (uint32_t)b;
}

uint32_t bit_length128(u128 x) {
  uint32_t b = 0;
  while (x) { ++b; x >>= 1; }
  return b;
}

struct WsView {
  char* base;
  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
};

// Timed launches: kernel-attached events.  ev[0] and ev[1] receive the
// kernel's own start and end (the dispatch's timestamps, hipExtLaunchKernel),
// so no marker packet sits between kernels and the elapsed time is the
// kernel's execution alone.  Without events: a plain launch.
template <typename... Formals, typename... Actuals>
void launch_timed(void (*k)(Formals...), uint32_t grid, uint32_t block, uint32_t shm, hipStream_t st,
                  hipEvent_t* ev, Actuals... a) {
  if (ev)
    hipExtLaunchKernelGGL(k, dim3(grid), dim3(block), shm, st, ev[0], ev[1], 0u, a...);
  else
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), shm, st, a...);
}

// Per-iteration event slots of a timed run (start, end of each kernel).
constexpr int kEvLeaf = 0, kEvHeavy = 2, kEvReduce = 4, kEvApply = 6, kEvPerIter = 8;

// mode: 0 packed FW keys, 1 full u64 loads, 2 full u128 loads, 3 extraction ranks
// ev (nullable): the iteration's kEvPerIter events; the leaf-credit, heavy-leaf
// and hot-node reduction kernels stamp their slots; used (when ev is given)
// receives a bit per slot pair that ran.
// hot_published: the hot keys at these loads are in the load update's table
// (64-bit Frank-Wolfe passes); otherwise every workgroup computes them.
int launch_leaf(const kdss_plan* P, const WsView& ws, int mode, const KeySrc& src, uint64_t* out,
                hipStream_t st, hipEvent_t* ev = nullptr, uint32_t* qlog = nullptr, bool reduce_hot = true,
                bool hot_published = false, uint32_t* used = nullptr) {
  const uint32_t ntiles = (uint32_t)P->tiles.size();
  if (ntiles == 0) return KDSS_OK;
  const uint32_t blocks = P->leaf_blocks;
  const Tile* tiles = ws.at<Tile>(P->off_tiles);
  const uint32_t* members = ws.at<uint32_t>(P->off_members);
  const uint32_t* hdr = ws.at<uint32_t>(P->off_hdr);
  const uint64_t* binom = ws.at<uint64_t>(P->off_binom);
  const uint32_t* hot = ws.at<uint32_t>(P->off_hot);
  const uint32_t* hot_base = ws.at<uint32_t>(P->off_hot_base);
  const uint32_t nhot = (uint32_t)P->hot.size();
  uint64_t* scratch = ws.at<uint64_t>(P->off_scratch);
  uint4* queue = ws.at<uint4>(P->off_queue);
  uint32_t* qcount = ws.at<uint32_t>(P->off_qcount);
  const uint32_t nbinom = (uint32_t)P->binom.size();
  const size_t table_off = hot_published ? P->off_hotkey_fw : P->off_hotkey;
  const uint32_t* xcd = P->sched == 2 ? ws.at<uint32_t>(P->off_xcd) : nullptr;
  hipEvent_t* ev_leaf = ev ? ev + kEvLeaf : nullptr;
  hipEvent_t* ev_heavy = ev ? ev + kEvHeavy : nullptr;
  // in place: every tile takes up its own heavy leaves; queue: none does
  const bool in_place = P->heavy == 2;
  const bool eight = P->heavy == 3;
#define KDSS_LEAF_V(KT, MASKED, LDSB)                                                                           \
  launch_timed(leaf_credit_kernel<KT, MASKED, LDSB>, blocks, kLeafThreads, 0, st, ev_leaf, tiles, ntiles, members, \
               hdr, binom, nbinom, P->k1, src, out, hot, hot_base, nhot, scratch, queue, qcount,                \
               ws.at<KT>(table_off), hot_published, xcd, in_place)
#define KDSS_LEAF(KT)                                                                                           \
  if (nbinom <= kBinomLds) {                                                                                     \
    if (P->gather == 2) KDSS_LEAF_V(KT, false, true);                                                            \
    else KDSS_LEAF_V(KT, true, true);                                                                            \
  } else {                                                                                                       \
    if (P->gather == 2) KDSS_LEAF_V(KT, false, false);                                                           \
    else KDSS_LEAF_V(KT, true, false);                                                                           \
  }                                                                                                              \
  if (!in_place)                                                                                                 \
    launch_timed(nbinom <= kHeavyBinomLds ? (eight ? heavy_kernel<KT, true, true> : heavy_kernel<KT, true, false>)   \
                                          : (eight ? heavy_kernel<KT, false, true> : heavy_kernel<KT, false, false>), \
                 P->heavy_blocks, 256,                                                                           \
                 0, st, ev_heavy, members, binom, P->k1, src, out, nhot, scratch, (const uint4*)queue,             \
                 (const uint32_t*)qcount, (const KT*)ws.at<KT>(table_off), nbinom)
  if (used) *used |= in_place ? 1u : 1u | 2u;
  switch (mode) {
    case 0: KDSS_LEAF(KPacked); break;
    case 1: KDSS_LEAF(KFull); break;
    case 2: KDSS_LEAF(KWide); break;
    default: KDSS_LEAF(KRank); break;
  }
#undef KDSS_LEAF
#undef KDSS_LEAF_V
  HIP_TRY(hipGetLastError(), "leaf credit launch");
  // hot-node totals over the slot entries (cleared again); also empties the queue
  const uint32_t grid = std::max(1u, (nhot + 3) / 4);   // a wavefront per hot node; block 0 empties the queue
  if (reduce_hot) {
    launch_timed(hot_reduce_kernel, grid, 256, 0, st, ev ? ev + kEvReduce : nullptr, scratch, hot, nhot, out,
                 qcount, qlog);
    HIP_TRY(hipGetLastError(), "hot reduce launch");
    if (used) *used |= 4u;
  }
  return KDSS_OK;
}

int fw_mode(const kdss_plan* P) { return P->width == 128 ? 2 : (P->key_mode == 0 ? 0 : 1); }

// One synchronous PBUpdate pass at loads d_r (64-bit) into out; hot-node
// totals go to the slot entries that the load update sums.  Events as for the
// leaf-credit pass (the last three mark its end).
int launch_pb(const kdss_plan* P, const WsView& ws, const void* d_r, uint64_t* out, hipStream_t st,
              hipEvent_t* ev, uint32_t* used) {
  const uint32_t ntiles = (uint32_t)P->tiles.size();
  const uint32_t split = P->pb_split, nhot = (uint32_t)P->hot.size();
  // The two kernels read r_{t-1} and only add credits, so they run side by
  // side: the register kernel on a second stream forked from st and joined
  // back before the load update (captured graphs keep the fork and join).
  hipStream_t reg_st = st;
  const bool both = split && split < ntiles && !P->one_stream;
  if (both) {
    if (!P->side_stream) {   // all three or none
      hipStream_t s2 = nullptr;
      hipEvent_t e1 = nullptr, e2 = nullptr;
      hipError_t e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&e2, hipEventDisableTiming);
      if (e == hipSuccess) e = injected_failure();
      if (e != hipSuccess) {
        if (e2) (void)hipEventDestroy(e2);
        if (e1) (void)hipEventDestroy(e1);
        if (s2) (void)hipStreamDestroy(s2);
        return hip_fail(e, "PBUpdate side stream");
      }
      P->side_stream = s2;
      P->ev_fork = e1;
      P->ev_join = e2;
    }
    reg_st = static_cast<hipStream_t>(P->side_stream);
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P->ev_fork), st), "PBUpdate fork");
    HIP_TRY(hipStreamWaitEvent(reg_st, static_cast<hipEvent_t>(P->ev_fork), 0), "PBUpdate fork");
  }
  if (split < ntiles) {   // the lane tiles of at most kPbRegRows rows, from registers
    const uint32_t blocks = std::min<uint32_t>((ntiles - split + 3) / 4, P->leaf_blocks);
    launch_timed(pb_reg_kernel, blocks, 256, 0, reg_st, ev ? ev + kEvHeavy : nullptr,
                 (const Tile*)ws.at<Tile>(P->off_tiles), split, ntiles, (const uint32_t*)ws.at<uint32_t>(P->off_members),
                 (const uint32_t*)ws.at<uint32_t>(P->off_hdr), (const uint64_t*)ws.at<uint64_t>(P->off_binom), P->k1,
                 static_cast<const uint64_t*>(d_r), (const uint32_t*)ws.at<uint32_t>(P->off_hot), nhot, out,
                 ws.at<uint64_t>(P->off_scratch));
    HIP_TRY(hipGetLastError(), "PBUpdate launch");
    if (used) *used |= 2u;
  }
  // big leaves and lane tiles of more than kPbRegRows rows, staged in LDS, in
  // one launch: one workgroup per tile of more than kPbMidRows rows, then
  // four wavefronts per workgroup for the rest
  if (split) {
    const uint32_t nbig = P->pb_mid, nmid = split - nbig;
    const uint32_t mid_blocks = nmid ? std::min<uint32_t>((nmid + 3) / 4, P->leaf_blocks) : 0u;
    const size_t rows = std::max<size_t>((size_t)4 * P->pb_rows_lo, nbig ? P->pb_rows : 0);
    launch_timed(pb_kernel, nbig + mid_blocks, 256, (uint32_t)(rows * 64 * 8), st, ev ? ev + kEvLeaf : nullptr,
                 (const Tile*)ws.at<Tile>(P->off_tiles), nbig, split, (const uint32_t*)ws.at<uint32_t>(P->off_members),
                 (const uint32_t*)ws.at<uint32_t>(P->off_hdr), (const uint64_t*)ws.at<uint64_t>(P->off_binom), P->k1,
                 static_cast<const uint64_t*>(d_r), (const uint32_t*)ws.at<uint32_t>(P->off_hot), nhot, out,
                 ws.at<uint64_t>(P->off_scratch), P->pb_rows_lo);
    HIP_TRY(hipGetLastError(), "PBUpdate launch");
    if (used) *used |= 1u;
  }
  if (both) {
    HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P->ev_join), reg_st), "PBUpdate join");
    HIP_TRY(hipStreamWaitEvent(st, static_cast<hipEvent_t>(P->ev_join), 0), "PBUpdate join");
  }
  return KDSS_OK;
}

KeySrc fw_src(const kdss_plan* P, const WsView& ws, const void* d_r) {
  (void)ws;
  KeySrc s{};
  s.id_bits = P->id_bits;
  s.r = static_cast<const uint64_t*>(d_r);
  s.rank = nullptr;
  return s;
}

// One iteration: credits at r_{t-1} into delta (hot nodes' into the slot
// entries) -- Frank-Wolfe's per-clique minimum, or PBUpdate's per-pair water
// fill -- then r_t = r_{t-1} + delta.  With 64-bit loads the hot-node
// reduction is part of the update kernel.
int launch_fw_step(const kdss_plan* P, const WsView& ws, void* d_r, hipStream_t st, hipEvent_t* ev,
                   uint32_t* qlog, uint32_t* used = nullptr) {
  uint64_t* delta = ws.at<uint64_t>(P->off_delta);
  const bool fused = P->width == 64 && !P->tiles.empty();
  int rc = P->opts.update == 1
               ? launch_pb(P, ws, d_r, delta, st, ev, used)
               : launch_leaf(P, ws, fw_mode(P), fw_src(P, ws, d_r), delta, st, ev, qlog, !fused, fused, used);
  if (rc) return rc;
  hipEvent_t* ev_apply = ev ? ev + kEvApply : nullptr;
  uint64_t* r = static_cast<uint64_t*>(d_r);
  if (P->width == 128) {
    launch_timed(apply128_kernel, grid_for(P->n), 256, 0, st, ev_apply, r, delta, P->n);
  } else if (fused) {
    const uint32_t nhot = (uint32_t)P->hot.size();
    const uint32_t hot_blocks = std::max(1u, (nhot + 3) / 4);   // block 0 also empties the queue
    launch_timed(apply64_hot_kernel, hot_blocks + grid_for(P->n / 2 + 1), 256, 0, st, ev_apply, r, delta, P->n,
                 ws.at<uint64_t>(P->off_scratch), (const uint32_t*)ws.at<uint32_t>(P->off_hot),
                 (const uint32_t*)ws.at<uint32_t>(P->off_hot_base), nhot, hot_blocks, ws.at<uint32_t>(P->off_qcount),
                 qlog, P->key_mode, P->id_bits, ws.at<uint64_t>(P->off_hotkey_fw));
  } else if ((reinterpret_cast<uintptr_t>(r) & 15u) == 0) {
    launch_timed(apply64_pairs_kernel, grid_for(P->n / 2 + 1), 256, 0, st, ev_apply, r, delta, P->n);
  } else {
    launch_timed(apply64_kernel, grid_for(P->n), 256, 0, st, ev_apply, r, delta, P->n);
  }
  HIP_TRY(hipGetLastError(), "apply launch");
  if (used) *used |= 8u;
  return KDSS_OK;
}

int launch_iteration(const kdss_plan* P, const WsView& ws, void* d_r, hipStream_t st) {
  return launch_fw_step(P, ws, d_r, st, nullptr, nullptr);
}

// Stable LSD radix sort of kw[0] (and kw[0][1] for 128-bit keys) with the
// permutation perm[0] over the low nbits bits; *cur receives the buffer index
// that holds the result.
int launch_radix(const kdss_plan* P, const WsView& ws, uint32_t nbits, int wide, hipStream_t st, int* cur_out) {
  const uint32_t n = P->n;
  uint64_t* kw[2][2] = {{ws.at<uint64_t>(P->off_kw[0][0]), ws.at<uint64_t>(P->off_kw[0][1])},
                        {ws.at<uint64_t>(P->off_kw[1][0]), ws.at<uint64_t>(P->off_kw[1][1])}};
  uint32_t* perm[2] = {ws.at<uint32_t>(P->off_perm[0]), ws.at<uint32_t>(P->off_perm[1])};
  uint32_t* hist = ws.at<uint32_t>(P->off_hist);
  uint32_t* dbase = ws.at<uint32_t>(P->off_dbase);
  int cur = 0;
  for (uint32_t sh = 0; sh < nbits; sh += 8) {
    const int use_hi = sh >= 64 ? 1 : 0;
    const uint64_t* src = use_hi ? kw[cur][1] : kw[cur][0];
    radix_hist_kernel<<<P->sort_blocks, kSortThreads, 0, st>>>(src, n, sh & 63u, hist, P->sort_blocks);
    radix_rowscan_kernel<<<256, 256, 0, st>>>(hist, P->sort_blocks, dbase);
    radix_digitscan_kernel<<<1, 256, 0, st>>>(dbase);
    radix_scatter_kernel<<<P->sort_blocks, kSortThreads, 0, st>>>(kw[cur][0], kw[cur][1], perm[cur], kw[cur ^ 1][0],
                                                                  kw[cur ^ 1][1], perm[cur ^ 1], n, sh & 63u, use_hi,
                                                                  wide, hist, P->sort_blocks, dbase);
    HIP_TRY(hipGetLastError(), "radix pass launch");
    cur ^= 1;
  }
  *cur_out = cur;
  return KDSS_OK;
}

// ----------------------------------------------------------------------------
// Top-s bound on rho* (single problem, 64-bit loads, zero start loads): with
// A_s = the sum of the s largest loads (the extraction order's first s),
// rho* <= max_s min(A_s, T C(s, k)) / (T s).  From s0, the first s with
// C(s, k) >= c_k, on every candidate is A_s (A_s <= T c_k) and A_s / s does
// not grow, so the maximum and its smallest s lie in s <= s0.  Every A_s is at
// most T c_k < 2^64; candidates are compared exactly (64 x 32-bit products).
// ----------------------------------------------------------------------------
constexpr uint32_t kTbThreads = 256;
constexpr uint32_t kTbItems = 4;

// (c1 / s1) beats (c2 / s2): a larger ratio, or an equal one at a smaller s;
// s = 0 marks "none yet"
__device__ inline bool tb_better(uint64_t c1, uint32_t s1, uint64_t c2, uint32_t s2) {
  if (s1 == 0) return false;
  if (s2 == 0) return true;
  const u128 a = (u128)c1 * s2, b = (u128)c2 * s1;
  return a != b ? a > b : s1 < s2;
}

// One workgroup: s = 1 .. slim in chunks of kTbThreads * kTbItems; per chunk
// a workgroup scan of the per-thread sums, then each thread's best candidate;
// the best over the workgroup goes to the device result.
__global__ __launch_bounds__(kTbThreads) void tb_prefix_kernel(const uint64_t* __restrict__ r,
                                                               const uint32_t* __restrict__ order, uint32_t slim,
                                                               const uint64_t* __restrict__ cbin, uint32_t T,
                                                               DevResult* d) {
  __shared__ uint64_t sc[2][kTbThreads];
  __shared__ uint64_t bc[kTbThreads];
  __shared__ uint32_t bz[kTbThreads];
  const uint32_t tid = threadIdx.x;
  uint64_t carry = 0, best = 0;
  uint32_t bsz = 0;
  for (uint32_t base = 0; base < slim; base += kTbThreads * kTbItems) {
    const uint32_t i0 = base + tid * kTbItems;
    uint64_t v[kTbItems], sum = 0;
    for (uint32_t q = 0; q < kTbItems; ++q) {
      v[q] = i0 + q < slim ? r[order[i0 + q]] : 0ull;
      sum += v[q];
    }
    // inclusive scan of the thread sums (Hillis-Steele, double-buffered)
    uint32_t cur = 0;
    sc[0][tid] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < kTbThreads; off <<= 1) {
      const uint64_t x = sc[cur][tid] + (tid >= off ? sc[cur][tid - off] : 0ull);
      sc[cur ^ 1][tid] = x;
      cur ^= 1;
      __syncthreads();
    }
    uint64_t run = carry + sc[cur][tid] - sum;
    for (uint32_t q = 0; q < kTbItems; ++q) {
      const uint32_t s = i0 + q + 1;
      if (s > slim) break;
      run += v[q];
      const u128 tc = (u128)T * cbin[s];
      const uint64_t c = tc < run ? (uint64_t)tc : run;
      if (tb_better(c, s, best, bsz)) { best = c; bsz = s; }
    }
    carry += sc[cur][kTbThreads - 1];
    __syncthreads();   // sc is rewritten by the next chunk
  }
  bc[tid] = best;
  bz[tid] = bsz;
  __syncthreads();
  for (uint32_t half = kTbThreads / 2; half > 0; half >>= 1) {
    if (tid < half && tb_better(bc[tid + half], bz[tid + half], bc[tid], bz[tid])) {
      bc[tid] = bc[tid + half];
      bz[tid] = bz[tid + half];
    }
    __syncthreads();
  }
  if (tid == 0) {
    d->tb_lo = bc[0];
    d->tb_hi = 0;
    d->tb_size = bz[0];
  }
}

// After an extraction at loads d_r: the top-s bound into the device result,
// when it applies (one problem, Frank-Wolfe, 64-bit loads, no start loads).
int launch_top_bound(const kdss_plan* P, const WsView& ws, const void* d_r, const uint64_t* d_r0, uint32_t T,
                     const uint32_t* d_order, hipStream_t st) {
  if (P->width != 64 || d_r0 || P->opts.update != 0 || P->node_off.size() != 2 || P->n == 0 ||
      P->tb_binom.size() < 2)
    return KDSS_OK;
  const uint32_t slim = (uint32_t)(P->tb_binom.size() - 1);
  tb_prefix_kernel<<<1, kTbThreads, 0, st>>>(static_cast<const uint64_t*>(d_r), d_order, slim,
                                             ws.at<uint64_t>(P->off_tb_binom), T, ws.at<DevResult>(P->off_dres));
  HIP_TRY(hipGetLastError(), "top-s bound launch");
  return KDSS_OK;
}

// Extraction at loads d_r; every load is <= bound.  The order lands in d_order
// and the best prefix and upper bound in the device result.
// d_counts (nullable, u64[n]) receives every prefix count K_i at index i - 1.
int launch_extract(const kdss_plan* P, const WsView& ws, const void* d_r, const uint64_t* d_r0, u128 bound,
                   uint32_t* d_order, hipStream_t st, uint64_t* d_counts = nullptr) {
  const uint32_t n = P->n;
  const int wide = P->width == 128 ? 1 : 0;
  const uint64_t* r = static_cast<const uint64_t*>(d_r);
  DevResult* dres = ws.at<DevResult>(P->off_dres);
  uint64_t* red = ws.at<uint64_t>(P->off_red);
  // upper bound numerator max (r - r0)
  max_partial_kernel<<<P->red_blocks, 256, 0, st>>>(r, d_r0, n, wide, red);
  max_final_kernel<<<1, 256, 0, st>>>(red, P->red_blocks, &dres->ub_lo, &dres->ub_hi);
  HIP_TRY(hipGetLastError(), "upper bound launch");
  // order: sort B - r ascending, stable over ascending ids
  uint64_t* kw[2][2] = {{ws.at<uint64_t>(P->off_kw[0][0]), ws.at<uint64_t>(P->off_kw[0][1])},
                        {ws.at<uint64_t>(P->off_kw[1][0]), ws.at<uint64_t>(P->off_kw[1][1])}};
  uint32_t* perm[2] = {ws.at<uint32_t>(P->off_perm[0]), ws.at<uint32_t>(P->off_perm[1])};
  sort_init_kernel<<<grid_for(n), 256, 0, st>>>(r, n, wide, (uint64_t)bound, (uint64_t)(bound >> 64), kw[0][0],
                                                kw[0][1], perm[0]);
  HIP_TRY(hipGetLastError(), "sort init launch");
  int cur = 0;
  int rc0 = launch_radix(P, ws, bit_length128(bound), wide, st, &cur);
  if (rc0) return rc0;
  // prefix clique counts via the leaf pass on position keys
  uint32_t* rank = ws.at<uint32_t>(P->off_keyp);
  uint64_t* cnt = ws.at<uint64_t>(P->off_cnt);
  rank_keys_kernel<<<grid_for(n), 256, 0, st>>>(perm[cur], n, rank, cnt);
  HIP_TRY(hipGetLastError(), "rank keys launch");
  KeySrc ks{};
  ks.rank = rank;
  int rc = launch_leaf(P, ws, 3, ks, cnt, st);
  if (rc) return rc;
  uint64_t* bsum = ws.at<uint64_t>(P->off_bsum);
  uint64_t* bbest = ws.at<uint64_t>(P->off_bbest);
  scan_blocksum_kernel<<<P->scan_blocks, kScanThreads, 0, st>>>(cnt, perm[cur], n, bsum);
  scan_exclusive_single_kernel<uint64_t><<<1, 1024, 0, st>>>(bsum, P->scan_blocks);
  scan_argmax_kernel<<<P->scan_blocks, kScanThreads, 0, st>>>(cnt, perm[cur], n, bsum, bbest);
  argmax_final_kernel<<<1, 256, 0, st>>>(bbest, P->scan_blocks, dres);
  if (d_counts) scan_prefix_kernel<<<P->scan_blocks, kScanThreads, 0, st>>>(cnt, perm[cur], n, bsum, d_counts);
  copy_u32_kernel<<<grid_for(n), 256, 0, st>>>(perm[cur], d_order, n);
  HIP_TRY(hipGetLastError(), "prefix count launch");
  return KDSS_OK;
}

// Exact 256-bit unsigned helpers for the optimality check (four 64-bit limbs,
// least significant first).
struct U256 {
  uint64_t w[4];
};
U256 u256_mul(u128 a, u128 b) {   // a * b
  const uint64_t x[2] = {(uint64_t)a, (uint64_t)(a >> 64)}, y[2] = {(uint64_t)b, (uint64_t)(b >> 64)};
  U256 r{{0, 0, 0, 0}};
  for (int i = 0; i < 2; ++i) {
    u128 carry = 0;
    for (int j = 0; j < 2; ++j) {
      const u128 t = (u128)x[i] * y[j] + r.w[i + j] + carry;
      r.w[i + j] = (uint64_t)t;
      carry = t >> 64;
    }
    r.w[i + 2] = (uint64_t)carry;
  }
  return r;
}
U256 u256_mul64(const U256& a, uint64_t b) {   // a * b, a < 2^192 here
  U256 r{{0, 0, 0, 0}};
  u128 carry = 0;
  for (int i = 0; i < 4; ++i) {
    const u128 t = (u128)a.w[i] * b + carry;
    r.w[i] = (uint64_t)t;
    carry = t >> 64;
  }
  return r;
}
int u256_cmp(const U256& a, const U256& b) {
  for (int i = 3; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
  return 0;
}
U256 u256_sub(const U256& a, const U256& b) {   // a - b, a >= b
  U256 r{{0, 0, 0, 0}};
  uint64_t borrow = 0;
  for (int i = 0; i < 4; ++i) {
    const u128 t = (u128)a.w[i] - b.w[i] - borrow;
    r.w[i] = (uint64_t)t;
    borrow = (uint64_t)(t >> 64) ? 1u : 0u;
  }
  return r;
}

// The bound num / den on rho* and the optimality check: certified when
// bound - K / i < 1 / (n (n - 1)), i.e. (num i - K den) n (n - 1) < den i.
void set_bound(kdss_result* o, u128 num, uint64_t den, int kind, bool may_certify) {
  o->bound_num.lo = (uint64_t)num;
  o->bound_num.hi = (uint64_t)(num >> 64);
  o->bound_den = den;
  o->bound_kind = kind;
  o->bound = den ? ((double)(uint64_t)(num >> 64) * 18446744073709551616.0 + (double)(uint64_t)num) / (double)den
                 : 0.0;
  o->certified = 0;
  if (!may_certify || den == 0) return;
  const u128 K = ((u128)o->dens_num.hi << 64) | o->dens_num.lo;
  const uint64_t i = o->size;
  if (i == 0) {   // no k-clique at all: density 0 and rho* = 0
    o->certified = (num == 0) ? 1 : 0;
    return;
  }
  const U256 a = u256_mul(num, i), b = u256_mul(K, den);
  if (u256_cmp(a, b) < 0) return;   // the bound is below the density: no claim
  const U256 diff = u256_sub(a, b);
  const uint64_t n = o->n;
  const U256 lhs = n >= 2 ? u256_mul64(u256_mul64(diff, n), n - 1) : U256{{0, 0, 0, 0}};
  o->certified = u256_cmp(lhs, u256_mul((u128)den, i)) < 0 ? 1 : 0;
}

void fill_result(const kdss_plan* P, const DevResult& d, uint32_t T, kdss_result* out) {
  std::memset(out, 0, sizeof(*out));
  out->T = T;
  out->n = P->n;
  out->size = d.size;
  out->width = P->width;
  out->dens_num.lo = d.dens_num;
  out->dens_num.hi = 0;
  out->ub_num.lo = d.ub_lo;
  out->ub_num.hi = d.ub_hi;
  out->c_k.lo = (uint64_t)P->c_k;
  out->c_k.hi = (uint64_t)(P->c_k >> 64);
  out->density = d.size ? (double)d.dens_num / (double)d.size : 0.0;
  const double ub = (double)d.ub_hi * 18446744073709551616.0 + (double)d.ub_lo;
  out->upper_bound = T ? ub / (double)T : 0.0;
  const bool fw = P->opts.update == 0;
  if (d.tb_size)
    set_bound(out, ((u128)d.tb_hi << 64) | d.tb_lo, (uint64_t)T * d.tb_size, 1, fw);
  else
    set_bound(out, ((u128)d.ub_hi << 64) | d.ub_lo, T, 0, fw);
}

int check_ws(const kdss_plan* P, void* d_ws, size_t ws_bytes) {
  if (!d_ws) return fail(KDSS_EINVAL, "null workspace");
  if (ws_bytes < P->ws_bytes) return fail(KDSS_EWORKSPACE, "workspace smaller than kdss_plan_info().workspace_bytes");
  if (P->uploaded_ws != d_ws) return fail(KDSS_EWORKSPACE, "workspace was not filled by kdss_plan_upload");
  return KDSS_OK;
}

int read_result(const kdss_plan* P, const WsView& ws, hipStream_t st, DevResult* h) {
  HIP_TRY(hipMemcpyAsync(h, ws.at<DevResult>(P->off_dres), sizeof(DevResult), hipMemcpyDeviceToHost, st),
          "result copy");
  HIP_TRY(hipStreamSynchronize(st), "stream synchronize");
  return KDSS_OK;
}

void drop_graph(kdss_plan* P) {
  if (P->graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(P->graph_exec));
  P->graph_exec = nullptr;
  P->graph_ws = nullptr;
  P->graph_r = nullptr;
}

// Captures use_graph consecutive iterations into one graph on a private
// stream (the caller's stream may be the null stream, which cannot be captured).
int ensure_graph(kdss_plan* P, const WsView& ws, void* d_r) {
  const uint32_t G = (uint32_t)P->opts.use_graph;
  if (P->graph_exec && P->graph_ws == ws.base && P->graph_r == d_r && P->graph_iters == G) return KDSS_OK;
  drop_graph(P);
  if (!P->capture_stream) {
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "capture stream");
    P->capture_stream = s;
  }
  hipStream_t cs = static_cast<hipStream_t>(P->capture_stream);
  HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
  int rc = KDSS_OK;
  for (uint32_t i = 0; i < G && !rc; ++i) rc = launch_iteration(P, ws, d_r, cs);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "graph instantiate");
  P->graph_exec = ex;
  P->graph_ws = ws.base;
  P->graph_r = d_r;
  P->graph_iters = G;
  return KDSS_OK;
}

// The hot-node slot entries are zero between passes; entry points clear them
// again (with a kernel, not a memset) in case an earlier pass was cut short.
void clear_hot_rows(const kdss_plan* P, const WsView& ws, hipStream_t st) {
  const size_t count = (size_t)kHotSlots * P->hot.size();
  if (count) fill_u64_kernel<<<grid_for(count), 256, 0, st>>>(ws.at<uint64_t>(P->off_scratch), 0ull, count);
}

// Start loads, zero credits and a cleared device result.
int start_run(kdss_plan* P, const WsView& ws, const uint64_t* d_r0, void* d_r, uint32_t T, hipStream_t st) {
  DevResult* dres = ws.at<DevResult>(P->off_dres);
  reset_result_kernel<<<1, 64, 0, st>>>(dres);
  clear_hot_rows(P, ws, st);
  init_loads_kernel<<<grid_for(P->n), 256, 0, st>>>(d_r0, static_cast<uint64_t*>(d_r), ws.at<uint64_t>(P->off_delta),
                                                    P->n, P->width == 128 ? 1 : 0, dres);
  HIP_TRY(hipGetLastError(), "init launch");
  if (d_r0) {   // a start load above r0_max would wrap the packed keys: refuse before the first iteration
    DevResult h;
    int rc = read_result(P, ws, st, &h);
    if (rc) return rc;
    if (h.r0max > P->r0_max) return fail(KDSS_EOVERFLOW, "a start load exceeds the plan's r0_max");
  }
  const uint32_t nhot = (uint32_t)P->hot.size();
  if (P->width == 64 && !P->tiles.empty() && nhot) {   // the iterations' leaf passes read the hot keys from a table
    hot_keys_kernel<<<(nhot + 255) / 256, 256, 0, st>>>(static_cast<const uint64_t*>(d_r), ws.at<uint32_t>(P->off_hot),
                                                         ws.at<uint32_t>(P->off_hot_base), nhot, P->key_mode,
                                                         P->id_bits, ws.at<uint64_t>(P->off_hotkey_fw));
    HIP_TRY(hipGetLastError(), "hot keys launch");
  }
  if (P->opts.time_kernels) {
    P->ev_used.assign(T, 0u);
    while (P->events.size() < (size_t)kEvPerIter * T) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e), "event create");
      P->events.push_back(e);
    }
  }
  return KDSS_OK;
}

// Iteration t (1-based): timed launches, a one-iteration graph replay, or plain launches.
int iterate(kdss_plan* P, const WsView& ws, void* d_r, uint32_t t, hipStream_t st) {
  if (P->opts.time_kernels) {
    hipEvent_t* ev = reinterpret_cast<hipEvent_t*>(P->events.data()) + (size_t)kEvPerIter * (t - 1);
    return launch_fw_step(P, ws, d_r, st, ev, ws.at<uint32_t>(P->off_qlog) + (t - 1), &P->ev_used[t - 1]);
  }
  if (P->opts.use_graph == 1) {
    int rc = ensure_graph(P, ws, d_r);
    if (rc) return rc;
    HIP_TRY(hipGraphLaunch(static_cast<hipGraphExec_t>(P->graph_exec), st), "graph launch");
    return KDSS_OK;
  }
  return launch_iteration(P, ws, d_r, st);
}

// Iterations t0 .. t0 + count - 1 with nothing between them: with use_graph
// = G > 1, as replays of one graph of G iterations, the rest one by one.
int iterate_span(kdss_plan* P, const WsView& ws, void* d_r, uint32_t t0, uint32_t count, hipStream_t st) {
  const uint32_t G = P->opts.time_kernels ? 0u : (uint32_t)std::max(0, P->opts.use_graph);
  uint32_t t = t0;
  if (G > 1 && count >= G) {
    int rc = ensure_graph(P, ws, d_r);
    if (rc) return rc;
    for (; t + G <= t0 + count; t += G)
      HIP_TRY(hipGraphLaunch(static_cast<hipGraphExec_t>(P->graph_exec), st), "graph launch");
  }
  for (; t < t0 + count; ++t) {
    int rc = G > 1 ? launch_iteration(P, ws, d_r, st) : iterate(P, ws, d_r, t, st);
    if (rc) return rc;
  }
  return KDSS_OK;
}

// After the stream is synchronised: add the timed kernel durations of T iterations.
int collect_timing(kdss_plan* P, const WsView& ws, uint32_t T) {
  if (!P->opts.time_kernels || P->tiles.empty()) return KDSS_OK;
  std::vector<uint32_t> q(T);
  HIP_TRY(hipMemcpy(q.data(), ws.at<uint32_t>(P->off_qlog), (size_t)T * 4, hipMemcpyDeviceToHost), "queue log");
  for (uint32_t v : q) P->timing.heavy_leaves += v;
  hipEvent_t* ev = reinterpret_cast<hipEvent_t*>(P->events.data());
  double* dst[4] = {&P->timing.leaf_ms, &P->timing.heavy_ms, &P->timing.reduce_ms, &P->timing.apply_ms};
  for (uint32_t t = 0; t < T && t < P->ev_used.size(); ++t) {
    for (int q = 0; q < 4; ++q) {
      if (!(P->ev_used[t] & (1u << q))) continue;
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ev[(size_t)kEvPerIter * t + 2 * q], ev[(size_t)kEvPerIter * t + 2 * q + 1]),
              "event elapsed");
      *dst[q] += ms;
    }
    if (P->ev_used[t] & 1u) P->timing.leaf_launches += 1;
    if (P->ev_used[t] & 8u) P->timing.apply_launches += 1;
  }
  return KDSS_OK;
}

}  // namespace

extern "C" {

#ifdef KDSS_FAULT_INJECTION
// after > 0: the after-th checked HIP call from now on fails; after <= 0: none.
void kdss_debug_inject_hip_failure(long after) { g_inject.store(after > 0 ? after : -1); }
#endif

void kdss_plan_free(kdss_plan* P) {
  if (!P) return;
  drop_graph(P);
  for (void* e : P->events) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
  if (P->capture_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(P->capture_stream));
  if (P->side_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(P->side_stream));
  if (P->ev_fork) (void)hipEventDestroy(static_cast<hipEvent_t>(P->ev_fork));
  if (P->ev_join) (void)hipEventDestroy(static_cast<hipEvent_t>(P->ev_join));
  delete P;
}

int kdss_plan_upload(kdss_plan* P, void* d_ws, size_t ws_bytes, void* stream) {
  return kdss::upload_plan(P, d_ws, ws_bytes, stream, false);
}

}  // extern "C"

namespace kdss {

int upload_plan(kdss_plan* P, void* d_ws, size_t ws_bytes, void* stream, bool fill_by_kernel) {
  if (!P || !d_ws) return fail(KDSS_EINVAL, "null argument");
  if (ws_bytes < P->ws_bytes) return fail(KDSS_EWORKSPACE, "workspace smaller than kdss_plan_info().workspace_bytes");
  hipStream_t st = static_cast<hipStream_t>(stream);
  WsView ws{static_cast<char*>(d_ws)};
  if (!P->members.empty())
    HIP_TRY(hipMemcpyAsync(ws.at<uint32_t>(P->off_members), P->members.data(), P->members.size() * 4,
                           hipMemcpyHostToDevice, st), "upload members");
  if (!P->hdr.empty())
    HIP_TRY(hipMemcpyAsync(ws.at<uint32_t>(P->off_hdr), P->hdr.data(), P->hdr.size() * 4, hipMemcpyHostToDevice, st),
            "upload headers");
  if (!P->tiles.empty())
    HIP_TRY(hipMemcpyAsync(ws.at<Tile>(P->off_tiles), P->tiles.data(), P->tiles.size() * sizeof(Tile),
                           hipMemcpyHostToDevice, st), "upload tiles");
  HIP_TRY(hipMemcpyAsync(ws.at<uint64_t>(P->off_binom), P->binom.data(), P->binom.size() * 8, hipMemcpyHostToDevice,
                         st), "upload binomials");
  if (!P->tb_binom.empty())
    HIP_TRY(hipMemcpyAsync(ws.at<uint64_t>(P->off_tb_binom), P->tb_binom.data(), P->tb_binom.size() * 8,
                           hipMemcpyHostToDevice, st), "upload bound binomials");
  if (!P->hot.empty()) {
    HIP_TRY(hipMemcpyAsync(ws.at<uint32_t>(P->off_hot), P->hot.data(), P->hot.size() * 4, hipMemcpyHostToDevice, st),
            "upload hot nodes");
    HIP_TRY(hipMemcpyAsync(ws.at<uint32_t>(P->off_hot_base), P->hot_base.data(), P->hot_base.size() * 4,
                           hipMemcpyHostToDevice, st), "upload hot node bases");
  }
  HIP_TRY(hipMemcpyAsync(ws.at<uint64_t>(P->off_nodeoff), P->node_off.data(), P->node_off.size() * 8,
                         hipMemcpyHostToDevice, st), "upload node offsets");
  HIP_TRY(hipMemcpyAsync(ws.at<uint32_t>(P->off_xcd), P->xcd_bounds, sizeof(P->xcd_bounds), hipMemcpyHostToDevice,
                         st), "upload XCD ranges");
  // the heavy-leaf queue and the hot-node slot entries start empty; every leaf
  // pass leaves them empty again
  if (fill_by_kernel) {
    fill_u64_kernel<<<1, 64, 0, st>>>(ws.at<uint64_t>(P->off_qcount), 0ull, 8);
    clear_hot_rows(P, ws, st);
    HIP_TRY(hipGetLastError(), "queue and hot rows reset");
  } else {
    HIP_TRY(hipMemsetAsync(ws.at<uint32_t>(P->off_qcount), 0, 64, st), "queue reset");
    if (!P->hot.empty())
      HIP_TRY(hipMemsetAsync(ws.at<uint64_t>(P->off_scratch), 0, (size_t)kHotSlots * P->hot.size() * 8, st),
              "hot rows reset");
  }
  HIP_TRY(hipStreamSynchronize(st), "upload synchronize");
  P->uploaded_ws = d_ws;
  return KDSS_OK;
}

}  // namespace kdss

extern "C" {

}  // extern "C"

namespace {

// T iterations from the loads d_start (nullable: zero), then the extraction.
// The run continues one that began at loads d_r0 (nullable: zero) t_offset
// iterations earlier: the upper bound and the certificate use r - r0 over
// t_offset + T iterations, and trace rows count from t_offset.
int run_impl(kdss_plan* P, void* d_ws, size_t ws_bytes, uint32_t T, uint32_t t_offset, const uint64_t* d_start,
             const uint64_t* d_r0, void* d_r, uint32_t* d_order, kdss_trace_row* h_trace, uint32_t trace_cap,
             kdss_result* h_res, void* stream) {
  if (!P || !d_r || !d_order || !h_res) return fail(KDSS_EINVAL, "null argument");
  if (T == 0 || T > P->T_max) return fail(KDSS_EINVAL, "T must be in 1..T_max");
  if ((uint64_t)t_offset + T > 0xFFFFFFFFull) return fail(KDSS_ERANGE, "t_offset + T exceeds 2^32 - 1");
  int rc = check_ws(P, d_ws, ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  WsView ws{static_cast<char*>(d_ws)};
  rc = start_run(P, ws, d_start, d_r, T, st);
  if (rc) return rc;
  const uint32_t every = P->opts.extract_every;
  const uint32_t T_all = t_offset + T;
  uint32_t rows = 0;
  if (!every || !h_trace) {
    rc = iterate_span(P, ws, d_r, 1, T, st);
    if (rc) return rc;
  }
  for (uint32_t t = 1; every && h_trace && t <= T; ++t) {
    rc = iterate(P, ws, d_r, t, st);
    if (rc) return rc;
    if (every && (t_offset + t) % every == 0 && t < T && h_trace && rows < trace_cap) {
      const u128 bound = (u128)P->r0_max + (u128)t * P->c_k;
      rc = launch_extract(P, ws, d_r, d_r0, bound, d_order, st);
      if (rc) return rc;
      DevResult h;
      rc = read_result(P, ws, st, &h);
      if (rc) return rc;
      kdss_trace_row& row = h_trace[rows++];
      row.t = t_offset + t;
      row.size = h.size;
      row.dens_num.lo = h.dens_num;
      row.dens_num.hi = 0;
      row.ub_num.lo = h.ub_lo;
      row.ub_num.hi = h.ub_hi;
    }
  }
  const u128 bound = (u128)P->r0_max + (u128)T * P->c_k;
  rc = launch_extract(P, ws, d_r, d_r0, bound, d_order, st);
  if (rc) return rc;
  rc = launch_top_bound(P, ws, d_r, d_r0, T_all, d_order, st);
  if (rc) return rc;
  DevResult h;
  rc = read_result(P, ws, st, &h);
  if (rc) return rc;
  rc = collect_timing(P, ws, T);
  if (rc) return rc;
  fill_result(P, h, T_all, h_res);
  if (every && h_trace && rows < trace_cap) {
    kdss_trace_row& row = h_trace[rows++];
    row.t = T_all;
    row.size = h.size;
    row.dens_num = h_res->dens_num;
    row.ub_num = h_res->ub_num;
  }
  return KDSS_OK;
}

}  // namespace

extern "C" {

int kdss_run(kdss_plan* P, void* d_ws, size_t ws_bytes, uint32_t T, const uint64_t* d_r0, void* d_r,
             uint32_t* d_order, kdss_trace_row* h_trace, uint32_t trace_cap, kdss_result* h_res, void* stream) {
  return run_impl(P, d_ws, ws_bytes, T, 0, d_r0, d_r0, d_r, d_order, h_trace, trace_cap, h_res, stream);
}

int kdss_run_resume(kdss_plan* P, void* d_ws, size_t ws_bytes, uint32_t T, uint32_t t_offset,
                    const uint64_t* d_start, const uint64_t* d_r0, void* d_r, uint32_t* d_order,
                    kdss_trace_row* h_trace, uint32_t trace_cap, kdss_result* h_res, void* stream) {
  if (!d_start) return fail(KDSS_EINVAL, "null checkpoint loads");
  return run_impl(P, d_ws, ws_bytes, T, t_offset, d_start, d_r0, d_r, d_order, h_trace, trace_cap, h_res, stream);
}

}  // extern "C"

int kdss::run_plan(kdss_plan* P, void* d_ws, size_t ws_bytes, uint32_t T, const uint64_t* d_r0, void* d_r,
                   uint32_t* d_order, kdss_result* h_res, void* stream) {
  return run_impl(P, d_ws, ws_bytes, T, 0, d_r0, d_r0, d_r, d_order, nullptr, 0, h_res, stream);
}

extern "C" {

int kdss_batch_run(kdss_plan* P, void* d_ws, size_t ws_bytes, uint32_t T, const uint64_t* d_r0, uint64_t* d_r,
                   uint32_t* d_order, kdss_result* h_res, uint32_t count, void* stream) {
  if (!P || !d_r || !d_order || !h_res) return fail(KDSS_EINVAL, "null argument");
  const uint32_t nprob = (uint32_t)(P->node_off.size() - 1);
  if (count != nprob) return fail(KDSS_ERANGE, "count does not match the plan's problems");
  if (T == 0 || T > P->T_max) return fail(KDSS_EINVAL, "T must be in 1..T_max");
  if (P->width != 64) return fail(KDSS_EUNSUPPORTED, "batches need 64-bit loads");
  int rc = check_ws(P, d_ws, ws_bytes);
  if (rc) return rc;
  // sort keys q << rbits | (B - r): B bounds every load of every problem
  u128 bound = 0;
  for (u128 ck : P->prob_ck) bound = std::max(bound, (u128)P->r0_max + (u128)T * ck);
  const uint32_t rbits = bit_length128(bound);
  const uint32_t qbits = bit_length128(nprob - 1);
  if (rbits + qbits > 64) return fail(KDSS_EUNSUPPORTED, "batch sort key exceeds 64 bits");
  hipStream_t st = static_cast<hipStream_t>(stream);
  WsView ws{static_cast<char*>(d_ws)};
  rc = start_run(P, ws, d_r0, d_r, T, st);
  if (rc) return rc;
  rc = iterate_span(P, ws, d_r, 1, T, st);
  if (rc) return rc;
  // segmented extraction
  const uint32_t n = P->n;
  const uint64_t* off = ws.at<uint64_t>(P->off_nodeoff);
  uint64_t* kw0 = ws.at<uint64_t>(P->off_kw[0][0]);
  uint32_t* perm0 = ws.at<uint32_t>(P->off_perm[0]);
  batch_sort_init_kernel<<<nprob, 256, 0, st>>>(d_r, off, rbits, (uint64_t)bound, kw0, perm0);
  HIP_TRY(hipGetLastError(), "batch sort init launch");
  int cur = 0;
  rc = launch_radix(P, ws, rbits + qbits, 0, st, &cur);
  if (rc) return rc;
  const uint32_t* perm = ws.at<uint32_t>(P->off_perm[cur]);
  uint32_t* rank = ws.at<uint32_t>(P->off_keyp);
  uint64_t* cnt = ws.at<uint64_t>(P->off_cnt);
  rank_keys_kernel<<<grid_for(n), 256, 0, st>>>(perm, n, rank, cnt);
  HIP_TRY(hipGetLastError(), "rank keys launch");
  KeySrc ks{};
  ks.rank = rank;
  rc = launch_leaf(P, ws, 3, ks, cnt, st);
  if (rc) return rc;
  uint64_t* bsum = ws.at<uint64_t>(P->off_bsum);
  uint64_t* prefix = ws.at<uint64_t>(P->off_prefix);
  DevResult* pres = ws.at<DevResult>(P->off_pres);
  scan_blocksum_kernel<<<P->scan_blocks, kScanThreads, 0, st>>>(cnt, perm, n, bsum);
  scan_exclusive_single_kernel<uint64_t><<<1, 1024, 0, st>>>(bsum, P->scan_blocks);
  scan_prefix_kernel<<<P->scan_blocks, kScanThreads, 0, st>>>(cnt, perm, n, bsum, prefix);
  segment_best_kernel<<<nprob, 256, 0, st>>>(prefix, off, d_r, d_r0, perm, d_order, pres);
  HIP_TRY(hipGetLastError(), "segment launch");
  std::vector<DevResult> h(nprob);
  DevResult hd;
  HIP_TRY(hipMemcpyAsync(h.data(), pres, sizeof(DevResult) * nprob, hipMemcpyDeviceToHost, st), "result copy");
  HIP_TRY(hipMemcpyAsync(&hd, ws.at<DevResult>(P->off_dres), sizeof(DevResult), hipMemcpyDeviceToHost, st),
          "result copy");
  HIP_TRY(hipStreamSynchronize(st), "stream synchronize");
  if (hd.r0max > P->r0_max) return fail(KDSS_EOVERFLOW, "a start load exceeds the plan's r0_max");
  rc = collect_timing(P, ws, T);
  if (rc) return rc;
  for (uint32_t q = 0; q < nprob; ++q) {
    kdss_result& o = h_res[q];
    std::memset(&o, 0, sizeof(o));
    o.T = T;
    o.n = (uint32_t)(P->node_off[q + 1] - P->node_off[q]);
    o.size = h[q].size;
    o.width = 64;
    o.dens_num.lo = h[q].dens_num;
    o.ub_num.lo = h[q].ub_lo;
    o.c_k.lo = (uint64_t)P->prob_ck[q];
    o.density = o.size ? (double)h[q].dens_num / (double)o.size : 0.0;
    o.upper_bound = (double)h[q].ub_lo / (double)T;
    set_bound(&o, h[q].ub_lo, T, 0, P->opts.update == 0);
  }
  return KDSS_OK;
}

int kdss_plan_set_timing(kdss_plan* P, int on) {
  if (!P) return fail(KDSS_EINVAL, "null argument");
  P->opts.time_kernels = on ? 1 : 0;
  return KDSS_OK;
}

int kdss_plan_set_launch(kdss_plan* P, uint32_t leaf_blocks, uint32_t heavy_blocks) {
  if (!P) return fail(KDSS_EINVAL, "null argument");
  if (leaf_blocks == 0 || leaf_blocks > kLeafBlocksMax || heavy_blocks == 0 || heavy_blocks > kHeavyBlocks)
    return fail(KDSS_ERANGE, "grid sizes must be in 1..8192 (leaf) and 1..16384 (heavy)");
  if (P->leaf_blocks != leaf_blocks || P->heavy_blocks != heavy_blocks) drop_graph(P);
  P->leaf_blocks = leaf_blocks;
  P->heavy_blocks = heavy_blocks;
  return KDSS_OK;
}

int kdss_plan_autotune(kdss_plan* P, void* d_ws, size_t ws_bytes, uint64_t* d_r, uint32_t warm, uint32_t iters,
                       kdss_tune_result* out, void* stream) {
  if (!P || !d_r || !out) return fail(KDSS_EINVAL, "null argument");
  if (iters == 0 || warm + iters > P->T_max) return fail(KDSS_EINVAL, "warm + iters must be in 1..T_max");
  int rc = check_ws(P, d_ws, ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  WsView ws{static_cast<char*>(d_ws)};
  const kdss_opts saved = P->opts;
  P->opts.time_kernels = 0;
  P->opts.use_graph = 0;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "event create");
  HIP_TRY(hipEventCreate(&e1), "event create");
  // leaf grids beyond the 2048 workgroups that stay resident balance the
  // strided tile walk's tail the same way
  const uint32_t leaf_c[] = {512, 1024, 1536, 1792, 2048, 4096, 8192};
  // heavy grids beyond what stays resident let the dispatcher balance the
  // queue's tail: new workgroups start as others finish
  const uint32_t heavy_c[] = {256, 512, 1024, 2048, 4096, 8192, 16384};
  std::memset(out, 0, sizeof(*out));
  out->best_ms = 1e30;
  // per-iteration time of the plan's current launch configuration
  auto time_config = [&](float* ms_per_iter) -> int {
    int r = start_run(P, ws, nullptr, d_r, warm + iters, st);
    for (uint32_t t = 1; !r && t <= warm; ++t) r = iterate(P, ws, d_r, t, st);
    if (!r && hipEventRecord(e0, st) != hipSuccess) r = fail(KDSS_EHIP, "event record");
    for (uint32_t t = warm + 1; !r && t <= warm + iters; ++t) r = iterate(P, ws, d_r, t, st);
    if (!r && hipEventRecord(e1, st) != hipSuccess) r = fail(KDSS_EHIP, "event record");
    float ms = 0.f;
    if (!r && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      r = fail(KDSS_EHIP, "event timing");
    *ms_per_iter = ms / iters;
    return r;
  };
  for (uint32_t lb : leaf_c) {
    for (uint32_t hb : heavy_c) {
      P->leaf_blocks = lb;
      P->heavy_blocks = hb;
      float ms = 0.f;
      rc = time_config(&ms);
      if (rc) break;
      const uint32_t idx = out->tried++;
      if (idx < 32) {
        out->leaf_blocks[idx] = lb;
        out->heavy_blocks[idx] = hb;
        out->ms[idx] = ms;
      }
      if (ms < out->best_ms) {
        out->best_ms = ms;
        out->best_leaf_blocks = lb;
        out->best_heavy_blocks = hb;
      }
    }
    if (rc) break;
  }
  out->best_gather = P->gather;
  out->best_schedule = P->sched;
  out->best_heavy = P->heavy;
  if (!rc) {
    out->gather_ms[P->gather - 1] = out->best_ms;
    out->schedule_ms[P->sched - 1] = out->best_ms;
    if (saved.gather == 0) {   // the mode was left to the library: try the other one at the best sizes
      const int current = P->gather;
      P->leaf_blocks = out->best_leaf_blocks;
      P->heavy_blocks = out->best_heavy_blocks;
      P->gather = 3 - current;
      float ms = 0.f;
      rc = time_config(&ms);
      if (!rc) {
        ++out->tried;
        out->gather_ms[P->gather - 1] = ms;
        if (ms < out->best_ms) {
          out->best_ms = ms;
          out->best_gather = P->gather;
        }
      }
      P->gather = out->best_gather;
    }
    if (!rc) out->heavy_ms[P->heavy - 1] = out->best_ms;
    if (!rc && saved.heavy == 0 && P->tiles.size() > 0) {   // the heavy-leaf mode was left to the library
      const int current = P->heavy;
      P->leaf_blocks = out->best_leaf_blocks;
      P->heavy_blocks = out->best_heavy_blocks;
      for (int m = 1; m <= 3 && !rc; ++m) {
        if (m == current) continue;
        P->heavy = m;
        float ms = 0.f;
        rc = time_config(&ms);
        if (!rc) {
          ++out->tried;
          out->heavy_ms[m - 1] = ms;
          if (ms < out->best_ms) {
            out->best_ms = ms;
            out->best_heavy = m;
          }
        }
      }
      P->heavy = out->best_heavy;
    }
    if (!rc) out->schedule_ms[P->sched - 1] = out->best_ms;
    if (!rc && saved.schedule == 0 && P->tiles.size() > 0) {   // the schedule was left to the library
      const int current = P->sched;
      P->leaf_blocks = out->best_leaf_blocks;
      P->heavy_blocks = out->best_heavy_blocks;
      P->sched = 3 - current;
      float ms = 0.f;
      rc = time_config(&ms);
      if (!rc) {
        ++out->tried;
        out->schedule_ms[P->sched - 1] = ms;
        if (ms < out->best_ms) {
          out->best_ms = ms;
          out->best_schedule = P->sched;
        }
      }
      P->sched = out->best_schedule;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->opts = saved;
  if (rc) return rc;
  P->leaf_blocks = out->best_leaf_blocks;
  P->heavy_blocks = out->best_heavy_blocks;
  drop_graph(P);
  return KDSS_OK;
}

int kdss_plan_tune_key(const kdss_plan* P, char* buf, size_t cap) {
  if (!P || !buf || cap == 0) return fail(KDSS_EINVAL, "null argument");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  // what the best launch depends on: the device, the kernel variant (load
  // width, key mode, update; gather, schedule and heavy-leaf options), the
  // clique sizes, and the shape of the work: leaves per size class and nodes
  // in half-octave buckets
  auto bucket = [](double x) { return x < 1 ? 0 : (int)std::lround(2.0 * std::log2(x)); };
  std::vector<uint32_t> ks(P->prob_k.begin(), P->prob_k.end());
  std::sort(ks.begin(), ks.end());
  ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
  std::string key = arch + "|w" + std::to_string(P->width) + "|km" + std::to_string(P->key_mode) + "|u" +
                    std::to_string(P->opts.update) + "|g" + std::to_string(P->opts.gather) + "|s" +
                    std::to_string(P->opts.schedule) + "|h" + std::to_string(P->opts.heavy) + "|k";
  for (size_t i = 0; i < ks.size(); ++i) key += (i ? "," : "") + std::to_string(ks[i]);
  key += "|q" + std::to_string(bucket((double)(P->node_off.size() - 1))) + "|n" + std::to_string(bucket(P->n)) +
         "|L";
  for (int c = 0; c < kNumClasses; ++c) key += (c ? "," : "") + std::to_string(bucket((double)P->class_leaves[c]));
  if (key.size() + 1 > cap) return fail(KDSS_ERANGE, "key buffer too small");
  std::memcpy(buf, key.c_str(), key.size() + 1);
  return KDSS_OK;
}

int kdss_plan_autotune_cached(kdss_plan* P, void* d_ws, size_t ws_bytes, uint64_t* d_r, uint32_t warm,
                              uint32_t iters, const char* cache_path, int* from_cache, kdss_tune_result* out,
                              void* stream) {
  if (!P || !d_r || !out || !cache_path || !from_cache) return fail(KDSS_EINVAL, "null argument");
  *from_cache = 0;
  char key[512];
  int rc = kdss_plan_tune_key(P, key, sizeof(key));
  if (rc) return rc;
  if (FILE* f = std::fopen(cache_path, "r")) {
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
      char k2[512];
      unsigned lb = 0, hb = 0;
      int g = 0, sc = 0, hm = 0;
      double ms = 0.0;
      if (std::sscanf(line, "%511s %u %u %d %d %d %lf", k2, &lb, &hb, &g, &sc, &hm, &ms) == 7 &&
          std::strcmp(k2, key) == 0 && lb >= 1 && lb <= kLeafBlocksMax && hb >= 1 && hb <= kHeavyBlocks &&
          (g == 1 || g == 2) && (sc == 1 || sc == 2) && hm >= 1 && hm <= 3) {
        std::memset(out, 0, sizeof(*out));
        out->best_leaf_blocks = lb;
        out->best_heavy_blocks = hb;
        out->best_gather = g;
        out->best_schedule = sc;
        out->best_heavy = hm;
        out->best_ms = ms;
        *from_cache = 1;
      }
    }
    std::fclose(f);
  }
  if (*from_cache) {
    P->leaf_blocks = out->best_leaf_blocks;
    P->heavy_blocks = out->best_heavy_blocks;
    P->gather = out->best_gather;
    P->sched = out->best_schedule;
    P->heavy = out->best_heavy;
    drop_graph(P);
    return KDSS_OK;
  }
  rc = kdss_plan_autotune(P, d_ws, ws_bytes, d_r, warm, iters, out, stream);
  if (rc) return rc;
  if (FILE* f = std::fopen(cache_path, "a")) {
    std::fprintf(f, "%s %u %u %d %d %d %.6f\n", key, out->best_leaf_blocks, out->best_heavy_blocks,
                 out->best_gather, out->best_schedule, out->best_heavy, out->best_ms);
    std::fclose(f);
  }
  return KDSS_OK;
}

int kdss_plan_timing(kdss_plan* P, kdss_timing* out, int reset) {
  if (!P || !out) return fail(KDSS_EINVAL, "null argument");
  *out = P->timing;
  if (reset) P->timing = kdss_timing{};
  return KDSS_OK;
}

int kdss_leaf_credit(kdss_plan* P, void* d_ws, size_t ws_bytes, const void* d_r, uint64_t* d_out, void* stream) {
  if (!P || !d_r || !d_out) return fail(KDSS_EINVAL, "null argument");
  int rc = check_ws(P, d_ws, ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  WsView ws{static_cast<char*>(d_ws)};
  fill_u64_kernel<<<grid_for(P->n), 256, 0, st>>>(d_out, 0ull, P->n);
  clear_hot_rows(P, ws, st);
  int mode = P->width == 128 ? 2 : 1;   // loads given directly: full keys
  KeySrc s{};
  s.r = static_cast<const uint64_t*>(d_r);
  rc = launch_leaf(P, ws, mode, s, d_out, st);
  if (rc) return rc;
  HIP_TRY(hipGetLastError(), "leaf credit launch");
  return KDSS_OK;
}

int kdss_extract(kdss_plan* P, void* d_ws, size_t ws_bytes, const void* d_r, const uint64_t* d_r0, uint32_t T,
                 uint32_t* d_order, kdss_result* h_res, void* stream) {
  return kdss_extract_counts(P, d_ws, ws_bytes, d_r, d_r0, T, d_order, nullptr, h_res, stream);
}

void kdss_batch_free(kdss_plan* P) { kdss_plan_free(P); }

int kdss_extract_counts(kdss_plan* P, void* d_ws, size_t ws_bytes, const void* d_r, const uint64_t* d_r0,
                        uint32_t T, uint32_t* d_order, uint64_t* d_counts, kdss_result* h_res, void* stream) {
  if (!P || !d_r || !d_order || !h_res) return fail(KDSS_EINVAL, "null argument");
  if (T == 0) return fail(KDSS_EINVAL, "T must be at least 1");
  if (d_counts && P->node_off.size() != 2) return fail(KDSS_EUNSUPPORTED, "prefix counts of a batch plan");
  int rc = check_ws(P, d_ws, ws_bytes);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  WsView ws{static_cast<char*>(d_ws)};
  DevResult* dres = ws.at<DevResult>(P->off_dres);
  reset_result_kernel<<<1, 64, 0, st>>>(dres);
  clear_hot_rows(P, ws, st);
  // the sort needs a bound on the loads: their maximum
  uint64_t* red = ws.at<uint64_t>(P->off_red);
  max_partial_kernel<<<P->red_blocks, 256, 0, st>>>(static_cast<const uint64_t*>(d_r), nullptr, P->n,
                                                    P->width == 128 ? 1 : 0, red);
  max_final_kernel<<<1, 256, 0, st>>>(red, P->red_blocks, &dres->pad1[0], &dres->pad1[1]);
  HIP_TRY(hipGetLastError(), "max launch");
  DevResult h;
  rc = read_result(P, ws, st, &h);
  if (rc) return rc;
  const u128 bound = ((u128)h.pad1[1] << 64) | h.pad1[0];
  rc = launch_extract(P, ws, d_r, d_r0, bound, d_order, st, d_counts);
  if (rc) return rc;
  rc = launch_top_bound(P, ws, d_r, d_r0, T, d_order, st);
  if (rc) return rc;
  rc = read_result(P, ws, st, &h);
  if (rc) return rc;
  fill_result(P, h, T, h_res);
  return KDSS_OK;
}

}  // extern "C"
