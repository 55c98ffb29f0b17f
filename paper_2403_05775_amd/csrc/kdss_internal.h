// Internal declarations shared by the host sources of the kdss library.
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <utility>
#include <string>
#include <vector>

#include "../../include/kdss.h"

struct kdss_plan;

namespace kdss {

using u128 = unsigned __int128;

// Records a detail message for kdss_last_error() and returns status.
int fail(int status, const std::string& msg);

// An allocator whose value-less construct() leaves trivial types uninitialised,
// so that large buffers filled in parallel are not zeroed first on one thread.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind { using other = NoInitAlloc<U>; };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) {}
  template <class U>
  void construct(U* p) noexcept { ::new ((void*)p) U; }
  template <class U, class... A>
  void construct(U* p, A&&... a) { ::new ((void*)p) U(std::forward<A>(a)...); }
};

// Host worker threads: OMP_NUM_THREADS when set, else the hardware's count (<= 256).
unsigned host_threads();

// f(thread, begin, end) over contiguous ranges of [0, count) on up to
// host_threads() threads, each range at least min_per_thread long; the same
// arguments always give the same ranges.
void parallel_ranges(uint64_t count, uint64_t min_per_thread,
                     const std::function<void(unsigned, uint64_t, uint64_t)>& f);

// ---- graph checks and degeneracy order (host) ----
int validate_csr(const kdss_csr* g);

struct Degeneracy {
  std::vector<uint32_t> order;   // nodes in peeling order
  std::vector<uint32_t> rank;    // rank[v] = position of v in order
  std::vector<uint32_t> core;    // core number of every node
  uint32_t degeneracy = 0;
};
void degeneracy_order(const kdss_csr* g, Degeneracy* out);

// ---- the k-pruned succinct clique tree, flattened to its leaves ----
// Leaf i owns members[off[i] .. off[i] + h[i] + p[i]): first its h hold nodes
// (every clique of the leaf contains them), then its p pivot nodes (any subset
// of them may be added).  Only leaves with h <= k <= h + p are kept (Lemma 4).
struct Sct {
  uint32_t n = 0, k = 0;
  std::vector<uint32_t> members;
  std::vector<uint64_t> off;     // leaves + 1 entries
  std::vector<uint8_t> h;
  std::vector<uint32_t> p;
  u128 c_k = 0;                  // sum over leaves of C(p, k - h)
  uint32_t s_max = 0;
  double build_seconds = 0.0;
  Degeneracy deg;
  uint64_t leaves() const { return h.size(); }
};

int build_sct(const kdss_csr* g, uint32_t k, uint32_t threads, Sct* out);
// The same search, keeping only the counts (leaves, members, s_max, c_k).
int count_sct(const kdss_csr* g, uint32_t k, uint32_t threads, kdss_tree_stats* stats);
int build_sct_impl(const kdss_csr* g, uint32_t k, uint32_t threads, Sct* out, kdss_tree_stats* stats);

// Binomial coefficient C(a, b) in 128 bits, saturating at 2^128 - 1.
u128 binom128(uint64_t a, uint64_t b);

// ---- device layout ----
// Leaves with at most 64 members are processed one leaf per lane: a "lane
// tile" is one round of up to 64 leaves of similar size, whose members are
// stored column-major (member x of the tile's leaf i at mbase + 64 x + i, short
// leaves padded), so every member load of a wavefront is one contiguous row.
// Leaves are grouped by size (kLaneBounds) and keep the tree's depth-first
// order inside a group, so neighbouring lanes usually share the leaf's root.
// Larger leaves ("big") are processed one per wavefront, members contiguous.
// Statistics are reported for the size buckets s <= 8, 16, 32, 64 and > 64.
constexpr int kNumClasses = 5;
constexpr int kBigClass = 4;
constexpr uint32_t kTileLane = 0, kTileBig = 4;
constexpr uint32_t kMaxBigLeaf = 4096;     // largest leaf the planner accepts
constexpr uint32_t kMaxK = 31;

// Word offset of member x of leaf i (lane i) inside a lane tile.
inline uint64_t lane_tile_offset(uint32_t x, uint32_t i) { return (uint64_t)64 * x + i; }
constexpr uint32_t kLaneBounds[] = {2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64};
constexpr int kNumLaneGroups = sizeof(kLaneBounds) / sizeof(kLaneBounds[0]);

// One tile = the work of one wavefront.
struct Tile {
  uint64_t mbase;    // first member of the tile
  uint32_t lbase;    // first leaf (index into the header array)
  uint32_t info;     // kind (3 bits: kTileLane / kTileBig) | leaf count (13 bits) << 3
                     // | largest leaf (16 bits) << 16
  uint32_t nbase;    // first node id of the tile's problem (packed keys use local ids)
  uint32_t pad[3];
};
static_assert(sizeof(Tile) == 32, "tile descriptor is 32 bytes");

// Launch geometry shared by the planner (workspace sizes) and the kernels.
constexpr uint32_t kSortThreads = 256, kSortItems = 8, kSortTile = kSortThreads * kSortItems;
constexpr uint32_t kScanThreads = 256, kScanItems = 4, kScanTile = kScanThreads * kScanItems;
constexpr uint32_t kRedThreads = 256, kRedTile = 4096;
constexpr uint32_t kBinomLds = 512;              // binomial tables up to this size live in LDS
constexpr uint32_t kHeavyBinomLds = 1024;        // ... in the heavy-leaf pass (s_max 64 at k <= 14)
// Hot nodes: the nodes that occur in the most leaves.  Their member ids carry
// kHotFlag | index into the hot table; every workgroup keeps their keys and
// credits in LDS and adds its nonzero credit totals, at its end, into one of
// kHotSlots slot entries per hot node (hot-node-major: slot b of hot node i is
// word i * kHotSlots + b, so one node's slots are read as one contiguous run).
constexpr uint32_t kHotMax = 512;
constexpr uint32_t kHotMinOccurrences = 32;
constexpr uint32_t kHotFlag = 0x80000000u;
constexpr uint32_t kLeafBlocksMax = 8192;        // leaf-credit grid, largest (2048 stay resident)
constexpr uint32_t kLeafBlocksDefault = 2048;    // eight workgroups per CU
constexpr uint32_t kHeavyBlocks = 16384;         // largest grid of the heavy-leaf kernel
constexpr uint32_t kHeavyBlocksDefault = 2048;   // its grid until set or tuned
constexpr uint32_t kHotSlots = 256;              // credit slots per hot node, shared by workgroups
constexpr double kMaskedGatherShare = 0.5;       // hot share from which masked gathers are the default
constexpr uint32_t kPbRegRows = 16;              // PBUpdate: lane tiles up to this many rows run from registers
constexpr uint32_t kPbMidRows = 32;              // PBUpdate: lane tiles up to this many rows share 4-wave workgroups
constexpr uint32_t kXcds = 8;                    // accelerator dies; workgroup b runs on die b mod 8

// Copies a plan's leaf stream and tables into the device workspace d_ws and
// empties its queue and hot-node slots (with kernels when fill_by_kernel, else
// with memsets); synchronises the stream.
int upload_plan(kdss_plan* P, void* d_ws, size_t ws_bytes, void* stream, bool fill_by_kernel);
// kdss_run without a trace.
int run_plan(kdss_plan* P, void* d_ws, size_t ws_bytes, uint32_t T, const uint64_t* d_r0, void* d_r,
             uint32_t* d_order, kdss_result* h_res, void* stream);

// Device-side result of an extraction.
struct DevResult {
  uint64_t dens_num;      // K_{i*}
  uint32_t size;          // i*
  uint32_t pad0;
  uint64_t ub_lo, ub_hi;  // max (r - r0)
  uint64_t r0max;         // largest start load seen
  uint64_t pad1[3];
  uint64_t tb_lo, tb_hi;  // top-s bound numerator min(A_s, T C(s, k)) at the best s
  uint32_t tb_size;       // that s (0: not computed)
  uint32_t pad2;
  uint64_t pad3[5];
};
static_assert(sizeof(DevResult) == 128, "device result is 128 bytes");

// Leaf header: h (5 bits), j = k - h (5 bits), p (22 bits).
inline uint32_t pack_leaf(uint32_t h, uint32_t j, uint32_t p) { return h | (j << 5) | (p << 10); }
inline uint32_t pack_tile_info(uint32_t kind, uint32_t leaves, uint32_t smax) {
  return kind | (leaves << 3) | (smax << 16);
}

}  // namespace kdss

// The host clique tree behind the opaque kdss_sct handle.
struct kdss_sct {
  kdss::Sct s;
};

// The device plan of one clique tree (opaque to callers as kdss_plan).
struct kdss_plan {
  uint32_t n = 0, k = 0, T_max = 0, id_bits = 0, s_max = 0;
  int width = 64;          // load width
  int key_mode = 0;        // 0 packed, 1 full
  int gather = 1;          // leaf-pass key gathers: 1 masked, 2 full
  int sched = 1;           // leaf-pass tile schedule: 1 strided, 2 XCD ranges
  int heavy = 1;           // heavy leaves: 1 queued (heavy kernel, four per batch), 2 in place, 3 queued (eight)
  uint32_t xcd_bounds[9] = {};   // XCD x takes tiles [xcd_bounds[x], xcd_bounds[x + 1])
  uint32_t pb_split = 0;   // PBUpdate: tiles [0, pb_split) are staged in LDS, the rest (lane tiles of
                           // at most kPbRegRows rows) kept in registers
  uint32_t pb_rows = 0;    // PBUpdate: staged rows of 64 members (largest tile or big leaf before pb_mid)
  uint32_t pb_mid = 0;     // PBUpdate: tiles [pb_mid, pb_split) are lane tiles of at most kPbMidRows rows
  uint32_t pb_rows_lo = 0; // PBUpdate: largest of those
  double hot_share = 0.0;  // hot nodes' share of all member occurrences
  uint64_t r0_max = 0;
  kdss::u128 c_k = 0;
  kdss_opts opts{};
  std::vector<uint32_t, kdss::NoInitAlloc<uint32_t>> members;   // class-major, tile order
  std::vector<uint32_t> hdr;          // one per leaf
  std::vector<kdss::Tile> tiles;
  std::vector<uint64_t> binom;        // C(a, b), a <= s_max, b <= k, row length k + 1
  uint64_t class_tiles[kdss::kNumClasses] = {}, class_leaves[kdss::kNumClasses] = {},
           class_members[kdss::kNumClasses] = {};
  // workspace layout (byte offsets)
  size_t off_members = 0, off_hdr = 0, off_tiles = 0, off_binom = 0, off_delta = 0,
         off_cnt = 0, off_kw[2][2] = {}, off_perm[2] = {}, off_keyp = 0, off_hist = 0, off_bsum = 0,
         off_bbest = 0, off_red = 0, off_dres = 0, ws_bytes = 0;
  uint32_t sort_blocks = 0, scan_blocks = 0, red_blocks = 0;
  uint32_t leaf_blocks = 0;            // persistent grid of the leaf-credit kernel
  std::vector<uint32_t> hot;           // original ids of the hot nodes
  std::vector<uint32_t> hot_base;      // first node id of each hot node's problem
  size_t off_hot = 0, off_hot_base = 0, off_scratch = 0, off_dbase = 0, off_queue = 0, off_qcount = 0;
  size_t off_qlog = 0;
  size_t off_xcd = 0;                  // the nine XCD range bounds (u32)
  size_t off_hotkey = 0;               // hot-node keys published by a leaf pass for its heavy pass
  size_t off_hotkey_fw = 0;            // hot-node keys at the current loads, kept by the load update
  uint32_t heavy_blocks = 0;           // grid of the heavy-leaf kernel
  uint32_t k1 = 0;                     // binomial table row length (largest k + 1)
  kdss::u128 bound_max = 0;            // largest r0_max + T_max * c_k over the problems
  std::vector<uint64_t> node_off;      // problem q owns ids node_off[q] .. node_off[q+1]-1
  std::vector<uint32_t> prob_k;
  std::vector<kdss::u128> prob_ck;
  size_t off_prefix = 0, off_pres = 0, off_nodeoff = 0;
  // top-s bound: C(s, k) for s = 0 .. its last entry, the first s with C(s, k) >= c_k
  // (saturated at 2^64 - 1; single problems with c_k < 2^64 only)
  std::vector<uint64_t> tb_binom;
  size_t off_tb_binom = 0;
  uint64_t lane_leaves = 0;            // leaves in lane tiles (queue capacity)
  // state of the device side
  void* uploaded_ws = nullptr;
  void* graph_exec = nullptr;          // hipGraphExec_t of one iteration
  void* graph_ws = nullptr;
  void* graph_r = nullptr;
  uint32_t graph_iters = 0;            // iterations the captured graph holds
  void* capture_stream = nullptr;
  // PBUpdate's register-tile kernel runs beside its LDS-tile kernel: a second
  // stream of the default priority and the fork / join events (made on first use)
  mutable void* side_stream = nullptr;
  mutable void* ev_fork = nullptr;
  mutable void* ev_join = nullptr;
  bool one_stream = false;   // set for the duration of a static run: no stream or event is made
  std::vector<void*> events;           // hipEvent_t pool for kernel timing
  std::vector<uint32_t> ev_used;       // per iteration: which kernels stamped their events
  kdss_timing timing{};
};
