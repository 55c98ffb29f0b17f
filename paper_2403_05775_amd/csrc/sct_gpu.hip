// The k-pruned succinct clique tree (paper: Sec. 2, Lemmas 3-5) built on the
// GPU.  The order comes from a level-synchronous peeling on the device: at
// level L, every node left with at most L remaining neighbours leaves in the
// same sub-round (ranks in id order within it, core number L), and L grows
// when none is left; a node then has at most L <= D (the degeneracy) later
// neighbours.  The graph is oriented along that order: out(v) holds v's later
// neighbours, ascending by id.
// The tree of a start node v is the pivoting recursion over out(v) (local
// indices, adjacency bitsets):
//   node (H, P, S): h = |H| = k: the leaf (H, {}); h + p + |S| < k: nothing;
//   S empty: the leaf (H, P) when p >= k - h; otherwise a pivot q of S with
//   the most neighbours in S: (H, P + q, S and N(q)), then for each w of S
//   not adjacent to q (w != q), in local order: (H + w, P, S and N(w) minus
//   the w handled before).
// Every k-clique of the graph lies in exactly one leaf (the tree of a node
// covers the cliques whose earliest node it is); the leaves may differ from
// the host build's, and any such tree gives the same results.
// A hub's tree can hold millions of leaves, so the work is split at the root:
// one thread per start node builds its bitsets once (out(x) of each member x
// merged with out(v): every edge inside out(v) is found once, from its
// earlier end) into a device store, picks the root pivot and lists the root's
// children that can hold a k-clique; then one thread per child ("task") runs
// the recursion below it with an explicit stack in a per-thread slice of
// global scratch sized by D (word i of thread t at i * threads + t, so a
// wavefront's equal-index accesses coalesce).  Start nodes run in decreasing
// |out(v)| and a node's tasks in its tree's order, so the leaves come out in
// the order a whole-tree recursion per node would give.  Nodes with
// |out(v)| + 1 < k hold no k-clique and are skipped.  Two passes over chunks
// of tasks: counts, then the leaves written at the prefix-sum offsets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "kdss_internal.h"

using kdss::u128;

namespace {

constexpr uint32_t kSctMaxLocal = 256;                 // largest degeneracy handled
constexpr uint32_t kSctMaxHold = 32;                   // hold list entries (k <= 31)
constexpr size_t kSctScratchBudget = size_t(8) << 30;  // per-chunk scratch bytes
constexpr uint32_t kPivotTask = 0x80000000u;           // task code: the root's pivot child

// Scratch words of one task thread for degeneracy D with W bitset words:
// frames (D + 2) * (2 W + 1) in 64-bit words; hold and pivot lists
// kSctMaxHold + D in 32-bit words.
inline size_t sct_words64(uint32_t D, uint32_t W) { return (size_t)(D + 2) * (2 * W + 1); }
inline size_t sct_words32(uint32_t D) { return kSctMaxHold + (size_t)D; }

int sct_hip_fail(hipError_t e, const char* what) {
  return kdss::fail(KDSS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define SCT_TRY(call, what)                              \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return sct_hip_fail(e_, what); \
  } while (0)

constexpr uint32_t kPeelTile = 1024;   // nodes per peeling workgroup (256 threads x 4)

__global__ __launch_bounds__(256) void peel_init_kernel(const uint64_t* __restrict__ rp, uint32_t n,
                                                        uint32_t* __restrict__ deg, uint32_t* __restrict__ rank) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  deg[v] = (uint32_t)(rp[v + 1] - rp[v]);
  rank[v] = ~0u;   // still in the graph
}

// The nodes of tile b (ids b * kPeelTile ..) still in the graph with at most L
// remaining neighbours: tcnt[b] = how many.
__global__ __launch_bounds__(256) void peel_count_kernel(const uint32_t* __restrict__ deg,
                                                         const uint32_t* __restrict__ rank, uint32_t n, uint32_t L,
                                                         uint32_t* __restrict__ tcnt) {
  __shared__ uint32_t tot;
  if (threadIdx.x == 0) tot = 0;
  __syncthreads();
  const uint32_t v0 = blockIdx.x * kPeelTile + threadIdx.x * 4;
  uint32_t c = 0;
  for (uint32_t i = 0; i < 4; ++i) {
    const uint32_t v = v0 + i;
    if (v < n && rank[v] == ~0u && deg[v] <= L) ++c;
  }
  if (c) atomicAdd(&tot, c);
  __syncthreads();
  if (threadIdx.x == 0) tcnt[blockIdx.x] = tot;
}

// The same nodes leave: rank = toff[b] + their position among the tile's, in
// id order (order[rank] = the node); core number L.
__global__ __launch_bounds__(256) void peel_assign_kernel(const uint32_t* __restrict__ deg,
                                                          uint32_t* __restrict__ rank, uint32_t* __restrict__ core,
                                                          uint32_t* __restrict__ order, uint32_t n, uint32_t L,
                                                          const uint32_t* __restrict__ toff) {
  __shared__ uint32_t sc[256];
  const uint32_t t = threadIdx.x;
  const uint32_t v0 = blockIdx.x * kPeelTile + t * 4;
  bool f[4];
  uint32_t c = 0;
  for (uint32_t i = 0; i < 4; ++i) {
    const uint32_t v = v0 + i;
    f[i] = v < n && rank[v] == ~0u && deg[v] <= L;
    c += f[i] ? 1u : 0u;
  }
  sc[t] = c;
  __syncthreads();
  for (uint32_t off = 1; off < 256; off <<= 1) {   // inclusive scan of the counts
    const uint32_t x = t >= off ? sc[t - off] : 0u;
    __syncthreads();
    sc[t] += x;
    __syncthreads();
  }
  uint32_t pos = toff[blockIdx.x] + sc[t] - c;
  for (uint32_t i = 0; i < 4; ++i)
    if (f[i]) {
      order[pos] = v0 + i;
      rank[v0 + i] = pos++;
      core[v0 + i] = L;
    }
}

// The sub-round's nodes (order[lo .. lo + cnt - 1]) are gone: each neighbour
// still in the graph loses one remaining neighbour.  One wavefront per
// removed node, its lanes over the node's row.
__global__ __launch_bounds__(256) void peel_drop_kernel(const uint64_t* __restrict__ rp,
                                                        const uint32_t* __restrict__ col,
                                                        const uint32_t* __restrict__ rank,
                                                        const uint32_t* __restrict__ order, uint32_t lo, uint32_t cnt,
                                                        uint32_t* __restrict__ deg) {
  const uint32_t i = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (i >= cnt) return;
  const uint32_t v = order[lo + i];
  for (uint64_t e = rp[v] + (threadIdx.x & 63u); e < rp[v + 1]; e += 64) {
    const uint32_t u = col[e];
    if (rank[u] == ~0u) atomicSub(&deg[u], 1u);
  }
}

// out-degree of every node along the order (rank): ocnt[v] = |out(v)|.
__global__ __launch_bounds__(256) void orient_count_kernel(const uint64_t* __restrict__ rp,
                                                           const uint32_t* __restrict__ col,
                                                           const uint32_t* __restrict__ rank, uint32_t n,
                                                           uint32_t* __restrict__ ocnt) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t rv = rank[v];
  uint32_t c = 0;
  for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) c += rank[col[e]] > rv;
  ocnt[v] = c;
}

// out(v) at orp[v], ascending by id (the row's order).
__global__ __launch_bounds__(256) void orient_fill_kernel(const uint64_t* __restrict__ rp,
                                                          const uint32_t* __restrict__ col,
                                                          const uint32_t* __restrict__ rank, uint32_t n,
                                                          const uint64_t* __restrict__ orp,
                                                          uint32_t* __restrict__ ocol) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t rv = rank[v];
  uint64_t at = orp[v];
  for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
    const uint32_t u = col[e];
    if (rank[u] > rv) ocol[at++] = u;
  }
}

// The first d bits set (d <= 64 W).
template <uint32_t W>
__device__ inline void all_bits(uint64_t (&S)[W], uint32_t d) {
  for (uint32_t w = 0; w < W; ++w) {
    const uint32_t lo = w * 64;
    S[w] = d >= lo + 64 ? ~0ull : (d > lo ? (1ull << (d - lo)) - 1 : 0ull);
  }
}

// The root's hold child for w (local index): S and N(w) minus the members of
// NQ (S's non-neighbours of the pivot, handled in local order) before w.
template <uint32_t W>
__device__ inline void hold_child(const uint64_t (&S)[W], const uint64_t (&NQ)[W], const uint64_t* A, uint32_t wi,
                                  uint64_t (&out)[W]) {
  for (uint32_t x = 0; x < W; ++x) {
    const uint64_t before = x < (wi >> 6) ? ~0ull : (x == (wi >> 6) ? (1ull << (wi & 63)) - 1 : 0ull);
    out[x] = S[x] & A[(size_t)wi * W + x] & ~(NQ[x] & before);
  }
}

// One thread per active start node perm[t] (t < nact).  D: the degeneracy
// (every |out(v)| is at most D, W * 64 >= D).  The node's bitsets live at
// abits + aoff[t], row i of W words at row i.  write = 0: builds the bitsets,
// picks the root pivot (qv[t]) and counts the root's children that can hold
// a k-clique (tcnt[t]): the pivot child (H = {v}, P = {q}) when
// 2 + |S and N(q)| >= k, and each hold child (H = {v, w}, P = {}) when
// 2 + |its S| >= k.  write = 1: their task records from toff[t], in the
// tree's order: t << 32 | code, code = q | kPivotTask or w.  *err: 1 = an
// out-list above D.
template <uint32_t W>
__global__ __launch_bounds__(64) void root_kernel(const uint64_t* __restrict__ orp, const uint32_t* __restrict__ ocol,
                                                  const uint32_t* __restrict__ perm, uint32_t k, uint32_t D,
                                                  uint32_t nact, uint64_t* __restrict__ abits,
                                                  const uint64_t* __restrict__ aoff, uint32_t* __restrict__ qv,
                                                  int write, uint32_t* __restrict__ tcnt,
                                                  const uint64_t* __restrict__ toff, uint64_t* __restrict__ tasks,
                                                  int* __restrict__ err) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nact) return;
  const uint32_t v = perm[t];
  const uint64_t ob = orp[v];
  const uint32_t d = (uint32_t)(orp[v + 1] - ob);
  const uint32_t* __restrict__ L = ocol + ob;
  if (d > D || d > W * 64) {
    atomicOr(err, 1);
    return;
  }
  uint64_t* __restrict__ A = abits + aoff[t];
  uint64_t S[W];
  all_bits<W>(S, d);
  uint32_t q = 0;
  if (!write) {
    for (uint32_t i = 0; i < d; ++i)
      for (uint32_t w = 0; w < W; ++w) A[(size_t)i * W + w] = 0;
    // edges inside out(v): merge out(x) with out(v), both ascending by id
    for (uint32_t i = 0; i < d; ++i) {
      const uint32_t x = L[i];
      uint64_t a = orp[x];
      const uint64_t ae = orp[x + 1];
      uint32_t j = 0;
      while (a < ae && j < d) {
        const uint32_t ya = ocol[a], yb = L[j];
        if (ya < yb) {
          ++a;
        } else if (ya > yb) {
          ++j;
        } else {
          A[(size_t)i * W + (j >> 6)] |= 1ull << (j & 63);
          A[(size_t)j * W + (i >> 6)] |= 1ull << (i & 63);
          ++a;
          ++j;
        }
      }
    }
    // root pivot: the member with the most neighbours in S (lowest index on ties)
    uint32_t best = 0;
    bool first = true;
    for (uint32_t i = 0; i < d; ++i) {
      uint32_t c = 0;
      for (uint32_t x = 0; x < W; ++x) c += __popcll(A[(size_t)i * W + x] & S[x]);
      if (first || c > best) { q = i; best = c; first = false; }
    }
    qv[t] = q;
  } else {
    q = qv[t];
  }
  uint64_t NQ[W];
  uint32_t cp = 0;
  for (uint32_t w = 0; w < W; ++w) {
    const uint64_t aq = A[(size_t)q * W + w];
    cp += __popcll(S[w] & aq);
    NQ[w] = S[w] & ~aq;
  }
  NQ[q >> 6] &= ~(1ull << (q & 63));
  const uint64_t base = write ? toff[t] : 0;
  uint32_t n = 0;
  if (2 + cp >= k) {
    if (write) tasks[base + n] = ((uint64_t)t << 32) | (q | kPivotTask);
    ++n;
  }
  for (uint32_t w = 0; w < W; ++w) {
    uint64_t bits = NQ[w];
    while (bits) {
      const uint32_t wi = w * 64 + (uint32_t)__ffsll((unsigned long long)bits) - 1;
      bits &= bits - 1;
      uint64_t C[W];
      hold_child<W>(S, NQ, A, wi, C);
      uint32_t c = 0;
      for (uint32_t x = 0; x < W; ++x) c += __popcll(C[x]);
      if (2 + c >= k) {
        if (write) tasks[base + n] = ((uint64_t)t << 32) | wi;
        ++n;
      }
    }
  }
  if (!write) tcnt[t] = n;
}

// One thread per task tasks[v0 + i] (i < count): the recursion below one of
// a root's children, from the start node's stored bitsets.  write = 0:
// counts[2 i] = leaves, counts[2 i + 1] = members.  write = 1: leaves from
// leaf_off[i], members from member_off[i]; hp[leaf] = h | p << 8.  *err:
// 2 = the stack would overflow (nothing is written out of bounds).
template <uint32_t W>
__global__ __launch_bounds__(64) void task_kernel(const uint64_t* __restrict__ orp, const uint32_t* __restrict__ ocol,
                                                  const uint32_t* __restrict__ perm, uint32_t k, uint32_t D,
                                                  const uint64_t* __restrict__ abits,
                                                  const uint64_t* __restrict__ aoff, const uint32_t* __restrict__ qv,
                                                  const uint64_t* __restrict__ tasks, uint64_t v0, uint32_t count,
                                                  uint64_t* __restrict__ s64, uint32_t* __restrict__ s32, int write,
                                                  uint64_t* __restrict__ counts, const uint64_t* __restrict__ leaf_off,
                                                  const uint64_t* __restrict__ member_off, uint32_t* __restrict__ hp,
                                                  uint32_t* __restrict__ members, int* __restrict__ err) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t rec = tasks[v0 + i];
  const uint32_t t = (uint32_t)(rec >> 32), code = (uint32_t)rec;
  const uint32_t v = perm[t];
  const uint64_t ob = orp[v];
  const uint32_t d = (uint32_t)(orp[v + 1] - ob);
  const uint32_t* __restrict__ L = ocol + ob;
  const uint64_t* __restrict__ A = abits + aoff[t];
  const size_t stride = count;
  const uint32_t nframes = D + 2;
  auto F = [&](uint32_t f, uint32_t w) -> uint64_t& { return s64[((size_t)f * (2 * W + 1) + w) * stride + i]; };
  auto Hl = [&](uint32_t x) -> uint32_t& { return s32[(size_t)x * stride + i]; };
  auto Pl = [&](uint32_t x) -> uint32_t& { return s32[((size_t)kSctMaxHold + x) * stride + i]; };
  uint64_t nleaves = 0, nmembers = 0;
  const uint64_t lo_leaf = write ? leaf_off[i] : 0, lo_mem = write ? member_off[i] : 0;
  auto emit = [&](uint32_t h, uint32_t p) {
    if (write) {
      hp[lo_leaf + nleaves] = h | (p << 8);
      uint64_t at = lo_mem + nmembers;
      for (uint32_t x = 0; x < h; ++x) members[at++] = Hl(x);
      for (uint32_t x = 0; x < p; ++x) members[at++] = Pl(x);
    }
    ++nleaves;
    nmembers += h + p;
  };
  // the root's child: its frame at depth 0
  uint64_t S[W];
  all_bits<W>(S, d);
  const uint32_t q = qv[t];
  Hl(0) = v;
  if (code & kPivotTask) {
    Pl(0) = L[q];
    for (uint32_t w = 0; w < W; ++w) F(0, w) = S[w] & A[(size_t)q * W + w];
    F(0, 2 * W) = ((uint64_t)1 << 16) | ((uint64_t)1 << 32);   // h 1, p 1, stage 0
  } else {
    uint64_t NQ[W], C[W];
    for (uint32_t w = 0; w < W; ++w) NQ[w] = S[w] & ~A[(size_t)q * W + w];
    NQ[q >> 6] &= ~(1ull << (q & 63));
    hold_child<W>(S, NQ, A, code, C);
    Hl(1) = L[code];
    for (uint32_t w = 0; w < W; ++w) F(0, w) = C[w];
    F(0, 2 * W) = (uint64_t)2 << 16;   // h 2, p 0, stage 0
  }
  uint32_t depth = 1;
  while (depth > 0) {
    const uint32_t f = depth - 1;
    const uint64_t meta = F(f, 2 * W);
    const uint32_t h = (uint32_t)(meta >> 16) & 0xFFFFu, p = (uint32_t)(meta >> 32) & 0xFFFFu;
    const uint32_t stage = (uint32_t)(meta >> 48);
    uint64_t Sf[W];
    for (uint32_t w = 0; w < W; ++w) Sf[w] = F(f, w);
    if (stage == 0) {
      uint32_t cs = 0;
      for (uint32_t w = 0; w < W; ++w) cs += __popcll(Sf[w]);
      if (h == k) { emit(h, 0); --depth; continue; }
      if (h + p + cs < k) { --depth; continue; }
      if (cs == 0) {
        if (p >= k - h) emit(h, p);
        --depth;
        continue;
      }
      // pivot: the member of S with the most neighbours in S (lowest index on ties)
      uint32_t qq = 0, best = 0;
      bool first = true;
      for (uint32_t w = 0; w < W; ++w) {
        uint64_t bits = Sf[w];
        while (bits) {
          const uint32_t x = w * 64 + (uint32_t)__ffsll((unsigned long long)bits) - 1;
          bits &= bits - 1;
          uint32_t c = 0;
          for (uint32_t y = 0; y < W; ++y) c += __popcll(A[(size_t)x * W + y] & Sf[y]);
          if (first || c > best) { qq = x; best = c; first = false; }
        }
      }
      if (depth == nframes || p >= D) { atomicOr(err, 2); return; }
      uint64_t Aq[W];
      for (uint32_t w = 0; w < W; ++w) Aq[w] = A[(size_t)qq * W + w];
      for (uint32_t w = 0; w < W; ++w) {
        uint64_t nn = Sf[w] & ~Aq[w];
        if (w == (qq >> 6)) nn &= ~(1ull << (qq & 63));
        F(f, W + w) = nn;
      }
      F(f, 2 * W) = (uint64_t)qq | ((uint64_t)h << 16) | ((uint64_t)p << 32) | (1ull << 48);
      Pl(p) = L[qq];
      for (uint32_t w = 0; w < W; ++w) F(depth, w) = Sf[w] & Aq[w];
      F(depth, 2 * W) = ((uint64_t)h << 16) | ((uint64_t)(p + 1) << 32);
      ++depth;
      continue;
    }
    // stage 1: the next non-neighbour of the pivot, as a hold node
    uint32_t w0 = W;
    uint64_t nw = 0;
    for (uint32_t w = 0; w < W; ++w) {
      nw = F(f, W + w);
      if (nw) { w0 = w; break; }
    }
    if (w0 == W) { --depth; continue; }
    const uint32_t wi = w0 * 64 + (uint32_t)__ffsll((unsigned long long)nw) - 1;
    F(f, W + w0) = nw & (nw - 1);
    if (depth == nframes || h >= kSctMaxHold) { atomicOr(err, 2); return; }
    Hl(h) = L[wi];
    for (uint32_t w = 0; w < W; ++w) F(depth, w) = Sf[w] & A[(size_t)wi * W + w];
    F(f, wi >> 6) = Sf[wi >> 6] & ~(1ull << (wi & 63));   // later branches exclude w
    F(depth, 2 * W) = ((uint64_t)(h + 1) << 16) | ((uint64_t)p << 32);
    ++depth;
  }
  if (!write) {
    counts[2 * (size_t)i] = nleaves;
    counts[2 * (size_t)i + 1] = nmembers;
  }
}

}  // namespace

namespace {

template <uint32_t W>
void launch_root(hipStream_t st, const uint64_t* orp, const uint32_t* ocol, const uint32_t* perm, uint32_t k,
                 uint32_t D, uint32_t nact, uint64_t* abits, const uint64_t* aoff, uint32_t* qv, int write,
                 uint32_t* tcnt, const uint64_t* toff, uint64_t* tasks, int* err) {
  root_kernel<W><<<(nact + 63) / 64, 64, 0, st>>>(orp, ocol, perm, k, D, nact, abits, aoff, qv, write, tcnt, toff,
                                                  tasks, err);
}

template <uint32_t W>
void launch_task(hipStream_t st, const uint64_t* orp, const uint32_t* ocol, const uint32_t* perm, uint32_t k,
                 uint32_t D, const uint64_t* abits, const uint64_t* aoff, const uint32_t* qv, const uint64_t* tasks,
                 uint64_t v0, uint32_t c, uint64_t* s64, uint32_t* s32, int write, uint64_t* counts,
                 const uint64_t* loff, const uint64_t* moff, uint32_t* hp, uint32_t* mem, int* err) {
  task_kernel<W><<<(c + 63) / 64, 64, 0, st>>>(orp, ocol, perm, k, D, abits, aoff, qv, tasks, v0, c, s64, s32, write,
                                               counts, loff, moff, hp, mem, err);
}

}  // namespace

// The build's device buffers are carved, 256-byte aligned, from the caller's
// workspace in the order they are needed; the leaves are written through a
// staging window (what is left at the end) chunk by chunk.
struct WsCarve {
  char* base;
  size_t cap, used;
  size_t left() const { return used < cap ? cap - used : 0; }
  int take(void** p, size_t bytes) {
    const size_t b = (std::max<size_t>(bytes, 8) + 255) & ~(size_t)255;
    if (used + b > cap)
      return kdss::fail(KDSS_EWORKSPACE, "GPU tree build workspace too small (" + std::to_string(used + b) +
                                             " bytes needed so far, " + std::to_string(cap) + " given)");
    *p = base + used;
    used += b;
    return KDSS_OK;
  }
};

constexpr size_t kSctStaging = size_t(512) << 20;   // suggested staging window for the leaves

// Per task thread: the recursion's scratch plus its count and offset entries.
inline size_t sct_task_bytes(uint32_t D, uint32_t W) { return sct_words64(D, W) * 8 + sct_words32(D) * 4 + 32; }

extern "C" int kdss_sct_build_gpu_workspace(const kdss_csr* g, uint32_t k, size_t* bytes) {
  if (!g || !bytes) return kdss::fail(KDSS_EINVAL, "null argument");
  if (k < 2) return kdss::fail(KDSS_EINVAL, "k must be at least 2");
  if (k > kdss::kMaxK) return kdss::fail(KDSS_ERANGE, "k must be at most 31");
  int rc = kdss::validate_csr(g);
  if (rc) return rc;
  kdss::Degeneracy deg;
  kdss::degeneracy_order(g, &deg);   // the device peeling reaches the same degeneracy
  const uint32_t D = deg.degeneracy;
  if (D > kSctMaxLocal) return kdss::fail(KDSS_EUNSUPPORTED, "the GPU tree build handles degeneracy up to 256");
  const uint32_t W = std::max<uint32_t>(1, (D + 63) / 64);
  const uint64_t n = g->n, nnz = g->nnz;
  auto al = [](size_t b) { return (std::max<size_t>(b, 8) + 255) & ~(size_t)255; };
  const uint64_t ntile = (n + kPeelTile - 1) / kPeelTile;
  size_t sz = al((n + 1) * 8) + al(nnz * 4) + 3 * al(n * 4) + al((n + 1) * 8) + al(nnz / 2 * 4) + al(n * 4) + al(4) +
              3 * al(n * 4) + 2 * al(ntile * 4);
  // roots: bitsets of the later neighbours (out-degrees sum to nnz / 2), offsets, pivots, task counts
  sz += al(nnz / 2 * W * 8) + al((n + 1) * 8) + 2 * al(n * 4) + al((n + 1) * 8);
  // tasks: at most one per later neighbour plus the pivot child of each start node
  const uint64_t ntask = nnz / 2 + n;
  sz += al(ntask * 8);
  const uint64_t chunk = std::max<uint64_t>(64, std::min<uint64_t>(std::max<uint64_t>(ntask, 1),
                                                                     kSctScratchBudget / sct_task_bytes(D, W)));
  sz += 5 * 256 + chunk * sct_task_bytes(D, W);
  sz += kSctStaging;
  *bytes = sz;
  return KDSS_OK;
}

extern "C" int kdss_sct_build_gpu(const kdss_csr* g, uint32_t k, void* d_ws, size_t ws_bytes, void* stream,
                                  kdss_sct** out) {
  using clock = std::chrono::steady_clock;
  if (!g || !out) return kdss::fail(KDSS_EINVAL, "null argument");
  if (k < 2) return kdss::fail(KDSS_EINVAL, "k must be at least 2");
  if (k > kdss::kMaxK) return kdss::fail(KDSS_ERANGE, "k must be at most 31");
  const auto t0 = clock::now();   // the build time includes the graph check, as the host build's does
  int rc = kdss::validate_csr(g);
  if (rc) return rc;
  if (!d_ws) return kdss::fail(KDSS_EWORKSPACE, "null workspace (see kdss_sct_build_gpu_workspace)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  kdss_sct* s = new (std::nothrow) kdss_sct();
  if (!s) return kdss::fail(KDSS_ENOMEM, "cannot allocate the tree handle");
  kdss::Sct& T = s->s;
  const uint32_t n = g->n;
  T.n = n;
  T.k = k;
  uint32_t D = 0, W = 1;   // the degeneracy and the bitset words, known after the peeling
  WsCarve carve{static_cast<char*>(d_ws), ws_bytes, 0};
  auto cleanup = [&]() {};
  auto alloc = [&](void** p, size_t bytes) -> int { return carve.take(p, bytes); };
  auto run = [&]() -> int {
    uint64_t *rp = nullptr, *orp = nullptr;
    uint32_t *col = nullptr, *rank = nullptr, *ocnt = nullptr, *ocol = nullptr, *perm = nullptr;
    int* derr = nullptr;
    int r = KDSS_OK;
    if ((r = alloc((void**)&rp, ((size_t)n + 1) * 8)) || (r = alloc((void**)&col, g->nnz * 4)) ||
        (r = alloc((void**)&rank, (size_t)n * 4)) || (r = alloc((void**)&ocnt, (size_t)n * 4)) ||
        (r = alloc((void**)&orp, ((size_t)n + 1) * 8)) || (r = alloc((void**)&ocol, g->nnz / 2 * 4)) ||
        (r = alloc((void**)&perm, (size_t)n * 4)) || (r = alloc((void**)&derr, sizeof(int))))
      return r;
    SCT_TRY(hipMemcpyAsync(rp, g->row_ptr, ((size_t)n + 1) * 8, hipMemcpyHostToDevice, st), "upload graph");
    if (g->nnz) SCT_TRY(hipMemcpyAsync(col, g->col, g->nnz * 4, hipMemcpyHostToDevice, st), "upload graph");
    SCT_TRY(hipMemsetAsync(derr, 0, sizeof(int), st), "clear flag");
    // the order: level-synchronous peeling (one synchronisation per sub-round)
    {
      uint32_t *pdeg = nullptr, *pcore = nullptr, *pord = nullptr, *ptc = nullptr, *pto = nullptr;
      const uint32_t ntile = (n + kPeelTile - 1) / kPeelTile;
      if ((r = alloc((void**)&pdeg, (size_t)n * 4)) || (r = alloc((void**)&pcore, (size_t)n * 4)) ||
          (r = alloc((void**)&pord, (size_t)n * 4)) || (r = alloc((void**)&ptc, (size_t)ntile * 4)) ||
          (r = alloc((void**)&pto, (size_t)ntile * 4)))
        return r;
      if (n) {
        peel_init_kernel<<<(n + 255) / 256, 256, 0, st>>>(rp, n, pdeg, rank);
        SCT_TRY(hipGetLastError(), "peeling launch");
      }
      std::vector<uint32_t> tc(ntile), to(ntile);
      uint32_t L = 0, done = 0;
      while (done < n) {
        peel_count_kernel<<<ntile, 256, 0, st>>>(pdeg, rank, n, L, ptc);
        SCT_TRY(hipGetLastError(), "peeling launch");
        SCT_TRY(hipMemcpyAsync(tc.data(), ptc, (size_t)ntile * 4, hipMemcpyDeviceToHost, st), "read peeling counts");
        SCT_TRY(hipStreamSynchronize(st), "stream synchronize");
        uint64_t tot = 0;
        for (uint32_t b = 0; b < ntile; ++b) {
          to[b] = done + (uint32_t)tot;
          tot += tc[b];
        }
        if (tot == 0) {   // nobody left with at most L remaining neighbours
          ++L;
          continue;
        }
        if (tot > n - done) return kdss::fail(KDSS_EUNSUPPORTED, "internal: the peeling removed a node twice");
        SCT_TRY(hipMemcpyAsync(pto, to.data(), (size_t)ntile * 4, hipMemcpyHostToDevice, st), "upload ranks");
        peel_assign_kernel<<<ntile, 256, 0, st>>>(pdeg, rank, pcore, pord, n, L, pto);
        SCT_TRY(hipGetLastError(), "peeling launch");
        peel_drop_kernel<<<(uint32_t)((tot + 3) / 4), 256, 0, st>>>(rp, col, rank, pord, done, (uint32_t)tot, pdeg);
        SCT_TRY(hipGetLastError(), "peeling launch");
        done += (uint32_t)tot;
        D = std::max(D, L);
      }
      T.deg.rank.resize(n);
      T.deg.core.resize(n);
      T.deg.order.resize(n);
      if (n) {
        SCT_TRY(hipMemcpyAsync(T.deg.rank.data(), rank, (size_t)n * 4, hipMemcpyDeviceToHost, st), "read order");
        SCT_TRY(hipMemcpyAsync(T.deg.core.data(), pcore, (size_t)n * 4, hipMemcpyDeviceToHost, st), "read cores");
        SCT_TRY(hipStreamSynchronize(st), "stream synchronize");
      }
      for (uint32_t v = 0; v < n; ++v) {
        if (T.deg.rank[v] >= n) return kdss::fail(KDSS_EUNSUPPORTED, "internal: a node left without a rank");
        T.deg.order[T.deg.rank[v]] = v;
      }
      T.deg.degeneracy = D;
    }
    if (D > kSctMaxLocal) return kdss::fail(KDSS_EUNSUPPORTED, "the GPU tree build handles degeneracy up to 256");
    W = std::max<uint32_t>(1, (D + 63) / 64);
    // orientation along the order: out-degrees, offsets on the host, lists
    std::vector<uint32_t> oc(n);
    if (n) {
      orient_count_kernel<<<(n + 255) / 256, 256, 0, st>>>(rp, col, rank, n, ocnt);
      SCT_TRY(hipGetLastError(), "orientation count launch");
      SCT_TRY(hipMemcpyAsync(oc.data(), ocnt, (size_t)n * 4, hipMemcpyDeviceToHost, st), "read out-degrees");
      SCT_TRY(hipStreamSynchronize(st), "stream synchronize");
    }
    std::vector<uint64_t> ob(n + 1, 0);
    for (uint32_t v = 0; v < n; ++v) {
      if (oc[v] > D) return kdss::fail(KDSS_EUNSUPPORTED, "internal: an out-degree above the degeneracy");
      ob[v + 1] = ob[v] + oc[v];
    }
    if (ob[n] != g->nnz / 2) return kdss::fail(KDSS_EUNSUPPORTED, "internal: the orientation lost edges");
    // start nodes that can hold a k-clique, by decreasing out-degree (ties by id)
    std::vector<uint64_t> bucket(D + 2, 0);
    for (uint32_t v = 0; v < n; ++v)
      if (oc[v] + 1 >= k) ++bucket[D - oc[v] + 1];
    for (uint32_t b = 1; b <= D + 1; ++b) bucket[b] += bucket[b - 1];
    const uint32_t active = (uint32_t)bucket[D + 1];
    std::vector<uint32_t> order(std::max<uint32_t>(active, 1));
    for (uint32_t v = 0; v < n; ++v)
      if (oc[v] + 1 >= k) order[bucket[D - oc[v]]++] = v;
    SCT_TRY(hipMemcpyAsync(orp, ob.data(), ((size_t)n + 1) * 8, hipMemcpyHostToDevice, st), "upload offsets");
    if (active) SCT_TRY(hipMemcpyAsync(perm, order.data(), (size_t)active * 4, hipMemcpyHostToDevice, st),
                        "upload start order");
    if (n) {
      orient_fill_kernel<<<(n + 255) / 256, 256, 0, st>>>(rp, col, rank, n, orp, ocol);
      SCT_TRY(hipGetLastError(), "orientation fill launch");
    }
    // the roots: bitsets into the store (row length W words, start node t at
    // aoff[t]), pivots and the number of tasks of each start node
    std::vector<uint64_t> ao((size_t)active + 1, 0);
    for (uint32_t t = 0; t < active; ++t) ao[t + 1] = ao[t] + (uint64_t)oc[order[t]] * W;
    uint64_t *abits = nullptr, *aoff = nullptr, *toff = nullptr, *tasks = nullptr;
    uint32_t *qv = nullptr, *tcnt = nullptr;
    if ((r = alloc((void**)&abits, ao[active] * 8)) || (r = alloc((void**)&aoff, ((size_t)active + 1) * 8)) ||
        (r = alloc((void**)&qv, (size_t)active * 4)) || (r = alloc((void**)&tcnt, (size_t)active * 4)) ||
        (r = alloc((void**)&toff, ((size_t)active + 1) * 8)))
      return r;
    SCT_TRY(hipMemcpyAsync(aoff, ao.data(), ((size_t)active + 1) * 8, hipMemcpyHostToDevice, st), "upload offsets");
    auto roots = [&](int write) {
      if (!active) return hipSuccess;
      switch (W) {
        case 1: launch_root<1>(st, orp, ocol, perm, k, D, active, abits, aoff, qv, write, tcnt, toff, tasks, derr); break;
        case 2: launch_root<2>(st, orp, ocol, perm, k, D, active, abits, aoff, qv, write, tcnt, toff, tasks, derr); break;
        case 3: launch_root<3>(st, orp, ocol, perm, k, D, active, abits, aoff, qv, write, tcnt, toff, tasks, derr); break;
        default: launch_root<4>(st, orp, ocol, perm, k, D, active, abits, aoff, qv, write, tcnt, toff, tasks, derr); break;
      }
      return hipGetLastError();
    };
    SCT_TRY(roots(0), "tree root launch");
    std::vector<uint32_t> tc(std::max<uint32_t>(active, 1));
    if (active) SCT_TRY(hipMemcpyAsync(tc.data(), tcnt, (size_t)active * 4, hipMemcpyDeviceToHost, st), "read tasks");
    int herr = 0;
    SCT_TRY(hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, st), "read flag");
    SCT_TRY(hipStreamSynchronize(st), "stream synchronize");
    if (herr & 1) return kdss::fail(KDSS_EUNSUPPORTED, "internal: an out-list above the degeneracy");
    std::vector<uint64_t> to((size_t)active + 1, 0);
    for (uint32_t t = 0; t < active; ++t) {
      if (tc[t] > oc[order[t]] + 1) return kdss::fail(KDSS_EUNSUPPORTED, "internal: more root children than nodes");
      to[t + 1] = to[t] + tc[t];
    }
    const uint64_t ntask = to[active];
    if ((r = alloc((void**)&tasks, ntask * 8))) return r;
    SCT_TRY(hipMemcpyAsync(toff, to.data(), ((size_t)active + 1) * 8, hipMemcpyHostToDevice, st), "upload offsets");
    SCT_TRY(roots(1), "tree root launch");
    // scratch for one chunk of tasks: up to half of what is left (the rest
    // stages the leaves), at least 64 tasks
    const size_t per_task = sct_task_bytes(D, W);
    const uint64_t fit = carve.left() > 6 * 256 ? (carve.left() / 2 - 6 * 256) / per_task : 0;
    const uint32_t chunk = (uint32_t)std::max<uint64_t>(
        64, std::min<uint64_t>({std::max<uint64_t>(ntask, 1), kSctScratchBudget / per_task, fit}));
    uint64_t *s64 = nullptr, *dcounts = nullptr, *loff = nullptr, *moff = nullptr;
    uint32_t *s32 = nullptr, *dhp = nullptr, *dmem = nullptr;
    if ((r = alloc((void**)&s64, (size_t)chunk * sct_words64(D, W) * 8)) ||
        (r = alloc((void**)&s32, (size_t)chunk * sct_words32(D) * 4)) ||
        (r = alloc((void**)&dcounts, (size_t)chunk * 16)) || (r = alloc((void**)&loff, (size_t)chunk * 8)) ||
        (r = alloc((void**)&moff, (size_t)chunk * 8)))
      return r;
    auto launch = [&](uint64_t v0, uint32_t c, int write, uint32_t* hp, uint32_t* mem) {
      switch (W) {
        case 1: launch_task<1>(st, orp, ocol, perm, k, D, abits, aoff, qv, tasks, v0, c, s64, s32, write, dcounts, loff, moff, hp, mem, derr); break;
        case 2: launch_task<2>(st, orp, ocol, perm, k, D, abits, aoff, qv, tasks, v0, c, s64, s32, write, dcounts, loff, moff, hp, mem, derr); break;
        case 3: launch_task<3>(st, orp, ocol, perm, k, D, abits, aoff, qv, tasks, v0, c, s64, s32, write, dcounts, loff, moff, hp, mem, derr); break;
        default: launch_task<4>(st, orp, ocol, perm, k, D, abits, aoff, qv, tasks, v0, c, s64, s32, write, dcounts, loff, moff, hp, mem, derr); break;
      }
      return hipGetLastError();
    };
    // pass 1: leaves and members per task
    std::vector<uint64_t> counts(2 * (size_t)ntask);
    for (uint64_t v0 = 0; v0 < ntask; v0 += chunk) {
      const uint32_t c = (uint32_t)std::min<uint64_t>(chunk, ntask - v0);
      SCT_TRY(launch(v0, c, 0, nullptr, nullptr), "tree count launch");
      SCT_TRY(hipMemcpyAsync(counts.data() + 2 * (size_t)v0, dcounts, (size_t)c * 16, hipMemcpyDeviceToHost, st),
              "read counts");
    }
    SCT_TRY(hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, st), "read flag");
    SCT_TRY(hipStreamSynchronize(st), "stream synchronize");
    if (herr & 2) return kdss::fail(KDSS_EUNSUPPORTED, "internal: the tree recursion went deeper than its stack");
    std::vector<uint64_t> lo((size_t)ntask + 1, 0), mo((size_t)ntask + 1, 0);
    for (uint64_t x = 0; x < ntask; ++x) {
      lo[x + 1] = lo[x] + counts[2 * x];
      mo[x + 1] = mo[x] + counts[2 * x + 1];
    }
    const uint64_t L = lo[ntask], M = mo[ntask];
    if (L >= (1ull << 40)) return kdss::fail(KDSS_ERANGE, "more than 2^40 leaves");
    // pass 2: chunks of tasks whose leaves fit the staging window write them
    // there (offsets relative to the chunk's first task); each chunk is then
    // copied to its place in the host arrays
    char* stage = carve.base + carve.used;
    const size_t stage_bytes = carve.left();
    std::vector<uint32_t> hpv(L);
    T.members.resize(M);
    std::vector<uint64_t> rl(chunk), rm(chunk);
    for (uint64_t v0 = 0; v0 < ntask;) {
      uint64_t v1 = v0;
      auto need = [&](uint64_t e) { return ((lo[e] - lo[v0]) * 4 + 255) / 256 * 256 + (mo[e] - mo[v0]) * 4; };
      while (v1 < ntask && v1 - v0 < chunk && need(v1 + 1) <= stage_bytes) ++v1;
      if (v1 == v0)
        return kdss::fail(KDSS_EWORKSPACE, "GPU tree build workspace too small: one root child's leaves need " +
                                               std::to_string(need(v0 + 1)) + " staging bytes, " +
                                               std::to_string(stage_bytes) + " left");
      const uint32_t c = (uint32_t)(v1 - v0);
      const uint64_t dl = lo[v1] - lo[v0], dm = mo[v1] - mo[v0];
      dhp = reinterpret_cast<uint32_t*>(stage);
      dmem = reinterpret_cast<uint32_t*>(stage + (dl * 4 + 255) / 256 * 256);
      for (uint32_t x = 0; x < c; ++x) {
        rl[x] = lo[v0 + x] - lo[v0];
        rm[x] = mo[v0 + x] - mo[v0];
      }
      SCT_TRY(hipMemcpyAsync(loff, rl.data(), (size_t)c * 8, hipMemcpyHostToDevice, st), "upload offsets");
      SCT_TRY(hipMemcpyAsync(moff, rm.data(), (size_t)c * 8, hipMemcpyHostToDevice, st), "upload offsets");
      SCT_TRY(launch(v0, c, 1, dhp, dmem), "tree write launch");
      if (dl) SCT_TRY(hipMemcpyAsync(hpv.data() + lo[v0], dhp, dl * 4, hipMemcpyDeviceToHost, st), "read leaves");
      if (dm)
        SCT_TRY(hipMemcpyAsync(T.members.data() + mo[v0], dmem, dm * 4, hipMemcpyDeviceToHost, st), "read leaves");
      SCT_TRY(hipStreamSynchronize(st), "stream synchronize");   // offsets and staging are reused
      v0 = v1;
    }
    T.h.resize(L);
    T.p.resize(L);
    T.off.resize(L + 1);
    // C(p, j) for p <= D, j <= k (every leaf has p <= D pivots)
    std::vector<u128> cb((size_t)(D + 1) * (k + 1));
    for (uint32_t pp = 0; pp <= D; ++pp)
      for (uint32_t jj = 0; jj <= k; ++jj) cb[(size_t)pp * (k + 1) + jj] = kdss::binom128(pp, jj);
    uint64_t at = 0;
    u128 ck = 0;
    uint32_t smax = 0;
    for (uint64_t i = 0; i < L; ++i) {
      const uint32_t h = hpv[i] & 0xFFu, p = hpv[i] >> 8;
      if (p > D || h > k) return kdss::fail(KDSS_EUNSUPPORTED, "internal: a leaf outside the tree's bounds");
      T.h[i] = (uint8_t)h;
      T.p[i] = p;
      T.off[i] = at;
      at += h + p;
      smax = std::max(smax, h + p);
      const u128 c = cb[(size_t)p * (k + 1) + (k - h)];
      if (ck + c < ck) return kdss::fail(KDSS_EOVERFLOW, "2^128 or more k-cliques");
      ck += c;
    }
    T.off[L] = at;
    T.c_k = ck;
    T.s_max = smax;
    return KDSS_OK;
  };
  rc = run();
  cleanup();
  if (rc) {
    delete s;
    return rc;
  }
  T.build_seconds = std::chrono::duration<double>(clock::now() - t0).count();
  *out = s;
  return KDSS_OK;
}
