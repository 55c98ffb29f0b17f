// The k-pruned succinct clique tree (paper: Sec. 2, Lemmas 3-5) built on the
// GPU: one thread per start node v.  v's later neighbours in the degeneracy
// order (at most the degeneracy, here at most kSctMaxLocal) get local indices
// and adjacency bitsets; the pivoting recursion then runs with an explicit
// stack, both in a per-thread slice of global scratch (word i of thread t at
// i * threads + t, so a wavefront's equal-index accesses coalesce):
//   node (H, P, S): h = |H| = k: the leaf (H, {}); h + p + |S| < k: nothing;
//   S empty: the leaf (H, P) when p >= k - h; otherwise a pivot q of S with
//   the most neighbours in S: (H, P + q, S and N(q)), then for each w of S
//   not adjacent to q (w != q), in local order: (H + w, P, S and N(w) minus
//   the w handled before).
// Every k-clique of the graph lies in exactly one leaf (the tree of a node
// covers the cliques whose earliest node it is); the leaves may differ from
// the host build's, and any such tree gives the same results.
// Two passes over chunks of start nodes: counts, then the leaves written at
// the prefix-sum offsets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "kdss_internal.h"

using kdss::u128;

namespace {

constexpr uint32_t kSctMaxLocal = 256;                 // largest later-neighbour set handled
constexpr uint32_t kSctWords = kSctMaxLocal / 64;      // bitset words
constexpr uint32_t kSctFrames = kSctMaxLocal + 2;      // recursion depth <= |S| + 1
constexpr uint32_t kFrameWords = 2 * kSctWords + 1;    // S, NN, (q | h << 16 | p << 32 | stage << 48)
constexpr uint32_t kWords64 = kSctMaxLocal * kSctWords + kSctFrames * kFrameWords;
constexpr uint32_t kWords32 = kSctMaxLocal + 32 + kSctMaxLocal;   // local ids, hold list, pivot list
constexpr uint32_t kChunk = 32768;                     // start nodes per launch

int sct_hip_fail(hipError_t e, const char* what) {
  return kdss::fail(KDSS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define SCT_TRY(call, what)                              \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return sct_hip_fail(e_, what); \
  } while (0)

__device__ inline bool has_edge_dev(const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col, uint32_t a,
                                    uint32_t b) {
  uint64_t lo = rp[a], hi = rp[a + 1];
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < b) lo = mid + 1;
    else hi = mid;
  }
  return lo < rp[a + 1] && col[lo] == b;
}

// One thread per start node v0 + tid.  write = 0: counts[2 t] = leaves,
// counts[2 t + 1] = members.  write = 1: leaves from leaf_off[t], members from
// member_off[t]; hp[leaf] = h | p << 8.  *err: 1 = a later-neighbour set above
// kSctMaxLocal, 2 = the stack would overflow (neither writes out of bounds).
__global__ __launch_bounds__(64) void sct_kernel(const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col,
                                                 const uint32_t* __restrict__ rank, uint32_t n, uint32_t k,
                                                 uint32_t v0, uint32_t count, uint64_t* __restrict__ s64,
                                                 uint32_t* __restrict__ s32, int write,
                                                 uint64_t* __restrict__ counts, const uint64_t* __restrict__ leaf_off,
                                                 const uint64_t* __restrict__ member_off, uint32_t* __restrict__ hp,
                                                 uint32_t* __restrict__ members, int* __restrict__ err) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const uint32_t v = v0 + t;
  const size_t stride = count;
  auto A = [&](uint32_t i, uint32_t w) -> uint64_t& { return s64[((size_t)i * kSctWords + w) * stride + t]; };
  auto F = [&](uint32_t f, uint32_t w) -> uint64_t& {
    return s64[((size_t)kSctMaxLocal * kSctWords + (size_t)f * kFrameWords + w) * stride + t];
  };
  auto L = [&](uint32_t i) -> uint32_t& { return s32[(size_t)i * stride + t]; };
  auto Hl = [&](uint32_t i) -> uint32_t& { return s32[((size_t)kSctMaxLocal + i) * stride + t]; };
  auto Pl = [&](uint32_t i) -> uint32_t& { return s32[((size_t)kSctMaxLocal + 32 + i) * stride + t]; };
  uint64_t nleaves = 0, nmembers = 0;
  uint64_t lo_leaf = write ? leaf_off[t] : 0, lo_mem = write ? member_off[t] : 0;
  // later neighbours of v (ascending ids, as in its row)
  uint32_t d = 0;
  const uint32_t rv = rank[v];
  for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
    const uint32_t u = col[e];
    if (rank[u] <= rv) continue;
    if (d == kSctMaxLocal) {
      atomicOr(err, 1);
      return;
    }
    L(d++) = u;
  }
  if (d + 1 >= k || (k == 2 && d >= 1)) {
    for (uint32_t i = 0; i < d; ++i)
      for (uint32_t w = 0; w < kSctWords; ++w) A(i, w) = 0;
    for (uint32_t i = 0; i < d; ++i)
      for (uint32_t j = i + 1; j < d; ++j)
        if (has_edge_dev(rp, col, L(i), L(j))) {
          A(i, j >> 6) |= 1ull << (j & 63);
          A(j, i >> 6) |= 1ull << (i & 63);
        }
    auto emit = [&](uint32_t h, uint32_t p) {
      if (write) {
        hp[lo_leaf + nleaves] = h | (p << 8);
        uint64_t at = lo_mem + nmembers;
        for (uint32_t i = 0; i < h; ++i) members[at++] = Hl(i);
        for (uint32_t i = 0; i < p; ++i) members[at++] = Pl(i);
      }
      ++nleaves;
      nmembers += h + p;
    };
    // root frame: H = {v}, P = {}, S = all later neighbours
    Hl(0) = v;
    for (uint32_t w = 0; w < kSctWords; ++w) {
      const uint32_t lo = w * 64;
      F(0, w) = d >= lo + 64 ? ~0ull : (d > lo ? (1ull << (d - lo)) - 1 : 0ull);
    }
    F(0, 2 * kSctWords) = (uint64_t)1 << 16;   // q 0, h 1, p 0, stage 0
    uint32_t depth = 1;
    while (depth > 0) {
      const uint32_t f = depth - 1;
      const uint64_t meta = F(f, 2 * kSctWords);
      const uint32_t h = (uint32_t)(meta >> 16) & 0xFFFFu, p = (uint32_t)(meta >> 32) & 0xFFFFu;
      const uint32_t stage = (uint32_t)(meta >> 48);
      if (stage == 0) {
        uint32_t cs = 0;
        for (uint32_t w = 0; w < kSctWords; ++w) cs += __popcll(F(f, w));
        if (h == k) { emit(h, 0); --depth; continue; }
        if (h + p + cs < k) { --depth; continue; }
        if (cs == 0) {
          if (p >= k - h) emit(h, p);
          --depth;
          continue;
        }
        // pivot: the member of S with the most neighbours in S (lowest index on ties)
        uint32_t q = 0, best = 0;
        bool first = true;
        for (uint32_t w = 0; w < kSctWords; ++w) {
          uint64_t bits = F(f, w);
          while (bits) {
            const uint32_t i = w * 64 + (uint32_t)__ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
            uint32_t c = 0;
            for (uint32_t x = 0; x < kSctWords; ++x) c += __popcll(A(i, x) & F(f, x));
            if (first || c > best) { q = i; best = c; first = false; }
          }
        }
        for (uint32_t w = 0; w < kSctWords; ++w) F(f, kSctWords + w) = F(f, w) & ~A(q, w);
        F(f, kSctWords + (q >> 6)) &= ~(1ull << (q & 63));
        F(f, 2 * kSctWords) = (uint64_t)q | ((uint64_t)h << 16) | ((uint64_t)p << 32) | (1ull << 48);
        if (depth == kSctFrames || p >= kSctMaxLocal) { atomicOr(err, 2); return; }
        Pl(p) = L(q);
        for (uint32_t w = 0; w < kSctWords; ++w) F(depth, w) = F(f, w) & A(q, w);
        F(depth, 2 * kSctWords) = ((uint64_t)h << 16) | ((uint64_t)(p + 1) << 32);
        ++depth;
        continue;
      }
      // stage 1: the next non-neighbour of the pivot, as a hold node
      uint32_t w0 = kSctWords;
      for (uint32_t w = 0; w < kSctWords; ++w)
        if (F(f, kSctWords + w)) { w0 = w; break; }
      if (w0 == kSctWords) { --depth; continue; }
      const uint32_t wi = w0 * 64 + (uint32_t)__ffsll((unsigned long long)F(f, kSctWords + w0)) - 1;
      F(f, kSctWords + w0) &= ~(1ull << (wi & 63));
      if (depth == kSctFrames || h >= 32) { atomicOr(err, 2); return; }
      Hl(h) = L(wi);
      for (uint32_t w = 0; w < kSctWords; ++w) F(depth, w) = F(f, w) & A(wi, w);
      F(f, wi >> 6) &= ~(1ull << (wi & 63));   // later branches exclude w
      F(depth, 2 * kSctWords) = ((uint64_t)(h + 1) << 16) | ((uint64_t)p << 32);
      ++depth;
    }
  }
  if (!write) {
    counts[2 * (size_t)t] = nleaves;
    counts[2 * (size_t)t + 1] = nmembers;
  }
}

}  // namespace

extern "C" int kdss_sct_build_gpu(const kdss_csr* g, uint32_t k, void* stream, kdss_sct** out) {
  using clock = std::chrono::steady_clock;
  if (!g || !out) return kdss::fail(KDSS_EINVAL, "null argument");
  if (k < 2) return kdss::fail(KDSS_EINVAL, "k must be at least 2");
  if (k > kdss::kMaxK) return kdss::fail(KDSS_ERANGE, "k must be at most 31");
  int rc = kdss::validate_csr(g);
  if (rc) return rc;
  const auto t0 = clock::now();
  hipStream_t st = static_cast<hipStream_t>(stream);
  kdss_sct* s = new (std::nothrow) kdss_sct();
  if (!s) return kdss::fail(KDSS_ENOMEM, "cannot allocate the tree handle");
  kdss::Sct& T = s->s;
  const uint32_t n = g->n;
  T.n = n;
  T.k = k;
  kdss::degeneracy_order(g, &T.deg);
  if (T.deg.degeneracy > kSctMaxLocal) {
    delete s;
    return kdss::fail(KDSS_EUNSUPPORTED, "the GPU tree build handles degeneracy up to 256");
  }
  std::vector<uint64_t> counts(2 * (size_t)n);
  std::vector<void*> bufs;
  auto cleanup = [&]() {
    for (void* p : bufs) (void)hipFree(p);
  };
  auto alloc = [&](void** p, size_t bytes) -> int {
    if (hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) return kdss::fail(KDSS_ENOMEM, "device memory");
    bufs.push_back(*p);
    return KDSS_OK;
  };
  uint64_t *rp = nullptr, *s64 = nullptr, *dcounts = nullptr, *loff = nullptr, *moff = nullptr;
  uint32_t *col = nullptr, *rank = nullptr, *s32 = nullptr, *dhp = nullptr, *dmem = nullptr;
  int* derr = nullptr;
  const uint32_t chunk = std::min<uint32_t>(std::max<uint32_t>(n, 1), kChunk);
  int rcx = KDSS_OK;
  if ((rcx = alloc((void**)&rp, ((size_t)n + 1) * 8)) || (rcx = alloc((void**)&col, g->nnz * 4)) ||
      (rcx = alloc((void**)&rank, (size_t)n * 4)) || (rcx = alloc((void**)&s64, (size_t)chunk * kWords64 * 8)) ||
      (rcx = alloc((void**)&s32, (size_t)chunk * kWords32 * 4)) ||
      (rcx = alloc((void**)&dcounts, (size_t)chunk * 16)) || (rcx = alloc((void**)&loff, (size_t)chunk * 8)) ||
      (rcx = alloc((void**)&moff, (size_t)chunk * 8)) || (rcx = alloc((void**)&derr, sizeof(int)))) {
    cleanup();
    delete s;
    return rcx;
  }
  auto run = [&]() -> int {
    SCT_TRY(hipMemcpyAsync(rp, g->row_ptr, ((size_t)n + 1) * 8, hipMemcpyHostToDevice, st), "upload graph");
    if (g->nnz) SCT_TRY(hipMemcpyAsync(col, g->col, g->nnz * 4, hipMemcpyHostToDevice, st), "upload graph");
    SCT_TRY(hipMemcpyAsync(rank, T.deg.rank.data(), (size_t)n * 4, hipMemcpyHostToDevice, st), "upload order");
    SCT_TRY(hipMemsetAsync(derr, 0, sizeof(int), st), "clear flag");
    // pass 1: leaves and members per start node
    for (uint32_t v0 = 0; v0 < n; v0 += chunk) {
      const uint32_t c = std::min(chunk, n - v0);
      sct_kernel<<<(c + 63) / 64, 64, 0, st>>>(rp, col, rank, n, k, v0, c, s64, s32, 0, dcounts, nullptr, nullptr,
                                               nullptr, nullptr, derr);
      SCT_TRY(hipGetLastError(), "tree count launch");
      SCT_TRY(hipMemcpyAsync(counts.data() + 2 * (size_t)v0, dcounts, (size_t)c * 16, hipMemcpyDeviceToHost, st),
              "read counts");
    }
    int herr = 0;
    SCT_TRY(hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, st), "read flag");
    SCT_TRY(hipStreamSynchronize(st), "stream synchronize");
    if (herr & 1) return kdss::fail(KDSS_EUNSUPPORTED, "a later-neighbour set above 256 nodes");
    if (herr & 2) return kdss::fail(KDSS_EUNSUPPORTED, "the tree recursion went deeper than its stack");
    std::vector<uint64_t> lo(n + 1, 0), mo(n + 1, 0);
    for (uint32_t v = 0; v < n; ++v) {
      lo[v + 1] = lo[v] + counts[2 * (size_t)v];
      mo[v + 1] = mo[v] + counts[2 * (size_t)v + 1];
    }
    const uint64_t L = lo[n], M = mo[n];
    if (L >= (1ull << 40)) return kdss::fail(KDSS_ERANGE, "more than 2^40 leaves");
    int r2 = alloc((void**)&dhp, L * 4);
    if (!r2) r2 = alloc((void**)&dmem, M * 4);
    if (r2) return r2;
    // pass 2: the leaves at their offsets (offsets relative to the chunk's first node)
    std::vector<uint64_t> cl(chunk), cm(chunk);
    for (uint32_t v0 = 0; v0 < n; v0 += chunk) {
      const uint32_t c = std::min(chunk, n - v0);
      for (uint32_t i = 0; i < c; ++i) {
        cl[i] = lo[v0 + i];
        cm[i] = mo[v0 + i];
      }
      SCT_TRY(hipMemcpyAsync(loff, cl.data(), (size_t)c * 8, hipMemcpyHostToDevice, st), "upload offsets");
      SCT_TRY(hipMemcpyAsync(moff, cm.data(), (size_t)c * 8, hipMemcpyHostToDevice, st), "upload offsets");
      sct_kernel<<<(c + 63) / 64, 64, 0, st>>>(rp, col, rank, n, k, v0, c, s64, s32, 1, nullptr, loff, moff, dhp,
                                               dmem, derr);
      SCT_TRY(hipGetLastError(), "tree write launch");
      SCT_TRY(hipStreamSynchronize(st), "stream synchronize");   // the host offset buffers are reused
    }
    std::vector<uint32_t> hpv(L);
    T.members.resize(M);
    if (L) SCT_TRY(hipMemcpyAsync(hpv.data(), dhp, L * 4, hipMemcpyDeviceToHost, st), "read leaves");
    if (M) SCT_TRY(hipMemcpyAsync(T.members.data(), dmem, M * 4, hipMemcpyDeviceToHost, st), "read leaves");
    SCT_TRY(hipStreamSynchronize(st), "stream synchronize");
    T.h.resize(L);
    T.p.resize(L);
    T.off.resize(L + 1);
    uint64_t at = 0;
    u128 ck = 0;
    uint32_t smax = 0;
    for (uint64_t i = 0; i < L; ++i) {
      const uint32_t h = hpv[i] & 0xFFu, p = hpv[i] >> 8;
      T.h[i] = (uint8_t)h;
      T.p[i] = p;
      T.off[i] = at;
      at += h + p;
      smax = std::max(smax, h + p);
      const u128 c = kdss::binom128(p, k - h);
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
