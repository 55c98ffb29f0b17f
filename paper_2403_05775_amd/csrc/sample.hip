// CPSample (paper: Algorithm 4): a clique tree of uniformly sampled k-cliques.
//
// Colour-increasing k-node paths are sampled uniformly (the CCPATH sampler the
// algorithm cites); the ones that are cliques are uniform k-cliques, and the
// distinct ones become leaves (C, {}) of a tree that the ordinary plan and run
// process: a leaf with h = k credits its minimum-load member once per
// iteration (Algorithm 4's loop) and counts once in every prefix that holds
// it (the extraction by rho'_k).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "kdss_internal.h"

using kdss::u128;

namespace {

int sample_hip_fail(hipError_t e, const char* what) {
  return kdss::fail(KDSS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define SAMPLE_TRY(call, what)                               \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return sample_hip_fail(e_, what);  \
  } while (0)

constexpr uint32_t kSampleThreads = 256, kSampleItems = 4, kSampleTile = kSampleThreads * kSampleItems;

// P_j(v) = sum over neighbours u with a higher colour of P_{j-1}(u); *overflow
// is set when a sum reaches 2^128.
__global__ __launch_bounds__(256) void path_count_kernel(const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col,
                                                         const uint32_t* __restrict__ color, uint32_t n,
                                                         const u128* __restrict__ prev, u128* __restrict__ cur,
                                                         int* __restrict__ overflow) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const uint32_t cv = color[v];
    u128 s = 0;
    bool ovf = false;
    for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
      const uint32_t u = col[e];
      if (color[u] <= cv) continue;
      const u128 w = prev[u];
      ovf |= s + w < s;
      s += w;
    }
    cur[v] = s;
    if (ovf) *overflow = 1;
  }
}

// inclusive prefix sums of a[0..n) (u128): block sums, one-thread scan of the
// block sums, then each block's prefixes
// Sums that wrap past 2^128 - 1 set *ovf (a carry shows as s + v < s).
__device__ __forceinline__ void add_checked(u128& s, u128 v, bool& wrapped) {
  const u128 t = s + v;
  wrapped |= t < s;
  s = t;
}

__global__ __launch_bounds__(kSampleThreads) void prefix_blocksum_kernel(const u128* __restrict__ a, uint32_t n,
                                                                         u128* __restrict__ bs, int* ovf) {
  __shared__ u128 part[kSampleThreads];
  const uint32_t base = blockIdx.x * kSampleTile + threadIdx.x * kSampleItems;
  u128 s = 0;
  bool wrapped = false;
  for (uint32_t q = 0; q < kSampleItems; ++q)
    if (base + q < n) add_checked(s, a[base + q], wrapped);
  part[threadIdx.x] = s;
  if (wrapped) atomicOr(ovf, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    u128 t = 0;
    bool w2 = false;
    for (uint32_t i = 0; i < kSampleThreads; ++i) add_checked(t, part[i], w2);
    bs[blockIdx.x] = t;
    if (w2) atomicOr(ovf, 1);
  }
}

__global__ void prefix_scan_kernel(u128* __restrict__ bs, uint32_t nb, int* ovf) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  u128 run = 0;
  bool wrapped = false;
  for (uint32_t b = 0; b < nb; ++b) {
    const u128 v = bs[b];
    bs[b] = run;
    add_checked(run, v, wrapped);
  }
  if (wrapped) atomicOr(ovf, 1);
}

__global__ __launch_bounds__(kSampleThreads) void prefix_write_kernel(const u128* __restrict__ a, uint32_t n,
                                                                      const u128* __restrict__ bs,
                                                                      u128* __restrict__ pre) {
  __shared__ u128 part[kSampleThreads];
  const uint32_t base = blockIdx.x * kSampleTile + threadIdx.x * kSampleItems;
  u128 s = 0;
  for (uint32_t q = 0; q < kSampleItems; ++q)
    if (base + q < n) s += a[base + q];
  part[threadIdx.x] = s;
  __syncthreads();
  u128 run = bs[blockIdx.x];
  for (uint32_t i = 0; i < threadIdx.x; ++i) run += part[i];
  for (uint32_t q = 0; q < kSampleItems; ++q)
    if (base + q < n) {
      run += a[base + q];
      pre[base + q] = run;
    }
}

__device__ bool adjacent(const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col, uint32_t a, uint32_t b) {
  uint64_t lo = rp[a], hi = rp[a + 1];
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < b) lo = mid + 1;
    else hi = mid;
  }
  return lo < rp[a + 1] && col[lo] == b;
}

// One sample per thread: the start by its share of [0, total) (binary search
// over the inclusive prefix sums), then each next node by its share among the
// higher-coloured neighbours, in adjacency order.  Writes the sorted ids and
// whether they form a clique.
__global__ __launch_bounds__(256) void sample_walk_kernel(const uint64_t* __restrict__ rp,
                                                          const uint32_t* __restrict__ col,
                                                          const uint32_t* __restrict__ color, uint32_t n, uint32_t k,
                                                          const u128* __restrict__ P, const u128* __restrict__ pre,
                                                          u128 total, const uint64_t* __restrict__ draws, uint64_t t,
                                                          uint32_t* __restrict__ out, uint8_t* __restrict__ valid) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < t; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t* d = draws + 2 * i * k;
    uint32_t path[32];
    const u128 x = (((u128)d[0] << 64) | d[1]) % total;
    uint32_t lo = 0, hi = n - 1;   // the first v with pre[v] > x (pre[n - 1] = total > x)
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo) / 2;
      if (pre[mid] > x) hi = mid;
      else lo = mid + 1;
    }
    uint32_t v = lo;
    path[0] = v;
    bool ok = true;
    for (uint32_t s = 1; s < k && ok; ++s) {
      const uint32_t j = k - s + 1;   // nodes left on the path, v included
      const u128 pj = P[(size_t)j * n + v];
      if (pj == 0) { ok = false; break; }   // cannot happen: v was drawn with a positive share
      u128 y = (((u128)d[2 * s] << 64) | d[2 * s + 1]) % pj;
      uint32_t next = 0xFFFFFFFFu;
      const uint32_t cv = color[v];
      for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
        const uint32_t u = col[e];
        if (color[u] <= cv) continue;
        const u128 w = P[(size_t)(j - 1) * n + u];
        if (y < w) { next = u; break; }
        y -= w;
      }
      if (next == 0xFFFFFFFFu) { ok = false; break; }
      v = next;
      path[s] = v;
    }
    bool clique = ok;
    for (uint32_t a = 0; a < k && clique; ++a)
      for (uint32_t b = a + 1; b < k && clique; ++b)
        if (!adjacent(rp, col, path[a], path[b])) clique = false;
    if (!ok)
      for (uint32_t a = 0; a < k; ++a) path[a] = 0;
    for (uint32_t a = 1; a < k; ++a) {   // ascending ids
      const uint32_t key = path[a];
      uint32_t b = a;
      for (; b > 0 && path[b - 1] > key; --b) path[b] = path[b - 1];
      path[b] = key;
    }
    for (uint32_t a = 0; a < k; ++a) out[i * k + a] = path[a];
    valid[i] = clique ? 1 : 0;
  }
}

// Greedy colouring: nodes by degree (descending, ties by ascending id), each
// the smallest colour none of its coloured neighbours has.
uint32_t greedy_colour(const kdss_csr* g, std::vector<uint32_t>& color) {
  const uint32_t n = g->n;
  std::vector<uint32_t> order(n), mark(n + 2, 0xFFFFFFFFu);
  std::iota(order.begin(), order.end(), 0u);
  auto deg = [&](uint32_t v) { return g->row_ptr[v + 1] - g->row_ptr[v]; };
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return deg(a) > deg(b); });
  color.assign(n, 0xFFFFFFFFu);
  uint32_t used = 0;
  for (uint32_t v : order) {
    for (uint64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e)
      if (color[g->col[e]] != 0xFFFFFFFFu) mark[color[g->col[e]]] = v;
    uint32_t c = 0;
    while (mark[c] == v) ++c;
    color[v] = c;
    used = std::max(used, c + 1);
  }
  return used;
}

// Device buffers carved from the caller's workspace (256-byte aligned pieces).
struct Carve {
  char* base;
  size_t cap, used;
  template <class T>
  int take(T** p, size_t count) {
    const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) & ~(size_t)255;
    if (base && used + bytes <= cap) *p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return KDSS_OK;
  }
};

// The pieces of one sampling call; with c.base == nullptr only the size is summed.
template <class F>
void sample_pieces(Carve& c, uint32_t n, uint64_t nnz, uint32_t k, uint64_t t, F&& bind) {
  const uint32_t nb = (n + kSampleTile - 1) / kSampleTile;
  uint64_t* rp = nullptr;
  uint32_t *col = nullptr, *dcolor = nullptr, *dout = nullptr;
  u128 *P = nullptr, *pre = nullptr, *bs = nullptr;
  uint64_t* draws = nullptr;
  uint8_t* dvalid = nullptr;
  int* ovf = nullptr;
  c.take(&rp, (size_t)n + 1);
  c.take(&col, nnz);
  c.take(&dcolor, n);
  c.take(&P, (size_t)(k + 1) * n);
  c.take(&pre, n);
  c.take(&bs, nb);
  c.take(&draws, (size_t)2 * t * k);
  c.take(&dout, (size_t)t * k);
  c.take(&dvalid, t);
  c.take(&ovf, 1);
  bind(rp, col, dcolor, P, pre, bs, draws, dout, dvalid, ovf, nb);
}

}  // namespace

extern "C" int kdss_sample_workspace(uint32_t n, uint64_t nnz, uint32_t k, uint64_t t, size_t* bytes) {
  if (!bytes) return kdss::fail(KDSS_EINVAL, "null argument");
  if (k < 2) return kdss::fail(KDSS_EINVAL, "k must be at least 2");
  if (k > kdss::kMaxK) return kdss::fail(KDSS_ERANGE, "k above 31");
  Carve c{nullptr, 0, 0};
  if (n > 0 && t > 0) sample_pieces(c, n, nnz, k, t, [](auto...) {});
  *bytes = c.used;
  return KDSS_OK;
}

extern "C" int kdss_sample_build(const kdss_csr* g, uint32_t k, uint64_t t, const uint64_t* h_draws, void* d_ws,
                                 size_t ws_bytes, void* stream, kdss_sample_info* info, kdss_sct** out) {
  using clock = std::chrono::steady_clock;
  if (!g || !out || (t && !h_draws)) return kdss::fail(KDSS_EINVAL, "null argument");
  if (k < 2) return kdss::fail(KDSS_EINVAL, "k must be at least 2");
  if (k > kdss::kMaxK) return kdss::fail(KDSS_ERANGE, "k above 31");
  int rc = kdss::validate_csr(g);
  if (rc) return rc;
  size_t need = 0;
  rc = kdss_sample_workspace(g->n, g->nnz, k, t, &need);
  if (rc) return rc;
  if (need > 0 && (!d_ws || ws_bytes < need))
    return kdss::fail(KDSS_EWORKSPACE, "sampler workspace smaller than kdss_sample_workspace() reports");
  const auto t0 = clock::now();
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t n = g->n;
  std::vector<uint32_t> color;
  const uint32_t ncolors = greedy_colour(g, color);
  kdss_sample_info inf{};
  inf.samples = t;
  inf.colors = ncolors;
  std::vector<uint32_t> cl((size_t)t * k);
  std::vector<uint8_t> valid(t);
  double dev_s = 0.0;
  if (n > 0 && t > 0) {
    uint64_t* rp = nullptr;
    uint32_t *col = nullptr, *dcolor = nullptr, *dout = nullptr;
    u128 *P = nullptr, *pre = nullptr, *bs = nullptr;
    uint64_t* draws = nullptr;
    uint8_t* dvalid = nullptr;
    int* ovf = nullptr;
    uint32_t nb = 0;
    Carve c{static_cast<char*>(d_ws), ws_bytes, 0};
    sample_pieces(c, n, g->nnz, k, t, [&](auto rp_, auto col_, auto dcolor_, auto P_, auto pre_, auto bs_,
                                          auto draws_, auto dout_, auto dvalid_, auto ovf_, uint32_t nb_) {
      rp = rp_; col = col_; dcolor = dcolor_; P = P_; pre = pre_; bs = bs_; draws = draws_; dout = dout_;
      dvalid = dvalid_; ovf = ovf_; nb = nb_;
    });
    SAMPLE_TRY(hipMemcpyAsync(rp, g->row_ptr, ((size_t)n + 1) * 8, hipMemcpyHostToDevice, st), "upload graph");
    if (g->nnz) SAMPLE_TRY(hipMemcpyAsync(col, g->col, g->nnz * 4, hipMemcpyHostToDevice, st), "upload graph");
    SAMPLE_TRY(hipMemcpyAsync(dcolor, color.data(), (size_t)n * 4, hipMemcpyHostToDevice, st), "upload colours");
    SAMPLE_TRY(hipMemcpyAsync(draws, h_draws, (size_t)2 * t * k * 8, hipMemcpyHostToDevice, st), "upload draws");
    std::vector<u128> ones(n, 1);
    SAMPLE_TRY(hipMemcpyAsync(P + n, ones.data(), (size_t)n * 16, hipMemcpyHostToDevice, st), "upload counts");
    SAMPLE_TRY(hipMemsetAsync(ovf, 0, sizeof(int), st), "clear flag");
    SAMPLE_TRY(hipStreamSynchronize(st), "stream synchronize");
    const auto t1 = clock::now();
    const uint32_t grid = std::min<uint32_t>((n + 255) / 256, 8192);
    for (uint32_t j = 2; j <= k; ++j)
      path_count_kernel<<<grid, 256, 0, st>>>(rp, col, dcolor, n, P + (size_t)(j - 1) * n, P + (size_t)j * n, ovf);
    prefix_blocksum_kernel<<<nb, kSampleThreads, 0, st>>>(P + (size_t)k * n, n, bs, ovf);
    prefix_scan_kernel<<<1, 64, 0, st>>>(bs, nb, ovf);
    prefix_write_kernel<<<nb, kSampleThreads, 0, st>>>(P + (size_t)k * n, n, bs, pre);
    SAMPLE_TRY(hipGetLastError(), "path count launch");
    u128 total = 0;
    int overflow = 0;
    SAMPLE_TRY(hipMemcpyAsync(&total, pre + (n - 1), 16, hipMemcpyDeviceToHost, st), "read total");
    SAMPLE_TRY(hipMemcpyAsync(&overflow, ovf, sizeof(int), hipMemcpyDeviceToHost, st), "read flag");
    SAMPLE_TRY(hipStreamSynchronize(st), "stream synchronize");
    // a path count, a block sum or the running total of the block sums wrapped
    if (overflow) return kdss::fail(KDSS_EOVERFLOW, "2^128 or more colour-increasing paths");
    inf.paths.lo = (uint64_t)total;
    inf.paths.hi = (uint64_t)(total >> 64);
    if (total > 0) {
      const uint32_t sgrid = (uint32_t)std::min<uint64_t>((t + 255) / 256, 8192);
      sample_walk_kernel<<<sgrid, 256, 0, st>>>(rp, col, dcolor, n, k, P, pre, total, draws, t, dout, dvalid);
      SAMPLE_TRY(hipGetLastError(), "sample launch");
      SAMPLE_TRY(hipMemcpyAsync(cl.data(), dout, (size_t)t * k * 4, hipMemcpyDeviceToHost, st), "read samples");
      SAMPLE_TRY(hipMemcpyAsync(valid.data(), dvalid, t, hipMemcpyDeviceToHost, st), "read samples");
    }
    SAMPLE_TRY(hipStreamSynchronize(st), "stream synchronize");
    dev_s = std::chrono::duration<double>(clock::now() - t1).count();
  }
  // the distinct sampled cliques, in lexicographic order
  std::vector<uint64_t> idx;
  for (uint64_t i = 0; i < t; ++i)
    if (valid[i]) idx.push_back(i);
  inf.cliques = idx.size();
  auto less = [&](uint64_t a, uint64_t b) {
    return std::lexicographical_compare(cl.begin() + a * k, cl.begin() + a * k + k, cl.begin() + b * k,
                                        cl.begin() + b * k + k);
  };
  auto same = [&](uint64_t a, uint64_t b) { return std::equal(cl.begin() + a * k, cl.begin() + a * k + k, cl.begin() + b * k); };
  std::sort(idx.begin(), idx.end(), less);
  idx.erase(std::unique(idx.begin(), idx.end(), same), idx.end());
  inf.distinct = idx.size();
  kdss_sct* s = new (std::nothrow) kdss_sct();
  if (!s) return kdss::fail(KDSS_ENOMEM, "cannot allocate the tree handle");
  kdss::Sct& T = s->s;
  T.n = n;
  T.k = k;
  T.members.resize(idx.size() * k);
  T.off.resize(idx.size() + 1);
  T.h.assign(idx.size(), (uint8_t)k);
  T.p.assign(idx.size(), 0u);
  for (size_t q = 0; q < idx.size(); ++q) {
    std::copy(cl.begin() + idx[q] * k, cl.begin() + idx[q] * k + k, T.members.begin() + q * k);
    T.off[q] = (uint64_t)q * k;
  }
  T.off[idx.size()] = (uint64_t)idx.size() * k;
  T.c_k = idx.size();
  T.s_max = idx.empty() ? 0 : k;
  const double total_s = std::chrono::duration<double>(clock::now() - t0).count();
  T.build_seconds = total_s;
  inf.device_seconds = dev_s;
  inf.host_seconds = total_s - dev_s;
  if (info) *info = inf;
  *out = s;
  return KDSS_OK;
}
