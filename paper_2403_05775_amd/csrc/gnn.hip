// Warm-start model for the Frank-Wolfe loads: a small message-passing network
// whose kernels run on gfx950 with BF16 operands and FP32 accumulation on the
// matrix cores (v_mfma_f32_32x32x16_bf16).  The model only chooses the integer
// start loads r0; the method's arithmetic is unchanged (a warm start is just
// Algorithm 2's "initialize r(u)").
//
// Layout conventions: activations are row-major BF16 (n rows); weights of a
// layer with K inputs are kept as W[K][64] (gradient layout) and Wt[64][K]
// (forward layout).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/kdss_gnn.h"
#include "kdss_internal.h"

using namespace kdss;

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One 32x32 BF16 product step over 16 k on gfx950's matrix cores (FP32 accumulate).
__device__ __forceinline__ f32x16 mfma16(s16x8 a, s16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// IEEE binary32 -> bfloat16, round to nearest, ties to even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x0040u);
  const uint32_t rounding = 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)((u + rounding) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

int hip_fail(hipError_t e, const char* what) { return fail(KDSS_EHIP, std::string(what) + ": " + hipGetErrorString(e)); }
#define HIP_TRY(call, what)                            \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, what);   \
  } while (0)

constexpr uint32_t kFeatureCols = 8;

uint32_t blocks_for(size_t n, uint32_t per, uint32_t cap = 65535) {
  size_t b = (n + per - 1) / per;
  return (uint32_t)std::max<size_t>(1, std::min<size_t>(b, cap));
}

// ---------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------

// The DAG that orients each edge from the earlier to the later node of the
// degeneracy order (out-degree <= degeneracy) is built on the device in three
// steps: out-degree per node, a scan into row offsets, and a fill that keeps
// each row's ascending id order.  One wavefront per node in the first and the
// last step.
__global__ __launch_bounds__(256) void orient_count_kernel(uint32_t n, uint64_t nnz,
                                                           const uint64_t* __restrict__ row_ptr,
                                                           const uint32_t* __restrict__ col,
                                                           const uint32_t* __restrict__ rank,
                                                           uint64_t* __restrict__ out_deg) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint32_t nw = gridDim.x * 4u;
  for (uint32_t u = wave; u < n; u += nw) {
    const uint32_t ru = rank[u];
    uint32_t c = 0;
    const uint64_t e_end = min(row_ptr[u + 1], nnz);
    for (uint64_t e = row_ptr[u] + lane; e < e_end; e += 64) {
      const uint32_t v = col[e];
      c += (v < n && rank[v] > ru) ? 1u : 0u;
    }
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
    if (lane == 0) out_deg[u] = c;
  }
}

constexpr uint32_t kScanItems = 8, kScanChunk = 256 * kScanItems;

// Inclusive scan of a[0..count) in chunks of 2048 (one workgroup each); the
// chunk totals go to part[].
__global__ __launch_bounds__(256) void scan_chunks_kernel(uint64_t* __restrict__ a, uint32_t count,
                                                          uint64_t* __restrict__ part) {
  __shared__ uint64_t wsum[4];
  const uint32_t base = blockIdx.x * kScanChunk + threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t run = 0;
#pragma unroll
  for (uint32_t i = 0; i < kScanItems; ++i) {
    v[i] = base + i < count ? a[base + i] : 0;
    run += v[i];
    v[i] = run;
  }
  // exclusive prefix of the thread totals across the workgroup
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  uint64_t x = run;
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint64_t off = x - run;
  for (uint32_t j = 0; j < w; ++j) off += wsum[j];
#pragma unroll
  for (uint32_t i = 0; i < kScanItems; ++i)
    if (base + i < count) a[base + i] = v[i] + off;
  if (threadIdx.x == 255) part[blockIdx.x] = off + run;
}

// Exclusive scan of the chunk totals (one workgroup, any count), then the
// offsets are added to every chunk.
__global__ __launch_bounds__(256) void scan_parts_kernel(uint64_t* __restrict__ part, uint32_t count) {
  __shared__ uint64_t wsum[4];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  for (uint32_t b = 0; b < count; b += 256) {
    const uint32_t i = b + threadIdx.x;
    const uint64_t own = i < count ? part[i] : 0;
    uint64_t x = own;
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(x, d);
      if (lane >= (uint32_t)d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint64_t off = carry + x - own;
    for (uint32_t j = 0; j < w; ++j) off += wsum[j];
    const uint64_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    if (i < count) part[i] = off;
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void scan_add_kernel(uint64_t* __restrict__ a, uint32_t count,
                                                       const uint64_t* __restrict__ part) {
  const uint32_t i = blockIdx.x * kScanChunk + threadIdx.x;
  const uint64_t off = part[blockIdx.x];
#pragma unroll
  for (uint32_t j = 0; j < kScanItems; ++j)
    if (i + j * 256u < count) a[i + j * 256u] += off;
}

__global__ __launch_bounds__(256) void orient_fill_kernel(uint32_t n, uint64_t nnz,
                                                          const uint64_t* __restrict__ row_ptr,
                                                          const uint32_t* __restrict__ col,
                                                          const uint32_t* __restrict__ rank,
                                                          const uint64_t* __restrict__ orp,
                                                          uint32_t* __restrict__ ocol) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint32_t nw = gridDim.x * 4u;
  const uint64_t below = (1ull << lane) - 1ull;
  for (uint32_t u = wave; u < n; u += nw) {
    const uint32_t ru = rank[u];
    uint64_t pos = orp[u];
    const uint64_t e_end = min(row_ptr[u + 1], nnz);
    for (uint64_t e0 = row_ptr[u]; e0 < e_end; e0 += 64) {
      const uint64_t e = e0 + lane;
      uint32_t v = 0;
      bool keep = false;
      if (e < e_end) {
        v = col[e];
        keep = v < n && rank[v] > ru;
      }
      const uint64_t m = __ballot(keep);
      if (keep) ocol[pos + (uint64_t)__popcll(m & below)] = v;
      pos += (uint64_t)__popcll(m);
    }
  }
}

// Triangles through every node on that DAG: a wavefront per node u; for every
// out-neighbour v of u and every out-neighbour w of v, w in N+(u) closes the
// triangle {u, v, w}, found once.  N+(u) goes into an open-addressing hash set
// in the wavefront's LDS slice (at most half full), so a membership test is
// one or two LDS reads; rows too long for the slice are binary-searched in
// global memory.  Four v are walked at a time, one 16-lane group each.
constexpr uint32_t kTriSlots = 2048;          // hash slots per wavefront
constexpr uint32_t kTriMaxStaged = kTriSlots / 2;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kGroupLanes = 16;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t tri_hash(uint32_t x, uint32_t bits) { return (x * 0x9E3779B1u) >> (32u - bits); }

__global__ __launch_bounds__(256) void triangle_kernel(uint32_t n, const uint64_t* __restrict__ orp,
                                                       const uint32_t* __restrict__ ocol,
                                                       uint32_t* __restrict__ tri) {
  __shared__ uint32_t sH[4][kTriSlots];
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t g = lane / kGroupLanes, q = lane % kGroupLanes;
  const uint32_t wave = blockIdx.x * 4u + wv;
  const uint32_t nw = gridDim.x * 4u;
  uint32_t* table = sH[wv];
  for (uint32_t u = wave; u < n; u += nw) {
    const uint64_t ub = orp[u], ue = orp[u + 1];
    const uint32_t d = (uint32_t)(ue - ub);
    if (d < 2) continue;
    const uint32_t* nu = ocol + ub;
    const bool staged = d <= kTriMaxStaged;
    uint32_t bits = 7;                         // table of 2^bits >= 2 d slots
    while ((1u << bits) < 2u * d && bits < 11) ++bits;
    const uint32_t mask = (1u << bits) - 1u;
    if (staged) {
      wave_lds_sync();   // earlier reads of the slice are done
      for (uint32_t i = lane; i <= mask; i += 64) table[i] = kEmpty;
      wave_lds_sync();
      for (uint32_t i = lane; i < d; i += 64) {
        const uint32_t key = nu[i];
        uint32_t h = tri_hash(key, bits);
        while (atomicCAS(&table[h], kEmpty, key) != kEmpty) h = (h + 1u) & mask;
      }
      wave_lds_sync();
    }
    uint32_t found_u = 0;
    for (uint32_t a0 = 0; a0 < d; a0 += 64) {
      // 64 out-neighbours v at a time, their row bounds loaded in parallel
      const uint32_t cnt = min(64u, d - a0);
      uint32_t my_v = 0;
      uint64_t my_b = 0, my_e = 0;
      if (lane < cnt) {
        my_v = nu[a0 + lane];
        my_b = orp[my_v];
        my_e = orp[my_v + 1];
      }
      for (uint32_t j0 = 0; j0 < cnt; j0 += 4) {
        const uint32_t j = j0 + g;
        const uint32_t v = __shfl(my_v, (int)(j & 63u));
        const uint64_t vb = __shfl(my_b, (int)(j & 63u)), ve = __shfl(my_e, (int)(j & 63u));
        uint32_t found = 0;
        if (j < cnt) {
          for (uint64_t x = vb + q; x < ve; x += kGroupLanes) {
            const uint32_t w = ocol[x];
            bool hit = false;
            if (staged) {
              uint32_t h = tri_hash(w, bits);
              for (;;) {
                const uint32_t y = table[h];
                if (y == w) { hit = true; break; }
                if (y == kEmpty) break;
                h = (h + 1u) & mask;
              }
            } else {
              uint32_t lo = 0, hi = d;
              while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (nu[mid] < w) lo = mid + 1; else hi = mid;
              }
              hit = lo < d && nu[lo] == w;
            }
            if (hit) {
              ++found;
              atomicAdd(tri + w, 1u);
            }
          }
        }
        for (uint32_t s2 = kGroupLanes / 2; s2 >= 1; s2 >>= 1) found += __shfl_xor(found, (int)s2);
        if (j < cnt && q == 0 && found) atomicAdd(tri + v, found);
        found_u += q == 0 ? found : 0u;
      }
    }
    for (int s2 = 32; s2 >= 1; s2 >>= 1) found_u += __shfl_xor(found_u, s2);
    if (lane == 0 && found_u) atomicAdd(tri + u, found_u);
  }
}

// x0[u] = [log1p(degree), log1p(core), log1p(triangles), 0, 0, 0, 0, 0] (8 columns, BF16)
__global__ __launch_bounds__(256) void features_kernel(uint32_t n, const uint64_t* __restrict__ row_ptr,
                                                       const uint32_t* __restrict__ core,
                                                       const uint32_t* __restrict__ tri, uint16_t* __restrict__ x0) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)n * kFeatureCols;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t u = i / kFeatureCols;
    const uint32_t c = (uint32_t)(i % kFeatureCols);
    float v = 0.f;
    if (c == 0) v = log1pf((float)(row_ptr[u + 1] - row_ptr[u]));
    else if (c == 1) v = log1pf((float)core[u]);
    else if (c == 2) v = log1pf((float)tri[u]);
    x0[i] = f2bf(v);
  }
}

// ---------------------------------------------------------------------------
// Mean aggregation over neighbours and its transpose
// ---------------------------------------------------------------------------

// One wavefront per node.  A row of F BF16 values is read in 16-byte pieces
// (eight values) by a group of F / 8 lanes; the G = 512 / F groups of a
// wavefront take every G-th neighbour, U = min(4, 64 / G) pieces in flight per
// lane, and are summed across groups at the end.  Neighbour ids (and, for the
// transpose, 1 / deg) are loaded 64 at a time, one per lane, and broadcast
// with shuffles.  Rows and row strides are multiples of 16 bytes.
__device__ __forceinline__ void add8(float (&s)[8], const uint4& w, float sc) {
  const uint32_t x[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    s[2 * i] += bf2f((uint16_t)(x[i] & 0xFFFFu)) * sc;
    s[2 * i + 1] += bf2f((uint16_t)(x[i] >> 16)) * sc;
  }
}

template <uint32_t F, bool kTranspose>
__device__ __forceinline__ void aggregate_row(uint32_t u, uint32_t lane, const uint64_t* __restrict__ row_ptr,
                                              const uint32_t* __restrict__ col, const uint4* __restrict__ src,
                                              uint32_t ld_vec, float (&s)[8]) {
  constexpr uint32_t LPR = F / 8, G = 64 / LPR;
  constexpr uint32_t U = G >= 16 ? 64 / G : 4;   // pieces in flight per lane
  const uint32_t g = lane / LPR, q = lane % LPR;
  const uint64_t b = row_ptr[u], e = row_ptr[u + 1];
  for (uint64_t c0 = b; c0 < e; c0 += 64) {
    const uint32_t cnt = (uint32_t)min<uint64_t>(64, e - c0);
    uint32_t my = 0;
    float myw = 1.f;
    if (lane < cnt) {
      my = col[c0 + lane];
      if (kTranspose) myw = 1.f / (float)(row_ptr[my + 1] - row_ptr[my]);
    }
    for (uint32_t j0 = 0; j0 < cnt; j0 += U * G) {
      uint4 w[U];
      float sc[U];
#pragma unroll
      for (uint32_t t = 0; t < U; ++t) {
        const uint32_t j = j0 + t * G + g;
        const uint32_t v = __shfl(my, (int)(j & 63u));
        sc[t] = kTranspose ? __shfl(myw, (int)(j & 63u)) : 1.f;
        w[t] = j < cnt ? src[(size_t)v * ld_vec + q] : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (uint32_t t = 0; t < U; ++t) add8(s, w[t], sc[t]);
    }
  }
#pragma unroll
  for (uint32_t d = LPR; d < 64; d <<= 1)
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] += __shfl_xor(s[i], (int)d);
}

__device__ __forceinline__ uint4 pack8(const float (&s)[8], float scale) {
  uint32_t x[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    x[i] = (uint32_t)f2bf(s[2 * i] * scale) | ((uint32_t)f2bf(s[2 * i + 1] * scale) << 16);
  return make_uint4(x[0], x[1], x[2], x[3]);
}

template <uint32_t F>
__global__ __launch_bounds__(256) void aggregate_kernel(uint32_t n, const uint64_t* __restrict__ row_ptr,
                                                        const uint32_t* __restrict__ col,
                                                        const uint4* __restrict__ h, uint4* __restrict__ out) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint32_t nw = gridDim.x * 4u;
  for (uint32_t u = wave; u < n; u += nw) {
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    aggregate_row<F, false>(u, lane, row_ptr, col, h, F / 8, s);
    const uint64_t deg = row_ptr[u + 1] - row_ptr[u];
    const float inv = deg ? 1.f / (float)deg : 0.f;
    if (lane < F / 8) out[(size_t)u * (F / 8) + lane] = pack8(s, inv);
  }
}

// out[v][f] = dself[v][f] + sum over u in N(v) of dagg[u][f] / deg(u)
// (the transpose of the mean aggregation; the graph is symmetric).
template <uint32_t F>
__global__ __launch_bounds__(256) void aggregate_backward_kernel(uint32_t n, const uint64_t* __restrict__ row_ptr,
                                                                 const uint32_t* __restrict__ col,
                                                                 const uint4* __restrict__ dagg,
                                                                 const uint4* __restrict__ dself,
                                                                 uint32_t ld_vec, uint4* __restrict__ out) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint32_t nw = gridDim.x * 4u;
  for (uint32_t v = wave; v < n; v += nw) {
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    aggregate_row<F, true>(v, lane, row_ptr, col, dagg, ld_vec, s);
    if (lane < F / 8) {
      add8(s, dself[(size_t)v * ld_vec + lane], 1.f);
      out[(size_t)v * (F / 8) + lane] = pack8(s, 1.f);
    }
  }
}

// ---------------------------------------------------------------------------
// Dense layers on the matrix cores
// ---------------------------------------------------------------------------

// Y[row][c] = act(sum_k X[row][k] * Bt[c][k] + bias[c]), c < 64, where
// X = [A1 (K1 columns, leading dim lda1) | A2 (K2 columns, lda2)], K = K1 + K2
// <= 128 a multiple of 16, K1 and K2 multiples of 8.  A workgroup computes 128
// rows; wavefront w computes rows 32 w .. 32 w + 31 as two 32x32 tiles, 16 k
// per instruction (v_mfma_f32_32x32x16_bf16).  Lane l holds
// A[l % 32][k0 + 8 (l / 32) .. + 7] and Bt[j0 + l % 32][k0 + 8 (l / 32) .. + 7]
// (one 16-byte load each; K1 is a multiple of 8, so a lane's eight k never
// straddle A1 and A2); accumulator v of lane l is row 8 (v / 4) + 4 (l / 32) +
// v % 4, column l % 32.
__global__ __launch_bounds__(256) void gemm_bt_kernel(uint32_t M, const uint16_t* __restrict__ A1, uint32_t K1,
                                                      uint32_t lda1, const uint16_t* __restrict__ A2, uint32_t K2,
                                                      uint32_t lda2, const uint16_t* __restrict__ Bt,
                                                      const float* __restrict__ bias, int relu,
                                                      uint16_t* __restrict__ Y, uint32_t ldy) {
  __shared__ __align__(16) uint16_t sB[64 * 128];
  const uint32_t K = K1 + K2;
  for (uint32_t i = threadIdx.x; i < 64u * K; i += blockDim.x) sB[i] = Bt[i];
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t li = lane & 31u, kq = (lane >> 5) * 8u;
  const uint32_t row = blockIdx.x * 128u + w * 32u + li;
  const bool rv = row < M;
  f32x16 acc0 = {}, acc1 = {};
  for (uint32_t k0 = 0; k0 < K; k0 += 16) {
    const uint32_t kk = k0 + kq;
    s16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
    if (rv) {
      const uint16_t* src = kk < K1 ? A1 + (size_t)row * lda1 + kk : A2 + (size_t)row * lda2 + (kk - K1);
      a = *reinterpret_cast<const s16x8*>(src);
    }
    const s16x8 b0 = *reinterpret_cast<const s16x8*>(&sB[li * K + kk]);
    const s16x8 b1 = *reinterpret_cast<const s16x8*>(&sB[(32u + li) * K + kk]);
    acc0 = mfma16(a, b0, acc0);
    acc1 = mfma16(a, b1, acc1);
  }
  const uint32_t rbase = blockIdx.x * 128u + w * 32u;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const uint32_t r = rbase + 8u * (v / 4) + (lane >> 5) * 4u + (v % 4);
    if (r >= M) continue;
    float y0 = acc0[v] + (bias ? bias[li] : 0.f);
    float y1 = acc1[v] + (bias ? bias[32u + li] : 0.f);
    if (relu) {
      y0 = fmaxf(y0, 0.f);
      y1 = fmaxf(y1, 0.f);
    }
    Y[(size_t)r * ldy + li] = f2bf(y0);
    Y[(size_t)r * ldy + 32u + li] = f2bf(y1);
  }
}

// dW[k][c] += sum_rows X[row][k] * dY[row][c];  db[c] += sum_rows dY[row][c].
// Each workgroup takes a band of rows in chunks of 32 staged in LDS; the four
// wavefronts own the K/32 x 2 output tiles; reduction over rows, 16 per MFMA:
// A[i][r] = X[r][i0 + i], B[r][j] = dY[r][j0 + j]; lane l supplies rows
// r = kk + 8 (l / 32) .. + 7 of column i0 + l % 32 (and of dY column j0 + l % 32).
__global__ __launch_bounds__(256) void gemm_wgrad_kernel(uint32_t M, const uint16_t* __restrict__ A1, uint32_t K1,
                                                         uint32_t lda1, const uint16_t* __restrict__ A2, uint32_t K2,
                                                         uint32_t lda2, const uint16_t* __restrict__ dY,
                                                         float* __restrict__ dW, float* __restrict__ db) {
  __shared__ __align__(16) uint16_t sX[32 * 128];
  __shared__ __align__(16) uint16_t sD[32 * 64];
  const uint32_t K = K1 + K2;
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t li = lane & 31u, rq = (lane >> 5) * 8u, vq = (lane >> 5) * 4u;
  const uint32_t ntile = ((K + 31u) / 32u) * 2u;   // 32-row tiles, the last one zero-padded
  f32x16 acc[2] = {{}, {}};
  float bsum = 0.f;
  const uint32_t band = (M + gridDim.x - 1) / gridDim.x;
  const uint32_t r_begin = blockIdx.x * band, r_end = min(M, r_begin + band);
  for (uint32_t r0 = r_begin; r0 < r_end; r0 += 32) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < 32u * K; i += blockDim.x) {
      const uint32_t r = r0 + i / K, k = i % K;
      uint16_t x = 0;
      if (r < r_end) x = k < K1 ? A1[(size_t)r * lda1 + k] : A2[(size_t)r * lda2 + (k - K1)];
      sX[i] = x;
    }
    for (uint32_t i = threadIdx.x; i < 32u * 64u; i += blockDim.x) {
      const uint32_t r = r0 + i / 64u;
      sD[i] = r < r_end ? dY[(size_t)r * 64u + (i % 64u)] : (uint16_t)0;
    }
    __syncthreads();
    if (threadIdx.x < 64)
      for (uint32_t r = 0; r < 32; ++r) bsum += bf2f(sD[r * 64u + threadIdx.x]);
#pragma unroll
    for (uint32_t t = 0; t < 2; ++t) {
      const uint32_t tile = w * 2u + t;
      if (tile >= ntile) continue;
      const uint32_t i0 = (tile >> 1) * 32u, j0 = (tile & 1u) * 32u;
      for (uint32_t kk = 0; kk < 32; kk += 16) {
        s16x8 a, b;
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) {
          a[q] = i0 + li < K ? (short)sX[(kk + rq + q) * K + i0 + li] : (short)0;
          b[q] = (short)sD[(kk + rq + q) * 64u + j0 + li];
        }
        acc[t] = mfma16(a, b, acc[t]);
      }
    }
  }
#pragma unroll
  for (uint32_t t = 0; t < 2; ++t) {
    const uint32_t tile = w * 2u + t;
    if (tile >= ntile) continue;
    const uint32_t i0 = (tile >> 1) * 32u, j0 = (tile & 1u) * 32u;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const uint32_t i = i0 + 8u * (v / 4) + vq + (v % 4);
      if (i < K) atomicAdd(dW + (size_t)i * 64u + j0 + li, acc[t][v]);
    }
  }
  if (db && threadIdx.x < 64) atomicAdd(db + threadIdx.x, bsum);
}

// dY *= (Y > 0)
__global__ __launch_bounds__(256) void relu_backward_kernel(size_t count, const uint16_t* __restrict__ y,
                                                            uint16_t* __restrict__ dy) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    if (!(bf2f(y[i]) > 0.f)) dy[i] = 0;
}

// ---------------------------------------------------------------------------
// Head, loss, optimiser, warm start
// ---------------------------------------------------------------------------

// pred[u] = sum_c h[u][c] w[c] + b
__global__ __launch_bounds__(256) void head_kernel(uint32_t n, const uint16_t* __restrict__ h,
                                                   const float* __restrict__ w, const float* __restrict__ b,
                                                   float* __restrict__ pred) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    float s = b[0];
    for (uint32_t c = 0; c < 64; ++c) s += bf2f(h[(size_t)u * 64u + c]) * w[c];
    pred[u] = s;
  }
}

// MSE over n nodes: loss += sum (pred - y)^2 / n; dh = dpred * w (BF16);
// dw[c] += sum dpred h[u][c]; dw[64] += sum dpred (the bias), dpred = 2 (pred - y) / n.
__global__ __launch_bounds__(256) void head_backward_kernel(uint32_t n, const uint16_t* __restrict__ h,
                                                            const float* __restrict__ w,
                                                            const float* __restrict__ pred,
                                                            const float* __restrict__ target,
                                                            uint16_t* __restrict__ dh, float* __restrict__ dw,
                                                            float* __restrict__ loss) {
  __shared__ float sw[65 * 4];
  float gw[65];
  for (int c = 0; c < 65; ++c) gw[c] = 0.f;
  float l = 0.f;
  const float inv_n = 1.f / (float)n;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    const float e = pred[u] - target[u];
    l += e * e * inv_n;
    const float d = 2.f * e * inv_n;
    for (uint32_t c = 0; c < 64; ++c) {
      gw[c] += d * bf2f(h[(size_t)u * 64u + c]);
      dh[(size_t)u * 64u + c] = f2bf(d * w[c]);
    }
    gw[64] += d;
  }
  // reduce over the wavefront, then over the four wavefronts
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  for (int c = 0; c < 66; ++c) {
    float x = c < 65 ? gw[c] : l;
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
    if (lane == 0) {
      if (c < 65) sw[c * 4 + wv] = x;
      else l = x;
    }
  }
  __syncthreads();
  if (threadIdx.x < 65) atomicAdd(dw + threadIdx.x, sw[threadIdx.x * 4] + sw[threadIdx.x * 4 + 1] +
                                                         sw[threadIdx.x * 4 + 2] + sw[threadIdx.x * 4 + 3]);
  if (lane == 0) atomicAdd(loss, l);
}

// Adam on FP32 master parameters (bias-corrected moments).
__global__ __launch_bounds__(256) void adam_kernel(uint32_t count, float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                   float b2, float eps, float c1, float c2) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// BF16 copies of a K x 64 FP32 weight: W[k][c] and its transpose Wt[c][k].
__global__ __launch_bounds__(256) void pack_weights_kernel(uint32_t K, const float* __restrict__ w32,
                                                           uint16_t* __restrict__ w, uint16_t* __restrict__ wt) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < K * 64u; i += gridDim.x * blockDim.x) {
    const uint32_t k = i / 64u, c = i % 64u;
    const uint16_t b = f2bf(w32[i]);
    if (w) w[i] = b;
    if (wt) wt[(size_t)c * K + k] = b;
  }
}

// r0[u] = round(t0 * expm1(pred[u])) clamped to [0, cap]; max into *rmax.
__global__ __launch_bounds__(256) void warm_start_kernel(uint32_t n, const float* __restrict__ pred, double t0,
                                                         uint64_t cap, uint64_t* __restrict__ r0,
                                                         unsigned long long* __restrict__ rmax) {
  unsigned long long mx = 0;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    double x = t0 * expm1((double)pred[u]);
    if (!(x > 0.0)) x = 0.0;
    uint64_t r = x >= (double)cap ? cap : (uint64_t)llrint(x);
    r0[u] = r;
    mx = r > mx ? r : mx;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    const unsigned long long o = __shfl_xor(mx, d);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & 63u) == 0 && mx) atomicMax(rmax, mx);
}

// Training target y[u] = log1p(r[u] / T) from a cold run's 64-bit loads.
__global__ __launch_bounds__(256) void label_kernel(uint32_t n, const uint64_t* __restrict__ r, double T,
                                                    float* __restrict__ y) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x)
    y[u] = (float)log1p((double)r[u] / T);
}

__global__ __launch_bounds__(256) void zero_f32_kernel(float* __restrict__ a, uint32_t count) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) a[i] = 0.f;
}

}  // namespace

extern "C" {

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

int kdss_gnn_features_workspace(uint32_t n, uint64_t nnz, size_t* bytes) {
  if (!bytes) return fail(KDSS_EINVAL, "null argument");
  const size_t parts = ((size_t)n + kScanChunk - 1) / kScanChunk;
  *bytes = 3 * al256((size_t)n * 4) + al256(((size_t)n + 1) * 8) + al256(std::max<size_t>(1, parts) * 8) +
           al256(std::max<uint64_t>(1, nnz) * 4);
  return KDSS_OK;
}

int kdss_gnn_features(const kdss_sct* s, const uint64_t* d_row_ptr, const uint32_t* d_col, uint64_t nnz,
                      int feature_set, uint16_t* d_x0, void* d_ws, size_t ws_bytes, void* stream) {
  if (!s || !d_row_ptr || !d_x0 || !d_ws || (nnz && !d_col)) return fail(KDSS_EINVAL, "null argument");
  if (feature_set != 0 && feature_set != 1) return fail(KDSS_EINVAL, "feature_set must be 0 or 1");
  const uint32_t n = s->s.n;
  size_t need = 0;
  kdss_gnn_features_workspace(n, nnz, &need);
  if (ws_bytes < need) return fail(KDSS_EWORKSPACE, "features workspace too small");
  if (n == 0) return KDSS_OK;
  const Degeneracy& dg = s->s.deg;
  const uint32_t parts = (uint32_t)(((size_t)n + kScanChunk - 1) / kScanChunk);
  char* p = static_cast<char*>(d_ws);
  uint32_t* d_rank = reinterpret_cast<uint32_t*>(p);
  uint32_t* d_core = reinterpret_cast<uint32_t*>(p + al256((size_t)n * 4));
  uint32_t* d_tri = reinterpret_cast<uint32_t*>(p + 2 * al256((size_t)n * 4));
  uint64_t* d_orp = reinterpret_cast<uint64_t*>(p + 3 * al256((size_t)n * 4));
  uint64_t* d_part = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(d_orp) + al256(((size_t)n + 1) * 8));
  uint32_t* d_ocol = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(d_part) + al256((size_t)parts * 8));
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the tree's host arrays outlive the copies
  HIP_TRY(hipMemcpyAsync(d_rank, dg.rank.data(), (size_t)n * 4, hipMemcpyHostToDevice, st), "upload order");
  HIP_TRY(hipMemcpyAsync(d_core, dg.core.data(), (size_t)n * 4, hipMemcpyHostToDevice, st), "upload cores");
  HIP_TRY(hipMemsetAsync(d_tri, 0, (size_t)n * 4, st), "clear triangles");
  HIP_TRY(hipMemsetAsync(d_orp, 0, 8, st), "clear offsets");
  const uint32_t wave_grid = blocks_for(n, 4, 16384);
  if (feature_set == 0) {   // triangles through every node (feature set 1 leaves the column 0)
    orient_count_kernel<<<wave_grid, 256, 0, st>>>(n, nnz, d_row_ptr, d_col, d_rank, d_orp + 1);
    scan_chunks_kernel<<<parts, 256, 0, st>>>(d_orp + 1, n, d_part);
    scan_parts_kernel<<<1, 256, 0, st>>>(d_part, parts);
    scan_add_kernel<<<parts, 256, 0, st>>>(d_orp + 1, n, d_part);
    orient_fill_kernel<<<wave_grid, 256, 0, st>>>(n, nnz, d_row_ptr, d_col, d_rank, d_orp, d_ocol);
    triangle_kernel<<<wave_grid, 256, 0, st>>>(n, d_orp, d_ocol, d_tri);
  }
  features_kernel<<<blocks_for((size_t)n * kFeatureCols, 256, 16384), 256, 0, st>>>(n, d_row_ptr, d_core, d_tri, d_x0);
  HIP_TRY(hipGetLastError(), "features launch");
  return KDSS_OK;
}

int kdss_gnn_aggregate(uint32_t n, const uint64_t* d_row_ptr, const uint32_t* d_col, const uint16_t* d_h,
                       uint32_t F, uint16_t* d_out, void* stream) {
  if (!d_row_ptr || (!d_col && n) || !d_h || !d_out) return fail(KDSS_EINVAL, "null argument");
  if (F != 8 && F != 16 && F != 32 && F != 64) return fail(KDSS_EINVAL, "F must be 8, 16, 32 or 64");
  if (n == 0) return KDSS_OK;
  if ((reinterpret_cast<uintptr_t>(d_h) | reinterpret_cast<uintptr_t>(d_out)) & 15u)
    return fail(KDSS_EINVAL, "h and out must be 16-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint4* h = reinterpret_cast<const uint4*>(d_h);
  uint4* out = reinterpret_cast<uint4*>(d_out);
  const uint32_t grid = blocks_for(n, 4, 16384);
  switch (F) {
    case 8: aggregate_kernel<8><<<grid, 256, 0, st>>>(n, d_row_ptr, d_col, h, out); break;
    case 16: aggregate_kernel<16><<<grid, 256, 0, st>>>(n, d_row_ptr, d_col, h, out); break;
    case 32: aggregate_kernel<32><<<grid, 256, 0, st>>>(n, d_row_ptr, d_col, h, out); break;
    default: aggregate_kernel<64><<<grid, 256, 0, st>>>(n, d_row_ptr, d_col, h, out); break;
  }
  HIP_TRY(hipGetLastError(), "aggregate launch");
  return KDSS_OK;
}

int kdss_gnn_aggregate_backward(uint32_t n, const uint64_t* d_row_ptr, const uint32_t* d_col, const uint16_t* d_dagg,
                                const uint16_t* d_dself, uint32_t F, uint32_t ld, uint16_t* d_out, void* stream) {
  if (!d_row_ptr || (!d_col && n) || !d_dagg || !d_dself || !d_out) return fail(KDSS_EINVAL, "null argument");
  if ((F != 8 && F != 16 && F != 32 && F != 64) || ld < F || ld % 8)
    return fail(KDSS_EINVAL, "F must be 8, 16, 32 or 64; ld >= F and a multiple of 8");
  if ((reinterpret_cast<uintptr_t>(d_dagg) | reinterpret_cast<uintptr_t>(d_dself) |
       reinterpret_cast<uintptr_t>(d_out)) & 15u)
    return fail(KDSS_EINVAL, "dagg, dself and out must be 16-byte aligned");
  if (n == 0) return KDSS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint4* da = reinterpret_cast<const uint4*>(d_dagg);
  const uint4* ds = reinterpret_cast<const uint4*>(d_dself);
  uint4* out = reinterpret_cast<uint4*>(d_out);
  const uint32_t grid = blocks_for(n, 4, 16384);
  switch (F) {
    case 8: aggregate_backward_kernel<8><<<grid, 256, 0, st>>>(n, d_row_ptr, d_col, da, ds, ld / 8, out); break;
    case 16: aggregate_backward_kernel<16><<<grid, 256, 0, st>>>(n, d_row_ptr, d_col, da, ds, ld / 8, out); break;
    case 32: aggregate_backward_kernel<32><<<grid, 256, 0, st>>>(n, d_row_ptr, d_col, da, ds, ld / 8, out); break;
    default: aggregate_backward_kernel<64><<<grid, 256, 0, st>>>(n, d_row_ptr, d_col, da, ds, ld / 8, out); break;
  }
  HIP_TRY(hipGetLastError(), "aggregate backward launch");
  return KDSS_OK;
}

int kdss_gnn_linear(uint32_t M, const uint16_t* d_a1, uint32_t K1, uint32_t lda1, const uint16_t* d_a2, uint32_t K2,
                    uint32_t lda2, const uint16_t* d_bt, const float* d_bias, int relu, uint16_t* d_y, uint32_t ldy,
                    void* stream) {
  if (!d_a1 || !d_bt || !d_y || (K2 && !d_a2)) return fail(KDSS_EINVAL, "null argument");
  auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
  if (K1 % 8 || K2 % 8 || (K1 + K2) % 16 || K1 + K2 == 0 || K1 + K2 > 128 || lda1 < K1 || (K2 && lda2 < K2) ||
      ldy < 64 || lda1 % 8 || (K2 && lda2 % 8) || !a16(d_a1) || (K2 && !a16(d_a2)) || !a16(d_bt))
    return fail(KDSS_EINVAL, "K1, K2 multiples of 8 with K1 + K2 a multiple of 16, at most 128; leading dims >= "
                             "widths and multiples of 8; A1, A2 and Bt 16-byte aligned");
  gemm_bt_kernel<<<blocks_for(M, 128, 1u << 30), 256, 0, static_cast<hipStream_t>(stream)>>>(
      M, d_a1, K1, lda1, d_a2, K2, lda2, d_bt, d_bias, relu, d_y, ldy);
  HIP_TRY(hipGetLastError(), "linear launch");
  return KDSS_OK;
}

int kdss_gnn_linear_wgrad(uint32_t M, const uint16_t* d_a1, uint32_t K1, uint32_t lda1, const uint16_t* d_a2,
                          uint32_t K2, uint32_t lda2, const uint16_t* d_dy, float* d_dw, float* d_db, void* stream) {
  if (!d_a1 || !d_dy || !d_dw || (K2 && !d_a2)) return fail(KDSS_EINVAL, "null argument");
  const uint32_t K = K1 + K2;
  if (K == 0 || K > 128 || K % 16 || K1 % 8 || K2 % 8 || lda1 < K1 || (K2 && lda2 < K2))
    return fail(KDSS_EINVAL, "K1, K2 multiples of 8 with K1 + K2 a multiple of 16, at most 128");
  gemm_wgrad_kernel<<<blocks_for(M, 2048, 256), 256, 0, static_cast<hipStream_t>(stream)>>>(
      M, d_a1, K1, lda1, d_a2, K2, lda2, d_dy, d_dw, d_db);
  HIP_TRY(hipGetLastError(), "weight gradient launch");
  return KDSS_OK;
}

int kdss_gnn_relu_backward(uint64_t count, const uint16_t* d_y, uint16_t* d_dy, void* stream) {
  if (!d_y || !d_dy) return fail(KDSS_EINVAL, "null argument");
  relu_backward_kernel<<<blocks_for(count, 256, 16384), 256, 0, static_cast<hipStream_t>(stream)>>>(count, d_y, d_dy);
  HIP_TRY(hipGetLastError(), "relu backward launch");
  return KDSS_OK;
}

int kdss_gnn_head(uint32_t n, const uint16_t* d_h, const float* d_w, float* d_pred, void* stream) {
  if (!d_h || !d_w || !d_pred) return fail(KDSS_EINVAL, "null argument");
  head_kernel<<<blocks_for(n, 256, 16384), 256, 0, static_cast<hipStream_t>(stream)>>>(n, d_h, d_w, d_w + 64, d_pred);
  HIP_TRY(hipGetLastError(), "head launch");
  return KDSS_OK;
}

int kdss_gnn_head_backward(uint32_t n, const uint16_t* d_h, const float* d_w, const float* d_pred,
                           const float* d_target, uint16_t* d_dh, float* d_dw, float* d_loss, void* stream) {
  if (!d_h || !d_w || !d_pred || !d_target || !d_dh || !d_dw || !d_loss || n == 0)
    return fail(KDSS_EINVAL, "null argument or n == 0");
  head_backward_kernel<<<blocks_for(n, 256, 2048), 256, 0, static_cast<hipStream_t>(stream)>>>(
      n, d_h, d_w, d_pred, d_target, d_dh, d_dw, d_loss);
  HIP_TRY(hipGetLastError(), "head backward launch");
  return KDSS_OK;
}

int kdss_gnn_adam(uint32_t count, float* d_p, const float* d_g, float* d_m, float* d_v, float lr, float b1, float b2,
                  float eps, uint32_t step, void* stream) {
  if (!d_p || !d_g || !d_m || !d_v || step == 0) return fail(KDSS_EINVAL, "null argument or step == 0");
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  adam_kernel<<<blocks_for(count, 256, 4096), 256, 0, static_cast<hipStream_t>(stream)>>>(count, d_p, d_g, d_m, d_v, lr,
                                                                                          b1, b2, eps, c1, c2);
  HIP_TRY(hipGetLastError(), "adam launch");
  return KDSS_OK;
}

int kdss_gnn_pack_weights(uint32_t K, const float* d_w32, uint16_t* d_w, uint16_t* d_wt, void* stream) {
  if (!d_w32 || (!d_w && !d_wt)) return fail(KDSS_EINVAL, "null argument");
  pack_weights_kernel<<<blocks_for((size_t)K * 64, 256, 4096), 256, 0, static_cast<hipStream_t>(stream)>>>(
      K, d_w32, d_w, d_wt);
  HIP_TRY(hipGetLastError(), "pack weights launch");
  return KDSS_OK;
}

// ---- the whole model: parameters in one FP32 array, workspace from the caller ----
namespace {

constexpr uint32_t kHidden = 64, kF0 = 8;
constexpr uint32_t kLayerK[3] = {2 * kF0, 2 * kHidden, 2 * kHidden};
constexpr size_t kOffW[3] = {KDSS_GNN_W1, KDSS_GNN_W2, KDSS_GNN_W3};
constexpr size_t kOffB[3] = {KDSS_GNN_B1, KDSS_GNN_B2, KDSS_GNN_B3};

struct ModelWs {   // byte layout of kdss_gnn_model_workspace
  uint16_t *w16[3], *wt16[3];   // BF16 weights K x 64 and 64 x K
  uint16_t *agg[3], *y[3];      // per layer: neighbour mean (n x F) and output (n x 64)
  float* pred;                  // n
  float* target;                // n (training)
  uint16_t *dy, *dx, *dh;       // n x 64, n x 128, n x 64 (training)
  float* grad;                  // KDSS_GNN_PARAMS (training)
  size_t bytes;
};

ModelWs model_layout(char* base, uint32_t n, int train) {
  ModelWs m{};
  size_t o = 0;
  auto take = [&](size_t b) {
    char* p = base ? base + o : nullptr;
    o += al256(std::max<size_t>(b, 4));
    return p;
  };
  for (int l = 0; l < 3; ++l) {
    m.w16[l] = reinterpret_cast<uint16_t*>(take((size_t)kLayerK[l] * kHidden * 2));
    m.wt16[l] = reinterpret_cast<uint16_t*>(take((size_t)kLayerK[l] * kHidden * 2));
  }
  const uint32_t F[3] = {kF0, kHidden, kHidden};
  for (int l = 0; l < 3; ++l) {
    m.agg[l] = reinterpret_cast<uint16_t*>(take((size_t)n * F[l] * 2));
    m.y[l] = reinterpret_cast<uint16_t*>(take((size_t)n * kHidden * 2));
  }
  m.pred = reinterpret_cast<float*>(take((size_t)n * 4));
  if (train) {
    m.target = reinterpret_cast<float*>(take((size_t)n * 4));
    m.dy = reinterpret_cast<uint16_t*>(take((size_t)n * kHidden * 2));
    m.dx = reinterpret_cast<uint16_t*>(take((size_t)n * 2 * kHidden * 2));
    m.dh = reinterpret_cast<uint16_t*>(take((size_t)n * kHidden * 2));
    m.grad = reinterpret_cast<float*>(take((size_t)KDSS_GNN_PARAMS * 4));
  }
  m.bytes = o;
  return m;
}

// BF16 copies of the three weights, then the forward pass into m.pred.
int model_forward(const ModelWs& m, uint32_t n, const uint64_t* rp, const uint32_t* col, const uint16_t* x0,
                  const float* params, void* stream) {
  for (int l = 0; l < 3; ++l) {
    int rc = kdss_gnn_pack_weights(kLayerK[l], params + kOffW[l], m.w16[l], m.wt16[l], stream);
    if (rc) return rc;
  }
  const uint16_t* h = x0;
  uint32_t F = kF0;
  for (int l = 0; l < 3; ++l) {
    int rc = kdss_gnn_aggregate(n, rp, col, h, F, m.agg[l], stream);
    if (!rc) rc = kdss_gnn_linear(n, h, F, F, m.agg[l], F, F, m.wt16[l], params + kOffB[l], 1, m.y[l], kHidden, stream);
    if (rc) return rc;
    h = m.y[l];
    F = kHidden;
  }
  return kdss_gnn_head(n, m.y[2], params + KDSS_GNN_HEAD, m.pred, stream);
}

int check_model_args(uint32_t n, const uint64_t* rp, const uint32_t* col, const uint16_t* x0, const void* params,
                     void* d_ws, size_t ws_bytes, int train) {
  if (!rp || !x0 || !params || !d_ws || (n && !col)) return fail(KDSS_EINVAL, "null argument");
  if (n == 0) return fail(KDSS_EINVAL, "the graph has no nodes");
  if ((reinterpret_cast<uintptr_t>(x0) & 15u) || (reinterpret_cast<uintptr_t>(d_ws) & 255u))
    return fail(KDSS_EINVAL, "x0 must be 16-byte and the workspace 256-byte aligned");
  if (ws_bytes < model_layout(nullptr, n, train).bytes)
    return fail(KDSS_EWORKSPACE, "model workspace smaller than kdss_gnn_model_workspace() reports");
  return KDSS_OK;
}

}  // namespace

int kdss_gnn_model_workspace(uint32_t n, int train, size_t* bytes) {
  if (!bytes) return fail(KDSS_EINVAL, "null argument");
  *bytes = model_layout(nullptr, n, train ? 1 : 0).bytes;
  return KDSS_OK;
}

int kdss_gnn_infer(uint32_t n, const uint64_t* d_row_ptr, const uint32_t* d_col, const uint16_t* d_x0,
                   const float* d_params, double t0, uint64_t cap, void* d_ws, size_t ws_bytes, float* d_pred,
                   uint64_t* d_r0, uint64_t* d_rmax, void* stream) {
  int rc = check_model_args(n, d_row_ptr, d_col, d_x0, d_params, d_ws, ws_bytes, 0);
  if (rc) return rc;
  if (!d_r0 || !d_rmax) return fail(KDSS_EINVAL, "null argument");
  const ModelWs m = model_layout(static_cast<char*>(d_ws), n, 0);
  rc = model_forward(m, n, d_row_ptr, d_col, d_x0, d_params, stream);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (d_pred) HIP_TRY(hipMemcpyAsync(d_pred, m.pred, (size_t)n * 4, hipMemcpyDeviceToDevice, st), "copy prediction");
  return kdss_gnn_warm_start(n, m.pred, t0, cap, d_r0, d_rmax, stream);
}

int kdss_gnn_train_step(uint32_t n, const uint64_t* d_row_ptr, const uint32_t* d_col, const uint16_t* d_x0,
                        const uint64_t* d_r, uint32_t T, float* d_params, float* d_m, float* d_v, uint32_t step,
                        float lr, void* d_ws, size_t ws_bytes, float* d_loss, void* stream) {
  int rc = check_model_args(n, d_row_ptr, d_col, d_x0, d_params, d_ws, ws_bytes, 1);
  if (rc) return rc;
  if (!d_r || !d_m || !d_v || !d_loss) return fail(KDSS_EINVAL, "null argument");
  if (T == 0 || step == 0) return fail(KDSS_EINVAL, "T and step must be at least 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ModelWs m = model_layout(static_cast<char*>(d_ws), n, 1);
  label_kernel<<<blocks_for(n, 256, 4096), 256, 0, st>>>(n, d_r, (double)T, m.target);
  zero_f32_kernel<<<blocks_for(KDSS_GNN_PARAMS, 256, 64), 256, 0, st>>>(m.grad, KDSS_GNN_PARAMS);
  HIP_TRY(hipGetLastError(), "label launch");
  rc = model_forward(m, n, d_row_ptr, d_col, d_x0, d_params, stream);
  if (rc) return rc;
  // loss and the head's gradient, then each layer back to front
  rc = kdss_gnn_head_backward(n, m.y[2], d_params + KDSS_GNN_HEAD, m.pred, m.target, m.dy, m.grad + KDSS_GNN_HEAD,
                              d_loss, stream);
  if (rc) return rc;
  const uint32_t F[3] = {kF0, kHidden, kHidden};
  uint16_t *dy = m.dy, *next = m.dh;   // the gradient at a layer's output, and the buffer for its input's
  for (int l = 2; l >= 0; --l) {
    const uint16_t* h = l ? m.y[l - 1] : d_x0;
    rc = kdss_gnn_relu_backward((uint64_t)n * kHidden, m.y[l], dy, stream);
    if (!rc) rc = kdss_gnn_linear_wgrad(n, h, F[l], F[l], m.agg[l], F[l], F[l], dy, m.grad + kOffW[l],
                                        m.grad + kOffB[l], stream);
    if (rc) return rc;
    if (l == 0) break;
    // dX = dY W^T: the self half into columns 0..f-1, the neighbour half into f..2f-1;
    // the input's gradient is the self half plus the mean's transpose of the other
    const uint32_t f = F[l];
    rc = kdss_gnn_linear(n, dy, kHidden, kHidden, nullptr, 0, 0, m.w16[l], nullptr, 0, m.dx, 2 * f, stream);
    if (!rc) rc = kdss_gnn_linear(n, dy, kHidden, kHidden, nullptr, 0, 0, m.w16[l] + (size_t)f * kHidden, nullptr, 0,
                                  m.dx + f, 2 * f, stream);
    if (!rc) rc = kdss_gnn_aggregate_backward(n, d_row_ptr, d_col, m.dx + f, m.dx, f, 2 * f, next, stream);
    if (rc) return rc;
    std::swap(dy, next);
  }
  return kdss_gnn_adam(KDSS_GNN_PARAMS, d_params, m.grad, d_m, d_v, lr, 0.9f, 0.999f, 1e-8f, step, stream);
}

int kdss_gnn_warm_start(uint32_t n, const float* d_pred, double t0, uint64_t cap, uint64_t* d_r0, uint64_t* d_rmax,
                        void* stream) {
  if (!d_pred || !d_r0 || !d_rmax) return fail(KDSS_EINVAL, "null argument");
  if (!(t0 >= 0.0)) return fail(KDSS_EINVAL, "t0 must be non-negative");
  warm_start_kernel<<<blocks_for(n, 256, 4096), 256, 0, static_cast<hipStream_t>(stream)>>>(
      n, d_pred, t0, cap, d_r0, reinterpret_cast<unsigned long long*>(d_rmax));
  HIP_TRY(hipGetLastError(), "warm start launch");
  return KDSS_OK;
}

}  // extern "C"
