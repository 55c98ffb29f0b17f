/*
 * k-clique densest subgraph search -- CPU ORACLE (test infrastructure only).
 *
 * This file is the plain, slow, obviously correct definition of what the
 * GPU path computes.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; no product code links it or calls it.  It shares
 * no source with the GPU library: it never builds a clique tree and enumerates
 * every k-clique explicitly.
 *
 * What it computes (paper: Sec. 2 "Convex programming CP(G)" and Algorithm 1,
 * the Frank-Wolfe framework; Sec. 3.2 Algorithm 2 for the iteration/extraction
 * skeleton):
 *
 *   r_0 = r0 (zero by default)
 *   for t = 1..T (synchronous: every clique reads r_{t-1}):
 *       d_t(u) = #{ C in C_k(V) : u = argmin_{v in C} (r_{t-1}(v), v) }
 *       r_t    = r_{t-1} + d_t
 *   pi  = nodes sorted by r_T non-increasing, ties by ascending id
 *   K_i = |C_k(pi[0..i))|,  i* = the largest i maximising K_i / i
 *   result: loads r_T, density K_{i*}/i*, node set pi[0..i*),
 *           upper bound max_u (r_T(u) - r0(u)) / T.
 *
 * Readings of points the paper leaves open (argmin ties go to the lowest id
 * where Algorithm 1 says "break ties arbitrarily"; synchronous updates; sort
 * direction and the largest-prefix tie rule from Definition 1) are listed with
 * their reasons in the design notes.  Loads are kept as unsigned 128-bit
 * integers so nothing here can overflow for any graph it can enumerate.
 *
 * Pins: the test suite checks this oracle against the paper's printed example
 * (Example 1: 9 triangles on 7 nodes, density 9/7, densest set {u1..u6} at
 * 4/3; Example 2's clique tree determines the graph), closed forms on complete
 * and disjoint-union graphs, Lemma 6 (sum of loads equals t * |C_k|), the
 * bound density <= rho* <= upper bound from brute force over all subsets on
 * graphs of at most 14 nodes, and a brute-force Frank-Wolfe over all k-subsets.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

enum {
    KOR_OK = 0,
    KOR_EINVAL = -1,      /* bad argument (k < 2, T == 0 for solve, null pointer) */
    KOR_EGRAPH = -2,      /* CSR is not a simple undirected graph */
    KOR_ENOMEM = -7,
};

typedef struct {
    uint32_t n;
    const uint64_t *row_ptr;
    const uint32_t *col;
} graph_t;

typedef struct {
    uint64_t c_k_lo, c_k_hi;      /* |C_k(V)| */
    uint32_t T;                   /* iterations run */
    uint32_t size;                /* i* */
    uint64_t dens_num;            /* K_{i*} */
    uint64_t ub_num_lo, ub_num_hi;/* max (r_T - r0); denominator T */
    double enum_seconds;          /* listing all k-cliques once */
    double iter_seconds;          /* the T Frank-Wolfe iterations */
    double extract_seconds;       /* final extraction */
    int threads;                  /* OpenMP threads used */
    int streamed;                 /* 1 if cliques were re-listed each iteration */
} kor_result;

typedef struct {                  /* one row per iteration when a trace is asked for */
    uint32_t t, size;
    uint64_t dens_num;
    uint64_t ub_num_lo, ub_num_hi;
} kor_trace_row;

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ---- graph validation: simple, undirected, rows sorted (Sec. 2 problem statement) ---- */

static int has_edge(const graph_t *g, uint32_t u, uint32_t v) {
    uint64_t lo = g->row_ptr[u], hi = g->row_ptr[u + 1];
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (g->col[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < g->row_ptr[u + 1] && g->col[lo] == v;
}

int kor_validate(uint32_t n, uint64_t nnz, const uint64_t *row_ptr, const uint32_t *col) {
    if (!row_ptr || (nnz && !col)) return KOR_EINVAL;
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return KOR_EGRAPH;
    graph_t g = {n, row_ptr, col};
    for (uint32_t u = 0; u < n; ++u) {
        if (row_ptr[u + 1] < row_ptr[u]) return KOR_EGRAPH;
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint32_t v = col[e];
            if (v >= n || v == u) return KOR_EGRAPH;                 /* range, self-loop */
            if (e > row_ptr[u] && col[e - 1] >= v) return KOR_EGRAPH; /* unsorted or repeated */
            if (!has_edge(&g, v, u)) return KOR_EGRAPH;               /* asymmetric */
        }
    }
    return KOR_OK;
}

/* ---- k-clique listing: every clique once, as ids c[0] < c[1] < ... < c[k-1] ---- */

typedef void (*clique_fn)(const uint32_t *c, int k, void *ctx);

typedef struct {
    const graph_t *g;
    int k;
    uint32_t *clique;     /* k entries */
    uint32_t *cand;       /* k levels x maxdeg */
    uint64_t maxdeg;
    clique_fn fn;
    void *ctx;
} lister_t;

/* cand (ncand ids, ascending) are the common neighbours of clique[0..depth)
 * that exceed clique[depth-1].  Extend by each of them in turn. */
static void list_rec(lister_t *L, int depth, const uint32_t *cand, uint64_t ncand) {
    for (uint64_t i = 0; i < ncand; ++i) {
        uint32_t v = cand[i];
        L->clique[depth] = v;
        if (depth + 1 == L->k) {
            L->fn(L->clique, L->k, L->ctx);
            continue;
        }
        /* next = cand[i+1..] intersected with N(v) */
        uint32_t *next = L->cand + (uint64_t)(depth + 1) * L->maxdeg;
        uint64_t nn = 0;
        uint64_t a = i + 1, b = L->g->row_ptr[v], be = L->g->row_ptr[v + 1];
        while (a < ncand && b < be) {
            uint32_t x = cand[a], y = L->g->col[b];
            if (x < y) ++a;
            else if (y < x) ++b;
            else { next[nn++] = x; ++a; ++b; }
        }
        if ((uint64_t)(depth + 1) + nn >= (uint64_t)L->k) list_rec(L, depth + 1, next, nn);
    }
}

static uint64_t max_degree(const graph_t *g) {
    uint64_t d = 0;
    for (uint32_t u = 0; u < g->n; ++u) {
        uint64_t x = g->row_ptr[u + 1] - g->row_ptr[u];
        if (x > d) d = x;
    }
    return d;
}

/* List every k-clique whose smallest id is u. */
static void list_from(lister_t *L, uint32_t u) {
    const graph_t *g = L->g;
    uint64_t b = g->row_ptr[u], e = g->row_ptr[u + 1];
    while (b < e && g->col[b] < u) ++b;      /* neighbours greater than u */
    L->clique[0] = u;
    if ((uint64_t)1 + (e - b) >= (uint64_t)L->k) list_rec(L, 1, g->col + b, e - b);
}

static int lister_init(lister_t *L, const graph_t *g, int k, clique_fn fn, void *ctx, uint64_t maxdeg) {
    L->g = g; L->k = k; L->fn = fn; L->ctx = ctx; L->maxdeg = maxdeg ? maxdeg : 1;
    L->clique = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k);
    L->cand = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k * (size_t)L->maxdeg);
    return (L->clique && L->cand) ? KOR_OK : KOR_ENOMEM;
}

static void lister_free(lister_t *L) { free(L->clique); free(L->cand); }

/* ---- counting and explicit listing (used by tests of the clique tree) ---- */

static void count_fn(const uint32_t *c, int k, void *ctx) { (void)c; (void)k; ++*(uint64_t *)ctx; }

static int set_threads(int threads) {
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
    return omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

int kor_count(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int k, int threads,
              uint64_t *count_lo, uint64_t *count_hi) {
    if (k < 1 || !row_ptr || !count_lo || !count_hi) return KOR_EINVAL;
    graph_t g = {n, row_ptr, col};
    uint64_t maxdeg = max_degree(&g);
    u128 total = 0;
    int err = KOR_OK;
    set_threads(threads);
    if (k == 1) { *count_lo = n; *count_hi = 0; return KOR_OK; }
#pragma omp parallel reduction(+ : total)
    {
        lister_t L;
        uint64_t local = 0;
        if (lister_init(&L, &g, k, count_fn, &local, maxdeg) != KOR_OK) {
#pragma omp atomic write
            err = KOR_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t u = 0; u < (int64_t)n; ++u) {
                list_from(&L, (uint32_t)u);
                total += local;
                local = 0;
            }
        }
        lister_free(&L);
    }
    *count_lo = (uint64_t)total;
    *count_hi = (uint64_t)(total >> 64);
    return err;
}

typedef struct { uint32_t *out; uint64_t cap, used; } fill_ctx;

static void fill_fn(const uint32_t *c, int k, void *ctx) {
    fill_ctx *f = (fill_ctx *)ctx;
    if (f->used < f->cap) memcpy(f->out + f->used * (uint64_t)k, c, sizeof(uint32_t) * (size_t)k);
    ++f->used;
}

/* Write all k-cliques (sorted ids; ordered by smallest id, then lexicographically)
 * into out[cap * k].  *count receives the total; KOR_ENOMEM if it exceeds cap.
 * Two passes over the roots: count the cliques of every root, then let each
 * root write at its prefix offset. */
int kor_list(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int k,
             uint32_t *out, uint64_t cap, uint64_t *count) {
    if (k < 2 || !row_ptr || !count) return KOR_EINVAL;
    graph_t g = {n, row_ptr, col};
    uint64_t maxdeg = max_degree(&g);
    uint64_t *start = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!start) return KOR_ENOMEM;
    int err = KOR_OK;
#pragma omp parallel
    {
        lister_t L;
        uint64_t local = 0;
        if (lister_init(&L, &g, k, count_fn, &local, maxdeg) != KOR_OK) {
#pragma omp atomic write
            err = KOR_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t u = 0; u < (int64_t)n; ++u) {
                local = 0;
                list_from(&L, (uint32_t)u);
                start[u + 1] = local;
            }
        }
        lister_free(&L);
    }
    for (uint32_t u = 0; u < n; ++u) start[u + 1] += start[u];
    *count = start[n];
    if (err || start[n] > cap) { free(start); return err ? err : KOR_ENOMEM; }
#pragma omp parallel
    {
        fill_ctx f = {NULL, 0, 0};
        lister_t L;
        if (lister_init(&L, &g, k, fill_fn, &f, maxdeg) != KOR_OK) {
#pragma omp atomic write
            err = KOR_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t u = 0; u < (int64_t)n; ++u) {
                f.out = out + start[u] * (uint64_t)k;
                f.cap = start[u + 1] - start[u];
                f.used = 0;
                list_from(&L, (uint32_t)u);
            }
        }
        lister_free(&L);
    }
    free(start);
    return err;
}

/* ---- synchronous Frank-Wolfe (Alg. 1, FW-2: each clique credits its minimum-load node) ---- */

typedef struct { const u128 *r; uint64_t *delta; } fw_ctx;

/* Ids in c are ascending, so a strict '<' keeps the lowest id among equal loads. */
static uint32_t argmin_load(const uint32_t *c, int k, const u128 *r) {
    uint32_t best = c[0];
    for (int i = 1; i < k; ++i)
        if (r[c[i]] < r[best]) best = c[i];
    return best;
}

static void fw_fn(const uint32_t *c, int k, void *ctx) {
    fw_ctx *f = (fw_ctx *)ctx;
    f->delta[argmin_load(c, k, f->r)] += 1;
}

/* ---- extraction (Alg. 1 / Alg. 2 tail: sort by load, best prefix density) ---- */

static const u128 *g_sort_r;   /* qsort has no context argument; the sort is single-threaded */

static int cmp_desc_load(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    if (g_sort_r[x] != g_sort_r[y]) return g_sort_r[x] > g_sort_r[y] ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct { const uint32_t *pos; uint64_t *hist; } pre_ctx;

static void prefix_fn(const uint32_t *c, int k, void *ctx) {
    pre_ctx *p = (pre_ctx *)ctx;
    uint32_t last = 0;
    for (int i = 0; i < k; ++i)
        if (p->pos[c[i]] > last) last = p->pos[c[i]];
    p->hist[last] += 1;   /* the clique lies in every prefix V_i with i > last */
}

typedef struct {
    const graph_t *g;
    int k;
    int stored;
    uint32_t *cliques;    /* c_k * k ids when stored */
    uint64_t nclq;
    uint64_t maxdeg;
    int nthreads;
} run_t;

/* Apply fn with per-thread context ctxs[thread] to every k-clique. */
static int for_each_clique(run_t *R, clique_fn fn, void **ctxs) {
    int err = KOR_OK;
    if (R->stored) {
#pragma omp parallel
        {
#ifdef _OPENMP
            void *ctx = ctxs[omp_get_thread_num()];
#else
            void *ctx = ctxs[0];
#endif
#pragma omp for schedule(static)
            for (int64_t i = 0; i < (int64_t)R->nclq; ++i)
                fn(R->cliques + (uint64_t)i * (uint64_t)R->k, R->k, ctx);
        }
        return KOR_OK;
    }
#pragma omp parallel
    {
#ifdef _OPENMP
        void *ctx = ctxs[omp_get_thread_num()];
#else
        void *ctx = ctxs[0];
#endif
        lister_t L;
        if (lister_init(&L, R->g, R->k, fn, ctx, R->maxdeg) != KOR_OK) {
#pragma omp atomic write
            err = KOR_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t u = 0; u < (int64_t)R->g->n; ++u) list_from(&L, (uint32_t)u);
        }
        lister_free(&L);
    }
    return err;
}

/* Extraction on loads r: writes order[n], returns (i*, K_{i*}); K_out
 * (nullable) receives every prefix count, K_out[i - 1] = K_i. */
static int extract(run_t *R, const u128 *r, uint32_t *order, uint32_t *size, uint64_t *dens_num,
                   uint64_t **hist_t, uint32_t *pos, uint64_t *K_out) {
    uint32_t n = R->g->n;
    for (uint32_t i = 0; i < n; ++i) order[i] = i;
    g_sort_r = r;
    qsort(order, n, sizeof(uint32_t), cmp_desc_load);
    for (uint32_t i = 0; i < n; ++i) pos[order[i]] = i;

    void *ctxs[1024];
    pre_ctx pc[1024];
    for (int t = 0; t < R->nthreads; ++t) {
        memset(hist_t[t], 0, sizeof(uint64_t) * (size_t)n);
        pc[t].pos = pos;
        pc[t].hist = hist_t[t];
        ctxs[t] = &pc[t];
    }
    int err = for_each_clique(R, prefix_fn, ctxs);
    if (err) return err;

    /* K_i = number of cliques inside the first i nodes; best ratio, ties -> larger i */
    uint64_t K = 0, bestK = 0;
    uint32_t best_i = 0;
    for (uint32_t i = 1; i <= n; ++i) {
        for (int t = 0; t < R->nthreads; ++t) K += hist_t[t][i - 1];
        if (K_out) K_out[i - 1] = K;
        if (K == 0) continue;
        if (best_i == 0 || (u128)K * best_i >= (u128)bestK * i) { bestK = K; best_i = i; }
    }
    *size = best_i;
    *dens_num = bestK;
    return KOR_OK;
}

static u128 upper_bound_num(const u128 *r, const uint64_t *r0, uint32_t n) {
    u128 best = 0;
    for (uint32_t u = 0; u < n; ++u) {
        u128 x = r[u] - (r0 ? (u128)r0[u] : 0);
        if (x > best) best = x;
    }
    return best;
}

/*
 * Full solve.  r_out_lo / r_out_hi receive the low and high 64 bits of r_T,
 * order_out the extraction order pi (its first result->size entries are the
 * node set).  trace (nullable) receives T rows: the extraction after every
 * iteration.  max_store_bytes bounds the memory used to keep the clique list;
 * above it cliques are listed again on every pass.
 */
int kor_solve(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int k, uint32_t T,
              const uint64_t *r0, int threads, uint64_t max_store_bytes,
              uint64_t *r_out_lo, uint64_t *r_out_hi, uint32_t *order_out,
              kor_result *res, kor_trace_row *trace) {
    if (k < 2 || T == 0 || !row_ptr || !r_out_lo || !r_out_hi || !order_out || !res) return KOR_EINVAL;
    memset(res, 0, sizeof(*res));
    graph_t g = {n, row_ptr, col};
    run_t R;
    memset(&R, 0, sizeof(R));
    R.g = &g;
    R.k = k;
    R.maxdeg = max_degree(&g);
    R.nthreads = set_threads(threads);
    if (R.nthreads > 1024) return KOR_EINVAL;
    res->threads = R.nthreads;
    int err = KOR_OK;

    double t0 = now_s();
    uint64_t c_lo = 0, c_hi = 0;
    err = kor_count(n, row_ptr, col, k, threads, &c_lo, &c_hi);
    if (err) return err;
    u128 c_k = ((u128)c_hi << 64) | c_lo;
    res->c_k_lo = c_lo;
    res->c_k_hi = c_hi;
    if (c_hi == 0 && c_lo * (u128)k * 4u <= (u128)max_store_bytes) {
        R.stored = 1;
        R.nclq = c_lo;
        R.cliques = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(c_lo ? c_lo : 1) * (size_t)k);
        if (!R.cliques) return KOR_ENOMEM;
        uint64_t got = 0;
        err = kor_list(n, row_ptr, col, k, R.cliques, c_lo, &got);
        if (err || got != c_lo) { free(R.cliques); return err ? err : KOR_EGRAPH; }
    }
    res->streamed = !R.stored;
    res->enum_seconds = now_s() - t0;

    u128 *r = (u128 *)malloc(sizeof(u128) * (size_t)(n ? n : 1));
    uint64_t **delta_t = (uint64_t **)calloc((size_t)R.nthreads, sizeof(uint64_t *));
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    int ok = r && delta_t && pos;
    for (int t = 0; ok && t < R.nthreads; ++t) {
        delta_t[t] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
        ok = delta_t[t] != NULL;
    }
    if (!ok) { err = KOR_ENOMEM; goto done; }
    for (uint32_t u = 0; u < n; ++u) r[u] = r0 ? (u128)r0[u] : 0;

    double t1 = now_s(), t_extract_in_loop = 0.0;
    for (uint32_t it = 1; it <= T; ++it) {
        void *ctxs[1024];
        fw_ctx fc[1024];
        for (int t = 0; t < R.nthreads; ++t) {
            memset(delta_t[t], 0, sizeof(uint64_t) * (size_t)n);
            fc[t].r = r;
            fc[t].delta = delta_t[t];
            ctxs[t] = &fc[t];
        }
        err = for_each_clique(&R, fw_fn, ctxs);     /* every clique reads r_{t-1} */
        if (err) goto done;
        for (uint32_t u = 0; u < n; ++u)            /* then r_t = r_{t-1} + d_t */
            for (int t = 0; t < R.nthreads; ++t) r[u] += delta_t[t][u];
        if (trace) {
            double te = now_s();
            kor_trace_row *row = &trace[it - 1];
            row->t = it;
            err = extract(&R, r, order_out, &row->size, &row->dens_num, delta_t, pos, NULL);
            if (err) goto done;
            u128 ub = upper_bound_num(r, r0, n);
            row->ub_num_lo = (uint64_t)ub;
            row->ub_num_hi = (uint64_t)(ub >> 64);
            t_extract_in_loop += now_s() - te;
        }
    }
    res->iter_seconds = now_s() - t1 - t_extract_in_loop;

    double t2 = now_s();
    res->T = T;
    if (c_k == 0) {
        for (uint32_t i = 0; i < n; ++i) order_out[i] = i;
        g_sort_r = r;
        qsort(order_out, n, sizeof(uint32_t), cmp_desc_load);
        res->size = 0;
        res->dens_num = 0;
    } else {
        err = extract(&R, r, order_out, &res->size, &res->dens_num, delta_t, pos, NULL);
        if (err) goto done;
    }
    u128 ub = upper_bound_num(r, r0, n);
    res->ub_num_lo = (uint64_t)ub;
    res->ub_num_hi = (uint64_t)(ub >> 64);
    res->extract_seconds = now_s() - t2;
    for (uint32_t u = 0; u < n; ++u) {
        r_out_lo[u] = (uint64_t)r[u];
        r_out_hi[u] = (uint64_t)(r[u] >> 64);
    }

done:
    if (delta_t)
        for (int t = 0; t < R.nthreads; ++t) free(delta_t[t]);
    free(delta_t);
    free(pos);
    free(r);
    free(R.cliques);
    return err;
}

/* Frank-Wolfe credits of one iteration from loads r (u64), for tests of the first step. */
int kor_credits(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int k,
                const uint64_t *r, uint64_t *d_out) {
    if (k < 2 || !row_ptr || !r || !d_out) return KOR_EINVAL;
    graph_t g = {n, row_ptr, col};
    u128 *rr = (u128 *)malloc(sizeof(u128) * (size_t)(n ? n : 1));
    if (!rr) return KOR_ENOMEM;
    for (uint32_t u = 0; u < n; ++u) { rr[u] = r[u]; d_out[u] = 0; }
    fw_ctx fc = {rr, d_out};
    lister_t L;
    int err = lister_init(&L, &g, k, fw_fn, &fc, max_degree(&g));
    if (!err)
        for (uint32_t u = 0; u < n; ++u) list_from(&L, u);
    lister_free(&L);
    free(rr);
    return err;
}

int kor_threads(int threads) { return set_threads(threads); }

/* Extraction alone on given loads r (u64): the order pi, i* and K_{i*};
 * K_out (nullable, n entries) receives K_i = |C_k(pi[0 .. i))| for i = 1..n. */
int kor_prefix_counts(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int k, const uint64_t *r,
                      int threads, uint32_t *order_out, uint32_t *size_out, uint64_t *dens_out,
                      uint64_t *K_out) {
    if (k < 2 || !row_ptr || !r || !order_out || !size_out || !dens_out) return KOR_EINVAL;
    graph_t g = {n, row_ptr, col};
    run_t R = {&g, k, 0, NULL, 0, max_degree(&g), set_threads(threads)};
    if (R.nthreads > 1024) R.nthreads = 1024;
    u128 *rr = (u128 *)malloc(sizeof(u128) * (size_t)(n ? n : 1));
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint64_t *hist_t[1024];
    int err = (rr && pos) ? KOR_OK : KOR_ENOMEM;
    int made = 0;
    for (; !err && made < R.nthreads; ++made) {
        hist_t[made] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
        if (!hist_t[made]) err = KOR_ENOMEM;
    }
    if (!err) {
        for (uint32_t u = 0; u < n; ++u) rr[u] = r[u];
        err = extract(&R, rr, order_out, size_out, dens_out, hist_t, pos, K_out);
    }
    for (int t = 0; t < made; ++t) free(hist_t[t]);
    free(rr);
    free(pos);
    return err;
}

int kor_extract(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int k, const uint64_t *r,
                int threads, uint32_t *order_out, uint32_t *size_out, uint64_t *dens_out) {
    return kor_prefix_counts(n, row_ptr, col, k, r, threads, order_out, size_out, dens_out, NULL);
}

/*
 * ---- PBUpdate: the paper's per-pair update (Algorithm 3) ----
 *
 * Input is a set of pairs (V_h, V_p) of a succinct clique tree (Sec. 3.1):
 * the k-cliques of a pair are V_h plus any (k - h)-subset of V_p.  This oracle
 * does not build the tree; it takes the pairs as given (the test suite checks
 * separately that the pairs it uses partition C_k(V)).
 *
 * One pair, following the algorithm's steps and notation:
 *   n_C = C(p, k - h) cliques to allocate; caps up(u) = C(p, k - h) for
 *   u in V_h and C(p - 1, k - h - 1) for u in V_p (the number of the pair's
 *   cliques that contain u);
 *   V_1 .. V_s = the nodes of the pair grouped by equal load, loads
 *   r_1 < .. < r_s;
 *   for i = 1, 2, ..: gap = r_{i+1} - r_i (infinite for the last plateau);
 *     while cliques remain, gap > 0 and V_i is not empty:
 *       w = min(min over V_i of up(u), gap, floor(n_C / |V_i|));
 *       w > 0: every u in V_i gains w (up(u) -= w), n_C -= w |V_i|, gap -= w;
 *       w = 0: n_C < |V_i|: n_C nodes of V_i gain 1 each, n_C = 0;
 *       nodes with up(u) = 0 leave V_i;
 *     what is left of V_i joins V_{i+1}.
 * The paper picks the nodes of the last step uniformly at random; here they
 * are the n_C nodes of V_i with the lowest ids (a deterministic reading).
 *
 * Two ways to apply it over the pairs of one iteration:
 *   sequential (the paper's Algorithm 2 loop): pairs in the given order, each
 *     reading the loads the pairs before it left;
 *   synchronous: every pair reads r_{t-1}; the increments of all pairs are
 *     summed and added at the end of the iteration (order independent).
 * Loads are u128 inside; the u64 outputs report overflow as an error.
 */
static u128 binom_u128(uint64_t a, uint64_t b) {
    if (b > a) return 0;
    if (b > a - b) b = a - b;
    u128 c = 1;
    for (uint64_t i = 1; i <= b; ++i) c = c * (a - b + i) / i;   /* exact at every step */
    return c;
}

typedef struct { uint32_t u; u128 cur, up; int alive; } pb_node;

static int cmp_pb_load_id(const void *a, const void *b) {
    const pb_node *x = (const pb_node *)a, *y = (const pb_node *)b;
    if (x->cur != y->cur) return x->cur < y->cur ? -1 : 1;
    return x->u < y->u ? -1 : (x->u > y->u ? 1 : 0);
}

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* One pair: reads loads r, adds the pair's allocation into add (may equal r). */
static int pb_pair(const uint32_t *mem, uint32_t h, uint32_t p, int k, const u128 *r, u128 *add) {
    if ((int)h > k || (uint32_t)(k - (int)h) > p) return KOR_OK;   /* the pair holds no k-clique */
    uint32_t j = (uint32_t)k - h, sz = h + p;
    u128 nC = binom_u128(p, j);
    pb_node *V = (pb_node *)malloc(sizeof(pb_node) * (size_t)sz);
    uint32_t *plat = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(sz + 1));
    uint32_t *pick = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)sz);
    if (!V || !plat || !pick) { free(V); free(plat); free(pick); return KOR_ENOMEM; }
    for (uint32_t x = 0; x < sz; ++x) {
        V[x].u = mem[x];
        V[x].cur = r[mem[x]];
        /* a pivot node lies in C(p - 1, j - 1) of the pair's cliques: none when
           j = 0 (h = k, Lemma 4's pair holding H alone), so it takes nothing */
        V[x].up = x < h ? binom_u128(p, j) : (j ? binom_u128(p - 1, j - 1) : 0);
        V[x].alive = V[x].up > 0;
    }
    /* plateaus: V sorted by (load, id); plateau q covers V[plat[q] .. plat[q + 1]) */
    qsort(V, sz, sizeof(pb_node), cmp_pb_load_id);
    uint32_t s = 0;
    for (uint32_t x = 0; x < sz; ++x)
        if (x == 0 || V[x].cur != V[x - 1].cur) plat[s++] = x;
    plat[s] = sz;
    /* the current set V_i is every alive node with index below plat[i + 1]
       that has not been removed: earlier plateaus merge into later ones */
    for (uint32_t i = 0; nC > 0 && i < s; ++i) {
        const uint32_t end = plat[i + 1];
        int inf_gap = (i + 1 >= s);
        u128 gap = inf_gap ? 0 : V[plat[i + 1]].cur - V[plat[i]].cur;
        for (;;) {
            uint64_t cnt = 0;
            u128 minup = 0;
            for (uint32_t x = 0; x < end; ++x)
                if (V[x].alive) {
                    if (cnt == 0 || V[x].up < minup) minup = V[x].up;
                    ++cnt;
                }
            if (nC == 0 || (!inf_gap && gap == 0) || cnt == 0) break;
            u128 w = minup;
            if (!inf_gap && gap < w) w = gap;
            if (nC / cnt < w) w = nC / cnt;
            if (w > 0) {
                for (uint32_t x = 0; x < end; ++x)
                    if (V[x].alive) { V[x].cur += w; V[x].up -= w; }
                nC -= w * cnt;
                if (!inf_gap) gap -= w;
            } else {
                /* fewer cliques left than nodes in V_i: the lowest ids gain 1 */
                uint32_t m = 0;
                for (uint32_t x = 0; x < end; ++x)
                    if (V[x].alive) pick[m++] = V[x].u;
                qsort(pick, m, sizeof(uint32_t), cmp_u32);
                for (uint32_t x = 0; x < end; ++x)
                    if (V[x].alive) {
                        for (uint64_t q = 0; q < (uint64_t)nC; ++q)
                            if (pick[q] == V[x].u) { V[x].cur += 1; V[x].up -= 1; break; }
                    }
                nC = 0;
            }
            for (uint32_t x = 0; x < end; ++x)
                if (V[x].alive && V[x].up == 0) V[x].alive = 0;
        }
        /* the rest of V_i has reached r_{i+1} and joins V_{i+1} (end grows with i) */
    }
    for (uint32_t x = 0; x < sz; ++x) add[V[x].u] += V[x].cur - r[V[x].u];
    free(V); free(plat); free(pick);
    return nC == 0 ? KOR_OK : KOR_EINVAL;
}

/* One pair at loads r (u64): the pair's allocation added into d (u64). */
int kor_pb_pair(uint32_t n, const uint32_t *mem, uint32_t h, uint32_t p, int k, const uint64_t *r, uint64_t *d) {
    if (k < 2 || !mem || !r || !d) return KOR_EINVAL;
    u128 *rr = (u128 *)calloc((size_t)(n ? n : 1), sizeof(u128));
    u128 *dd = (u128 *)calloc((size_t)(n ? n : 1), sizeof(u128));
    if (!rr || !dd) { free(rr); free(dd); return KOR_ENOMEM; }
    for (uint32_t u = 0; u < n; ++u) rr[u] = r[u];
    int err = pb_pair(mem, h, p, k, rr, dd);
    for (uint32_t u = 0; !err && u < n; ++u) {
        if (dd[u] + d[u] > (u128)UINT64_MAX) err = KOR_EINVAL;
        d[u] += (uint64_t)dd[u];
    }
    free(rr); free(dd);
    return err;
}

/*
 * T iterations of PBUpdate over the pairs (members of pair q at
 * mem[off[q] .. off[q] + h[q] + p[q]), hold nodes first); r holds r_0 on entry
 * and r_T on return.  synchronous = 0: the paper's sequential pass.
 */
int kor_pb_run(uint32_t n, uint64_t npairs, const uint32_t *h, const uint32_t *p, const uint64_t *off,
               const uint32_t *mem, int k, uint32_t T, int synchronous, uint64_t *r, double *seconds) {
    if (k < 2 || !r || (npairs && (!h || !p || !off || !mem))) return KOR_EINVAL;
    u128 *cur = (u128 *)malloc(sizeof(u128) * (size_t)(n ? n : 1));
    u128 *nxt = (u128 *)malloc(sizeof(u128) * (size_t)(n ? n : 1));
    if (!cur || !nxt) { free(cur); free(nxt); return KOR_ENOMEM; }
    for (uint32_t u = 0; u < n; ++u) cur[u] = r[u];
    double t0 = now_s();
    int err = KOR_OK;
    for (uint32_t t = 1; !err && t <= T; ++t) {
        if (synchronous) {
            for (uint32_t u = 0; u < n; ++u) nxt[u] = cur[u];
            for (uint64_t q = 0; !err && q < npairs; ++q) err = pb_pair(mem + off[q], h[q], p[q], k, cur, nxt);
            u128 *sw = cur; cur = nxt; nxt = sw;
        } else {
            for (uint64_t q = 0; !err && q < npairs; ++q) err = pb_pair(mem + off[q], h[q], p[q], k, cur, cur);
        }
    }
    if (seconds) *seconds = now_s() - t0;
    for (uint32_t u = 0; !err && u < n; ++u) {
        if (cur[u] > (u128)UINT64_MAX) err = KOR_EINVAL;
        r[u] = (uint64_t)cur[u];
    }
    free(cur); free(nxt);
    return err;
}

/*
 * ---- CPSample (Algorithm 4): uniform k-clique samples from k-color paths ----
 *
 * Colouring: nodes in order of degree (descending, ties by ascending id), each
 * taking the smallest colour no already coloured neighbour has; adjacent nodes
 * differ.  A k-color path is a path v_1 .. v_k whose colours increase; a
 * k-clique sorted by colour is exactly one such path, so a uniform k-color path
 * that happens to be a clique is a uniform k-clique (the paper's CCPATH
 * sampler, read as colour-increasing paths).
 *   P_j(v) = number of colour-increasing paths of j nodes starting at v:
 *   P_1(v) = 1, P_j(v) = sum over neighbours u with c(u) > c(v) of P_{j-1}(u).
 * Sample i uses the given random draws R(i, s) (two u64 each, high word first):
 *   v_1 = the node (ascending ids) whose share of [0, sum_v P_k(v)) holds
 *         R(i, 0) mod sum_v P_k(v);
 *   v_{s+1}: x = R(i, s) mod P_{k-s+1}(v_s); the neighbours u of v_s with
 *         c(u) > c(v_s), in adjacency order, take shares P_{k-s}(u); v_{s+1}
 *         is the one whose share holds x.
 * The path is a sample; it is kept (valid) when every pair of its nodes is
 * adjacent.  Its ids are returned sorted.
 */
static uint32_t *g_deg_order_deg;
static int cmp_deg_desc(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    if (g_deg_order_deg[x] != g_deg_order_deg[y]) return g_deg_order_deg[x] > g_deg_order_deg[y] ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int kor_color(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t *color) {
    if (!row_ptr || !color) return KOR_EINVAL;
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint32_t *deg = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    uint32_t *seen = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n + 2));
    if (!order || !deg || !seen) { free(order); free(deg); free(seen); return KOR_ENOMEM; }
    for (uint32_t v = 0; v < n; ++v) {
        order[v] = v;
        deg[v] = (uint32_t)(row_ptr[v + 1] - row_ptr[v]);
        color[v] = UINT32_MAX;
    }
    g_deg_order_deg = deg;
    qsort(order, n, sizeof(uint32_t), cmp_deg_desc);
    for (uint32_t c = 0; c < n + 2; ++c) seen[c] = UINT32_MAX;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t v = order[i];
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (color[col[e]] != UINT32_MAX) seen[color[col[e]]] = v;   /* colours taken around v */
        uint32_t c = 0;
        while (seen[c] == v) ++c;
        color[v] = c;
    }
    free(order); free(deg); free(seen);
    return KOR_OK;
}

int kor_sample(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int k, uint64_t t,
               const uint64_t *draws, uint32_t *cliques, uint8_t *valid, uint64_t *paths_lo, uint64_t *paths_hi) {
    if (k < 2 || !row_ptr || (t && (!draws || !cliques || !valid))) return KOR_EINVAL;
    uint32_t *color = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    u128 *P = (u128 *)calloc((size_t)(n ? n : 1) * (size_t)(k + 1), sizeof(u128));   /* P[j * n + v] */
    if (!color || !P) { free(color); free(P); return KOR_ENOMEM; }
    int err = kor_color(n, row_ptr, col, color);
    for (uint32_t v = 0; !err && v < n; ++v) P[1 * (size_t)n + v] = 1;
    for (int j = 2; !err && j <= k; ++j)
        for (uint32_t v = 0; v < n; ++v) {
            u128 s = 0;
            for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
                if (color[col[e]] > color[v]) s += P[(size_t)(j - 1) * n + col[e]];
            P[(size_t)j * n + v] = s;
        }
    u128 total = 0;
    for (uint32_t v = 0; !err && v < n; ++v) total += P[(size_t)k * n + v];
    if (paths_lo) *paths_lo = (uint64_t)total;
    if (paths_hi) *paths_hi = (uint64_t)(total >> 64);
    graph_t g = {n, row_ptr, col};
    uint32_t path[64];
    for (uint64_t i = 0; !err && i < t; ++i) {
        valid[i] = 0;
        for (int s = 0; s < k; ++s) cliques[i * (uint64_t)k + s] = 0;
        if (total == 0) continue;
        const uint64_t *d = draws + 2 * i * (uint64_t)k;
        u128 x = ((((u128)d[0]) << 64) | d[1]) % total;
        uint32_t v = 0;
        for (; v < n; ++v) {                       /* the start node's share */
            u128 w = P[(size_t)k * n + v];
            if (x < w) break;
            x -= w;
        }
        path[0] = v;
        for (int s = 1; s < k; ++s) {
            const int j = k - s + 1;                /* nodes left on the path, v included */
            u128 y = ((((u128)d[2 * s]) << 64) | d[2 * s + 1]) % P[(size_t)j * n + v];
            uint32_t next = UINT32_MAX;
            for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                uint32_t u = col[e];
                if (color[u] <= color[v]) continue;
                u128 w = P[(size_t)(j - 1) * n + u];
                if (y < w) { next = u; break; }
                y -= w;
            }
            v = next;
            path[s] = v;
        }
        int clique = 1;
        for (int a = 0; clique && a < k; ++a)
            for (int b = a + 1; clique && b < k; ++b)
                if (!has_edge(&g, path[a], path[b])) clique = 0;
        qsort(path, (size_t)k, sizeof(uint32_t), cmp_u32);
        for (int s = 0; s < k; ++s) cliques[i * (uint64_t)k + s] = path[s];
        valid[i] = (uint8_t)clique;
    }
    free(color); free(P);
    return err;
}

/* Synchronous Frank-Wolfe (every listed clique credits its minimum-load node)
 * and the extraction, over a given list of k-cliques (ids ascending within a
 * clique): Algorithm 4's loop and its rho'_k extraction over the sample set. */
int kor_solve_list(uint32_t n, const uint32_t *cliques, uint64_t nclq, int k, uint32_t T, uint64_t *r_out,
                   uint32_t *order_out, uint32_t *size_out, uint64_t *dens_out) {
    if (k < 2 || T == 0 || !r_out || !order_out || !size_out || !dens_out || (nclq && !cliques)) return KOR_EINVAL;
    graph_t g = {n, NULL, NULL};
    run_t R;
    memset(&R, 0, sizeof(R));
    R.g = &g;
    R.k = k;
    R.stored = 1;
    R.nclq = nclq;
    R.cliques = (uint32_t *)cliques;
    R.nthreads = 1;
    set_threads(1);
    u128 *r = (u128 *)calloc((size_t)(n ? n : 1), sizeof(u128));
    uint64_t *delta = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    int err = (r && delta && pos) ? KOR_OK : KOR_ENOMEM;
    for (uint32_t it = 1; !err && it <= T; ++it) {
        memset(delta, 0, sizeof(uint64_t) * (size_t)n);
        fw_ctx fc = {r, delta};
        void *ctxs[1] = {&fc};
        err = for_each_clique(&R, fw_fn, ctxs);
        for (uint32_t u = 0; !err && u < n; ++u) r[u] += delta[u];
    }
    if (!err) {
        uint64_t *hist[1] = {delta};
        err = extract(&R, r, order_out, size_out, dens_out, hist, pos, NULL);
    }
    for (uint32_t u = 0; !err && u < n; ++u) r_out[u] = (uint64_t)r[u];
    free(r); free(delta); free(pos);
    return err;
}
