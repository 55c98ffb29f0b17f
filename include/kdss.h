/*
 * kdss -- k-clique densest subgraph search on MI355X (gfx950).
 *
 * The library runs the hot path of PSCTL (paper: Sec. 3, Algorithm 2) with the
 * Frank-Wolfe step of the convex program CP(G) (Sec. 2, Algorithm 1), batched
 * through the succinct clique tree (SCT, Sec. 2, Lemmas 3-5):
 *
 *   1. build the k-pruned SCT of the graph on the host (timed separately);
 *   2. T synchronous Frank-Wolfe iterations on the GPU: every leaf (hold set H,
 *      pivot set P) credits each member u with the exact number of the leaf's
 *      k-cliques whose minimum-load member is u (loads compared as (r(u), id(u)),
 *      lower id first on equal loads), and the credits are added to r;
 *   3. order the nodes by r non-increasing (ties: lower id first), count the
 *      k-cliques inside every prefix, and return the prefix with the highest
 *      k-clique density |C_k(S)|/|S| (Sec. 2), the longest one on ties.
 *
 * Every count is an exact integer; results do not depend on the SCT's shape
 * or on the order in which leaves are processed.
 *
 * Conventions for every entry point:
 *  - Return value: KDSS_OK (0) or a negative status below; kdss_last_error()
 *    then gives a thread-local message.  No call aborts or throws.
 *  - Host pointers are marked "host", device pointers "device".  The caller
 *    owns every buffer it passes; the library owns only the opaque handles it
 *    returns, which *_free releases (NULL is accepted).
 *  - The library allocates no device memory: the caller passes one device
 *    workspace of the size kdss_plan_info() reports.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *    enqueued on it in order; a call that fills a host result synchronises
 *    that stream before returning.
 *  - Handles are not safe for concurrent use from several threads.
 *  - Node ids are 32-bit; loads are u64, or u128 (two u64 per node: low word
 *    first) when a run could exceed 2^64 - 1.
 */
#ifndef KDSS_H
#define KDSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KDSS_OK 0
#define KDSS_EINVAL (-1)      /* bad argument: null pointer, k < 2, T == 0, ... */
#define KDSS_EGRAPH (-2)      /* the CSR is not a simple undirected graph      */
#define KDSS_ERANGE (-3)      /* a size exceeds a documented limit            */
#define KDSS_EOVERFLOW (-4)   /* an exact count would not fit its integer     */
#define KDSS_EWORKSPACE (-5)  /* workspace too small or not the uploaded one  */
#define KDSS_EHIP (-6)        /* a HIP runtime call failed                    */
#define KDSS_ENOMEM (-7)      /* host allocation failed                       */
#define KDSS_EUNSUPPORTED (-8)/* a case this build does not handle            */

typedef struct kdss_sct kdss_sct;     /* host clique tree (owned by the library) */
typedef struct kdss_plan kdss_plan;   /* device layout of one tree               */

/* Simple undirected graph G(V, E) (Sec. 2): n nodes, symmetric adjacency with
 * rows sorted ascending, no self-loops, no repeated neighbours.  Host arrays:
 * row_ptr[n + 1] (row_ptr[0] = 0, row_ptr[n] = nnz = 2|E|), col[nnz]. */
typedef struct {
    uint32_t n;
    uint64_t nnz;
    const uint64_t *row_ptr;
    const uint32_t *col;
} kdss_csr;

typedef struct { uint64_t lo, hi; } kdss_u128;

typedef struct {
    uint32_t k, n;
    uint64_t leaves;          /* |P_k|: leaves with h <= k <= h + p (Lemma 4)   */
    uint64_t members;         /* sum over those leaves of h + p                 */
    uint32_t s_max;           /* largest h + p                                  */
    uint32_t degeneracy;      /* delta of Sec. 2                                */
    kdss_u128 c_k;            /* |C_k(V)| = sum of C(p, k - h) (Lemma 5)        */
    double build_seconds;     /* host SCT construction, wall clock              */
} kdss_tree_stats;

typedef struct {
    int width;                /* 0: choose; 64 or 128: force the load width     */
    int use_graph;            /* G >= 1: replay the iterations as a hipGraph of
                                 G iterations (captured on first use; with
                                 extract_every, one iteration per replay)     */
    uint32_t extract_every;   /* 0: extract after iteration T only; e > 0: also
                                 after every e-th iteration, into the trace     */
    int time_kernels;         /* 1: time every iteration kernel of kdss_run
                                 with kernel-attached hipEvents (plain
                                 launches, no graph); see kdss_plan_timing    */
    int gather;               /* key gathers of the leaf-credit pass:
                                 0: choose (masked when hot nodes hold at least
                                    half of the member occurrences; autotune
                                    may switch);
                                 1: masked: only members inside the lane's leaf
                                    that are not hot are gathered;
                                 2: full: every row's key is gathered (no
                                    branch, more loads in flight)              */
    int update;               /* the per-iteration update:
                                 0: Frank-Wolfe (Algorithm 1): every k-clique
                                    credits its minimum-load member;
                                 1: PBUpdate (Algorithm 3), synchronous: every
                                    pair of the tree water-fills its C(p, k - h)
                                    cliques onto its lowest-load members, up to
                                    each member's clique count in the pair, all
                                    pairs reading r_{t-1}; a remainder smaller
                                    than the lowest plateau goes to its lowest
                                    ids.  The paper applies the pairs one after
                                    another; this variant sums them, so it does
                                    not depend on the pair order.  64-bit loads
                                    only.  The result's upper bound is certified
                                    only for update 0.                         */
    int schedule;             /* which tiles a workgroup of the persistent
                                 leaf-credit grid takes:
                                 0: choose (strided; autotune may switch);
                                 1: strided: wavefront w takes tiles w,
                                    w + W, w + 2W, .. of the whole list;
                                 2: XCD ranges: the tile list is cut into 8
                                    ranges of equal work, and the workgroups
                                    b = x, x + 8, .. take range x in strides,
                                    so each of the 8 XCDs (which run the
                                    workgroups with b mod 8 = x) walks one
                                    contiguous range and its L2 holds that
                                    range's keys.  Batches of Frank-Wolfe
                                    problems list their tiles problem by
                                    problem.  Grids under 8 workgroups run
                                    strided.                                  */
    int heavy;                /* leaves with more than four pivot members
                                 below their hold minimum ("heavy"):
                                 0: choose (queue; autotune may switch);
                                 1: queue: the leaf-credit kernel queues them
                                    and a second kernel spreads them over its
                                    grid, one leaf per wavefront, four per
                                    batch;
                                 2: in place: the wavefront that finds them
                                    takes them up at once, four at a time,
                                    while its tile's rows are still cached,
                                    and no second kernel runs (faster when
                                    heavy leaves are spread over many tiles
                                    and the loads fit in the caches; slower
                                    when they crowd into a few tiles);
                                 3: queue, eight leaves per batch (64-bit
                                    keys; four otherwise): more in flight per
                                    wavefront, faster on queues of millions,
                                    slower on short ones                    */
} kdss_opts;

typedef struct {              /* accumulated by kdss_run when time_kernels = 1  */
    uint64_t leaf_launches;   /* Frank-Wolfe credit passes timed                */
    double leaf_ms;           /* leaf-credit kernel, summed (hipEvent time)     */
    double heavy_ms;          /* heavy-leaf kernel that follows it (0 with
                                 heavy leaves in place: none runs)             */
    double reduce_ms;         /* hot-node reduction that completes the pass     */
    uint64_t apply_launches;
    double apply_ms;          /* load update r += credits                       */
    uint64_t heavy_leaves;    /* leaves queued for the heavy-leaf kernel, summed
                                 (0 with heavy leaves in place)                */
} kdss_timing;

typedef struct {
    uint64_t workspace_bytes; /* device workspace that kdss_plan_upload/run need */
    uint64_t stream_bytes;    /* leaf stream: members + headers + tile table     */
    int width;                /* load width of runs with this plan: 64 or 128   */
    int key_mode;             /* 0: packed 64-bit keys (r << id_bits | id);
                                 1: full (r, id) keys                           */
    uint32_t id_bits;
    uint32_t T_max;
    uint64_t tiles[5];        /* per size class: s <= 8, 16, 32, 64, > 64       */
    uint64_t leaves[5];
    uint64_t members[5];
    int gather;               /* gather mode of later runs: 1 masked, 2 full   */
    int update;               /* 0 Frank-Wolfe, 1 PBUpdate (synchronous)       */
    int schedule;             /* tile schedule of later runs: 1 strided, 2 XCD ranges */
    uint32_t hot_nodes;       /* nodes whose keys and credits live in LDS       */
    double hot_share;         /* their share of all member occurrences          */
    int heavy;                /* heavy leaves of later runs: 1 queue, 2 in place,
                                 3 queue with eight per batch                 */
} kdss_plan_stats;

typedef struct {
    uint32_t T;               /* iterations run                                 */
    uint32_t size;            /* i*: the node set is order[0 .. size)           */
    uint32_t n;
    int width;                /* load width used: 64 or 128                     */
    kdss_u128 dens_num;       /* K_{i*} = |C_k(order[0 .. i*))|                 */
    kdss_u128 ub_num;         /* max_u (r_T(u) - r0(u)); the bound is ub_num/T  */
    kdss_u128 c_k;
    double density;           /* dens_num / size (0 when size == 0)             */
    double upper_bound;       /* ub_num / T                                     */
    /* A certified bound on rho* = max_S |C_k(S)| / |S| and an optimality check
     * (Frank-Wolfe runs).  Any node set S of s nodes has |C_k(S)| <=
     * (sum of its (r - r0)) / T, since the cliques inside S put their weight
     * inside S, and |C_k(S)| <= C(s, k); so rho* <= max_s min(A_s, T C(s, k))
     * / (T s), A_s = the s largest (r - r0).  bound_kind 1: this top-s bound
     * (single problems with 64-bit loads and no start loads); 0: the plain
     * bound ub_num / T.  Two densities with denominators <= n differ by at
     * least 1 / (n (n - 1)), so certified = 1 when bound - density is below
     * that: the density is then rho*.  PBUpdate runs report bound_kind 0 and
     * certified 0 (their loads need not bound rho*).                         */
    kdss_u128 bound_num;      /* the bound is bound_num / bound_den             */
    uint64_t bound_den;
    int bound_kind;
    int certified;
    double bound;
} kdss_result;

typedef struct {              /* one extraction during a run                    */
    uint32_t t, size;
    kdss_u128 dens_num;
    kdss_u128 ub_num;
} kdss_trace_row;

/* Name of a status code, and the detail of the calling thread's last error. */
const char *kdss_status_string(int status);
const char *kdss_last_error(void);

/* Checks that g is a simple undirected graph in the form described above.
 * KDSS_OK, KDSS_EINVAL (null arrays) or KDSS_EGRAPH. Host only. */
int kdss_csr_validate(const kdss_csr *g);

/* Builds the k-pruned succinct clique tree of g (Sec. 2 "Succinct Clique Tree",
 * Lemmas 3-5) on the host with up to `threads` threads (0: all cores).  Only
 * leaves with h <= k <= h + p are kept (Lemma 4).  Every k-clique of g lies in
 * exactly one kept leaf.  g's arrays are read during the call only.
 * Errors: KDSS_EINVAL (k < 2, null), KDSS_EGRAPH, KDSS_ERANGE (k > 31),
 * KDSS_EOVERFLOW (|C_k| >= 2^128), KDSS_ENOMEM. */
int kdss_sct_build(const kdss_csr *g, uint32_t k, uint32_t threads, kdss_sct **out);

/* The same tree built on the current device on `stream`: the graph check on
 * the host; on the device a degeneracy order by level-synchronous peeling
 * (every node left with at most L remaining neighbours leaves in one
 * sub-round, ranked by id within it, and L grows when none is left; the
 * tree's core numbers are the levels), the graph oriented along it (each node
 * keeps its later neighbours), then, per start node, the local adjacency
 * bitsets of its later neighbours (built once, kept in a device store), the
 * root pivot and the root's children; one thread per root child runs the
 * pivoting recursion below it with an explicit stack, heaviest start nodes
 * first; a counting pass and a writing pass over chunks of children.  The
 * leaves may differ from kdss_sct_build's (another valid tree: every k-clique
 * in exactly one kept leaf), so every result computed on it is the same.
 * Device memory is the caller's workspace d_ws (ws_bytes): the graph, the
 * order, the oriented lists, the root bitsets and tasks, one chunk's recursion
 * scratch (at most half of what is left, at most 8 GiB) and, in the rest, a
 * staging window through which each chunk's leaves are copied back to the host.
 * The call synchronises the stream (once per peeling sub-round too);
 * build_seconds covers the whole call.
 * Errors: as kdss_sct_build, plus KDSS_EUNSUPPORTED (degeneracy above 256,
 * found by the peeling), KDSS_EWORKSPACE (d_ws NULL, too small for the fixed
 * parts, or one root child's leaves larger than the staging window) and
 * KDSS_EHIP. */
int kdss_sct_build_gpu(const kdss_csr *g, uint32_t k, void *d_ws, size_t ws_bytes, void *stream,
                       kdss_sct **out);

/* A workspace size (bytes) with which kdss_sct_build_gpu runs g at k: the
 * fixed parts bounded from n and nnz (the bitsets by nnz / 2 later neighbours
 * times ceil(degeneracy / 64) words, the degeneracy from a host peeling), one
 * chunk of recursion scratch, and a 512 MiB staging window.  Host only.
 * Errors: as kdss_sct_build_gpu's argument and graph checks, and
 * KDSS_EUNSUPPORTED for degeneracy above 256. */
int kdss_sct_build_gpu_workspace(const kdss_csr *g, uint32_t k, size_t *bytes);

int kdss_sct_info(const kdss_sct *s, kdss_tree_stats *out);

/* Sizes the k-pruned tree of g before (or instead of) building it: the same
 * search as kdss_sct_build (Sec. 2 "Succinct Clique Tree", Lemmas 3-5, the
 * same leaves), keeping only the counts.  out (host) receives k, n, the kept
 * leaves |P_k|, their members, s_max, the degeneracy, c_k = |C_k(V)| (Lemma
 * 5) and the seconds taken (build_seconds).  Host memory stays O(n + m)
 * whatever the tree's size.  Errors as kdss_sct_build. */
int kdss_sct_count(const kdss_csr *g, uint32_t k, uint32_t threads, kdss_tree_stats *out);

/* Copies the kept leaves to host arrays: h[i], p[i] per leaf and the members
 * (leaf by leaf, its h hold nodes first, then its p pivot nodes).
 * KDSS_ERANGE if a capacity is too small. */
int kdss_sct_export(const kdss_sct *s, uint32_t *h, uint32_t *p, uint32_t *members,
                    uint64_t leaf_cap, uint64_t member_cap);

/* Core number of every node (a by-product of the degeneracy order); core[n].
 * KDSS_EUNSUPPORTED for a tree of sampled cliques (kdss_sample_build). */
int kdss_sct_core_numbers(const kdss_sct *s, uint32_t *core, uint32_t n);

void kdss_sct_free(kdss_sct *s);

/* ---- CPSample (Algorithm 4): a tree of uniformly sampled k-cliques ----
 * Samples t colour-increasing k-node paths uniformly (the CCPATH sampler the
 * algorithm cites): nodes are coloured greedily in order of degree
 * (descending, ties by ascending id), each taking the smallest colour no
 * coloured neighbour has; P_j(v), the number of colour-increasing paths of j
 * nodes from v, is counted for j = 1..k; a sample picks its start with weight
 * P_k(v) and each next node among the higher-coloured neighbours with weight
 * P_{j-1}(u), using the caller's random draws: h_draws (host) holds t * k
 * pairs of u64 (high word, then low word), pair s of sample i being step s's
 * 128-bit draw, reduced mod the step's total.  A k-clique sorted by colour is
 * exactly one such path, so the samples that are cliques are uniform
 * k-cliques.  The distinct sampled cliques C become the leaves (C, {}) of the
 * returned tree: a plan and kdss_run on it run Algorithm 4's loop (here
 * synchronous) over the sample set and its extraction by
 * rho'_k(V_i) = |C_k(V_i) with sampled C| / i.  The path counts and walks run
 * on the current device on `stream`, in the caller's device workspace d_ws of
 * ws_bytes >= kdss_sample_workspace(n, nnz, k, t) bytes (the graph, the path
 * counts P_1..P_k and their prefix sums in 128 bits, the draws and the walks;
 * NULL when that size is 0); the call synchronises the stream.  Colouring and
 * the de-duplication run on the host.
 * Errors: KDSS_EINVAL (k < 2, null draws with t > 0), KDSS_EGRAPH,
 * KDSS_ERANGE (k > 31), KDSS_EOVERFLOW (2^128 or more paths, seen as a
 * wrapped path count, block sum or running total), KDSS_EWORKSPACE,
 * KDSS_ENOMEM, KDSS_EHIP. */
typedef struct {
    uint64_t samples;         /* t                                             */
    uint64_t cliques;         /* samples that are k-cliques                    */
    uint64_t distinct;        /* distinct sampled cliques (the tree's leaves)  */
    kdss_u128 paths;          /* colour-increasing k-node paths in g           */
    uint32_t colors;          /* colours used                                  */
    double device_seconds;    /* path counts and walks (synchronised)          */
    double host_seconds;      /* colouring, uploads, de-duplication, the tree  */
} kdss_sample_info;

int kdss_sample_build(const kdss_csr *g, uint32_t k, uint64_t t, const uint64_t *h_draws, void *d_ws,
                      size_t ws_bytes, void *stream, kdss_sample_info *info, kdss_sct **out);

/* Device workspace (bytes) of kdss_sample_build for n nodes, nnz directed
 * edges, clique size k and t samples (0 when n or t is 0).  Host only. */
int kdss_sample_workspace(uint32_t n, uint64_t nnz, uint32_t k, uint64_t t, size_t *bytes);

/* Lays out s for the GPU, for runs of at most T_max iterations whose start
 * loads r0 are all <= r0_max.  Chooses the load width (u64 when
 * r0_max + T_max * |C_k| < 2^64, else u128) and the key mode.  opts may be NULL.
 * Errors: KDSS_EINVAL, KDSS_EOVERFLOW (|C_k| >= 2^64, or u128 needed but
 * width 64 forced), KDSS_EUNSUPPORTED (a leaf larger than 4096 members, or
 * more than 2^31 nodes). */
int kdss_plan_create(const kdss_sct *s, uint32_t T_max, uint64_t r0_max, const kdss_opts *opts,
                     kdss_plan **out);
int kdss_plan_info(const kdss_plan *p, kdss_plan_stats *out);

/* Device workspace (bytes, into *bytes) that a plan of s with these arguments
 * needs: kdss_plan_info().workspace_bytes of that plan, without keeping it.
 * Errors as kdss_plan_create. */
int kdss_workspace_size(const kdss_sct *s, uint32_t T_max, uint64_t r0_max, const kdss_opts *opts,
                        size_t *bytes);

/* Kernel durations gathered by kdss_run with opts.time_kernels = 1 since the
 * plan was created or the last reset (reset != 0 clears them after copying).
 * Each duration is the kernel's own execution span: the runtime stamps the
 * dispatch's start and end into the launch's events (hipExtLaunchKernel), so
 * no marker packet sits between the kernels of a timed run. */
int kdss_plan_timing(kdss_plan *p, kdss_timing *out, int reset);

/* Switches the plan's kernel timing (opts.time_kernels) on or off for later runs. */
int kdss_plan_set_timing(kdss_plan *p, int on);
void kdss_plan_free(kdss_plan *p);

/* Copies the leaf stream, tile table and binomial table into the device
 * workspace d_ws (ws_bytes >= workspace_bytes) on `stream`.  Must precede
 * kdss_run on that workspace.  Errors: KDSS_EWORKSPACE, KDSS_EHIP. */
int kdss_plan_upload(kdss_plan *p, void *d_ws, size_t ws_bytes, void *stream);

/* Runs T (1 <= T <= T_max) synchronous Frank-Wolfe iterations (Algorithm 2's
 * loop with Algorithm 1's per-clique step) from loads d_r0 (device u64[n];
 * NULL = all zero; every entry must be <= r0_max), then the extraction.
 * Outputs (device, caller-owned): d_r receives r_T (u64[n], or u128[n] as
 * 2n u64 when the plan's width is 128); d_order receives the order pi (u32[n]),
 * whose first h_res->size entries are the node set.  h_trace (host, nullable)
 * receives one row per extraction when opts->extract_every > 0, at most
 * trace_cap rows.  h_res (host) is filled after the stream is synchronised.
 * Errors: KDSS_EINVAL, KDSS_EWORKSPACE, KDSS_EOVERFLOW (an r0 entry exceeds
 * r0_max: found when the start loads are read, before the first iteration), KDSS_EHIP. */
int kdss_run(kdss_plan *p, void *d_ws, size_t ws_bytes, uint32_t T, const uint64_t *d_r0,
             void *d_r, uint32_t *d_order, kdss_trace_row *h_trace, uint32_t trace_cap,
             kdss_result *h_res, void *stream);

/* Continues a run from a checkpoint (Algorithm 2's loop is a map r_{t-1} ->
 * r_t, so T more iterations from r_t equal iterations t + 1 .. t + T of one
 * run).  d_start (device u64[n]) holds the checkpoint loads r_{t_offset} of a
 * run that began at d_r0 (device u64[n], nullable = zero); every d_start entry
 * must be <= the plan's r0_max (create the plan with r0_max >= the largest
 * checkpoint load).  Runs T iterations from d_start, then the extraction; the
 * upper bound and certificate use r - r0 over t_offset + T iterations, h_res->T
 * and trace rows count from t_offset, so the result equals that of one
 * kdss_run of t_offset + T iterations from d_r0, bit for bit.  Outputs and the
 * other errors as kdss_run; KDSS_ERANGE when t_offset + T >= 2^32. */
int kdss_run_resume(kdss_plan *p, void *d_ws, size_t ws_bytes, uint32_t T, uint32_t t_offset,
                    const uint64_t *d_start, const uint64_t *d_r0, void *d_r, uint32_t *d_order,
                    kdss_trace_row *h_trace, uint32_t trace_cap, kdss_result *h_res, void *stream);

/* One-shot (Algorithm 2 end to end): builds g's k-pruned tree on host threads,
 * lays it out for T iterations with start loads <= r0_max, and, when the
 * caller's buffers are large enough, uploads it into d_ws, runs kdss_run (T
 * iterations from d_r0, nullable) and the extraction, and frees the tree and
 * plan.  *ws_needed (host) always receives the workspace the plan needs, and
 * h_res->width / h_res->n the load width and node count; when d_ws is NULL, or
 * ws_bytes < *ws_needed, or r_words (u64 words at d_r) < n (2n for 128-bit
 * loads), nothing runs and KDSS_EWORKSPACE is returned, so a caller can size
 * its buffers with a first call.  The library allocates no device memory.
 * Synchronises the stream.  Other errors as kdss_sct_build, kdss_plan_create
 * and kdss_run. */
int kdss_solve(const kdss_csr *g, uint32_t k, uint32_t T, const kdss_opts *opts, const uint64_t *d_r0,
               uint64_t r0_max, void *d_ws, size_t ws_bytes, size_t *ws_needed, void *d_r, size_t r_words,
               uint32_t *d_order, kdss_result *h_res, void *stream);

/* One leaf-credit pass (Algorithm 1's per-clique step, batched by Lemma 5) at loads
 * d_r (device, the plan's width): d_out[u] (device u64[n], overwritten) =
 * the number of k-cliques whose minimum (r, id) member is u.  Enqueued only. */
int kdss_leaf_credit(kdss_plan *p, void *d_ws, size_t ws_bytes, const void *d_r,
                     uint64_t *d_out, void *stream);

/* The extraction alone (Algorithm 2, last three lines) at loads d_r after T
 * iterations from d_r0 (nullable): order into d_order (device u32[n]), result
 * into h_res (host; synchronises the stream). */
int kdss_extract(kdss_plan *p, void *d_ws, size_t ws_bytes, const void *d_r,
                 const uint64_t *d_r0, uint32_t T, uint32_t *d_order, kdss_result *h_res,
                 void *stream);

/* kdss_extract that also writes every prefix count of Algorithm 2's scoring:
 * d_counts[i - 1] = K_i = |C_k(order[0 .. i))| for i = 1..n (device u64[n],
 * caller-owned; each k-clique counted once, Lemma 4), so K_i / i is the
 * k-clique density (Sec. 2) of every prefix.  d_counts may be NULL.
 * KDSS_EUNSUPPORTED for batch plans with d_counts. */
int kdss_extract_counts(kdss_plan *p, void *d_ws, size_t ws_bytes, const void *d_r, const uint64_t *d_r0,
                        uint32_t T, uint32_t *d_order, uint64_t *d_counts, kdss_result *h_res, void *stream);

/* ---- runs without device allocation ----
 * For callers that cannot allocate device memory (tight serving loops, code
 * that must not call hipMalloc): kdss_run with the plan's workspace taken from
 * a static device array of KDSS_STATIC_WORKSPACE_BYTES that the library holds
 * on every GPU it runs on until the process ends.  Each call copies the plan's
 * leaf stream and tables into the current device's array (kdss_plan_upload's
 * work; the stream is synchronised), clears its queue and hot-node slots with
 * kernels, then runs T iterations from d_r0 (device u64[n], nullable, entries
 * <= r0_max) and the extraction with plain launches (the plan's use_graph,
 * time_kernels and extract_every are ignored).  d_r, d_order and h_res as in
 * kdss_run; the result equals kdss_run's bit for bit.  The call makes no
 * device allocation.  All calls on one GPU share its array: calls that
 * overlap on one GPU (from several threads or streams) race and are not
 * allowed.  After the call the plan is uploaded to the array, not to any
 * earlier workspace (kdss_plan_upload again before kdss_run there).
 * Errors: KDSS_ERANGE when kdss_plan_info().workspace_bytes exceeds
 * KDSS_STATIC_WORKSPACE_BYTES; others as kdss_run. */
#define KDSS_STATIC_WORKSPACE_BYTES (64u << 20)
int kdss_run_static(kdss_plan *p, uint32_t T, const uint64_t *d_r0, void *d_r, uint32_t *d_order,
                    kdss_result *h_res, void *stream);

/* ---- launch tuning (autotuned tile schedules) ----
 * The leaf-credit and heavy-leaf kernels run persistent grids; their sizes
 * decide how tiles and queued heavy leaves are spread over the 256 CUs. */

typedef struct {
    uint32_t tried;               /* configurations timed                      */
    uint32_t best_leaf_blocks, best_heavy_blocks;
    double best_ms;               /* per iteration, best configuration         */
    uint32_t leaf_blocks[32], heavy_blocks[32];
    double ms[32];                /* per iteration, each grid-size pair (the
                                     first 32 of the 49 timed)                 */
    int best_gather;              /* gather mode kept (1 masked, 2 full)       */
    double gather_ms[2];          /* per iteration at the best grid sizes with
                                     masked / full gathers (0: not timed)      */
    int best_schedule;            /* tile schedule kept (1 strided, 2 XCD ranges) */
    double schedule_ms[2];        /* per iteration with each schedule at the
                                     best grid sizes and gather (0: not timed) */
    int best_heavy;               /* heavy leaves kept (1 queue, 2 in place,
                                     3 queue with eight per batch)             */
    double heavy_ms[3];           /* per iteration with each heavy-leaf mode at
                                     the best launch otherwise (0: not timed)  */
} kdss_tune_result;

/* Sets the grid sizes (leaf-credit 1..8192, heavy-leaf 1..16384 workgroups) used by later runs. */
int kdss_plan_set_launch(kdss_plan *p, uint32_t leaf_blocks, uint32_t heavy_blocks);

/* Times `iters` iterations after `warm` untimed ones (from zero loads) for each
 * candidate pair of grid sizes on the plan's own data, keeps the fastest and
 * reports all (out, host).  Then each choice the plan's options left to the
 * library (the gather mode, then the heavy-leaf mode, then the tile schedule)
 * has its other values timed at the best launch so far, the fastest kept.  d_r (device, the plan's load width) is scratch.
 * warm + iters must not exceed T_max.  Synchronises the stream. */
int kdss_plan_autotune(kdss_plan *p, void *d_ws, size_t ws_bytes, uint64_t *d_r, uint32_t warm, uint32_t iters,
                       kdss_tune_result *out, void *stream);

/* The key under which kdss_plan_autotune_cached files a plan's tuning (host
 * string, NUL-terminated, into buf[cap]): the current device's architecture,
 * the kernel variant (load width, key mode, update, gather, schedule and
 * heavy-leaf options), the problems' clique sizes, and half-octave buckets of
 * the problem count, node count and leaves per size class.  KDSS_ERANGE if cap is too small. */
int kdss_plan_tune_key(const kdss_plan *p, char *buf, size_t cap);

/* kdss_plan_autotune through a tuning cache: a text file (cache_path, host)
 * of lines "key leaf_blocks heavy_blocks gather schedule heavy ms".  When the file holds the
 * plan's key (the last such line wins) its launch is applied without timing
 * anything (*from_cache = 1; out carries only the best_* fields); otherwise the
 * plan is tuned as by kdss_plan_autotune and a line is appended (*from_cache =
 * 0).  Errors as kdss_plan_autotune. */
int kdss_plan_autotune_cached(kdss_plan *p, void *d_ws, size_t ws_bytes, uint64_t *d_r, uint32_t warm,
                              uint32_t iters, const char *cache_path, int *from_cache, kdss_tune_result *out,
                              void *stream);

/* ---- batches: many problems (graph, k) in one launch per iteration ----
 * (each problem is exactly the problem of
 * kdss_run, and its result equals a solo run bit for bit) */

/* Lays out `count` trees (each with its own graph and k) as one plan: problem q
 * owns the node ids node_off[q] .. node_off[q+1]-1 of one concatenated id
 * space (kdss_batch_offsets), every iteration is one persistent launch over all
 * leaves, and leaves carry their own k.  The trees are read during the call
 * only.  r0_max bounds every start load.  Errors as kdss_plan_create;
 * KDSS_EUNSUPPORTED for more than 2^31 nodes in total. */
int kdss_batch_create(const kdss_sct *const *trees, uint32_t count, uint32_t T_max, uint64_t r0_max,
                      const kdss_opts *opts, kdss_plan **out);

/* node_off[count + 1] (host): first node id of every problem, then the total. */
int kdss_batch_offsets(const kdss_plan *p, uint64_t *node_off, uint32_t count);

/* Runs T iterations for every problem of a batch plan, then every problem's
 * extraction.  d_r0 (device u64[total], nullable), d_r (device u64[total]) and
 * d_order (device u32[total]) use the concatenated id space; problem q's order
 * occupies d_order[node_off[q] .. node_off[q+1]) and holds its local ids, its
 * node set being the first h_res[q].size of them.  h_res (host) receives one
 * result per problem.  Batches use 64-bit loads (KDSS_EUNSUPPORTED otherwise,
 * or when log2(count) + log2(largest bound) exceeds 64 bits).  Other errors as
 * kdss_run. */
int kdss_batch_run(kdss_plan *p, void *d_ws, size_t ws_bytes, uint32_t T, const uint64_t *d_r0, uint64_t *d_r,
                   uint32_t *d_order, kdss_result *h_res, uint32_t count, void *stream);

/* Releases a batch plan (the same as kdss_plan_free; NULL is accepted). */
void kdss_batch_free(kdss_plan *p);

#ifdef __cplusplus
}
#endif

#endif /* KDSS_H */
