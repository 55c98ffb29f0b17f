"""Seeded synthetic graph generators.

These produce the inputs of every run: simple undirected graphs in CSR form
(``row_ptr`` uint64[n+1], ``col`` uint32[2m], each row sorted, symmetric, no
self-loops or duplicates).  They hold none of the k-clique densest-subgraph
arithmetic, so both the GPU path and the CPU oracle may take their graphs from
here.

Random numbers come from SplitMix64 used as a counter-based generator: the
i-th output of a stream with key ``s`` is ``mix(s + (i + 1) * 0x9E3779B97F4A7C15)``
where ``mix`` is SplitMix64's output function (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014).  Uniform doubles are
``(x >> 11) * 2**-53``.  A "seeded shuffle" is the order of ``n`` random 64-bit
keys (argsort, stable).

Stand-ins for the paper's datasets (Table 3: SNAP/KONECT social, web and
collaboration graphs) are Chung-Lu power-law graphs with an optional planted
near-clique, R-MAT graphs, and Erdos-Renyi graphs with a planted clique.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = 1.0 / float(1 << 53)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class Stream:
    """One independent SplitMix64 stream, identified by (seed, stream id)."""

    def __init__(self, seed: int, stream: int = 0):
        with np.errstate(over="ignore"):
            k = np.array([(seed * 0x100000001B3 + stream * 0x632BE59BD9B4E019) & (2**64 - 1)],
                         dtype=np.uint64)
            self.key = np.uint64(_mix(k + _GAMMA)[0])
        self.pos = 0

    def u64(self, count: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            i = np.arange(self.pos, self.pos + count, dtype=np.uint64) + np.uint64(1)
            out = _mix(self.key + i * _GAMMA)
        self.pos += count
        return out

    def uniform(self, count: int) -> np.ndarray:
        return (self.u64(count) >> np.uint64(11)).astype(np.float64) * _TWO_M53

    def shuffle_order(self, n: int) -> np.ndarray:
        """A seeded random permutation of range(n) (order of random keys)."""
        return np.argsort(self.u64(n), kind="stable").astype(np.int64)

    def integers(self, lo: int, hi: int, count: int = 1) -> np.ndarray:
        """Uniform integers in [lo, hi] (inclusive) by floor(U * width)."""
        width = hi - lo + 1
        return lo + np.minimum((self.uniform(count) * width).astype(np.int64), width - 1)


def sample_draws(seed: int, t: int, k: int) -> np.ndarray:
    """The random draws of t k-color path samples: uint64[t, k, 2], two words
    (high, low) per step; stream 97 of the seed.  Both the GPU sampler and
    the CPU reference take them as input."""
    return Stream(seed, 97).u64(2 * k * t).reshape(t, k, 2)


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray   # uint64[n+1]
    col: np.ndarray       # uint32[row_ptr[n]]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1]) // 2


def csr_from_edges(n: int, lo: np.ndarray, hi: np.ndarray, name: str = "") -> Graph:
    """Symmetric CSR from distinct undirected edges given as lo < hi pairs."""
    lo = np.asarray(lo, dtype=np.int64)
    hi = np.asarray(hi, dtype=np.int64)
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    key = np.sort((src << np.int64(32)) | dst)
    src = key >> np.int64(32)
    dst = key & np.int64(0xFFFFFFFF)
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.uint32), name=name)


def _dedupe(n: int, a: np.ndarray, b: np.ndarray):
    """Drop self-loops and repeated pairs, keeping first occurrences in draw order."""
    keep = a != b
    a, b = a[keep], b[keep]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = lo * np.int64(n) + hi
    _, first = np.unique(key, return_index=True)
    first.sort()
    return lo[first], hi[first]


def _relabel(n: int, lo: np.ndarray, hi: np.ndarray, rs: Stream):
    """Apply a seeded random relabelling of the node ids."""
    order = rs.shuffle_order(n)
    new_id = np.empty(n, dtype=np.int64)
    new_id[order] = np.arange(n, dtype=np.int64)
    a, b = new_id[lo], new_id[hi]
    return np.minimum(a, b), np.maximum(a, b)


def _planted(rs_nodes: Stream, rs_edges: Stream, n: int, size: int, prob: float):
    nodes = rs_nodes.shuffle_order(n)[:size]
    iu, ju = np.triu_indices(size, 1)
    if prob < 1.0:
        keep = rs_edges.uniform(iu.size) < prob
        iu, ju = iu[keep], ju[keep]
    return nodes[iu].astype(np.int64), nodes[ju].astype(np.int64)


def erdos_renyi(n: int, p: float, seed: int = 0, planted_clique: int = 0,
                relabel: bool = True) -> Graph:
    """G(n, p): pair (u, v), u < v, taken in lexicographic order, is an edge iff
    its uniform draw is below p; plus an optional clique on ``planted_clique``
    nodes chosen by a seeded shuffle (stream 1).  Relabelled by stream 2."""
    rs = Stream(seed, 0)
    iu, ju = np.triu_indices(n, 1)
    keep = rs.uniform(iu.size) < p
    lo, hi = iu[keep].astype(np.int64), ju[keep].astype(np.int64)
    if planted_clique:
        plo, phi = _planted(Stream(seed, 1), None, n, planted_clique, 1.0)
        lo, hi = _dedupe(n, np.concatenate([lo, plo]), np.concatenate([hi, phi]))
    if relabel:
        lo, hi = _relabel(n, lo, hi, Stream(seed, 2))
    return csr_from_edges(n, lo, hi, name=f"er{n}_p{p}_s{seed}_k{planted_clique}")


def chung_lu_weights(n: int, m: int, beta: float) -> np.ndarray:
    """Expected degrees w_i proportional to (i+1)^(-1/(beta-1)), summing to 2m."""
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (beta - 1.0))
    return w * (2.0 * m / w.sum())


def chung_lu(n: int, m: int, beta: float, seed: int = 0, planted: int = 0,
             planted_p: float = 0.9, relabel: bool = True) -> Graph:
    """Chung-Lu power-law graph with exactly m distinct edges.

    Endpoints are drawn independently with probability proportional to w
    (inverse CDF, stream 0); self-loops and repeated pairs are dropped and
    draws continue until m distinct edges exist (first occurrences kept).
    An optional near-clique on ``planted`` nodes (stream 1), each pair present
    with probability ``planted_p`` (stream 3), is added on top.  Node ids are
    then relabelled by a seeded shuffle (stream 2).
    """
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds the number of node pairs")
    w = chung_lu_weights(n, m, beta)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    rs = Stream(seed, 0)
    lo = np.empty(0, dtype=np.int64)
    hi = np.empty(0, dtype=np.int64)
    rounds = 0
    while lo.size < m:
        need = m - lo.size
        batch = int(need * 1.25) + 1024
        u = np.minimum(np.searchsorted(cdf, rs.uniform(batch), side="right"), n - 1)
        v = np.minimum(np.searchsorted(cdf, rs.uniform(batch), side="right"), n - 1)
        lo, hi = _dedupe(n, np.concatenate([lo, u.astype(np.int64)]),
                         np.concatenate([hi, v.astype(np.int64)]))
        rounds += 1
        if rounds > 200:
            raise RuntimeError("Chung-Lu sampling did not reach m distinct edges")
    lo, hi = lo[:m], hi[:m]
    if planted:
        plo, phi = _planted(Stream(seed, 1), Stream(seed, 3), n, planted, planted_p)
        lo, hi = _dedupe(n, np.concatenate([lo, plo]), np.concatenate([hi, phi]))
    if relabel:
        lo, hi = _relabel(n, lo, hi, Stream(seed, 2))
    return csr_from_edges(n, lo, hi, name=f"cl{n}_m{m}_b{beta}_s{seed}_pl{planted}")


def rmat(scale: int, edge_factor: int = 8, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 0, relabel: bool = True) -> Graph:
    """R-MAT: edge_factor * 2^scale draws, each choosing one of the four
    quadrants per level with probabilities (a, b, c, 1-a-b-c); the graph is
    symmetrised, loops and repeats dropped.  Relabelled by stream 2."""
    n = 1 << scale
    draws = edge_factor * n
    rs = Stream(seed, 0)
    u = np.zeros(draws, dtype=np.int64)
    v = np.zeros(draws, dtype=np.int64)
    for level in range(scale):
        x = rs.uniform(draws)
        bit = np.int64(1 << (scale - 1 - level))
        right = (x >= a) & (x < a + b) | (x >= a + b + c)
        down = x >= a + b
        u += np.where(down, bit, 0)
        v += np.where(right, bit, 0)
    lo, hi = _dedupe(n, u, v)
    if relabel:
        lo, hi = _relabel(n, lo, hi, Stream(seed, 2))
    return csr_from_edges(n, lo, hi, name=f"rmat{scale}_ef{edge_factor}_s{seed}")


def batch_member_params(index: int, base_seed: int = 1000, n_lo: int = 1000,
                        n_hi: int = 50000, d_lo: float = 8.0, d_hi: float = 40.0,
                        b_lo: float = 2.2, b_hi: float = 2.8):
    """(n, m, beta, seed) of member ``index`` of a batch of Chung-Lu graphs:
    n uniform in [n_lo, n_hi], average degree uniform in [d_lo, d_hi], exponent
    uniform in [b_lo, b_hi], m = round(n * d / 2); seed base_seed + index."""
    seed = base_seed + index
    rs = Stream(seed, 7)
    n = int(rs.integers(n_lo, n_hi)[0])
    d, beta = rs.uniform(2)
    d = d_lo + (d_hi - d_lo) * d
    beta = b_lo + (b_hi - b_lo) * beta
    m = min(int(round(n * d / 2.0)), n * (n - 1) // 2)
    return n, m, float(beta), seed


def batch_member(index: int, **kw) -> Graph:
    n, m, beta, seed = batch_member_params(index, **kw)
    return chung_lu(n, m, beta, seed=seed)


def from_edge_list(n: int, edges, name: str = "") -> Graph:
    """CSR from an explicit list of undirected (u, v) pairs (test fixtures)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if e.size == 0:
        return Graph(n=n, row_ptr=np.zeros(n + 1, dtype=np.uint64),
                     col=np.zeros(0, dtype=np.uint32), name=name)
    lo, hi = _dedupe(n, e[:, 0], e[:, 1])
    return csr_from_edges(n, lo, hi, name=name)


def complete_graph(n: int) -> Graph:
    iu, ju = np.triu_indices(n, 1)
    return csr_from_edges(n, iu.astype(np.int64), ju.astype(np.int64), name=f"K{n}")


def hub_core_size(n: int, m: int, beta: float) -> int:
    """Number of nodes whose Chung-Lu weight reaches sqrt(2m) (the saturated core)."""
    w = chung_lu_weights(n, m, beta)
    return int(np.count_nonzero(w >= math.sqrt(2.0 * m)))
