"""Brute force on tiny graphs (n <= 14), written straight from the definitions
of Sec. 2: k-cliques as all k-subsets whose pairs are all edges, k-clique
density |C_k(S)|/|S|, the Frank-Wolfe step of Algorithm 1 (each clique credits
one unit to its minimum-load member), and the best prefix of the load order.
It uses no clique tree and no clique-listing recursion, so it is independent of
both the oracle and the GPU path."""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def adjacency(g) -> np.ndarray:
    a = np.zeros((g.n, g.n), dtype=bool)
    rp = g.row_ptr.astype(np.int64)
    for u in range(g.n):
        for e in range(rp[u], rp[u + 1]):
            a[u, int(g.col[e])] = True
    return a


def cliques(g, k) -> list[tuple[int, ...]]:
    a = adjacency(g)
    out = []
    for c in itertools.combinations(range(g.n), k):
        if all(a[x, y] for x, y in itertools.combinations(c, 2)):
            out.append(c)
    return out


def frank_wolfe(n, cl, T, r0=None):
    """Synchronous: all cliques of iteration t read the loads of iteration t-1;
    ties between equal loads go to the lowest id."""
    r = [0] * n if r0 is None else [int(x) for x in r0]
    for _ in range(T):
        d = [0] * n
        for c in cl:
            d[min(c, key=lambda v: (r[v], v))] += 1
        r = [r[u] + d[u] for u in range(n)]
    return r


def best_prefix(n, cl, r):
    """Order by load non-increasing (ties: lower id first); among prefixes with
    the highest density take the longest.  Returns (order, i*, K_{i*})."""
    order = sorted(range(n), key=lambda v: (-r[v], v))
    best, best_i, best_K = Fraction(-1), 0, 0
    if not cl:
        return order, 0, 0
    for i in range(1, n + 1):
        s = set(order[:i])
        K = sum(1 for c in cl if s.issuperset(c))
        if K and Fraction(K, i) >= best:
            best, best_i, best_K = Fraction(K, i), i, K
    return order, best_i, best_K


def max_density(n, cl) -> Fraction:
    """rho* = max over non-empty subsets S of |C_k(S)| / |S| (subset-sum transform)."""
    f = np.zeros(1 << n, dtype=np.int64)
    for c in cl:
        f[sum(1 << v for v in c)] += 1
    for b in range(n):
        bit = 1 << b
        idx = np.arange(1 << n)
        sel = (idx & bit) != 0
        f[sel] += f[idx[sel] ^ bit]
    best = Fraction(0)
    for S in range(1, 1 << n):
        if f[S]:
            x = Fraction(int(f[S]), bin(S).count("1"))
            if x > best:
                best = x
    return best
