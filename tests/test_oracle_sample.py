"""Pins of the oracle's CPSample pieces (Algorithm 4).

* Colouring: proper, at most max degree + 1 colours.
* Path counts: the number of colour-increasing k-node paths equals a
  brute-force depth-first enumeration.
* Samples: every sample is a colour-increasing path; it is flagged a clique
  exactly when all its pairs are adjacent; over many draws every such path
  appears with about the same frequency (uniform), so every k-clique does.
* Frank-Wolfe and the extraction over a clique list equal the brute-force
  definitions, and over the full list they equal the full solve.
"""
from __future__ import annotations

import itertools
from collections import Counter

import numpy as np
import pytest

from paper_2403_05775_amd import synth
from tests import _brute as B


def increasing_paths(g, color, k):
    a = B.adjacency(g)
    out = []

    def walk(path):
        if len(path) == k:
            out.append(tuple(path))
            return
        v = path[-1]
        for u in range(g.n):
            if a[v, u] and color[u] > color[v]:
                walk(path + [u])

    for v in range(g.n):
        walk([v])
    return out


@pytest.mark.parametrize("seed", range(4))
def test_colouring_and_path_counts(oracle_mod, seed):
    g = synth.erdos_renyi(14, 0.45, seed=seed, planted_clique=5)
    c = oracle_mod.color(g.n, g.row_ptr, g.col)
    a = B.adjacency(g)
    assert all(c[u] != c[v] for u in range(g.n) for v in range(g.n) if a[u, v])
    assert int(c.max()) <= int(a.sum(axis=1).max())
    for k in (2, 3, 4):
        s = oracle_mod.sample(g.n, g.row_ptr, g.col, k, synth.sample_draws(seed, 1, k))
        assert s["paths"] == len(increasing_paths(g, c, k))


def test_samples_are_uniform_increasing_paths(oracle_mod):
    g = synth.erdos_renyi(12, 0.5, seed=4, planted_clique=5)
    k = 3
    c = oracle_mod.color(g.n, g.row_ptr, g.col)
    paths = increasing_paths(g, c, k)
    cl = set(B.cliques(g, k))
    t = 300 * len(paths)
    s = oracle_mod.sample(g.n, g.row_ptr, g.col, k, synth.sample_draws(11, t, k))
    assert s["paths"] == len(paths)
    keyed = {tuple(sorted(p)): p for p in paths}   # a path's node set determines it (colours increase)
    seen = Counter(tuple(int(x) for x in row) for row in s["cliques"])
    assert set(seen) == set(keyed)                  # every sample is an increasing path, every path appears
    counts = np.array([seen[key] for key in keyed])
    assert counts.min() > 0.75 * 300 and counts.max() < 1.25 * 300
    for row, v in zip(s["cliques"], s["valid"]):
        assert bool(v) == (tuple(int(x) for x in row) in cl)


@pytest.mark.parametrize("seed", range(4))
def test_solve_over_a_clique_list(oracle_mod, seed):
    g = synth.erdos_renyi(12, 0.55, seed=seed)
    full = B.cliques(g, 3)
    rs = np.random.default_rng(seed)
    part = [c for c in full if rs.uniform() < 0.6]
    for cl, T in ((part, 5), (full, 7)):
        got = oracle_mod.solve_list(g.n, np.array(cl, dtype=np.uint32).reshape(-1, 3), 3, T)
        r = B.frank_wolfe(g.n, cl, T)
        order, i_star, K = B.best_prefix(g.n, cl, r)
        assert got["r"].tolist() == r
        assert (got["size"], got["dens_num"]) == (i_star, K)
        assert got["order"].tolist() == order
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, 3, 7)
    got = oracle_mod.solve_list(g.n, np.array(full, dtype=np.uint32).reshape(-1, 3), 3, 7)
    assert got["r"].tolist() == ref["r"].tolist() and (got["size"], got["dens_num"]) == (ref["size"],
                                                                                        ref["dens_num"])
