"""Pins of the certified bound on rho* and of the optimality check.

* Brute force over all node subsets (graphs of at most 13 nodes): rho* lies
  between the density found and the top-s bound, and the top-s bound is never
  above the plain bound max (r - r0) / T.
* Complete graphs: the top-s bound equals rho(K_n) = C(n, k) / n after any
  number of iterations, so the optimum is certified.
* A certified density is the brute-force optimum.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2403_05775_amd import synth
from tests import _brute as B


def rho_star(g, k):
    return B.max_density(g.n, B.cliques(g, k))


@pytest.mark.parametrize("seed", range(8))
def test_bound_brackets_optimum(oracle_mod, seed):
    O = oracle_mod
    rs = np.random.default_rng(seed)
    n = int(rs.integers(7, 14))
    g = synth.erdos_renyi(n, float(rs.uniform(0.35, 0.75)), seed=seed)
    k = int(rs.integers(2, 5))
    star = rho_star(g, k)
    for T in (1, 3, 20):
        res = O.solve(g.n, g.row_ptr, g.col, k, T)
        bound = O.top_bound(res["r"], None, T, k)
        dens = Fraction(res["dens_num"], res["size"]) if res["size"] else Fraction(0)
        assert dens <= star <= bound
        assert bound <= Fraction(res["ub_num"], T)
        if O.certified(res["dens_num"], res["size"], bound, g.n):
            assert dens == star


@pytest.mark.parametrize("n,k", [(7, 3), (9, 4), (6, 2)])
def test_bound_on_complete_graphs(oracle_mod, n, k):
    g = synth.complete_graph(n)
    for T in (1, 5):
        res = oracle_mod.solve(g.n, g.row_ptr, g.col, k, T)
        bound = oracle_mod.top_bound(res["r"], None, T, k)
        assert bound == Fraction(math.comb(n, k), n)
        assert oracle_mod.certified(res["dens_num"], res["size"], bound, n)


def test_bound_with_start_loads(oracle_mod):
    """With start loads the bound uses r - r0 (the loads the iterations added)."""
    g = synth.erdos_renyi(11, 0.6, seed=3)
    r0 = np.array([5, 0, 9, 1, 0, 3, 0, 0, 7, 2, 4], dtype=np.uint64)
    res = oracle_mod.solve(g.n, g.row_ptr, g.col, 3, 6, r0=r0)
    bound = oracle_mod.top_bound(res["r"], r0, 6, 3)
    assert rho_star(g, 3) <= bound <= Fraction(res["ub_num"], 6)
