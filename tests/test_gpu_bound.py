"""The certified bound on rho* (top-s bound) and the optimality check through
the C-ABI, against the oracle's bound computed from its own loads."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2403_05775_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_05775_amd import kdss
    kdss.lib()
    return kdss


@pytest.mark.parametrize("seed", range(6))
def test_top_bound_matches_oracle(K, oracle_mod, seed):
    rs = synth.Stream(seed, 83)
    n = int(rs.integers(30, 600)[0])
    g = synth.chung_lu(n, int(rs.integers(2 * n, 8 * n)[0]), 2.3, seed=seed, planted=int(rs.integers(5, 25)[0]))
    k = int(rs.integers(3, 7)[0])
    T = int(rs.integers(1, 120)[0])
    print(f"bound seed={seed} n={n} k={k} T={T}", flush=True)
    sol = K.solve(g, k, T)
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, k, T)
    want = oracle_mod.top_bound(ref["r"], None, T, k)
    assert sol.bound_kind == 1
    assert Fraction(sol.bound_num, sol.bound_den) == want
    assert sol.certified == oracle_mod.certified(ref["dens_num"], ref["size"], want, g.n)


@pytest.mark.parametrize("k,T", [(2, 5), (3, 2)])
def test_top_bound_long_prefix(K, oracle_mod, k, T):
    """A dense graph: the bound's prefix (up to the first s with C(s, k) >= c_k,
    about 2,100 nodes at k = 2) spans several chunks of the bound kernel."""
    g = synth.erdos_renyi(3000, 0.5 if k == 2 else 0.1, seed=31)
    print(f"long prefix k={k} T={T} m={g.m}", flush=True)
    sol = K.solve(g, k, T)
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, k, T)
    want = oracle_mod.top_bound(ref["r"], None, T, k)
    s0 = next(s for s in range(g.n + 1) if math.comb(s, k) >= ref["c_k"])
    assert k > 2 or s0 > 2048
    assert Fraction(sol.bound_num, sol.bound_den) == want


def test_top_bound_without_cliques(K, oracle_mod):
    g = synth.erdos_renyi(200, 0.02, seed=3)
    sol = K.solve(g, 7, 4)
    assert sol.c_k == 0 and sol.bound_kind == 1 and sol.bound_num == 0


def test_complete_graph_is_certified(K, oracle_mod):
    g = synth.complete_graph(40)
    sol = K.solve(g, 4, 3)
    assert Fraction(sol.bound_num, sol.bound_den) == Fraction(math.comb(40, 4), 40)
    assert sol.certified and (sol.dens_num, sol.size) == (math.comb(40, 4), 40)


def test_planted_clique_certified_after_enough_iterations(K, oracle_mod):
    g = synth.erdos_renyi(300, 0.03, seed=5, planted_clique=20)
    sol = K.solve(g, 4, 400)
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, 4, 400)
    want = oracle_mod.top_bound(ref["r"], None, 400, 4)
    assert Fraction(sol.bound_num, sol.bound_den) == want
    assert sol.certified == oracle_mod.certified(ref["dens_num"], ref["size"], want, g.n)


def test_plain_bound_where_top_bound_does_not_apply(K):
    g = synth.chung_lu(500, 4000, 2.3, seed=9, planted=15)
    r0 = (synth.Stream(9, 84).u64(g.n) % np.uint64(6)).astype(np.uint64)
    for kw in (dict(r0=r0), dict(update=1)):
        sol = K.solve(g, 4, 10, **kw)
        assert sol.bound_kind == 0
        assert Fraction(sol.bound_num, sol.bound_den) == Fraction(sol.ub_num, 10)
        if kw.get("update"):
            assert not sol.certified   # PBUpdate loads need not bound rho*
