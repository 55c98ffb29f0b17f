"""Plant plausible slips in a copy of the oracle and check that a pin catches each.

This is evidence that the pins in test_oracle_pins.py constrain the oracle: a
mutated oracle (tie rule, sort direction, argmax tie rule, prefix index,
per-thread reduction, credits that ignore the loads, exclusive prefix counts)
must fail at least one of them.  Mutations are made on
the CPU, in a temporary copy of the source.
"""
from __future__ import annotations

import math
import shutil
from fractions import Fraction

import numpy as np
import pytest

from paper_2403_05775_amd import synth
from tests import _brute as B
from tests.test_oracle_pins import example_graph

MUTATIONS = {
    "highest id wins ties": ("if (r[c[i]] < r[best]) best = c[i];", "if (r[c[i]] <= r[best]) best = c[i];"),
    "ascending load order": ("return g_sort_r[x] > g_sort_r[y] ? -1 : 1;", "return g_sort_r[x] > g_sort_r[y] ? 1 : -1;"),
    "shortest best prefix": ("(u128)K * best_i >= (u128)bestK * i", "(u128)K * best_i > (u128)bestK * i"),
    "prefix by first node": ("if (p->pos[c[i]] > last) last = p->pos[c[i]];", "if (p->pos[c[i]] < last) last = p->pos[c[i]];"),
    "one thread's credits": ("for (int t = 0; t < R.nthreads; ++t) r[u] += delta_t[t][u];", "r[u] += delta_t[0][u];"),
    "credit the maximum": ("if (r[c[i]] < r[best]) best = c[i];", "if (r[c[i]] > r[best]) best = c[i];"),
    "credits ignore the loads": ("for (uint32_t u = 0; u < n; ++u) { rr[u] = r[u]; d_out[u] = 0; }",
                                 "for (uint32_t u = 0; u < n; ++u) { rr[u] = 0; d_out[u] = 0; }"),
    "exclusive prefix counts": ("for (int t = 0; t < R->nthreads; ++t) K += hist_t[t][i - 1];\n"
                                "        if (K_out) K_out[i - 1] = K;",
                                "if (K_out) K_out[i - 1] = K;\n"
                                "        for (int t = 0; t < R->nthreads; ++t) K += hist_t[t][i - 1];"),
}


def _pins(O, path):
    """A compact run of the pins: raises AssertionError if any fails."""
    g, _, vals = example_graph()
    cl = B.cliques(g, 3)
    # Example 1 printed optimum
    res = O.solve(g.n, g.row_ptr, g.col, 3, 64, libpath=path)
    assert Fraction(res["dens_num"], res["size"]) == Fraction(*vals["densest_density"])
    # first iteration from r = 0: lowest id of each clique
    r1 = O.solve(g.n, g.row_ptr, g.col, 3, 1, libpath=path)["r"]
    assert r1.tolist() == [sum(1 for c in cl if min(c) == u) for u in range(g.n)]
    # K_n closed form
    kn = synth.complete_graph(9)
    assert O.solve(kn.n, kn.row_ptr, kn.col, 3, 1, libpath=path)["r"].tolist() == \
        [math.comb(8 - i, 2) for i in range(9)]
    # equal-density tie: the longest prefix
    e = [(i, j) for i in range(4) for j in range(i + 1, 4)]
    e += [(4 + i, 4 + j) for i in range(4) for j in range(i + 1, 4)]
    g2 = synth.from_edge_list(8, e)
    r0 = np.array([10, 10, 10, 10, 0, 0, 0, 0], dtype=np.uint64)
    assert O.solve(g2.n, g2.row_ptr, g2.col, 3, 1, r0=r0, libpath=path)["size"] == 8
    # Lemma 6 with several threads
    g3 = synth.chung_lu(400, 3000, 2.3, seed=1)
    ck = O.count(g3.n, g3.row_ptr, g3.col, 3, libpath=path)
    r = O.solve(g3.n, g3.row_ptr, g3.col, 3, 3, threads=4, libpath=path)["r"]
    assert int(np.sum(r.astype(object))) == 3 * ck
    # brute-force Frank-Wolfe on a tiny graph
    g4 = synth.erdos_renyi(10, 0.55, seed=3)
    cl4 = B.cliques(g4, 3)
    rb = B.frank_wolfe(10, cl4, 4)
    res4 = O.solve(g4.n, g4.row_ptr, g4.col, 3, 4, libpath=path)
    assert res4["r"].tolist() == rb
    _, i_star, K = B.best_prefix(10, cl4, rb)
    assert (res4["size"], res4["dens_num"]) == (i_star, K)
    # one credit pass at tied, non-zero loads
    r5 = [5, 0, 3, 1, 2, 0, 4]
    d5 = O.credits(g.n, g.row_ptr, g.col, 3, np.array(r5, dtype=np.uint64), libpath=path)
    assert d5.tolist() == [a - b for a, b in zip(B.frank_wolfe(g.n, cl, 1, r5), r5)]
    # every prefix count at those loads
    order5 = sorted(range(g.n), key=lambda v: (-r5[v], v))
    K5 = [sum(1 for c in cl if set(c) <= set(order5[:i])) for i in range(1, g.n + 1)]
    assert O.prefix_counts(g.n, g.row_ptr, g.col, 3, np.array(r5, dtype=np.uint64), libpath=path)["K"].tolist() == K5


def test_unmutated_oracle_passes(oracle_mod):
    _pins(oracle_mod, None)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(oracle_mod, tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(oracle_mod.SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {old}"
    msrc = tmp_path / "kdss_oracle_mut.c"
    msrc.write_text(src.replace(old, new))
    out = str(tmp_path / f"libmut_{abs(hash(name))}.so")
    oracle_mod.build(force=True, src=str(msrc), out=out)
    with pytest.raises(AssertionError):
        _pins(oracle_mod, out)
