"""Pins of the oracle's PBUpdate (the paper's per-pair update, Algorithm 3).

* Example 3 of the paper: the first two pair updates from zero loads.
* Brute force: a unit-by-unit water fill (each of the pair's C(p, k - h)
  cliques goes to the node of lowest (current load, id) that is still below
  its cap) gives the same allocation as the algorithm's plateau steps.
* Invariants: a pair allocates exactly its C(p, k - h) cliques and no node more
  than its cap; the synchronous pass does not depend on the pair order; both
  passes add T * sum_q C(p_q, k - h_q) to the loads.
Mutations of the oracle source (remainder to the highest ids, pivot caps
C(p, j), no gap limit, a synchronous pass that reads updated loads) must each
fail one of them.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

from paper_2403_05775_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pbupdate_example3.txt")


def read_steps():
    steps = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        key, _, rest = line.partition(" ")
        assert key == "step"
        h, p, g = (part.split() for part in rest.split(";"))
        steps.append(([int(x) for x in h], [int(x) for x in p], sorted(int(x) for x in g)))
    return steps


def caps(h, p, k):
    j = k - len(h)
    return {**{u: math.comb(len(p), j) for u in h}, **{u: math.comb(len(p) - 1, j - 1) if j else 0 for u in p}}


def unit_fill(h, p, k, r):
    """Brute force: the pair's cliques one at a time, each to the lowest
    (current load, id) node below its cap."""
    j = k - len(h)
    if j < 0 or j > len(p):
        return {}
    cap = caps(h, p, k)
    cur = {u: int(r[u]) for u in h + p}
    inc = {u: 0 for u in h + p}
    for _ in range(math.comb(len(p), j)):
        u = min((x for x in h + p if inc[x] < cap[x]), key=lambda x: (cur[x], x))
        cur[u] += 1
        inc[u] += 1
    return inc


def random_pair(rs, n, kmax=6):
    k = int(rs.integers(2, kmax + 1))
    h = int(rs.integers(1, k + 1))
    p = int(rs.integers(k - h, 9))   # h = k with p > 0: the pair holds H alone (Lemma 4)
    nodes = rs.permutation(n)[: h + p].tolist()
    return nodes[:h], nodes[h:], k


def _pb_pins(O, path):
    # Example 3
    r = np.zeros(7, dtype=np.uint64)
    for h, p, gain in read_steps():
        d = O.pb_pair(7, h + p, len(h), len(p), 3, r, libpath=path)
        assert sorted(np.flatnonzero(d).tolist()) == gain and set(d[gain].tolist()) == {1}
        r = r + d
    # a pair with h = k and p > 0 holds the one clique H (Lemma 4): the pivot
    # nodes are in none of its cliques, and H's least (load, id) node takes it
    d = O.pb_pair(5, [0, 1, 2, 3, 4], 3, 2, 3, np.array([2, 1, 1, 0, 0], dtype=np.uint64), libpath=path)
    assert d.tolist() == [0, 1, 0, 0, 0]
    # brute force on random tiny pairs, loads with many ties
    rs = np.random.default_rng(7)
    for _ in range(300):
        n = 12
        h, p, k = random_pair(rs, n)
        r = rs.integers(0, 4, n).astype(np.uint64) * np.uint64(rs.integers(1, 3))
        d = O.pb_pair(n, h + p, len(h), len(p), k, r, libpath=path)
        want = unit_fill(h, p, k, r)
        assert {u: int(d[u]) for u in h + p} == want, (h, p, k, r.tolist())
        assert int(d.sum()) == math.comb(len(p), k - len(h))
    # synchronous passes do not depend on the pair order; both add T * sum C(p, k - h)
    pairs = [random_pair(rs, 30, kmax=4) for _ in range(40)]
    for kk in (3, 4):
        ps = [(h, p) for h, p, k in pairs if len(h) <= kk <= len(h) + len(p)]
        hs = np.array([len(h) for h, _ in ps])
        pp = np.array([len(p) for _, p in ps])
        mem = np.array([u for h, p in ps for u in h + p], dtype=np.uint32)
        total = sum(math.comb(len(p), kk - len(h)) for h, p in ps)
        a = O.pb_run(30, hs, pp, mem, kk, 5, True, libpath=path)["r"]
        perm = rs.permutation(len(ps))
        mem2 = np.array([u for q in perm for u in ps[q][0] + ps[q][1]], dtype=np.uint32)
        b = O.pb_run(30, hs[perm], pp[perm], mem2, kk, 5, True, libpath=path)["r"]
        assert np.array_equal(a, b)
        assert int(a.astype(object).sum()) == 5 * total
        c = O.pb_run(30, hs, pp, mem, kk, 5, False, libpath=path)["r"]
        assert int(c.astype(object).sum()) == 5 * total


def test_pb_pins(oracle_mod):
    _pb_pins(oracle_mod, None)


def test_pb_sequential_reads_earlier_pairs(oracle_mod):
    """The paper's loop applies pairs one after another: on Example 3's two
    pairs the second sees the first (u4 is no longer lowest); the synchronous
    pass lets both read zero loads."""
    steps = read_steps()
    hs = np.array([len(h) for h, _, _ in steps])
    pp = np.array([len(p) for _, p, _ in steps])
    mem = np.array([u for h, p, _ in steps for u in h + p], dtype=np.uint32)
    seq = oracle_mod.pb_run(7, hs, pp, mem, 3, 1, False)["r"]
    syn = oracle_mod.pb_run(7, hs, pp, mem, 3, 1, True)["r"]
    assert seq.tolist() == [0, 0, 0, 1, 1, 1, 1]
    # synchronous: ({4}, {5, 6}) gives u4 one; ({3}, {4, 5, 6}) at zero loads: four
    # nodes tie, floor(3 / 4) = 0, so the three lowest ids u3, u4, u5 gain one
    assert syn.tolist() == [0, 0, 0, 1, 2, 1, 0]


def test_pb_on_tree_pairs_reaches_densest(oracle_mod):
    """On the example graph, sequential PBUpdate over Example 2's pairs orders
    the densest set {u1..u6} (Example 1) first after enough iterations."""
    from tests.test_oracle_pins import example_graph
    g, pairs, vals = example_graph()
    hs = np.array([len(h) for h, _ in pairs])
    pp = np.array([len(p) for _, p in pairs])
    mem = np.array([u for h, p in pairs for u in h + p], dtype=np.uint32)
    r = oracle_mod.pb_run(g.n, hs, pp, mem, 3, 60, False)["r"]
    ex = oracle_mod.extract(g.n, g.row_ptr, g.col, 3, r)
    assert (ex["dens_num"], ex["size"]) == (8, 6)
    assert sorted(ex["order"][: ex["size"]].tolist()) == vals["densest_set"]


PB_MUTATIONS = {
    "remainder to the highest ids": ("return x < y ? -1 : (x > y ? 1 : 0);\n}\n\n/* One pair",
                                     "return x < y ? 1 : (x > y ? -1 : 0);\n}\n\n/* One pair"),
    "pivot caps C(p, j)": ("binom_u128(p - 1, j - 1)", "binom_u128(p, j)"),
    "no gap limit": ("if (!inf_gap && gap < w) w = gap;", ""),
    "synchronous pass reads updated loads": ("err = pb_pair(mem + off[q], h[q], p[q], k, cur, nxt);",
                                             "err = pb_pair(mem + off[q], h[q], p[q], k, nxt, nxt);"),
}


@pytest.mark.parametrize("name", sorted(PB_MUTATIONS))
def test_pb_mutation_is_caught(oracle_mod, tmp_path, name):
    old, new = PB_MUTATIONS[name]
    src = open(oracle_mod.SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {old}"
    msrc = tmp_path / "kdss_oracle_mut.c"
    msrc.write_text(src.replace(old, new))
    out = str(tmp_path / f"libpbmut_{abs(hash(name))}.so")
    oracle_mod.build(force=True, src=str(msrc), out=out)
    with pytest.raises((AssertionError, RuntimeError)):
        _pb_pins(oracle_mod, out)
