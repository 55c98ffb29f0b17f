"""Parity at the benchmarked sizes, in the launch configurations bench.py times.

* Chung-Lu n = 1,000,000, m = 10,000,000, k = 5, T = 200: the oracle runs the
  whole problem (its clique listing fits in memory), so loads, order, density,
  upper bound and every prefix count K_i are compared bit for bit.
* The 2048-problem batch (512 Chung-Lu graphs x k in {3, 4, 6, 8}, T = 64, one
  plan, the bench's tuned launch): every problem equals its solo run, and the
  oracle on every problem with at most 2e5 k-cliques (about 750).
* The warm-start evaluation graph (n = 2,000,000, m = 40,000,000, k = 6) and
  R-MAT scale 16 (k = 6): too many cliques for the oracle's listing, so
  properties that hold at any size are checked: Lemma 6 (the loads grow by
  exactly T c_k), the order is the sort of the loads (descending, ties by
  ascending id), and density <= upper bound; and one credit pass at seeded,
  tied loads is compared on sampled nodes with a per-node count (the
  (k - 1)-cliques among the neighbours above the node, by the oracle's
  counter); the same sampled pass on R-MAT scale 18.  R-MAT scale 12 is
  compared with the oracle bit for bit at both load widths.
"""
from __future__ import annotations

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


def say(msg):
    print(msg, flush=True)


_graphs = {}


def warm_start_graph():
    """The 2M / 40M evaluation graph, generated once for the module's tests."""
    if "2m" not in _graphs:
        _graphs["2m"] = synth.chung_lu(2_000_000, 40_000_000, 2.5, seed=90000)
    return _graphs["2m"]


def loads(x):
    return [int(v) for v in (x if isinstance(x, list) else x.tolist())]


def assert_properties(g, sol, T, r0=None):
    """Lemma 6, order = sort of the loads, density <= upper bound (64-bit loads)."""
    assert not isinstance(sol.r, list)
    r = sol.r.astype(np.uint64)
    base = np.zeros(g.n, dtype=np.uint64) if r0 is None else np.asarray(r0, dtype=np.uint64)
    assert np.all(r >= base)
    grow = r - base
    assert int(grow.astype(object).sum()) == T * sol.c_k          # Lemma 6
    order = sol.order.astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(g.n))
    ro = r[order]
    assert np.all(ro[:-1] >= ro[1:])                               # loads non-increasing
    tie = ro[:-1] == ro[1:]
    assert np.all(order[:-1][tie] < order[1:][tie])                # ties by ascending id
    assert sol.ub_num == int(grow.max())
    assert sol.dens_num * T <= sol.ub_num * max(sol.size, 1)        # density <= upper bound


def test_chung_lu_1m_bit_exact(K, oracle_mod):
    say("chung-lu 1M k=5 T=200: generating")
    g = synth.chung_lu(1_000_000, 10_000_000, 2.5, seed=0, planted=40, planted_p=0.9)
    say("chung-lu 1M k=5 T=200: GPU")
    sol = K.solve(g, 5, 200)
    say("chung-lu 1M k=5 T=200: oracle")
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, 5, 200)
    assert loads(sol.r) == loads(ref["r"])
    assert np.array_equal(sol.order, ref["order"])
    assert (sol.size, sol.dens_num, sol.ub_num, sol.c_k) == (ref["size"], ref["dens_num"], ref["ub_num"],
                                                            ref["c_k"])
    say("chung-lu 1M k=5 T=200: GPU, heavy leaves in place")
    sol2 = K.solve(g, 5, 200, heavy=2)
    assert loads(sol2.r) == loads(ref["r"]) and np.array_equal(sol2.order, ref["order"])
    assert (sol2.size, sol2.dens_num, sol2.ub_num) == (ref["size"], ref["dens_num"], ref["ub_num"])
    say("chung-lu 1M: certified bound")
    want = oracle_mod.top_bound(ref["r"], None, 200, 5)
    from fractions import Fraction
    assert sol.bound_kind == 1 and Fraction(sol.bound_num, sol.bound_den) == want
    assert sol.certified == oracle_mod.certified(ref["dens_num"], ref["size"], want, g.n)
    say("chung-lu 1M: every prefix count K_i at r_200")
    tree = K.Tree(g, 5)
    plan = K.Plan(tree, 200)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    rt = torch.from_numpy(np.asarray(ref["r"], dtype=np.uint64).view(np.int64).copy()).cuda()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    cnt = torch.empty(g.n, dtype=torch.int64, device="cuda")
    plan.extract_counts(ws, rt, order, cnt, 200)
    torch.cuda.synchronize()
    want_k = oracle_mod.prefix_counts(g.n, g.row_ptr, g.col, 5, ref["r"])
    assert np.array_equal(order.cpu().numpy().view(np.uint32), want_k["order"])
    assert np.array_equal(cnt.cpu().numpy().view(np.uint64), want_k["K"])
    assert int(want_k["K"][-1]) == ref["c_k"]
    plan.close()
    tree.close()


def test_batch_512_every_problem(K, oracle_mod):
    """The full batch in the bench's launch (tuning cache), every one of its
    2048 problems against its own solo run (loads, order, i*, K_{i*}, upper
    bound), and against the oracle on every problem with at most 2e5 k-cliques
    (about 750 problems; the oracle finishes each in a fraction of a second)."""
    from paper_2403_05775_amd import gnn
    say("batch 512 x 4: generating")
    graphs = gnn.generate(512, base_seed=1000, n_lo=1000, n_hi=50000, workers=16, log=lambda *_: None)
    jobs = [(g, k) for g in graphs for k in (3, 4, 6, 8)]
    trees = [K.Tree(g, k) for g, k in jobs]
    T = 64
    say("batch 512 x 4: plan and run")
    b = K.Batch(trees, T)
    ws = b.alloc_workspace()
    b.upload(ws)
    r = torch.empty(b.n, dtype=torch.int64, device="cuda")
    order = torch.empty(b.n, dtype=torch.int32, device="cuda")
    b.autotune_cached(ws, r, warm=T // 2, iters=5)
    res = b.run(ws, T, r, order)
    torch.cuda.synchronize()
    rr = r.cpu().numpy().view(np.uint64)
    oo = order.cpu().numpy().view(np.uint32)
    off = b.node_off.astype(np.int64)
    del ws
    b.close()
    torch.cuda.empty_cache()
    ck = [t.stats().c_k.value for t in trees]
    checked = 0
    for q, (g, k) in enumerate(jobs):
        if q % 256 == 0:
            say(f"batch problem {q}: solo runs")
        plan = K.Plan(trees[q], T)
        pws = plan.alloc_workspace()
        plan.upload(pws)
        pr = plan.alloc_loads()
        po = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
        sres, _ = plan.run(pws, T, pr, po)
        torch.cuda.synchronize()
        assert np.array_equal(rr[off[q]:off[q + 1]], pr.cpu().numpy().view(np.uint64)[: g.n]), q
        assert np.array_equal(oo[off[q]:off[q + 1]], po.cpu().numpy().view(np.uint32)[: g.n]), q
        assert (res[q].size, res[q].dens_num.value, res[q].ub_num.value) == \
            (sres.size, sres.dens_num.value, sres.ub_num.value), q
        plan.close()
        if 0 < ck[q] <= 200_000:
            ref = oracle_mod.solve(g.n, g.row_ptr, g.col, k, T, threads=16)
            assert rr[off[q]:off[q + 1]].tolist() == loads(ref["r"]), q
            assert (res[q].size, res[q].dens_num.value, res[q].ub_num.value) == \
                (ref["size"], ref["dens_num"], ref["ub_num"]), q
            checked += 1
    say(f"batch: {len(jobs)} problems equal their solo runs; {checked} also equal the oracle")
    assert checked >= 500
    for t in trees:
        t.close()


def _local_credit(oracle_mod, g, k, r, u):
    """The k-cliques whose minimum (load, id) member is u, counted one node at a
    time: the (k - 1)-cliques among u's neighbours w with (r[w], w) > (r[u], u),
    by the oracle's own counter on that induced subgraph."""
    nb = g.col[g.row_ptr[u]:g.row_ptr[u + 1]].astype(np.int64)
    sel = nb[(r[nb] > r[u]) | ((r[nb] == r[u]) & (nb > u))]
    if k == 2:
        return len(sel)
    mark = np.full(g.n, -1, dtype=np.int64)
    mark[sel] = np.arange(len(sel))
    edges = []
    for i, w in enumerate(sel):
        j = mark[g.col[g.row_ptr[w]:g.row_ptr[w + 1]]]
        j = j[j > i]
        edges.extend((i, int(x)) for x in j)
    sub = synth.from_edge_list(len(sel), edges)
    return oracle_mod.count(sub.n, sub.row_ptr, sub.col, k - 1) if sub.n else 0


def _sampled_credits(K, oracle_mod, g, k, seed, samples=48, max_degree=400, heavy_modes=(1,)):
    """One credit pass on the GPU at seeded loads with many ties, compared on
    sampled nodes (degree at most max_degree, so each count stays small) with
    the per-node count, and the total with c_k (every clique credits exactly
    one member); once per heavy-leaf mode (1 queue, 2 in place), the two
    passes equal node for node."""
    tree = K.Tree(g, k)
    rs = synth.Stream(seed, 83)
    r = (rs.u64(g.n) % np.uint64(4)).astype(np.uint64)
    deg = np.diff(g.row_ptr.astype(np.int64))
    cand = np.nonzero((deg > 0) & (deg <= max_degree))[0]
    picks = cand[(rs.u64(samples) % np.uint64(len(cand))).astype(np.int64)]
    big = cand[np.argsort(deg[cand])[-4:]]   # and the four largest neighbourhoods allowed
    want = {int(u): _local_credit(oracle_mod, g, k, r, int(u)) for u in np.concatenate([picks, big])}
    first = None
    for heavy in heavy_modes:
        say(f"  credit pass, heavy-leaf mode {heavy}")
        plan = K.Plan(tree, 1, heavy=heavy)
        ws = plan.alloc_workspace()
        plan.upload(ws)
        rt = torch.from_numpy(r.view(np.int64).copy()).cuda()
        out = torch.empty(g.n, dtype=torch.int64, device="cuda")
        plan.leaf_credit(ws, rt, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint64)
        del ws, rt, out
        plan.close()
        assert int(got.astype(object).sum()) == tree.stats().c_k.value
        for u, c in want.items():
            assert int(got[u]) == c, (heavy, u)
        if first is None:
            first = got
        else:
            assert np.array_equal(got, first)
    tree.close()


def test_warm_start_graph_sampled_credits(K, oracle_mod):
    """The 2M / 40M graph at k = 6 (2.1e10 cliques, too many for the oracle's
    listing): one credit pass at tied loads, sampled node by node."""
    say("chung-lu 2M m=40M k=6: sampled credits")
    g = warm_start_graph()
    _sampled_credits(K, oracle_mod, g, 6, seed=5)


def test_rmat_16_sampled_credits(K, oracle_mod):
    say("rmat 16 k=6: sampled credits")
    _sampled_credits(K, oracle_mod, synth.rmat(16, 8, seed=0), 6, seed=6, max_degree=200, heavy_modes=(1, 2))


def test_rmat_18_sampled_credits(K, oracle_mod):
    """R-MAT scale 18 at k = 6, the largest R-MAT graph one GPU holds (8.3e8
    leaves, a 41 GB leaf stream): one credit pass, sampled node by node."""
    say("rmat 18 k=6: sampled credits (tree build about a minute)")
    _sampled_credits(K, oracle_mod, synth.rmat(18, 8, seed=0), 6, seed=7, samples=32, max_degree=150,
                     heavy_modes=(1, 2))


def test_warm_start_graph_properties(K):
    from paper_2403_05775_amd import gnn
    say("chung-lu 2M m=40M k=6: generating")
    g = warm_start_graph()
    tree = K.Tree(g, 6)
    dev = torch.device("cuda:0")
    dg = gnn.DeviceGraph(g, tree, dev)
    model = gnn.Model(device=dev)
    import os
    if os.path.exists(gnn.WEIGHTS_FILE):
        with np.load(gnn.WEIGHTS_FILE) as z:
            model.load(z)
    r0, rmax = model.warm_start(dg, 50)
    r0h = r0.cpu().numpy().view(np.uint64)
    assert rmax == int(r0h.max())
    tree.close()
    for T, start in ((3, None), (3, r0h)):
        say(f"chung-lu 2M k=6 T={T} {'warm' if start is not None else 'cold'}: GPU")
        sol = K.solve(g, 6, T, r0=start)
        assert_properties(g, sol, T, start)


@pytest.mark.parametrize("width", [0, 128])
def test_rmat_12_bit_exact(K, oracle_mod, width):
    g = synth.rmat(12, 8, seed=0)
    say(f"rmat 12 k=6 T=100 width={width}")
    sol = K.solve(g, 6, 100, width=width)
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, 6, 100)
    assert loads(sol.r) == loads(ref["r"])
    assert np.array_equal(sol.order, ref["order"])
    assert (sol.size, sol.dens_num, sol.ub_num) == (ref["size"], ref["dens_num"], ref["ub_num"])


def test_rmat_16_properties(K):
    """The run's invariants, and the same run with heavy leaves in place (the
    tuned launch for this graph) equal to it bit for bit."""
    g = synth.rmat(16, 8, seed=0)
    say("rmat 16 k=6 T=100")
    sol = K.solve(g, 6, 100)
    assert_properties(g, sol, 100)
    say("rmat 16 k=6 T=100, heavy leaves in place")
    sol2 = K.solve(g, 6, 100, heavy=2)
    assert np.array_equal(sol2.r, sol.r) and np.array_equal(sol2.order, sol.order)
    assert (sol2.size, sol2.dens_num, sol2.ub_num) == (sol.size, sol.dens_num, sol.ub_num)
