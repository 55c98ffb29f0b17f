"""Batches: many (graph, k) problems in one launch per iteration; each problem's
result must equal its solo run and the oracle bit for bit."""
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


def _problems(count, seed0):
    probs = []
    for i in range(count):
        rs = synth.Stream(seed0 + i, 91)
        n = int(rs.integers(40, 900)[0])
        m = int(rs.integers(2 * n, 7 * n)[0])
        g = synth.chung_lu(n, m, 2.1 + 0.7 * float(rs.uniform(1)[0]), seed=seed0 + i,
                           planted=int(rs.integers(0, 25)[0]))
        k = [3, 4, 6, 8, 2, 5][i % 6]
        probs.append((g, k))
    return probs


def run_batch(K, probs, T, r0s=None, use_graph=False, tune=False, gather=0):
    trees = [K.Tree(g, k) for g, k in probs]
    r0_max = 0 if r0s is None else int(max(int(np.max(x)) if x.size else 0 for x in r0s))
    b = K.Batch(trees, T, r0_max=r0_max, use_graph=use_graph, gather=gather)
    if gather:
        assert b.stats().gather == gather
    ws = b.alloc_workspace()
    b.upload(ws)
    r = torch.empty(b.n, dtype=torch.int64, device="cuda")
    order = torch.empty(b.n, dtype=torch.int32, device="cuda")
    r0 = None
    if r0s is not None:
        r0 = torch.from_numpy(np.concatenate(r0s).astype(np.uint64).view(np.int64)).cuda()
    if tune:
        tr = b.autotune(ws, r, warm=2, iters=2)
        assert tr.tried >= 4 and tr.best_ms > 0
    res = b.run(ws, T, r, order, r0=r0)
    torch.cuda.synchronize()
    rr = r.cpu().numpy().view(np.uint64)
    oo = order.cpu().numpy().view(np.uint32)
    off = b.node_off.astype(np.int64)
    out = []
    for q in range(len(probs)):
        out.append(dict(r=rr[off[q]:off[q + 1]], order=oo[off[q]:off[q + 1]], size=res[q].size,
                        dens_num=res[q].dens_num.value, ub_num=res[q].ub_num.value, c_k=res[q].c_k.value))
    return out


def same(a, ref):
    assert np.array_equal(a["r"], ref["r"])
    assert np.array_equal(a["order"], ref["order"])
    assert (a["size"], a["dens_num"], a["ub_num"], a["c_k"]) == (ref["size"], ref["dens_num"], ref["ub_num"],
                                                                   ref["c_k"])


@pytest.mark.parametrize("gather", [1, 2])
def test_batch_matches_oracle(K, oracle_mod, gather):
    probs = _problems(18, 300)
    print(f"batch of 18 problems, T=15, gather mode {gather}", flush=True)
    out = run_batch(K, probs, 15, gather=gather)
    for (g, k), got in zip(probs, out):
        same(got, oracle_mod.solve(g.n, g.row_ptr, g.col, k, 15))


def test_batch_warm_start_and_graph(K, oracle_mod):
    probs = _problems(9, 700)
    r0s = [(synth.Stream(i, 93).u64(g.n) % np.uint64(7)).astype(np.uint64) for i, (g, k) in enumerate(probs)]
    print("batch of 9 problems with warm starts, graph replay, T=11", flush=True)
    out = run_batch(K, probs, 11, r0s=r0s, use_graph=True)
    for (g, k), r0, got in zip(probs, r0s, out):
        same(got, oracle_mod.solve(g.n, g.row_ptr, g.col, k, 11, r0=r0))


def test_batch_equals_solo_after_autotune(K):
    probs = _problems(6, 900) + [(synth.chung_lu(20000, 150000, 2.3, seed=5, planted=30), 5)]
    print("batch vs solo after autotune, T=20", flush=True)
    out = run_batch(K, probs, 20, tune=True)
    for (g, k), got in zip(probs, out):
        sol = K.solve(g, k, 20)
        same(got, dict(r=sol.r, order=sol.order, size=sol.size, dens_num=sol.dens_num, ub_num=sol.ub_num,
                       c_k=sol.c_k))


def test_batch_with_degenerate_members(K, oracle_mod):
    """Members with no edges, a single node, k above the clique number and a
    complete graph, between ordinary ones: each equals its own oracle run."""
    probs = [(synth.from_edge_list(20, []), 3), (synth.chung_lu(300, 1500, 2.3, seed=71, planted=12), 4),
             (synth.from_edge_list(1, []), 2), (synth.complete_graph(7), 8), (synth.complete_graph(15), 5),
             (synth.chung_lu(500, 2500, 2.4, seed=72), 3)]
    print("batch with degenerate members, T=6", flush=True)
    out = run_batch(K, probs, 6)
    for (g, k), got in zip(probs, out):
        same(got, oracle_mod.solve(g.n, g.row_ptr, g.col, k, 6))
