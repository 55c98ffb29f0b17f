"""PBUpdate (the paper's per-pair update, Algorithm 3), synchronous variant:
the HIP path through the C-ABI against the CPU oracle's synchronous pass over
the same pairs (the tree's leaves, exported), bit for bit: loads, then the
extraction on those loads (order, i*, K_{i*})."""
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


def oracle_pb(O, K, g, k, T, r0=None):
    tree = K.Tree(g, k)
    h, p, mem = tree.export()
    tree.close()
    r = O.pb_run(g.n, h, p, mem, k, T, True, r0=r0)["r"]
    ex = O.extract(g.n, g.row_ptr, g.col, k, r)
    return r, ex


def check(K, O, g, k, T, r0=None, label="", **kw):
    print(f"PBUpdate {label} n={g.n} k={k} T={T}", flush=True)
    sol = K.solve(g, k, T, r0=r0, update=1, **kw)
    assert sol.plan_stats.update == 1
    r, ex = oracle_pb(O, K, g, k, T, r0)
    assert np.array_equal(sol.r, r), label
    assert np.array_equal(sol.order, ex["order"]), label
    assert (sol.size, sol.dens_num) == (ex["size"], ex["dens_num"]), label
    base = np.zeros(g.n, dtype=np.uint64) if r0 is None else np.asarray(r0, dtype=np.uint64)
    assert int((sol.r - base).astype(object).sum()) == T * sol.c_k   # every pair allocates all its cliques
    return sol


@pytest.mark.parametrize("seed", range(6))
def test_pb_random_graphs(K, oracle_mod, seed):
    rs = synth.Stream(seed, 81)
    n = int(rs.integers(40, 500)[0])
    m = int(rs.integers(n, 6 * n)[0])
    g = synth.chung_lu(n, m, 2.1 + 0.8 * float(rs.uniform(1)[0]), seed=seed, planted=int(rs.integers(0, 20)[0]))
    k = int(rs.integers(3, 8)[0])
    T = int(rs.integers(1, 30)[0])
    r0 = (rs.u64(n) % np.uint64(5)).astype(np.uint64) if seed % 2 else None
    check(K, oracle_mod, g, k, T, r0, f"seed={seed}")


@pytest.mark.parametrize("k,planted", [(3, 70), (5, 30), (6, 70)])
def test_pb_size_classes(K, oracle_mod, k, planted):
    """Lane tiles of every size and, with a planted 70-clique, leaves of more
    than 64 members (one per wavefront)."""
    g = synth.erdos_renyi(260, 0.12, seed=7, planted_clique=planted)
    sol = check(K, oracle_mod, g, k, 7, None, f"size classes planted={planted}")
    if planted > 64:
        assert sol.plan_stats.leaves[4] > 0


def test_pb_example_graph(K, oracle_mod):
    from tests.test_oracle_pins import example_graph
    g, _, vals = example_graph()
    sol = check(K, oracle_mod, g, 3, 40, None, "example graph")
    assert (sol.dens_num, sol.size) == (8, 6)   # Example 1: {u1..u6}, density 4/3


def test_pb_graph_replay_and_batch(K, oracle_mod):
    g = synth.chung_lu(3000, 20000, 2.3, seed=11, planted=25)
    a = K.solve(g, 4, 12, update=1, use_graph=True)
    r, ex = oracle_pb(oracle_mod, K, g, 4, 12)
    assert np.array_equal(a.r, r) and (a.size, a.dens_num) == (ex["size"], ex["dens_num"])
    # a batch of problems, each equal to its solo run
    probs = [(synth.chung_lu(300 + 40 * i, 2500 + 200 * i, 2.3, seed=40 + i, planted=10), 3 + i % 4) for i in range(5)]
    trees = [K.Tree(pg, pk) for pg, pk in probs]
    b = K.Batch(trees, 9, update=1)
    assert b.stats().update == 1
    ws = b.alloc_workspace()
    b.upload(ws)
    rr = torch.empty(b.n, dtype=torch.int64, device="cuda")
    order = torch.empty(b.n, dtype=torch.int32, device="cuda")
    res = b.run(ws, 9, rr, order)
    torch.cuda.synchronize()
    rh = rr.cpu().numpy().view(np.uint64)
    off = b.node_off.astype(np.int64)
    for q, (pg, pk) in enumerate(probs):
        ro, exo = oracle_pb(oracle_mod, K, pg, pk, 9)
        assert np.array_equal(rh[off[q]:off[q + 1]], ro), q
        assert (res[q].size, res[q].dens_num.value) == (exo["size"], exo["dens_num"]), q
    for t in trees:
        t.close()


def test_pb_chung_lu_1m_sampled(K, oracle_mod):
    """The benchmarked graph (n = 1,000,000, m = 10,000,000, k = 5) in the bench's
    launch configuration, 8 iterations, loads compared with the oracle in full."""
    g = synth.chung_lu(1_000_000, 10_000_000, 2.5, seed=0, planted=40, planted_p=0.9)
    tree = K.Tree(g, 5)
    h, p, mem = tree.export()
    plan = K.Plan(tree, 8, update=1)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    plan.autotune(ws, r, warm=2, iters=2)
    res, _ = plan.run(ws, 8, r, order)
    torch.cuda.synchronize()
    got = r.cpu().numpy().view(np.uint64)
    print("chung-lu 1M PBUpdate: oracle", flush=True)
    want = oracle_mod.pb_run(g.n, h, p, mem, 5, 8, True)["r"]
    assert np.array_equal(got, want)
    assert int(got.astype(object).sum()) == 8 * tree.stats().c_k.value
    tree.close()


@pytest.mark.parametrize("case", ["no_cliques", "k2_one_iteration", "complete_k4_ties", "star_k2_r0"])
def test_pb_edge_cases(K, oracle_mod, case):
    """No k-cliques, k = 2 with a single iteration, a complete graph (every
    load tied: the remainder rule decides), a star with start loads."""
    r0 = None
    if case == "no_cliques":
        g, k, T = synth.erdos_renyi(200, 0.02, seed=4), 6, 5
    elif case == "k2_one_iteration":
        g, k, T = synth.chung_lu(500, 3000, 2.3, seed=6), 2, 1
    elif case == "complete_k4_ties":
        g, k, T = synth.complete_graph(12), 4, 7
    else:
        g, k, T = synth.from_edge_list(30, [(0, i) for i in range(1, 30)]), 2, 6
        r0 = (synth.Stream(7, 89).u64(g.n) % np.uint64(5)).astype(np.uint64)
    sol = check(K, oracle_mod, g, k, T, r0=r0, label=case)
    if case == "no_cliques":
        assert sol.c_k == 0 and sol.size == 0
