"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Loads, order, node set, density and upper bound must be bit-exact: every count
is an integer and the synchronous update does not depend on leaf order."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2403_05775_amd import synth
from tests.test_oracle_pins import example_graph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_05775_amd import kdss
    kdss.lib()
    return kdss


def ref(O, g, k, T, r0=None, trace=False):
    return O.solve(g.n, g.row_ptr, g.col, k, T, r0=r0, trace=trace)


def assert_same(sol, res, T, label=""):
    r_gpu = sol.r if isinstance(sol.r, list) else sol.r.tolist()
    r_ref = res["r"] if isinstance(res["r"], list) else res["r"].tolist()
    assert [int(x) for x in r_gpu] == [int(x) for x in r_ref], f"loads differ {label}"
    assert sol.c_k == res["c_k"], label
    assert np.array_equal(sol.order, res["order"]), f"order differs {label}"
    assert (sol.size, sol.dens_num, sol.ub_num) == (res["size"], res["dens_num"], res["ub_num"]), label
    assert sol.T == T


def test_example_graph(K, oracle_mod):
    g, _, vals = example_graph()
    for T in (1, 2, 5, 64):
        print(f"example graph k=3 T={T}", flush=True)
        sol = K.solve(g, 3, T)
        assert_same(sol, ref(oracle_mod, g, 3, T), T, f"T={T}")
    sol = K.solve(g, 3, 64)
    assert sorted(sol.nodes.tolist()) == vals["densest_set"]


def test_er_planted_trace(K, oracle_mod):
    """ER G(200, 0.08) seed 0 + planted 12-clique, k = 3, T = 64, extraction after every iteration."""
    g = synth.erdos_renyi(200, 0.08, seed=0, planted_clique=12)
    print("er200 k=3 T=64 trace", flush=True)
    sol = K.solve(g, 3, 64, extract_every=1)
    res = ref(oracle_mod, g, 3, 64, trace=True)
    assert_same(sol, res, 64)
    assert len(sol.trace) == 64
    for a, b in zip(sol.trace, res["trace"]):
        assert (a["t"], a["size"], a["dens_num"], a["ub_num"]) == (b["t"], b["size"], b["dens_num"], b["ub_num"])
    # the planted 12-clique is the densest subgraph here: density C(12,3)/12 = 55/3
    assert sol.size == 12 and sol.dens_num == 220


@pytest.mark.parametrize("seed", range(10))
def test_random_graphs(K, oracle_mod, seed):
    rs = synth.Stream(seed, 61)
    n = int(rs.integers(30, 400)[0])
    m = int(rs.integers(n, 6 * n)[0])
    beta = 2.1 + 0.8 * float(rs.uniform(1)[0])
    planted = int(rs.integers(0, 20)[0])
    g = synth.chung_lu(n, m, beta, seed=seed, planted=planted)
    k = int(rs.integers(2, 8)[0])
    T = int(rs.integers(1, 40)[0])
    r0 = None
    if seed % 3 == 1:
        r0 = (rs.u64(n) % np.uint64(4)).astype(np.uint64)       # many ties
    elif seed % 3 == 2:
        r0 = (rs.u64(n) % np.uint64(1000)).astype(np.uint64)
    heavy = 1 + seed % 3   # heavy leaves queued, in place, or queued eight per batch
    print(f"random seed={seed} n={n} m={m} k={k} T={T} r0={'yes' if r0 is not None else 'no'} heavy={heavy}",
          flush=True)
    sol = K.solve(g, k, T, r0=r0, heavy=heavy)
    assert_same(sol, ref(oracle_mod, g, k, T, r0=r0), T, f"seed={seed}")


@pytest.mark.parametrize("k,planted", [(2, 70), (3, 70), (4, 70), (5, 30), (6, 30), (8, 30)])
def test_every_size_class(K, oracle_mod, k, planted):
    """Leaves of 2..64 members, and above 64 with a planted 70-clique (kept small
    enough for the oracle to list every k-clique)."""
    g = synth.erdos_renyi(260, 0.12, seed=7, planted_clique=planted)
    T = 6
    print(f"size classes k={k} planted={planted}", flush=True)
    want = ref(oracle_mod, g, k, T)
    for heavy in (1, 2, 3):
        sol = K.solve(g, k, T, heavy=heavy)
        if planted > 64:
            assert sol.plan_stats.leaves[4] > 0
        assert_same(sol, want, T, f"k={k} heavy={heavy}")


def test_graph_replay_and_determinism(K, oracle_mod):
    g = synth.chung_lu(3000, 20000, 2.3, seed=11, planted=25)
    print("graph replay k=4 T=30", flush=True)
    a = K.solve(g, 4, 30, use_graph=True)
    b = K.solve(g, 4, 30)
    c = K.solve(g, 4, 30)
    assert_same(a, ref(oracle_mod, g, 4, 30), 30)
    for x in (b, c):
        assert np.array_equal(a.r, x.r) and np.array_equal(a.order, x.order) and a.size == x.size


def test_full_keys_and_wide_loads(K, oracle_mod):
    """Start loads near 2^62 force full (load, id) keys; near 2^64 force 128-bit loads."""
    g = synth.chung_lu(600, 5000, 2.3, seed=12, planted=15)
    rs = synth.Stream(12, 71)
    base = np.uint64(2**62)
    r0 = base + (rs.u64(g.n) % np.uint64(3)).astype(np.uint64)
    print("full keys", flush=True)
    sol = K.solve(g, 4, 7, r0=r0)
    assert sol.plan_stats.key_mode == 1 and sol.width == 64
    assert_same(sol, ref(oracle_mod, g, 4, 7, r0=r0), 7)
    r0w = np.uint64(2**64 - 50) + (rs.u64(g.n) % np.uint64(5)).astype(np.uint64)
    print("wide loads", flush=True)
    sol = K.solve(g, 4, 7, r0=r0w)
    assert sol.width == 128
    res = ref(oracle_mod, g, 4, 7, r0=r0w)
    assert isinstance(res["r"], list)
    assert_same(sol, res, 7)
    print("forced width 128", flush=True)
    sol = K.solve(g, 3, 5, width=128)
    assert sol.width == 128
    assert_same(sol, ref(oracle_mod, g, 3, 5), 5)


@pytest.mark.parametrize("gather", [1, 2])
def test_gather_modes(K, oracle_mod, gather):
    """Both key-gather modes of the leaf pass (masked: non-hot members inside
    the leaf only; full: every row), with packed keys, (load, id) keys and
    128-bit loads, from cold and tied start loads."""
    g = synth.chung_lu(4000, 30000, 2.2, seed=21, planted=28)
    rs = synth.Stream(21, 72)
    ties = (rs.u64(g.n) % np.uint64(3)).astype(np.uint64)
    high = np.uint64(2**62) + (rs.u64(g.n) % np.uint64(3)).astype(np.uint64)
    for k, T, r0, width, key_mode in ((4, 25, None, 0, 0), (5, 9, ties, 0, 0), (4, 7, high, 0, 1),
                                      (3, 5, None, 128, 1)):
        print(f"gather {gather} k={k} T={T} width={width}", flush=True)
        sol = K.solve(g, k, T, r0=r0, width=width, gather=gather)
        assert sol.plan_stats.gather == gather and sol.plan_stats.key_mode == key_mode
        assert sol.plan_stats.hot_nodes > 0
        assert_same(sol, ref(oracle_mod, g, k, T, r0=r0), T, f"gather={gather} k={k}")


@pytest.mark.parametrize("gather", [1, 2])
def test_heavy_leaves_in_place(K, oracle_mod, gather):
    """Heavy leaves (more than four pivot members below the hold minimum) taken
    up in place by the tile's wavefront instead of the queue: packed keys,
    (load, id) keys and 128-bit loads (two leaves at a time), extraction
    included; the same graphs queue heavy leaves in the other mode, and in
    place none is queued and no heavy kernel runs."""
    g = synth.chung_lu(4000, 30000, 2.2, seed=21, planted=28)
    rs = synth.Stream(21, 73)
    ties = (rs.u64(g.n) % np.uint64(3)).astype(np.uint64)
    high = np.uint64(2**62) + (rs.u64(g.n) % np.uint64(3)).astype(np.uint64)
    for k, T, r0, width, key_mode in ((4, 25, None, 0, 0), (5, 9, ties, 0, 0), (4, 7, high, 0, 1),
                                      (6, 5, None, 128, 1)):
        print(f"heavy in place, gather {gather} k={k} T={T} width={width}", flush=True)
        sol = K.solve(g, k, T, r0=r0, width=width, gather=gather, heavy=2)
        assert sol.plan_stats.heavy == 2 and sol.plan_stats.key_mode == key_mode
        assert_same(sol, ref(oracle_mod, g, k, T, r0=r0), T, f"in place gather={gather} k={k}")
    tree = K.Tree(g, 5)
    counts = {}
    for heavy in (1, 2, 3):
        plan = K.Plan(tree, 9, time_kernels=True, gather=gather, heavy=heavy)
        ws = plan.alloc_workspace()
        plan.upload(ws)
        r = plan.alloc_loads()
        order = torch.empty(g.n, dtype=torch.int32, device="cuda")
        print(f"heavy mode {heavy}: timed run", flush=True)
        plan.run(ws, 9, r, order)
        torch.cuda.synchronize()
        tm = plan.timing()
        counts[heavy] = (tm.heavy_leaves, tm.heavy_ms)
        assert np.array_equal(r.cpu().numpy().view(np.uint64)[: g.n], ref(oracle_mod, g, 5, 9)["r"])
        plan.close()
    tree.close()
    assert counts[1][0] > 0 and counts[1][1] > 0
    assert counts[2] == (0, 0.0)
    assert counts[3][0] == counts[1][0] and counts[3][1] > 0   # the same queue, eight per batch


def test_heavy_in_place_credits_at_tied_loads(K, oracle_mod):
    """One credit pass with heavy leaves in place, at loads with many ties, and
    a batch of problems with different k: each equals the oracle."""
    from paper_2403_05775_amd import kdss
    g = synth.chung_lu(2000, 16000, 2.2, seed=13, planted=30)
    for k in (3, 5, 7):
        tree = kdss.Tree(g, k)
        plan = kdss.Plan(tree, 1, heavy=2)
        ws = plan.alloc_workspace()
        plan.upload(ws)
        for trial in range(2):
            rs = synth.Stream(200 + trial, 81)
            r = (rs.u64(g.n) % np.uint64(2 + 5 * trial)).astype(np.uint64)
            rt = torch.from_numpy(r.view(np.int64).copy()).cuda()
            out = torch.empty(g.n, dtype=torch.int64, device="cuda")
            print(f"in-place leaf credit k={k} trial={trial}", flush=True)
            plan.leaf_credit(ws, rt, out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint64), oracle_mod.credits(g.n, g.row_ptr, g.col, k, r))
        plan.close()
        tree.close()
    T = 6
    probs = [(synth.chung_lu(500 + 150 * i, 4000 + 900 * i, 2.2, seed=60 + i, planted=14 + i), 3 + i % 5)
             for i in range(6)]
    b = kdss.Batch([kdss.Tree(gq, kq) for gq, kq in probs], T, heavy=2)
    assert b.stats().heavy == 2
    wsb = b.alloc_workspace()
    b.upload(wsb)
    rb = torch.empty(b.n, dtype=torch.int64, device="cuda")
    ob = torch.empty(b.n, dtype=torch.int32, device="cuda")
    print("in-place heavy leaves, batch", flush=True)
    resb = b.run(wsb, T, rb, ob)
    torch.cuda.synchronize()
    rr = rb.cpu().numpy().view(np.uint64)
    oo = ob.cpu().numpy().view(np.uint32)
    for q, (gq, kq) in enumerate(probs):
        want = ref(oracle_mod, gq, kq, T)
        lo, hi = int(b.node_off[q]), int(b.node_off[q + 1])
        assert np.array_equal(rr[lo:hi], want["r"]), q
        assert np.array_equal(oo[lo:hi], want["order"]), q
        assert (resb[q].size, resb[q].dens_num.value, resb[q].ub_num.value) == \
            (want["size"], want["dens_num"], want["ub_num"]), q


@pytest.mark.parametrize("gather", [1, 2])
def test_binomial_table_in_memory(K, oracle_mod, gather):
    """A plan whose binomial table does not fit in LDS (s_max = 130 at k = 3:
    131 x 4 entries), so every pass reads it from memory.  The graph's lane
    tiles hold leaves with 1-4, 5-8 and more than 8 low members at the tied
    loads used (about 100 of each of the last two per trial); one credit pass
    per trial and heavy-leaf mode, and a run, equal the oracle."""
    from paper_2403_05775_amd import kdss
    g = synth.erdos_renyi(400, 0.08, seed=17, planted_clique=130)
    tree = kdss.Tree(g, 3)
    assert tree.stats().s_max == 130
    for heavy in (1, 2):
        plan = kdss.Plan(tree, 1, gather=gather, heavy=heavy)
        ws = plan.alloc_workspace()
        plan.upload(ws)
        for trial in range(2):
            rs = synth.Stream(300 + trial, 81)
            r = (rs.u64(g.n) % np.uint64(2 + 5 * trial)).astype(np.uint64)
            rt = torch.from_numpy(r.view(np.int64).copy()).cuda()
            out = torch.empty(g.n, dtype=torch.int64, device="cuda")
            print(f"binomials in memory: gather {gather} heavy {heavy} trial {trial}", flush=True)
            plan.leaf_credit(ws, rt, out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint64), oracle_mod.credits(g.n, g.row_ptr, g.col, 3, r))
        plan.close()
    tree.close()
    print(f"binomials in memory: gather {gather}, run T=12", flush=True)
    sol = K.solve(g, 3, 12, gather=gather)
    assert_same(sol, ref(oracle_mod, g, 3, 12), 12, f"binomials in memory, gather={gather}")


def test_leaf_credit_with_forced_ties(K, oracle_mod):
    """One credit pass at arbitrary loads with many equal values (ties by id)."""
    from paper_2403_05775_amd import kdss
    g = synth.chung_lu(2000, 16000, 2.2, seed=13, planted=30)
    for k in (3, 5):
        tree = kdss.Tree(g, k)
        plan = kdss.Plan(tree, 1)
        ws = plan.alloc_workspace()
        plan.upload(ws)
        for trial in range(3):
            rs = synth.Stream(100 + trial, 81)
            r = (rs.u64(g.n) % np.uint64(3 + 7 * trial)).astype(np.uint64)
            rt = torch.from_numpy(r.view(np.int64).copy()).cuda()
            out = torch.empty(g.n, dtype=torch.int64, device="cuda")
            print(f"leaf credit k={k} trial={trial}", flush=True)
            plan.leaf_credit(ws, rt, out)
            torch.cuda.synchronize()
            got = out.cpu().numpy().view(np.uint64)
            want = oracle_mod.credits(g.n, g.row_ptr, g.col, k, r)
            assert np.array_equal(got, want)
        plan.close()
        tree.close()


def test_extract_alone(K, oracle_mod):
    """The extraction at the oracle's own loads gives the oracle's answer."""
    from paper_2403_05775_amd import kdss
    g = synth.chung_lu(1500, 12000, 2.4, seed=14, planted=20)
    res = ref(oracle_mod, g, 4, 9)
    tree = kdss.Tree(g, 4)
    plan = kdss.Plan(tree, 9)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    rt = torch.from_numpy(res["r"].view(np.int64).copy()).cuda()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    print("extract alone", flush=True)
    out = plan.extract(ws, rt, order, 9)
    assert (out.size, out.dens_num.value, out.ub_num.value) == (res["size"], res["dens_num"], res["ub_num"])
    assert np.array_equal(order.cpu().numpy().view(np.uint32), res["order"])


def test_no_cliques(K, oracle_mod):
    g = synth.complete_graph(6)
    print("k above clique number", flush=True)
    sol = K.solve(g, 7, 3)
    assert sol.c_k == 0 and sol.size == 0 and sol.dens_num == 0 and sol.ub_num == 0
    assert np.all(sol.r == 0)
    assert_same(sol, ref(oracle_mod, g, 7, 3), 3)


@pytest.mark.parametrize("leaf_blocks", [1, 3, 7, 9])
def test_small_leaf_grids(K, oracle_mod, leaf_blocks):
    """Grids far smaller than the tile count: the tiles past the first stride
    come from the tile counters (fewer counters than eight when the grid is
    smaller), and every tile is processed once."""
    from paper_2403_05775_amd import kdss
    g = synth.chung_lu(4000, 30000, 2.3, seed=23, planted=25)
    T = 7
    tree = kdss.Tree(g, 4)
    plan = kdss.Plan(tree, T)
    plan.set_launch(leaf_blocks, 3)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    print(f"leaf grid {leaf_blocks}, {sum(plan.stats().tiles)} tiles", flush=True)
    assert sum(plan.stats().tiles) > 4 * leaf_blocks
    res, _ = plan.run(ws, T, r, order)
    torch.cuda.synchronize()
    want = ref(oracle_mod, g, 4, T)
    assert np.array_equal(r.cpu().numpy().view(np.uint64)[: g.n], want["r"])
    assert np.array_equal(order.cpu().numpy().view(np.uint32), want["order"])
    assert (res.size, res.dens_num.value, res.ub_num.value) == (want["size"], want["dens_num"], want["ub_num"])


@pytest.mark.parametrize("leaf_blocks", [5, 8, 13, 64, 2048])
def test_xcd_range_schedule(K, oracle_mod, leaf_blocks):
    """The XCD-range tile schedule: every tile once whatever the grid (under 8
    workgroups it runs strided; 13 gives the dies uneven workgroup counts), on
    a single problem with big leaves and on a batch listed problem by problem."""
    from paper_2403_05775_amd import kdss
    g = synth.erdos_renyi(300, 0.1, seed=9, planted_clique=70)
    T = 5
    tree = kdss.Tree(g, 4)
    plan = kdss.Plan(tree, T, schedule=2)
    assert plan.stats().schedule == 2
    plan.set_launch(leaf_blocks, 7)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    print(f"xcd schedule, grid {leaf_blocks}, single", flush=True)
    res, _ = plan.run(ws, T, r, order)
    torch.cuda.synchronize()
    want = ref(oracle_mod, g, 4, T)
    assert np.array_equal(r.cpu().numpy().view(np.uint64)[: g.n], want["r"])
    assert (res.size, res.dens_num.value) == (want["size"], want["dens_num"])
    probs = [(synth.chung_lu(400 + 90 * i, 3000 + 500 * i, 2.3, seed=50 + i, planted=12), 3 + i % 4)
             for i in range(6)]
    b = kdss.Batch([kdss.Tree(gq, kq) for gq, kq in probs], T, schedule=2)
    b.set_launch(leaf_blocks, 5)
    wsb = b.alloc_workspace()
    b.upload(wsb)
    rb = torch.empty(b.n, dtype=torch.int64, device="cuda")
    ob = torch.empty(b.n, dtype=torch.int32, device="cuda")
    print(f"xcd schedule, grid {leaf_blocks}, batch", flush=True)
    resb = b.run(wsb, T, rb, ob)
    torch.cuda.synchronize()
    rr = rb.cpu().numpy().view(np.uint64)
    oo = ob.cpu().numpy().view(np.uint32)
    for q, (gq, kq) in enumerate(probs):
        want = ref(oracle_mod, gq, kq, T)
        lo, hi = int(b.node_off[q]), int(b.node_off[q + 1])
        assert np.array_equal(rr[lo:hi], want["r"]), q
        assert np.array_equal(oo[lo:hi], want["order"]), q
        assert (resb[q].size, resb[q].dens_num.value) == (want["size"], want["dens_num"]), q


@pytest.mark.parametrize("G,heavy", [(4, 1), (8, 1), (8, 2), (4, 3)])
def test_multi_iteration_graphs(K, oracle_mod, G, heavy):
    """Iterations replayed as graphs of G iterations (21 = 2 or 5 replays plus
    the rest one by one), three runs in a row with the oracle checked after
    each; and a batch plan with 4-iteration graphs; heavy leaves queued or in
    place (a graph without the heavy kernel)."""
    from paper_2403_05775_amd import kdss
    g = synth.chung_lu(3000, 20000, 2.3, seed=11, planted=25)
    T = 21
    want = ref(oracle_mod, g, 4, T)
    tree = kdss.Tree(g, 4)
    plan = kdss.Plan(tree, T, use_graph=G, heavy=heavy)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for rep in range(3):
        print(f"graphs of {G} iterations, heavy mode {heavy}, run {rep}", flush=True)
        res, _ = plan.run(ws, T, r, order)
        torch.cuda.synchronize()
        assert np.array_equal(r.cpu().numpy().view(np.uint64)[: g.n], want["r"]), rep
        assert np.array_equal(order.cpu().numpy().view(np.uint32), want["order"]), rep
        assert (res.size, res.dens_num.value, res.ub_num.value) == (want["size"], want["dens_num"], want["ub_num"])
    probs = [(synth.chung_lu(400 + 90 * i, 3000 + 500 * i, 2.3, seed=50 + i, planted=12), 3 + i % 4)
             for i in range(4)]
    b = kdss.Batch([kdss.Tree(gq, kq) for gq, kq in probs], 9, use_graph=4, heavy=heavy)
    wsb = b.alloc_workspace()
    b.upload(wsb)
    rb = torch.empty(b.n, dtype=torch.int64, device="cuda")
    ob = torch.empty(b.n, dtype=torch.int32, device="cuda")
    for rep in range(2):
        resb = b.run(wsb, 9, rb, ob)
        torch.cuda.synchronize()
        rr = rb.cpu().numpy().view(np.uint64)
        for q, (gq, kq) in enumerate(probs):
            w = ref(oracle_mod, gq, kq, 9)
            lo, hi = int(b.node_off[q]), int(b.node_off[q + 1])
            assert np.array_equal(rr[lo:hi], w["r"]), (rep, q)
            assert (resb[q].size, resb[q].dens_num.value) == (w["size"], w["dens_num"]), (rep, q)
