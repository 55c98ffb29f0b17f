"""The clique tree built on the GPU (kdss_sct_build_gpu): its leaves expand to
every k-clique exactly once (against the oracle's listing), and runs on it give
the oracle's results bit for bit; on the 1M-node workload it agrees with the
host-built tree in c_k and in every load."""
from __future__ import annotations

import itertools
import math

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


def expand(tree, k):
    h, p, m = tree.export()
    out, at = [], 0
    for hh, pp in zip(h.tolist(), p.tolist()):
        hold, piv = m[at:at + hh].tolist(), m[at + hh:at + hh + pp].tolist()
        at += hh + pp
        for extra in itertools.combinations(piv, k - hh):
            out.append(tuple(sorted(hold + list(extra))))
    return out


@pytest.mark.parametrize("seed,k", [(0, 2), (1, 3), (2, 4), (3, 5), (4, 6), (5, 3)])
def test_gpu_tree_expands_to_every_clique_once(K, oracle_mod, seed, k):
    rs = synth.Stream(seed, 87)
    n = int(rs.integers(30, 300)[0])
    g = synth.chung_lu(n, int(rs.integers(2 * n, 8 * n)[0]), 2.2, seed=seed, planted=int(rs.integers(5, 25)[0]))
    print(f"gpu tree seed={seed} n={g.n} k={k}", flush=True)
    t = K.GpuTree(g, k)
    got = expand(t, k)
    want = [tuple(c) for c in oracle_mod.list_cliques(g.n, g.row_ptr, g.col, k).tolist()]
    assert len(got) == len(set(got)) and sorted(got) == sorted(want)
    assert t.stats().c_k.value == len(want)
    t.close()


@pytest.mark.parametrize("k,planted", [(3, 70), (5, 30), (4, 30)])
def test_gpu_tree_runs_match_oracle(K, oracle_mod, k, planted):
    g = synth.erdos_renyi(260, 0.12, seed=7, planted_clique=planted)
    t = K.GpuTree(g, k)
    assert t.stats().c_k.value == oracle_mod.count(g.n, g.row_ptr, g.col, k)
    plan = K.Plan(t, 9)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    res, _ = plan.run(ws, 9, r, order)
    torch.cuda.synchronize()
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, k, 9)
    assert np.array_equal(r.cpu().numpy().view(np.uint64)[: g.n], ref["r"])
    assert np.array_equal(order.cpu().numpy().view(np.uint32), ref["order"])
    assert (res.size, res.dens_num.value, res.ub_num.value) == (ref["size"], ref["dens_num"], ref["ub_num"])
    t.close()


def test_gpu_tree_chung_lu_1m(K):
    g = synth.chung_lu(1_000_000, 10_000_000, 2.5, seed=0, planted=40, planted_p=0.9)
    host = K.Tree(g, 5)
    gpu = K.GpuTree(g, 5)
    hs, gs = host.stats(), gpu.stats()
    print(f"host build {hs.build_seconds:.2f} s, GPU build {gs.build_seconds:.2f} s; "
          f"leaves {hs.leaves} / {gs.leaves}", flush=True)
    assert gs.c_k.value == hs.c_k.value and gs.degeneracy == hs.degeneracy
    out = []
    for t in (host, gpu):
        plan = K.Plan(t, 20)
        ws = plan.alloc_workspace()
        plan.upload(ws)
        r = plan.alloc_loads()
        order = torch.empty(g.n, dtype=torch.int32, device="cuda")
        res, _ = plan.run(ws, 20, r, order)
        torch.cuda.synchronize()
        out.append((r.cpu().numpy().view(np.uint64).copy(), res.size, res.dens_num.value))
        del ws
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1:] == out[1][1:]
    host.close()
    gpu.close()


@pytest.mark.parametrize("n,p,k", [(300, 0.55, 3), (300, 0.55, 4), (420, 0.62, 3)])
def test_gpu_tree_dense_graphs(K, oracle_mod, n, p, k):
    """Dense graphs whose degeneracy needs three (146) and four (236) bitset
    words per node: c_k equals the host tree's and the oracle's count, and a
    run on the GPU-built tree equals the oracle bit for bit."""
    g = synth.erdos_renyi(n, p, seed=5)
    t = K.GpuTree(g, k)
    st = t.stats()
    print(f"dense n={n} p={p} k={k}: degeneracy {st.degeneracy}, {st.leaves} leaves", flush=True)
    assert st.degeneracy > 128
    host = K.Tree(g, k)
    assert st.c_k.value == host.stats().c_k.value == oracle_mod.count(g.n, g.row_ptr, g.col, k)
    host.close()
    T = 3
    plan = K.Plan(t, T)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    res, _ = plan.run(ws, T, r, order)
    torch.cuda.synchronize()
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, k, T)
    assert np.array_equal(r.cpu().numpy().view(np.uint64)[: g.n], ref["r"])
    assert (res.size, res.dens_num.value, res.ub_num.value) == (ref["size"], ref["dens_num"], ref["ub_num"])
    t.close()


@pytest.mark.parametrize("case", ["empty", "no_edges", "star_k2", "k_above_clique_number", "triangle_k3"])
def test_gpu_tree_edge_cases(K, oracle_mod, case):
    """Degenerate inputs: no nodes, no edges, stars (k = 2: every edge is a
    leaf), k above the clique number (no leaves), one triangle."""
    if case == "empty":
        g, k = synth.from_edge_list(0, []), 3
    elif case == "no_edges":
        g, k = synth.from_edge_list(50, []), 2
    elif case == "star_k2":
        g, k = synth.from_edge_list(40, [(0, i) for i in range(1, 40)]), 2
    elif case == "k_above_clique_number":
        g, k = synth.complete_graph(7), 8
    else:
        g, k = synth.from_edge_list(3, [(0, 1), (1, 2), (0, 2)]), 3
    print(f"edge case {case}: n={g.n} k={k}", flush=True)
    t = K.GpuTree(g, k)
    st = t.stats()
    want = oracle_mod.count(g.n, g.row_ptr, g.col, k) if g.n else 0
    assert st.c_k.value == want
    got = sorted(expand(t, k)) if st.leaves else []
    want_list = sorted(tuple(c) for c in oracle_mod.list_cliques(g.n, g.row_ptr, g.col, k).tolist()) if want else []
    assert got == want_list
    t.close()


def test_gpu_tree_rejects_degeneracy_above_256(K):
    with pytest.raises(K.KdssError) as e:
        K.GpuTree(synth.complete_graph(300), 3)   # degeneracy 299
    assert e.value.status == K.EUNSUPPORTED


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gpu_tree_core_numbers(K, seed):
    """The device peeling gives every node its core number (unique, so equal to
    the host peeling's) and an order with at most the degeneracy later
    neighbours per node."""
    rs = synth.Stream(seed, 88)
    n = int(rs.integers(500, 20000)[0])
    g = synth.chung_lu(n, int(rs.integers(2 * n, 10 * n)[0]), 2.2 + 0.5 * float(rs.uniform(1)[0]), seed=seed,
                       planted=int(rs.integers(0, 30)[0]))
    host, gpu = K.Tree(g, 3), K.GpuTree(g, 3)
    assert np.array_equal(gpu.core_numbers(), host.core_numbers())
    assert gpu.stats().degeneracy == host.stats().degeneracy
    assert gpu.stats().c_k.value == host.stats().c_k.value
    host.close()
    gpu.close()


def test_gpu_tree_small_workspace_stages_in_chunks(K):
    """Workspaces far below the suggested size (about 7 MB of fixed parts here,
    3.9 MB of leaves): the recursion runs in smaller chunks and the leaves come
    back through a small staging window in several chunks; every tree built
    equals the one built with the suggested size.  Sizes too small for the fixed
    parts or for one root child's leaves are refused with KDSS_EWORKSPACE."""
    g = synth.chung_lu(20000, 200000, 2.3, seed=61, planted=30)
    k = 4
    big = K.GpuTree(g, k)
    hb, pb, mb = big.export()
    ck = big.stats().c_k.value
    ok = 0
    for mib in (12, 10, 9, 8, 7.5, 7):
        nbytes = int(mib * (1 << 20))
        print(f"gpu tree with {nbytes} workspace bytes", flush=True)
        try:
            small = K.GpuTree(g, k, ws_bytes=nbytes)
        except K.KdssError as e:
            assert e.status == K.EWORKSPACE
            continue
        hs, ps, ms = small.export()
        assert np.array_equal(hs, hb) and np.array_equal(ps, pb) and np.array_equal(ms, mb)
        assert small.stats().c_k.value == ck
        small.close()
        ok += 1
    assert ok >= 2
    with pytest.raises(K.KdssError) as e:
        K.GpuTree(g, k, ws_bytes=1 << 16)
    assert e.value.status == K.EWORKSPACE
    big.close()
