"""Host-side tests of the C-ABI library: exports, graph checks, the clique tree
builder and the planner.  No GPU call is made here."""
from __future__ import annotations

import ctypes as C
import itertools
import math
import os
import re

import numpy as np
import pytest

from paper_2403_05775_amd import kdss, synth
from tests.test_oracle_pins import example_graph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = "".join(open(os.path.join(ROOT, "include", h)).read() for h in ("kdss.h", "kdss_gnn.h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kdss_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = kdss.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(kdss.EXPORTS) | (set(names) - set(kdss.EXPORTS))
    for name in kdss.EXPORTS:
        assert name in names
    assert sum(1 for x in names if x.startswith("kdss_gnn_")) >= 12


def test_status_strings():
    L = kdss.lib()
    for code in range(0, -9, -1):
        assert L.kdss_status_string(code)
    assert L.kdss_status_string(0) == b"ok"


def test_validate_codes():
    good = synth.from_edge_list(4, [(0, 1), (1, 2), (2, 3)])
    assert kdss.validate(good) == kdss.OK
    bad = synth.Graph(n=4, row_ptr=good.row_ptr.copy(), col=np.array([1, 2, 0, 1, 3, 2], np.uint32))
    assert kdss.validate(bad) == kdss.EGRAPH
    bad2 = synth.Graph(n=4, row_ptr=np.array([0, 0, 2, 4, 5], np.uint64), col=np.array([0, 2, 1, 3, 2], np.uint32))
    assert kdss.validate(bad2) == kdss.EGRAPH
    with pytest.raises(kdss.KdssError) as e:
        kdss.Tree(bad, 3)
    assert e.value.status == kdss.EGRAPH


def test_validate_large_graph_reports_the_first_fault():
    """Rows are checked on several host threads; the fault reported is the one
    a row-by-row pass meets first."""
    g = synth.chung_lu(50_000, 300_000, 2.4, seed=3)
    assert kdss.validate(g) == kdss.OK
    rp = g.row_ptr
    # drop the symmetric copy of one edge late in the graph: row u keeps v,
    # row v's entry for u becomes a duplicate of its neighbour (breaking order)
    u = 45_000
    while rp[u + 1] == rp[u]:
        u += 1
    v = int(g.col[rp[u]])
    col = g.col.copy()
    pos = int(rp[v]) + int(np.searchsorted(g.col[rp[v]:rp[v + 1]], u))
    col[pos] = g.n - 1 if u != g.n - 1 else 0
    bad = synth.Graph(n=g.n, row_ptr=rp, col=col)
    assert kdss.validate(bad) == kdss.EGRAPH
    # a self-loop in an early row as well: that one is reported
    w = 10
    while rp[w + 1] == rp[w]:
        w += 1
    col2 = col.copy()
    col2[rp[w]] = w
    with pytest.raises(kdss.KdssError) as e:
        kdss.Tree(synth.Graph(n=g.n, row_ptr=rp, col=col2), 3)
    assert e.value.status == kdss.EGRAPH and f"node {w}" in str(e.value)


def test_tree_argument_errors():
    g = synth.complete_graph(6)
    for k, code in [(1, kdss.EINVAL), (0, kdss.EINVAL), (32, kdss.ERANGE)]:
        with pytest.raises(kdss.KdssError) as e:
            kdss.Tree(g, k)
        assert e.value.status == code


def expand(h, p, m, k):
    out, off = [], 0
    for hh, pp in zip(h, p):
        H = [int(x) for x in m[off: off + hh]]
        P = [int(x) for x in m[off + hh: off + hh + pp]]
        off += hh + pp
        for c in itertools.combinations(P, k - hh):
            out.append(tuple(sorted(H + list(c))))
    return out


def test_example_tree_matches_paper_pairs():
    """Example 2 prints five pairs, each with one hold node; the library's tree of
    the same graph has the same number of leaves and the same pair sizes, and for
    k = 3 (Lemma 5) encodes the 9 triangles of Example 1."""
    g, pairs, vals = example_graph()
    t = kdss.Tree(g, 3)
    h, p, m = t.export()
    assert len(h) == len(pairs)
    assert sorted(zip(h.tolist(), p.tolist())) == sorted((len(a), len(b)) for a, b in pairs)
    assert t.stats().c_k.value == vals["triangles"][0]
    assert len(set(expand(h, p, m, 3))) == 9


@pytest.mark.parametrize("seed", range(8))
def test_tree_expansion_equals_enumeration(oracle_mod, seed):
    """Lemma 4: the kept leaves partition C_k(V); every leaf is a clique; h <= k <= h + p."""
    rs = synth.Stream(seed, 51)
    n = int(rs.integers(20, 45)[0])
    g = synth.erdos_renyi(n, 0.35, seed=seed, planted_clique=int(rs.integers(0, 12)[0]))
    A = set()
    rp = g.row_ptr.astype(np.int64)
    for u in range(n):
        for e in range(rp[u], rp[u + 1]):
            A.add((u, int(g.col[e])))
    for k in range(2, 9):
        t = kdss.Tree(g, k)
        h, p, m = t.export()
        assert np.all(h <= k) and np.all(h + p >= k)
        off = 0
        for hh, pp in zip(h, p):
            leaf = [int(x) for x in m[off: off + hh + pp]]
            off += hh + pp
            assert all((a, b) in A for a, b in itertools.combinations(leaf, 2))
        got = expand(h, p, m, k)
        ref = {tuple(int(x) for x in c) for c in oracle_mod.list_cliques(g.n, g.row_ptr, g.col, k)}
        assert len(got) == len(set(got)) == len(ref)
        assert set(got) == ref
        assert t.stats().c_k.value == len(ref)
        assert t.stats().members == int(np.sum(h + p))


def test_tree_power_law_counts(oracle_mod):
    g = synth.chung_lu(3000, 30000, 2.3, seed=4, planted=25)
    for k in (3, 5, 7):
        t = kdss.Tree(g, k)
        assert t.stats().c_k.value == oracle_mod.count(g.n, g.row_ptr, g.col, k)


def test_tree_independent_of_threads():
    g = synth.chung_lu(5000, 40000, 2.4, seed=2)
    a = kdss.Tree(g, 4, threads=1).export()
    b = kdss.Tree(g, 4, threads=7).export()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_core_numbers_match_peeling():
    g = synth.chung_lu(500, 3000, 2.3, seed=3)
    core = kdss.Tree(g, 3).core_numbers()
    # peeling by repeatedly removing a minimum-degree node (quadratic, tiny n)
    adj = [set() for _ in range(g.n)]
    rp = g.row_ptr.astype(np.int64)
    for u in range(g.n):
        for e in range(rp[u], rp[u + 1]):
            adj[u].add(int(g.col[e]))
    alive = set(range(g.n))
    deg = {u: len(adj[u]) for u in alive}
    ref = np.zeros(g.n, dtype=np.int64)
    cur = 0
    while alive:
        u = min(alive, key=lambda x: (deg[x], x))
        cur = max(cur, deg[u])
        ref[u] = cur
        alive.remove(u)
        for v in adj[u]:
            if v in alive:
                deg[v] -= 1
    assert np.array_equal(core.astype(np.int64), ref)


def test_plan_layout_and_errors():
    g = synth.chung_lu(2000, 20000, 2.3, seed=5, planted=30)
    t = kdss.Tree(g, 4)
    ts = t.stats()
    p = kdss.Plan(t, 50)
    s = p.stats()
    assert sum(s.leaves) == ts.leaves and sum(s.members) == ts.members
    assert s.width == 64 and s.workspace_bytes > s.stream_bytes
    with pytest.raises(kdss.KdssError) as e:
        kdss.Plan(t, 0)
    assert e.value.status == kdss.EINVAL
    with pytest.raises(kdss.KdssError) as e:
        kdss.Plan(t, 10, r0_max=2**64 - 2, width=64)
    assert e.value.status == kdss.EOVERFLOW
    assert kdss.Plan(t, 10, r0_max=2**64 - 2).stats().width == 128
    assert kdss.Plan(t, 10, width=128).stats().width == 128
    assert kdss.Plan(t, 10, r0_max=2**60).stats().key_mode == 1


def test_gather_mode_option():
    g = synth.chung_lu(3000, 30000, 2.2, seed=6, planted=30)
    t = kdss.Tree(g, 4)
    s = kdss.Plan(t, 10).stats()
    assert 0 < s.hot_nodes <= 512 and 0.0 < s.hot_share <= 1.0
    # left to the library: masked gathers once hot nodes hold half the occurrences
    assert s.gather == (1 if s.hot_share >= 0.5 else 2)
    assert kdss.Plan(t, 10, gather=1).stats().gather == 1
    assert kdss.Plan(t, 10, gather=2).stats().gather == 2
    for bad in (-1, 3):
        with pytest.raises(kdss.KdssError) as e:
            kdss.Plan(t, 10, gather=bad)
        assert e.value.status == kdss.EINVAL
    # hot nodes: the (at most 512) nodes with the most member occurrences, at
    # least 32 each; the share is their part of all occurrences
    _, _, mem = t.export()
    occ = np.bincount(mem, minlength=g.n)
    cand = np.flatnonzero(occ >= 32)
    cand = cand[np.lexsort((cand, -occ[cand]))][:512]
    assert s.hot_nodes == cand.size
    assert abs(s.hot_share - occ[cand].sum() / occ.sum()) < 1e-12


def test_update_option():
    g = synth.chung_lu(2000, 20000, 2.3, seed=5, planted=30)
    t = kdss.Tree(g, 4)
    assert kdss.Plan(t, 10).stats().update == 0
    assert kdss.Plan(t, 10, update=1).stats().update == 1
    for kw in (dict(update=2), dict(update=-1), dict(update=1, width=128), dict(update=1, r0_max=2**64 - 2)):
        with pytest.raises(kdss.KdssError) as e:
            kdss.Plan(t, 10, **kw)
        assert e.value.status == kdss.EINVAL, kw


def test_heavy_leaf_option():
    """Heavy leaves: queued (four per heavy-kernel batch) unless in place or
    eight per batch is asked for; other values refused."""
    g = synth.chung_lu(2000, 20000, 2.3, seed=5, planted=30)
    t = kdss.Tree(g, 4)
    assert kdss.Plan(t, 10).stats().heavy == 1
    assert kdss.Plan(t, 10, heavy=1).stats().heavy == 1
    assert kdss.Plan(t, 10, heavy=2).stats().heavy == 2
    assert kdss.Plan(t, 10, heavy=3).stats().heavy == 3
    assert kdss.Batch([t], 10, heavy=2).stats().heavy == 2
    for h in (4, -1):
        with pytest.raises(kdss.KdssError) as e:
            kdss.Plan(t, 10, heavy=h)
        assert e.value.status == kdss.EINVAL, h


def test_sample_build_arguments_and_empty_sample():
    g = synth.chung_lu(300, 2000, 2.3, seed=4, planted=10)
    c, keep = kdss._csr(g)
    L = kdss.lib()
    h = C.c_void_p()
    assert L.kdss_sample_build(C.byref(c), 4, 5, None, None, 0, None, None, C.byref(h)) == kdss.EINVAL  # no draws
    assert L.kdss_sample_build(C.byref(c), 1, 0, None, None, 0, None, None, C.byref(h)) == kdss.EINVAL  # k < 2
    assert L.kdss_sample_build(C.byref(c), 32, 0, None, None, 0, None, None, C.byref(h)) == kdss.ERANGE  # k > 31
    # the workspace: graph, k + 1 rows of 128-bit path counts, prefix sums, draws, walks
    need = C.c_size_t(0)
    assert L.kdss_sample_workspace(g.n, int(c.nnz), 4, 5, C.byref(need)) == 0
    al = lambda b: (b + 255) // 256 * 256
    n, nnz, nb = g.n, int(c.nnz), (g.n + 1023) // 1024
    assert need.value == sum(al(x) for x in (8 * (n + 1), 4 * nnz, 4 * n, 16 * 5 * n, 16 * n, 16 * nb,
                                             16 * 5 * 4, 4 * 5 * 4, 5, 4))
    assert L.kdss_sample_workspace(g.n, int(c.nnz), 4, 0, C.byref(need)) == 0 and need.value == 0
    draws = np.ones(5 * 4 * 2, dtype=np.uint64)
    assert L.kdss_sample_build(C.byref(c), 4, 5, draws.ctypes.data_as(C.POINTER(C.c_uint64)), None, 0, None, None,
                               C.byref(h)) == kdss.EWORKSPACE
    # no samples: no device work, an empty tree with no core numbers
    t = kdss.SampleTree(g, 4, np.zeros((0, 4, 2), dtype=np.uint64))
    st = t.stats()
    assert (st.leaves, st.members, st.c_k.value, t.info.samples, t.info.colors > 0) == (0, 0, 0, 0, True)
    with pytest.raises(kdss.KdssError) as e:
        t.core_numbers()
    assert e.value.status == kdss.EUNSUPPORTED


def test_gpu_tree_build_rejects_bad_arguments_before_device_work():
    g = synth.complete_graph(6)
    for k, code in [(1, kdss.EINVAL), (32, kdss.ERANGE)]:
        with pytest.raises(kdss.KdssError) as e:
            kdss.GpuTree(g, k)
        assert e.value.status == code
    bad = synth.Graph(n=4, row_ptr=np.array([0, 0, 2, 4, 5], np.uint64), col=np.array([0, 2, 1, 3, 2], np.uint32))
    with pytest.raises(kdss.KdssError) as e:
        kdss.GpuTree(bad, 3)
    assert e.value.status == kdss.EGRAPH


def test_run_rejects_bad_arguments_before_device_work():
    g = synth.complete_graph(8)
    t = kdss.Tree(g, 3)
    p = kdss.Plan(t, 5)
    L = kdss.lib()
    res = kdss.Result()
    # null workspace / not uploaded workspace / T out of range: host checks only
    assert L.kdss_run(p._h, None, 0, 3, None, C.c_void_p(8), C.c_void_p(8), None, 0, C.byref(res), None) == kdss.EINVAL
    assert L.kdss_run(p._h, C.c_void_p(256), p.workspace_bytes, 3, None, C.c_void_p(8), C.c_void_p(8), None, 0,
                      C.byref(res), None) == kdss.EWORKSPACE
    assert L.kdss_run(p._h, C.c_void_p(256), p.workspace_bytes, 9, None, C.c_void_p(8), C.c_void_p(8), None, 0,
                      C.byref(res), None) == kdss.EINVAL
    assert L.kdss_run(p._h, C.c_void_p(256), 16, 3, None, C.c_void_p(8), C.c_void_p(8), None, 0,
                      C.byref(res), None) == kdss.EWORKSPACE
    assert b"workspace" in L.kdss_last_error()


def test_batch_plan_layout():
    probs = [(synth.chung_lu(300 + 50 * i, 2000 + 300 * i, 2.3, seed=i), 3 + i % 4) for i in range(5)]
    trees = [kdss.Tree(g, k) for g, k in probs]
    b = kdss.Batch(trees, 30)
    assert b.count == 5
    assert b.node_off.tolist() == list(np.cumsum([0] + [g.n for g, _ in probs]))
    st = b.stats()
    assert sum(st.leaves) == sum(t.stats().leaves for t in trees)
    assert sum(st.members) == sum(t.stats().members for t in trees)
    with pytest.raises(kdss.KdssError) as e:
        b.set_launch(0, 10)
    assert e.value.status == kdss.ERANGE
    b.set_launch(512, 256)


def test_workspace_size_matches_plan():
    g = synth.chung_lu(2000, 20000, 2.3, seed=5, planted=30)
    t = kdss.Tree(g, 4)
    for T, r0_max, width in ((50, 0, 0), (10, 2**60, 0), (10, 0, 128), (7, 3, 64)):
        assert t.workspace_size(T, r0_max, width) == kdss.Plan(t, T, r0_max, width=width).workspace_bytes
    with pytest.raises(kdss.KdssError) as e:
        t.workspace_size(0)
    assert e.value.status == kdss.EINVAL


def test_solve_sizes_buffers_before_device_work():
    """kdss_solve with no workspace builds and lays out the tree, reports the
    workspace and load width, and runs nothing (no device call)."""
    g = synth.chung_lu(1500, 12000, 2.3, seed=2, planted=20)
    L = kdss.lib()
    c, keep = kdss._csr(g)
    need = C.c_size_t(0)
    res = kdss.Result()
    o = kdss.Opts(0, 0, 0, 0, 0, 0)
    rc = L.kdss_solve(C.byref(c), 4, 20, C.byref(o), None, 0, None, 0, C.byref(need), None, 0, None, C.byref(res),
                      None)
    assert rc == kdss.EWORKSPACE
    assert need.value == kdss.Plan(kdss.Tree(g, 4), 20).workspace_bytes
    assert (res.width, res.n) == (64, g.n)
    o128 = kdss.Opts(128, 0, 0, 0, 0, 0)
    rc = L.kdss_solve(C.byref(c), 4, 20, C.byref(o128), None, 0, None, 0, C.byref(need), None, 0, None,
                      C.byref(res), None)
    assert rc == kdss.EWORKSPACE and res.width == 128
    # argument and graph errors come first
    assert L.kdss_solve(None, 4, 20, None, None, 0, None, 0, C.byref(need), None, 0, None, C.byref(res),
                        None) == kdss.EINVAL
    assert L.kdss_solve(C.byref(c), 1, 20, None, None, 0, None, 0, C.byref(need), None, 0, None, C.byref(res),
                        None) == kdss.EINVAL
    assert L.kdss_solve(C.byref(c), 4, 0, None, None, 0, None, 0, C.byref(need), None, 0, None, C.byref(res),
                        None) == kdss.EINVAL


def test_resume_and_counts_reject_bad_arguments_before_device_work():
    g = synth.complete_graph(8)
    t = kdss.Tree(g, 3)
    p = kdss.Plan(t, 5)
    L = kdss.lib()
    res = kdss.Result()
    v = C.c_void_p(8)
    assert L.kdss_run_resume(p._h, C.c_void_p(256), p.workspace_bytes, 3, 2, None, None, v, v, None, 0,
                             C.byref(res), None) == kdss.EINVAL           # no checkpoint loads
    assert L.kdss_run_resume(p._h, C.c_void_p(256), p.workspace_bytes, 3, 2**32 - 2, v, None, v, v, None, 0,
                             C.byref(res), None) == kdss.ERANGE           # t_offset + T past 2^32 - 1
    assert L.kdss_run_resume(p._h, C.c_void_p(256), p.workspace_bytes, 3, 2, v, None, v, v, None, 0,
                             C.byref(res), None) == kdss.EWORKSPACE       # not uploaded
    assert L.kdss_extract_counts(p._h, C.c_void_p(256), p.workspace_bytes, v, None, 0, v, v, C.byref(res),
                                 None) == kdss.EINVAL                     # T = 0
    b = kdss.Batch([t, kdss.Tree(g, 4)], 5)
    assert L.kdss_extract_counts(b._h, C.c_void_p(256), b.workspace_bytes, v, None, 3, v, v, C.byref(res),
                                 None) == kdss.EUNSUPPORTED               # batch plans: no prefix counts
    b.close()
    L.kdss_batch_free(None)


@pytest.mark.parametrize("k", [3, 5, 6])
def test_tree_count_equals_build(k):
    """kdss_sct_count sizes the same tree kdss_sct_build keeps."""
    for g in (synth.chung_lu(3000, 30000, 2.3, seed=8, planted=30), synth.rmat(11, 8, seed=0)):
        t = kdss.Tree(g, k)
        a, b = t.stats(), kdss.tree_count(g, k)
        for f in ("k", "n", "leaves", "members", "s_max", "degeneracy"):
            assert getattr(a, f) == getattr(b, f), f
        assert a.c_k.value == b.c_k.value
        assert kdss.tree_count(g, k, threads=1).leaves == a.leaves


def test_schedule_option():
    g = synth.chung_lu(2000, 20000, 2.3, seed=5, planted=30)
    t = kdss.Tree(g, 4)
    assert kdss.Plan(t, 10).stats().schedule == 1
    assert kdss.Plan(t, 10, schedule=1).stats().schedule == 1
    assert kdss.Plan(t, 10, schedule=2).stats().schedule == 2
    for bad in (-1, 3):
        with pytest.raises(kdss.KdssError) as e:
            kdss.Plan(t, 10, schedule=bad)
        assert e.value.status == kdss.EINVAL
