"""The C-ABI calls beyond the plain run, on the GPU, against the oracle:

* kdss_extract_counts: every prefix count K_i = |C_k(order[0 .. i))| (Algorithm
  2's prefix scoring) element by element against the oracle's prefix counts,
  for every leaf size class, both key modes and 128-bit loads;
* kdss_run_resume: a run cut at a checkpoint and resumed equals the uncut run
  bit for bit (loads, order, density, upper bound, certificate, trace rows);
* kdss_solve: the one-shot call equals the oracle;
* start loads above the plan's r0_max are refused before the first iteration.
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


def dev_u64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64).copy()).cuda()


def host_u64(t, n):
    return t.cpu().numpy().view(np.uint64)[:n].copy()


def counts_case(K, O, g, k, r, width=0):
    """GPU prefix counts at loads r (u64[n]) against the oracle's."""
    tree = K.Tree(g, k)
    plan = K.Plan(tree, 1, r0_max=int(r.max()) if g.n else 0, width=width)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    if plan.width == 128:
        w = np.zeros(2 * g.n, dtype=np.uint64)
        w[0::2] = r
        rt = dev_u64(w)
    else:
        rt = dev_u64(r)
    order = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    cnt = torch.empty(max(g.n, 1), dtype=torch.int64, device="cuda")
    res = plan.extract_counts(ws, rt, order, cnt, 1)
    torch.cuda.synchronize()
    want = O.prefix_counts(g.n, g.row_ptr, g.col, k, r)
    assert np.array_equal(order.cpu().numpy().view(np.uint32)[: g.n], want["order"])
    assert np.array_equal(host_u64(cnt, g.n), want["K"])
    assert (res.size, res.dens_num.value) == (want["size"], want["dens_num"])
    plan.close()
    tree.close()
    return plan


@pytest.mark.parametrize("k,planted", [(2, 70), (3, 70), (5, 30), (6, 30), (8, 30)])
def test_prefix_counts_every_size_class(K, oracle_mod, k, planted):
    """Leaves of 2..64 members and above 64 (a planted 70-clique); loads with ties."""
    g = synth.erdos_renyi(260, 0.12, seed=7, planted_clique=planted)
    rs = synth.Stream(k, 91)
    r = (rs.u64(g.n) % np.uint64(7)).astype(np.uint64)
    say(f"prefix counts k={k} planted={planted}")
    counts_case(K, oracle_mod, g, k, r)


@pytest.mark.parametrize("seed", range(4))
def test_prefix_counts_random_graphs(K, oracle_mod, seed):
    """Power-law graphs with a ragged last scan tile (n not a multiple of 1024),
    packed keys, (load, id) keys and 128-bit loads."""
    rs = synth.Stream(seed, 93)
    n = int(rs.integers(1100, 5000)[0])
    g = synth.chung_lu(n, 8 * n, 2.3, seed=300 + seed, planted=20)
    k = 3 + seed % 3
    r = (rs.u64(n) % np.uint64(50)).astype(np.uint64)
    if seed == 2:
        r = r + np.uint64(2**62)
    say(f"prefix counts seed={seed} n={n} k={k}")
    counts_case(K, oracle_mod, g, k, r, width=128 if seed == 3 else 0)


def test_prefix_counts_after_a_run(K, oracle_mod):
    """K_i at the loads of a 40-iteration run (the extraction order kdss_run
    used): the best prefix of the run is the argmax of K_i / i."""
    g = synth.erdos_renyi(200, 0.08, seed=0, planted_clique=12)
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, 3, 40)
    say("prefix counts after 40 iterations")
    counts_case(K, oracle_mod, g, 3, ref["r"])
    want = oracle_mod.prefix_counts(g.n, g.row_ptr, g.col, 3, ref["r"])["K"].astype(object)
    ratios = [(int(want[i]), i + 1) for i in range(g.n)]
    best = max(range(g.n), key=lambda i: (ratios[i][0] / ratios[i][1], i))
    assert best + 1 == ref["size"] == 12


def _run(K, plan, ws, T, n, r0=None, trace_cap=0):
    r = plan.alloc_loads()
    order = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    res, trace = plan.run(ws, T, r, order, r0=r0, trace_cap=trace_cap)
    torch.cuda.synchronize()
    return res, trace, r, order


@pytest.mark.parametrize("case", ["cold", "warm", "wide", "trace"])
def test_resume_equals_uncut_run(K, oracle_mod, case):
    g = synth.chung_lu(3000, 24000, 2.3, seed=31, planted=25)
    k, T1, T2 = 4, 7, 11
    rs = synth.Stream(31, 95)
    r0 = (rs.u64(g.n) % np.uint64(20)).astype(np.uint64) if case == "warm" else None
    tree = K.Tree(g, k)
    ck = tree.stats().c_k.value
    r0_max = (0 if r0 is None else int(r0.max())) + T1 * ck
    every = 2 if case == "trace" else 0
    plan = K.Plan(tree, T1 + T2, r0_max=r0_max, width=128 if case == "wide" else 0, extract_every=every)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    r0_t = None if r0 is None else dev_u64(r0)
    cap = (T1 + T2) // every + 1 if every else 0
    say(f"resume {case}: uncut run of {T1 + T2}")
    full, ftrace, fr, fo = _run(K, plan, ws, T1 + T2, g.n, r0_t, cap)
    say(f"resume {case}: {T1} then {T2}")
    part, _, pr, _ = _run(K, plan, ws, T1, g.n, r0_t)
    ckpt = K.loads_to_numpy(pr, g.n, plan.width)
    assert not isinstance(ckpt, list)
    start = dev_u64(ckpt)
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    res, rtrace = plan.resume(ws, T2, T1, start, r, order, r0=r0_t, trace_cap=cap)
    torch.cuda.synchronize()
    assert K.loads_to_numpy(r, g.n, plan.width).tolist() == K.loads_to_numpy(fr, g.n, plan.width).tolist()
    assert np.array_equal(order.cpu().numpy(), fo.cpu().numpy())
    for f in ("T", "size", "width", "bound_den", "bound_kind", "certified"):
        assert getattr(res, f) == getattr(full, f), f
    for f in ("dens_num", "ub_num", "c_k", "bound_num"):
        assert getattr(res, f).value == getattr(full, f).value, f
    if every:
        # rows of the resumed part: iterations past the checkpoint
        want = [row for row in ftrace if row["t"] > T1]
        assert rtrace == want
    # and both equal the oracle
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, k, T1 + T2, r0=r0)
    assert [int(x) for x in K.loads_to_numpy(r, g.n, plan.width)] == [int(x) for x in ref["r"]]
    assert (res.size, res.dens_num.value, res.ub_num.value) == (ref["size"], ref["dens_num"], ref["ub_num"])
    plan.close()
    tree.close()


def test_resume_rejects_checkpoint_above_r0_max(K):
    g = synth.chung_lu(800, 6000, 2.3, seed=32, planted=12)
    tree = K.Tree(g, 3)
    plan = K.Plan(tree, 5, r0_max=10)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    start = np.full(g.n, 3, dtype=np.uint64)
    start[17] = 11
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    say("resume with a checkpoint load above r0_max")
    with pytest.raises(K.KdssError) as e:
        plan.resume(ws, 3, 4, dev_u64(start), r, order)
    assert e.value.status == K.EOVERFLOW
    # refused before any iteration: the loads are the start loads
    assert np.array_equal(host_u64(r, g.n), start)
    plan.close()
    tree.close()


def test_start_loads_above_r0_max_refused_before_iterating(K):
    g = synth.chung_lu(800, 6000, 2.3, seed=33, planted=12)
    tree = K.Tree(g, 4)
    plan = K.Plan(tree, 9, r0_max=100)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    r0 = np.full(g.n, 100, dtype=np.uint64)
    r0[g.n - 1] = 2**63
    say("start loads above r0_max")
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(K.KdssError) as e:
        plan.run(ws, 9, r, order, r0=dev_u64(r0))
    assert e.value.status == K.EOVERFLOW
    torch.cuda.synchronize()
    assert np.array_equal(host_u64(r, g.n), r0)
    # the plan still runs correctly afterwards
    r0[g.n - 1] = 100
    res, _ = plan.run(ws, 9, r, order, r0=dev_u64(r0))
    torch.cuda.synchronize()
    assert int(host_u64(r, g.n).astype(object).sum()) - 100 * g.n == 9 * tree.stats().c_k.value
    plan.close()
    tree.close()


@pytest.mark.parametrize("width", [0, 128])
def test_one_shot_solve(K, oracle_mod, width):
    g = synth.erdos_renyi(200, 0.08, seed=0, planted_clique=12)
    rs = synth.Stream(5, 97)
    r0 = (rs.u64(g.n) % np.uint64(9)).astype(np.uint64)
    say(f"kdss_solve width={width}")
    res, r, order = K.solve_one_shot(g, 3, 30, r0=r0, width=width)
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, 3, 30, r0=r0)
    assert res.width == (128 if width else 64)
    assert [int(x) for x in r] == [int(x) for x in ref["r"]]
    assert np.array_equal(order, ref["order"])
    assert (res.size, res.dens_num.value, res.ub_num.value) == (ref["size"], ref["dens_num"], ref["ub_num"])


def test_timed_run_matches_untimed(K, oracle_mod):
    """Kernel-attached events (time_kernels) change nothing in the results and
    give one leaf-credit and one load-update duration per iteration."""
    g = synth.chung_lu(5000, 40000, 2.3, seed=34, planted=25)
    tree = K.Tree(g, 4)
    T = 12
    plain = K.Plan(tree, T)
    timed = K.Plan(tree, T, time_kernels=True)
    outs = []
    for plan in (plain, timed):
        ws = plan.alloc_workspace()
        plan.upload(ws)
        res, _, r, order = _run(K, plan, ws, T, g.n)
        outs.append((res, host_u64(r, g.n), order.cpu().numpy()))
    say("timed run")
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])
    assert (outs[0][0].size, outs[0][0].dens_num.value) == (outs[1][0].size, outs[1][0].dens_num.value)
    tm = timed.timing(reset=True)
    assert tm.leaf_launches == T and tm.apply_launches == T
    assert tm.leaf_ms > 0 and tm.heavy_ms > 0 and tm.apply_ms > 0 and tm.reduce_ms == 0
    assert timed.timing().leaf_launches == 0
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, 4, T)
    assert np.array_equal(outs[1][1], ref["r"])


def test_tuning_cache(K, tmp_path):
    """A tuned launch is filed under the plan's key and applied from the file."""
    g = synth.chung_lu(5000, 40000, 2.3, seed=35, planted=25)
    tree = K.Tree(g, 4)
    plan = K.Plan(tree, 16)
    ws = plan.alloc_workspace()
    plan.upload(ws)
    r = plan.alloc_loads()
    key = plan.tune_key()
    assert key.startswith("gfx") and "|k4|" in key
    cache = str(tmp_path / "tune.txt")
    say("tuning cache: tune and file")
    a, hit = plan.autotune_cached(ws, r, warm=3, iters=2, cache_path=cache)
    assert not hit and a.tried >= 20
    line = open(cache).read().split()
    assert line[0] == key and int(line[1]) == a.best_leaf_blocks and int(line[2]) == a.best_heavy_blocks
    assert (int(line[3]), int(line[4]), int(line[5])) == (a.best_gather, a.best_schedule, a.best_heavy)
    assert a.best_heavy in (1, 2, 3) and all(a.heavy_ms[m] > 0 for m in range(3))
    plan2 = K.Plan(tree, 16)
    b, hit = plan2.autotune_cached(ws, r, warm=3, iters=2, cache_path=cache)
    assert hit and (b.best_leaf_blocks, b.best_heavy_blocks, b.best_gather, b.best_heavy) == \
        (a.best_leaf_blocks, a.best_heavy_blocks, a.best_gather, a.best_heavy)
    assert plan2.stats().gather == a.best_gather and plan2.stats().heavy == a.best_heavy
