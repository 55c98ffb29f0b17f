"""kdss_run_static (the entry point for callers that cannot allocate device
memory) against kdss_run on the same plans: loads, order and every result
field equal, on two calls in a row (the second on a smaller problem, so the
static workspace holds the first call's leftovers), with start loads and with
128-bit loads; a plan larger than the static workspace is refused."""
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


def fields(res):
    return (res.T, res.size, res.n, res.width, res.dens_num.value, res.ub_num.value, res.c_k.value,
            res.bound_num.value, res.bound_den, res.bound_kind, res.certified)


def both(K, g, k, T, r0=None, width=0, heavy=0, update=0):
    tree = K.Tree(g, k)
    r0_max = 0 if r0 is None else int(r0.max())
    plan = K.Plan(tree, T, r0_max=r0_max, width=width, use_graph=True, heavy=heavy, update=update)
    assert plan.workspace_bytes <= K.STATIC_WORKSPACE_BYTES
    r0_t = None if r0 is None else torch.from_numpy(r0.view(np.int64).copy()).cuda()
    # the static entry point first: nothing of this plan is in any workspace yet
    rs = plan.alloc_loads()
    os_ = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    got = plan.run_static(T, rs, os_, r0=r0_t)
    torch.cuda.synchronize()
    ws = plan.alloc_workspace()
    plan.upload(ws)
    rw = plan.alloc_loads()
    ow = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    want, _ = plan.run(ws, T, rw, ow, r0=r0_t)
    torch.cuda.synchronize()
    assert np.array_equal(rs.cpu().numpy(), rw.cpu().numpy())
    assert np.array_equal(os_.cpu().numpy(), ow.cpu().numpy())
    assert fields(got) == fields(want)
    plan.close()
    tree.close()
    return got


def test_static_run_twice_second_smaller(K, oracle_mod):
    big = synth.chung_lu(20000, 160000, 2.3, seed=41, planted=30)
    small = synth.erdos_renyi(200, 0.08, seed=0, planted_clique=12)
    say("static run: 20k-node Chung-Lu, k=4, T=30")
    a = both(K, big, 4, 30)
    say("static run: ER(200) + K12, k=3, T=64")
    b = both(K, small, 3, 64)
    ref = oracle_mod.solve(small.n, small.row_ptr, small.col, 3, 64)
    assert (b.size, b.dens_num.value, b.ub_num.value) == (ref["size"], ref["dens_num"], ref["ub_num"])
    assert a.n == big.n


def test_static_run_heavy_leaves_in_place(K, oracle_mod):
    """The static entry point with heavy leaves taken up in place (no heavy
    kernel in the replayed iterations) equals kdss_run and the oracle."""
    g = synth.chung_lu(6000, 50000, 2.2, seed=43, planted=28)
    say("static run: 6k-node Chung-Lu, k=5, T=20, heavy leaves in place")
    got = both(K, g, 5, 20, heavy=2)
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, 5, 20)
    assert (got.size, got.dens_num.value, got.ub_num.value) == (ref["size"], ref["dens_num"], ref["ub_num"])


def test_static_run_pbupdate(K, oracle_mod):
    """PBUpdate through the static entry point (its two pass kernels one after
    the other on the caller's stream) equals kdss_run (side by side on two
    streams, replayed as a graph) and the oracle's synchronous pass."""
    g = synth.chung_lu(6000, 50000, 2.2, seed=44, planted=28)
    say("static run: 6k-node Chung-Lu, k=4, T=15, PBUpdate")
    got = both(K, g, 4, 15, update=1)
    tree = K.Tree(g, 4)
    h, p, mem = tree.export()
    tree.close()
    r = oracle_mod.pb_run(g.n, h, p, mem, 4, 15, True)["r"]
    ex = oracle_mod.extract(g.n, g.row_ptr, g.col, 4, r)
    assert (got.size, got.dens_num.value) == (ex["size"], ex["dens_num"])


def test_static_run_start_loads_and_wide(K):
    g = synth.chung_lu(3000, 24000, 2.3, seed=42, planted=20)
    rs = synth.Stream(42, 99)
    r0 = (rs.u64(g.n) % np.uint64(50)).astype(np.uint64)
    say("static run: start loads")
    both(K, g, 4, 12, r0=r0)
    say("static run: 128-bit loads")
    both(K, synth.erdos_renyi(500, 0.05, seed=3, planted_clique=10), 3, 9, width=128)


def test_static_run_rejects_oversized_plan(K):
    g = synth.chung_lu(1_500_000, 3_000_000, 2.5, seed=43)
    tree = K.Tree(g, 3)
    plan = K.Plan(tree, 10)
    assert plan.workspace_bytes > K.STATIC_WORKSPACE_BYTES
    r = plan.alloc_loads()
    order = torch.empty(g.n, dtype=torch.int32, device="cuda")
    say("static run: oversized plan")
    with pytest.raises(K.KdssError) as e:
        plan.run_static(10, r, order)
    assert e.value.status == K.ERANGE
    plan.close()
    tree.close()
