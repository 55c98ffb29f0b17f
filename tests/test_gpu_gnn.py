"""Warm-start model kernels against FP32 references (BF16 operands, FP32 accumulation).

Tolerances follow from the arithmetic: inputs are exact BF16 values and sums are
FP32, so a GEMM output differs from the FP32 reference by at most its BF16
rounding (relative 2^-8) plus FP32 summation-order error; reductions over many
rows (weight gradients) are compared at a relative 1e-3."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2403_05775_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_05775_amd import gnn
    gnn._lib()
    return gnn


def rand_bf16(G, shape, seed, scale=1.0):
    rs = synth.Stream(seed, 5)
    x = torch.from_numpy(((rs.uniform(int(np.prod(shape))) * 2 - 1) * scale).astype(np.float32).reshape(shape))
    return G.float_to_bf16_rne(x).cuda()


def f(G, t):
    return G.bf16_to_float(t.cpu())


def test_bf16_rounding_ties_to_even(G):
    """FP32 -> BF16 in the kernels rounds to nearest, ties to even (IEEE definition)."""
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -2.5, 3.0e38, 1e-40, 0.0, -0.0,
                     1 + 2 ** -8 + 2 ** -20, 65504.0, 1.00390625], dtype=np.float32)
    w32 = torch.zeros((1, 64), dtype=torch.float32)
    w32[0, : vals.size] = torch.from_numpy(vals)
    w32 = w32.cuda()
    w16 = torch.empty((1, 64), dtype=torch.int16, device="cuda")
    G._ck(G._lib().kdss_gnn_pack_weights(1, G._p(w32), G._p(w16), None, G._s()), "pack")
    torch.cuda.synchronize()
    got = w16.cpu().numpy().view(np.uint16)[0, : vals.size]
    u = vals.view(np.uint32).astype(np.uint64)
    want = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    assert np.array_equal(got, want)
    assert got[1] == 0x3F80 and got[2] == 0x3F82   # 1 + 2^-8 ties down to even, 1 + 3 * 2^-8 up


@pytest.mark.parametrize("M,K1,K2,relu", [(1000, 32, 32, 1), (777, 64, 64, 1), (4096, 64, 0, 0), (33, 64, 64, 0),
                                          (2049, 8, 8, 1)])
def test_linear_matches_fp32(G, M, K1, K2, relu):
    a1 = rand_bf16(G, (M, K1), 1)
    a2 = rand_bf16(G, (M, max(K2, 8)), 2)[:, :K2].contiguous() if K2 else None
    K = K1 + K2
    bt = rand_bf16(G, (64, K), 3, 0.2)
    bias = torch.from_numpy(np.linspace(-0.5, 0.5, 64).astype(np.float32)).cuda()
    y = torch.empty((M, 64), dtype=torch.int16, device="cuda")
    G._ck(G._lib().kdss_gnn_linear(M, G._p(a1), K1, K1, G._p(a2), K2, max(K2, 1) if K2 else 0, G._p(bt),
                                   G._p(bias), relu, G._p(y), 64, G._s()), "linear")
    torch.cuda.synchronize()
    x = f(G, a1) if not K2 else torch.cat([f(G, a1), f(G, a2)], 1)
    ref = x.double() @ f(G, bt).double().T + bias.cpu().double()
    if relu:
        ref = ref.clamp_min(0)
    got = f(G, y).double()
    assert torch.all((got - ref).abs() <= 2 ** -8 * ref.abs() + 1e-5), (got - ref).abs().max()


@pytest.mark.parametrize("M,K1,K2", [(5000, 32, 32), (3333, 64, 64), (4001, 8, 8)])
def test_weight_gradient(G, M, K1, K2):
    a1 = rand_bf16(G, (M, K1), 4)
    a2 = rand_bf16(G, (M, K2), 5)
    dy = rand_bf16(G, (M, 64), 6)
    dw = torch.zeros((K1 + K2, 64), dtype=torch.float32, device="cuda")
    db = torch.zeros(64, dtype=torch.float32, device="cuda")
    G._ck(G._lib().kdss_gnn_linear_wgrad(M, G._p(a1), K1, K1, G._p(a2), K2, K2, G._p(dy), G._p(dw), G._p(db),
                                         G._s()), "wgrad")
    torch.cuda.synchronize()
    x = torch.cat([f(G, a1), f(G, a2)], 1).double()
    d = f(G, dy).double()
    ref = x.T @ d
    assert torch.allclose(dw.cpu().double(), ref, rtol=1e-3, atol=1e-3)
    assert torch.allclose(db.cpu().double(), d.sum(0), rtol=1e-3, atol=1e-3)


def small_graph():
    return synth.chung_lu(3000, 20000, 2.3, seed=21, planted=20)


def test_aggregate_and_transpose(G):
    g = small_graph()
    dg_rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
    dg_col = torch.from_numpy(g.col.view(np.int32)).cuda()
    n = g.n
    deg = np.diff(g.row_ptr.astype(np.int64))
    for F in (8, 16, 32, 64):
        h = rand_bf16(G, (n, F), 7)
        out = torch.empty((n, F), dtype=torch.int16, device="cuda")
        G._ck(G._lib().kdss_gnn_aggregate(n, G._p(dg_rp), G._p(dg_col), G._p(h), F, G._p(out), G._s()), "agg")
        torch.cuda.synchronize()
        hf = f(G, h).double().numpy()
        ref = np.zeros((n, F))
        rp = g.row_ptr.astype(np.int64)
        for u in range(n):
            if deg[u]:
                ref[u] = hf[g.col[rp[u]:rp[u + 1]]].mean(0)
        got = f(G, out).double().numpy()
        assert np.all(np.abs(got - ref) <= 2 ** -8 * np.abs(ref) + 1e-5)
        # transpose: <agg(h), d> == <h, agg^T(d)> up to rounding
        d = rand_bf16(G, (n, 2 * F), 8)
        outb = torch.empty((n, F), dtype=torch.int16, device="cuda")
        G._ck(G._lib().kdss_gnn_aggregate_backward(n, G._p(dg_rp), G._p(dg_col), G._p(d[:, F:]), G._p(d), F,
                                                   2 * F, G._p(outb), G._s()), "agg backward")
        torch.cuda.synchronize()
        df = f(G, d).double().numpy()
        refb = df[:, :F].copy()
        for u in range(n):
            if deg[u]:
                refb[g.col[rp[u]:rp[u + 1]]] += df[u, F:] / deg[u]
        gotb = f(G, outb).double().numpy()
        assert np.all(np.abs(gotb - refb) <= 2 ** -8 * np.abs(refb) + 1e-4)


@pytest.mark.parametrize("size", ["small", "many-chunks"])
def test_features_triangles(G, oracle_mod, size):
    """Column 2 is log1p of the triangles through each node (triangles listed by the
    oracle).  The larger graph has more than 256 scan chunks of 2048 offsets and
    rows longer than one wavefront."""
    from paper_2403_05775_amd import kdss
    g = small_graph() if size == "small" else synth.chung_lu(600_000, 1_500_000, 2.5, seed=22)
    tree = kdss.Tree(g, 3)
    x0 = G.features(tree, torch.from_numpy(g.row_ptr.astype(np.int64)).cuda(),
                    torch.from_numpy(g.col.view(np.int32)).cuda(), int(g.row_ptr[-1]))
    torch.cuda.synchronize()
    tri = np.zeros(g.n, dtype=np.int64)
    for c in oracle_mod.list_cliques(g.n, g.row_ptr, g.col, 3):
        tri[c] += 1
    core = tree.core_numbers()
    deg = np.diff(g.row_ptr.astype(np.int64))
    got = f(G, x0).numpy()
    want = np.stack([np.log1p(deg), np.log1p(core), np.log1p(tri)], 1).astype(np.float32)
    want16 = G.bf16_to_float(G.float_to_bf16_rne(torch.from_numpy(want))).numpy()
    assert np.allclose(got[:, :3], want16, rtol=2 ** -7, atol=1e-6)
    assert np.all(got[:, 3:] == 0)


def test_model_gradients_match_reference(G):
    """Full forward/backward of the kernels vs a float64 torch model that rounds
    activations to BF16 at the same points (finite parameters, same data)."""
    from paper_2403_05775_amd import kdss
    g = small_graph()
    tree = kdss.Tree(g, 5)
    dg = G.DeviceGraph(g, tree)
    dg.target = torch.linspace(0, 3, g.n, dtype=torch.float32, device="cuda")
    model = G.Model(seed=3)
    model.zero_grad()
    pred, acts = model.forward(dg)
    loss = model.backward(dg, pred, acts, dg.target)
    torch.cuda.synchronize()
    # reference
    n = g.n
    rp = g.row_ptr.astype(np.int64)
    deg = torch.from_numpy(np.maximum(np.diff(rp), 1)).double()
    rows = torch.from_numpy(np.repeat(np.arange(n), np.diff(rp)))
    cols = torch.from_numpy(g.col.astype(np.int64))
    A = torch.sparse_coo_tensor(torch.stack([rows, cols]), torch.ones(cols.numel(), dtype=torch.float64),
                                (n, n)).coalesce()

    def r16(x):
        return G.bf16_to_float(G.float_to_bf16_rne(x.float())).double()

    def st(x):   # rounded value forward, identity gradient backward
        return r16(x.detach()) + (x - x.detach())

    params = [p.cpu().double().clone().requires_grad_(True) for p in model.params]
    h = f(G, dg.x0).double()
    for li in range(3):
        agg = st(torch.sparse.mm(A, h) / deg[:, None])
        W = params[2 * li]
        Wr = r16(W.detach())  # the kernels use the BF16 copy of W
        y = torch.cat([h, agg], 1) @ (Wr + (W - W.detach())) + params[2 * li + 1]
        h = st(torch.relu(y))
    predr = h @ params[6][:64] + params[6][64]
    lref = ((predr - dg.target.cpu().double()) ** 2).mean()
    lref.backward()
    lref = float(lref.detach())
    assert abs(float(loss.item()) - lref) <= 1e-2 * lref
    assert torch.allclose(pred.cpu().double(), predr.detach(), rtol=2e-2, atol=2e-2)
    for gk, pr in zip(model.grads, params):
        ref = pr.grad
        scale = ref.abs().max().item() + 1e-6
        assert (gk.cpu().double() - ref).abs().max().item() <= 0.05 * scale


def test_training_reduces_loss_and_warm_start(G, oracle_mod):
    from paper_2403_05775_amd import kdss
    graphs = [synth.chung_lu(2000 + 300 * i, 15000 + 2000 * i, 2.3, seed=40 + i, planted=15) for i in range(4)]
    data = []
    for g in graphs:
        tree = kdss.Tree(g, 4)
        dg = G.DeviceGraph(g, tree)
        dg.loads, dg.T = G.cold_loads(g, tree, 30), 30
        w = dg.loads.to(torch.float64)
        dg.target = torch.log1p(w / 30).to(torch.float32)
        data.append(dg)
    model = G.Model(seed=1)
    hist = G.train(model, data, epochs=12, lr=3e-3, log=lambda *_: None)
    assert hist[-1] < hist[0]
    # the warm start is an ordinary start load: the run stays exact
    g = graphs[0]
    r0, rmax = model.warm_start(data[0], t0=5)
    torch.cuda.synchronize()
    r0h = r0.cpu().numpy().view(np.uint64)
    assert rmax == int(r0h.max())
    sol = kdss.solve(g, 4, 9, r0=r0h)
    ref = oracle_mod.solve(g.n, g.row_ptr, g.col, 4, 9, r0=r0h)
    assert np.array_equal(sol.r, ref["r"]) and (sol.size, sol.dens_num) == (ref["size"], ref["dens_num"])


def test_library_step_equals_kernel_by_kernel_step(G):
    """kdss_gnn_train_step (label, forward, backward, Adam in one call) against
    the same kernels called one by one: the label transform log1p(r / T) is
    compared with float64, the loss and parameters after the step within the
    float atomics' reordering, and kdss_gnn_infer's prediction and integer
    start loads with the forward pass and kdss_gnn_warm_start bit for bit."""
    from paper_2403_05775_amd import kdss
    g = synth.chung_lu(3000, 24000, 2.3, seed=44, planted=15)
    tree = kdss.Tree(g, 4)
    dg = G.DeviceGraph(g, tree)
    dg.loads, dg.T = G.cold_loads(g, tree, 25), 25
    r = dg.loads.cpu().numpy().view(np.uint64).astype(np.float64)
    dg.target = torch.from_numpy(np.log1p(r / 25).astype(np.float32)).cuda()
    a, b = G.Model(seed=5), G.Model(seed=5)
    # library step
    loss_a = torch.zeros(1, dtype=torch.float32, device="cuda")
    a.train_step(dg, 2e-3, loss_a)
    # kernel by kernel
    b.zero_grad()
    pred, acts = b.forward(dg)
    loss_b = b.backward(dg, pred, acts, dg.target)
    b.adam(2e-3)
    torch.cuda.synchronize()
    assert abs(float(loss_a.item()) - float(loss_b.item())) <= 1e-5 * float(loss_b.item())
    assert torch.allclose(a.flat, b.flat, rtol=1e-4, atol=1e-6)
    # inference: the same forward kernels, so the same bits
    pa = torch.empty(g.n, dtype=torch.float32, device="cuda")
    r0a, ma = a.warm_start(dg, 40, pred=pa)
    a.pack()   # the kernel-level forward reads the BF16 copies of the current weights
    pb, _ = a.forward(dg)
    r0b = torch.empty(g.n, dtype=torch.int64, device="cuda")
    mb = torch.zeros(1, dtype=torch.int64, device="cuda")
    G._ck(G._lib().kdss_gnn_warm_start(g.n, G._p(pb), 40.0, 1 << 62, G._p(r0b), G._p(mb), G._s()), "warm start")
    torch.cuda.synchronize()
    assert torch.equal(pa, pb) and torch.equal(r0a, r0b) and ma == int(mb.item())


def test_feature_set_without_triangles(G):
    """Feature set 1 keeps degree and core number and leaves the triangle column 0."""
    from paper_2403_05775_amd import kdss
    g = small_graph()
    tree = kdss.Tree(g, 3)
    rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
    col = torch.from_numpy(g.col.view(np.int32)).cuda()
    nnz = int(g.row_ptr[-1])
    x0 = G.features(tree, rp, col, nnz, 0)
    x1 = G.features(tree, rp, col, nnz, 1)
    torch.cuda.synchronize()
    assert torch.equal(x0[:, :2], x1[:, :2]) and torch.equal(x0[:, 3:], x1[:, 3:])
    assert int((x1[:, 2] != 0).sum()) == 0 and int((x0[:, 2] != 0).sum()) > 0
