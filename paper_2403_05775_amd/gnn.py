"""Warm start for Frank-Wolfe from a small message-passing network.

Orchestration only: every feature, layer, gradient and optimiser step runs in
the HIP kernels of libkdss.so (``include/kdss_gnn.h``); torch holds the device
buffers.  The model predicts y(u) ~ log1p(r*(u) / T) -- the per-iteration load
of node u after a long cold run -- and the warm start is
r0 = round(t0 * expm1(y)), fed to ``kdss_run`` unchanged, so the method's
arithmetic (and exactness) is untouched.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import time

import numpy as np

from . import kdss, synth

HIDDEN = 64
F0 = 8           # feature columns (3 used, padded to one 8-wide matrix-core step)
LAYERS = [(F0, F0), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN)]   # (self columns, neighbour columns)
WEIGHTS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gnn_weights.npz")
PARAMS = 17665   # KDSS_GNN_PARAMS

_bound = False


def _lib():
    global _bound
    L = kdss.lib()
    if not _bound:
        vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
        L.kdss_gnn_features_workspace.argtypes = [u32, u64, C.POINTER(C.c_size_t)]
        L.kdss_gnn_features.argtypes = [vp, vp, vp, u64, C.c_int, vp, vp, C.c_size_t, vp]
        L.kdss_gnn_model_workspace.argtypes = [u32, C.c_int, C.POINTER(C.c_size_t)]
        L.kdss_gnn_infer.argtypes = [u32, vp, vp, vp, vp, C.c_double, u64, vp, C.c_size_t, vp, vp, vp, vp]
        L.kdss_gnn_train_step.argtypes = [u32, vp, vp, vp, vp, u32, vp, vp, vp, u32, C.c_float, vp, C.c_size_t,
                                          vp, vp]
        L.kdss_gnn_aggregate.argtypes = [u32, vp, vp, vp, u32, vp, vp]
        L.kdss_gnn_aggregate_backward.argtypes = [u32, vp, vp, vp, vp, u32, u32, vp, vp]
        L.kdss_gnn_linear.argtypes = [u32, vp, u32, u32, vp, u32, u32, vp, vp, C.c_int, vp, u32, vp]
        L.kdss_gnn_linear_wgrad.argtypes = [u32, vp, u32, u32, vp, u32, u32, vp, vp, vp, vp]
        L.kdss_gnn_relu_backward.argtypes = [u64, vp, vp, vp]
        L.kdss_gnn_head.argtypes = [u32, vp, vp, vp, vp]
        L.kdss_gnn_head_backward.argtypes = [u32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.kdss_gnn_adam.argtypes = [u32, vp, vp, vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, u32, vp]
        L.kdss_gnn_pack_weights.argtypes = [u32, vp, vp, vp, vp]
        L.kdss_gnn_warm_start.argtypes = [u32, vp, C.c_double, u64, vp, vp, vp]
        _bound = True
    return L


def _p(t):
    return None if t is None else t.data_ptr()


def _s():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _ck(status, where):
    kdss._check(status, where)


class DeviceGraph:
    """A graph's CSR on the device, its features and (optionally) labels."""

    def __init__(self, graph, tree=None, device="cuda", feature_set=0):
        import torch
        self.n = graph.n
        self.row_ptr = torch.from_numpy(graph.row_ptr.astype(np.int64)).to(device)
        col = graph.col if graph.col.size else np.zeros(1, np.uint32)
        self.col = torch.from_numpy(col.view(np.int32)).to(device)
        own = tree is None
        tree = tree or kdss.Tree(graph, 3)
        self.nnz = int(graph.row_ptr[graph.n])
        self.x0 = features(tree, self.row_ptr, self.col, self.nnz, feature_set)
        if own:
            tree.close()
        self.target = None
        self.loads = None     # a cold run's loads (u64 as int64, device) and its T, for training
        self.T = 0

    @classmethod
    def resident(cls, n, row_ptr, col, nnz):
        """A graph whose CSR is already on the device; x0 is left for the caller."""
        self = cls.__new__(cls)
        self.n, self.row_ptr, self.col, self.nnz = n, row_ptr, col, nnz
        self.x0 = None
        self.target = None
        return self


def features(tree, d_row_ptr, d_col, nnz, feature_set=0):
    """x0 (n x 8 BF16 as int16) = log1p of degree, core number, triangle count
    (feature set 0; set 1 leaves the triangle column 0), then zeros."""
    import torch
    nbytes = C.c_size_t(0)
    _ck(_lib().kdss_gnn_features_workspace(tree.n, nnz, C.byref(nbytes)), "kdss_gnn_features_workspace")
    ws = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=d_row_ptr.device)
    x0 = torch.empty((max(tree.n, 1), F0), dtype=torch.int16, device=d_row_ptr.device)
    _ck(_lib().kdss_gnn_features(tree._h, _p(d_row_ptr), _p(d_col), nnz, feature_set, _p(x0), _p(ws), ws.numel(),
                                 _s()), "kdss_gnn_features")
    return x0[: tree.n]


def bf16_to_float(t):
    """BF16 bits held in an int16 tensor -> float32 tensor (exact)."""
    import torch
    return (t.to(torch.int32) << 16).view(torch.float32)


def float_to_bf16_rne(x):
    """float32 -> BF16 bits with round to nearest even (torch reference of the kernels' rounding)."""
    import torch
    u = x.contiguous().view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r & 0xFFFF).to(torch.int32).to(torch.int16)


class Model:
    """Parameters (FP32 masters + BF16 copies), Adam state, and the kernels' forward/backward."""

    def __init__(self, device="cuda", seed=0):
        import torch
        self.device = device
        rs = synth.Stream(seed, 77)
        host = []
        for (ks, kn) in LAYERS:
            K = ks + kn
            scale = math.sqrt(6.0 / (K + HIDDEN))
            host.append(((rs.uniform(K * HIDDEN) * 2 - 1) * scale).astype(np.float32).reshape(K, HIDDEN))
            host.append(np.zeros(HIDDEN, dtype=np.float32))
        head = ((rs.uniform(HIDDEN + 1) * 2 - 1) * math.sqrt(6.0 / (HIDDEN + 1))).astype(np.float32)
        head[HIDDEN] = 0.0
        host.append(head)
        # one flat FP32 array in the library's layout (W1 b1 W2 b2 W3 b3 head);
        # params, grads and the Adam moments are views into flat arrays
        self.flat = torch.from_numpy(np.concatenate([h.reshape(-1) for h in host])).to(device)
        assert self.flat.numel() == PARAMS
        self.flat_grad = torch.zeros_like(self.flat)
        self.flat_m = torch.zeros_like(self.flat)
        self.flat_v = torch.zeros_like(self.flat)

        def views(t):
            out, at = [], 0
            for h in host:
                out.append(t[at:at + h.size].view(h.shape))
                at += h.size
            return out
        self.params = views(self.flat)
        self.grads = views(self.flat_grad)
        self.m = views(self.flat_m)
        self.v = views(self.flat_v)
        self._ws = {}
        self.w16 = [torch.empty(p.shape, dtype=torch.int16, device=device) for p in self.params[0:6:2]]
        self.wt16 = [torch.empty((HIDDEN, p.shape[0]), dtype=torch.int16, device=device) for p in self.params[0:6:2]]
        self.step_count = 0
        self.pack()

    def pack(self):
        for i, w in enumerate(self.params[0:6:2]):
            _ck(_lib().kdss_gnn_pack_weights(w.shape[0], _p(w), _p(self.w16[i]), _p(self.wt16[i]), _s()),
                "kdss_gnn_pack_weights")

    def state(self):
        return {f"p{i}": p.cpu().numpy() for i, p in enumerate(self.params)}

    def load(self, state):
        import torch
        for i, p in enumerate(self.params):
            p.copy_(torch.from_numpy(np.asarray(state[f"p{i}"], dtype=np.float32)))
        self.pack()

    def forward(self, dg):
        """Returns (pred FP32 [n], activations for backward)."""
        import torch
        L = _lib()
        n = dg.n
        acts = []
        h, F = dg.x0, F0
        for li in range(3):
            agg = torch.empty((n, F), dtype=torch.int16, device=self.device)
            _ck(L.kdss_gnn_aggregate(n, _p(dg.row_ptr), _p(dg.col), _p(h), F, _p(agg), _s()), "aggregate")
            y = torch.empty((n, HIDDEN), dtype=torch.int16, device=self.device)
            _ck(L.kdss_gnn_linear(n, _p(h), F, F, _p(agg), F, F, _p(self.wt16[li]), _p(self.params[2 * li + 1]), 1,
                                  _p(y), HIDDEN, _s()), "linear")
            acts.append((h, agg, F, y))
            h, F = y, HIDDEN
        pred = torch.empty(n, dtype=torch.float32, device=self.device)
        _ck(L.kdss_gnn_head(n, _p(h), _p(self.params[6]), _p(pred), _s()), "head")
        return pred, acts

    def backward(self, dg, pred, acts, target):
        """Accumulates gradients into self.grads; returns the loss tensor (FP32 [1])."""
        import torch
        L = _lib()
        n = dg.n
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        h3 = acts[-1][3]
        dy = torch.empty((n, HIDDEN), dtype=torch.int16, device=self.device)
        _ck(L.kdss_gnn_head_backward(n, _p(h3), _p(self.params[6]), _p(pred), _p(target), _p(dy),
                                     _p(self.grads[6]), _p(loss), _s()), "head backward")
        for li in (2, 1, 0):
            h, agg, F, y = acts[li]
            _ck(L.kdss_gnn_relu_backward(n * HIDDEN, _p(y), _p(dy), _s()), "relu backward")
            _ck(L.kdss_gnn_linear_wgrad(n, _p(h), F, F, _p(agg), F, F, _p(dy), _p(self.grads[2 * li]),
                                        _p(self.grads[2 * li + 1]), _s()), "weight gradient")
            if li == 0:
                break
            # dX = dY W^T: 64 self columns then 64 neighbour columns (ld 128)
            dx = torch.empty((n, 2 * F), dtype=torch.int16, device=self.device)
            w16 = self.w16[li]
            _ck(L.kdss_gnn_linear(n, _p(dy), HIDDEN, HIDDEN, None, 0, 0, _p(w16[0:F]), None, 0, _p(dx), 2 * F,
                                  _s()), "data gradient")
            _ck(L.kdss_gnn_linear(n, _p(dy), HIDDEN, HIDDEN, None, 0, 0, _p(w16[F:2 * F]), None, 0,
                                  _p(dx[:, F:]), 2 * F, _s()), "data gradient")
            dh = torch.empty((n, F), dtype=torch.int16, device=self.device)
            _ck(L.kdss_gnn_aggregate_backward(n, _p(dg.row_ptr), _p(dg.col), _p(dx[:, F:]), _p(dx), F, 2 * F,
                                              _p(dh), _s()), "aggregate backward")
            dy = dh
        return loss

    def zero_grad(self):
        for g in self.grads:
            g.zero_()

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        L = _lib()
        for p, g, m, v in zip(self.params, self.grads, self.m, self.v):
            _ck(L.kdss_gnn_adam(p.numel(), _p(p), _p(g), _p(m), _p(v), lr, b1, b2, eps, self.step_count, _s()),
                "adam")
        self.pack()

    def workspace(self, n, train):
        import torch
        key = (n, bool(train))
        if key not in self._ws:
            b = C.c_size_t(0)
            _ck(_lib().kdss_gnn_model_workspace(n, 1 if train else 0, C.byref(b)), "kdss_gnn_model_workspace")
            self._ws = {key: torch.empty(b.value, dtype=torch.uint8, device=self.device)}
        return self._ws[key]

    def warm_start(self, dg, t0, cap=1 << 62, sync=True, pred=None):
        """r0 (device uint64 as int64) and its maximum (an int when sync, else the
        device scalar): the forward pass and the rounding in one library call."""
        import torch
        ws = self.workspace(dg.n, False)
        r0 = torch.empty(dg.n, dtype=torch.int64, device=self.device)
        rmax = torch.zeros(1, dtype=torch.int64, device=self.device)
        _ck(_lib().kdss_gnn_infer(dg.n, _p(dg.row_ptr), _p(dg.col), _p(dg.x0), _p(self.flat), float(t0), cap, _p(ws),
                                  ws.numel(), _p(pred), _p(r0), _p(rmax), _s()), "kdss_gnn_infer")
        return r0, (int(rmax.item()) if sync else rmax)

    def train_step(self, dg, lr, loss):
        """One Adam step on one graph (library call: label, forward, backward, Adam);
        the graph's mean squared error is added into loss (device FP32 [1])."""
        self.step_count += 1
        ws = self.workspace(dg.n, True)
        _ck(_lib().kdss_gnn_train_step(dg.n, _p(dg.row_ptr), _p(dg.col), _p(dg.x0), _p(dg.loads), dg.T,
                                       _p(self.flat), _p(self.flat_m), _p(self.flat_v), self.step_count, lr, _p(ws),
                                       ws.numel(), _p(loss), _s()), "kdss_gnn_train_step")


def cold_loads(graph, tree, T, device="cuda"):
    """A cold run's loads r_T (u64 as int64 on the device) for a graph's tree;
    the training step turns them into the target log1p(r_T / T)."""
    import torch
    plan = kdss.Plan(tree, T, width=64)
    ws = plan.alloc_workspace(device)
    plan.upload(ws)
    r = plan.alloc_loads(device)
    order = torch.empty(max(graph.n, 1), dtype=torch.int32, device=device)
    plan.run(ws, T, r, order)
    plan.close()
    return r[:graph.n]


def generate(count, base_seed=10000, n_lo=10_000, n_hi=200_000, workers=6, first=0, log=print):
    """Chung-Lu graphs first .. first + count - 1 of the seeded family (n in
    [n_lo, n_hi], average degree 8-40, exponent 2.2-2.8), made on worker threads
    (the process that drives the GPU is never forked)."""
    import concurrent.futures as cf
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        graphs = list(ex.map(_member, [(i, base_seed, n_lo, n_hi) for i in range(first, first + count)]))
    log(f"{count} graphs generated in {time.time() - t0:.0f} s")
    return graphs


def prepare(graphs, k=6, T=200, device="cuda", log=print, feature_set=0):
    """Features and cold-run loads at (k, T) on the device; the host graphs are
    released as they are consumed."""
    import torch
    out = []
    t1 = time.time()
    for i in range(len(graphs)):
        g = graphs[i]
        graphs[i] = None
        tree = kdss.Tree(g, k)
        dg = DeviceGraph(g, tree, device, feature_set)
        dg.loads = cold_loads(g, tree, T, device)
        dg.T = T
        # the target as the training step computes it (for the kernel-level path)
        w = dg.loads.to(torch.float64)
        dg.target = torch.log1p(torch.where(w < 0, w + 2.0 ** 64, w) / T).to(torch.float32)
        tree.close()
        out.append(dg)
        if len(out) % 25 == 0 or len(out) == len(graphs):
            log(f"{len(out)}/{len(graphs)} graphs labelled ({time.time() - t1:.0f} s)")
    return out


def training_set(count, k=6, T=200, base_seed=10000, n_lo=10_000, n_hi=200_000, workers=6, device="cuda",
                 first=0, log=print, feature_set=0):
    """generate() then prepare()."""
    return prepare(generate(count, base_seed, n_lo, n_hi, workers, first, log), k, T, device, log, feature_set)


def _member(args):
    i, base, lo, hi = args
    return synth.batch_member(i, base_seed=base, n_lo=lo, n_hi=hi)


def evaluate(model, data):
    """Mean loss over graphs: the forward pass in the library, the mean squared
    error against log1p(r / T)."""
    import torch
    tot = 0.0
    for dg in data:
        pred = torch.empty(dg.n, dtype=torch.float32, device=model.device)
        model.warm_start(dg, 1.0, pred=pred)
        tot += float(((pred - dg.target) ** 2).mean().item())
    return tot / max(1, len(data))


def train(model, data, epochs=3, lr=1e-3, seed=0, val=None, log=print):
    """One Adam step per graph (MSE over its nodes; one kdss_gnn_train_step
    call), graphs in a seeded shuffled order each epoch.  Returns the mean
    training loss of each epoch."""
    import torch
    rs = synth.Stream(seed, 78)
    hist = []
    loss = torch.zeros(1, dtype=torch.float32, device=model.device)
    for ep in range(epochs):
        order = rs.shuffle_order(len(data))
        loss.zero_()
        for i in order:
            model.train_step(data[int(i)], lr, loss)
        hist.append(float(loss.item()) / len(data))
        msg = f"epoch {ep + 1}: mean loss {hist[-1]:.4f}"
        if val:
            msg += f", held-out {evaluate(model, val):.4f}"
        log(msg)
    return hist


def main(argv=None):
    """Trains the model on the seeded Chung-Lu family and saves its FP32
    parameters (with the training settings as meta_* entries)."""
    import argparse
    ap = argparse.ArgumentParser(prog="python -m paper_2403_05775_amd.gnn", description=main.__doc__)
    ap.add_argument("--graphs", type=int, default=2000, help="training graphs (seeds 10000 + i)")
    ap.add_argument("--held-out", type=int, default=8, help="validation graphs (seeds 20000 + i)")
    ap.add_argument("--k", type=int, default=6)
    ap.add_argument("--T", type=int, default=200, help="cold iterations behind each label")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--workers", type=int, default=6, help="graph generator processes")
    ap.add_argument("--out", default=WEIGHTS_FILE)
    ap.add_argument("--feature-set", type=int, default=0, help="0: degree, core, triangles; 1: degree, core")
    ap.add_argument("--curve", default="", help="graph counts for a held-out loss curve, e.g. 50,100,200,300")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    g_val = generate(args.held_out, base_seed=20000, workers=args.workers, log=log)
    g_train = generate(args.graphs, workers=args.workers, log=log)
    val = prepare(g_val, k=args.k, T=args.T, log=log, feature_set=args.feature_set)
    data = prepare(g_train, k=args.k, T=args.T, log=log, feature_set=args.feature_set)
    log(f"data ready in {time.time() - t0:.0f} s")
    model = None
    if args.curve:
        # held-out loss after training on the first c graphs, for each c (the
        # run on all graphs, when listed last, is the saved model)
        curve = {}
        for c in (int(x) for x in args.curve.split(",")):
            m = Model(seed=0)
            hist = train(m, data[:c], epochs=args.epochs, lr=args.lr, log=lambda *_: None)
            curve[c] = evaluate(m, val)
            log(f"curve: {c} graphs -> held-out loss {curve[c]:.5f} (last epoch's training loss {hist[-1]:.5f})")
            if c >= len(data):
                model = m
        print("CURVE " + " ".join(f"{c}:{v:.6f}" for c, v in curve.items()), flush=True)
    if model is None:
        model = Model(seed=0)
        hist = train(model, data, epochs=args.epochs, lr=args.lr, val=val, log=log)
    state = model.state()
    state.update(meta_graphs=np.int64(args.graphs), meta_k=np.int64(args.k), meta_T=np.int64(args.T),
                 meta_epochs=np.int64(args.epochs), meta_train_loss=np.float64(hist[-1]),
                 meta_held_out_loss=np.float64(evaluate(model, val)),
                 meta_feature_set=np.int64(args.feature_set))
    np.savez(args.out, **state)
    log(f"saved {args.out} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
