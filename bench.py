"""Benchmark: synchronous Frank-Wolfe over the k-pruned SCT on one MI355X.

Workload (default, batch-512): 512 Chung-Lu power-law graphs (n uniform in
[1000, 50000], average degree 8-40, exponent 2.2-2.8, seeds 1000 + g), each at
k = 3, 4, 6 and 8: 2048 problems, 3.3e8 leaves and 5.0e9 members per iteration,
in one plan with one launch per kernel per iteration; T = 64; u32 ids, u64
loads.  The other configurations are named workloads (--workload): chung-lu-1m
(n = 1,000,000, m = 10,000,000, exponent 2.5, planted 40-node near-clique,
k = 5, T = 200), er-200, rmat-16, gnn-warm-2m, and the paper's other parts.

A step is one whole pass of the hot path on inputs already resident in HBM:
start loads, T leaf-credit + load-update iterations, and the extraction
(radix sort, prefix clique counts, exact best prefix).  The clique-tree build
on the host is reported separately (the paper also excludes it).

Prints one JSON line: SCT-leaf updates/s (leaves * T per second of step time),
the leaf-credit kernel's roofline figures from kernel-attached HIP events over
the timed steps, and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_WAVE_INSTS = 256 * 2.4e9     # one wave64 VALU instruction per CU per cycle
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_2403_05775_amd", "csrc", "kernels.hip")

WORKLOADS = {
    "chung-lu-1m": dict(kind="chung_lu", n=1_000_000, m=10_000_000, beta=2.5, seed=0, planted=40,
                        planted_p=0.9, k=5, T=200),
    "er-200": dict(kind="er", n=200, p=0.08, seed=0, planted=12, k=3, T=64, cpu_full=True),
    # the paper's own update rule (PBUpdate, synchronous over the tree's pairs)
    # on the default workload's graph; the oracle's synchronous pass samples 5
    # iterations
    "pbupdate-1m": dict(kind="chung_lu", n=1_000_000, m=10_000_000, beta=2.5, seed=0, planted=40,
                        planted_p=0.9, k=5, T=200, update=1, cpu_iters=5),
    # CPSample (Algorithm 4): 2,000,000 k-color path samples (draw seed 1) on
    # R-MAT scale 16 at k = 4, then Frank-Wolfe over the distinct sampled
    # cliques; on the Chung-Lu default graph only about 3e-5 of the paths are
    # cliques at k = 5, too few to use
    "cpsample-rmat16": dict(kind="sample", graph=dict(kind="rmat", scale=16, edge_factor=8, seed=0), k=4,
                            t=2_000_000, draw_seed=1, T=64),
    # the clique tree of the default workload's graph built on the GPU (one
    # thread per start node); a step is one whole build, host order included
    "sctbuild-1m": dict(kind="sctbuild", graph=dict(kind="chung_lu", n=1_000_000, m=10_000_000, beta=2.5, seed=0,
                                                    planted=40, planted_p=0.9), k=5),
    # 512 Chung-Lu graphs (n in [1k, 50k], average degree 8-40, exponent 2.2-2.8,
    # seeds 1000 + g), each at k = 3, 4, 6, 8: 2048 problems in one plan
    "batch-512": dict(kind="batch", graphs=512, ks=(3, 4, 6, 8), T=64),
    # R-MAT (a, b, c) = (0.57, 0.19, 0.19), edge factor 8, seed 0, k = 6, T = 100,
    # at scale 16: the scale-27 graph's clique tree is far beyond host memory
    # (members grow about 28x per two scales); the oracle samples 1 iteration
    "rmat-16": dict(kind="rmat", scale=16, edge_factor=8, seed=0, k=6, T=100, cpu_iters=1),
    # the same family at scale 18 (262,144 nodes, 1,969,522 edges): the largest
    # scale whose k = 6 clique tree (8.3e8 leaves, 1.02e10 members, a 44 GB
    # leaf stream) one GPU holds; scale 19 needs about 200 GB of stream plus a
    # 61 GB heavy-leaf queue, and scale 27 about 10^19 members (tree-growth mode)
    "rmat-18": dict(kind="rmat", scale=18, edge_factor=8, seed=0, k=6, T=100, cpu_iters=0),
    # warm start vs cold start on an unseen Chung-Lu graph, n = 2M, m = 40M,
    # exponent 2.5, seed 90000; k = 6; the reference density is the best over a
    # 4T cold run with an extraction after every iteration
    "gnn-warm-2m": dict(kind="gnn", n=2_000_000, m=40_000_000, beta=2.5, seed=90000, k=6, T=200, t0=50,
                        gap=0.01),
}


def _batch_graph(i):
    from paper_2403_05775_amd import synth
    return synth.batch_member(i)


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """Threads the oracle uses: the box's share (at most 16), or fewer cores."""
    return min(16, os.cpu_count() or 1)


def rooflines(tm, L, M, n, width=64, concurrent=False):
    """HBM roofline fractions from the kernel durations of the timed region
    (kernel-attached HIP events; averages per launch), with the algorithmic
    bytes of one iteration: the leaf stream (4 B per member, 4 B per leaf
    header) and w B per node to read the loads, plus w B per node to write them
    in the load update (w = 8 for 64-bit loads).  concurrent: the pass's two
    kernels run side by side (PBUpdate), so the pass takes the longer of them."""
    nl = max(1, tm.leaf_launches)
    leaf_us = 1000.0 * tm.leaf_ms / nl
    heavy_us = 1000.0 * tm.heavy_ms / nl
    reduce_us = 1000.0 * tm.reduce_ms / nl
    apply_us = 1000.0 * tm.apply_ms / max(1, tm.apply_launches)
    w = width // 8
    pass_bytes = 4 * M + 4 * L + w * n
    iter_bytes = pass_bytes + w * n
    pass_us = (max(leaf_us, heavy_us) if concurrent else leaf_us + heavy_us) + reduce_us
    iter_us = pass_us + apply_us

    def frac(b, us):
        gbs = b / (us * 1e-6) / 1e9 if us > 0 else 0.0
        return gbs, gbs / HBM_PEAK_GBS

    a_leaf, f_leaf = frac(pass_bytes, leaf_us)
    a_pass, f_pass = frac(pass_bytes, pass_us)
    a_iter, f_iter = frac(iter_bytes, iter_us)
    return dict(leaf_us=leaf_us, heavy_us=heavy_us, reduce_us=reduce_us, apply_us=apply_us, pass_bytes=pass_bytes,
                iter_bytes=iter_bytes, leaf=(a_leaf, f_leaf), credit_pass=(a_pass, f_pass, pass_us),
                iteration=(a_iter, f_iter, iter_us), heavy_per_iter=tm.heavy_leaves / nl)


def roofline_fields(rf, kernel, workload, counters_key):
    """The line's roofline object (the leaf-credit kernel) and the two wider scopes."""
    traffic = counter_field(counters_key, "hbm_bytes_per_launch")
    valu = counter_field(counters_key, "valu_insts_per_launch")
    out = {"roofline": {"bound": "hbm", "achieved": rf["leaf"][0], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": rf["leaf"][1], "traffic": traffic, "kernel": kernel,
                        "bytes_per_launch": rf["pass_bytes"], "us_per_launch": rf["leaf_us"],
                        "timing": "kernel-attached HIP events (hipExtLaunchKernel) over the timed steps"},
           "credit_pass": {"kernels": ("pb_kernel beside pb_reg_kernel (two streams; the longer counts)"
                                       if kernel == "pb_kernel" else "leaf_credit + heavy_leaf")
                                      + (" + hot_reduce" if rf["reduce_us"] else ""),
                           "us": rf["credit_pass"][2], "achieved": rf["credit_pass"][0], "frac": rf["credit_pass"][1]},
           "iteration": {"kernels": "credit pass + load update", "us": rf["iteration"][2],
                         "bytes": rf["iter_bytes"], "achieved": rf["iteration"][0], "frac": rf["iteration"][1]},
           "kernel_us": {"leaf_credit": rf["leaf_us"], "heavy_leaf": rf["heavy_us"],
                         "hot_reduce": rf["reduce_us"] or None, "apply": rf["apply_us"]},
           "heavy_leaves_per_iteration": rf["heavy_per_iter"]}
    if valu:
        # one wave64 VALU instruction per CU per cycle: 256 CUs x 2.4 GHz
        peak = VALU_PEAK_WAVE_INSTS
        got = valu / (rf["leaf_us"] * 1e-6)
        out["valu_issue"] = {"bound": "alu", "insts_per_launch": valu, "achieved": got, "peak": peak,
                             "unit": "wave-instructions/s", "frac": got / peak,
                             "formula": "SQ_INSTS_VALU per launch / leaf-credit duration; peak = 256 CUs x "
                                        "2.4e9 cycles/s x 1 wave64 VALU instruction per CU per cycle"}
    return out


def batch_bench(w, args):
    """The batch workload: all problems in one plan, one launch per kernel per
    iteration; a step runs T iterations and every problem's extraction."""
    import concurrent.futures as cf
    import torch
    from paper_2403_05775_amd import kdss
    t0 = time.time()
    count = args.batch_graphs or w["graphs"]
    with cf.ProcessPoolExecutor(max_workers=host_cores()) as ex:
        graphs = list(ex.map(_batch_graph, range(count), chunksize=4))
    log(f"{count} graphs generated ({time.time() - t0:.1f} s), total n={sum(g.n for g in graphs)}")
    t1 = time.time()
    jobs = [(g, k) for g in graphs for k in w["ks"]]
    with cf.ThreadPoolExecutor(max_workers=host_cores()) as ex:
        trees = list(ex.map(lambda gk: kdss.Tree(gk[0], gk[1], threads=1), jobs))
    build_s = time.time() - t1
    L = sum(t.stats().leaves for t in trees)
    M = sum(t.stats().members for t in trees)
    cks = [t.stats().c_k.value for t in trees]
    log(f"{len(trees)} trees built in {build_s:.1f} s: leaves={L} members={M}")
    T = w["T"]
    t2 = time.time()
    b = kdss.Batch(trees, T, use_graph=args.graph, schedule=args.schedule, gather=launch_gather(args),
                   heavy=args.heavy)
    plan_s = time.time() - t2
    n_total = b.n
    for t in trees:
        t.close()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ws = b.alloc_workspace(dev)
    b.upload(ws)
    r = torch.empty(n_total, dtype=torch.int64, device=dev)
    order = torch.empty(n_total, dtype=torch.int32, device=dev)
    tune, cached = tune_launch(b, ws, r, T, args)
    st = b.stats()
    log(f"plan {plan_s:.1f} s, workspace {b.workspace_bytes / 1e9:.1f} GB, key mode {st.key_mode}")
    for i in range(args.warmup):
        b.run(ws, T, r, order)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for i in range(args.steps):
        res = b.run(ws, T, r, order)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - ts) / args.steps
    tm = profiled_steps(b, lambda: b.run(ws, T, r, order), args)
    step_bytes = T * (4 * M + 4 * L + 16 * n_total) + (4 * M + 4 * L)
    out = {
        "metric": "SCT-leaf updates/s", "value": L * T / (ms / 1000.0), "unit": "leaf-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"batch-512: {count} Chung-Lu graphs (n in [1000, 50000], average degree 8-40, "
                               f"exponent 2.2-2.8, seeds 1000+g) x k in {list(w['ks'])}, T={T}",
                   "problems": len(jobs), "n_total": n_total, "leaves": L, "members": M,
                   "key_mode": st.key_mode, "gather": "masked" if st.gather == 1 else "full",
                   "hot_share": round(st.hot_share, 4), "heavy_leaves": heavy_name(st.heavy),
                   "parallelism": "single GPU, one launch per kernel per iteration for all problems",
                   "hip_graph_iterations": args.graph},
        "hbm_gbps_algorithmic": step_bytes / (ms / 1000.0) / 1e9,
        "host_build_s": build_s, "plan_s": plan_s,
        "launch": launch_fields(tune, cached),
        "size_classes": size_classes(st),
        "densest_sizes_first8": [x.size for x in res[:8]],
    }
    if tm is not None:
        out["kernel_ms_per_step"] = kernel_time_sum(tm) / args.steps
        out["kernel_time_within_step"] = kernel_time_sum(tm) / args.steps <= ms * 1.001
        rf = rooflines(tm, L, M, n_total)
        out.update(roofline_fields(rf, "leaf_credit_kernel<KPacked>", "batch-512", "batch-512"))
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline_batch(jobs, cks, T)
    print(json.dumps(out))


def size_classes(ps):
    """Leaves, members and lane tiles per size class s = h + p."""
    return {name: {"leaves": int(ps.leaves[c]), "members": int(ps.members[c]), "tiles": int(ps.tiles[c])}
            for c, name in enumerate(("s<=8", "s<=16", "s<=32", "s<=64", "s>64"))}


def tune_launch(plan, ws, r, T, args):
    """Grid sizes and gather mode: from the committed tuning cache when it holds
    this plan's key, else timed on the plan's own data at steady state (T/2
    untimed iterations from zero loads, then 5 timed) and filed in the cache;
    always outside the timed region."""
    if args.launch:
        lb, hb, ga = (int(x) for x in args.launch.split(","))
        plan.set_launch(lb, hb)
        log(f"launch: leaf {lb} heavy {hb} (given), gather {plan.stats().gather}, schedule {plan.stats().schedule}")
        return None, False
    if args.no_autotune or T < 8:
        return None, False
    warm = max(3, T // 2)
    iters = min(5, T - warm)
    cache = args.tune_cache or None
    if cache:
        tune, cached = plan.autotune_cached(ws, r, warm=warm, iters=iters, cache_path=cache)
    else:
        tune, cached = plan.autotune(ws, r, warm=warm, iters=iters), False
    log(f"launch: leaf {tune.best_leaf_blocks} heavy {tune.best_heavy_blocks} gather {tune.best_gather} "
        f"({'tuning cache' if cached else f'tuned, {tune.best_ms * 1000:.2f} us/iter'}; key {plan.tune_key()})")
    return tune, cached


def launch_gather(args):
    return int(args.launch.split(",")[2]) if args.launch else 0


HEAVY_MODES = {1: "queue", 2: "in place", 3: "queue, eight per batch"}


def heavy_name(mode):
    """Where leaves with more than four low members are credited."""
    return {1: "queued for the heavy kernel (four per batch)", 2: "in place, by the tile's wavefront",
            3: "queued for the heavy kernel (eight per batch)"}[mode]


def launch_fields(tune, cached):
    if tune is None:
        return "defaults"
    out = {"leaf_blocks": tune.best_leaf_blocks, "heavy_blocks": tune.best_heavy_blocks,
           "gather": "masked" if tune.best_gather == 1 else "full",
           "schedule": "strided" if tune.best_schedule == 1 else "XCD ranges",
           "heavy_leaves": HEAVY_MODES[tune.best_heavy], "from_tuning_cache": cached,
           "tuned_us_per_iter": tune.best_ms * 1000}
    if not cached:
        out["gather_us"] = {"masked": tune.gather_ms[0] * 1000, "full": tune.gather_ms[1] * 1000}
        out["schedule_us"] = {"strided": tune.schedule_ms[0] * 1000, "XCD ranges": tune.schedule_ms[1] * 1000}
        out["heavy_us"] = {HEAVY_MODES[m]: tune.heavy_ms[m - 1] * 1000 for m in (1, 2, 3)}
    return out


def cpu_baseline_batch(jobs, cks, T, budget_s=15.0):
    """The oracle (clique listing, then T synchronous iterations and the
    extraction) on a bounded sample of the batch's problems: problems in a
    seeded shuffle, skipping those with more than 2e7 k-cliques (listing
    memory), until budget_s seconds of iterations + extraction; listing
    excluded as the tree build is on the GPU side."""
    import numpy as np
    from oracle import oracle as O
    O.build()
    cores = host_cores()
    rng = np.random.default_rng(2048)
    idx = [int(q) for q in rng.permutation(len(jobs)) if 0 < cks[int(q)] <= 2e7]
    leaves_done, secs, listing, probs = 0, 0.0, 0.0, 0
    from paper_2403_05775_amd import kdss
    for q in idx:
        g, k = jobs[q]
        res = O.solve(g.n, g.row_ptr, g.col, k, T, threads=cores)
        secs += res["iter_seconds"] + res["extract_seconds"]
        listing += res["enum_seconds"]
        leaves_done += kdss.tree_count(g, k).leaves
        probs += 1
        if secs >= budget_s:
            break
    return dict(value=leaves_done * T / secs, unit="leaf-updates/s", cores=cores, kind="oracle",
                cpu=cpu_model(),
                sample=f"{probs} of the {len(jobs)} problems (seeded shuffle, c_k <= 2e7), each {T} synchronous "
                       f"iterations + extraction ({secs:.1f} s); leaves counted as the GPU plan's; the oracle's "
                       f"k-clique listing ({listing:.1f} s) excluded", seconds=secs)


def _within(K, i, K_ref, i_ref, gap):
    """K / i >= (1 - gap) K_ref / i_ref, exactly (gap rounded to ten-thousandths)."""
    h = round(gap * 10000)
    return 10000 * K * i_ref >= (10000 - h) * K_ref * i


def gnn_bench(w, args):
    """Time to a 1% density gap from the model's warm start vs from zero loads.

    Untimed: the graph, its tree, a 4T cold reference run (extraction after
    every iteration) that fixes rho_ref and the cold iteration count t_c, and a
    warm trace that fixes t_w (t_w = 0 when the start loads alone are within the
    gap).  Timed, each on inputs resident in HBM: cold = t_c iterations plus the
    extraction; warm = features + model + r0 + t_w iterations plus the
    extraction.  The tree build is excluded from both."""
    import numpy as np
    import torch
    from paper_2403_05775_amd import gnn, kdss, synth
    k, T, t0, gap = w["k"], w["T"], w["t0"], (args.gap or w["gap"])
    t_start = time.time()
    g = synth.chung_lu(w["n"], w["m"], w["beta"], seed=w["seed"])
    log(f"graph {g.name}: n={g.n} m={g.m} ({time.time() - t_start:.1f} s)")
    tree = kdss.Tree(g, k)
    ts = tree.stats()
    log(f"tree k={k}: leaves={ts.leaves} members={ts.members} c_k={ts.c_k.value} build={ts.build_seconds:.1f} s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rp = torch.from_numpy(g.row_ptr.astype(np.int64)).to(dev)
    col = torch.from_numpy(g.col.view(np.int32)).to(dev)
    nnz = int(g.row_ptr[-1])
    n = g.n
    model = gnn.Model(device=dev)
    wfile = args.gnn_weights or gnn.WEIGHTS_FILE
    trained = os.path.exists(wfile) and not args.gnn_untrained
    meta = {}
    if trained:
        with np.load(wfile) as z:
            model.load(z)
            meta = {x: z[x].item() for x in z.files if x.startswith("meta_")}
    log(f"model: {'trained ' + str(meta) if trained else 'untrained (random init)'}")
    order = torch.empty(n, dtype=torch.int32, device=dev)

    def free(plan):
        plan.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    # reference: 4T cold iterations, extraction after each
    Tref = 4 * T
    pref = kdss.Plan(tree, Tref, extract_every=1)
    ws = pref.alloc_workspace(dev)
    pref.upload(ws)
    r = pref.alloc_loads(dev)
    _, trace = pref.run(ws, Tref, r, order, trace_cap=Tref + 1)
    best = trace[0]
    for row in trace:
        if row["dens_num"] * best["size"] > best["dens_num"] * row["size"]:
            best = row
    K_ref, i_ref = best["dens_num"], best["size"]
    t_cold = next(row["t"] for row in trace if _within(row["dens_num"], row["size"], K_ref, i_ref, gap))
    r_ref = kdss.loads_to_numpy(r, n, pref.width)
    r_ref = np.asarray(r_ref, dtype=np.float64)
    ideal = np.rint(t0 * r_ref / Tref).astype(np.uint64)
    log(f"cold reference: rho_ref={K_ref}/{i_ref}={K_ref / max(i_ref, 1):.2f} (best at t={best['t']}), "
        f"t_cold={t_cold}")
    del ws, r
    free(pref)

    # warm traces: the model's start and the start taken from the reference loads
    dg = gnn.DeviceGraph.resident(n, rp, col, nnz)
    fset = int(meta.get("meta_feature_set", 0))
    dg.x0 = gnn.features(tree, rp, col, nnz, fset)
    r0, rmax = model.warm_start(dg, t0)
    r0_ideal = torch.from_numpy(ideal.view(np.int64)).to(dev)
    pw = kdss.Plan(tree, Tref, r0_max=max(rmax, int(ideal.max())), extract_every=1)
    assert pw.width == 64
    ws = pw.alloc_workspace(dev)
    pw.upload(ws)
    r = pw.alloc_loads(dev)

    def first_within(start):
        res0 = pw.extract(ws, start, order, 1, r0=start)
        curve = [(0, res0.dens_num.value, res0.size)]
        if _within(res0.dens_num.value, res0.size, K_ref, i_ref, gap):
            return 0, curve
        _, tr = pw.run(ws, Tref, r, order, r0=start, trace_cap=Tref + 1)
        curve += [(row["t"], row["dens_num"], row["size"]) for row in tr]
        for t, K, i in curve:
            if _within(K, i, K_ref, i_ref, gap):
                return t, curve
        return None, curve

    t_warm, curve_w = first_within(r0)
    t_ideal, _ = first_within(r0_ideal)
    log(f"warm: t_warm={t_warm} (start density {curve_w[0][1]}/{curve_w[0][2]}), "
        f"reference-loads start: t={t_ideal}")
    del ws, r, r0_ideal
    free(pw)

    # timed runs (no per-iteration extraction)
    t_run = max(1, t_cold, t_warm or 1)
    pt = kdss.Plan(tree, t_run, r0_max=rmax)
    ws = pt.alloc_workspace(dev)
    pt.upload(ws)
    r = pt.alloc_loads(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    parts = {"features": 0.0, "model": 0.0, "frank_wolfe_and_extraction": 0.0}

    def cold_once():
        res, _ = pt.run(ws, t_cold, r, order)
        return res

    def warm_once(split=False):
        ev[0].record()
        dg.x0 = gnn.features(tree, rp, col, nnz, fset)
        ev[1].record()
        r0w, _ = model.warm_start(dg, t0, sync=False)
        ev[2].record()
        if t_warm == 0:
            res = pt.extract(ws, r0w, order, 1, r0=r0w)
        else:
            res, _ = pt.run(ws, t_warm, r, order, r0=r0w)
        ev[3].record()
        if split:
            torch.cuda.synchronize()
            parts["features"] += ev[0].elapsed_time(ev[1])
            parts["model"] += ev[1].elapsed_time(ev[2])
            parts["frank_wolfe_and_extraction"] += ev[2].elapsed_time(ev[3])
        return res

    def timed(fn, **kw):
        for _ in range(args.warmup):
            fn(**kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            res = fn(**kw)
        torch.cuda.synchronize()
        return 1000.0 * (time.perf_counter() - t1) / args.steps, res

    cold_ms, res_c = timed(cold_once)
    warm_ms = None
    res_w = None
    if t_warm is not None:
        warm_ms, res_w = timed(warm_once)
        for _ in range(max(1, args.steps)):
            warm_once(split=True)
        for key in parts:
            parts[key] /= max(1, args.steps)
    log(f"cold {cold_ms:.2f} ms ({t_cold} iterations), warm {warm_ms} ms ({t_warm} iterations)")
    out = {
        "metric": "time to 1% density gap, GNN-warm vs cold PSCTL",
        "value": warm_ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": warm_ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 loads; bf16 model with fp32 accumulation", "data": "synthetic",
        "config": {"workload": f"gnn-warm-2m: {g.name}, k={k}, gap {gap:.1%}", "n": n, "m": g.m, "k": k,
                   "leaves": ts.leaves, "members": ts.members, "c_k": ts.c_k.value, "t0": t0,
                   "reference_iterations": Tref, "parallelism": "single GPU"},
        "cold_ms": cold_ms, "speedup": (cold_ms / warm_ms) if warm_ms else None,
        "t_cold": t_cold, "t_warm": t_warm, "t_start_from_reference_loads": t_ideal,
        "rho_ref": [K_ref, i_ref], "rho_cold": [res_c.dens_num.value, res_c.size],
        "rho_warm": [res_w.dens_num.value, res_w.size] if res_w is not None else None,
        "warm_breakdown_ms": parts if warm_ms else None,
        "model": {"trained": trained, **meta},
        "sct_build_s": ts.build_seconds,
    }
    print(json.dumps(out))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_graph(w):
    from paper_2403_05775_amd import synth
    if w["kind"] == "chung_lu":
        return synth.chung_lu(w["n"], w["m"], w["beta"], seed=w["seed"], planted=w["planted"],
                              planted_p=w["planted_p"])
    if w["kind"] == "rmat":
        return synth.rmat(w["scale"], w["edge_factor"], seed=w["seed"])
    return synth.erdos_renyi(w["n"], w["p"], seed=w["seed"], planted_clique=w["planted"])


def kernel_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def sample_bench(w, args):
    """CPSample: the sample tree is built once (sampler timed on its own, like
    the tree build); a step runs T Frank-Wolfe iterations over the distinct
    sampled cliques and the rho'_k extraction."""
    import numpy as np
    import torch
    from paper_2403_05775_amd import kdss, synth
    g = make_graph(w["graph"])
    k, t, T = w["k"], w["t"], w["T"]
    draws = synth.sample_draws(w["draw_seed"], t, k)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tree = kdss.SampleTree(g, k, draws)
    tree.close()
    tree = kdss.SampleTree(g, k, draws)   # the second build is the timed one (the first loads the kernels)
    info = tree.info
    L = tree.stats().leaves
    log(f"{t} samples: {info.cliques} cliques, {info.distinct} distinct, {info.paths.value} colour-increasing "
        f"paths, {info.colors} colours; device {info.device_seconds:.3f} s, host {info.host_seconds:.3f} s")
    plan = kdss.Plan(tree, T, use_graph=True)
    ws = plan.alloc_workspace(dev)
    plan.upload(ws)
    r = plan.alloc_loads(dev)
    order = torch.empty(g.n, dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        res, _ = plan.run(ws, T, r, order)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, _ = plan.run(ws, T, r, order)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / args.steps
    out = {
        "metric": "SCT-leaf updates/s", "value": L * T / (ms / 1000.0), "unit": "leaf-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"cpsample-rmat16: {g.name}, k={k}, {t} samples, T={T}", "n": g.n, "m": g.m, "k": k,
                   "samples": t, "T": T, "leaves": L, "parallelism": "single GPU, hipGraph iterations"},
        "sampler": {"cliques": info.cliques, "distinct": info.distinct, "paths": info.paths.value,
                    "colors": info.colors, "device_s": info.device_seconds, "host_s": info.host_seconds,
                    "samples_per_s_device": t / info.device_seconds if info.device_seconds else None,
                    "clique_fraction": info.cliques / t if t else 0.0},
        "result": {"size": res.size, "dens_num": res.dens_num.value, "density_sampled": res.density},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        O.build()
        h, p, mem = tree.export()
        cl = mem.reshape(-1, k)
        s0 = time.perf_counter()
        O.solve_list(g.n, cl, k, T)
        secs = time.perf_counter() - s0
        out["cpu_baseline"] = dict(value=L * T / secs, unit="leaf-updates/s", cores=1, kind="oracle",
                                   sample=f"the same distinct sample set, {T} synchronous Frank-Wolfe iterations "
                                          f"and the extraction ({secs:.2f} s), one thread", seconds=secs)
    tree.close()
    print(json.dumps(out))


def sctbuild_bench(w, args):
    """The GPU clique-tree build: a step is one kdss_sct_build_gpu call (host
    degeneracy order, device orientation and recursion, leaves back to the
    host); the figure is k-cliques covered per second.  The host build of the
    same tree is timed beside it, and the CPU baseline is the oracle counting
    the same k-cliques."""
    import torch
    from paper_2403_05775_amd import kdss
    g = make_graph(w["graph"])
    k = w["k"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    for _ in range(max(1, args.warmup)):
        kdss.GpuTree(g, k).close()
    secs = []
    for _ in range(args.steps):
        t = kdss.GpuTree(g, k)
        st = t.stats()
        secs.append(st.build_seconds)
        t.close()
    ms = 1000.0 * sum(secs) / len(secs)
    host = kdss.Tree(g, k)
    hs = host.stats()
    host.close()
    ck = st.c_k.value
    log(f"GPU tree build: {ms:.1f} ms ({st.leaves} leaves, {st.members} members, degeneracy {st.degeneracy}); "
        f"host build {1000 * hs.build_seconds:.1f} ms")
    out = {
        "metric": "k-cliques covered by the built tree per second", "value": ck / (ms / 1000.0),
        "unit": "k-cliques/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"sctbuild-1m: {g.name}, k={k}", "n": g.n, "m": g.m, "k": k, "c_k": ck,
                   "leaves": st.leaves, "members": st.members, "degeneracy": st.degeneracy,
                   "parallelism": "single GPU"},
        "host_build_ms": 1000.0 * hs.build_seconds,
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        O.build()
        cores = min(16, os.cpu_count() or 1)
        s0 = time.perf_counter()
        n_or = O.count(g.n, g.row_ptr, g.col, k, threads=cores)
        secs_or = time.perf_counter() - s0
        if n_or != ck:
            raise SystemExit(f"the oracle counts {n_or} k-cliques, the GPU tree covers {ck}")
        out["cpu_baseline"] = dict(value=ck / secs_or, unit="k-cliques/s", cores=cores, kind="oracle",
                                   sample=f"the same graph and k: the oracle's k-clique count ({secs_or:.2f} s)",
                                   seconds=secs_or)
    print(json.dumps(out))


def counters_file(workload):
    return os.path.join(PROFILES, f"leaf_credit_{workload}_counters.txt")


def counter_field(workload, field):
    """A per-launch figure of the leaf-credit kernel from the committed
    rocprofv3 counter runs, only while they describe the current kernel source."""
    path = counters_file(workload)
    if not os.path.exists(path):
        return None
    c = json.load(open(path))
    if c.get("kernel_sha256_16") != kernel_hash() or c.get("workload") != workload:
        return None
    return c.get(field)


def cpu_baseline_pb(g, w, tree, L, sample_T):
    """The CPU oracle's synchronous PBUpdate over the same pairs (the tree's
    leaves, exported), sample_T iterations."""
    from oracle import oracle as O
    O.build()
    h, p, mem = tree.export()
    res = O.pb_run(g.n, h, p, mem, w["k"], sample_T, True)
    secs = res["seconds"]
    return dict(value=L * sample_T / secs, unit="leaf-updates/s", cores=1, kind="oracle", cpu=cpu_model(),
                sample=f"same graph, k and pairs, {sample_T} synchronous PBUpdate iterations ({secs:.2f} s), "
                       f"one thread", seconds=secs)


def cpu_baseline(g, w, L, sample_T):
    """The CPU oracle (clique listing + synchronous Frank-Wolfe) on the same graph,
    sample_T iterations; listing excluded like the tree build on the GPU side."""
    from oracle import oracle as O
    O.build()
    res = O.solve(g.n, g.row_ptr, g.col, w["k"], sample_T, threads=host_cores())
    secs = res["iter_seconds"] + res["extract_seconds"]
    return dict(value=L * sample_T / secs, unit="leaf-updates/s", cores=res["threads"], kind="oracle",
                cpu=cpu_model(),
                sample=f"same graph and k, {sample_T} iterations + extraction ({secs:.2f} s); "
                       f"its k-clique listing ({res['enum_seconds']:.1f} s, c_k={res['c_k']}) excluded",
                seconds=secs, listing_seconds=res["enum_seconds"])


def cpu_baseline_full(g, w, L, budget_s=5.0):
    """A workload the oracle finishes in milliseconds: the whole run (listing,
    T iterations, extraction), repeated for about budget_s seconds, on one
    core and on all of the machine's cores."""
    from oracle import oracle as O
    O.build()
    out = {}
    for label, threads in (("single_core", 1), ("all_cores", host_cores())):
        reps, secs = 0, 0.0
        while secs < budget_s or reps < 3:
            s0 = time.perf_counter()
            O.solve(g.n, g.row_ptr, g.col, w["k"], w["T"], threads=threads)
            secs += time.perf_counter() - s0
            reps += 1
        out[label] = dict(value=L * w["T"] * reps / secs, ms_per_run=1000.0 * secs / reps, cores=threads, runs=reps)
    best = out["all_cores"]
    return dict(value=best["value"], unit="leaf-updates/s", cores=best["cores"], kind="oracle", cpu=cpu_model(),
                sample=f"the whole workload (listing, {w['T']} iterations, extraction), {best['runs']} runs",
                seconds=best["ms_per_run"] / 1000.0, single_core=out["single_core"], all_cores=out["all_cores"])


def counters_mode(w, args):
    """A short run for rocprofv3 counter passes: the bench's launch (tuning
    cache), then 20 iterations of the workload (the last 20 leaf-credit
    dispatches), then a plain 1 GiB device copy (three times) that calibrates
    the byte counters."""
    import torch
    from paper_2403_05775_amd import kdss
    if w["kind"] == "batch":
        import concurrent.futures as cf
        count = args.batch_graphs or w["graphs"]
        with cf.ProcessPoolExecutor(max_workers=host_cores()) as ex:
            graphs = list(ex.map(_batch_graph, range(count), chunksize=4))
        jobs = [(g, k) for g in graphs for k in w["ks"]]
        with cf.ThreadPoolExecutor(max_workers=host_cores()) as ex:
            trees = list(ex.map(lambda gk: kdss.Tree(gk[0], gk[1], threads=1), jobs))
        plan = kdss.Batch(trees, w["T"])
        n = plan.n
    else:
        g = make_graph(w)
        plan = kdss.Plan(kdss.Tree(g, w["k"]), w["T"])
        n = g.n
    ws = plan.alloc_workspace("cuda:0")
    plan.upload(ws)
    r = torch.empty(max(n, 1) * (2 if plan.width == 128 else 1), dtype=torch.int64, device="cuda:0")
    order = torch.empty(max(n, 1), dtype=torch.int32, device="cuda:0")
    tune_launch(plan, ws, r, w["T"], args)
    if w["kind"] == "batch":
        plan.run(ws, 20, r, order)
    else:
        plan.run(ws, 20, r, order)
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counters_run": "done", "workload": w}))


def _db_rows(db):
    import sqlite3
    c = sqlite3.connect(db)
    cols = [r[1] for r in c.execute("pragma table_info(counters_collection)")]
    ki, ci, vi, di = (cols.index(x) for x in ("kernel_name", "counter_name", "value", "dispatch_id"))
    per = {}
    for row in c.execute("select * from counters_collection"):
        key = (row[ki], row[di])
        per[key] = per.get(key, 0.0) + row[vi]
    return per


def summarize_counters(workload, fetch_db, write_db, valu_db, command):
    """Per-launch HBM bytes of the leaf-credit kernel from FETCH_SIZE / WRITE_SIZE
    runs, each divided by the factor the same counter shows for a 1 GiB copy,
    and its VALU wave-instructions (SQ_INSTS_VALU) per launch."""
    out = {"workload": workload, "kernel_sha256_16": kernel_hash(), "command": command}

    def leaf_values(db):
        per = _db_rows(db)
        # the last 20 dispatches: the run after the tuning launches
        leaf = [v for (k, d), v in sorted(per.items(), key=lambda kv: kv[0][1])
                if "leaf_credit_kernel" in k and "KPacked" in k][-20:]
        other = [v for (k, d), v in per.items() if "anonymous namespace" not in k]
        return leaf, (max(other) if other else None)

    for name, db in (("fetch", fetch_db), ("write", write_db)):
        leaf, copy = leaf_values(db)
        leaf_kib = sum(leaf) / len(leaf)
        factor = copy * 1024.0 / COPY_BYTES if copy else None
        out[name] = {"leaf_kib_per_dispatch": leaf_kib, "dispatches": len(leaf), "copy_kib": copy,
                     "copy_bytes": COPY_BYTES, "factor": factor,
                     "bytes_per_launch": leaf_kib * 1024.0 / factor if factor else None}
    out["hbm_bytes_per_launch"] = out["fetch"]["bytes_per_launch"] + out["write"]["bytes_per_launch"]
    if valu_db:
        leaf, _ = leaf_values(valu_db)
        out["valu_insts_per_launch"] = sum(leaf) / len(leaf)
    return out


def summarize_trace(db, command, bench_json=None):
    """Kernel-trace statistics (rocprofv3 --kernel-trace --stats) as markdown;
    with the JSON line the traced bench printed, also its launch and its own
    (kernel-attached event) per-launch durations, to compare."""
    import sqlite3
    c = sqlite3.connect(db)
    lines = ["# Kernel trace: " + command, "",
             "Durations from the dispatch records (end - start), per kernel and grid size "
             "(the tuning launches run the other grid sizes).", "",
             "| kernel | workgroups | calls | total us | average us | min us | max us |",
             "|---|---|---|---|---|---|---|"]
    rows = c.execute("select name, grid_x / max(workgroup_x, 1), count(*), sum(end - start), avg(end - start), "
                     "min(end - start), max(end - start) from kernels group by name, grid_x "
                     "order by sum(end - start) desc limit 30")
    for name, wg, calls, tot, avg, mn, mx in rows:
        short = name.replace("(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| {short} | {wg} | {calls} | {tot / 1e3:.1f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | "
                     f"{mx / 1e3:.2f} |")
    if bench_json:
        try:
            line = json.loads(open(bench_json).read().strip().splitlines()[-1])
        except (OSError, ValueError, IndexError):
            line = None
        if line:
            lines += ["", "The traced bench's own line (same run):", "",
                      f"- launch: {json.dumps(line.get('launch'))}",
                      f"- per-launch durations from kernel-attached events, us: {json.dumps(line.get('kernel_us'))}",
                      f"- ms_per_step {line.get('ms_per_step'):.3f} (under the profiler), roofline frac "
                      f"{(line.get('roofline') or {}).get('frac')}"]
    return "\n".join(lines) + "\n"


COPY_BYTES = 1 << 30


def tree_growth(args):
    """Sizes of the k-pruned clique tree of R-MAT graphs (a, b, c) = (0.57, 0.19,
    0.19), edge factor 8, seed 0, over a range of scales, counted without
    building the tree (kdss_sct_count, host threads); a log-linear fit of leaves,
    members and c_k per scale step extrapolates to scale 27, where the leaf
    stream (4 B per member + 4 B per leaf, read by every iteration) is compared
    with one GPU's 288 GB of HBM."""
    import math
    from paper_2403_05775_amd import kdss, synth
    lo, hi = (int(x) for x in args.scales.split("-"))
    rows = []
    for sc in range(lo, hi + 1):
        t0 = time.time()
        g = synth.rmat(sc, 8, seed=0)
        gen_s = time.time() - t0
        st = kdss.tree_count(g, args.k)
        row = dict(scale=sc, n=g.n, m=g.m, leaves=st.leaves, members=st.members, s_max=st.s_max,
                   degeneracy=st.degeneracy, c_k=st.c_k.value, count_s=round(st.build_seconds, 2),
                   generate_s=round(gen_s, 2))
        rows.append(row)
        log(json.dumps(row))

    def fit(key):
        pts = [(r["scale"], math.log(r[key])) for r in rows if r[key] > 0][-3:]
        xs, ys = [p[0] for p in pts], [p[1] for p in pts]
        xm, ym = sum(xs) / len(xs), sum(ys) / len(ys)
        b = sum((x - xm) * (y - ym) for x, y in pts) / max(1e-12, sum((x - xm) ** 2 for x in xs))
        return math.exp(b), (lambda sc: math.exp(ym + b * (sc - xm)))

    out = {"mode": "tree-growth", "k": args.k, "graph": "R-MAT (0.57, 0.19, 0.19), edge factor 8, seed 0",
           "rows": rows, "fit_on_scales": [r["scale"] for r in rows][-3:]}
    target = 27
    ext = {}
    for key in ("leaves", "members", "c_k"):
        f, at = fit(key)
        ext[key] = {"growth_per_scale": f, "at_scale_27": at(target)}
    stream_bytes = 4 * ext["members"]["at_scale_27"] + 4 * ext["leaves"]["at_scale_27"]
    out["extrapolated"] = ext
    out["scale_27_leaf_stream_bytes"] = stream_bytes
    out["hbm_bytes"] = 288e9
    out["scale_27_fits_one_gpu"] = stream_bytes < 288e9
    out["largest_scale_fitting_288GB"] = max(
        (sc for sc in range(lo, target + 1)
         if 4 * fit("members")[1](sc) + 4 * fit("leaves")[1](sc) < 288e9), default=None)
    print(json.dumps(out))


def single_bench(w, args):
    """One plan (one graph, one k): a step is start loads + T iterations + the
    extraction on inputs resident in HBM.  The timed steps launch plainly; the
    same number of steps after them, with kernel-attached HIP events on every
    iteration kernel, give the per-launch durations of the roofline fields."""
    import torch
    from paper_2403_05775_amd import kdss
    t0 = time.time()
    g = make_graph(w)
    log(f"graph {g.name}: n={g.n} m={g.m} ({time.time() - t0:.1f} s)")
    tree = kdss.Tree(g, w["k"])
    ts = tree.stats()
    log(f"tree k={w['k']}: leaves={ts.leaves} members={ts.members} s_max={ts.s_max} "
        f"c_k={ts.c_k.value} build={ts.build_seconds:.2f} s")
    T = w["T"]
    update = w.get("update", 0)
    plan = kdss.Plan(tree, T, use_graph=args.graph, update=update, schedule=args.schedule, gather=launch_gather(args),
                     heavy=args.heavy)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ws = plan.alloc_workspace(dev)
    plan.upload(ws)
    r = plan.alloc_loads(dev)
    order = torch.empty(g.n, dtype=torch.int32, device=dev)
    tune, cached = tune_launch(plan, ws, r, T, args)
    ps = plan.stats()
    for i in range(args.warmup):
        res, _ = plan.run(ws, T, r, order)
        log(f"warmup {i + 1}/{args.warmup}: size={res.size} density={res.density:.3f}")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        res, _ = plan.run(ws, T, r, order)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1000.0 * elapsed / args.steps
    tm = profiled_steps(plan, lambda: plan.run(ws, T, r, order), args)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step; i*={res.size} "
        f"density={res.dens_num.value}/{res.size}={res.density:.4f} ub={res.upper_bound:.4f}")
    L, M, n = ts.leaves, ts.members, g.n
    step_bytes = T * (4 * M + 4 * L + 16 * n) + (4 * M + 4 * L)
    out = {
        "metric": "SCT-leaf updates/s",
        "value": L * T / (ms_per_step / 1000.0),
        "unit": "leaf-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {g.name}, k={w['k']}, T={T}", "n": n, "m": g.m,
                   "k": w["k"], "T": T, "leaves": L, "members": M, "c_k": ts.c_k.value,
                   "parallelism": "single GPU", "hip_graph_iterations": args.graph,
                   "gather": "masked" if ps.gather == 1 else "full", "hot_share": round(ps.hot_share, 4),
                   "heavy_leaves": heavy_name(ps.heavy),
                   "update": "PBUpdate (synchronous)" if update else "Frank-Wolfe"},
        "hbm_gbps_algorithmic": step_bytes / (ms_per_step / 1000.0) / 1e9,
        "sct_build_s": ts.build_seconds,
        "result": {"size": res.size, "dens_num": res.dens_num.value, "ub_num": res.ub_num.value,
                   "density": res.density, "upper_bound": res.upper_bound,
                   "bound": {"num": res.bound_num.value, "den": res.bound_den, "value": res.bound,
                             "kind": "top-s" if res.bound_kind == 1 else "max load",
                             "certified_optimal": bool(res.certified),
                             "gap": (res.bound - res.density) / res.bound if res.bound else 0.0}},
        "size_classes": size_classes(ps),
        "launch": launch_fields(tune, cached),
        "cpu_baseline": None,
    }
    if tm is not None:
        # the kernels of a step fit inside it (a profiler attached to the run
        # can stretch the event-stamped steps; the line then says so)
        # (PBUpdate's two pass kernels run side by side: the longer one counts)
        out["kernel_time_within_step"] = kernel_time_sum(tm, bool(update)) / args.steps <= ms_per_step * 1.001
        rf = rooflines(tm, L, M, n, ps.width, concurrent=bool(update))
        kname = "pb_kernel" if update else "leaf_credit_kernel<KPacked>"
        out.update(roofline_fields(rf, kname, args.workload, args.workload))
        out["kernel_ms_per_step"] = kernel_time_sum(tm, bool(update)) / args.steps
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        if update:
            out["cpu_baseline"] = cpu_baseline_pb(g, w, tree, L, w.get("cpu_iters", args.cpu_sample_iters))
        elif w.get("cpu_full"):
            out["cpu_baseline"] = cpu_baseline_full(g, w, L)
        elif w.get("cpu_iters") == 0:
            out["cpu_baseline"] = None
            out["cpu_baseline_skipped"] = (f"the oracle would list all {ts.c_k.value} k-cliques for every iteration "
                                           f"(about 1.5e7 per second on 16 threads: over half an hour per iteration)")
        else:
            out["cpu_baseline"] = cpu_baseline(g, w, L, w.get("cpu_iters", args.cpu_sample_iters))
    print(json.dumps(out))


def kernel_time_sum(tm, concurrent=False):
    """Kernel time of the timed steps; with concurrent pass kernels (PBUpdate)
    the pass counts as the longer of its two kernels."""
    pass_ms = max(tm.leaf_ms, tm.heavy_ms) if concurrent else tm.leaf_ms + tm.heavy_ms
    return pass_ms + tm.reduce_ms + tm.apply_ms


def profiled_steps(plan, step, args):
    """Right after the timed steps, the same number of steps of the same plan
    (same launch) with kernel-attached HIP events on every iteration kernel:
    the runtime stamps each dispatch's own start and end, so the durations are
    the kernels' execution spans (what rocprofv3's kernel trace reports).  The
    events cost time between kernels, so the step time comes from the plain
    steps before (timed steps launch plainly, also when the plain steps replay
    graphs)."""
    import torch
    plan.set_timing(True)
    plan.timing(reset=True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    tm = plan.timing(reset=True)
    plan.set_timing(False)
    return tm


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch-512", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=20)
    ap.add_argument("--graph", type=int, default=0, metavar="G",
                    help="replay the iterations as hipGraphs of G iterations (0: plain launches)")
    ap.add_argument("--no-autotune", action="store_true", help="default grid sizes and gather mode")
    ap.add_argument("--launch", default="", help="LEAF,HEAVY,GATHER: a given launch instead of the tuned one")
    ap.add_argument("--schedule", type=int, default=0, help="tile schedule: 0 tuned, 1 strided, 2 XCD ranges")
    ap.add_argument("--heavy", type=int, default=0,
                    help="heavy leaves: 0 tuned, 1 queued for the heavy kernel, 2 in place by the tile's wavefront, "
                         "3 queued, eight per heavy-kernel batch")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2403_05775_amd", "tune_cache.txt"),
                    help="tuning cache file ('' to tune without one)")
    ap.add_argument("--scales", default="12-20", help="tree-growth mode: R-MAT scales lo-hi")
    ap.add_argument("--k", type=int, default=6, help="tree-growth mode: clique size")
    ap.add_argument("--mode", default="bench", choices=["bench", "counters", "tree-growth"],
                    help="counters: short run for rocprofv3 --pmc passes (with a copy calibration)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DB", "WRITE_DB", "VALU_DB"))
    ap.add_argument("--summarize-trace", metavar="DB")
    ap.add_argument("--bench-json", default="", help="summarize-trace: the traced bench's JSON output")
    ap.add_argument("--command", default="", help="command line recorded in a summary")
    ap.add_argument("--out", default="")
    ap.add_argument("--batch-graphs", type=int, default=0, help="graphs in the batch workload (default 512)")
    ap.add_argument("--gnn-untrained", action="store_true", help="warm start from a randomly initialised model")
    ap.add_argument("--gnn-weights", default="", help="warm-start weights (.npz; default: the package's)")
    ap.add_argument("--gap", type=float, default=0.0, help="warm-start workload: density gap (default 0.01)")
    args = ap.parse_args()
    if args.summarize_counters:
        res = summarize_counters(args.workload, *args.summarize_counters, args.command)
        with open(args.out or counters_file(args.workload), "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res))
        return
    if args.summarize_trace:
        md = summarize_trace(args.summarize_trace, args.command, args.bench_json or None)
        if args.out:
            open(args.out, "w").write(md)
        print(md)
        return
    if args.mode == "tree-growth":
        tree_growth(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    w = WORKLOADS[args.workload]
    if args.mode == "counters":
        counters_mode(w, args)
        return
    kind = w["kind"]
    if kind == "batch":
        batch_bench(w, args)
    elif kind == "sample":
        sample_bench(w, args)
    elif kind == "sctbuild":
        sctbuild_bench(w, args)
    elif kind == "gnn":
        gnn_bench(w, args)
    else:
        single_bench(w, args)


if __name__ == "__main__":
    main()
