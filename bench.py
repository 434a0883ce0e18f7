#!/usr/bin/env python3
"""Benchmark: MeshGraphNet processor edge-updates/s, forward + backward,
BF16 against plain FP32, 15 layers, one MI355X.

A step is one full training pass of the hot path over the workload:
forward (encoders, 15 fused edge + node processor layers, decoder), masked
MSE gradient, and the hand-written backward with all parameter gradients.
Inputs (graph, partition plan, parameters, features, targets) are resident
in HBM before the timed region starts; the kNN graph build and the
partitioner run once beforehand and are reported separately and in an
end-to-end total (kNN + partitioning + one step).

Two tape policies are timed, for both precisions, each BF16 leg against the
plain FP32 leg of the same policy: "keep" (the forward also stores every
edge's hidden activation z, so the edge adjoint skips the first product;
the headline) and "recompute" (per-layer checkpoints only, every edge MLP
recomputed in the backward).  A second form of the edge forward is timed
beside them as a variant (keep policy): "split", the first layer
re-associated over its input blocks with per-node projections of W1 (the
headline is the gathered form, which applies the 3H x H layer per edge).

edge-updates/s = E_useful * L / t_step.

Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3

WORKLOADS = {
    # name: config index (synth.CONFIGS)
    "ellipsoid-200k": 2,
    "ellipsoid-ms-400k": 3,
    "ellipsoid-ms-1m-24p": 4,
    "car-ms-4m-16p": 5,
    "car-ms-2m-21p-h512": 6,
}
# partitions per batch when --wave-parts is not given: every part in one batch
# where its tape and workspace fit in HBM (288 GB), else waves of this many
# (about 90 GB at H = 256 and 110 GB at H = 512)
DEFAULT_WAVE_PARTS = {"car-ms-4m-16p": 2, "car-ms-2m-21p-h512": 3}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_bytes(name: str, n: int, E: int, H: int, s: int, fused: int = 0, de_in: float = 1.0,
                 ztape: bool = False, atape: bool = False, split: bool = False) -> float | None:
    """Algorithmic HBM bytes of one launch of a processor kernel: each input
    read once, each output written once (s = bytes per stored latent; FP32
    adjoints are 4 bytes).  `fused`: the edge adjoint accumulates dW2 (1), or
    dW2 and the e-block of dW1 (2), itself, so z and du are not written (and
    with 1 the e-block is a separate product that reads da and e again).
    `de_in`: fraction of launches that read an incoming edge adjoint de' (all
    but the last layer).  `atape`: the forward also writes the
    pre-activation a (SiLU), which the adjoint reads too.  `ztape`: the
    forward writes z for the adjoint, which reads it instead of h_s and h_r.
    `split`: the edge forward's split form, which reads the FP32 node
    projections of W1 instead of h."""
    if name == "edge_fwd" and split:
        # per edge: e read, e' (and z, a) written; per node: the projections
        # W1_r h + b1 and W1_s h (FP32) read; per receiver: m (FP32) written
        return E * (2 + (1 if ztape else 0) + (1 if atape else 0)) * H * s + n * (8 * H + 4 * H)
    if name == "node_proj":
        return n * (H * s + 8 * H)
    if name == "edge_fwd":
        # per edge: e and the gathered h_s read, e' (and z) written; per
        # receiver: h_r read, m (FP32) written
        return E * (3 + (1 if ztape else 0) + (1 if atape else 0)) * H * s + n * (H * s + 4 * H)
    if name == "edge_bwd":
        # per edge: de' (FP32) read, de (FP32) and da written, and
        #   both fused, z on the tape: z, e read
        #   dW2 fused, z on the tape:  z read
        #   fused, recompute:          h_s, e read
        #   unfused, z on the tape:    z read, du written
        #   unfused, recompute:        h_s, e read, z, du written
        # per receiver: h_r (not with ztape), dm (FP32) read, S_r (FP32) written
        if ztape:
            lat = 3 if fused == 2 else 2
        else:
            lat = 3 if fused else 5
        per_edge = (lat + (1 if atape else 0)) * H * s + 4 * H * (1 + de_in)
        return E * per_edge + n * ((0 if ztape else H * s) + 8 * H)
    if name == "node_fwd":
        return n * (2 * H * s + 4 * H)
    if name == "node_bwd":
        # h, m (FP32), dh' (FP32) read; dh_mid, dm (FP32) and da written (z and
        # du too where dW2 is not fused: BF16 at H = 128 fuses it)
        return n * (2 * H * s + 16 * H + (0 if (s == 2 and H == 128) else 2 * H * s))
    return None


def kernel_flops(name: str, n: int, E: int, H: int, fused: int = 0, ztape: bool = False,
                 split: bool = False) -> float | None:
    """Dense multiply-add flops of one launch (2 per MAC)."""
    if name == "edge_fwd":
        return E * (4.0 if split else 8.0) * H * H
    if name == "node_proj":
        return n * 4.0 * H * H
    if name == "edge_bwd":
        # recompute (3H x H unless z is on the tape, H x H), W2^T du, W1e^T da;
        # fused: du^T z (1), and da^T e (2)
        return E * (12.0 + 2.0 * fused - (6.0 if ztape else 0.0)) * H * H
    if name == "node_fwd":
        return n * 6.0 * H * H
    if name == "node_bwd":
        return n * (14.0 if H == 128 else 12.0) * H * H
    return None


def kernel_source_hash() -> str:
    """Hash of the device-code sources (.hip and .hpp; the host-side
    api.cpp only picks among the kernels, and a traffic record names the
    instantiation it measured); HBM counters taken on other sources are
    stale."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_17164_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/traffic_<kernel>_<workload>.json), if it was taken on
    the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(cfg_idx: int, layers: int, hidden: int):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    the same geometry / multi-scale recipe at 1/32 of the points (1/128 at
    H = 256, 1/2048 at H = 512, to keep the same order of work), full depth
    and width, one forward + backward."""
    from oracle import graph as og
    from oracle import model as om
    from synth import CONFIGS, init_params, make_inputs
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        cores = os.cpu_count() or 1
    cfg = CONFIGS[cfg_idx]
    div = 32 * (hidden // 128) ** (2 if hidden <= 256 else 3)
    levels = tuple(max(200, lv // div) for lv in cfg.levels)
    inp = make_inputs(cfg, levels=levels)
    G = og.build_graph(inp.pos, levels, cfg.k_intra, cfg.k_cross if len(levels) > 1 else 0)
    d = om.Desc(hidden=hidden, layers=layers, node_in=cfg.node_in, activation=cfg.activation)
    params = init_params(om.param_entries(d), cfg.seed("weights")).astype(np.float64)
    t0 = time.perf_counter()
    om.step_full(d, params, G, inp.node_in, inp.pos, inp.edge_norm, inp.targets)
    t = time.perf_counter() - t0
    return {"value": G.n_edges * layers / t, "unit": "edge-updates/s", "cores": int(cores), "kind": "oracle",
            "sample": f"FP64 oracle fwd+bwd on the same recipe at levels {list(levels)} "
                      f"({G.n_edges} edges, {layers} layers, H={hidden}); {t:.1f} s"}


def study(args):
    """Studies on one GPU, one partition per batch (Sec. V.F.1-2, III.D).

    offload: the 3-level 400k-point ellipsoid in two halo partitions, with
    the per-layer checkpoints on the device and offloaded to host memory.
    memory: peak device memory of a training step against the partition
    count (1 to 32, equal sizes, 15-hop halos) on the 1-level and the
    3-level graph of the same 400k points, both tape placements.
    Prints one JSON line per run."""
    import torch

    from paper_2411_17164_amd import api
    from synth import CONFIGS, init_params, make_inputs

    cfg = CONFIGS[3]
    H, L = cfg.hidden, cfg.layers
    dev = torch.device("cuda:0")
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    if args.study == "inference":
        return study_inference(args, cfg, to)
    if args.study == "offload":
        plan = [("3-level", cfg.levels, [2])]
    else:
        plan = [("1-level", (cfg.levels[-1],), [1, 2, 4, 8, 16, 32]), ("3-level", cfg.levels, [1, 2, 4, 8, 16, 32])]
    model = api.Model(H, L, precision="bf16")
    entries = [(kind, shape) for (_, _, _, kind, shape, _) in model.param_tensors()]
    params = to(init_params(entries, cfg.seed("weights")))
    for gname, levels, part_counts in plan:
        inp = make_inputs(cfg, levels=levels)
        pos, node_in, tgt = to(inp.pos), to(inp.node_in), to(inp.targets)
        kctx = api.Context(0)
        g = kctx.build_knn(pos, [int(x) for x in inp.level_end], cfg.k_intra, cfg.k_cross if len(levels) > 1 else 0)
        N, E = g.info()
        out = torch.zeros(N, 4, device=dev)
        d_out, loss = torch.zeros_like(out), torch.zeros(1, device=dev)
        d_params, acc = torch.zeros_like(params), torch.zeros_like(params)
        for P in part_counts:
            sizes = None if P == 1 else [N // P + (1 if i < N % P else 0) for i in range(P)]
            ps = api.Partset.halo(g, inp.pos, sizes, L)
            infos = [ps.info(p) for p in range(P)]
            E_proc = sum(i[2] for i in infos)
            for offload in (False, True):
                ctx = api.Context(0)
                ctx.set_offload(offload)

                def step():
                    acc.zero_()
                    for p in range(P):  # one partition at a time, gradients aggregated
                        ctx.forward(model, params, ps, [p], node_in, pos, inp.edge_norm, out, keep_tape=True)
                        ctx.mse_grad(out, tgt, N, d_out, loss)
                        ctx.backward(model, params, d_out, d_params)
                        api.grad_accumulate(acc, d_params)

                step()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    step()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / args.steps * 1e3
                line = {"study": args.study, "graph": gname, "nodes": N, "edges": E, "partitions": P, "halo": L,
                        "offload": offload, "ms_per_step": round(ms, 2),
                        "device_workspace_gb": round(ctx.memory() / 1e9, 3),
                        "pinned_host_gb": round(ctx.host_memory() / 1e9, 3),
                        "processed_edges": E_proc, "max_part_edges": max(i[2] for i in infos),
                        "edge_updates_per_s": E * L / (ms * 1e-3), "dtype": "bf16", "data": "synthetic"}
                print(json.dumps(line), flush=True)
                del ctx


def study_inference(args, cfg, to):
    """Inference and the optimizer on the 400k-point 3-level graph (Sec. III.D,
    V.D): forward without a tape over the whole graph and over 4 halo
    partitions one at a time (halo rows dropped, inner rows re-assembled),
    and a full training step with the Adam update.  One JSON line each."""
    import torch

    from paper_2411_17164_amd import api
    from synth import init_params, make_inputs

    H, L = cfg.hidden, cfg.layers
    inp = make_inputs(cfg)
    pos, node_in, tgt = to(inp.pos), to(inp.node_in), to(inp.targets)
    ctx = api.Context(0)
    g = ctx.build_knn(pos, [int(x) for x in inp.level_end], cfg.k_intra, cfg.k_cross)
    N, E = g.info()
    model = api.Model(H, L, precision="bf16")
    entries = [(kind, shape) for (_, _, _, kind, shape, _) in model.param_tensors()]
    params = to(init_params(entries, cfg.seed("weights")))
    out = torch.zeros(N, 4, device=params.device)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps * 1e3

    for P in (1, 4):
        sizes = None if P == 1 else [N // P + (1 if i < N % P else 0) for i in range(P)]
        ps = api.Partset.halo(g, inp.pos, sizes, L)
        E_proc = sum(ps.info(p)[2] for p in range(P))

        def infer():
            for p in range(P):
                ctx.forward(model, params, ps, [p], node_in, pos, inp.edge_norm, out, keep_tape=False)

        ms = timed(infer)
        print(json.dumps({"study": "inference", "graph": "3-level", "nodes": N, "edges": E, "partitions": P,
                          "processed_edges": E_proc, "ms_per_forward": round(ms, 2),
                          "edge_updates_per_s": E * L / (ms * 1e-3), "dtype": "bf16", "data": "synthetic"}),
              flush=True)
    full = api.Partset.halo(g, inp.pos, None, L)
    d_out, loss = torch.zeros_like(out), torch.zeros(1, device=out.device)
    d_params = torch.zeros_like(params)
    opt = api.Adam(ctx, params, clip_norm=32.0)

    def train():
        ctx.forward(model, params, full, [0], node_in, pos, inp.edge_norm, out, keep_tape=True)
        ctx.mse_grad(out, tgt, N, d_out, loss)
        ctx.backward(model, params, d_out, d_params)
        opt.step(d_params, api.cosine_lr(opt.t, 1000, 1e-3, 1e-6))

    ms = timed(train)
    print(json.dumps({"study": "train", "graph": "3-level", "nodes": N, "edges": E, "ms_per_step": round(ms, 2),
                      "edge_updates_per_s": E * L / (ms * 1e-3), "loss": float(loss.item()), "dtype": "bf16",
                      "data": "synthetic"}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ellipsoid-ms-400k", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--tape", choices=["keep", "recompute", "both"], default="both",
                    help="tape policy: keep the edge MLPs' hidden activations, recompute them from the "
                         "per-layer checkpoints, or time both (the first listed is the headline)")
    ap.add_argument("--edge-form", choices=["gather", "split", "both"], default="both",
                    help="edge forward: the gathered 3H first layer (the headline), the split form with "
                         "per-node projections of W1 (a variant, keep policy only), or both")
    ap.add_argument("--graph", action="store_true", help="replay each step from a captured HIP graph")
    ap.add_argument("--edge-rows", type=int, default=0)
    ap.add_argument("--node-rows", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--edge-waves", type=int, default=0)
    ap.add_argument("--adjoint-edge-rows", type=int, default=0, help="edge tile rows of the edge adjoint")
    ap.add_argument("--adjoint-edge-waves", type=int, default=0, help="waves per workgroup of the edge adjoint")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default tiles")
    ap.add_argument("--wave-parts", type=int, default=0,
                    help="partitions per batch (wave) for partitioned workloads (0 = the workload's default: "
                         "all in one batch where it fits in HBM)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 256 MiB device copy first (to scale HBM counters)")
    ap.add_argument("--study", choices=["offload", "memory", "inference"],
                    help="memory studies instead of the benchmark line (one JSON line per run)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(partitions would be spread over GPUs with one gradient all-reduce)", file=sys.stderr)
        sys.exit(2)

    if args.study:
        study(args)
        return

    import torch

    from paper_2411_17164_amd import api
    from synth import CONFIGS, init_params, make_inputs

    cfg = CONFIGS[WORKLOADS[args.workload]]
    H, L = cfg.hidden, cfg.layers
    dev = torch.device("cuda:0")
    log(f"[bench] workload {args.workload}: generating inputs")
    inp = make_inputs(cfg)
    levels = [int(x) for x in inp.level_end]
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    pos, node_in, tgt = to(inp.pos), to(inp.node_in), to(inp.targets)
    if args.calib_copy:
        a = torch.ones(64 << 20, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ctx = api.Context(0)
    ctx.set_tiles(args.edge_rows, args.node_rows, args.grid, args.edge_waves)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = ctx.build_knn(pos, levels, cfg.k_intra, cfg.k_cross if len(levels) > 1 else 0)
    t_knn = time.perf_counter() - t0
    N, E = g.info()
    t0 = time.perf_counter()
    n_parts = cfg.n_parts
    ps = api.Partset.halo(g, inp.pos, inp.part_sizes if n_parts > 1 else None, L)
    t_part = time.perf_counter() - t0
    infos = [ps.info(p) for p in range(n_parts)]
    E_proc = int(sum(i[2] for i in infos))
    wp = args.wave_parts if args.wave_parts > 0 else DEFAULT_WAVE_PARTS.get(args.workload, n_parts)
    waves = [list(range(i, min(i + wp, n_parts))) for i in range(0, n_parts, wp)]
    wave_sizes = [(sum(infos[p][0] + infos[p][1] for p in w), sum(infos[p][2] for p in w)) for w in waves]
    log(f"[bench] graph N={N} E={E} (processed {E_proc}, {n_parts} parts in {len(waves)} waves) "
        f"kNN {t_knn * 1e3:.1f} ms, plan {t_part * 1e3:.1f} ms")

    results = {}
    if H == 512 and not args.no_fp32:
        log("[bench] H = 512 runs in the BF16 form only: no FP32 leg")
    precs = ["bf16"] if args.no_fp32 or H == 512 else ["bf16", "fp32"]
    policies = {"keep": [True], "recompute": [False], "both": [True, False]}[args.tape]
    forms = {"gather": [False], "split": [True], "both": [False, True]}[args.edge_form]
    # legs: (name, precision, keep_hidden, split form); the first is the headline
    legs = [(p + ("_split" if split else "") + ("" if keep else "_recompute"), p, keep, split)
            for split in forms for keep in policies if keep or not split for p in precs]
    if not legs:
        sys.exit("the split edge form runs with the keep tape policy only")
    for leg, prec, keep, split in legs:
        ctx = api.Context(0)  # a context per leg, so that its workspace is the leg's own
        ctx.set_tiles(args.edge_rows, args.node_rows, args.grid, args.edge_waves)
        ctx.set_bwd_tiles(args.adjoint_edge_rows, args.adjoint_edge_waves)
        ctx.set_tape(keep)
        ctx.set_edge_split(split)
        model = api.Model(H, L, node_in=cfg.node_in, activation=cfg.activation, precision=prec)
        entries = [(kind, shape) for (_, _, _, kind, shape, _) in model.param_tensors()]
        params = to(init_params(entries, cfg.seed("weights")))
        out = torch.zeros(N, 4, device=dev)
        d_out = torch.zeros_like(out)
        loss = torch.zeros(1, device=dev)
        d_params = torch.zeros_like(params)
        acc = torch.zeros_like(params) if len(waves) > 1 else None

        def step():
            if acc is None:
                ctx.forward(model, params, ps, waves[0], node_in, pos, inp.edge_norm, out, keep_tape=True)
                ctx.mse_grad(out, tgt, N, d_out, loss)
                ctx.backward(model, params, d_out, d_params)
                return
            acc.zero_()
            for w in waves:  # gradient aggregation over partition waves
                ctx.forward(model, params, ps, w, node_in, pos, inp.edge_norm, out, keep_tape=True)
                ctx.mse_grad(out, tgt, N, d_out, loss)
                ctx.backward(model, params, d_out, d_params)
                api.grad_accumulate(acc, d_params)

        tuned = None
        if H == 512 and not args.no_autotune:
            log("[bench] H = 512: default tiles (64-row wide edge forward, 32-row edge adjoint, 16-row node), no autotuning")
        elif not args.no_autotune and not (args.edge_rows or args.node_rows or args.grid or args.edge_waves
                                           or args.adjoint_edge_rows or args.adjoint_edge_waves):
            ctx.set_tiles(0, 0, 0, 0)
            tuned = ctx.autotune(model, params, ps, waves[0], node_in, pos, inp.edge_norm, out, d_out, d_params)
            tuned = tuned[:4] + ctx.get_bwd_tiles() + tuned[4:]
            log(f"[bench] {leg}: autotuned edge_rows={tuned[0]} node_rows={tuned[1]} grid={tuned[2]} "
                f"edge_waves={tuned[3]} adjoint_edge_rows={tuned[4]} adjoint_edge_waves={tuned[5]} "
                f"({tuned[6]:.2f} ms)")
        log(f"[bench] {leg}: warmup {args.warmup}")
        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        run = step
        if args.graph:  # every wave's batch plan is cached by now: the whole step is captured
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr):
                step()
            run = gr.replay
            run()
            torch.cuda.synchronize()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            run()
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        ev = e0.elapsed_time(e1) / 1e3 / args.steps
        log(f"[bench] {leg}: {wall * 1e3:.2f} ms/step wall, {ev * 1e3:.2f} ms/step events, loss {loss.item():.5f}")
        # per-kernel breakdown from one extra (untimed) step
        ctx.set_timing(True)
        step()
        torch.cuda.synchronize()
        tk = ctx.timings()
        ctx.set_timing(False)
        results[leg] = dict(wall=wall, ev=ev, kernels=tk, mem=ctx.memory(), tiles=tuned, keep=keep, split=split)
        log(f"[bench] {leg} kernels: " + ", ".join(f"{k} {v[0]:.2f}ms/{v[1]}" for k, v in
                                                     sorted(tk.items(), key=lambda kv: -kv[1][0])))
        del params, out, d_out, d_params, ctx
        torch.cuda.empty_cache()

    head = legs[0][0]
    bf = results[head]
    value = E * L / bf["wall"]
    # dominant kernel of the headline BF16 step and its roofline
    kern = bf["kernels"]
    ztape = bf["keep"]  # the edge adjoint reads z from the forward's tape (tape policy keep)
    # the BF16 edge adjoint at H = 128 fuses its weight gradients: dW2 only on
    # its 32-row tiles with the z tape, dW2 and the e-block of dW1 otherwise
    adj_rows = (bf["tiles"][4] or bf["tiles"][0]) if bf["tiles"] else (args.adjoint_edge_rows or args.edge_rows or 64)
    fused = 0 if H != 128 else (1 if (ztape and adj_rows == 32) else 2)
    atape = ztape and cfg.activation != "relu"  # ... and, under SiLU, a
    de_in = (L - 1) / L
    kb = lambda k, n_w, e_w: kernel_bytes(k, n_w, e_w, H, 2, fused, de_in, ztape, atape, bf["split"])  # noqa: E731
    dom = max((k for k in kern if kb(k, N, E) is not None), key=lambda k: kern[k][0])
    avg_ms = kern[dom][0] / kern[dom][1]
    # launches of a processor kernel per step: L per wave (edge/node kernels)
    per_step = kern[dom][1]
    tot_bytes = sum(kb(dom, n_w, e_w) for n_w, e_w in wave_sizes) * per_step / len(waves)
    tot_flops = sum(kernel_flops(dom, n_w, e_w, H, fused, ztape, bf["split"])
                    for n_w, e_w in wave_sizes) * per_step / len(waves)
    by = tot_bytes / per_step
    fl = tot_flops / per_step
    achieved = by / (avg_ms * 1e-3) / 1e9
    tflops = fl / (avg_ms * 1e-3) / 1e12
    # the bound is the roof the kernel's arithmetic intensity meets first: HBM
    # below the BF16 ridge point (peak flops / peak bandwidth), MFMA above it
    mfma_bound = fl / by > BF16_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    roofline = {"kernel": dom, "bound": "mfma" if mfma_bound else "hbm",
                "achieved": round(tflops, 2) if mfma_bound else round(achieved, 1),
                "peak": BF16_PEAK_TFLOPS if mfma_bound else HBM_PEAK_GBS,
                "unit": "TFLOP/s" if mfma_bound else "GB/s",
                "frac": round(tflops / BF16_PEAK_TFLOPS if mfma_bound else achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.workload, dom), "source_hash": kernel_source_hash(),
                "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": by,
                "algorithmic_flops_per_launch": fl, "hbm_gbs": round(achieved, 1),
                "mfma_tflops": round(tflops, 2), "mfma_frac_bf16": round(tflops / BF16_PEAK_TFLOPS, 4)}
    line = {
        "metric": "processor edge-updates/s fwd+bwd, BF16 vs FP32 plain, 15 layers, 1 MI355X",
        "value": value,
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(bf["wall"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": args.workload, "nodes": N, "edges": E, "hidden": H, "layers": L,
                   "levels": levels, "k": [cfg.k_intra, cfg.k_cross], "partitions": n_parts,
                   "halo": L if n_parts > 1 else 0, "waves": len(waves), "processed_edges": E_proc,
                   "parallelism": "halo-partition batches" if n_parts > 1 else "none",
                   "graph_replay": bool(args.graph), "activation": cfg.activation,
                   "node_in": cfg.node_in},
        "processed_edge_updates_per_s": E_proc * L / bf["wall"],
        "roofline": roofline,
        "knn_build_ms": round(t_knn * 1e3, 2),
        "partition_plan_ms": round(t_part * 1e3, 2),
    }
    line["tape"] = "keep hidden activations" if bf["keep"] else "checkpoints only (recompute)"
    line["edge_form"] = "split (per-node W1 projections)" if bf["split"] else "gathered 3H first layer"
    line["end_to_end_ms"] = round((t_knn + t_part) * 1e3 + bf["wall"] * 1e3, 3)
    for leg, r in results.items():
        if leg == head:
            continue
        line[f"{leg}_value"] = E * L / r["wall"]
        line[f"{leg}_ms_per_step"] = round(r["wall"] * 1e3, 3)
    # BF16 against plain FP32 under the same tape policy
    for sfx in ("", "_recompute", "_split"):
        if "bf16" + sfx in results and "fp32" + sfx in results:
            line["bf16_over_fp32" + sfx] = round(results["fp32" + sfx]["wall"] / results["bf16" + sfx]["wall"], 3)
    line["tiles"] = {p: (dict(zip(["edge_rows", "node_rows", "grid", "edge_waves", "adjoint_edge_rows",
                                   "adjoint_edge_waves"], r["tiles"][:6]))
                         if r["tiles"] else None) for p, r in results.items()}
    line["kernels_ms"] = {p: {k: round(v[0], 3) for k, v in r["kernels"].items()} for p, r in results.items()}
    line["device_workspace_gb"] = {p: round(r["mem"] / 1e9, 2) for p, r in results.items()}
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(WORKLOADS[args.workload], L, H)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
