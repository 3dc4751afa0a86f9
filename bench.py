"""Benchmark: optimisation steps/s of the per-pixel stochastic gradient
estimator at the paper's scale on one MI355X.

One step = estimate_grad over every (pair, view) item (8 antithetic pairs x
4 views of a 1024^2 render of a 46080-triangle mesh with 1024^2 albedo,
normal and roughness maps, GGX shading, L2 loss) followed by the Adam step
over all 7 409 158 parameters.  Inputs (parameters, targets) are resident in
HBM before the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config paper]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "optimisation steps/s at 1024², 50K tris (batched vs plain); % of HBM peak"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes of the fused raster/shade/loss/scatter kernel (k_tile):
# per pixel-estimate the target pixel is read once (12 B), the only per-pixel
# HBM input once the + and - renders stay on chip.
BYTES_PER_PIXEL_ESTIMATE = 12
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tile_traffic.json")


# Vector issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 VALU
# instruction per SIMD every 4 cycles.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def code_digest(paths):
    """SHA-256 of the kernel sources with comments and blank space removed:
    the counters stay valid across comment edits and go stale with any
    change of the code itself."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in paths:
        src = open(os.path.join(ROOT, f)).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def profiled_counters(kernel):
    """The committed rocprofv3 counters of `kernel` (HBM bytes and VALU
    instructions per launch), or None when they were taken on another kernel
    or the kernel code changed since."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if code_digest(rec["sources"]) != rec.get("kernel_code_sha256") or rec.get("kernel") != kernel:
        return None
    return rec


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counters, or None."""
    rec = profiled_counters(kernel)
    return None if rec is None else rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def progress(msg):
    """A progress line on stderr (the result stays the one JSON line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gate(torch, ms=100.0):
    """Hold the stream with a short device-side spin so the host can queue a
    timed sequence ahead of the GPU: the per-kernel event intervals then hold
    no host launch gaps."""
    if hasattr(torch.cuda, "_sleep"):
        torch.cuda._sleep(int(ms * 1e-3 * 2.4e9))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="paper",
                    choices=["paper", "mid", "tiny", "batch64", "soup", "layers", "subdiv", "atomics"])
    ap.add_argument("--soup-steps", type=int, default=100, help="Adam steps per run of the soup config")
    ap.add_argument("--cpu-reps", type=int, default=3, help="oracle: whole steps timed per core count")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mode", default="both", choices=["both", "graph", "batched", "plain"])
    ap.add_argument("--probe-copy-mib", type=int, default=0,
                    help="after the run, copy a float32 buffer of this many MiB 3 times (a kernel of "
                         "known traffic, to calibrate profiler byte counters)")
    return ap.parse_args()


def run_mode(ctx, sc, th, m, v, tg, eps, steps, warmup, tuning, api, torch):
    ctx.set_tuning(*tuning)
    Q, K = ctx.new_accumulators()
    n_pairs = sc.n_pairs
    t = 0

    def one_step():
        nonlocal t
        t += 1
        ctx.estimate_grad(th, sc.views, tg, sc.seed, t, n_pairs, eps, Q=Q, K=K)
        ctx.step(th, m, v, t, Q, K, eps, n_pairs, kind=api.ADAM, averaging=api.AVG_COUNT, lr=sc.lr)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    ctx.timing_read(reset=True)
    ctx.timing_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    gate(torch)
    w0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        one_step()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ctx.timing_enable(False)
    tm = ctx.timing_read(reset=True)
    ev_ms = start.elapsed_time(stop)
    # one extra estimate to count contributions (sum of K) of a step
    Q2, K2 = ctx.new_accumulators()
    ctx.estimate_grad(th, sc.views, tg, sc.seed, t + 1, n_pairs, eps, Q=Q2, K=K2)
    torch.cuda.synchronize()
    contributions = int(K2.to(torch.int64).sum().item())
    return {"ms_per_step": ev_ms / steps, "wall_ms_per_step": 1e3 * wall / steps, "timing": tm,
            "contributions_per_step": contributions}


def host_cpu():
    """Model name and usable core count of the host that runs the oracle."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, usable


def cpu_baseline(sc, reps=3, threads=None):
    """The oracle timed on whole optimisation steps: the estimate over every
    (pair, view) item plus the Adam step, on one host core and on all usable
    host cores (a thread pool over the items; the oracle releases the
    interpreter lock inside each call).  Each item's integer sums go to its
    thread's own accumulators, added at the end, so Q and K are bit-identical
    to the single-threaded step (checked).  Median of `reps` steps per core
    count.  Signs, renders, differences, scatter and descent all run in the
    oracle; the targets are inputs, rendered before timing."""
    import concurrent.futures as cf
    import statistics

    import numpy as np

    import oracle
    model, usable = host_cpu()
    if threads is None:
        # the machine's CPU share for one GPU is 16 cores, whatever the machine has
        threads = max(1, min(usable, int(os.environ.get("OMP_NUM_THREADS", "16")), 16))
    o = oracle.Oracle(sc)
    theta = sc.flat_params()
    views = sc.views
    items = [(n, v) for n in range(sc.n_pairs) for v in range(len(views))]
    targets = [o.render(sc.flat_params(True), vw)[0] for vw in views]

    def item(n, v, Q, K):
        s = oracle.signs(sc.seed, 1, n, 0, o.d)[None]
        o.estimate(theta, [views[v]], [targets[v]], sc.seed, 1, 1, sc.eps, signs_=s, Q=Q, K=K)

    def one_step(nthr):
        t0 = time.perf_counter()
        if nthr == 1:
            Q = np.zeros(o.d, np.int64)
            K = np.zeros(o.G, np.uint32)
            for (n, v) in items:
                item(n, v, Q, K)
        else:
            accs = [(np.zeros(o.d, np.int64), np.zeros(o.G, np.uint32)) for _ in range(nthr)]

            def work(w):
                for (n, v) in items[w::nthr]:
                    item(n, v, accs[w][0], accs[w][1])

            with cf.ThreadPoolExecutor(nthr) as ex:
                list(ex.map(work, range(nthr)))
            Q, K = accs[0]
            for q, k in accs[1:]:
                Q += q
                K += k
        th = theta.copy()
        m = np.zeros(o.d, np.float32)
        vv = np.zeros(o.d, np.float32)
        o.step(th, m, vv, 1, Q.copy(), K.copy(), sc.eps, sc.n_pairs, kind=0, averaging=0, lr=sc.lr)
        return time.perf_counter() - t0, Q, K, th

    legs = {}
    ref = None
    for nthr in sorted({1, threads}):
        runs = []
        for _ in range(reps):
            dt, Q, K, th = one_step(nthr)
            runs.append(dt)
            if ref is None:
                ref = (Q, K, th)
            elif not (np.array_equal(Q, ref[0]) and np.array_equal(K, ref[1]) and np.array_equal(th, ref[2])):
                raise RuntimeError("oracle step differs between core counts")
        med = statistics.median(runs)
        legs[nthr] = {"value": 1.0 / med, "unit": "steps/s", "cores": nthr, "s_per_step_runs": runs}
        progress(f"cpu baseline: {nthr} thread(s), {med:.2f} s/step (median of {reps})")
    top = legs[threads]
    px = sc.n_pairs * sum(v.width * v.height for v in views)
    return {"value": top["value"], "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"whole steps: all {len(items)} (pair, view) items of an estimate plus the Adam step; "
                      f"median of {reps} per core count; threads over items, integer sums bit-identical "
                      f"to one thread",
            "pixel_estimates_per_s": px * top["value"],
            "single_core": legs[1], "all_cores": top, "nproc": usable, "cpu_model": model}


def run_graph_mode(sc_list, tg_list, steps, warmup, api, batch_mod, torch, dev, tile=16, caps=None):
    """The batching form: every scene's step as one launch per kernel,
    captured once as a HIP graph and replayed."""
    bt = batch_mod.Batch(sc_list, sc_list[0].n_pairs, dev, tile_px=tile, seed=sc_list[0].seed, first_step=1,
                         targets=tg_list, kind=api.ADAM, averaging=api.AVG_COUNT, bin_capacities=caps)
    for _ in range(warmup):
        bt.step(use_graph=True)
    torch.cuda.synchronize()
    # the optimisation moves the mesh; the per-kernel pass below restarts from
    # this state so that it times the same steps as the graph replays
    snap = ([t.clone() for t in bt.theta], [t.clone() for t in bt.m], [t.clone() for t in bt.v], bt.get_step())
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        bt.step(use_graph=True)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ev_ms = start.elapsed_time(stop)
    # per-kernel durations: the same kernels launched directly, with events
    for dst, src in zip(bt.theta + bt.m + bt.v, snap[0] + snap[1] + snap[2]):
        dst.copy_(src)
    bt.set_step(snap[3])
    torch.cuda.synchronize()
    bt.timing_read(reset=True)
    bt.timing_enable(True)
    gate(torch)
    for _ in range(steps):
        bt.step(use_graph=False)
    bt.timing_enable(False)
    tm = bt.timing_read(reset=True)
    st = bt.stats()
    return {"ms_per_step": ev_ms / steps, "wall_ms_per_step": 1e3 * wall / steps, "timing": tm,
            "stats": st, "batch": bt}


def run_sequential_plain(sc_list, tg_list, steps, warmup, api, torch, dev, tile=16, caps=None, seed=0):
    """Each scene stepped on its own with one raster launch per item.  The
    signs are drawn as in the batch: one seed, the scene's index in the
    Philox counter."""
    ctxs, th, m, v = [], [], [], []
    for b, sc in enumerate(sc_list):
        c = api.Context(sc, dev, tuning=(tile, 256 if caps is None else caps[b], 1))
        c.set_scene_index(b)
        ctxs.append(c)
        th.append(torch.tensor(sc.flat_params(), device=dev))
        m.append(torch.zeros_like(th[-1]))
        v.append(torch.zeros_like(th[-1]))
    t = 0

    def one_step():
        nonlocal t
        t += 1
        for b, sc in enumerate(sc_list):
            Q, K = ctxs[b].estimate_grad(th[b], sc.views, tg_list[b], seed, t, sc.n_pairs, sc.eps)
            ctxs[b].step(th[b], m[b], v[b], t, Q, K, sc.eps, sc.n_pairs, kind=api.ADAM, averaging=api.AVG_COUNT,
                         lr=sc.lr)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        one_step()
    stop.record()
    torch.cuda.synchronize()
    return {"ms_per_step": start.elapsed_time(stop) / steps, "ctxs": ctxs, "theta": th, "m": m, "v": v,
            "steps_done": t}


def batch_equality(g, p, sc_list, tg_list, seed, torch):
    """Equal gradient accuracy of the two forms, checked on the runs just
    timed: every scene's parameters and Adam moments after the same number
    of steps from the same start, and then the Q and K of one more estimate
    (the batch's against each scene's own context), compared bit for bit."""
    bt = g["batch"]
    torch.cuda.synchronize()
    if bt.get_step() != p["steps_done"] + 1:
        raise RuntimeError(f"step counters differ: batch at {bt.get_step()}, plain did {p['steps_done']}")
    state_bad = [b for b in range(len(sc_list))
                 if not (torch.equal(bt.theta[b], p["theta"][b]) and torch.equal(bt.m[b], p["m"][b])
                         and torch.equal(bt.v[b], p["v"][b]))]
    t = bt.get_step()
    for b in range(len(sc_list)):
        bt.Q[b].zero_()
        bt.K[b].zero_()
    bt.estimate()
    est_bad = []
    for b, sc in enumerate(sc_list):
        Q, K = p["ctxs"][b].estimate_grad(bt.theta[b], sc.views, tg_list[b], seed, t, sc.n_pairs, sc.eps)
        if not (torch.equal(Q, bt.Q[b]) and torch.equal(K, bt.K[b])):
            est_bad.append(b)
    torch.cuda.synchronize()
    return {"scenes": len(sc_list), "steps_compared": p["steps_done"], "theta_m_v_equal": not state_bad,
            "estimate_Q_K_equal": not est_bad, "differing_scenes": sorted(set(state_bad) | set(est_bad))}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2404_09758_amd import api, autotune, batch, scenes
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.config == "batch64":
        return main_batch64(args, torch, api, autotune, batch, scenes, dev)
    if args.config == "soup":
        return main_soup(args, torch, api, scenes, dev)
    if args.config == "layers":
        return main_layers(args, torch, api, autotune, scenes, dev)
    if args.config == "atomics":
        return main_atomics(args, torch, dev)
    sc = scenes.CONFIGS[args.config]()
    ctx = api.Context(sc, dev, tuning=(16, 256, 0))
    th0 = torch.tensor(sc.flat_params(), device=dev)
    tgt_th = torch.tensor(sc.flat_params(True), device=dev)
    tg = torch.cat([ctx.render(tgt_th, v, ids=False, uv=False)[0].reshape(-1) for v in sc.views])
    eps = sc.eps
    px_per_step = sc.n_pairs * sum(v.width * v.height for v in sc.views)
    # launch shape from the autotuner (untimed)
    (tile, cap, _), tune_report = autotune.tune_scene(ctx, th0, sc.views, tg, sc.n_pairs, eps)
    progress(f"autotune: tile {tile}, bin capacity {cap}")
    results = {}
    modes = {"batched": (tile, cap, 0), "plain": (tile, cap, 1)}
    order = ["graph", "batched", "plain"] if args.mode == "both" else [args.mode]
    if sc.subdiv_levels > 0:
        order = [m for m in order if m != "graph"] or ["batched"]     # the batch form is mesh-only
    for name in order:
        if name == "graph":
            results[name] = run_graph_mode([sc], [tg], args.steps, args.warmup, api, batch, torch, dev, tile=tile,
                                           caps=[cap])
            progress(f"mode graph: {results[name]['ms_per_step']:.3f} ms/step")
            continue
        th = th0.clone()
        m = torch.zeros_like(th)
        v = torch.zeros_like(th)
        results[name] = run_mode(ctx, sc, th, m, v, tg, eps, args.steps, args.warmup, modes[name], api, torch)
        progress(f"mode {name}: {results[name]['ms_per_step']:.3f} ms/step")
    main_mode = order[0]
    r = results[main_mode]
    tm = r["timing"]
    tile_avg_ms = tm["tile_ms"] / max(tm["tile_launches"], 1)
    launches_per_step = tm["tile_launches"] / args.steps
    alg_bytes_launch = BYTES_PER_PIXEL_ESTIMATE * px_per_step / launches_per_step
    # the graph-captured step is a one-scene batch, whose tile kernel takes the
    # scene in its arguments; the host-driven modes (all items in one launch,
    # or one launch per item) run the context's tile kernel
    kernel = f"k_tile_b1<{tile}>" if main_mode == "graph" else f"k_tile<{tile},0,false>"
    traffic = measured_traffic(kernel) if args.config == "paper" else None
    achieved = alg_bytes_launch / (tile_avg_ms * 1e-3) / 1e9
    out = {
        # the headline metric names the paper-scale workload; other workloads say which they are
        "metric": METRIC if args.config == "paper" else f"optimisation steps/s, {args.config} workload",
        "value": 1e3 / r["ms_per_step"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {sc.views[0].width}x{sc.views[0].height} px, "
                               f"{ctx.tri.shape[0]} tris"
                               + (f" (Catmull-Clark x{sc.subdiv_levels} of {sc.n_tris})" if sc.subdiv_levels else "")
                               + f", {len(sc.views)} views x {sc.n_pairs} pairs, "
                               f"d={sc.n_params}, {['unlit', 'lambert', 'ggx'][sc.shading]}",
                   "mode": main_mode, "tile_px": tile, "bin_capacity": cap,
                   "pixel_estimates_per_step": px_per_step},
        "autotune": {str(k): v for k, v in tune_report.items()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "kernel_avg_ms": tile_avg_ms,
                     "alg_bytes_per_launch": alg_bytes_launch},
        "kernels_ms_per_step": {k[:-3]: tm[k] / args.steps for k in tm if k.endswith("_ms")},
        "pixel_estimates_per_s": px_per_step * 1e3 / r["ms_per_step"],
    }
    # the HBM target of the raster/scatter pass: half of peak.  The fused
    # kernel issues far more vector instructions than its bytes need, so it
    # meets vector issue long before HBM (see "issue")
    out["roofline"]["target_frac"] = 0.5
    out["roofline"]["target_met"] = out["roofline"]["frac"] >= 0.5
    rec = profiled_counters(kernel) if args.config == "paper" else None
    if rec is not None and "valu_wave_instructions_per_launch" in rec:
        # the ceiling the kernel actually meets: vector instruction issue
        rate = rec["valu_wave_instructions_per_launch"] / (tile_avg_ms * 1e-3)
        out["issue"] = {"valu_wave_instructions_per_launch": rec["valu_wave_instructions_per_launch"],
                        "achieved_per_s": rate, "peak_per_s": VALU_ISSUE_PEAK, "frac": rate / VALU_ISSUE_PEAK}
    for name, rr in results.items():
        out[f"{name}_steps_per_s"] = 1e3 / rr["ms_per_step"]
    if args.probe_copy_mib > 0:
        n = args.probe_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 4 * n
    if not args.no_cpu:
        progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_reps)
    print(json.dumps(out), flush=True)


def main_batch64(args, torch, api, autotune, batch, scenes, dev):
    """64 independent scenes of uneven size: one graph-captured batched step
    against 64 sequential plain steps.  The two are then checked equal bit
    for bit (parameters and moments after the timed steps, and one more
    estimate's Q and K per scene); the run fails if any scene differs."""
    n = 64
    scs = [scenes.make_batch_scene(b) for b in range(n)]
    tgs = []
    for sc in scs:
        c = api.Context(sc, dev)
        tt = torch.tensor(sc.flat_params(True), device=dev)
        tgs.append(torch.cat([c.render(tt, v, ids=False, uv=False)[0].reshape(-1) for v in sc.views]))
        del c
    px = sum(sc.n_pairs * sum(v.width * v.height for v in sc.views) for sc in scs)
    tile, caps, tune_report = autotune.tune_batch(scs, tgs, scs[0].n_pairs, dev, seed=scs[0].seed)
    progress(f"autotune: tile {tile}")
    g = run_graph_mode(scs, tgs, args.steps, args.warmup, api, batch, torch, dev, tile=tile, caps=caps)
    progress(f"graph: {g['ms_per_step']:.3f} ms/step")
    p = run_sequential_plain(scs, tgs, args.steps, args.warmup, api, torch, dev, tile=tile, caps=caps,
                             seed=scs[0].seed)
    progress(f"sequential plain: {p['ms_per_step']:.3f} ms/step")
    eq = batch_equality(g, p, scs, tgs, scs[0].seed, torch)
    progress(f"equality: {eq}")
    tm = g["timing"]
    tile_avg_ms = tm["tile_ms"] / max(tm["tile_launches"], 1)
    alg = BYTES_PER_PIXEL_ESTIMATE * px / (tm["tile_launches"] / args.steps)
    achieved = alg / (tile_avg_ms * 1e-3) / 1e9
    out = {
        "metric": "optimisation steps/s of 64 uneven scenes (graph-captured batched step vs 64 sequential plain steps)",
        "value": 1e3 / g["ms_per_step"], "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": g["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch64: {n} scenes, F in [{min(s.n_tris for s in scs)}, "
                               f"{max(s.n_tris for s in scs)}], 4 pairs x 1 view each, lambert, "
                               f"{px} pixel-estimates per step", "mode": "graph", "tile_px": tile,
                   "bin_capacity_max": max(caps)},
        "autotune": {str(k): v for k, v in tune_report.items()},
        "stats": g["stats"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": f"k_tile_b<{tile}>",
                     "kernel_avg_ms": tile_avg_ms, "alg_bytes_per_launch": alg},
        "kernels_ms_per_step": {k[:-3]: tm[k] / args.steps for k in tm if k.endswith("_ms")},
        "graph_steps_per_s": 1e3 / g["ms_per_step"],
        "sequential_plain_steps_per_s": 1e3 / p["ms_per_step"],
        "speedup_vs_sequential_plain": p["ms_per_step"] / g["ms_per_step"],
        "pixel_estimates_per_s": px * 1e3 / g["ms_per_step"],
        "equal_results": eq,
    }
    print(json.dumps(out), flush=True)
    if eq["differing_scenes"]:
        sys.exit(1)


def main_soup(args, torch, api, scenes, dev):
    """Per-pixel (Eq. 8) vs full-image (Eq. 4) estimation on triangle soups
    of 1K / 10K / 100K triangles (12 parameters each), 512^2 px, N = 128
    pairs per step, Adam with lr = eps: the loss after --soup-steps steps
    relative to the initial loss, and the step time (the validation of
    Sec. 6.1 on a synthetic target image)."""
    from paper_2404_09758_amd import autotune
    rows = []
    for n in (1024, 10240, 102400):
        sc = scenes.make_soup(n)
        tg = torch.tensor(sc.target_image, device=dev).reshape(-1)
        probe = api.Context(sc, dev, tuning=(16, 256, 0))
        th = torch.tensor(sc.flat_params(), device=dev)
        tuning, _ = autotune.tune_scene(probe, th, sc.views, tg, sc.n_pairs, sc.eps, reps=1)
        del probe
        for name, full, averaging in (("per_pixel_count", False, api.AVG_COUNT),
                                      ("per_pixel_pairs", False, api.AVG_PAIRS),
                                      ("full_image", True, api.AVG_PAIRS)):
            ctx = api.Context(sc, dev, tuning=tuning)
            th = torch.tensor(sc.flat_params(), device=dev)
            m = torch.zeros_like(th)
            v = torch.zeros_like(th)
            l0 = float(ctx.loss(th, sc.views, tg).sum())
            Q, K = ctx.new_accumulators()
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            start.record()
            for t in range(1, args.soup_steps + 1):
                ctx.estimate_grad(th, sc.views, tg, sc.seed, t, sc.n_pairs, sc.eps, Q=Q, K=K, full_image=full)
                ctx.step(th, m, v, t, Q, K, sc.eps, sc.n_pairs, kind=api.ADAM, averaging=averaging, lr=sc.lr)
                if t % 20 == 0:
                    torch.cuda.synchronize()
                    progress(f"soup {n} {name}: step {t} of {args.soup_steps}")
            stop.record()
            torch.cuda.synchronize()
            l1 = float(ctx.loss(th, sc.views, tg).sum())
            rows.append({"triangles": n, "d": sc.n_params, "estimator": name, "loss_ratio": l1 / l0,
                         "ms_per_step": start.elapsed_time(stop) / args.soup_steps, "tile_px": tuning[0],
                         "bin_capacity": tuning[1], "tile_overflows": ctx.stats()["tile_overflows"],
                         "full_scans": ctx.stats()["full_scans"]})
            progress(f"soup {n} {name}: loss ratio {l1 / l0:.4f}, {rows[-1]['ms_per_step']:.2f} ms/step, "
                     f"tuning {tuning}, overflows {rows[-1]['tile_overflows']}, full scans {rows[-1]['full_scans']}")
            del ctx
    out = {"metric": f"L2 loss after {args.soup_steps} Adam steps / initial loss (N=128 pairs/step, 512^2)",
           "config": {"workload": "soup: 1K/10K/100K-triangle soups, 12 params per triangle, unlit, "
                                  "value-noise target"},
           "data": "synthetic", "n_gpus": 1, "rows": rows}
    print(json.dumps(out), flush=True)


def main_layers(args, torch, api, autotune, scenes, dev):
    """Semi-transparent geometry: the same 20480-triangle, 512^2, 4-view x
    8-pair step with 0 (opaque), 2 and 4 composited layers per pixel; per
    layer count the step rate, the raster/scatter kernel's time and its
    algorithmic bandwidth, and the oracle on one (pair, view) item."""
    rows = []
    for layers in (0, 2, 4):
        sc = scenes.make_layered(layers)
        ctx = api.Context(sc, dev, tuning=(16, 256, 0))
        th0 = torch.tensor(sc.flat_params(), device=dev)
        tt = torch.tensor(sc.flat_params(True), device=dev)
        tg = torch.cat([ctx.render(tt, v, ids=False, uv=False)[0].reshape(-1) for v in sc.views])
        tiles = (8, 16) if layers > 0 else (8, 16, 32)
        (tile, cap, _), _ = autotune.tune_scene(ctx, th0, sc.views, tg, sc.n_pairs, sc.eps, tiles=tiles)
        th = th0.clone()
        m = torch.zeros_like(th)
        v = torch.zeros_like(th)
        r = run_mode(ctx, sc, th, m, v, tg, sc.eps, args.steps, args.warmup, (tile, cap, 0), api, torch)
        tm = r["timing"]
        px = sc.n_pairs * sum(vw.width * vw.height for vw in sc.views)
        tile_ms = tm["tile_ms"] / max(tm["tile_launches"], 1)
        alg = BYTES_PER_PIXEL_ESTIMATE * px / (tm["tile_launches"] / args.steps)
        row = {"layers": layers, "steps_per_s": 1e3 / r["ms_per_step"], "ms_per_step": r["ms_per_step"],
               "tile_px": tile, "bin_capacity": cap, "pixel_estimates_per_s": px * 1e3 / r["ms_per_step"],
               "contributions_per_step": r["contributions_per_step"],
               "roofline": {"bound": "hbm", "achieved": alg / (tile_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": alg / (tile_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                            "kernel": f"k_tile<{tile},0,{'true' if layers else 'false'}>",
                            "kernel_avg_ms": tile_ms},
               "kernels_ms_per_step": {k[:-3]: tm[k] / args.steps for k in tm if k.endswith("_ms")}}
        if not args.no_cpu:
            cb = cpu_baseline(sc, args.cpu_reps)
            row["cpu_baseline"] = cb
        rows.append(row)
        progress(f"layers {layers}: {row['steps_per_s']:.1f} steps/s")
        del ctx
    out = {"metric": "optimisation steps/s with semi-transparent layers (512^2, 20480 tris, 4 views x 8 pairs)",
           "unit": "steps/s", "higher_is_better": True, "dtype": "f32", "data": "synthetic", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "config": {"workload": "layers: icosphere 20480 tris, 512^2 px, lambert, RGBA albedo 512^2, "
                                  "0 / 2 / 4 composited layers"},
           "rows": rows}
    print(json.dumps(out), flush=True)


def main_atomics(args, torch, dev):
    """The atomic ceiling of the scatter's flush: agent-scope 64- and 32-bit
    atomic adds (no value returned) by address pattern -- adjacent lanes on
    adjacent elements, one element per 128-byte line, hashed (as a flush of
    hashed groups), and a wave's 64 lanes on one element -- into a 256 MiB
    buffer, timed with HIP events on the launch stream (median of 5)."""
    import statistics

    from paper_2404_09758_amd import _lib as L
    lib = L.load()
    nbytes = 256 << 20
    n_ops = 1 << 26
    buf = torch.zeros(nbytes // 8, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    names = {L.PROBE_CONTIGUOUS: "contiguous", L.PROBE_LINES: "one_per_line", L.PROBE_SCATTERED: "scattered",
             L.PROBE_CONFLICTING: "conflicting"}
    rows = []
    for width in (64, 32):
        for pat, name in names.items():
            def launch():
                st = lib.dr_probe_atomics(buf.data_ptr(), nbytes, width, pat, n_ops, stream)
                if st != 0:
                    raise RuntimeError(f"dr_probe_atomics: {L.STATUS.get(st, st)}")
            launch()
            torch.cuda.synchronize()
            times = []
            for _ in range(5):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                launch()
                b.record()
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b))
            ms = statistics.median(times)
            rows.append({"width_bits": width, "pattern": name, "ops": n_ops, "ms": ms,
                         "atomics_per_s": n_ops / (ms * 1e-3),
                         "operand_bytes_per_s": n_ops * width / 8 / (ms * 1e-3)})
            progress(f"atomics {width}-bit {name}: {rows[-1]['atomics_per_s'] / 1e9:.1f} G/s")
    out = {"metric": "agent-scope atomic adds per second by address pattern (256 MiB buffer)",
           "unit": "atomics/s", "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"atomics: {n_ops} no-return atomic adds per launch, 64- and 32-bit, "
                                  "4 address patterns"},
           "rows": rows}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
