"""Autotuner of the raster launch shape: tile size and bin capacity.

Results never depend on the tuning (a bin that overflows falls back to
testing every triangle), only the speed does.  For each candidate tile size
the tuner measures the largest bin occupancy of a scene with a generous
capacity, sizes the capacity at the next power of two above 1.5x that
(other pairs and steps move the triangles, so the margin keeps overflows
rare), then times the candidates and keeps the fastest.
"""
from __future__ import annotations

import time

import torch

from . import api, batch

TILES = (8, 16, 32)
PROBE_CAPACITY = 4096


def _pow2_at_least(x):
    p = 16
    while p < x:
        p *= 2
    return p


def capacity_for(max_bin):
    return min(_pow2_at_least(int(max_bin * 1.5) + 1), 1 << 16)


def probe_max_bin(ctx, theta, views, targets, eps, tile, seed=0):
    """Largest bin occupancy of one estimate (one pair) with tile size `tile`."""
    saved = ctx.tuning
    ctx.set_tuning(tile, PROBE_CAPACITY, 1)
    ctx.reset_stats()
    Q, K = ctx.new_accumulators()
    ctx.estimate_grad(theta, views, targets, seed, 1, 1, eps, Q=Q, K=K)
    st = ctx.stats()
    ctx.set_tuning(*saved)
    return int(st["max_bin"])


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune_scene(ctx, theta, views, targets, n_pairs, eps, tiles=TILES, reps=3, items_per_launch=0):
    """Pick (tile_px, bin_capacity) for one scene; returns (tuning, report)."""
    report = {}
    best = None
    Q, K = ctx.new_accumulators()
    for tile in tiles:
        cap = capacity_for(probe_max_bin(ctx, theta, views, targets, eps, tile))
        ctx.set_tuning(tile, cap, items_per_launch)
        sec = _time(lambda: ctx.estimate_grad(theta, views, targets, 0, 1, n_pairs, eps, Q=Q, K=K), reps)
        report[tile] = {"bin_capacity": cap, "ms": 1e3 * sec}
        if best is None or sec < best[0]:
            best = (sec, (tile, cap, items_per_launch))
    ctx.set_tuning(*best[1])
    return best[1], report


def tune_batch(scenes, targets, n_pairs, device, tiles=TILES, reps=3, **batch_kw):
    """Pick the batch's tile size and every scene's bin capacity.
    targets[b]: scene b's views' images (device tensor).  Returns
    (tile_px, capacities, report)."""
    caps_by_tile = {}
    for tile in tiles:
        caps = []
        for b, sc in enumerate(scenes):
            ctx = api.Context(sc, device, tuning=(tile, PROBE_CAPACITY, 1))
            th = torch.tensor(sc.flat_params(), device=device)
            caps.append(capacity_for(probe_max_bin(ctx, th, sc.views, targets[b], sc.eps, tile)))
            del ctx
        caps_by_tile[tile] = caps
    report = {}
    best = None
    for tile in tiles:
        bt = batch.Batch(scenes, n_pairs, device, tile_px=tile, bin_capacities=caps_by_tile[tile], targets=targets,
                         **batch_kw)
        sec = _time(lambda: bt.estimate(), reps)
        st = bt.stats()
        report[tile] = {"ms": 1e3 * sec, "max_capacity": max(caps_by_tile[tile]), "overflows": st["tile_overflows"]}
        del bt
        if best is None or sec < best[0]:
            best = (sec, tile)
    return best[1], caps_by_tile[best[1]], report
