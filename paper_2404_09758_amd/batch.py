"""Python binding of the batching form (dr_batch_*): many independent
scenes stepped together, one launch per kernel, optionally replayed as a
HIP graph.  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np
import torch

from . import _lib as L
from .api import AVG_COUNT, ADAM, Context, DRError, _floats, make_optim, make_view


class Batch:
    """scenes: scenes.Scene objects.  Each scene's parameters (flat theta),
    Adam moments and accumulators are device tensors owned by this object
    (`theta[b]`, `m[b]`, `v[b]`, `Q[b]`, `K[b]`); targets[b] is the scene's
    views' images concatenated (rendered from its target parameters when not
    given).  bin_capacities: per scene (0 = the context default)."""

    def __init__(self, scenes: Sequence, n_pairs, device=None, tile_px=16, kind=ADAM, averaging=AVG_COUNT,
                 seed=0, first_step=1, bin_capacities=None, targets=None, lr=None, beta1=0.9, beta2=0.999,
                 eps_hat=1e-8):
        self.lib = L.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.scenes = list(scenes)
        n = len(self.scenes)
        self.n_pairs = int(n_pairs)
        self.ctx = []
        self.theta, self.m, self.v, self.Q, self.K, self.targets = [], [], [], [], [], []
        self._views = []
        with torch.cuda.device(self.device):
            for b, sc in enumerate(self.scenes):
                cap = 256 if bin_capacities is None else int(bin_capacities[b]) or 256
                ctx = Context(sc, self.device, tuning=(tile_px, cap, 0))
                ctx.set_scene_index(b)
                self.ctx.append(ctx)
                th = torch.tensor(sc.flat_params(), device=self.device)
                self.theta.append(th)
                self.m.append(torch.zeros_like(th))
                self.v.append(torch.zeros_like(th))
                Q, K = ctx.new_accumulators()
                self.Q.append(Q)
                self.K.append(K)
                if targets is None:
                    tt = torch.tensor(sc.flat_params(True), device=self.device)
                    tg = torch.cat([ctx.render(tt, vw, ids=False, uv=False)[0].reshape(-1) for vw in sc.views])
                else:
                    tg = targets[b]
                    if isinstance(tg, (list, tuple)):
                        tg = torch.cat([t.reshape(-1) for t in tg])
                self.targets.append(tg.contiguous())
            arr = (L.BatchScene * n)()
            for b, sc in enumerate(self.scenes):
                vws = (L.View * len(sc.views))(*[make_view(v) for v in sc.views])
                self._views.append(vws)
                e = list(sc.eps) + [0.0] * (1 + L.MAX_TEX - len(sc.eps))
                lrs = list(lr[b] if lr is not None else sc.lr)
                lrs = lrs + [0.0] * (1 + L.MAX_TEX - len(lrs))
                arr[b].ctx = self.ctx[b].h
                arr[b].views = vws
                arr[b].n_views = len(sc.views)
                arr[b].targets = self.targets[b].data_ptr()
                arr[b].theta = self.theta[b].data_ptr()
                arr[b].m = self.m[b].data_ptr()
                arr[b].v = self.v[b].data_ptr()
                arr[b].Q = self.Q[b].data_ptr()
                arr[b].K = self.K[b].data_ptr()
                arr[b].eps = _floats(e, 1 + L.MAX_TEX)
                arr[b].lr = _floats(lrs, 1 + L.MAX_TEX)
                arr[b].bin_capacity = 0
            self._arr = arr
            o = make_optim(kind, averaging, [], beta1, beta2, eps_hat)
            h = C.c_void_p()
            torch.cuda.synchronize(self.device)
            st = self.lib.dr_batch_create(C.byref(h), arr, n, self.n_pairs, int(tile_px), C.byref(o), C.c_uint64(seed),
                                          C.c_uint32(first_step),
                                          C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
            if st != 0:
                raise DRError(f"dr_batch_create failed: {L.STATUS.get(st, st)}")
            self.h = h
        self.tile_px = tile_px

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                self.lib.dr_batch_destroy(h)
            except Exception:
                pass
            self.h = None

    def _call(self, name, *args):
        st = getattr(self.lib, name)(self.h, *args)
        if st != 0:
            msg = self.lib.dr_batch_last_error(self.h)
            raise DRError(f"{name}: {L.STATUS.get(st, st)}: {msg.decode() if msg else ''}")

    def estimate(self):
        self._call("dr_batch_estimate")

    def step(self, use_graph=True):
        self._call("dr_batch_step", int(bool(use_graph)))

    def set_step(self, t):
        self._call("dr_batch_set_step", C.c_uint32(t))

    def get_step(self):
        t = C.c_uint32()
        self._call("dr_batch_get_step", C.byref(t))
        return int(t.value)

    def timing_enable(self, on=True):
        self._call("dr_batch_timing_enable", int(bool(on)))

    def timing_read(self, reset=True):
        t = L.Timing()
        self._call("dr_batch_timing_read", C.byref(t), int(bool(reset)))
        return {k: getattr(t, k) for k, _ in L.Timing._fields_}

    def stats(self):
        s = L.Stats()
        self._call("dr_batch_stats", C.byref(s))
        return {"tile_overflows": s.tile_overflows, "saturations": s.saturations, "nonfinite": s.nonfinite,
                "max_bin": s.max_bin, "full_scans": s.full_scans}
