"""Python binding of the C ABI: argument marshalling only.

Every step of the estimator runs in the HIP kernels of libdr.so; PyTorch
provides the device memory (tensors) and the stream.  Calls are queued on
torch's current stream of the context's device.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np
import torch

from . import _lib as L

ADAM, SGD = 0, 1
AVG_COUNT, AVG_PAIRS = 0, 1


class DRError(RuntimeError):
    pass


def _check_tensor(t, dtype, device, numel=None, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must live on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


def make_view(v) -> L.View:
    out = L.View()
    out.width = int(v.width)
    out.height = int(v.height)
    vp = np.asarray(v.view_proj, np.float32).reshape(16)
    for i in range(16):
        out.view_proj[i] = float(vp[i])
    cp = np.asarray(v.cam_pos, np.float32)
    for i in range(3):
        out.cam_pos[i] = float(cp[i])
    out.near_w = float(np.float32(getattr(v, "near", 0.1)))
    return out


def _floats(vals, n):
    arr = (C.c_float * n)()
    for i, x in enumerate(list(vals)[:n]):
        arr[i] = float(np.float32(x))
    return arr


def make_optim(kind, averaging, lr, beta1=0.9, beta2=0.999, eps_hat=1e-8) -> L.Optim:
    o = L.Optim()
    o.kind = int(kind)
    o.averaging = int(averaging)
    lr = list(lr) if lr is not None else []
    o.lr = _floats(lr + [0.0] * (1 + L.MAX_TEX - len(lr)), 1 + L.MAX_TEX)
    o.beta1, o.beta2, o.eps_hat = float(beta1), float(beta2), float(eps_hat)
    return o


def subdivide(tri, corner_uv, n_verts, levels):
    """Catmull-Clark tessellation of a triangle control mesh by the library
    (dr_subdivide, host): dict(tri, corner_uv, n_fine, rowptr, cols, w)."""
    lib = L.load()
    tri = np.ascontiguousarray(tri, np.int32)
    cuv = np.ascontiguousarray(corner_uv, np.float32)
    nv, nt, nnz = C.c_int32(), C.c_int32(), C.c_int64()
    st = lib.dr_subdivide_sizes(tri.ctypes.data, int(n_verts), int(tri.shape[0]), int(levels), C.byref(nv),
                                C.byref(nt), C.byref(nnz))
    if st != 0:
        raise DRError(f"dr_subdivide_sizes failed: {L.STATUS.get(st, st)}")
    out = {"tri": np.zeros((nt.value, 3), np.int32), "corner_uv": np.zeros((nt.value, 3, 2), np.float32),
           "rowptr": np.zeros(nv.value + 1, np.int32), "cols": np.zeros(max(nnz.value, 1), np.int32),
           "w": np.zeros(max(nnz.value, 1), np.float32), "n_fine": nv.value}
    st = lib.dr_subdivide(tri.ctypes.data, cuv.ctypes.data, int(n_verts), int(tri.shape[0]), int(levels),
                          out["tri"].ctypes.data, out["corner_uv"].ctypes.data, out["rowptr"].ctypes.data,
                          out["cols"].ctypes.data, out["w"].ctypes.data)
    if st != 0:
        raise DRError(f"dr_subdivide failed: {L.STATUS.get(st, st)}")
    out["cols"], out["w"] = out["cols"][: nnz.value], out["w"][: nnz.value]
    return out


class Context:
    """A scene bound to one GPU: topology, UVs, texture shapes and shading.

    tuning: (tile_px, bin_capacity, items_per_launch); items_per_launch 1 is
    one raster launch per (pair, view) ("plain"), 0 is all of them in one
    launch ("batched")."""

    def __init__(self, scene, device=None, tuning=(16, 256, 1)):
        self.lib = L.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("the estimator runs on a GPU device")
        levels = int(getattr(scene, "subdiv_levels", 0))
        with torch.cuda.device(self.device):
            tri, cuv, n_verts = scene.tri, scene.corner_uv, int(scene.pos.shape[0])
            self.surface = None
            if levels > 0:
                # scene.tri / corner_uv are the control mesh: tessellate it
                self.surface = subdivide(scene.tri, scene.corner_uv, n_verts, levels)
                tri, cuv = self.surface["tri"], self.surface["corner_uv"]
            self.tri = torch.as_tensor(np.ascontiguousarray(tri, np.int32), device=self.device)
            self.corner_uv = torch.as_tensor(np.ascontiguousarray(cuv, np.float32), device=self.device)
            shapes = [tuple(t.shape) for t in scene.tex]
            s = L.Scene()
            s.n_verts = n_verts if levels == 0 else int(self.surface["n_fine"])
            s.n_tris = int(self.tri.shape[0])
            if levels > 0:
                self.sub = [torch.as_tensor(self.surface[k], device=self.device) for k in ("rowptr", "cols", "w")]
                s.n_ctrl = n_verts
                s.sub_rowptr, s.sub_cols, s.sub_w = (t.data_ptr() for t in self.sub)
            s.tri = self.tri.data_ptr()
            s.corner_uv = self.corner_uv.data_ptr()
            s.n_tex = len(shapes)
            for t, (h, w, c) in enumerate(shapes):
                s.tex_h[t], s.tex_w[t], s.tex_c[t] = int(h), int(w), int(c)
            s.shading = int(scene.shading)
            s.tex_mode = int(getattr(scene, "tex_mode", 0))
            ld = np.asarray(scene.light_dir, np.float32)
            lc = np.asarray(scene.light_rgb, np.float32)
            for i in range(3):
                s.light_dir[i] = float(ld[i])
                s.light_rgb[i] = float(lc[i])
            s.ambient = float(np.float32(scene.ambient))
            s.diffuse = float(np.float32(getattr(scene, "diffuse", 0.9)))
            s.layers = int(getattr(scene, "layers", 0))
            self.layers = s.layers
            self._scene = s
            self.n_tex = len(shapes)
            tn = L.Tuning(*tuning)
            h = C.c_void_p()
            st = self.lib.dr_create(C.byref(h), C.byref(s), C.byref(tn),
                                    C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
            if st != 0:
                raise DRError(f"dr_create failed: {L.STATUS.get(st, st)}")
            self.h = h
        self.d = int(self.lib.dr_param_count(self.h))
        self.G = int(self.lib.dr_group_count(self.h))
        self.tuning = tuple(tuning)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                self.lib.dr_destroy(h)
            except Exception:
                pass
            self.h = None

    # ------------------------------------------------------------------
    def _call(self, name, *args):
        self.lib.dr_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        st = getattr(self.lib, name)(self.h, *args)
        if st != 0:
            msg = self.lib.dr_last_error(self.h)
            raise DRError(f"{name}: {L.STATUS.get(st, st)}: {msg.decode() if msg else ''}")

    def set_tuning(self, tile_px, bin_capacity, items_per_launch):
        tn = L.Tuning(int(tile_px), int(bin_capacity), int(items_per_launch))
        self._call("dr_set_tuning", C.byref(tn))
        self.tuning = (tile_px, bin_capacity, items_per_launch)

    def set_adaptive_bins(self, on=True):
        """Raise the bin capacity after an estimate whose bins overflowed."""
        self._call("dr_set_adaptive_bins", int(bool(on)))

    def get_tuning(self):
        """The launch shape in force: (tile_px, bin_capacity, items_per_launch)."""
        t = L.Tuning()
        self._call("dr_get_tuning", C.byref(t))
        return (t.tile_px, t.bin_capacity, t.items_per_launch)

    def _eps(self, eps):
        e = list(eps) + [0.0] * (1 + L.MAX_TEX - len(eps))
        return _floats(e, 1 + L.MAX_TEX)

    def render(self, theta, view, pert=None, rgb=True, ids=True, uv=True):
        """pert: None or dict(seed, step, pair, scene_index, sign, eps).
        Semi-transparent scenes return deep ids [H,W,L] and uv [H,W,L,2]."""
        dp = _check_tensor(theta, torch.float32, self.device, self.d, "theta")
        W, H = int(view.width), int(view.height)
        out_rgb = torch.empty((H, W, 3), dtype=torch.float32, device=self.device) if rgb else None
        deep = (self.layers,) if self.layers > 0 else ()
        out_id = torch.empty((H, W) + deep, dtype=torch.int32, device=self.device) if ids else None
        out_uv = torch.empty((H, W) + deep + (2,), dtype=torch.float32, device=self.device) if uv else None
        p = None
        if pert is not None:
            p = L.Perturb()
            p.seed = int(pert.get("seed", 0))
            p.step = int(pert.get("step", 0))
            p.pair = int(pert.get("pair", 0))
            p.scene_index = int(pert.get("scene_index", 0))
            p.sign = int(pert["sign"])
            p.eps = self._eps(pert["eps"])
        vw = make_view(view)
        self._call("dr_render", C.c_void_p(dp), C.byref(vw), C.byref(p) if p is not None else None,
                   C.c_void_p(out_rgb.data_ptr() if rgb else 0), C.c_void_p(out_id.data_ptr() if ids else 0),
                   C.c_void_p(out_uv.data_ptr() if uv else 0))
        return out_rgb, out_id, out_uv

    def loss(self, theta, views: Sequence, targets):
        """Per-view L2 image error (float64 tensor [n_views])."""
        dp = _check_tensor(theta, torch.float32, self.device, self.d, "theta")
        if isinstance(targets, (list, tuple)):
            targets = torch.cat([t.reshape(-1) for t in targets])
        need = sum(3 * int(v.width) * int(v.height) for v in views)
        dt = _check_tensor(targets, torch.float32, self.device, need, "targets")
        out = torch.empty(len(views), dtype=torch.float64, device=self.device)
        vws = (L.View * len(views))(*[make_view(v) for v in views])
        self._call("dr_loss", C.c_void_p(dp), vws, len(views), C.c_void_p(dt), C.c_void_p(out.data_ptr()))
        return out

    def signs(self, seed, step, pair, scene_index=0):
        words = (self.d + 31) // 32
        bits = torch.empty(words, dtype=torch.int32, device=self.device)
        self._call("dr_signs", C.c_uint64(seed), C.c_uint32(step), C.c_uint32(pair), C.c_uint32(scene_index),
                   C.c_void_p(bits.data_ptr()))
        return bits

    def new_accumulators(self):
        Q = torch.zeros(self.d, dtype=torch.int64, device=self.device)
        K = torch.zeros(self.G, dtype=torch.int32, device=self.device)
        return Q, K

    def estimate_grad(self, theta, views: Sequence, targets, seed, step, n_pairs, eps, Q=None, K=None,
                      full_image=False, image_grad=False, noalloc=False):
        """Eq. 8 (per pixel) or, with full_image, Eq. 4, summed over pairs and
        views into Q, K.  targets: one float32 tensor holding the views'
        [H,W,3] images concatenated (or a list of them).  image_grad: targets
        hold dL/dI of a downstream loss instead, and each pixel scatters
        <dL/dI, I+ - I-> (the image form; per pixel only).  noalloc: the
        per-pixel loss form through dr_estimate_grad_noalloc, whose scratch
        is the library's static device array (no device allocation)."""
        if full_image and image_grad:
            raise ValueError("the image form is a per-pixel estimator")
        if noalloc and (full_image or image_grad):
            raise ValueError("the allocation-free call is the per-pixel loss form")
        dp = _check_tensor(theta, torch.float32, self.device, self.d, "theta")
        if isinstance(targets, (list, tuple)):
            targets = torch.cat([t.reshape(-1) for t in targets])
        need = sum(3 * int(v.width) * int(v.height) for v in views)
        dt = _check_tensor(targets, torch.float32, self.device, need, "targets")
        if Q is None or K is None:
            Q, K = self.new_accumulators()
        dq = _check_tensor(Q, torch.int64, self.device, self.d, "Q")
        dk = _check_tensor(K, torch.int32, self.device, self.G, "K")
        vws = (L.View * len(views))(*[make_view(v) for v in views])
        fn = "dr_estimate_grad_full" if full_image else ("dr_estimate_grad_image" if image_grad else "dr_estimate_grad")
        if noalloc:
            fn = "dr_estimate_grad_noalloc"
        self._call(fn, C.c_void_p(dp), vws, len(views),
                   C.c_void_p(dt), C.c_uint64(seed),
                   C.c_uint32(step), int(n_pairs), self._eps(eps), C.c_void_p(dq), C.c_void_p(dk))
        return Q, K

    def decode_grad(self, Q, K, eps, averaging=AVG_COUNT, n_pairs=1):
        dq = _check_tensor(Q, torch.int64, self.device, self.d, "Q")
        dk = _check_tensor(K, torch.int32, self.device, self.G, "K")
        g = torch.empty(self.d, dtype=torch.float32, device=self.device)
        self._call("dr_decode_grad", C.c_void_p(dq), C.c_void_p(dk), self._eps(eps), int(averaging),
                   int(n_pairs), C.c_void_p(g.data_ptr()))
        return g

    def step(self, theta, m, v, t, Q, K, eps, n_pairs, kind=ADAM, averaging=AVG_COUNT, lr=None,
             beta1=0.9, beta2=0.999, eps_hat=1e-8):
        """One descent step (Adam or SGD) on theta; Q and K are zeroed."""
        dp = _check_tensor(theta, torch.float32, self.device, self.d, "theta")
        dm = _check_tensor(m, torch.float32, self.device, self.d, "m") if m is not None else 0
        dv = _check_tensor(v, torch.float32, self.device, self.d, "v") if v is not None else 0
        dq = _check_tensor(Q, torch.int64, self.device, self.d, "Q")
        dk = _check_tensor(K, torch.int32, self.device, self.G, "K")
        o = make_optim(kind, averaging, lr, beta1, beta2, eps_hat)
        self._call("dr_step", C.c_void_p(dp), C.c_void_p(dm), C.c_void_p(dv), C.c_uint32(t), C.c_void_p(dq),
                   C.c_void_p(dk), self._eps(eps), int(n_pairs), C.byref(o))

    def timing_enable(self, on=True):
        self._call("dr_timing_enable", int(bool(on)))

    def timing_read(self, reset=True):
        t = L.Timing()
        self._call("dr_timing_read", C.byref(t), int(bool(reset)))
        return {k: getattr(t, k) for k, _ in L.Timing._fields_}

    def set_scene_index(self, b):
        self._call("dr_set_scene_index", C.c_uint32(b))

    def stats(self):
        s = L.Stats()
        self._call("dr_stats", C.byref(s))
        return {"tile_overflows": s.tile_overflows, "saturations": s.saturations, "nonfinite": s.nonfinite,
                "max_bin": s.max_bin, "full_scans": s.full_scans}

    def reset_stats(self):
        self._call("dr_reset_stats")
