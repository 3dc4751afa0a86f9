"""ctypes binding of the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It takes plain numpy
arrays and scene-like objects (duck-typed: tri, corner_uv, tex, shading, ...)
and never imports the GPU library or its binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

MAX_TEX = 3
BG_ID = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain C, no contraction, no fast math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Scene_(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tris", C.c_int32),
                ("tri", C.c_void_p), ("corner_uv", C.c_void_p),
                ("n_tex", C.c_int32),
                ("tex_w", C.c_int32 * MAX_TEX), ("tex_h", C.c_int32 * MAX_TEX),
                ("tex_c", C.c_int32 * MAX_TEX),
                ("shading", C.c_int32), ("tex_mode", C.c_int32),
                ("light_dir", C.c_float * 3), ("light_rgb", C.c_float * 3),
                ("ambient", C.c_float), ("diffuse", C.c_float), ("layers", C.c_int32),
                ("n_ctrl", C.c_int32), ("sub_rowptr", C.c_void_p), ("sub_cols", C.c_void_p),
                ("sub_w", C.c_void_p)]


class View_(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("view_proj", C.c_float * 16),
                ("cam_pos", C.c_float * 3), ("near_w", C.c_float)]


class Optim_(C.Structure):
    _fields_ = [("kind", C.c_int32), ("averaging", C.c_int32), ("lr", C.c_float * (1 + MAX_TEX)),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps_hat", C.c_float)]


class Stats_(C.Structure):
    _fields_ = [("saturations", C.c_uint64), ("nonfinite", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        vp = C.c_void_p
        L.or_philox4x64_10.argtypes = [vp, vp, vp]
        L.or_signs.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64, vp]
        L.or_param_count.argtypes = [vp]
        L.or_param_count.restype = C.c_int64
        L.or_group_count.argtypes = [vp]
        L.or_group_count.restype = C.c_int64
        L.or_render.argtypes = [vp, vp, vp, C.c_int, vp, vp, vp, vp, vp]
        L.or_pixel_loss.argtypes = [vp, vp, vp, C.c_int, vp, vp, vp, vp]
        L.or_quantize.argtypes = [C.c_float, vp]
        L.or_quantize.restype = C.c_int64
        L.or_estimate.argtypes = [vp, vp, vp, C.c_int32, vp, C.c_uint64, C.c_uint32, C.c_int32,
                                  C.c_uint32, vp, vp, vp, vp, vp, vp]
        L.or_estimate_full.argtypes = L.or_estimate.argtypes
        L.or_estimate_image.argtypes = L.or_estimate.argtypes
        L.or_decode.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, vp]
        L.or_step.argtypes = [vp, vp, vp, vp, C.c_uint32, vp, vp, vp, C.c_int32, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def make_view(v) -> View_:
    out = View_()
    out.width = int(v.width)
    out.height = int(v.height)
    vp = np.asarray(v.view_proj, np.float32).reshape(16)
    for i in range(16):
        out.view_proj[i] = float(vp[i])
    for i in range(3):
        out.cam_pos[i] = float(np.float32(v.cam_pos[i]))
    out.near_w = float(np.float32(getattr(v, "near", 0.1)))
    return out


def philox4x64_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint64)
    k = _c(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def signs(seed: int, step: int, pair: int, scene: int, d: int) -> np.ndarray:
    s = np.zeros(d, np.int8)
    lib().or_signs(seed, step, pair, scene, d, _ptr(s))
    return s


def quantize(delta: float) -> int:
    st = Stats_()
    return int(lib().or_quantize(float(np.float32(delta)), C.byref(st)))


class Oracle:
    """The oracle bound to one scene (topology, UVs, texture shapes, shading)."""

    def __init__(self, scene, tex_shapes=None, shading=None, tex_mode=None):
        levels = int(getattr(scene, "subdiv_levels", 0))
        n_verts = int(scene.pos.shape[0]) if hasattr(scene, "pos") else int(scene.n_verts)
        self.surface = None
        if levels > 0:
            # scene.tri / corner_uv are the control mesh (Sec. 6.3)
            from . import subdiv
            self.surface = subdiv.catmull_clark(scene.tri, n_verts, scene.corner_uv, levels)
            self.tri = _c(self.surface["tri"], np.int32)
            self.corner_uv = _c(self.surface["corner_uv"], np.float32)
        else:
            self.tri = _c(scene.tri, np.int32)
            self.corner_uv = _c(scene.corner_uv, np.float32)
        shapes = tex_shapes if tex_shapes is not None else [t.shape for t in scene.tex]
        s = Scene_()
        s.n_verts = n_verts if levels == 0 else int(self.surface["n_fine"])
        s.n_tris = int(self.tri.shape[0])
        if levels > 0:
            s.n_ctrl = n_verts
            s.sub_rowptr = _ptr(self.surface["rowptr"])
            s.sub_cols = _ptr(self.surface["cols"])
            s.sub_w = _ptr(self.surface["w"])
        s.tri = _ptr(self.tri)
        s.corner_uv = _ptr(self.corner_uv)
        s.n_tex = len(shapes)
        for t, (h, w, c) in enumerate(shapes):
            s.tex_h[t], s.tex_w[t], s.tex_c[t] = int(h), int(w), int(c)
        s.shading = int(scene.shading if shading is None else shading)
        s.tex_mode = int(getattr(scene, "tex_mode", 0) if tex_mode is None else tex_mode)
        ld = np.asarray(getattr(scene, "light_dir", (0.57735026, 0.57735026, 0.57735026)), np.float32)
        lc = np.asarray(getattr(scene, "light_rgb", (1.0, 1.0, 1.0)), np.float32)
        for i in range(3):
            s.light_dir[i] = float(ld[i])
            s.light_rgb[i] = float(lc[i])
        s.ambient = float(np.float32(getattr(scene, "ambient", 0.1)))
        s.diffuse = float(np.float32(getattr(scene, "diffuse", 0.9)))
        s.layers = int(getattr(scene, "layers", 0))
        self.layers = s.layers
        self.s = s
        self.d = int(lib().or_param_count(C.byref(s)))
        self.G = int(lib().or_group_count(C.byref(s)))
        self.n_blocks = 1 + s.n_tex

    def _eps(self, eps):
        e = np.zeros(1 + MAX_TEX, np.float32)
        e[: len(eps)] = np.asarray(eps, np.float32)
        return e

    def render(self, theta, view, signs_=None, sign=+1, eps=None):
        th = _c(theta, np.float32)
        assert th.shape == (self.d,)
        W, H = int(view.width), int(view.height)
        rgb = np.zeros((H, W, 3), np.float32)
        deep = (self.layers,) if self.layers > 0 else ()
        ids = np.zeros((H, W) + deep, np.uint32)
        uv = np.zeros((H, W) + deep + (2,), np.float32)
        sg = None if signs_ is None else _c(signs_, np.int8)
        e = self._eps(eps if eps is not None else [0.0])
        vw = make_view(view)
        rc = lib().or_render(C.byref(self.s), _ptr(th), _ptr(sg), int(sign), _ptr(e), C.byref(vw),
                             _ptr(rgb), _ptr(ids), _ptr(uv))
        assert rc == 0
        return rgb, ids, uv

    def pixel_loss(self, theta, view, target, signs_=None, sign=+1, eps=None):
        th = _c(theta, np.float32)
        W, H = int(view.width), int(view.height)
        f = np.zeros((H, W), np.float32)
        sg = None if signs_ is None else _c(signs_, np.int8)
        e = self._eps(eps if eps is not None else [0.0])
        vw = make_view(view)
        tg = _c(target, np.float32)
        rc = lib().or_pixel_loss(C.byref(self.s), _ptr(th), _ptr(sg), int(sign), _ptr(e), C.byref(vw),
                                 _ptr(tg), _ptr(f))
        assert rc == 0
        return f

    def estimate(self, theta, views, targets, seed, step, n_pairs, eps, scene_index=0, signs_=None,
                 Q=None, K=None, want_g64=False, full_image=False, image_grad=False):
        """Eq. 8 summed over pairs and views (full_image=True: Eq. 4).
        image_grad=True: `targets` are the views' gradients dL/dI of a
        downstream loss and the per-pixel difference is <g, I+ - I->."""
        th = _c(theta, np.float32)
        vws = (View_ * len(views))(*[make_view(v) for v in views])
        tg = np.concatenate([_c(t, np.float32).reshape(-1) for t in targets])
        Q = np.zeros(self.d, np.int64) if Q is None else Q
        K = np.zeros(self.G, np.uint32) if K is None else K
        G64 = np.zeros(self.d, np.float64) if want_g64 else None
        sg = None if signs_ is None else _c(signs_, np.int8).reshape(-1)
        if sg is not None:
            assert sg.size == n_pairs * self.d
        st = Stats_()
        e = self._eps(eps)
        assert not (full_image and image_grad)
        fn = lib().or_estimate_full if full_image else (lib().or_estimate_image if image_grad else lib().or_estimate)
        rc = fn(C.byref(self.s), _ptr(th), vws, len(views), _ptr(tg), int(seed), int(step),
                               int(n_pairs), int(scene_index), _ptr(e), _ptr(sg), _ptr(Q), _ptr(K),
                               _ptr(G64), C.byref(st))
        assert rc == 0
        return Q, K, G64, {"saturations": st.saturations, "nonfinite": st.nonfinite}

    def decode(self, Q, K, eps, averaging, n_pairs):
        g = np.zeros(self.d, np.float32)
        e = self._eps(eps)
        lib().or_decode(C.byref(self.s), _ptr(_c(Q, np.int64)), _ptr(_c(K, np.uint32)), _ptr(e),
                        int(averaging), int(n_pairs), _ptr(g))
        return g

    def step(self, theta, m, v, t, Q, K, eps, n_pairs, kind=0, averaging=0, lr=None,
             beta1=0.9, beta2=0.999, eps_hat=1e-8):
        """In place on theta, m, v, Q, K (all contiguous numpy arrays)."""
        for a, dt in ((theta, np.float32), (m, np.float32), (v, np.float32), (Q, np.int64), (K, np.uint32)):
            assert a.dtype == dt and a.flags["C_CONTIGUOUS"]
        o = Optim_()
        o.kind = int(kind)
        o.averaging = int(averaging)
        lrs = np.zeros(1 + MAX_TEX, np.float32)
        lrs[: len(lr)] = np.asarray(lr, np.float32)
        for i in range(1 + MAX_TEX):
            o.lr[i] = float(lrs[i])
        o.beta1, o.beta2, o.eps_hat = float(beta1), float(beta2), float(eps_hat)
        st = Stats_()
        e = self._eps(eps)
        rc = lib().or_step(C.byref(self.s), _ptr(theta), _ptr(m), _ptr(v), int(t), _ptr(Q), _ptr(K),
                           _ptr(e), int(n_pairs), C.byref(o), C.byref(st))
        assert rc == 0
        return {"saturations": st.saturations, "nonfinite": st.nonfinite}
