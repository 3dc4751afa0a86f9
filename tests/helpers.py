"""Small hand-built scenes for the pins (no estimator arithmetic here)."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class V:
    """A view: view_proj maps world to clip space."""
    width: int
    height: int
    view_proj: np.ndarray
    cam_pos: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))
    near: float = 0.1


def ndc_view(w, h):
    """Identity projection: world x, y, z are NDC and clip w = 1."""
    return V(w, h, np.eye(4, dtype=np.float32), np.array([0, 0, 3], np.float32))


@dataclass
class SimpleScene:
    tri: np.ndarray
    corner_uv: np.ndarray
    pos: np.ndarray
    tex: list
    shading: int = 0
    tex_mode: int = 0
    light_dir: np.ndarray = field(default_factory=lambda: np.array([0, 0, 1], np.float32))
    light_rgb: np.ndarray = field(default_factory=lambda: np.ones(3, np.float32))
    ambient: float = 0.1
    diffuse: float = 0.9
    layers: int = 0

    @property
    def n_verts(self):
        return self.pos.shape[0]

    def flat(self, pos=None, tex=None):
        pos = self.pos if pos is None else pos
        tex = self.tex if tex is None else tex
        return np.concatenate([np.asarray(pos, np.float32).reshape(-1)]
                              + [np.asarray(t, np.float32).reshape(-1) for t in tex])


def quad_scene(tex, z=0.0, extent=1.0, uv_scale=1.0, shading=0):
    """Two triangles covering [-extent, extent]^2 at depth z, UV = [0,1]^2
    (u right, v down on screen)."""
    e = extent
    pos = np.array([(-e, e, z), (e, e, z), (e, -e, z), (-e, -e, z)], np.float32)
    tri = np.array([(0, 3, 1), (1, 3, 2)], np.int32)
    uvv = np.array([(0, 0), (1, 0), (1, 1), (0, 1)], np.float32) * uv_scale
    corner_uv = uvv[tri].astype(np.float32)
    return SimpleScene(tri, corner_uv, pos, [np.asarray(tex, np.float32)], shading=shading)


def grid_scene(n, jitter, seed, z=0.0, lo=-0.9, hi=0.9, tex=None):
    """A planar n x n grid of quads over [lo, hi]^2 split into triangles,
    interior vertices jittered; a watertight tessellation of the square."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(lo, hi, n + 1)
    P = np.array([(x, y, z) for y in xs for x in xs], np.float64)
    step = (hi - lo) / n
    for j in range(1, n):
        for i in range(1, n):
            k = j * (n + 1) + i
            P[k, :2] += rng.uniform(-jitter, jitter, 2) * step
    tris = []
    for j in range(n):
        for i in range(n):
            a = j * (n + 1) + i
            b, c, d = a + 1, a + n + 1, a + n + 2
            if (i + j) % 2:
                tris += [(a, b, d), (a, d, c)]
            else:
                tris += [(a, b, c), (b, d, c)]
    tri = np.array(tris, np.int32)
    corner_uv = np.zeros((len(tri), 3, 2), np.float32)
    if tex is None:
        tex = np.full((4, 4, 3), 0.5, np.float32)
    return SimpleScene(tri, corner_uv, P.astype(np.float32), [tex])


def sphere_scene(freq, splits=0, res=(96, 80), shading=0, tex_shapes=((48, 48, 3),), seed=0, views=1,
                 tex_mode=0, eps=None):
    """A small seeded sphere scene (scenes.Scene) with arbitrary texture
    shapes and view size, for parity cases that span several tiles."""
    from paper_2404_09758_amd import scenes as S
    rng = np.random.default_rng(seed)
    v, f, uv = S._sphere_scene(freq, splits)
    tex = [rng.uniform(0.05, 0.95, s).astype(np.float32) for s in tex_shapes]
    ttex = [rng.uniform(0.05, 0.95, s).astype(np.float32) for s in tex_shapes]
    tpos = S._radial_displace(v, seed + 7, amp=0.08).astype(np.float32)
    W, Hh = res
    vs = [S.look_at_view(W, Hh, 37.0 * k + 10.0, 15.0) for k in range(views)]
    if eps is None:
        fy = 1.0 / np.tan(np.radians(S.FOVY_DEG) / 2)
        eps = [1.5 * (S.CAM_DIST / fy) * 2.0 / Hh] + [1.0 / 255.0] * len(tex_shapes)
    return S.Scene("sphere", f.astype(np.int32), uv, v.astype(np.float32), tex, tpos, ttex, vs,
                   shading=shading, tex_mode=tex_mode, ambient=0.1 if shading == 1 else 0.03,
                   light_rgb=np.full(3, 1.0 if shading != 2 else 3.0, np.float32),
                   eps=list(eps), lr=list(eps), n_pairs=1)


def stack_scene(tex, layers, n_quads=3, shading=0):
    """n_quads axis-aligned quads at NDC depths -0.5, 0, 0.5, ... (front to
    back), each shifted right and down from the one before so that they
    overlap partly.  Quad k maps to the k-th of n_quads vertical strips of
    the RGBA texture, its UVs on texel centres (so its samples never read a
    neighbouring strip)."""
    tex = np.asarray(tex, np.float32)
    Ht, Wt, _ = tex.shape
    pos, tri, cuv = [], [], []
    for k in range(n_quads):
        x0, y0, z = -0.8 + 0.35 * k, 0.8 - 0.35 * k, -0.5 + 0.5 * k
        e = 0.9
        base = len(pos)
        pos += [(x0, y0, z), (x0 + e, y0, z), (x0 + e, y0 - e, z), (x0, y0 - e, z)]
        u0 = (k * Wt / n_quads + 0.5) / Wt
        u1 = ((k + 1) * Wt / n_quads - 0.5) / Wt
        v0, v1 = 0.5 / Ht, (Ht - 0.5) / Ht
        uvv = [(u0, v0), (u1, v0), (u1, v1), (u0, v1)]
        for t in ((0, 3, 1), (1, 3, 2)):
            tri.append(tuple(base + i for i in t))
            cuv.append([uvv[i] for i in t])
    return SimpleScene(np.array(tri, np.int32), np.array(cuv, np.float32), np.array(pos, np.float32), [tex],
                       shading=shading, layers=layers)


# ------------------------------------------------------- large triangles --

def _rot(ax_deg, ay_deg):
    ax, ay = np.radians(ax_deg), np.radians(ay_deg)
    rx = np.array([[1, 0, 0], [0, np.cos(ax), -np.sin(ax)], [0, np.sin(ax), np.cos(ax)]])
    ry = np.array([[np.cos(ay), 0, np.sin(ay)], [0, 1, 0], [-np.sin(ay), 0, np.cos(ay)]])
    return ry @ rx


def _quad(extent, z, rot, uv_scale):
    e = extent
    local = np.array([(-e, e, 0.0), (e, e, 0.0), (e, -e, 0.0), (-e, -e, 0.0)])
    pos = local @ rot.T + np.array([0.0, 0.0, z])
    tri = np.array([(0, 3, 1), (1, 3, 2)], np.int64)
    uvv = np.array([(0, 0), (1, 0), (1, 1), (0, 1)], np.float64) * uv_scale
    return pos, tri, uvv[tri]


def big_quad_scene(res, shading=0, seed=0, tex_shapes=((48, 64, 3),)):
    """Two triangles of a slanted quad that fills the whole view (each
    triangle spans the screen, far beyond 128 px from 256 px on), textured
    with a repeating UV map, seen in perspective from the default camera."""
    from paper_2404_09758_amd import scenes as S
    rng = np.random.default_rng(300 + seed)
    pos, tri, cuv = _quad(2.6, -0.3, _rot(20.0, 30.0), 2.3)
    tex = [rng.uniform(0.05, 0.95, s).astype(np.float32) for s in tex_shapes]
    ttex = [rng.uniform(0.05, 0.95, s).astype(np.float32) for s in tex_shapes]
    tpos = (pos + rng.normal(0.0, 0.01, pos.shape)).astype(np.float32)
    vs = [S.look_at_view(res, res, 0.0, 0.0), S.look_at_view(res, res - 24, 12.0, -8.0)]
    eps = [2e-3] + [1.0 / 255.0] * len(tex_shapes)
    return S.Scene("bigquad", tri.astype(np.int32), cuv.astype(np.float32), pos.astype(np.float32), tex, tpos,
                   ttex, vs, shading=shading, ambient=0.1 if shading == 1 else 0.03,
                   light_rgb=np.full(3, 1.0 if shading != 2 else 3.0, np.float32), eps=eps, lr=list(eps),
                   n_pairs=1)


def closeup_sphere_scene(res=512, shading=1, seed=0, dist=1.4):
    """The 320-triangle icosphere seen from close by (camera 0.4 above the
    surface): its nearest triangles span several hundred pixels."""
    from paper_2404_09758_amd import scenes as S
    rng = np.random.default_rng(400 + seed)
    v, f, uv = S._sphere_scene(4)
    tex = [rng.uniform(0.05, 0.95, (64, 64, 3)).astype(np.float32)]
    ttex = [rng.uniform(0.05, 0.95, (64, 64, 3)).astype(np.float32)]
    tpos = S._radial_displace(v, seed + 11, amp=0.05).astype(np.float32)
    vs = [S.look_at_view(res, res, 25.0, 10.0, dist=dist), S.look_at_view(res, res - 40, 140.0, -30.0, dist=dist)]
    eps = [1e-3, 1.0 / 255.0]
    return S.Scene("closeup", f.astype(np.int32), uv, v.astype(np.float32), tex, tpos, ttex, vs, shading=shading,
                   ambient=0.1, eps=eps, lr=list(eps), n_pairs=1)


def mixed_bin_scene(res=(264, 232), freq=16, shading=1, seed=0):
    """A fine icosphere (triangles of a few pixels) in front of a large
    background quad (two triangles spanning the view): the sphere's tiles
    hold both many small triangles and one large one."""
    from paper_2404_09758_amd import scenes as S
    rng = np.random.default_rng(500 + seed)
    v, f, uv = S._sphere_scene(freq)
    qp, qt, quv = _quad(3.2, -1.6, np.eye(3), 1.0)
    pos = np.concatenate([v, qp]).astype(np.float32)
    tri = np.concatenate([f, qt + len(v)]).astype(np.int32)
    cuv = np.concatenate([uv, quv.astype(np.float32)]).astype(np.float32)
    tex = [rng.uniform(0.05, 0.95, (40, 56, 3)).astype(np.float32)]
    ttex = [rng.uniform(0.05, 0.95, (40, 56, 3)).astype(np.float32)]
    tv = S._radial_displace(v, seed + 13, amp=0.06)
    tpos = np.concatenate([tv, qp]).astype(np.float32)
    W, Hh = res
    vs = [S.look_at_view(W, Hh, 15.0, 5.0)]
    fy = 1.0 / np.tan(np.radians(S.FOVY_DEG) / 2)
    eps = [1.5 * (S.CAM_DIST / fy) * 2.0 / Hh, 1.0 / 255.0]
    return S.Scene("mixed", tri, cuv, pos, tex, tpos, ttex, vs, shading=shading, ambient=0.1, eps=eps,
                   lr=list(eps), n_pairs=1)


def tri_spans_px(sc, view):
    """Pixel bounding-box spans (max of width, height) of the triangles with
    every vertex in front of the near plane, from a float64 projection."""
    P = np.concatenate([sc.pos.astype(np.float64), np.ones((sc.n_verts, 1))], 1) @ \
        view.view_proj.astype(np.float64).T
    ok = P[:, 3] > view.near
    sx = (P[:, 0] / P[:, 3] * 0.5 + 0.5) * view.width
    sy = (0.5 - P[:, 1] / P[:, 3] * 0.5) * view.height
    t = sc.tri
    good = ok[t].all(1)
    span = np.maximum(np.ptp(sx[t], axis=1), np.ptp(sy[t], axis=1))
    return span[good], sx, sy


def tile_bin_counts(sc, view, tile):
    """Triangles whose clipped pixel bounding box touches each tile (the
    binning's occupancy, from a float64 projection)."""
    span, sx, sy = tri_spans_px(sc, view)
    P = np.concatenate([sc.pos.astype(np.float64), np.ones((sc.n_verts, 1))], 1) @ \
        view.view_proj.astype(np.float64).T
    good = (P[:, 3] > view.near)[sc.tri].all(1)
    tx = -(-view.width // tile)
    ty = -(-view.height // tile)
    cnt = np.zeros((ty, tx), np.int64)
    big = np.zeros((ty, tx), bool)
    for t in np.nonzero(good)[0]:
        xs, ys = sx[sc.tri[t]], sy[sc.tri[t]]
        x0, x1 = max(int(np.floor(xs.min())), 0), min(int(np.floor(xs.max())), view.width - 1)
        y0, y1 = max(int(np.floor(ys.min())), 0), min(int(np.floor(ys.max())), view.height - 1)
        if x0 > x1 or y0 > y1:
            continue
        cnt[y0 // tile:y1 // tile + 1, x0 // tile:x1 // tile + 1] += 1
        if max(np.ptp(xs), np.ptp(ys)) >= 128:
            big[y0 // tile:y1 // tile + 1, x0 // tile:x1 // tile + 1] = True
    return cnt, big
