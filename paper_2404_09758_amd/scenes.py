"""Seeded synthetic scene generators.

This module produces the inputs of the estimator (meshes, per-corner UVs,
textures, cameras, lights) as plain numpy arrays.  It holds none of the
estimator's arithmetic: no perturbation, raster, shading, loss or scatter.
Both the GPU library and the CPU oracle consume exactly these arrays.

The paper's own assets (cow, skull, dancer, the teaser surface) are not
available, so seeded geodesic icospheres stand in for them, at the scale the
paper reports: 1024^2 renders of ~50K triangles with 1024^2 PBR maps (teaser
caption), and d = 3*vertices + 3*texels parameters (the performance table of
the nvDiffRast comparison, Sec. 6.2).

Parameter layout shared by every consumer (Sec. 4.1, Table 1: theta holds
geometry and textures):
    theta = [ positions (V,3) | texture 0 (H0,W0,C0) | texture 1 | ... ]
Texture roles: 0 = albedo (RGB), 1 = tangent-space normal map (RGB),
2 = roughness (R).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SHADING_UNLIT = 0
SHADING_LAMBERT = 1
SHADING_GGX = 2

TEX_FOOTPRINT = 0   # the 2x2 bilinear footprint texels contribute
TEX_NEAREST = 1     # only the texel nearest the sample contributes (Sec. 4.4)

AVG_COUNT = 0       # divide each gradient by its contribution count
AVG_PAIRS = 1       # divide by the number of antithetic pairs (Eq. 9)

OPT_ADAM = 0
OPT_SGD = 1

FOVY_DEG = 45.0
NEAR = 0.1
FAR = 10.0
CAM_DIST = 3.0


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
                  (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
                  (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    f = np.array(f, dtype=np.int64)
    # enforce outward counter-clockwise winding
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def geodesic_icosphere(freq: int):
    """Unit geodesic icosphere of frequency `freq`: F = 20 n^2, V = 10 n^2 + 2.

    Each icosahedron face is split into a triangular grid of n^2 triangles,
    whose points are projected to the unit sphere.  Winding is outward CCW.
    """
    if freq < 1:
        raise ValueError("freq must be >= 1")
    iv, ifaces = _icosahedron()
    n = freq
    verts: list = []
    index: dict = {}

    def vid(p):
        p = p / np.linalg.norm(p)
        key = (round(p[0], 9), round(p[1], 9), round(p[2], 9))
        k = index.get(key)
        if k is None:
            k = len(verts)
            index[key] = k
            verts.append(p)
        return k

    tris = []
    for (ia, ib, ic) in ifaces:
        a, b, c = iv[ia], iv[ib], iv[ic]
        grid = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                grid[(i, j)] = vid(a + (b - a) * (i / n) + (c - a) * (j / n))
        for i in range(n):
            for j in range(n - i):
                tris.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j < n - 1:
                    tris.append((grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]))
    v = np.array(verts, dtype=np.float64)
    f = np.array(tris, dtype=np.int64)
    assert len(v) == 10 * n * n + 2 and len(f) == 20 * n * n
    return v, f


def midpoint_split(v: np.ndarray, f: np.ndarray):
    """One 1-to-4 midpoint split; midpoints stay on the flat faces."""
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    uniq, inv = np.unique(e, axis=0, return_inverse=True)
    inv = inv.reshape(3, len(f)).T + len(v)
    mid = 0.5 * (v[uniq[:, 0]] + v[uniq[:, 1]])
    nv = np.concatenate([v, mid], axis=0)
    a, b, c = f[:, 0], f[:, 1], f[:, 2]
    mab, mbc, mca = inv[:, 0], inv[:, 1], inv[:, 2]
    nf = np.stack([np.stack([a, mab, mca], 1), np.stack([mab, b, mbc], 1),
                   np.stack([mca, mbc, c], 1), np.stack([mab, mbc, mca], 1)], axis=1)
    return nv, nf.reshape(-1, 3)


def spherical_corner_uv(v: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Per-corner spherical UVs [F,3,2] with the seam fixed per triangle.

    u = atan2(z, x)/(2 pi) + 1/2, v = acos(y)/pi on the unit direction.  A
    triangle straddling the seam gets u += 1 on its corners below 1/2; a
    corner at a pole takes the mean u of the triangle's other corners.
    """
    d = v / np.linalg.norm(v, axis=1, keepdims=True)
    u = np.arctan2(d[:, 2], d[:, 0]) / (2 * math.pi) + 0.5
    w = np.arccos(np.clip(d[:, 1], -1.0, 1.0)) / math.pi
    cu = u[f].copy()
    cv = w[f].copy()
    wrap = (cu.max(1) - cu.min(1)) > 0.5
    cu[wrap] = np.where(cu[wrap] < 0.5, cu[wrap] + 1.0, cu[wrap])
    pole = np.abs(d[f][:, :, 1]) > 1.0 - 1e-9
    for k in range(3):
        rows = np.nonzero(pole[:, k])[0]
        others = [j for j in range(3) if j != k]
        cu[rows, k] = 0.5 * (cu[rows, others[0]] + cu[rows, others[1]])
    return np.stack([cu, cv], axis=2).astype(np.float32)


# --------------------------------------------------------------------------
# value noise
# --------------------------------------------------------------------------

def _smooth(t):
    return t * t * (3.0 - 2.0 * t)


def value_noise_3d(p: np.ndarray, seed: int, octaves=4, f0=1.5, gain=0.5, period=64):
    """Seeded 3D value noise in [0,1): lattice values U[0,1), smoothstep."""
    rng = np.random.default_rng(seed)
    table = rng.random((octaves, period, period, period))
    total = np.zeros(len(p))
    norm = 0.0
    amp = 1.0
    for o in range(octaves):
        q = (p * (f0 * 2 ** o)) + 17.0
        i0 = np.floor(q).astype(np.int64)
        t = _smooth(q - i0)
        acc = np.zeros(len(p))
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    wgt = ((t[:, 0] if dx else 1 - t[:, 0]) * (t[:, 1] if dy else 1 - t[:, 1])
                           * (t[:, 2] if dz else 1 - t[:, 2]))
                    val = table[o, (i0[:, 0] + dx) % period, (i0[:, 1] + dy) % period,
                                (i0[:, 2] + dz) % period]
                    acc += wgt * val
        total += amp * acc
        norm += amp
        amp *= gain
    return total / norm


def value_noise_2d(h: int, w: int, seed: int, channels=1, octaves=4, f0=4, gain=0.5):
    """Seeded tileable 2D value noise image [h,w,channels] in [0,1)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((h, w, channels))
    ys = (np.arange(h) + 0.5) / h
    xs = (np.arange(w) + 0.5) / w
    for c in range(channels):
        norm = 0.0
        amp = 1.0
        for o in range(octaves):
            fr = int(f0 * 2 ** o)
            lat = rng.random((fr, fr))
            gx = xs * fr
            gy = ys * fr
            x0 = np.floor(gx).astype(np.int64)
            y0 = np.floor(gy).astype(np.int64)
            tx = _smooth(gx - x0)[None, :]
            ty = _smooth(gy - y0)[:, None]
            a = lat[y0[:, None] % fr, x0[None, :] % fr]
            b = lat[y0[:, None] % fr, (x0[None, :] + 1) % fr]
            cc = lat[(y0[:, None] + 1) % fr, x0[None, :] % fr]
            d = lat[(y0[:, None] + 1) % fr, (x0[None, :] + 1) % fr]
            val = (a * (1 - tx) + b * tx) * (1 - ty) + (cc * (1 - tx) + d * tx) * ty
            out[:, :, c] += amp * val
            norm += amp
            amp *= gain
        out[:, :, c] /= norm
    return out


def normal_map_from_height(hgt: np.ndarray, strength=4.0) -> np.ndarray:
    """Tangent-space normal map (encoded (n+1)/2) from a periodic height field."""
    h = hgt[:, :, 0]
    dx = (np.roll(h, -1, axis=1) - np.roll(h, 1, axis=1)) * 0.5 * h.shape[1] / 64.0
    dy = (np.roll(h, -1, axis=0) - np.roll(h, 1, axis=0)) * 0.5 * h.shape[0] / 64.0
    n = np.stack([-dx * strength, -dy * strength, np.ones_like(h)], axis=2)
    n /= np.linalg.norm(n, axis=2, keepdims=True)
    return 0.5 * n + 0.5


# --------------------------------------------------------------------------
# cameras and lights
# --------------------------------------------------------------------------

@dataclass
class View:
    width: int
    height: int
    view_proj: np.ndarray      # float32 [4,4], row-major, acts on column vectors
    cam_pos: np.ndarray        # float32 [3]
    near: float = NEAR         # vertices with clip w below this are culled


def look_at_view(width, height, azimuth_deg, elevation_deg, dist=CAM_DIST,
                 fovy_deg=FOVY_DEG, near=NEAR, far=FAR) -> View:
    """Right-handed y-up look-at camera aimed at the origin, GL-style
    perspective; built in float64 and rounded to float32 once."""
    az = math.radians(azimuth_deg)
    el = math.radians(elevation_deg)
    eye = np.array([dist * math.cos(el) * math.sin(az), dist * math.sin(el),
                    dist * math.cos(el) * math.cos(az)])
    fwd = -eye / np.linalg.norm(eye)
    up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    true_up = np.cross(right, fwd)
    view = np.eye(4)
    view[0, :3] = right
    view[1, :3] = true_up
    view[2, :3] = -fwd
    view[:3, 3] = -view[:3, :3] @ eye
    aspect = width / height
    fy = 1.0 / math.tan(math.radians(fovy_deg) / 2)
    proj = np.zeros((4, 4))
    proj[0, 0] = fy / aspect
    proj[1, 1] = fy
    proj[2, 2] = (far + near) / (near - far)
    proj[2, 3] = 2 * far * near / (near - far)
    proj[3, 2] = -1.0
    vp = (proj @ view).astype(np.float32)
    return View(width, height, vp, eye.astype(np.float32), float(near))


def unit_light(direction=(1.0, 1.0, 1.0)) -> np.ndarray:
    d = np.asarray(direction, dtype=np.float64)
    return (d / np.linalg.norm(d)).astype(np.float32)


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------

@dataclass
class Scene:
    """Fixed scene data plus the initial and target parameter sets."""
    name: str
    tri: np.ndarray                 # int32 [F,3]
    corner_uv: np.ndarray           # float32 [F,3,2]
    pos: np.ndarray                 # float32 [V,3] initial positions
    tex: list                       # float32 [H,W,C] initial textures
    target_pos: np.ndarray
    target_tex: list
    views: list                     # [View]
    shading: int = SHADING_UNLIT
    tex_mode: int = TEX_FOOTPRINT
    light_dir: np.ndarray = field(default_factory=unit_light)
    light_rgb: np.ndarray = field(default_factory=lambda: np.ones(3, np.float32))
    ambient: float = 0.1
    diffuse: float = 0.9
    eps: list = field(default_factory=list)     # per block: pos, tex0, tex1, ...
    lr: list = field(default_factory=list)      # per block
    n_pairs: int = 1
    optimizer: int = OPT_ADAM
    averaging: int = AVG_COUNT
    steps: int = 1
    seed: int = 0
    layers: int = 0                 # 0 opaque; 1..4 semi-transparent (albedo RGBA)
    subdiv_levels: int = 0          # > 0: tri / corner_uv / pos are a Catmull-Clark control mesh

    @property
    def n_verts(self):
        return int(self.pos.shape[0])

    @property
    def n_tris(self):
        return int(self.tri.shape[0])

    @property
    def n_params(self):
        return param_count(self.n_verts, [t.shape for t in self.tex])

    def flat_params(self, target=False) -> np.ndarray:
        pos = self.target_pos if target else self.pos
        tex = self.target_tex if target else self.tex
        return np.concatenate([pos.reshape(-1)] + [t.reshape(-1) for t in tex]).astype(np.float32)


def param_count(n_verts: int, tex_shapes) -> int:
    """d = 3 V + sum over textures of H W C."""
    return 3 * n_verts + sum(int(h) * int(w) * int(c) for (h, w, c) in tex_shapes)


def texel_classes(tex_shapes):
    """Textures sharing one resolution share their texel groups.

    Returns (class_of_texture, class_sizes) in order of first appearance."""
    classes = []
    cls = []
    for (h, w, _c) in tex_shapes:
        key = (int(h), int(w))
        if key not in classes:
            classes.append(key)
        cls.append(classes.index(key))
    return cls, classes


def group_count(n_verts: int, tex_shapes) -> int:
    _, classes = texel_classes(tex_shapes)
    return n_verts + sum(h * w for (h, w) in classes)


def _sphere_scene(freq, splits=0):
    v, f = geodesic_icosphere(freq)
    for _ in range(splits):
        v, f = midpoint_split(v, f)
    uv = spherical_corner_uv(v, f)
    return v, f, uv


def make_tiny(seed=1) -> Scene:
    """64x64 px, 320-triangle icosphere, 64^2 RGB albedo, unlit, 1 view."""
    v, f, uv = _sphere_scene(4)
    rng_a = np.random.default_rng(seed * 1000 + 1)
    rng_b = np.random.default_rng(seed * 1000 + 2)
    rng_c = np.random.default_rng(seed * 1000 + 3)
    tex0 = rng_a.random((64, 64, 3)).astype(np.float32)
    tgt_tex = rng_b.random((64, 64, 3)).astype(np.float32)
    tgt_pos = (v + rng_c.normal(0.0, 0.02, size=v.shape)).astype(np.float32)
    return Scene("tiny", f.astype(np.int32), uv, v.astype(np.float32), [tex0], tgt_pos, [tgt_tex],
                 [look_at_view(64, 64, 0.0, 0.0)], shading=SHADING_UNLIT,
                 eps=[1e-3, 1e-2], lr=[3e-5, 5e-3], n_pairs=1, optimizer=OPT_SGD, steps=50,
                 seed=seed)


def _radial_displace(v, seed, amp=0.1):
    d = v / np.linalg.norm(v, axis=1, keepdims=True)
    n = value_noise_3d(d, seed)
    return d * (1.0 + amp * (2.0 * n - 1.0))[:, None] * np.linalg.norm(v, axis=1, keepdims=True)


def make_mid(seed=2, res=512, views=8, pairs=16) -> Scene:
    """512^2 px, 20480-triangle icosphere, 512^2 RGBA8 albedo as fp32 RGB,
    Lambert, 8 ring views, 16 pairs, Adam lr 1e-3, count averaging."""
    v, f, uv = _sphere_scene(32)
    tex0 = np.full((res, res, 3), 128.0 / 255.0, dtype=np.float32)
    noise = value_noise_2d(res, res, seed * 1000 + 11, channels=3)
    tgt_tex = (np.round(noise * 255.0) / 255.0).astype(np.float32)
    tgt_pos = _radial_displace(v, seed * 1000 + 12).astype(np.float32)
    fy = 1.0 / math.tan(math.radians(FOVY_DEG) / 2)
    eps_pos = 1.5 * (CAM_DIST / fy) * 2.0 / res      # ~1.5 px at distance 3
    vs = [look_at_view(res, res, 45.0 * k, 0.0) for k in range(views)]
    return Scene("mid", f.astype(np.int32), uv, v.astype(np.float32), [tex0], tgt_pos, [tgt_tex], vs,
                 shading=SHADING_LAMBERT, eps=[eps_pos, 1.0 / 255.0], lr=[1e-3, 1e-3],
                 n_pairs=pairs, optimizer=OPT_ADAM, steps=100, seed=seed)


def make_layered(layers: int, seed=9, res=512, views=4, pairs=8) -> Scene:
    """Semi-transparent variant of the mid workload (Sec. 4.4 "Transparent
    geometry"): the 20480-triangle icosphere at 512^2 px, Lambert, with a
    512^2 RGBA albedo whose fourth channel is the opacity (initial 0.5,
    target a value-noise field in [0.3, 0.9]); the `layers` nearest
    fragments of each pixel are composited, so the back of the sphere shows
    through its front.  layers = 0 gives the opaque scene with the same
    colour channels, for comparison.  4 ring views, 8 pairs, Adam."""
    v, f, uv = _sphere_scene(32)
    c = 4 if layers > 0 else 3
    tex0 = np.full((res, res, c), 0.5, dtype=np.float32)
    tgt = np.empty((res, res, c), np.float32)
    tgt[..., :3] = value_noise_2d(res, res, seed * 1000 + 11, channels=3)
    if c == 4:
        tgt[..., 3] = 0.3 + 0.6 * value_noise_2d(res, res, seed * 1000 + 13, channels=1)[..., 0]
    tgt_pos = _radial_displace(v, seed * 1000 + 12).astype(np.float32)
    fy = 1.0 / math.tan(math.radians(FOVY_DEG) / 2)
    eps_pos = 1.5 * (CAM_DIST / fy) * 2.0 / res
    vs = [look_at_view(res, res, 90.0 * k + 20.0, 15.0) for k in range(views)]
    return Scene(f"layered{layers}", f.astype(np.int32), uv, v.astype(np.float32), [tex0], tgt_pos, [tgt], vs,
                 shading=SHADING_LAMBERT, eps=[eps_pos, 1.0 / 255.0], lr=[eps_pos, 1.0 / 255.0],
                 n_pairs=pairs, optimizer=OPT_ADAM, steps=1, seed=seed, layers=layers)


def make_subdiv(seed=4, res=1024, tex_res=1024, views=4, pairs=8, control_freq=10, levels=2,
                 shading=SHADING_GGX) -> Scene:
    """Subdivision-surface variant of the paper workload (Sec. 6.3 and the
    teaser: a 2K-triangle control mesh, two Catmull-Clark levels, about 50K
    triangles): the control mesh is a frequency-10 geodesic icosphere (2000
    triangles, 1002 vertices) whose vertices are the position parameters;
    two levels give 24 000 quads = 48 000 tessellated triangles.  Albedo,
    normal and roughness maps at 1024^2, GGX, 4 views, 8 pairs, Adam with
    lr = eps.  The target displaces the control vertices radially."""
    v, f, uv = _sphere_scene(control_freq)
    t = tex_res
    if shading == SHADING_GGX:
        tex = [np.full((t, t, 3), 0.5, np.float32), np.empty((t, t, 3), np.float32),
               np.full((t, t, 1), 0.5, np.float32)]
        tex[1][:] = (0.5, 0.5, 1.0)
        hgt = value_noise_2d(t, t, seed * 1000 + 32, channels=1, f0=8)
        tgt = [value_noise_2d(t, t, seed * 1000 + 31, channels=3).astype(np.float32),
               normal_map_from_height(hgt).astype(np.float32),
               (0.2 + 0.6 * value_noise_2d(t, t, seed * 1000 + 33, channels=1)).astype(np.float32)]
    else:
        tex = [np.full((t, t, 3), 0.5, np.float32)]
        tgt = [value_noise_2d(t, t, seed * 1000 + 31, channels=3).astype(np.float32)]
    tgt_pos = _radial_displace(v, seed * 1000 + 34).astype(np.float32)
    fy = 1.0 / math.tan(math.radians(FOVY_DEG) / 2)
    eps_pos = 1.5 * (CAM_DIST / fy) * 2.0 / res
    q = 1.0 / 255.0
    eps = [eps_pos] + [q] * len(tex)
    vs = [look_at_view(res, res, 90.0 * k, 20.0) for k in range(views)]
    return Scene("subdiv", f.astype(np.int32), uv, v.astype(np.float32), tex, tgt_pos, tgt, vs,
                 shading=shading, light_rgb=np.full(3, 3.0 if shading == SHADING_GGX else 1.0, np.float32),
                 ambient=0.03 if shading == SHADING_GGX else 0.1, eps=eps, lr=list(eps), n_pairs=pairs,
                 optimizer=OPT_ADAM, steps=1, seed=seed, subdiv_levels=levels)


def make_paper(seed=3, res=1024, tex_res=1024, views=4, pairs=8, control_freq=12, splits=2) -> Scene:
    """1024^2 px, 46080-triangle sphere (frequency-12 control, two 1-to-4
    splits), albedo/normal/roughness maps at 1024^2, GGX, 4 views, 8 pairs."""
    v, f, uv = _sphere_scene(control_freq, splits)
    t = tex_res
    albedo = np.full((t, t, 3), 0.5, np.float32)
    normal = np.empty((t, t, 3), np.float32)
    normal[:] = (0.5, 0.5, 1.0)
    rough = np.full((t, t, 1), 0.5, np.float32)
    tgt_alb = value_noise_2d(t, t, seed * 1000 + 21, channels=3).astype(np.float32)
    hgt = value_noise_2d(t, t, seed * 1000 + 22, channels=1, f0=8)
    tgt_nrm = normal_map_from_height(hgt).astype(np.float32)
    tgt_rgh = (0.2 + 0.6 * value_noise_2d(t, t, seed * 1000 + 23, channels=1)).astype(np.float32)
    tgt_pos = _radial_displace(v, seed * 1000 + 24).astype(np.float32)
    fy = 1.0 / math.tan(math.radians(FOVY_DEG) / 2)
    eps_pos = 1.5 * (CAM_DIST / fy) * 2.0 / res
    q = 1.0 / 255.0
    vs = [look_at_view(res, res, 90.0 * k, 20.0) for k in range(views)]
    return Scene("paper", f.astype(np.int32), uv, v.astype(np.float32), [albedo, normal, rough],
                 tgt_pos, [tgt_alb, tgt_nrm, tgt_rgh], vs, shading=SHADING_GGX, ambient=0.03,
                 light_rgb=np.full(3, 3.0, np.float32),
                 eps=[eps_pos, q, q, q], lr=[eps_pos, q, q, q], n_pairs=pairs,
                 optimizer=OPT_ADAM, steps=1, seed=seed)


def make_octa_small(seed=4, res=16) -> Scene:
    """16x16 px check scene: octahedron with one projected 1-to-4 split
    (32 triangles / 18 vertices), 16^2 RGB albedo, unlit."""
    v = np.array([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)], np.float64)
    f = np.array([(0, 2, 4), (4, 2, 1), (1, 2, 5), (5, 2, 0),
                  (4, 3, 0), (1, 3, 4), (5, 3, 1), (0, 3, 5)], np.int64)
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    v, f = midpoint_split(v, f)
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    uv = spherical_corner_uv(v, f)
    rng = np.random.default_rng(seed * 1000 + 31)
    tex0 = rng.random((16, 16, 3)).astype(np.float32)
    tgt_tex = rng.random((16, 16, 3)).astype(np.float32)
    tgt_pos = (v + rng.normal(0.0, 0.05, size=v.shape)).astype(np.float32)
    return Scene("octa", f.astype(np.int32), uv, v.astype(np.float32), [tex0], tgt_pos, [tgt_tex],
                 [look_at_view(res, res, 30.0, 15.0)], shading=SHADING_UNLIT,
                 eps=[1e-3, 1e-2], lr=[1e-3, 1e-2], n_pairs=256, optimizer=OPT_ADAM, seed=seed)


def make_diff_run(seed=5, res=256) -> Scene:
    """256^2 px, frequency-16 icosphere (5120 triangles), 256^2 albedo, unlit."""
    v, f, uv = _sphere_scene(16)
    rng = np.random.default_rng(seed * 1000 + 41)
    tex0 = np.full((256, 256, 3), 0.5, np.float32)
    tgt_tex = value_noise_2d(256, 256, seed * 1000 + 42, channels=3).astype(np.float32)
    tgt_pos = _radial_displace(v, seed * 1000 + 43).astype(np.float32)
    del rng
    return Scene("diff", f.astype(np.int32), uv, v.astype(np.float32), [tex0], tgt_pos, [tgt_tex],
                 [look_at_view(res, res, 0.0, 0.0)], shading=SHADING_UNLIT,
                 eps=[1e-3, 1e-2], lr=[1e-3, 1e-2], n_pairs=64, optimizer=OPT_ADAM, seed=seed)


def make_batch_scene(b: int, seed=6) -> Scene:
    """Scene b of the 64-scene batch: F log-uniform in [1e3, 5e4], render
    size and texture side drawn from {128,256,512,1024}, Lambert, 1 view,
    4 pairs, Adam."""
    rng = np.random.default_rng(seed * 100000 + b)
    t_b = math.exp(rng.uniform(math.log(1e3), math.log(5e4)))
    freq = max(1, int(round(math.sqrt(t_b / 20.0))))
    res = int(rng.choice([128, 256, 512, 1024]))
    ts = int(rng.choice([128, 256, 512, 1024]))
    v, f, uv = _sphere_scene(freq)
    tex0 = np.full((ts, ts, 3), 0.5, np.float32)
    tgt_tex = value_noise_2d(ts, ts, seed * 100000 + 500 + b, channels=3).astype(np.float32)
    tgt_pos = _radial_displace(v, seed * 100000 + 900 + b).astype(np.float32)
    fy = 1.0 / math.tan(math.radians(FOVY_DEG) / 2)
    eps_pos = 1.5 * (CAM_DIST / fy) * 2.0 / res
    az = float(rng.uniform(0.0, 360.0))
    return Scene(f"batch{b}", f.astype(np.int32), uv, v.astype(np.float32), [tex0], tgt_pos, [tgt_tex],
                 [look_at_view(res, res, az, 10.0)], shading=SHADING_LAMBERT,
                 eps=[eps_pos, 1.0 / 255.0], lr=[eps_pos, 1.0 / 255.0], n_pairs=4,
                 optimizer=OPT_ADAM, seed=seed + b)


CONFIGS = {
    "tiny": make_tiny,
    "mid": make_mid,
    "paper": make_paper,
    "octa": make_octa_small,
    "diff": make_diff_run,
    "subdiv": make_subdiv,
}


def make_soup(n_tris: int, res: int = 512, seed: int = 7, pairs: int = 128) -> Scene:
    """Triangle soup of the per-pixel vs full-image validation (Sec. 6.1):
    n_tris independent triangles, each with 12 parameters (its 3 vertices and
    one RGB colour), unlit, seen from the front.  The colour of triangle t is
    texel t of an h x w colour map with exactly n_tris texels (h the largest
    divisor of n_tris not above its square root), whose corner UVs all sit
    on that texel's centre; nearest-texel mode credits only that texel, so
    d = 9 n_tris + 3 n_tris = 12 n_tris, the count of Sec. 6.1.  The target
    is a seeded value-noise image (the paper's target image is not
    available), so `target_pos`/`target_tex` are unused."""
    rng = np.random.default_rng(seed * 1000 + n_tris)
    half = CAM_DIST * math.tan(math.radians(FOVY_DEG) / 2)
    centres = np.stack([rng.uniform(-half, half, n_tris), rng.uniform(-half, half, n_tris),
                        rng.uniform(-0.2, 0.2, n_tris)], 1)
    size = 2.5 * 2 * half / math.sqrt(n_tris)
    offs = rng.normal(0.0, size / 2, (n_tris, 3, 3))
    offs[:, :, 2] *= 0.1
    pos = (centres[:, None, :] + offs).reshape(-1, 3)
    tri = np.arange(3 * n_tris, dtype=np.int64).reshape(n_tris, 3)
    a, b, c = pos[tri[:, 0]], pos[tri[:, 1]], pos[tri[:, 2]]
    flip = np.cross(b - a, c - a)[:, 2] < 0                 # face the camera (+z)
    tri[flip] = tri[flip][:, [0, 2, 1]]
    h = max(k for k in range(1, math.isqrt(n_tris) + 1) if n_tris % k == 0)
    w = n_tris // h
    tx, ty = np.arange(n_tris) % w, np.arange(n_tris) // w
    uv = np.stack([(tx + 0.5) / w, (ty + 0.5) / h], 1).astype(np.float32)
    corner_uv = np.repeat(uv[:, None, :], 3, axis=1)
    colours = rng.uniform(0.0, 1.0, (h, w, 3)).astype(np.float32)
    fy = 1.0 / math.tan(math.radians(FOVY_DEG) / 2)
    eps_pos = 1.5 * (CAM_DIST / fy) * 2.0 / res
    sc = Scene(f"soup{n_tris}", tri.astype(np.int32), corner_uv, pos.astype(np.float32), [colours],
               pos.astype(np.float32), [colours], [look_at_view(res, res, 0.0, 0.0)], shading=SHADING_UNLIT,
               tex_mode=TEX_NEAREST, eps=[eps_pos, 1.0 / 64.0], lr=[eps_pos, 1.0 / 64.0], n_pairs=pairs,
               optimizer=OPT_ADAM, seed=seed)
    sc.target_image = value_noise_2d(res, res, seed * 1000 + 77, channels=3, f0=2).astype(np.float32)
    return sc
