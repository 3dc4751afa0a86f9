"""Pins of the subdivision-surface parameterisation (Sec. 6.3): the oracle's
Catmull-Clark map against textbook values and invariants, the library's own
tessellation (host code, no GPU) against the oracle's, and the one-hot
estimator on a control vertex against the quantised Eq. 3."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import subdiv
from paper_2404_09758_amd import scenes as S
from tests import helpers as H


def _cube():
    V = [(x, y, z) for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)]
    ix = {v: i for i, v in enumerate(V)}
    F = [[(-1, -1, -1), (-1, 1, -1), (1, 1, -1), (1, -1, -1)], [(-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)],
         [(-1, -1, -1), (1, -1, -1), (1, -1, 1), (-1, -1, 1)], [(-1, 1, -1), (-1, 1, 1), (1, 1, 1), (1, 1, -1)],
         [(-1, -1, -1), (-1, -1, 1), (-1, 1, 1), (-1, 1, -1)], [(1, -1, -1), (1, 1, -1), (1, 1, 1), (1, -1, 1)]]
    return V, [[ix[c] for c in f] for f in F], ix


def _point(row, V):
    return tuple(sum(w * Fraction(V[i][c]) for i, w in row.items()) for c in range(3))


def test_cube_points_are_the_textbook_values():
    """Catmull and Clark's rules on the cube [-1, 1]^3: a corner's vertex
    point is (5/9, 5/9, 5/9) (times its signs), an edge point
    (3/4, 3/4, 0), a face point the face centre."""
    V, F, ix = _cube()
    faces, n, M = subdiv.refine_rational(F, 8, 1)
    assert n == 8 + 12 + 6 and len(faces) == 24
    assert _point(M[ix[(1, 1, 1)]], V) == (Fraction(5, 9),) * 3
    assert _point(M[ix[(-1, 1, -1)]], V) == (Fraction(-5, 9), Fraction(5, 9), Fraction(-5, 9))
    pts = {_point(M[j], V) for j in range(8, 20)}
    assert (Fraction(3, 4), Fraction(3, 4), Fraction(0)) in pts
    assert {_point(M[j], V) for j in range(20, 26)} == {(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1),
                                                        (0, 0, -1)}


def _torus_quads(n):
    idx = lambda i, j: (i % n) * n + (j % n)
    return [[idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)] for i in range(n) for j in range(n)]


def test_regular_quad_masks_are_the_bicubic_bspline_masks():
    """On a regular quad grid (a torus, valence 4 everywhere) one level gives
    the uniform bicubic B-spline masks: vertex point 9/16 centre, 3/32 edge
    neighbours, 1/64 diagonal ones; edge point 3/8 on the edge's ends and
    1/16 on the four vertices beside it."""
    n = 6
    faces, _, M = subdiv.refine_rational(_torus_quads(n), n * n, 1)
    idx = lambda i, j: (i % n) * n + (j % n)
    v = M[idx(2, 3)]
    assert v[idx(2, 3)] == Fraction(9, 16)
    assert all(v[idx(2 + di, 3 + dj)] == Fraction(3, 32) for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)))
    assert all(v[idx(2 + di, 3 + dj)] == Fraction(1, 64) for di, dj in ((1, 1), (1, -1), (-1, 1), (-1, -1)))
    assert len(v) == 9
    # the edge (2,3)-(3,3): the first edge point whose row holds both ends
    e_rows = [M[j] for j in range(n * n, len(M) - len(faces) // 4)]
    e = [r for r in e_rows if r.get(idx(2, 3)) == Fraction(3, 8) and r.get(idx(3, 3)) == Fraction(3, 8)]
    assert len(e) == 1
    assert sorted(w for k, w in e[0].items() if k not in (idx(2, 3), idx(3, 3))) == [Fraction(1, 16)] * 4


def test_rows_are_affine_combinations_and_counts_follow_euler():
    v, f, uv = S._sphere_scene(2)                 # 42 vertices, 80 triangles, 120 edges
    faces, n, M = subdiv.refine_rational([list(t) for t in f], 42, 2)
    assert n == (42 + 120 + 80) + 2 * 240 + 240 and len(faces) == 960
    assert all(sum(r.values()) == 1 for r in M)
    assert all(w > 0 for r in M for w in r.values())
    out = subdiv.catmull_clark(f, 42, uv, 2)
    assert out["tri"].shape == (1920, 3) and out["n_fine"] == n
    # fp32 weights are the rationals rounded once
    k = 0
    for j, r in enumerate(M):
        for i in sorted(r):
            assert out["cols"][k] == i and out["w"][k] == np.float32(float(r[i]))
            k += 1
    # tessellated positions of the sphere stay near it (the limit surface shrinks a little)
    P = np.asarray(v, np.float64)
    fine = np.array([sum(float(w) * P[i] for i, w in r.items()) for r in M])
    rad = np.linalg.norm(fine, axis=1)
    assert rad.min() > 0.85 and rad.max() <= 1.0 + 1e-12


def test_face_varying_uvs_stay_inside_the_control_triangle():
    v, f, uv = S._sphere_scene(2)
    out = subdiv.catmull_clark(f, 42, uv, 2)
    cu = uv.reshape(-1, 3, 2).astype(np.float64)
    fu = out["corner_uv"].astype(np.float64)
    for t in range(0, 1920, 7):
        ctrl = t // 24                             # 3 quads x 4 x 2 triangles per control triangle
        for c in range(3):
            # barycentrics of the fine corner in the control triangle's UV triangle
            b = np.linalg.solve(np.vstack([cu[ctrl].T, np.ones(3)]), np.r_[fu[t, c], 1.0])
            assert np.all(b > -1e-5) and np.allclose(np.round(b * 24), b * 24, atol=2e-3)


@pytest.mark.parametrize("levels", [1, 2])
def test_library_tessellation_equals_the_oracles(levels):
    """The library's own builder (C++, host) and the oracle's give the same
    triangles, corner UVs and weights, bit for bit."""
    from paper_2404_09758_amd import api
    v, f, uv = S._sphere_scene(3)
    a = api.subdivide(f, uv, v.shape[0], levels)
    b = subdiv.catmull_clark(f, v.shape[0], uv, levels)
    assert a["n_fine"] == b["n_fine"]
    for k in ("tri", "rowptr", "cols"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["w"].view(np.uint32), b["w"].view(np.uint32))
    assert np.array_equal(a["corner_uv"].view(np.uint32), b["corner_uv"].view(np.uint32))


def test_library_rejects_open_meshes_and_bad_levels():
    from paper_2404_09758_amd import api
    tri = np.array([[0, 1, 2]], np.int32)
    uv = np.zeros((1, 3, 2), np.float32)
    with pytest.raises(api.DRError):
        api.subdivide(tri, uv, 3, 1)                 # an open mesh: edges with one face
    v, f, uvs = S._sphere_scene(1)
    with pytest.raises(api.DRError):
        api.subdivide(f, uvs, v.shape[0], 3)
    with pytest.raises(api.DRError):
        api.subdivide(f + 1000, uvs, v.shape[0], 1)


def small_subdiv_scene(shading=S.SHADING_UNLIT, res=32, levels=2, freq=1, tex=8, seed=3):
    """A frequency-1 icosphere control mesh (20 triangles), `levels` levels."""
    v, f, uv = S._sphere_scene(freq)
    rng = np.random.default_rng(seed)
    texs = [rng.uniform(0.1, 0.9, (tex, tex, 3)).astype(np.float32)]
    sc = H.SimpleScene(f.astype(np.int32), uv, v.astype(np.float32), texs, shading=shading,
                       light_dir=S.unit_light())
    sc.subdiv_levels = levels
    sc.view = S.look_at_view(res, res, 20.0, 10.0)
    return sc


@pytest.mark.parametrize("shading", [S.SHADING_UNLIT, S.SHADING_LAMBERT])
def test_subdiv_onehot_equals_full_image_finite_difference(shading, oracle_lib):
    """Pin T2 on a subdivision surface: with s = e_i for a control-vertex
    coordinate (or a texel), the per-pixel estimator equals the quantised
    Eq. 3 over all pixels bit for bit -- every pixel whose colour moves with
    the control vertex has it in its set (the union of the control vertices
    its triangle's corners combine)."""
    sc = small_subdiv_scene(shading)
    o = oracle.Oracle(sc)
    assert o.d == 3 * 12 + 8 * 8 * 3
    theta = sc.flat()
    rng = np.random.default_rng(4)
    tgt = rng.random((32, 32, 3)).astype(np.float32)
    eps = [2e-2, 5e-2]
    params = list(range(36)) + list(36 + rng.choice(192, 8, replace=False))
    nonzero = 0
    for i in params:
        s = np.zeros((1, o.d), np.int8)
        s[0, i] = 1 if i % 2 else -1
        Q, K, _, _ = o.estimate(theta, [sc.view], [tgt], 0, 1, 1, eps, signs_=s)
        fp = o.pixel_loss(theta, sc.view, tgt, signs_=s[0], sign=+1, eps=eps)
        fm = o.pixel_loss(theta, sc.view, tgt, signs_=s[0], sign=-1, eps=eps)
        brute = sum(oracle.quantize(x) for x in (fp - fm).reshape(-1))
        assert Q[i] == int(s[0, i]) * brute, i
        nonzero += brute != 0
    assert nonzero >= len(params) // 2


def test_tessellated_positions_match_the_exact_map(oracle_lib):
    """The oracle's fp32 tessellation (row-ordered sums) renders the same
    image as the surface whose vertices are the exact rational map applied
    in float64 and rounded once: identical IDs away from a handful of
    edge pixels, colours within fp32 rounding elsewhere."""
    sc = small_subdiv_scene(S.SHADING_LAMBERT, res=48)
    o = oracle.Oracle(sc)
    v, f, _ = S._sphere_scene(1)
    _, _, M = subdiv.refine_rational([list(t) for t in f], v.shape[0], 2)
    P = np.asarray(sc.pos, np.float64)
    exact = np.array([sum(float(w) * P[i] for i, w in r.items()) for r in M]).astype(np.float32)
    plain = H.SimpleScene(o.surface["tri"], o.surface["corner_uv"], exact, sc.tex, shading=sc.shading,
                          light_dir=sc.light_dir)
    rgb_a, id_a, _ = o.render(sc.flat(), sc.view)
    rgb_b, id_b, _ = oracle.Oracle(plain).render(plain.flat(), sc.view)
    same = id_a == id_b
    assert (id_a != oracle.BG_ID).sum() > 500
    assert same.mean() > 0.99
    assert np.abs(rgb_a[same] - rgb_b[same]).max() < 1e-4
