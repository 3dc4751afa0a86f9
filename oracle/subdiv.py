"""Catmull-Clark refinement of a control mesh, in exact rational arithmetic.

TEST INFRASTRUCTURE ONLY (part of the oracle): only the tests, the smoke
check and the CPU baseline leg of the benchmark may use it.

Sec. 6.3 "Subdivision surfaces" optimises the control mesh of a
Catmull-Clark surface (Catmull and Clark 1978) tessellated on the fly: each
tessellated vertex is a fixed linear combination of control vertices, so a
pixel depends on the control vertices that the corners of its tessellated
triangle combine.  This module computes that linear map S (fine vertex ->
control weights) level by level with fractions.Fraction, so every weight is
the exact rational the refinement rules give, and rounds each weight to fp32
once at the end.

Refinement rules of one level, on a closed manifold mesh of polygons:
  face point   f = average of the face's vertices;
  edge point   e = (a + b + f1 + f2) / 4 for the edge (a, b) between faces f1, f2;
  vertex point v' = (Q + 2 R + (n - 3) v) / n, n = valence, Q = average of the
               adjacent face points, R = average of the midpoints of the
               adjacent edges.
Numbering of the refined mesh (a convention the GPU library's own builder
follows as well): vertex points first (vertex i keeps index i), then edge
points in order of first appearance (faces in order, each face's edges
(v_k, v_k+1) in order), then face points in face order.  Face f with
vertices v_0..v_{m-1} becomes the quads (v'_k, e(v_k, v_k+1), f', e(v_k-1, v_k))
for k = 0..m-1, in that order.  After the last level each quad
(q0, q1, q2, q3) is split into the triangles (q0, q1, q2) and (q0, q2, q3).

Texture coordinates are face-varying and refined linearly inside each
control triangle (the refinement points' positions within the triangle,
without smoothing): a fine corner's UV is sum_k (n_k / 24) uv_k over the
control triangle's corners, the n_k integers (the barycentrics of two
levels have denominators dividing 24), evaluated in float64 as
((n0 ua + n1 ub) + n2 uc) / 24 and rounded to fp32.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _refine(faces, n_verts, bary=None):
    """One Catmull-Clark level.  faces: list of vertex-index lists.  Returns
    (new_faces, n_new, M, new_bary): M[j] is the list of (old index,
    Fraction) of new vertex j; bary (optional) maps each face's corners to
    barycentric Fractions triples and is carried to the new faces."""
    edge_id = {}
    edges = []                      # (a, b) in first-appearance orientation
    edge_faces = []
    for fi, f in enumerate(faces):
        m = len(f)
        for k in range(m):
            a, b = f[k], f[(k + 1) % m]
            key = (min(a, b), max(a, b))
            if key not in edge_id:
                edge_id[key] = len(edges)
                edges.append((a, b))
                edge_faces.append([])
            edge_faces[edge_id[key]].append(fi)
    n_e, n_f = len(edges), len(faces)
    e0, f0 = n_verts, n_verts + n_e

    def face_point(fi):
        f = faces[fi]
        w = Fraction(1, len(f))
        acc = {}
        for v in f:
            acc[v] = acc.get(v, Fraction(0)) + w
        return acc

    fps = [face_point(fi) for fi in range(n_f)]

    def add(acc, terms, scale):
        for v, w in terms.items():
            acc[v] = acc.get(v, Fraction(0)) + w * scale

    M = [None] * (n_verts + n_e + n_f)
    for ei, (a, b) in enumerate(edges):
        fl = edge_faces[ei]
        if len(fl) != 2:
            raise ValueError("the control mesh must be a closed manifold")
        acc = {}
        add(acc, {a: Fraction(1)}, Fraction(1, 4))
        add(acc, {b: Fraction(1)}, Fraction(1, 4))
        add(acc, fps[fl[0]], Fraction(1, 4))
        add(acc, fps[fl[1]], Fraction(1, 4))
        M[e0 + ei] = acc
    for fi in range(n_f):
        M[f0 + fi] = dict(fps[fi])
    vfaces = [[] for _ in range(n_verts)]
    vnbrs = [set() for _ in range(n_verts)]
    for fi, f in enumerate(faces):
        m = len(f)
        for k in range(m):
            vfaces[f[k]].append(fi)
            vnbrs[f[k]].add(f[(k + 1) % m])
            vnbrs[f[k]].add(f[(k - 1) % m])
    for v in range(n_verts):
        n = len(vnbrs[v])
        if n == 0:
            M[v] = {v: Fraction(1)}
            continue
        acc = {}
        for fi in vfaces[v]:                        # Q / n
            add(acc, fps[fi], Fraction(1, n * n))
        for w_ in vnbrs[v]:                         # 2 R / n, R = avg (v + w) / 2
            add(acc, {v: Fraction(1), w_: Fraction(1)}, Fraction(1, n * n))
        add(acc, {v: Fraction(1)}, Fraction(n - 3, n))
        M[v] = acc
    new_faces, new_bary = [], []
    for fi, f in enumerate(faces):
        m = len(f)
        for k in range(m):
            a, b, p = f[k], f[(k + 1) % m], f[(k - 1) % m]
            eab = e0 + edge_id[(min(a, b), max(a, b))]
            epa = e0 + edge_id[(min(p, a), max(p, a))]
            new_faces.append([a, eab, f0 + fi, epa])
            if bary is not None:
                B = bary[fi]
                mid = lambda x, y: tuple((x[i] + y[i]) / 2 for i in range(3))
                cen = tuple(sum(B[j][i] for j in range(m)) / m for i in range(3))
                new_bary.append([B[k], mid(B[k], B[(k + 1) % m]), cen, mid(B[(k - 1) % m], B[k])])
    return new_faces, n_verts + n_e + n_f, M, (new_bary if bary is not None else None)


def _compose(M2, M1):
    """(M2 o M1): rows of M2 over level-1 vertices, M1 over level-0."""
    out = []
    for row in M2:
        acc = {}
        for j, w in row.items():
            for i, w1 in M1[j].items():
                acc[i] = acc.get(i, Fraction(0)) + w * w1
        out.append({i: w for i, w in acc.items() if w != 0})
    return out


def refine_rational(faces, n_verts, levels):
    """The exact map after `levels` levels: (faces, n_fine, rows) with rows[j]
    a dict control index -> Fraction.  faces may be any polygons."""
    M = [{i: Fraction(1)} for i in range(n_verts)]
    cur, n = [list(f) for f in faces], n_verts
    for _ in range(levels):
        cur, n_new, Ml, _ = _refine(cur, n)
        M = _compose(Ml, M)
        n = n_new
    return cur, n, M


def catmull_clark(tri, n_verts, corner_uv, levels):
    """Refine a triangle control mesh `levels` (>= 1) times and triangulate.

    Returns dict(tri int32 [F_f, 3], n_fine, rowptr int32 [n_fine + 1],
    cols int32 [nnz] (ascending within a row), w float32 [nnz],
    corner_uv float32 [F_f, 3, 2]); row j of (rowptr, cols, w) is fine
    vertex j as a combination of control vertices."""
    tri = np.asarray(tri, np.int64)
    cuv = np.asarray(corner_uv, np.float32).reshape(-1, 3, 2)
    faces = [list(map(int, t)) for t in tri]
    one, zero = Fraction(1), Fraction(0)
    bary = [[(one, zero, zero), (zero, one, zero), (zero, zero, one)] for _ in faces]
    owner = list(range(len(faces)))             # control triangle of each face
    M = [{i: one} for i in range(n_verts)]
    cur, n = faces, n_verts
    for _ in range(levels):
        nf_before = [len(f) for f in cur]
        cur2, n_new, Ml, bary = _refine(cur, n, bary)
        owner = [owner[fi] for fi, m in enumerate(nf_before) for _ in range(m)]
        M = _compose(Ml, M)
        cur, n = cur2, n_new
    out_tri, out_uv = [], []
    for fi, q in enumerate(cur):
        B = bary[fi]
        uv = cuv[owner[fi]].astype(np.float64)
        for (i0, i1, i2) in ((0, 1, 2), (0, 2, 3)):
            out_tri.append((q[i0], q[i1], q[i2]))
            corners = []
            for c in (i0, i1, i2):
                nb = [int(B[c][k] * 24) for k in range(3)]
                assert all(Fraction(nb[k], 24) == B[c][k] for k in range(3))
                corners.append([((nb[0] * uv[0, a] + nb[1] * uv[1, a]) + nb[2] * uv[2, a]) / 24.0
                                for a in range(2)])
            out_uv.append(corners)
    rowptr = [0]
    cols, w = [], []
    for row in M:
        for i in sorted(row):
            cols.append(i)
            w.append(float(row[i]))      # Fraction -> nearest double
        rowptr.append(len(cols))
    # nearest double, then nearest float: both sides use this same rounding
    w32 = np.asarray(w, np.float64).astype(np.float32)
    return {"tri": np.asarray(out_tri, np.int32), "n_fine": n, "rowptr": np.asarray(rowptr, np.int32),
            "cols": np.asarray(cols, np.int32), "w": w32,
            "corner_uv": np.asarray(out_uv, np.float64).astype(np.float32)}
