// dr_subdiv.cpp -- host-side Catmull-Clark tessellation of a control mesh
// (Sec. 6.3 "Subdivision surfaces"): the fixed sparse map from control
// vertices to the tessellated surface's vertices, the tessellated
// triangles and their face-varying texture coordinates.
//
// Weights are kept as exact rationals through both levels and rounded once,
// num / den in double (both below 2^53, so the quotient is the correctly
// rounded value) and then to float.  Numbering, face order and the
// face-varying UV rule are the ones dr.h documents for dr_subdivide.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <numeric>
#include <vector>

#include "dr.h"

namespace {

struct Rat {
    long long n = 0, d = 1;
};

long long gcd_ll(long long a, long long b) {
    if (a < 0) a = -a;
    while (b) {
        long long t = a % b;
        a = b;
        b = t;
    }
    return a;
}

Rat norm(long long n, long long d) {
    if (d < 0) { n = -n; d = -d; }
    long long g = gcd_ll(n, d);
    if (g == 0) g = 1;
    return Rat{n / g, d / g};
}

Rat add(Rat a, Rat b) {
    long long g = gcd_ll(a.d, b.d);
    long long l = a.d / g * b.d;
    return norm(a.n * (l / a.d) + b.n * (l / b.d), l);
}

Rat mul(Rat a, Rat b) {
    long long g1 = gcd_ll(a.n, b.d), g2 = gcd_ll(b.n, a.d);
    if (g1 == 0) g1 = 1;
    if (g2 == 0) g2 = 1;
    return norm((a.n / g1) * (b.n / g2), (a.d / g2) * (b.d / g1));
}

using Row = std::map<int, Rat>;          // control (or previous-level) index -> weight

void acc(Row& r, int i, Rat w) {
    auto it = r.find(i);
    if (it == r.end()) r.emplace(i, w);
    else it->second = add(it->second, w);
}

void acc_row(Row& r, const Row& src, Rat s) {
    for (auto& kv : src) acc(r, kv.first, mul(kv.second, s));
}

// Barycentric position of a refinement point inside its control triangle,
// as integers over 24 (exact for two levels).
struct Bary {
    int b[3];
};

struct Mesh {
    std::vector<std::vector<int>> faces;
    std::vector<std::vector<Bary>> bary;     // per face corner
    std::vector<int> owner;                  // control triangle of each face
    int n_verts = 0;
};

// One level: returns the refined mesh and M (new vertex -> previous vertices).
bool refine(const Mesh& in, Mesh& out, std::vector<Row>& M) {
    const int n = in.n_verts;
    std::map<std::pair<int, int>, int> edge_id;
    std::vector<std::pair<int, int>> edges;
    std::vector<std::vector<int>> edge_faces;
    for (size_t fi = 0; fi < in.faces.size(); ++fi) {
        const auto& f = in.faces[fi];
        int m = (int)f.size();
        for (int k = 0; k < m; ++k) {
            int a = f[k], b = f[(k + 1) % m];
            auto key = std::make_pair(std::min(a, b), std::max(a, b));
            auto it = edge_id.find(key);
            int e;
            if (it == edge_id.end()) {
                e = (int)edges.size();
                edge_id.emplace(key, e);
                edges.emplace_back(a, b);
                edge_faces.emplace_back();
            } else {
                e = it->second;
            }
            edge_faces[e].push_back((int)fi);
        }
    }
    const int n_e = (int)edges.size(), n_f = (int)in.faces.size();
    const int e0 = n, f0 = n + n_e;
    std::vector<Row> fp(n_f);
    for (int fi = 0; fi < n_f; ++fi) {
        const auto& f = in.faces[fi];
        Rat w = norm(1, (long long)f.size());
        for (int v : f) acc(fp[fi], v, w);
    }
    M.assign((size_t)(n + n_e + n_f), Row());
    const Rat q4 = norm(1, 4);
    for (int e = 0; e < n_e; ++e) {
        if (edge_faces[e].size() != 2) return false;         // not a closed manifold
        Row& r = M[e0 + e];
        acc(r, edges[e].first, q4);
        acc(r, edges[e].second, q4);
        acc_row(r, fp[edge_faces[e][0]], q4);
        acc_row(r, fp[edge_faces[e][1]], q4);
    }
    for (int fi = 0; fi < n_f; ++fi) M[f0 + fi] = fp[fi];
    std::vector<std::vector<int>> vfaces(n);
    std::vector<std::vector<int>> vnbrs(n);
    for (int fi = 0; fi < n_f; ++fi) {
        const auto& f = in.faces[fi];
        int m = (int)f.size();
        for (int k = 0; k < m; ++k) {
            vfaces[f[k]].push_back(fi);
            vnbrs[f[k]].push_back(f[(k + 1) % m]);
            vnbrs[f[k]].push_back(f[(k + m - 1) % m]);
        }
    }
    for (int v = 0; v < n; ++v) {
        auto& nb = vnbrs[v];
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        long long val = (long long)nb.size();
        Row& r = M[v];
        if (val == 0) {
            acc(r, v, norm(1, 1));
            continue;
        }
        Rat inv2 = norm(1, val * val);
        for (int fi : vfaces[v]) acc_row(r, fp[fi], inv2);           // Q / n
        for (int w : nb) {                                          // 2 R / n
            acc(r, v, inv2);
            acc(r, w, inv2);
        }
        acc(r, v, norm(val - 3, val));                              // (n - 3) v / n
    }
    out.faces.clear();
    out.bary.clear();
    out.owner.clear();
    for (int fi = 0; fi < n_f; ++fi) {
        const auto& f = in.faces[fi];
        const auto& B = in.bary[fi];
        int m = (int)f.size();
        Bary cen{{0, 0, 0}};
        for (int j = 0; j < m; ++j)
            for (int c = 0; c < 3; ++c) cen.b[c] += B[j].b[c];
        for (int c = 0; c < 3; ++c) {
            if (cen.b[c] % m) return false;                      // more levels than the UV rule covers
            cen.b[c] /= m;
        }
        for (int k = 0; k < m; ++k) {
            int a = f[k], b = f[(k + 1) % m], p = f[(k + m - 1) % m];
            int eab = e0 + edge_id[std::make_pair(std::min(a, b), std::max(a, b))];
            int epa = e0 + edge_id[std::make_pair(std::min(p, a), std::max(p, a))];
            out.faces.push_back({a, eab, f0 + fi, epa});
            Bary mab, mpa;
            for (int c = 0; c < 3; ++c) {
                int s1 = B[k].b[c] + B[(k + 1) % m].b[c], s2 = B[(k + m - 1) % m].b[c] + B[k].b[c];
                if ((s1 & 1) || (s2 & 1)) return false;
                mab.b[c] = s1 / 2;
                mpa.b[c] = s2 / 2;
            }
            out.bary.push_back({B[k], mab, cen, mpa});
            out.owner.push_back(in.owner[fi]);
        }
    }
    out.n_verts = n + n_e + n_f;
    return true;
}

struct Built {
    std::vector<int> tri;
    std::vector<float> uv;
    std::vector<int> rowptr, cols;
    std::vector<float> w;
    int n_fine = 0;
};

dr_status build(const int32_t* tri, const float* corner_uv, int32_t n_verts, int32_t n_tris, int32_t levels,
                Built& out) {
    if (!tri || n_verts < 3 || n_tris < 1 || levels < 1 || levels > 2) return DR_E_INVALID;
    for (long long i = 0; i < 3ll * n_tris; ++i)
        if (tri[i] < 0 || tri[i] >= n_verts) return DR_E_INVALID;
    Mesh cur;
    cur.n_verts = n_verts;
    for (int t = 0; t < n_tris; ++t) {
        cur.faces.push_back({tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]});
        cur.bary.push_back({Bary{{24, 0, 0}}, Bary{{0, 24, 0}}, Bary{{0, 0, 24}}});
        cur.owner.push_back(t);
    }
    std::vector<Row> S(n_verts);
    for (int i = 0; i < n_verts; ++i) S[i].emplace(i, norm(1, 1));
    for (int l = 0; l < levels; ++l) {
        Mesh nxt;
        std::vector<Row> M;
        if (!refine(cur, nxt, M)) return DR_E_INVALID;
        std::vector<Row> S2(M.size());
        for (size_t j = 0; j < M.size(); ++j)
            for (auto& kv : M[j]) acc_row(S2[j], S[kv.first], kv.second);
        S.swap(S2);
        cur = std::move(nxt);
    }
    out.n_fine = cur.n_verts;
    out.rowptr.assign(1, 0);
    for (auto& row : S) {
        for (auto& kv : row) {
            if (kv.second.n == 0) continue;
            out.cols.push_back(kv.first);
            out.w.push_back((float)((double)kv.second.n / (double)kv.second.d));
        }
        out.rowptr.push_back((int)out.cols.size());
    }
    static const int split[2][3] = {{0, 1, 2}, {0, 2, 3}};
    for (size_t fi = 0; fi < cur.faces.size(); ++fi) {
        const auto& q = cur.faces[fi];
        const float* cu = corner_uv ? corner_uv + 6ll * cur.owner[fi] : nullptr;
        for (int h = 0; h < 2; ++h)
            for (int k = 0; k < 3; ++k) {
                int c = split[h][k];
                out.tri.push_back(q[c]);
                const Bary& b = cur.bary[fi][c];
                for (int a = 0; a < 2; ++a) {
                    float u = 0.0f;
                    if (cu) {
                        double x = ((double)b.b[0] * (double)cu[a] + (double)b.b[1] * (double)cu[2 + a]) +
                                   (double)b.b[2] * (double)cu[4 + a];
                        u = (float)(x / 24.0);
                    }
                    out.uv.push_back(u);
                }
            }
    }
    return DR_OK;
}

}  // namespace

extern "C" dr_status dr_subdivide_sizes(const int32_t* tri, int32_t n_verts, int32_t n_tris, int32_t levels,
                                        int32_t* n_fine_verts, int32_t* n_fine_tris, int64_t* nnz) {
    if (!n_fine_verts || !n_fine_tris || !nnz) return DR_E_INVALID;
    Built b;
    dr_status s = build(tri, nullptr, n_verts, n_tris, levels, b);
    if (s) return s;
    *n_fine_verts = b.n_fine;
    *n_fine_tris = (int32_t)(b.tri.size() / 3);
    *nnz = (int64_t)b.cols.size();
    return DR_OK;
}

extern "C" dr_status dr_subdivide(const int32_t* tri, const float* corner_uv, int32_t n_verts, int32_t n_tris,
                                  int32_t levels, int32_t* fine_tri, float* fine_corner_uv, int32_t* rowptr,
                                  int32_t* cols, float* w) {
    if (!corner_uv || !fine_tri || !fine_corner_uv || !rowptr || !cols || !w) return DR_E_INVALID;
    Built b;
    dr_status s = build(tri, corner_uv, n_verts, n_tris, levels, b);
    if (s) return s;
    std::memcpy(fine_tri, b.tri.data(), b.tri.size() * sizeof(int32_t));
    std::memcpy(fine_corner_uv, b.uv.data(), b.uv.size() * sizeof(float));
    std::memcpy(rowptr, b.rowptr.data(), b.rowptr.size() * sizeof(int32_t));
    std::memcpy(cols, b.cols.data(), b.cols.size() * sizeof(int32_t));
    std::memcpy(w, b.w.data(), b.w.size() * sizeof(float));
    return DR_OK;
}
