/* oracle.c -- CPU oracle of the per-pixel stochastic gradient estimator.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded restatement of
 * the method, used to check the GPU library.  Nothing in the product path
 * may load it.  It shares no code with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared.
 *
 * Precision.  The paper does not state one; the render/loss path runs in
 * fp32, the precision of the kernels it checks, because floating point
 * decides integers here (the visible triangle, the fixed-point code of
 * each loss difference).  Every fp32 expression is written with explicit
 * parenthesisation and is evaluated without contraction.  The unquantised
 * gradient accumulator and the decode are fp64.
 *
 * Where the paper is silent (the random hash, camera, fill rule, depth
 * interpolation, texture filter, shading formulas, accumulator format,
 * averaging) the readings below are this project's; each is marked
 * "reading".
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define BG_ID 0xFFFFFFFFu

/* ------------------------------------------------------------------ */
/* Random signs (Alg. 1 "randomsign"; reading: Philox4x64-10)           */
/* ------------------------------------------------------------------ */

/* Philox4x64 round constants, from Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11). */
static const uint64_t PH_M0 = 0xD2E7470EE14C6C93ull;
static const uint64_t PH_M1 = 0xCA5A826395121157ull;
static const uint64_t PH_W0 = 0x9E3779B97F4A7C15ull;
static const uint64_t PH_W1 = 0xBB67AE8584CAA73Bull;

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PH_W0; k1 += PH_W1; }
        unsigned __int128 p0 = (unsigned __int128)PH_M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)PH_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Reading: counter = (i div 256, pair, step, scene), key = (seed, 0); the
 * 256 output bits of a block give the signs of 256 consecutive parameters,
 * bit (i mod 256) of the output words in order; a set bit means -1.  Each
 * sign is +1 or -1 with probability 1/2 (Sec. 3, Eq. 4). */
void or_signs(uint64_t seed, uint32_t step, uint32_t pair, uint32_t scene, int64_t d, int8_t* s) {
    uint64_t key[2] = {seed, 0};
    for (int64_t base = 0; base < d; base += 256) {
        uint64_t ctr[4] = {(uint64_t)(base >> 8), pair, step, scene};
        uint64_t r[4];
        or_philox4x64_10(ctr, key, r);
        for (int j = 0; j < 256 && base + j < d; ++j) {
            uint64_t bit = (r[j >> 6] >> (j & 63)) & 1u;
            s[base + j] = bit ? (int8_t)-1 : (int8_t)1;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Parameter layout (Sec. 4.1: theta = geometry then textures)          */
/* ------------------------------------------------------------------ */

/* Position groups: the control vertices of a subdivision surface, else
 * the mesh's vertices. */
static int64_t n_pos(const or_scene* sc) { return sc->n_ctrl > 0 ? sc->n_ctrl : sc->n_verts; }

int64_t or_param_count(const or_scene* sc) {
    int64_t d = 3 * n_pos(sc);
    for (int t = 0; t < sc->n_tex; ++t)
        d += (int64_t)sc->tex_w[t] * sc->tex_h[t] * sc->tex_c[t];
    return d;
}

static int64_t tex_offset(const or_scene* sc, int t) {
    int64_t off = 3 * n_pos(sc);
    for (int k = 0; k < t; ++k) off += (int64_t)sc->tex_w[k] * sc->tex_h[k] * sc->tex_c[k];
    return off;
}

/* Reading: textures of equal resolution share one set of texel groups,
 * because a sample reads the same texel coordinates in all of them.
 * Classes are numbered in order of first appearance. */
typedef struct {
    int n;                       /* number of classes                    */
    int of_tex[OR_MAX_TEX];      /* class of each texture                */
    int first[OR_MAX_TEX];       /* first texture of each class          */
    int64_t offset[OR_MAX_TEX];  /* first group index of each class      */
} classes_t;

static classes_t texel_classes(const or_scene* sc) {
    classes_t c;
    memset(&c, 0, sizeof(c));
    int64_t off = n_pos(sc);
    for (int t = 0; t < sc->n_tex; ++t) {
        int found = -1;
        for (int j = 0; j < t; ++j)
            if (sc->tex_w[j] == sc->tex_w[t] && sc->tex_h[j] == sc->tex_h[t]) { found = c.of_tex[j]; break; }
        if (found >= 0) {
            c.of_tex[t] = found;
        } else {
            c.of_tex[t] = c.n;
            c.first[c.n] = t;
            c.offset[c.n] = off;
            off += (int64_t)sc->tex_w[t] * sc->tex_h[t];
            c.n++;
        }
    }
    return c;
}

int64_t or_group_count(const or_scene* sc) {
    classes_t c = texel_classes(sc);
    int64_t g = n_pos(sc);
    for (int k = 0; k < c.n; ++k) g += (int64_t)sc->tex_w[c.first[k]] * sc->tex_h[c.first[k]];
    return g;
}

/* Block of parameter i: 0 = positions, 1 + t = texture t. */
static int block_of(const or_scene* sc, int64_t i) {
    int64_t off = 3 * n_pos(sc);
    if (i < off) return 0;
    for (int t = 0; t < sc->n_tex; ++t) {
        off += (int64_t)sc->tex_w[t] * sc->tex_h[t] * sc->tex_c[t];
        if (i < off) return 1 + t;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Perturbation (Alg. 1): theta +- s (.) eps, one fp32 add per entry    */
/* ------------------------------------------------------------------ */

static float* perturbed_copy(const or_scene* sc, const float* theta, const int8_t* s, int sign,
                             const float* eps) {
    int64_t d = or_param_count(sc);
    float* p = (float*)malloc(sizeof(float) * (size_t)(d > 0 ? d : 1));
    if (!p) return NULL;
    for (int64_t i = 0; i < d; ++i) {
        float e = eps ? eps[block_of(sc, i)] : 0.0f;
        if (s == NULL || s[i] == 0 || e == 0.0f) {
            p[i] = theta[i];
        } else {
            float se = (s[i] > 0) ? e : -e;           /* s_i eps_i, exact          */
            p[i] = (sign > 0) ? (theta[i] + se) : (theta[i] - se);
        }
    }
    return p;
}

/* ------------------------------------------------------------------ */
/* Rasterizer R (Sec. 4.3-4.4): colour + ID buffer + UV buffer          */
/* ------------------------------------------------------------------ */

typedef struct {
    int valid;
    int32_t X, Y;      /* snapped screen position, 1/256 pixel units     */
    float z;           /* depth in [0,1] (NDC z mapped)                  */
    float iw;          /* 1 / clip w                                     */
} vtx_t;

/* Reading: clip = M [x y z 1]^T summed left to right; NDC by division;
 * pixel (0,0) at the top-left; snap to 1/256 pixel by round-half-even;
 * vertices behind the near plane or beyond +-2^22 subpixels are invalid
 * and cull their triangles (no clipping). */
static vtx_t transform_vertex(const or_view* vw, const float* p) {
    const float* M = vw->view_proj;
    float x = p[0], y = p[1], z = p[2];
    float cx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
    float cy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
    float cz = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
    float cw = ((M[12] * x + M[13] * y) + M[14] * z) + M[15];
    vtx_t v;
    memset(&v, 0, sizeof(v));
    if (!(cw >= vw->near_w)) return v;
    float nx = cx / cw, ny = cy / cw, nz = cz / cw;
    float sx = (nx * 0.5f + 0.5f) * (float)vw->width;
    float sy = (0.5f - ny * 0.5f) * (float)vw->height;
    float fx = sx * 256.0f, fy = sy * 256.0f;
    if (!(fabsf(fx) <= 4194304.0f) || !(fabsf(fy) <= 4194304.0f)) return v;
    v.valid = 1;
    v.X = (int32_t)rintf(fx);
    v.Y = (int32_t)rintf(fy);
    v.z = nz * 0.5f + 0.5f;
    v.iw = 1.0f / cw;
    return v;
}

typedef struct {
    int ok;
    int order[3];          /* normalised corner order -> original corner   */
    int32_t X[3], Y[3];
    float z[3], iw[3];
    int64_t area2;         /* twice the signed area, > 0 after normalising */
    int topleft[3];        /* edge k (opposite vertex k) is top or left     */
    float z0, zx, zy;      /* depth plane                                   */
    float ia;              /* 1 / area2, formed once per triangle           */
} tri_setup_t;

/* Reading: triangles are made counter-clockwise in the y-down pixel frame
 * by swapping corners 1 and 2 when the signed area is negative; zero area
 * culls.  There is no back-face culling: depth alone decides. */
static tri_setup_t setup_triangle(const vtx_t* vt, const int32_t* tri, int32_t t) {
    tri_setup_t s;
    memset(&s, 0, sizeof(s));
    const vtx_t* a = &vt[tri[3 * t + 0]];
    const vtx_t* b = &vt[tri[3 * t + 1]];
    const vtx_t* c = &vt[tri[3 * t + 2]];
    if (!a->valid || !b->valid || !c->valid) return s;
    int64_t area2 = (int64_t)(b->X - a->X) * (int64_t)(c->Y - a->Y)
                  - (int64_t)(b->Y - a->Y) * (int64_t)(c->X - a->X);
    if (area2 == 0) return s;
    int o1 = 1, o2 = 2;
    if (area2 < 0) { o1 = 2; o2 = 1; area2 = -area2; }
    s.order[0] = 0; s.order[1] = o1; s.order[2] = o2;
    const vtx_t* v[3] = {a, (o1 == 1) ? b : c, (o1 == 1) ? c : b};
    for (int k = 0; k < 3; ++k) {
        s.X[k] = v[k]->X; s.Y[k] = v[k]->Y; s.z[k] = v[k]->z; s.iw[k] = v[k]->iw;
    }
    s.area2 = area2;
    /* Edge k runs from vertex k+1 to vertex k+2.  With y pointing down and
     * positive area, a top edge is horizontal going right and a left edge
     * goes up (Direct3D-style top-left rule). */
    for (int k = 0; k < 3; ++k) {
        int ia = (k + 1) % 3, ib = (k + 2) % 3;
        int32_t dx = s.X[ib] - s.X[ia], dy = s.Y[ib] - s.Y[ia];
        s.topleft[k] = (dy < 0) || (dy == 0 && dx > 0);
    }
    /* Reading: depth is the plane through the three snapped vertices,
     * evaluated at the sample from vertex 0. */
    float d1 = s.z[1] - s.z[0], d2 = s.z[2] - s.z[0];
    float fX1 = (float)(s.X[1] - s.X[0]), fY1 = (float)(s.Y[1] - s.Y[0]);
    float fX2 = (float)(s.X[2] - s.X[0]), fY2 = (float)(s.Y[2] - s.Y[0]);
    float fa = (float)area2;
    s.z0 = s.z[0];
    s.zx = (d1 * fY2 - d2 * fY1) / fa;
    s.zy = (d2 * fX1 - d1 * fX2) / fa;
    s.ia = 1.0f / fa;
    s.ok = 1;
    return s;
}

/* Edge function of edge (a -> b) at sample (px, py), exact in int64. */
static int64_t edge_fn(int32_t xa, int32_t ya, int32_t xb, int32_t yb, int32_t px, int32_t py) {
    return (int64_t)(xb - xa) * (int64_t)(py - ya) - (int64_t)(yb - ya) * (int64_t)(px - xa);
}

static void edges_at(const tri_setup_t* s, int32_t px, int32_t py, int64_t E[3]) {
    for (int k = 0; k < 3; ++k) {
        int ia = (k + 1) % 3, ib = (k + 2) % 3;
        E[k] = edge_fn(s->X[ia], s->Y[ia], s->X[ib], s->Y[ib], px, py);
    }
}

static int covers(const tri_setup_t* s, const int64_t E[3]) {
    for (int k = 0; k < 3; ++k)
        if (!(E[k] > 0 || (E[k] == 0 && s->topleft[k]))) return 0;
    return 1;
}

static float depth_at(const tri_setup_t* s, int32_t px, int32_t py) {
    float z = (s->z0 + s->zx * (float)(px - s->X[0])) + s->zy * (float)(py - s->Y[0]);
    if (!(z > 0.0f)) z = 0.0f;
    return z;
}

static uint32_t f2u(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Visibility: for every pixel centre, the covering triangle of least
 * (depth, triangle index) -- an exact z-buffer with ties broken towards
 * the lower index.  Written as one pass over triangles and their bounding
 * boxes, keeping the per-pixel minimum of the packed key depth<<32 | id. */
static void rasterize_ids(const or_scene* sc, const tri_setup_t* ts, int W, int H, uint32_t* id) {
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)W * H);
    for (int64_t p = 0; p < (int64_t)W * H; ++p) key[p] = ~0ull;
    for (int32_t t = 0; t < sc->n_tris; ++t) {
        const tri_setup_t* s = &ts[t];
        if (!s->ok) continue;
        int32_t xmin = s->X[0], xmax = s->X[0], ymin = s->Y[0], ymax = s->Y[0];
        for (int k = 1; k < 3; ++k) {
            if (s->X[k] < xmin) xmin = s->X[k];
            if (s->X[k] > xmax) xmax = s->X[k];
            if (s->Y[k] < ymin) ymin = s->Y[k];
            if (s->Y[k] > ymax) ymax = s->Y[k];
        }
        int x0 = (xmin >> 8) - 1, x1 = (xmax >> 8) + 1, y0 = (ymin >> 8) - 1, y1 = (ymax >> 8) + 1;
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (x1 > W - 1) x1 = W - 1;
        if (y1 > H - 1) y1 = H - 1;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                int32_t px = 256 * x + 128, py = 256 * y + 128;
                int64_t E[3];
                edges_at(s, px, py, E);
                if (!covers(s, E)) continue;
                uint64_t k = ((uint64_t)f2u(depth_at(s, px, py)) << 32) | (uint32_t)t;
                if (k < key[(int64_t)y * W + x]) key[(int64_t)y * W + x] = k;
            }
    }
    for (int64_t p = 0; p < (int64_t)W * H; ++p)
        id[p] = (key[p] == ~0ull) ? BG_ID : (uint32_t)(key[p] & 0xFFFFFFFFu);
    free(key);
}

/* Visibility of semi-transparent geometry (Sec. 4.4 "Transparent
 * geometry": front-to-back rendering after a sort, with a deep ID buffer):
 * for every pixel centre, the L covering triangles of least (depth,
 * triangle index), in increasing order -- the exact per-pixel front-to-back
 * order, kept by insertion into a sorted list of L packed keys. */
static void rasterize_deep(const or_scene* sc, const tri_setup_t* ts, int W, int H, int L, uint32_t* id) {
    int64_t n = (int64_t)W * H * L;
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < n; ++p) key[p] = ~0ull;
    for (int32_t t = 0; t < sc->n_tris; ++t) {
        const tri_setup_t* s = &ts[t];
        if (!s->ok) continue;
        int32_t xmin = s->X[0], xmax = s->X[0], ymin = s->Y[0], ymax = s->Y[0];
        for (int k = 1; k < 3; ++k) {
            if (s->X[k] < xmin) xmin = s->X[k];
            if (s->X[k] > xmax) xmax = s->X[k];
            if (s->Y[k] < ymin) ymin = s->Y[k];
            if (s->Y[k] > ymax) ymax = s->Y[k];
        }
        int x0 = (xmin >> 8) - 1, x1 = (xmax >> 8) + 1, y0 = (ymin >> 8) - 1, y1 = (ymax >> 8) + 1;
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (x1 > W - 1) x1 = W - 1;
        if (y1 > H - 1) y1 = H - 1;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                int32_t px = 256 * x + 128, py = 256 * y + 128;
                int64_t E[3];
                edges_at(s, px, py, E);
                if (!covers(s, E)) continue;
                uint64_t k = ((uint64_t)f2u(depth_at(s, px, py)) << 32) | (uint32_t)t;
                uint64_t* list = key + ((int64_t)y * W + x) * L;
                if (k >= list[L - 1]) continue;
                int j = L - 1;
                while (j > 0 && list[j - 1] > k) {
                    list[j] = list[j - 1];
                    --j;
                }
                list[j] = k;
            }
    }
    for (int64_t p = 0; p < n; ++p) id[p] = (key[p] == ~0ull) ? BG_ID : (uint32_t)(key[p] & 0xFFFFFFFFu);
    free(key);
}

/* ------------------------------------------------------------------ */
/* Attributes and shading at a pixel (Sec. 4.4 "Textures")              */
/* ------------------------------------------------------------------ */

typedef struct {
    float b[3];        /* screen-space barycentrics, normalised order     */
    float pc[3];       /* b_k / w_k                                       */
    float S;           /* sum of pc                                       */
    float iS;          /* 1 / S                                           */
    float u, v;        /* perspective-correct texture coordinates         */
} attr_t;

/* Reading: b_k = E_k * (1 / area2) in fp32, the reciprocal formed once per
 * triangle; perspective-correct interpolation multiplies the 1/w-weighted
 * sums by the reciprocal of their total; sums run over the normalised
 * corner order. */
static attr_t attributes(const or_scene* sc, const tri_setup_t* s, int32_t t, int32_t px, int32_t py) {
    attr_t a;
    int64_t E[3];
    edges_at(s, px, py, E);
    for (int k = 0; k < 3; ++k) a.b[k] = (float)E[k] * s->ia;
    for (int k = 0; k < 3; ++k) a.pc[k] = a.b[k] * s->iw[k];
    a.S = (a.pc[0] + a.pc[1]) + a.pc[2];
    a.iS = 1.0f / a.S;
    const float* cuv = sc->corner_uv + 6 * (int64_t)t;
    float u0 = cuv[2 * s->order[0]], u1 = cuv[2 * s->order[1]], u2 = cuv[2 * s->order[2]];
    float v0 = cuv[2 * s->order[0] + 1], v1 = cuv[2 * s->order[1] + 1], v2 = cuv[2 * s->order[2] + 1];
    a.u = ((a.pc[0] * u0 + a.pc[1] * u1) + a.pc[2] * u2) * a.iS;
    a.v = ((a.pc[0] * v0 + a.pc[1] * v1) + a.pc[2] * v2) * a.iS;
    return a;
}

typedef struct {
    int xa, xb, ya, yb;    /* the 2x2 footprint (wrap in u, clamp in v)   */
    float fx, fy;
} fp_t;

/* Reading: bilinear filter with texel centres at half-integers; u wraps
 * (repeat), v clamps to the edge. */
static fp_t footprint(float u, float v, int W, int H) {
    fp_t f;
    float x = u * (float)W - 0.5f;
    float y = v * (float)H - 0.5f;
    if (!(fabsf(x) < 16777216.0f)) x = 0.0f;
    if (!(fabsf(y) < 16777216.0f)) y = 0.0f;
    float x0f = floorf(x), y0f = floorf(y);
    f.fx = x - x0f;
    f.fy = y - y0f;
    int x0 = (int)x0f, y0 = (int)y0f;
    f.xa = ((x0 % W) + W) % W;
    f.xb = (((x0 + 1) % W) + W) % W;
    f.ya = y0 < 0 ? 0 : (y0 > H - 1 ? H - 1 : y0);
    f.yb = (y0 + 1) < 0 ? 0 : ((y0 + 1) > H - 1 ? H - 1 : (y0 + 1));
    return f;
}

static void sample_tex(const or_scene* sc, const float* th, int t, float u, float v, float* out) {
    int W = sc->tex_w[t], H = sc->tex_h[t], C = sc->tex_c[t];
    const float* tx = th + tex_offset(sc, t);
    fp_t f = footprint(u, v, W, H);
    float w00 = (1.0f - f.fx) * (1.0f - f.fy);
    float w10 = f.fx * (1.0f - f.fy);
    float w01 = (1.0f - f.fx) * f.fy;
    float w11 = f.fx * f.fy;
    for (int c = 0; c < C; ++c) {
        float t00 = tx[((int64_t)f.ya * W + f.xa) * C + c];
        float t10 = tx[((int64_t)f.ya * W + f.xb) * C + c];
        float t01 = tx[((int64_t)f.yb * W + f.xa) * C + c];
        float t11 = tx[((int64_t)f.yb * W + f.xb) * C + c];
        out[c] = ((w00 * t00 + w10 * t10) + w01 * t01) + w11 * t11;
    }
}

static void normalize3(float* x) {
    float l2 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
    if (l2 > 0.0f) {
        float inv = 1.0f / sqrtf(l2);
        x[0] = x[0] * inv; x[1] = x[1] * inv; x[2] = x[2] * inv;
    } else {
        x[0] = 0.0f; x[1] = 0.0f; x[2] = 0.0f;
    }
}

static float dot3(const float* a, const float* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

static void cross3(const float* a, const float* b, float* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

#define OR_PI 3.14159265f
#define OR_INV_PI 0.318309886f

/* Shade pixel (px,py) covered by triangle t of the (perturbed) scene th.
 * Readings: unlit = albedo; Lambert = albedo (ambient + diffuse max(0,n.l))
 * light with the face normal; GGX = Cook-Torrance with GGX distribution,
 * Smith-Schlick geometry (k = alpha/2), Schlick Fresnel (F0 = 0.04) and a
 * tangent-space normal map in the face's UV frame.  The colour depends only
 * on the triangle's three vertices and on the texels of its footprint. */
static void shade(const or_scene* sc, const or_view* vw, const float* th, const float* pos, const tri_setup_t* s,
                  int32_t t, int32_t px, int32_t py, float* rgb, float* uv_out, float* alpha_out) {
    attr_t a = attributes(sc, s, t, px, py);
    uv_out[0] = a.u;
    uv_out[1] = a.v;
    float alb[4] = {0.0f, 0.0f, 0.0f, 1.0f};
    if (sc->n_tex > 0) sample_tex(sc, th, 0, a.u, a.v, alb);
    /* Reading: the opacity of a semi-transparent surface is the albedo's
     * fourth channel, clamped to [0, 1]. */
    float al = alb[3];
    if (!(al > 0.0f)) al = 0.0f;
    if (al > 1.0f) al = 1.0f;
    *alpha_out = al;
    if (sc->shading == 0) {
        rgb[0] = alb[0]; rgb[1] = alb[1]; rgb[2] = alb[2];
        return;
    }
    const int32_t* ti = sc->tri + 3 * (int64_t)t;
    float p[3][3];
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 3; ++c) p[k][c] = pos[3 * (int64_t)ti[k] + c];
    float e1[3], e2[3], nf[3];
    for (int c = 0; c < 3; ++c) { e1[c] = p[1][c] - p[0][c]; e2[c] = p[2][c] - p[0][c]; }
    cross3(e1, e2, nf);
    normalize3(nf);
    if (sc->shading == 1) {
        float ndl = dot3(nf, sc->light_dir);
        if (!(ndl > 0.0f)) ndl = 0.0f;
        float sh = sc->ambient + sc->diffuse * ndl;
        for (int c = 0; c < 3; ++c) rgb[c] = alb[c] * (sh * sc->light_rgb[c]);
        return;
    }
    /* GGX */
    const float* cuv = sc->corner_uv + 6 * (int64_t)t;
    float du1 = cuv[2] - cuv[0], dv1 = cuv[3] - cuv[1];
    float du2 = cuv[4] - cuv[0], dv2 = cuv[5] - cuv[1];
    float r = du1 * dv2 - du2 * dv1;
    float T[3], B[3];
    for (int c = 0; c < 3; ++c) T[c] = e1[c] * dv2 - e2[c] * dv1;
    if (r < 0.0f) { T[0] = -T[0]; T[1] = -T[1]; T[2] = -T[2]; }
    float nt = dot3(nf, T);
    for (int c = 0; c < 3; ++c) T[c] = T[c] - nf[c] * nt;
    normalize3(T);
    cross3(nf, T, B);
    float nm[3] = {0.5f, 0.5f, 1.0f};
    if (sc->n_tex > 1) sample_tex(sc, th, 1, a.u, a.v, nm);
    float tn[3];
    for (int c = 0; c < 3; ++c) tn[c] = 2.0f * nm[c] - 1.0f;
    float n[3];
    for (int c = 0; c < 3; ++c) n[c] = (T[c] * tn[0] + B[c] * tn[1]) + nf[c] * tn[2];
    normalize3(n);
    float rough = 0.5f;
    if (sc->n_tex > 2) sample_tex(sc, th, 2, a.u, a.v, &rough);
    float P[3];
    for (int c = 0; c < 3; ++c) {
        float q0 = p[s->order[0]][c], q1 = p[s->order[1]][c], q2 = p[s->order[2]][c];
        P[c] = ((a.pc[0] * q0 + a.pc[1] * q1) + a.pc[2] * q2) * a.iS;
    }
    float V[3] = {vw->cam_pos[0] - P[0], vw->cam_pos[1] - P[1], vw->cam_pos[2] - P[2]};
    normalize3(V);
    const float* L = sc->light_dir;
    float Hh[3] = {L[0] + V[0], L[1] + V[1], L[2] + V[2]};
    normalize3(Hh);
    float ndl = dot3(n, L), ndv = dot3(n, V), ndh = dot3(n, Hh), vdh = dot3(V, Hh);
    if (!(ndl > 0.0f)) ndl = 0.0f;
    if (!(ndv > 0.0f)) ndv = 0.0f;
    if (!(ndh > 0.0f)) ndh = 0.0f;
    if (!(vdh > 0.0f)) vdh = 0.0f;
    float alpha = rough * rough;
    if (!(alpha > 0.002f)) alpha = 0.002f;
    float a2 = alpha * alpha;
    /* D G F / (4 n.l n.v) with D = a2 / (pi dd^2) and the Smith-Schlick
     * G = n.l / gl * n.v / gv: the factors n.l n.v cancel, leaving one
     * division, a2 F / (4 pi dd^2 gl gv). */
    float dd = (ndh * ndh) * (a2 - 1.0f) + 1.0f;
    float k = alpha * 0.5f;
    float gl = ndl * (1.0f - k) + k;
    float gv = ndv * (1.0f - k) + k;
    float om = 1.0f - vdh;
    float om5 = ((om * om) * (om * om)) * om;
    float F = 0.04f + 0.96f * om5;
    float spec = 0.0f;
    if (ndl > 0.0f && ndv > 0.0f) spec = (a2 * F) / ((((4.0f * OR_PI) * dd) * dd) * (gl * gv));
    for (int c = 0; c < 3; ++c)
        rgb[c] = ((alb[c] * OR_INV_PI + spec) * sc->light_rgb[c]) * ndl + sc->ambient * alb[c];
}

typedef struct {
    int W, H;
    float* th;             /* perturbed parameters                         */
    float* pos;            /* mesh vertex positions [n_verts, 3]           */
    vtx_t* vt;
    tri_setup_t* ts;
} frame_t;

/* Vertex positions of the tessellated surface from the (perturbed) control
 * vertices: per vertex and coordinate, the weighted terms of its row added
 * in row order to a zero start, each weight times coordinate an fp32
 * product. */
static void subdivide_positions(const or_scene* sc, const float* ctrl, float* pos) {
    for (int32_t j = 0; j < sc->n_verts; ++j)
        for (int c = 0; c < 3; ++c) {
            float acc = 0.0f;
            for (int32_t k = sc->sub_rowptr[j]; k < sc->sub_rowptr[j + 1]; ++k)
                acc = acc + sc->sub_w[k] * ctrl[3 * (int64_t)sc->sub_cols[k] + c];
            pos[3 * (int64_t)j + c] = acc;
        }
}

static int build_frame(frame_t* fr, const or_scene* sc, const float* theta, const int8_t* s, int sign,
                       const float* eps, const or_view* vw) {
    fr->W = vw->width;
    fr->H = vw->height;
    fr->th = perturbed_copy(sc, theta, s, sign, eps);
    fr->pos = fr->th;
    if (sc->n_ctrl > 0) {
        fr->pos = (float*)malloc(sizeof(float) * 3 * (size_t)(sc->n_verts > 0 ? sc->n_verts : 1));
        if (!fr->pos || !fr->th) return -1;
        subdivide_positions(sc, fr->th, fr->pos);
    }
    fr->vt = (vtx_t*)malloc(sizeof(vtx_t) * (size_t)(sc->n_verts > 0 ? sc->n_verts : 1));
    fr->ts = (tri_setup_t*)malloc(sizeof(tri_setup_t) * (size_t)(sc->n_tris > 0 ? sc->n_tris : 1));
    if (!fr->th || !fr->vt || !fr->ts) return -1;
    for (int32_t j = 0; j < sc->n_verts; ++j) fr->vt[j] = transform_vertex(vw, fr->pos + 3 * (int64_t)j);
    for (int32_t t = 0; t < sc->n_tris; ++t) fr->ts[t] = setup_triangle(fr->vt, sc->tri, t);
    return 0;
}

static void free_frame(frame_t* fr) {
    if (fr->pos != fr->th) free(fr->pos);
    free(fr->th);
    free(fr->vt);
    free(fr->ts);
}

static int n_layers(const or_scene* sc) { return sc->layers > 0 ? sc->layers : 1; }

/* id [H,W,L], uv [H,W,L,2].  Opaque: the visible triangle's colour.
 * Semi-transparent (reading): the listed fragments composited front to
 * back over a black background, C = sum_k T_k alpha_k c_k with T_0 = 1 and
 * T_{k+1} = T_k (1 - alpha_k), accumulated in list order. */
static int render_frame(const or_scene* sc, const or_view* vw, frame_t* fr, float* rgb, uint32_t* id,
                        float* uv) {
    int W = fr->W, H = fr->H, L = n_layers(sc);
    if (sc->layers > 0) rasterize_deep(sc, fr->ts, W, H, L, id);
    else rasterize_ids(sc, fr->ts, W, H, id);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t p = (int64_t)y * W + x;
            float out[3] = {0.0f, 0.0f, 0.0f}, T = 1.0f;
            for (int l = 0; l < L; ++l) {
                int64_t e = p * L + l;
                float c[3] = {0.0f, 0.0f, 0.0f}, w[2] = {0.0f, 0.0f}, al = 1.0f;
                if (id[e] != BG_ID)
                    shade(sc, vw, fr->th, fr->pos, &fr->ts[id[e]], (int32_t)id[e], 256 * x + 128, 256 * y + 128, c, w,
                          &al);
                uv[2 * e + 0] = w[0]; uv[2 * e + 1] = w[1];
                if (sc->layers == 0) {
                    out[0] = c[0]; out[1] = c[1]; out[2] = c[2];
                } else if (id[e] != BG_ID) {
                    float wt = T * al;
                    for (int ch = 0; ch < 3; ++ch) out[ch] = out[ch] + wt * c[ch];
                    T = T * (1.0f - al);
                }
            }
            rgb[3 * p + 0] = out[0]; rgb[3 * p + 1] = out[1]; rgb[3 * p + 2] = out[2];
        }
    return 0;
}

int or_render(const or_scene* sc, const float* theta, const int8_t* s, int sign, const float* eps,
              const or_view* view, float* rgb, uint32_t* id, float* uv) {
    int64_t np = (int64_t)view->width * view->height;
    int64_t ne = np * n_layers(sc);
    frame_t fr;
    if (build_frame(&fr, sc, theta, s, sign, eps, view)) return -1;
    float* c = (float*)malloc(sizeof(float) * 3 * (size_t)np);
    uint32_t* i = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)ne);
    float* w = (float*)malloc(sizeof(float) * 2 * (size_t)ne);
    render_frame(sc, view, &fr, c, i, w);
    if (rgb) memcpy(rgb, c, sizeof(float) * 3 * (size_t)np);
    if (id) memcpy(id, i, sizeof(uint32_t) * (size_t)ne);
    if (uv) memcpy(uv, w, sizeof(float) * 2 * (size_t)ne);
    free(c); free(i); free(w);
    free_frame(&fr);
    return 0;
}

/* f_{w,h} = || I_{w,h}(theta) - I_{w,h} ||^2 (Table 1), channels r, g, b in order. */
static float pixel_l2(const float* c, const float* t) {
    float dr = c[0] - t[0], dg = c[1] - t[1], db = c[2] - t[2];
    return (dr * dr + dg * dg) + db * db;
}

int or_pixel_loss(const or_scene* sc, const float* theta, const int8_t* s, int sign, const float* eps,
                  const or_view* view, const float* target, float* f) {
    int64_t np = (int64_t)view->width * view->height;
    float* rgb = (float*)malloc(sizeof(float) * 3 * (size_t)np);
    if (or_render(sc, theta, s, sign, eps, view, rgb, NULL, NULL)) return -1;
    for (int64_t p = 0; p < np; ++p) f[p] = pixel_l2(rgb + 3 * p, target + 3 * p);
    free(rgb);
    return 0;
}

/* Reading: the accumulator is int64 fixed point with 32 fraction bits, so
 * sums do not depend on the order of the additions. */
int64_t or_quantize(float delta, or_stats* st) {
    if (isnan(delta)) {
        if (st) st->nonfinite++;
        return 0;
    }
    if (fabsf(delta) > 32.0f) {
        if (st) st->saturations++;
        return delta > 0.0f ? ((int64_t)1 << 37) : -((int64_t)1 << 37);
    }
    return (int64_t)nearbyint((double)delta * 4294967296.0);
}

/* ------------------------------------------------------------------ */
/* Contribution set of a pixel (Sec. 4.4; reading: union over the two   */
/* perturbed renders -- and over the layers of a deep ID buffer -- each */
/* group once)                                                          */
/* ------------------------------------------------------------------ */

#define MAX_SET 1024

typedef struct {
    int n;
    int64_t g[MAX_SET];
} gset_t;

static void set_add(gset_t* s, int64_t g) {
    for (int i = 0; i < s->n; ++i)
        if (s->g[i] == g) return;
    if (s->n == MAX_SET) abort();        /* a contribution set this large is a bug */
    s->g[s->n++] = g;
}

static int class_active(const or_scene* sc, const classes_t* c, const float* eps, int cls) {
    for (int t = 0; t < sc->n_tex; ++t)
        if (c->of_tex[t] == cls && eps[1 + t] != 0.0f) return 1;
    return 0;
}

/* Groups one render contributes at a pixel: the visible triangle's three
 * vertices (ID buffer) and, per texel class, the texels its sample read
 * (UV buffer): the bilinear footprint, or the nearest texel. */
static void groups_of(const or_scene* sc, const float* eps, uint32_t id, const float* uv, gset_t* out) {
    if (id == BG_ID) return;
    if (eps[0] != 0.0f)
        for (int k = 0; k < 3; ++k) {
            int32_t v = sc->tri[3 * (int64_t)id + k];
            if (sc->n_ctrl > 0) {
                /* Sec. 6.3: the control vertices the corner combines */
                for (int32_t j = sc->sub_rowptr[v]; j < sc->sub_rowptr[v + 1]; ++j) set_add(out, sc->sub_cols[j]);
            } else {
                set_add(out, v);
            }
        }
    classes_t c = texel_classes(sc);
    for (int cls = 0; cls < c.n; ++cls) {
        if (!class_active(sc, &c, eps, cls)) continue;
        int t = c.first[cls];
        int W = sc->tex_w[t], H = sc->tex_h[t];
        int64_t base = c.offset[cls];
        fp_t f = footprint(uv[0], uv[1], W, H);
        if (sc->tex_mode == 1) {
            int xn = (f.fx >= 0.5f) ? f.xb : f.xa;
            int yn = (f.fy >= 0.5f) ? f.yb : f.ya;
            set_add(out, base + (int64_t)yn * W + xn);
        } else {
            set_add(out, base + (int64_t)f.ya * W + f.xa);
            set_add(out, base + (int64_t)f.ya * W + f.xb);
            set_add(out, base + (int64_t)f.yb * W + f.xa);
            set_add(out, base + (int64_t)f.yb * W + f.xb);
        }
    }
}

/* Parameters of a group: a vertex's x, y, z, or one texel's channels in
 * every texture of the class. */
static int params_of(const or_scene* sc, int64_t g, int64_t* out) {
    int n = 0;
    if (g < n_pos(sc)) {
        for (int c = 0; c < 3; ++c) out[n++] = 3 * g + c;
        return n;
    }
    classes_t c = texel_classes(sc);
    for (int cls = 0; cls < c.n; ++cls) {
        int t0 = c.first[cls];
        int64_t size = (int64_t)sc->tex_w[t0] * sc->tex_h[t0];
        if (g >= c.offset[cls] && g < c.offset[cls] + size) {
            int64_t texel = g - c.offset[cls];
            for (int t = 0; t < sc->n_tex; ++t)
                if (c.of_tex[t] == cls)
                    for (int ch = 0; ch < sc->tex_c[t]; ++ch)
                        out[n++] = tex_offset(sc, t) + texel * sc->tex_c[t] + ch;
        }
    }
    return n;
}

/* ------------------------------------------------------------------ */
/* Estimator: Eq. 8 per pixel, accumulated over pairs and views (Eq. 9) */
/* ------------------------------------------------------------------ */

/* The per-pixel difference that Eq. 8 scatters.  Loss form: f+ - f- of
 * the per-pixel L2 error against the target t (Table 1).  Image form: t is
 * the gradient g of a downstream loss with respect to the pixel's colour
 * and the difference is <g, I+ - I->, the change of that loss to first
 * order, so that the estimator approximates the vector-Jacobian product of
 * the render with g. */
static float pixel_delta(const float* ip, const float* im, const float* t, int image_form) {
    if (!image_form) return pixel_l2(ip, t) - pixel_l2(im, t);
    float d0 = ip[0] - im[0], d1 = ip[1] - im[1], d2 = ip[2] - im[2];
    return (t[0] * d0 + t[1] * d1) + t[2] * d2;
}

static int estimate_per_pixel(const or_scene* sc, const float* theta, const or_view* views, int32_t n_views,
                              const float* targets, int image_form, uint64_t seed, uint32_t step,
                              int32_t n_pairs, uint32_t scene_index, const float* eps, const int8_t* signs,
                              int64_t* Q, uint32_t* K, double* G64, or_stats* st) {
    int64_t d = or_param_count(sc);
    int8_t* s = (int8_t*)malloc((size_t)(d > 0 ? d : 1));
    if (!s) return -1;
    int64_t params[3 * 64];
    for (int32_t n = 0; n < n_pairs; ++n) {
        /* P: the sign vector of this pair. */
        if (signs) memcpy(s, signs + (int64_t)n * d, (size_t)d);
        else or_signs(seed, step, (uint32_t)n, scene_index, d, s);
        const float* tgt = targets;
        for (int32_t v = 0; v < n_views; ++v) {
            const or_view* vw = &views[v];
            int64_t np = (int64_t)vw->width * vw->height;
            /* R: render theta + s eps and theta - s eps. */
            float* rgb[2];
            uint32_t* id[2];
            float* uv[2];
            int L = n_layers(sc);
            for (int k = 0; k < 2; ++k) {
                rgb[k] = (float*)malloc(sizeof(float) * 3 * (size_t)np);
                id[k] = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(np * L));
                uv[k] = (float*)malloc(sizeof(float) * 2 * (size_t)(np * L));
                frame_t fr;
                if (build_frame(&fr, sc, theta, s, k == 0 ? +1 : -1, eps, vw)) return -1;
                render_frame(sc, vw, &fr, rgb[k], id[k], uv[k]);
                free_frame(&fr);
            }
            /* G: per pixel, the loss difference goes to the parameters of
             * the groups that contributed to the pixel (Alg. 2). */
            for (int64_t p = 0; p < np; ++p) {
                float delta = pixel_delta(rgb[0] + 3 * p, rgb[1] + 3 * p, tgt + 3 * p, image_form);
                gset_t set;
                set.n = 0;
                for (int k = 0; k < 2; ++k)
                    for (int l = 0; l < L; ++l) groups_of(sc, eps, id[k][p * L + l], uv[k] + 2 * (p * L + l), &set);
                if (set.n == 0) continue;
                int64_t q = or_quantize(delta, st);
                for (int gi = 0; gi < set.n; ++gi) {
                    int64_t g = set.g[gi];
                    K[g] += 1;
                    int np_ = params_of(sc, g, params);
                    for (int j = 0; j < np_; ++j) {
                        int64_t i = params[j];
                        float e = eps[block_of(sc, i)];
                        if (e == 0.0f || s[i] == 0) continue;
                        Q[i] += (int64_t)s[i] * q;
                        if (G64) G64[i] += (double)s[i] * (double)delta / (2.0 * (double)e);
                    }
                }
            }
            for (int k = 0; k < 2; ++k) { free(rgb[k]); free(id[k]); free(uv[k]); }
            tgt += 3 * np;
        }
    }
    free(s);
    return 0;
}

int or_estimate(const or_scene* sc, const float* theta, const or_view* views, int32_t n_views,
                const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                uint32_t scene_index, const float* eps, const int8_t* signs, int64_t* Q, uint32_t* K,
                double* G64, or_stats* st) {
    return estimate_per_pixel(sc, theta, views, n_views, targets, 0, seed, step, n_pairs, scene_index, eps,
                              signs, Q, K, G64, st);
}

int or_estimate_image(const or_scene* sc, const float* theta, const or_view* views, int32_t n_views,
                      const float* grad_image, uint64_t seed, uint32_t step, int32_t n_pairs,
                      uint32_t scene_index, const float* eps, const int8_t* signs, int64_t* Q, uint32_t* K,
                      double* G64, or_stats* st) {
    return estimate_per_pixel(sc, theta, views, n_views, grad_image, 1, seed, step, n_pairs, scene_index, eps,
                              signs, Q, K, G64, st);
}

/* Eq. 4 (the full-image estimator of Sec. 3 and 6.1): every parameter of
 * an active block receives s_i times the quantised difference of the whole
 * image, q = sum over pixels of q_p (fixed point, so the sum is exact); every
 * group of an active block counts one contribution per (pair, view). */
int or_estimate_full(const or_scene* sc, const float* theta, const or_view* views, int32_t n_views,
                     const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                     uint32_t scene_index, const float* eps, const int8_t* signs, int64_t* Q, uint32_t* K,
                     double* G64, or_stats* st) {
    int64_t d = or_param_count(sc);
    int64_t G = or_group_count(sc);
    int8_t* s = (int8_t*)malloc((size_t)(d > 0 ? d : 1));
    if (!s) return -1;
    classes_t cl = texel_classes(sc);
    for (int32_t n = 0; n < n_pairs; ++n) {
        if (signs) memcpy(s, signs + (int64_t)n * d, (size_t)d);
        else or_signs(seed, step, (uint32_t)n, scene_index, d, s);
        const float* tgt = targets;
        for (int32_t v = 0; v < n_views; ++v) {
            const or_view* vw = &views[v];
            int64_t np = (int64_t)vw->width * vw->height;
            float* rgb[2];
            for (int k = 0; k < 2; ++k) {
                rgb[k] = (float*)malloc(sizeof(float) * 3 * (size_t)np);
                uint32_t* id = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(np * n_layers(sc)));
                float* uv = (float*)malloc(sizeof(float) * 2 * (size_t)(np * n_layers(sc)));
                frame_t fr;
                if (build_frame(&fr, sc, theta, s, k == 0 ? +1 : -1, eps, vw)) return -1;
                render_frame(sc, vw, &fr, rgb[k], id, uv);
                free_frame(&fr);
                free(id);
                free(uv);
            }
            int64_t qsum = 0;
            double dsum = 0.0;
            for (int64_t p = 0; p < np; ++p) {
                float delta = pixel_l2(rgb[0] + 3 * p, tgt + 3 * p) - pixel_l2(rgb[1] + 3 * p, tgt + 3 * p);
                qsum += or_quantize(delta, st);
                dsum += (double)delta;
            }
            for (int64_t i = 0; i < d; ++i) {
                float e = eps[block_of(sc, i)];
                if (e == 0.0f || s[i] == 0) continue;
                Q[i] += (int64_t)s[i] * qsum;
                if (G64) G64[i] += (double)s[i] * dsum / (2.0 * (double)e);
            }
            for (int64_t g = 0; g < G; ++g) {
                int active;
                if (g < n_pos(sc)) {
                    active = eps[0] != 0.0f;
                } else {
                    active = 0;
                    for (int c = 0; c < cl.n; ++c) {
                        int64_t size = (int64_t)sc->tex_w[cl.first[c]] * sc->tex_h[cl.first[c]];
                        if (g >= cl.offset[c] && g < cl.offset[c] + size) active = class_active(sc, &cl, eps, c);
                    }
                }
                if (active) K[g] += 1;
            }
            for (int k = 0; k < 2; ++k) free(rgb[k]);
            tgt += 3 * np;
        }
    }
    free(s);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Decode and descent (Sec. 5)                                          */
/* ------------------------------------------------------------------ */

static int64_t group_of_param(const or_scene* sc, int64_t i) {
    if (i < 3 * n_pos(sc)) return i / 3;
    int t = block_of(sc, i) - 1;
    classes_t c = texel_classes(sc);
    int64_t texel = (i - tex_offset(sc, t)) / sc->tex_c[t];
    return c.offset[c.of_tex[t]] + texel;
}

/* Reading: g_i = Q_i 2^-32 / (2 eps_i D_i), D_i the contribution count of
 * the parameter's group (or the number of pairs, Eq. 9).  A parameter with
 * no contribution (count 0) or eps_i = 0 has no gradient. */
int or_decode(const or_scene* sc, const int64_t* Q, const uint32_t* K, const float* eps,
              int32_t averaging, int32_t n_pairs, float* grad) {
    int64_t d = or_param_count(sc);
    for (int64_t i = 0; i < d; ++i) {
        float e = eps[block_of(sc, i)];
        double D = (averaging == 0) ? (double)K[group_of_param(sc, i)] : (double)n_pairs;
        if (e == 0.0f || D == 0.0) { grad[i] = 0.0f; continue; }
        grad[i] = (float)(((double)Q[i] * (1.0 / 4294967296.0)) / (2.0 * (double)e * D));
    }
    return 0;
}

int or_step(const or_scene* sc, float* theta, float* m, float* v, uint32_t t, int64_t* Q, uint32_t* K,
            const float* eps, int32_t n_pairs, const or_optim* opt, or_stats* st) {
    int64_t d = or_param_count(sc);
    int64_t G = or_group_count(sc);
    float* g = (float*)malloc(sizeof(float) * (size_t)(d > 0 ? d : 1));
    or_decode(sc, Q, K, eps, opt->averaging, n_pairs, g);
    /* Adam (Kingma and Ba), bias-corrected with the global step t >= 1;
     * the constants are formed in double and rounded to float once. */
    float b1 = opt->beta1, b2 = opt->beta2;
    float omb1 = (float)(1.0 - (double)b1), omb2 = (float)(1.0 - (double)b2);
    float bc1 = (float)(1.0 - pow((double)b1, (double)t));
    float bc2 = (float)(1.0 - pow((double)b2, (double)t));
    for (int64_t i = 0; i < d; ++i) {
        int b = block_of(sc, i);
        if (eps[b] == 0.0f) continue;
        if (opt->averaging == 0 && K[group_of_param(sc, i)] == 0) continue;
        float gi = g[i];
        if (!isfinite(gi)) {
            if (st) st->nonfinite++;
            continue;
        }
        float lr = opt->lr[b];
        if (opt->kind == 1) {
            theta[i] = theta[i] - lr * gi;
        } else {
            m[i] = b1 * m[i] + omb1 * gi;
            v[i] = b2 * v[i] + omb2 * (gi * gi);
            float mh = m[i] / bc1;
            float vh = v[i] / bc2;
            theta[i] = theta[i] - lr * (mh / (sqrtf(vh) + opt->eps_hat));
        }
    }
    memset(Q, 0, sizeof(int64_t) * (size_t)d);
    memset(K, 0, sizeof(uint32_t) * (size_t)G);
    free(g);
    return 0;
}
