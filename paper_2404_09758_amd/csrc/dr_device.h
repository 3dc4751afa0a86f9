// dr_device.h -- device-side data layout and per-pixel arithmetic of the
// per-pixel stochastic gradient estimator (gfx950).
//
// Every floating-point expression is written with explicit parentheses
// and compiled with -ffp-contract=off, so each result is the correctly
// rounded fp32 value of the stated operation sequence; divisions and square
// roots are the correctly rounded ones.  This fixed operation order is what
// makes the triangle IDs, the loss differences and hence the fixed-point
// gradient sums reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DRD_BG 0xFFFFFFFFu
#define DRD_MAX_TEX 3
#define DRD_MAX_LAYERS 4
#define DRD_MAX_VIEWS 16
#define DRD_PI 3.14159265f
#define DRD_INV_PI 0.318309886f

// Scene constants, passed by value to every kernel.
struct DScene {
    int n_verts, n_tris;
    const int* tri;             // [F,3]
    const float* cuv;           // [F,3,2]
    int n_tex;
    int tex_w[DRD_MAX_TEX], tex_h[DRD_MAX_TEX], tex_c[DRD_MAX_TEX];
    long long tex_off[DRD_MAX_TEX];      // first parameter of each texture
    int tex_cls[DRD_MAX_TEX];            // texel class of each texture
    int n_cls;
    int cls_w[DRD_MAX_TEX], cls_h[DRD_MAX_TEX];
    long long cls_goff[DRD_MAX_TEX];     // first group of each class
    int shading, tex_mode;
    int layers;                          // 0 opaque; 1..4 composited fragments
    // subdivision surface: n_ctrl > 0 control vertices are the position
    // parameters; tessellated vertex j = sum_k sub_w[k] ctrl[sub_cols[k]],
    // and tessellated triangle t credits the control vertices
    // tri_cols[tri_rowptr[t] .. tri_rowptr[t+1]) (the union of its corners')
    int n_vg;                            // position groups: n_ctrl, else n_verts
    int n_ctrl;
    const int* sub_rowptr;
    const int* sub_cols;
    const float* sub_w;
    const int* tri_rowptr;
    const int* tri_cols;
    float light[3], light_rgb[3], ambient, diffuse;
    long long d, G;
    int words;                           // ceil(d / 32) sign words per pair
};

struct DView {
    int W, H;
    float M[16];
    float cam[3];
    float near_w;
    int tiles_x, tiles_y;
    long long tgt_off;                   // first float of this view's target
};

struct DViews {
    DView v[DRD_MAX_VIEWS];
};

// Perturbation of one launch: per-block eps and the sign bits of the pairs.
struct DPert {
    const uint32_t* bits;                // [pairs, words] or null (no perturbation)
    float eps[1 + DRD_MAX_TEX];
};

// Raster half of a triangle record (48 B): snapped vertices in normalised
// (positive-area) order, flags, 1 / area and the depth plane.  The first
// 32 B hold all that the shading reads from it; the pixel box is recomputed
// from the corners where it is needed (tri_box).
struct __align__(16) TriR {
    int X[3], Y[3];
    unsigned flags;                      // bit0 valid, bit1+k top-left edge k, bit4 swapped
    float ia;                            // 1 / area2
    float z0, zx, zy;
    int pad;
};

// Shading half (48 B): 1/w in normalised order and the perturbed world
// positions in the original corner order.
struct __align__(16) TriS {
    float iw[3];
    float p[9];
};

// Per-face shading frame: the unit face normal and (GGX) the tangent frame
// of the face's UV map, formed per shaded pixel from the shading record
// (measured as fast as storing it per triangle, and 64 B per triangle and
// render less to write).
struct TriF {
    float nf[3];
    float T[3];
    float B[3];
};

static_assert(sizeof(TriR) == 48, "TriR layout");
static_assert(sizeof(TriS) == 48, "TriS layout");

#define TRI_VALID 1u
#define TRI_SWAPPED 16u
#define TRI_SMALL 32u          // bbox spans < 2^15 subpixels: 32-bit edge functions are exact

// ---------------------------------------------------------------- signs --

__device__ __forceinline__ void philox4x64_10(unsigned long long c0, unsigned long long c1,
                                              unsigned long long c2, unsigned long long c3,
                                              unsigned long long k0, unsigned long long k1,
                                              unsigned long long out[4]) {
    const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        unsigned long long hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        unsigned long long hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        unsigned long long n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// theta_i perturbed by sgn * s_i * eps (one fp32 add or subtract).
__device__ __forceinline__ float pval(const float* __restrict__ th, long long i, float e,
                                      const uint32_t* __restrict__ pb, float sgn) {
    float x = th[i];
    if (pb == nullptr || e == 0.0f) return x;
    unsigned w = pb[i >> 5];
    float se = ((w >> (unsigned)(i & 31)) & 1u) ? -e : e;
    return (sgn > 0.0f) ? (x + se) : (x - se);
}

__device__ __forceinline__ int sign_of(const uint32_t* __restrict__ pb, long long i) {
    return ((pb[i >> 5] >> (unsigned)(i & 31)) & 1u) ? -1 : 1;
}

// ------------------------------------------------------------ geometry --

struct Vtx {
    int valid;
    int X, Y;
    float z, iw;
};

__device__ __forceinline__ Vtx xform(const DView& v, float x, float y, float z) {
    const float* M = v.M;
    float cx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3];
    float cy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7];
    float cz = ((M[8] * x + M[9] * y) + M[10] * z) + M[11];
    float cw = ((M[12] * x + M[13] * y) + M[14] * z) + M[15];
    Vtx o;
    o.valid = 0; o.X = 0; o.Y = 0; o.z = 0.0f; o.iw = 0.0f;
    if (!(cw >= v.near_w)) return o;
    float nx = cx / cw, ny = cy / cw, nz = cz / cw;
    float sx = (nx * 0.5f + 0.5f) * (float)v.W;
    float sy = (0.5f - ny * 0.5f) * (float)v.H;
    float fx = sx * 256.0f, fy = sy * 256.0f;
    if (!(fabsf(fx) <= 4194304.0f) || !(fabsf(fy) <= 4194304.0f)) return o;
    o.valid = 1;
    o.X = (int)rintf(fx);
    o.Y = (int)rintf(fy);
    o.z = nz * 0.5f + 0.5f;
    o.iw = 1.0f / cw;
    return o;
}

// Edge k of a normalised triangle runs from vertex k+1 to vertex k+2.
__device__ __forceinline__ long long edge_at(int xa, int ya, int xb, int yb, int px, int py) {
    return (long long)(xb - xa) * (long long)(py - ya) - (long long)(yb - ya) * (long long)(px - xa);
}

__device__ __forceinline__ bool inside(const TriR& r, int px, int py, long long& e0, long long& e1,
                                       long long& e2) {
    e0 = edge_at(r.X[1], r.Y[1], r.X[2], r.Y[2], px, py);
    e1 = edge_at(r.X[2], r.Y[2], r.X[0], r.Y[0], px, py);
    e2 = edge_at(r.X[0], r.Y[0], r.X[1], r.Y[1], px, py);
    bool ok0 = (e0 > 0) || (e0 == 0 && (r.flags & 2u));
    bool ok1 = (e1 > 0) || (e1 == 0 && (r.flags & 4u));
    bool ok2 = (e2 > 0) || (e2 == 0 && (r.flags & 8u));
    return ok0 && ok1 && ok2;
}

// The same coverage test for triangles flagged TRI_SMALL: every product is
// below 2^30 in magnitude, so 24-bit multiplies give the exact values.
__device__ __forceinline__ bool inside_small(const TriR& r, int px, int py) {
    int e0 = __mul24(r.X[2] - r.X[1], py - r.Y[1]) - __mul24(r.Y[2] - r.Y[1], px - r.X[1]);
    int e1 = __mul24(r.X[0] - r.X[2], py - r.Y[2]) - __mul24(r.Y[0] - r.Y[2], px - r.X[2]);
    int e2 = __mul24(r.X[1] - r.X[0], py - r.Y[0]) - __mul24(r.Y[1] - r.Y[0], px - r.X[0]);
    bool ok0 = (e0 > 0) || (e0 == 0 && (r.flags & 2u));
    bool ok1 = (e1 > 0) || (e1 == 0 && (r.flags & 4u));
    bool ok2 = (e2 > 0) || (e2 == 0 && (r.flags & 8u));
    return ok0 && ok1 && ok2;
}

// Pixel box of a triangle clipped to [px0, cx1] x [py0, cy1] (px0, py0 >= 0):
// the pixels whose centre 256 x + 128 lies within the snapped corners'
// bounds.  Empty when x0 > x1 or y0 > y1.
__device__ __forceinline__ void tri_box(const TriR& r, int px0, int py0, int cx1, int cy1, int& x0, int& x1,
                                        int& y0, int& y1) {
    int xmin = min(r.X[0], min(r.X[1], r.X[2])), xmax = max(r.X[0], max(r.X[1], r.X[2]));
    int ymin = min(r.Y[0], min(r.Y[1], r.Y[2])), ymax = max(r.Y[0], max(r.Y[1], r.Y[2]));
    x0 = max((xmin + 127) >> 8, px0);
    x1 = min((xmax - 128) >> 8, cx1);
    y0 = max((ymin + 127) >> 8, py0);
    y1 = min((ymax - 128) >> 8, cy1);
}

__device__ __forceinline__ float depth_at(const TriR& r, int px, int py) {
    float z = (r.z0 + r.zx * (float)(px - r.X[0])) + r.zy * (float)(py - r.Y[0]);
    if (!(z > 0.0f)) z = 0.0f;
    return z;
}

// ------------------------------------------------------------- sampling --

struct Foot {
    int xa, xb, ya, yb;
    float fx, fy;
};

__device__ __forceinline__ Foot footprint(float u, float v, int W, int H) {
    Foot f;
    float x = u * (float)W - 0.5f;
    float y = v * (float)H - 0.5f;
    if (!(fabsf(x) < 16777216.0f)) x = 0.0f;
    if (!(fabsf(y) < 16777216.0f)) y = 0.0f;
    float x0f = floorf(x), y0f = floorf(y);
    f.fx = x - x0f;
    f.fy = y - y0f;
    int x0 = (int)x0f, y0 = (int)y0f;
    // x0 mod W (non-negative); UVs within a period or two need no division
    int xa;
    if (x0 >= 0 && x0 < W) xa = x0;
    else if (x0 >= W && x0 < 2 * W) xa = x0 - W;
    else if (x0 < 0 && x0 >= -W) xa = x0 + W;
    else {
        xa = x0 % W;
        if (xa < 0) xa += W;
    }
    f.xa = xa;
    f.xb = (xa + 1 == W) ? 0 : xa + 1;
    f.ya = y0 < 0 ? 0 : (y0 > H - 1 ? H - 1 : y0);
    int y1 = y0 + 1;
    f.yb = y1 < 0 ? 0 : (y1 > H - 1 ? H - 1 : y1);
    return f;
}

// Global-memory views of device pointers (address space 1).  Loads and
// atomics through them compile to global_* instructions instead of flat_*
// ones, so the compiler can wait on each request by itself instead of on
// all outstanding memory and LDS traffic together.
#define DRD_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ T gload(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const DRD_GLOBAL T*)p;
#else
    return *p;             // host pass: parsed, never run
#endif
}

// Bilinear sample of one texture with C channels per texel (C consecutive
// parameters per texel), perturbed as by pval.  All four texels' values and
// sign words are requested before any is used.  The perturbed value is
// x + (s_i ? -es : es) with es = +-eps by the render's sign: x - y and
// x + (-y) are the same IEEE operation, so this equals pval's result.
// 64-bit word at a 4-byte aligned address (one load of two sign words)
typedef unsigned long long __attribute__((aligned(4))) drd_u64_a4;

template <int C>
__device__ __forceinline__ void sample_texels(const DRD_GLOBAL float* th, const DRD_GLOBAL uint32_t* pb,
                                              long long base, int W, float e, float sgn, const Foot& f,
                                              float* out) {
    const DRD_GLOBAL float* tt = th + base;
    const bool pert = pb != nullptr && e != 0.0f;
    const DRD_GLOBAL uint32_t* pw = pb + (base >> 5);
    unsigned bb = (unsigned)(base & 31);
    // s_i (sgn e) is e (>= 0) with its sign bit set to the sign bit s_i
    // holds -- complemented for the minus render: the IEEE value of
    // +-e exactly, so x + it is the same operation as pval's
    const unsigned eb = __float_as_uint(e);
    const unsigned flip = (sgn > 0.0f) ? 0u : 0xFFFFFFFFu;
    float wx[2] = {1.0f - f.fx, f.fx};
    float acc[C];
    // row by row (ya, then yb), two texels each: the weighted sum keeps its
    // order ((w00 t00 + w10 t10) + w01 t01) + w11 t11
#pragma unroll
    for (int row = 0; row < 2; ++row) {
        int yy = row ? f.yb : f.ya;
        float wy = row ? f.fy : 1.0f - f.fy;
        // texel offsets within the texture: W, H <= 32768 and C <= 4 keep
        // them below 2^32
        unsigned o[2];
        const unsigned ro = __umul24((unsigned)yy, (unsigned)W);      // W, H <= 32768: exact
        o[0] = (ro + (unsigned)f.xa) * C;
        o[1] = (ro + (unsigned)f.xb) * C;
        float x[2][C];
        if (C == 1 && f.xb == f.xa + 1) {
            // the row's two single-channel texels are adjacent: one 8 B read
            typedef float __attribute__((ext_vector_type(2), aligned(4))) f2a4;
            f2a4 v = *(const DRD_GLOBAL f2a4*)(tt + o[0]);
            x[0][0] = v.x;
            x[1][0] = v.y;
        } else {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int c = 0; c < C; ++c) x[k][c] = tt[(unsigned long long)o[k] + c];
        }
        if (pert) {
            // parameter base + o has its sign at bit (base + o) mod 32 of
            // word (base + o) / 32.  One 64-bit read at that word holds the
            // texel's C bits and, when xb = xa + 1, the next texel's C bits
            // right after them (at most bit 31 + 2 C < 64); a wrapped xb
            // reads its own.  The sign buffers carry a spare word at the
            // end, so the read past a pair's last word stays in bounds (its
            // bits belong to no parameter of the texel).
            unsigned r = (o[0] & 31u) + bb;
            unsigned long long w = *(const DRD_GLOBAL drd_u64_a4*)(pw + (o[0] >> 5) + (r >> 5));
            unsigned win[2];
            win[0] = __builtin_amdgcn_alignbit((unsigned)(w >> 32), (unsigned)w, r & 31u);
            win[1] = win[0] >> C;
            if (f.xb != f.xa + 1) {
                unsigned rb = (o[1] & 31u) + bb;
                unsigned long long wb = *(const DRD_GLOBAL drd_u64_a4*)(pw + (o[1] >> 5) + (rb >> 5));
                win[1] = __builtin_amdgcn_alignbit((unsigned)(wb >> 32), (unsigned)wb, rb & 31u);
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const unsigned wk = win[k] ^ flip;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    x[k][c] = x[k][c] + __uint_as_float(((wk << (31 - c)) & 0x80000000u) | eb);
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float t0 = (wx[0] * wy) * x[0][c], t1 = (wx[1] * wy) * x[1][c];
            acc[c] = row ? ((acc[c] + t0) + t1) : (t0 + t1);
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = acc[c];
}

// Bilinear sample of texture t of the perturbed scene (theta + sgn s eps)
// over a precomputed footprint.  out has room for 4 channels; channels at
// and beyond the texture's count keep their values.
__device__ __forceinline__ void sample_tex(const DScene& sc, const float* __restrict__ th,
                                           const uint32_t* __restrict__ pb, float e, float sgn, int t,
                                           const Foot& f, float* out) {
    int W = sc.tex_w[t], C = sc.tex_c[t];
    long long base = sc.tex_off[t];
    const DRD_GLOBAL float* gth = (const DRD_GLOBAL float*)th;
    const DRD_GLOBAL uint32_t* gpb = (const DRD_GLOBAL uint32_t*)pb;
    if (C == 3) sample_texels<3>(gth, gpb, base, W, e, sgn, f, out);
    else if (C == 1) sample_texels<1>(gth, gpb, base, W, e, sgn, f, out);
    else if (C == 4) sample_texels<4>(gth, gpb, base, W, e, sgn, f, out);
    else sample_texels<2>(gth, gpb, base, W, e, sgn, f, out);
}

// Correctly rounded square root and reciprocal for operands in a normal
// range, in fewer instructions than the general sequences.
// sqrt_rn: for x in [2^-96, 2^126] the hardware square root (within 1 ulp)
// corrected by the residuals of its two neighbours -- the correction the
// compiler's sqrtf applies, without its scaling of tiny inputs and its
// handling of 0, inf and NaN.  rcp_rn: for |y| in [2^-125, 2^125] the
// hardware reciprocal refined by one Newton step with fused multiply-adds.
// Both are checked against sqrtf and 1.0f / y for every operand of those
// ranges (dr_probe_math); operands outside them take sqrtf and division.
#define DRD_SQRT_LO 0x0F800000u        // 2^-96
#define DRD_SQRT_HI 0x7E800000u        // 2^126
#define DRD_RCP_LO 0x01000000u         // 2^-125
#define DRD_RCP_HI 0x7E000000u         // 2^125

__device__ __forceinline__ float sqrt_rn_fast(float x) {
    float s = __builtin_amdgcn_sqrtf(x);
    float sm = __uint_as_float(__float_as_uint(s) - 1u), sp = __uint_as_float(__float_as_uint(s) + 1u);
    float rm = __builtin_fmaf(-sm, s, x), rp = __builtin_fmaf(-sp, s, x);
    s = (rm <= 0.0f) ? sm : s;
    return (rp > 0.0f) ? sp : s;
}

__device__ __forceinline__ float rcp_rn_fast(float y) {
    float r = __builtin_amdgcn_rcpf(y);
    float e = __builtin_fmaf(-y, r, 1.0f);
    return __builtin_fmaf(e, r, r);
}

__device__ __forceinline__ bool sqrt_fast_ok(float x) {
    unsigned b = __float_as_uint(x);
    return b >= DRD_SQRT_LO && b <= DRD_SQRT_HI;            // positive, in range
}

__device__ __forceinline__ bool rcp_fast_ok(float y) {
    unsigned b = __float_as_uint(y) & 0x7FFFFFFFu;
    return b >= DRD_RCP_LO && b <= DRD_RCP_HI;
}

// sqrtf(x), correctly rounded
__device__ __forceinline__ float sqrt_rn(float x) { return sqrt_fast_ok(x) ? sqrt_rn_fast(x) : sqrtf(x); }

// 1.0f / y, correctly rounded
__device__ __forceinline__ float rcp_rn(float y) { return rcp_fast_ok(y) ? rcp_rn_fast(y) : 1.0f / y; }

__device__ __forceinline__ void nrm3(float* x) {
    float l2 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
    if (l2 > 0.0f) {
        float inv = rcp_rn(sqrt_rn(l2));                     // 1 / sqrt(l2), each correctly rounded
        x[0] = x[0] * inv; x[1] = x[1] * inv; x[2] = x[2] * inv;
    } else {
        x[0] = 0.0f; x[1] = 0.0f; x[2] = 0.0f;
    }
}

__device__ __forceinline__ float dot3(const float* a, const float* b) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

__device__ __forceinline__ void cross3(const float* a, const float* b, float* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Face frame of a triangle from its perturbed corners p (original order)
// and corner UVs: the unit face normal and, for GGX, the tangent frame.
// A triangle's corner UVs (original corner order), read once per shaded
// pixel and render for both the face frame and the attributes.
struct CornerUV {
    float c[6];
};

__device__ __forceinline__ CornerUV load_cuv(const DScene& sc, unsigned t) {
    return gload((const CornerUV*)(sc.cuv + 6 * (long long)t));
}

__device__ __forceinline__ void face_frame(int shading, const float* p, const CornerUV& cu, TriF& F) {
    const float* cuv = cu.c;
    float e1v[3], e2v[3], nf[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { e1v[c] = p[3 + c] - p[c]; e2v[c] = p[6 + c] - p[c]; }
    cross3(e1v, e2v, nf);
    nrm3(nf);
#pragma unroll
    for (int c = 0; c < 3; ++c) { F.nf[c] = nf[c]; F.T[c] = 0.0f; F.B[c] = 0.0f; }
    if (shading != 2) return;
    float du1 = cuv[2] - cuv[0], dv1 = cuv[3] - cuv[1], du2 = cuv[4] - cuv[0], dv2 = cuv[5] - cuv[1];
    float rr = du1 * dv2 - du2 * dv1;
    float T[3], B[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) T[c] = e1v[c] * dv2 - e2v[c] * dv1;
    if (rr < 0.0f) { T[0] = -T[0]; T[1] = -T[1]; T[2] = -T[2]; }
    float nt = dot3(nf, T);
#pragma unroll
    for (int c = 0; c < 3; ++c) T[c] = T[c] - nf[c] * nt;
    nrm3(T);
    cross3(nf, T, B);
#pragma unroll
    for (int c = 0; c < 3; ++c) { F.T[c] = T[c]; F.B[c] = B[c]; }
}

// Perspective-correct attributes of pixel (px,py) on triangle t: the
// 1/w-weighted barycentrics, the reciprocal of their sum and the UV.
struct Attr {
    float pc0, pc1, pc2, iS, u, v;
};

__device__ __forceinline__ Attr frag_attr(const DScene& sc, const TriR& r, const TriS& s, const CornerUV& cu, int px,
                                          int py) {
    // edge functions as floats; for a TRI_SMALL triangle they fit in 32 bits
    // and convert in one instruction, to the same values
    float f0, f1, f2;
    if (r.flags & TRI_SMALL) {
        int e0 = __mul24(r.X[2] - r.X[1], py - r.Y[1]) - __mul24(r.Y[2] - r.Y[1], px - r.X[1]);
        int e1 = __mul24(r.X[0] - r.X[2], py - r.Y[2]) - __mul24(r.Y[0] - r.Y[2], px - r.X[2]);
        int e2 = __mul24(r.X[1] - r.X[0], py - r.Y[0]) - __mul24(r.Y[1] - r.Y[0], px - r.X[0]);
        f0 = (float)e0; f1 = (float)e1; f2 = (float)e2;
    } else {
        long long e0, e1, e2;
        (void)inside(r, px, py, e0, e1, e2);
        f0 = (float)e0; f1 = (float)e1; f2 = (float)e2;
    }
    float b0 = f0 * r.ia, b1 = f1 * r.ia, b2 = f2 * r.ia;
    float pc0 = b0 * s.iw[0], pc1 = b1 * s.iw[1], pc2 = b2 * s.iw[2];
    float S = (pc0 + pc1) + pc2;
    float iS = rcp_rn(S);
    bool sw = (r.flags & TRI_SWAPPED) != 0u;
    const float* cuv = cu.c;
    float cu0 = cuv[0], cv0 = cuv[1], cu1 = cuv[2], cv1 = cuv[3], cu2 = cuv[4], cv2 = cuv[5];
    float un1 = sw ? cu2 : cu1, vn1 = sw ? cv2 : cv1, un2 = sw ? cu1 : cu2, vn2 = sw ? cv1 : cv2;
    Attr a;
    a.pc0 = pc0; a.pc1 = pc1; a.pc2 = pc2; a.iS = iS;
    a.u = ((pc0 * cu0 + pc1 * un1) + pc2 * un2) * iS;
    a.v = ((pc0 * cv0 + pc1 * vn1) + pc2 * vn2) * iS;
    return a;
}

// Colour, opacity and UV of pixel (px,py) (subpixel sample coordinates)
// covered by triangle t: perspective-correct attributes, then unlit /
// Lambert / GGX.  foot0 receives the bilinear footprint of texel class 0 at
// the pixel; opacity the albedo's fourth channel clamped to [0, 1] (1 for a
// three-channel albedo).
__device__ __forceinline__ void shade_pixel(const DScene& sc, const DView& vw, const float* __restrict__ th,
                                            const uint32_t* __restrict__ pb, const float* eps, float sgn,
                                            const TriR& r, const TriS& s, const TriF& fr, const CornerUV& cu,
                                            int px, int py,
                                            float* rgb, float* uvo, Foot& foot0, float& opacity) {
    Attr a = frag_attr(sc, r, s, cu, px, py);
    float pc0 = a.pc0, pc1 = a.pc1, pc2 = a.pc2, iS = a.iS, u = a.u, v = a.v;
    bool sw = (r.flags & TRI_SWAPPED) != 0u;
    int o1 = sw ? 2 : 1, o2 = sw ? 1 : 2;
    uvo[0] = u;
    uvo[1] = v;
    float alb[4] = {0.0f, 0.0f, 0.0f, 1.0f};
    if (sc.n_tex > 0) {
        foot0 = footprint(u, v, sc.cls_w[0], sc.cls_h[0]);
        sample_tex(sc, th, pb, eps[1], sgn, 0, foot0, alb);
    }
    float al = alb[3];
    if (!(al > 0.0f)) al = 0.0f;
    if (al > 1.0f) al = 1.0f;
    opacity = al;
    if (sc.shading == 0) {
        rgb[0] = alb[0]; rgb[1] = alb[1]; rgb[2] = alb[2];
        return;
    }
    const float* nf = fr.nf;
    if (sc.shading == 1) {
        float ndl = dot3(nf, sc.light);
        if (!(ndl > 0.0f)) ndl = 0.0f;
        float sh = sc.ambient + sc.diffuse * ndl;
#pragma unroll
        for (int c = 0; c < 3; ++c) rgb[c] = alb[c] * (sh * sc.light_rgb[c]);
        return;
    }
    // GGX with a tangent-space normal map in the face's UV frame
    float nm[4] = {0.5f, 0.5f, 1.0f, 0.0f};
    if (sc.n_tex > 1) {
        int c1 = sc.tex_cls[1];
        Foot f1 = (c1 == 0) ? foot0 : footprint(u, v, sc.cls_w[c1], sc.cls_h[c1]);
        sample_tex(sc, th, pb, eps[2], sgn, 1, f1, nm);
    }
    float tn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) tn[c] = 2.0f * nm[c] - 1.0f;
    float n[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) n[c] = (fr.T[c] * tn[0] + fr.B[c] * tn[1]) + nf[c] * tn[2];
    nrm3(n);
    float rough4[4] = {0.5f, 0.0f, 0.0f, 0.0f};
    if (sc.n_tex > 2) {
        int c2 = sc.tex_cls[2];
        Foot f2 = (c2 == 0) ? foot0 : footprint(u, v, sc.cls_w[c2], sc.cls_h[c2]);
        sample_tex(sc, th, pb, eps[3], sgn, 2, f2, rough4);
    }
    float P[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float q0 = s.p[c], q1 = s.p[3 * o1 + c], q2 = s.p[3 * o2 + c];
        P[c] = ((pc0 * q0 + pc1 * q1) + pc2 * q2) * iS;
    }
    float V[3] = {vw.cam[0] - P[0], vw.cam[1] - P[1], vw.cam[2] - P[2]};
    nrm3(V);
    const float* L = sc.light;
    float Hh[3] = {L[0] + V[0], L[1] + V[1], L[2] + V[2]};
    nrm3(Hh);
    float ndl = dot3(n, L), ndv = dot3(n, V), ndh = dot3(n, Hh), vdh = dot3(V, Hh);
    if (!(ndl > 0.0f)) ndl = 0.0f;
    if (!(ndv > 0.0f)) ndv = 0.0f;
    if (!(ndh > 0.0f)) ndh = 0.0f;
    if (!(vdh > 0.0f)) vdh = 0.0f;
    float alpha = rough4[0] * rough4[0];
    if (!(alpha > 0.002f)) alpha = 0.002f;
    float a2 = alpha * alpha;
    // D G F / (4 n.l n.v) with D = a2 / (pi dd^2) and Smith-Schlick
    // G = n.l / gl * n.v / gv: n.l n.v cancel, leaving one division
    float dd = (ndh * ndh) * (a2 - 1.0f) + 1.0f;
    float k = alpha * 0.5f;
    float gl = ndl * (1.0f - k) + k;
    float gv = ndv * (1.0f - k) + k;
    float om = 1.0f - vdh;
    float om5 = ((om * om) * (om * om)) * om;
    float F = 0.04f + 0.96f * om5;
    float spec = 0.0f;
    if (ndl > 0.0f && ndv > 0.0f) spec = (a2 * F) / ((((4.0f * DRD_PI) * dd) * dd) * (gl * gv));
#pragma unroll
    for (int c = 0; c < 3; ++c)
        rgb[c] = ((alb[c] * DRD_INV_PI + spec) * sc.light_rgb[c]) * ndl + sc.ambient * alb[c];
}

// Fixed-point code of a loss difference: round-half-even(delta * 2^32),
// clamped to +-2^37; NaN gives 0.  flag: 1 saturated, 2 NaN.
__device__ __forceinline__ long long quantize(float delta, int& flag) {
    flag = 0;
    if (delta != delta) { flag = 2; return 0; }
    if (fabsf(delta) > 32.0f) {
        flag = 1;
        return delta > 0.0f ? (1ll << 37) : -(1ll << 37);
    }
    return (long long)rintf(delta * 4294967296.0f);
}

// The per-pixel difference that Eq. 8 scatters, from the colours of the two
// renders.  Loss form (img == 0): f+ - f- with f the L2 error against the
// target t (Table 1).  Image form (img != 0): t is the gradient g of a
// downstream loss with respect to the pixel's colour and the difference is
// <g, I+ - I->, the first-order change of that loss, so that the estimator
// approximates the vector-Jacobian product of the render.
__device__ __forceinline__ float pixel_delta(const float* p, const float* m, const float* t_, int img) {
    const DRD_GLOBAL float* t = (const DRD_GLOBAL float*)t_;
    float t0 = t[0], t1 = t[1], t2 = t[2];
    if (img) {
        float d0 = p[0] - m[0], d1 = p[1] - m[1], d2 = p[2] - m[2];
        return (t0 * d0 + t1 * d1) + t2 * d2;
    }
    float dr0 = p[0] - t0, dg0 = p[1] - t1, db0 = p[2] - t2;
    float dr1 = m[0] - t0, dg1 = m[1] - t1, db1 = m[2] - t2;
    float fp = (dr0 * dr0 + dg0 * dg0) + db0 * db0;
    float fm = (dr1 * dr1 + dg1 * dg1) + db1 * db1;
    return fp - fm;
}
