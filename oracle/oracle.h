/* oracle.h -- CPU oracle of the per-pixel stochastic gradient estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Everything here is a plain, slow, single-threaded restatement of the
 * paper's method:
 *   - Eq. 8 (per-pixel stochastic finite difference) and Eq. 9 (average of
 *     N antithetic estimates), executed as Algorithm 1 (P: perturb) and
 *     Algorithm 2 (G: gradient), Sec. 4.3;
 *   - the per-primitive contribution sets of Sec. 4.4 (ID buffer -> the
 *     triangle's vertices, UV buffer -> the texels the sample reads);
 *   - Adam with beta1 = 0.9, beta2 = 0.999 (Sec. 5, gradient-descent
 *     optimizer).
 * All pointers are host pointers.  Arrays are row-major and contiguous.
 */
#ifndef DR_ORACLE_H
#define DR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_TEX 3

typedef struct {
    int32_t n_verts, n_tris;
    const int32_t* tri;        /* [F,3] vertex indices                       */
    const float* corner_uv;    /* [F,3,2] per-corner texture coordinates     */
    int32_t n_tex;             /* 0..3: albedo, normal map, roughness        */
    int32_t tex_w[OR_MAX_TEX], tex_h[OR_MAX_TEX], tex_c[OR_MAX_TEX];
    int32_t shading;           /* 0 unlit, 1 Lambert, 2 GGX                  */
    int32_t tex_mode;          /* 0 bilinear footprint, 1 nearest texel      */
    float light_dir[3];        /* unit vector towards the light              */
    float light_rgb[3];
    float ambient;
    float diffuse;
    int32_t layers;            /* 0 opaque; 1..8 semi-transparent: the       */
                               /* nearest `layers` fragments of a pixel are   */
                               /* composited front to back, alpha = channel 3 */
                               /* of the albedo (which then has 4 channels)   */
    /* Subdivision surface (Sec. 6.3): when n_ctrl > 0 the position        */
    /* parameters are n_ctrl control vertices and the n_verts vertices of  */
    /* tri are the tessellated surface, vertex j = sum over k in           */
    /* [rowptr[j], rowptr[j+1]) of w[k] * control vertex cols[k].          */
    int32_t n_ctrl;
    const int32_t* sub_rowptr;
    const int32_t* sub_cols;
    const float* sub_w;
} or_scene;

typedef struct {
    int32_t width, height;
    float view_proj[16];       /* row-major, applied to column vectors       */
    float cam_pos[3];
    float near_w;              /* vertices with clip w below this are culled */
} or_view;

typedef struct {
    int32_t kind;              /* 0 Adam, 1 SGD                              */
    int32_t averaging;         /* 0 by contribution count, 1 by pair count   */
    float lr[1 + OR_MAX_TEX];  /* per block                                  */
    float beta1, beta2, eps_hat;
} or_optim;

typedef struct {
    uint64_t saturations;      /* |delta| > 32 clamped                       */
    uint64_t nonfinite;        /* NaN delta (dropped) or non-finite update   */
} or_stats;

/* Philox4x64-10 (Salmon et al., SC'11) on one counter block. */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Rademacher sign vector of pair n at step t for scene b: s[i] in {-1,+1}. */
void or_signs(uint64_t seed, uint32_t step, uint32_t pair, uint32_t scene, int64_t d,
              int8_t* s);

int64_t or_param_count(const or_scene* sc);
int64_t or_group_count(const or_scene* sc);

/* Render theta (perturbed by sign*s*eps when s != NULL) from one view.
 * rgb [H,W,3], id [H,W,L] (0xFFFFFFFF = background or an empty layer),
 * uv [H,W,L,2], with L = max(1, layers); any output may be NULL.  Returns 0
 * on success. */
int or_render(const or_scene* sc, const float* theta, const int8_t* s, int sign,
              const float* eps, const or_view* view, float* rgb, uint32_t* id, float* uv);

/* Per-pixel L2 error f_{w,h} of a render against target [H,W,3] (Table 1). */
int or_pixel_loss(const or_scene* sc, const float* theta, const int8_t* s, int sign,
                  const float* eps, const or_view* view, const float* target, float* f);

/* Fixed-point code of a loss difference: round-half-even(delta * 2^32),
 * clamped to +-2^37; NaN -> 0. */
int64_t or_quantize(float delta, or_stats* st);

/* Eq. 9 accumulated over n_pairs antithetic pairs and n_views views.
 *   Q   int64 [d]  += s_i * q_p              (fixed point, 32 fraction bits)
 *   K   uint32 [G] += 1 per (pair, view, pixel) whose contribution set holds g
 *   G64 double [d] += s_i * delta_p / (2 eps_i)   (optional, unquantised)
 * signs == NULL draws s^(n) from Philox (seed, step, pair, scene); otherwise
 * signs is an int8 [n_pairs, d] table with entries in {-1, 0, +1}. */
int or_estimate(const or_scene* sc, const float* theta, const or_view* views, int32_t n_views,
                const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                uint32_t scene_index, const float* eps, const int8_t* signs,
                int64_t* Q, uint32_t* K, double* G64, or_stats* st);

/* The image form of or_estimate: grad_image holds, per view, the [H,W,3]
 * gradient g of a downstream loss with respect to the rendered colours, and
 * the per-pixel difference is <g_p, I+_p - I-_p> (channels r, g, b in that
 * order) in place of f+_p - f-_p.  Everything else is as for or_estimate. */
int or_estimate_image(const or_scene* sc, const float* theta, const or_view* views, int32_t n_views,
                      const float* grad_image, uint64_t seed, uint32_t step, int32_t n_pairs,
                      uint32_t scene_index, const float* eps, const int8_t* signs,
                      int64_t* Q, uint32_t* K, double* G64, or_stats* st);

/* Eq. 4, the full-image estimator: like or_estimate, but every parameter
 * (of a block with eps != 0) receives s_i * sum_p q_p of the whole image and
 * every such group counts one contribution per (pair, view). */
int or_estimate_full(const or_scene* sc, const float* theta, const or_view* views, int32_t n_views,
                     const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                     uint32_t scene_index, const float* eps, const int8_t* signs,
                     int64_t* Q, uint32_t* K, double* G64, or_stats* st);

/* Decode the fixed-point sums into float gradients (averaged). */
int or_decode(const or_scene* sc, const int64_t* Q, const uint32_t* K, const float* eps,
              int32_t averaging, int32_t n_pairs, float* grad);

/* One descent step (Adam or SGD) on theta, then Q and K are zeroed. */
int or_step(const or_scene* sc, float* theta, float* m, float* v, uint32_t t, int64_t* Q,
            uint32_t* K, const float* eps, int32_t n_pairs, const or_optim* opt, or_stats* st);

#ifdef __cplusplus
}
#endif
#endif
