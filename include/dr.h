/* dr.h -- per-pixel stochastic gradient estimator for MI355X (gfx950).
 *
 * C ABI of the library that turns a non-differentiable rasterizer into a
 * differentiable one by stochastic finite differences evaluated per pixel
 * (Deliot, Heitz, Belcour 2024).  The operations follow the paper's
 * statement of the problem: a scene theta in R^d (geometry and textures,
 * Sec. 4.1 / Table 1) is rendered to an image I(theta); the objective is the
 * L2 error f = || I(theta) - I ||^2 against a target; its gradient is
 * estimated with Eq. 8 (one antithetic pair of Rademacher perturbations,
 * each pixel's loss difference credited only to the parameters that pixel
 * used) and averaged over N pairs (Eq. 9) before a descent step (Sec. 5).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers owned by the caller (the library
 *    never frees them), contiguous, 4-byte aligned (8 for int64), on the
 *    GPU the context was created on.  Struct arguments are host memory and
 *    are copied before the call returns.
 *  - Calls are asynchronous on the context's HIP stream; results are ready
 *    once that stream is synchronised.  dr_stats synchronises it.
 *  - Errors are returned as dr_status codes (never aborts or exceptions);
 *    dr_last_error gives the message of the last failing call.  An invalid
 *    argument is detected on the host and nothing is launched.
 *  - A context serves one stream and is not thread-safe; calls on one
 *    context must not overlap.
 *
 * Flat parameter layout (shared by theta, Q, the Adam moments and the
 * signs):  [ positions V x 3 (x,y,z) | texture 0 (H0,W0,C0) | texture 1 |
 * texture 2 ], row-major texels, channels innermost.  Blocks: 0 =
 * positions, 1 + t = texture t.  Textures: 0 albedo (3 channels), 1
 * tangent-space normal map (3), 2 roughness (1).
 *
 * Contribution groups (the unit of the counts K): one group per vertex,
 * then one per texel of each distinct texture resolution ("texel class",
 * numbered in order of first appearance): textures of equal resolution
 * share their texel groups because a sample reads the same texel
 * coordinates in all of them.
 */
#ifndef DR_H
#define DR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DR_MAX_TEX 3
#define DR_MAX_LAYERS 4
#define DR_MAX_VIEWS 16
#define DR_BG_ID 0xFFFFFFFFu

typedef enum {
    DR_OK = 0,
    DR_E_INVALID = -1,      /* bad argument, detected on the host           */
    DR_E_OOM = -2,          /* device allocation failed                      */
    DR_E_HIP = -3,          /* HIP runtime or launch error                   */
    DR_E_UNSUPPORTED = -4   /* valid but not supported by this build         */
} dr_status;

enum { DR_UNLIT = 0, DR_LAMBERT = 1, DR_GGX = 2 };
enum { DR_TEX_FOOTPRINT = 0, DR_TEX_NEAREST = 1 };
enum { DR_AVG_COUNT = 0, DR_AVG_PAIRS = 1 };
enum { DR_ADAM = 0, DR_SGD = 1 };

typedef struct dr_ctx dr_ctx;

/* Fixed scene data.  tri and corner_uv are device pointers that must stay
 * valid for the life of the context. */
typedef struct {
    int32_t n_verts, n_tris;
    const int32_t* tri;          /* [F,3] vertex indices                      */
    const float* corner_uv;      /* [F,3,2] per-corner texture coordinates    */
    int32_t n_tex;               /* 0..3                                      */
    int32_t tex_w[DR_MAX_TEX], tex_h[DR_MAX_TEX], tex_c[DR_MAX_TEX];
    int32_t shading;             /* DR_UNLIT | DR_LAMBERT | DR_GGX            */
    int32_t tex_mode;            /* DR_TEX_FOOTPRINT | DR_TEX_NEAREST         */
    float light_dir[3];          /* unit vector towards the light             */
    float light_rgb[3];
    float ambient, diffuse;
    int32_t layers;              /* 0: opaque.  1..DR_MAX_LAYERS: semi-       */
                                 /* transparent (Sec. 4.4): the `layers`      */
                                 /* nearest fragments of each pixel, in depth */
                                 /* order, composited front to back over      */
                                 /* black; opacity = the albedo's fourth      */
                                 /* channel (tex_c[0] must then be 4),        */
                                 /* clamped to [0, 1].  Needs tile_px <= 16.  */
    /* Subdivision surface (Sec. 6.3): n_ctrl > 0 makes the position
     * parameters n_ctrl control vertices (theta starts with 3 * n_ctrl
     * coordinates) and tri / corner_uv / n_verts the tessellated surface
     * (see dr_subdivide), whose vertex j is, per coordinate, the sum over k
     * in [sub_rowptr[j], sub_rowptr[j+1]) of sub_w[k] times control vertex
     * sub_cols[k], added in that order from zero (device pointers, valid
     * for the life of the context).  A pixel's vertex groups are then the
     * control vertices its triangle's corners combine.  Opaque scenes only
     * (layers == 0); not available in a dr_batch.  n_ctrl == 0: the mesh's
     * own vertices are the parameters. */
    int32_t n_ctrl;
    const int32_t* sub_rowptr;   /* [n_verts + 1]                             */
    const int32_t* sub_cols;     /* [nnz], ascending within a row             */
    const float* sub_w;          /* [nnz]                                     */
} dr_scene;

/* A camera: clip = view_proj * [x y z 1]^T (row-major); pixel (0,0) is the
 * top-left.  Vertices with clip w < near_w cull their triangles. */
typedef struct {
    int32_t width, height;
    float view_proj[16];
    float cam_pos[3];
    float near_w;
} dr_view;

/* Launch shape.  Raster tiles are tile_px (8, 16 or 32) pixels square,
 * each with a bin of bin_capacity triangles; the entries of a bin past its
 * capacity go to a spill list of the render (8192 entries), which the
 * overflowing tile reads after its bin; only when that list is full does
 * the tile test every triangle of the render.  items_per_launch is the number of
 * (pair, view) items one raster launch covers: 1 = one launch per item
 * ("plain"), 0 = every item of the call in one launch ("batched").
 * Results never depend on these values. */
typedef struct {
    int32_t tile_px;
    int32_t bin_capacity;
    int32_t items_per_launch;
} dr_tuning;

/* A perturbation of theta (Alg. 1): theta + sign * s (.) eps, with s the
 * Rademacher vector of (seed, step, pair, scene_index). */
typedef struct {
    uint64_t seed;
    uint32_t step, pair, scene_index;
    int32_t sign;                /* +1 or -1                                  */
    float eps[1 + DR_MAX_TEX];   /* per block; 0 leaves the block unperturbed */
} dr_perturb;

typedef struct {
    int32_t kind;                /* DR_ADAM | DR_SGD                          */
    int32_t averaging;           /* DR_AVG_COUNT | DR_AVG_PAIRS               */
    float lr[1 + DR_MAX_TEX];    /* per block                                 */
    float beta1, beta2, eps_hat;
} dr_optim;

typedef struct {
    uint64_t tile_overflows;     /* (tile, render) bins that overflowed       */
    uint64_t saturations;        /* loss differences clamped to |delta| = 32  */
    uint64_t nonfinite;          /* NaN differences dropped; non-finite
                                    gradients skipped by dr_step              */
    uint64_t max_bin;            /* largest bin occupancy seen (triangles)    */
    uint64_t full_scans;         /* overflowing bins whose render's spill list
                                    (8192 entries) was full, so the tile tested
                                    every triangle of the render              */
} dr_stats_t;

/* Create a context for one scene on the current HIP device; stream is a
 * hipStream_t (NULL = default stream); tune NULL picks 16 px tiles, 256
 * triangles per bin and one launch per item. */
dr_status dr_create(dr_ctx** out, const dr_scene* scene, const dr_tuning* tune, void* stream);
dr_status dr_destroy(dr_ctx* ctx);
dr_status dr_set_stream(dr_ctx* ctx, void* stream);
dr_status dr_set_tuning(dr_ctx* ctx, const dr_tuning* tune);
/* Catmull-Clark tessellation of a closed manifold triangle control mesh
 * (Sec. 6.3; Catmull and Clark 1978), on the host: `levels` (1 or 2)
 * refinements, then every quad (q0, q1, q2, q3) split into (q0, q1, q2) and
 * (q0, q2, q3).  Rules per level: face point = mean of the face's vertices;
 * edge point = (a + b + f1 + f2) / 4; vertex point = (Q + 2 R + (n - 3) v) / n
 * with n the valence, Q the mean of the adjacent face points and R the mean
 * of the adjacent edge midpoints.  Numbering: vertex points first (vertex i
 * keeps index i), then edge points in order of first appearance (faces in
 * order, edges (v_k, v_k+1)), then face points; face (v_0 .. v_m-1) becomes
 * the quads (v'_k, e(v_k, v_k+1), f', e(v_k-1, v_k)), k = 0 .. m-1.
 * Weights are exact rationals rounded once (num / den in double, then to
 * float).  Texture coordinates are face-varying and refined linearly in the
 * control triangle: fine corner UV = ((n0 ua + n1 ub) + n2 uc) / 24 in double,
 * rounded to float, with n_k / 24 the corner's barycentrics.
 * All pointers are HOST pointers.  dr_subdivide_sizes reports the output
 * sizes; dr_subdivide fills fine_tri [F_f,3], fine_corner_uv [F_f,3,2],
 * rowptr [n_fine + 1], cols and w [nnz] (the sub_* arrays of dr_scene).
 * DR_E_INVALID for indices out of range, a mesh that is not a closed
 * manifold, or levels outside 1..2. */
dr_status dr_subdivide_sizes(const int32_t* tri, int32_t n_verts, int32_t n_tris, int32_t levels,
                             int32_t* n_fine_verts, int32_t* n_fine_tris, int64_t* nnz);
dr_status dr_subdivide(const int32_t* tri, const float* corner_uv, int32_t n_verts, int32_t n_tris,
                       int32_t levels, int32_t* fine_tri, float* fine_corner_uv, int32_t* rowptr,
                       int32_t* cols, float* w);

/* Adaptive bin capacity (default on): after an estimate whose largest tile
 * bin exceeded bin_capacity (an overflowing tile also reads the render's
 * spill list, exact but slower), a later dr_estimate_grad* call raises
 * the capacity to the next power of two above 1.5x that bin (at most 2^16),
 * reallocating the bins once.  The figure is read back asynchronously, so
 * the raise may come one call later.  Results never depend on it.
 * dr_get_tuning reports the launch shape in force. */
dr_status dr_set_adaptive_bins(dr_ctx* ctx, int32_t on);
dr_status dr_get_tuning(const dr_ctx* ctx, dr_tuning* out);

/* Counter word 3 of the sign stream of dr_estimate_grad (default 0): the
 * index of this scene in a batch, so that a scene stepped alone draws the
 * same signs as in a dr_batch. */
dr_status dr_set_scene_index(dr_ctx* ctx, uint32_t scene_index);
int64_t dr_param_count(const dr_ctx* ctx);       /* d                         */
int64_t dr_group_count(const dr_ctx* ctx);       /* number of groups G        */

/* The rasterizer R extended with ID and UV buffers (Sec. 4.4): render theta
 * (perturbed when pert != NULL) from one view.  rgb [H,W,3] float, id [H,W]
 * uint32 (DR_BG_ID where no triangle covers the pixel centre), uv [H,W,2]
 * float (0 on background); any output may be NULL.  For a semi-transparent
 * scene id and uv are deep buffers, [H,W,layers] and [H,W,layers,2], front
 * to back, unused layers DR_BG_ID and 0. */
dr_status dr_render(dr_ctx* ctx, const float* theta, const dr_view* view, const dr_perturb* pert,
                    float* rgb, uint32_t* id, float* uv);

/* The objective of Table 1: f(theta) = || I(theta) - I ||^2 = sum over
 * pixels of f_{w,h}, per view.  targets as for dr_estimate_grad; loss
 * [n_views] double (device), each the sum of the per-pixel fp32 errors in
 * a fixed order (reproducible run to run). */
dr_status dr_loss(dr_ctx* ctx, const float* theta, const dr_view* views, int32_t n_views,
                  const float* targets, double* loss);

/* The sign vector of one pair (Alg. 1, randomsign): bit i of the uint32
 * words bits[ceil(d/32)] set means s_i = -1. */
dr_status dr_signs(dr_ctx* ctx, uint64_t seed, uint32_t step, uint32_t pair, uint32_t scene_index,
                   uint32_t* bits);

/* Eq. 8 for n_pairs antithetic pairs over n_views views (Eq. 9 numerator),
 * accumulated into the caller's buffers:
 *   Q [d] int64:  Q_i += s_i * round(delta_p * 2^32)   over every pixel p
 *                 (of every pair and view) whose contribution set holds i;
 *   K [G] uint32: K_g += 1 per (pair, view, pixel) whose set holds group g.
 * The contribution set of a pixel is the union over the two renders of
 * the visible triangle's three vertices (ID buffer) and the texels its
 * sample read (UV buffer).  targets: device, the views' [H,W,3] float
 * images concatenated in view order.  eps: host, per block (>= 0). */
dr_status dr_estimate_grad(dr_ctx* ctx, const float* theta, const dr_view* views, int32_t n_views,
                           const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                           const float* eps, int64_t* Q, uint32_t* K);

/* Eq. 4, the full-image estimator (the baseline Sec. 6.1 compares against):
 * the same renders, but every parameter of a block with eps > 0 receives
 *   Q_i += s_i * sum over the image of round(delta_p * 2^32)
 * per (pair, view), and every group of such a block counts K_g += 1 per
 * (pair, view).  Arguments as for dr_estimate_grad. */
dr_status dr_estimate_grad_full(dr_ctx* ctx, const float* theta, const dr_view* views, int32_t n_views,
                                const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                                const float* eps, int64_t* Q, uint32_t* K);

/* The image form of dr_estimate_grad, for a loss computed downstream of the
 * render: grad_image (device, the views' [H,W,3] float images concatenated
 * in view order, like targets) holds dL/dI, and each pixel scatters
 *   delta_p = <g_p, I+_p - I-_p>   (channels r, g, b summed in that order)
 * in place of f+_p - f-_p, so that Eq. 8 estimates the vector-Jacobian
 * product of the render with g; with g = 2 (I - T) it equals the L2 form
 * wherever the colour is linear in the parameters.  Contribution sets,
 * Q, K, eps and errors are as for dr_estimate_grad. */
dr_status dr_estimate_grad_image(dr_ctx* ctx, const float* theta, const dr_view* views, int32_t n_views,
                                 const float* grad_image, uint64_t seed, uint32_t step, int32_t n_pairs,
                                 const float* eps, int64_t* Q, uint32_t* K);

/* dr_estimate_grad without any device allocation, for callers that cannot
 * allocate: code being captured into a HIP graph, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same arguments, results (bit for bit)
 * and errors as dr_estimate_grad, except that:
 *  - all scratch (sign bits, triangle records, bins, per-pair group sums,
 *    tessellated positions) comes from one static device array of
 *    DR_NOALLOC_SCRATCH_BYTES, which every GPU the library is loaded on
 *    holds until the process ends;
 *  - a call whose scratch would exceed that size (after lowering the
 *    items per raster launch as far as one) returns DR_E_INVALID and
 *    launches nothing; dr_last_error states the bytes it needed;
 *  - the bin capacity is the context's current one (no adaptive raise:
 *    an overflowing bin is exact but slower), and no timing events are
 *    recorded;
 *  - every call on one GPU shares that GPU's array: calls that overlap on
 *    one GPU (from several contexts or streams) race and give wrong
 *    results.  Calls ordered on one stream are safe; each call clears the
 *    part of the array that must start at zero.
 * The array's device address is looked up by dr_create on the context's
 * device; no call here allocates or frees memory. */
#define DR_NOALLOC_SCRATCH_BYTES (128ull << 20)
dr_status dr_estimate_grad_noalloc(dr_ctx* ctx, const float* theta, const dr_view* views, int32_t n_views,
                                   const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                                   const float* eps, int64_t* Q, uint32_t* K);

/* Decode Q, K into float gradients: g_i = Q_i 2^-32 / (2 eps_i D_i) with
 * D_i = K of the parameter's group (DR_AVG_COUNT) or n_pairs (DR_AVG_PAIRS,
 * Eq. 9); 0 where eps_i = 0 or D_i = 0.  grad [d] float. */
dr_status dr_decode_grad(dr_ctx* ctx, const int64_t* Q, const uint32_t* K, const float* eps,
                         int32_t averaging, int32_t n_pairs, float* grad);

/* The descent step (Sec. 5, shader D): decode as dr_decode_grad, then Adam
 * (bias-corrected with step t >= 1) or SGD on theta with per-block learning
 * rates; parameters with eps_i = 0, or (count averaging) with K = 0, are
 * not updated.  m, v [d] float are the Adam moments.  Q and K are zeroed. */
dr_status dr_step(dr_ctx* ctx, float* theta, float* m, float* v, uint32_t t, int64_t* Q, uint32_t* K,
                  const float* eps, int32_t n_pairs, const dr_optim* opt);

/* Per-kernel timing: while enabled, HIP events are recorded on the
 * context's stream around every launch of the estimator's kernels;
 * dr_timing_read synchronises the stream and returns the summed durations
 * (milliseconds) and launch counts since the last reset (reset != 0 clears
 * them after reading). */
typedef struct {
    double signs_ms, setup_ms, tile_ms, fold_ms, step_ms;
    int64_t signs_launches, setup_launches, tile_launches, fold_launches, step_launches;
} dr_timing_t;

dr_status dr_timing_enable(dr_ctx* ctx, int enable);
dr_status dr_timing_read(dr_ctx* ctx, dr_timing_t* out, int reset);

/* Device-side condition counters since the last reset (synchronises). */
dr_status dr_stats(dr_ctx* ctx, dr_stats_t* out);
dr_status dr_reset_stats(dr_ctx* ctx);

/* ---------------------------------------------------------------- batch
 * The batching form: one optimisation step of many independent scenes of
 * uneven size, each with n_pairs antithetic pairs over its views, run with
 * one launch per kernel -- one raster/shade/scatter launch covers every
 * (scene, pair, view, tile) unit, costliest scenes first -- followed by one
 * Adam/SGD launch over all scenes' parameters.  The step number lives on
 * the device and advances with each step, so the whole step can be captured
 * once as a HIP graph and replayed.  Scene b draws its signs with counter
 * word 3 = b (dr_set_scene_index), so each scene's Q and K are those of
 * dr_estimate_grad on that scene alone. */
typedef struct dr_batch dr_batch;

typedef struct {
    dr_ctx* ctx;                 /* the scene (topology, UVs, textures, shading)  */
    const dr_view* views;        /* host, copied; 1..16 views                     */
    int32_t n_views;
    const float* targets;        /* device: the views' [H,W,3] images, concatenated */
    float* theta, * m, * v;      /* device [d]: parameters and Adam moments       */
    int64_t* Q;                  /* device [d] and [G]: accumulators, zeroed by   */
    uint32_t* K;                 /*   each step                                   */
    float eps[1 + DR_MAX_TEX];   /* per block                                     */
    float lr[1 + DR_MAX_TEX];    /* per block                                     */
    int32_t bin_capacity;        /* 0: the context's tuning                       */
} dr_batch_scene;

/* Arrays passed in scenes[] must stay valid for the life of the batch.
 * tile_px: 8, 16 or 32 for every scene; first_step >= 1.  Scenes must be
 * opaque (layers == 0; DR_E_UNSUPPORTED otherwise). */
dr_status dr_batch_create(dr_batch** out, const dr_batch_scene* scenes, int32_t n_scenes, int32_t n_pairs,
                          int32_t tile_px, const dr_optim* opt, uint64_t seed, uint32_t first_step,
                          void* stream);
dr_status dr_batch_destroy(dr_batch* b);
/* Eq. 8 summed over every scene's pairs and views into its Q and K, at the
 * current step (the step counter does not advance). */
dr_status dr_batch_estimate(dr_batch* b);
/* One optimisation step of every scene (estimate, then descent), after
 * which the step counter advances.  use_graph != 0 captures the step as a
 * HIP graph on first use and replays it afterwards.  The step adds to its
 * estimate whatever Q holds when Q may be non-zero -- on the first step,
 * and after dr_batch_estimate (such a step runs without the graph) -- and
 * leaves Q zero; Q must not be written between steps otherwise. */
dr_status dr_batch_step(dr_batch* b, int use_graph);
dr_status dr_batch_set_step(dr_batch* b, uint32_t step);      /* synchronous; step >= 1 */
dr_status dr_batch_get_step(dr_batch* b, uint32_t* step);     /* synchronous */
dr_status dr_batch_stats(dr_batch* b, dr_stats_t* out);       /* synchronous */
/* Per-kernel timing of direct (not graph-replayed) launches, as dr_timing_*. */
dr_status dr_batch_timing_enable(dr_batch* b, int enable);
dr_status dr_batch_timing_read(dr_batch* b, dr_timing_t* out, int reset);
const char* dr_batch_last_error(const dr_batch* b);

/* ---------------------------------------------------------- measurement
 * Throughput probe of the device-scope atomic adds that the scatter's
 * flush issues (Alg. 2 accumulates with AtomicAdd; here each tile adds its
 * per-group sums with one 64-bit and one 32-bit agent-scope atomic per
 * group).  Launches n_ops atomic adds of 1 (width_bits 32 or 64, no value
 * returned) on the stream into the device buffer buf of `bytes` bytes
 * (8-byte aligned, caller-owned; its contents are changed), operation i
 * addressing element e(i) of the buffer, n = bytes / (width_bits / 8):
 *   DR_PROBE_CONTIGUOUS   e = i mod n (adjacent lanes, adjacent elements)
 *   DR_PROBE_LINES        e = (i * 128 / elem_bytes) mod n (one per 128 B line)
 *   DR_PROBE_SCATTERED    e = hash(i) mod n (unrelated lines, as a flush of
 *                         hashed groups)
 *   DR_PROBE_CONFLICTING  e = (i / 64) mod n (a wave's 64 lanes on one element)
 * Asynchronous; DR_E_INVALID for a bad argument (nothing launched). */
enum { DR_PROBE_CONTIGUOUS = 0, DR_PROBE_LINES = 1, DR_PROBE_SCATTERED = 2, DR_PROBE_CONFLICTING = 3 };
dr_status dr_probe_atomics(void* buf, int64_t bytes, int32_t width_bits, int32_t pattern, int64_t n_ops,
                           void* stream);

/* Self-check of the shading's short correctly rounded sequences: for every
 * float whose bit pattern lies in [lo, hi] (lo <= hi), the library's fast
 * square root (op DR_PROBE_SQRT, valid for [2^-96, 2^126]) or reciprocal
 * (DR_PROBE_RCP, valid for magnitudes in [2^-125, 2^125]) against the
 * compiler's correctly rounded sqrtf or 1.0f / x.  Adds the number of
 * operands where they differ to *bad and lowers *first to the least such
 * bit pattern (device pointers; the caller sets them to 0 and 0xFFFFFFFF).
 * Asynchronous on the stream. */
enum { DR_PROBE_SQRT = 0, DR_PROBE_RCP = 1 };
dr_status dr_probe_math(int32_t op, uint32_t lo, uint32_t hi, uint64_t* bad, uint32_t* first, void* stream);

const char* dr_status_str(dr_status s);
const char* dr_last_error(const dr_ctx* ctx);     /* "" when none; ctx may be NULL */

#ifdef __cplusplus
}
#endif
#endif
