// dr_launch.h -- argument blocks and launchers of the estimator kernels
// (shared by the kernels and the host side of the C ABI).
#pragma once

#include "dr_device.h"

struct SetupArgs {
    DScene sc;
    DViews views;
    DPert pert;
    const float* theta;
    int n_views;            // views per pair (item -> pair = item / n_views)
    int item0;              // first item of this launch
    int nsign;              // 1 (render) or 2 (+ and -)
    float sgn[2];
    int tile;               // tile size in pixels
    int cap;                // bin capacity
    int max_tiles;          // tile slots per (item, sign)
    TriR* recR;
    TriS* recS;
    unsigned* counts;
    unsigned* bins;
};

struct TileArgs {
    DScene sc;
    DViews views;
    DPert pert;
    const float* theta;
    int n_views;
    int item0;
    int nsign;
    float sgn[2];
    int cap;
    int max_tiles;
    const TriR* recR;
    const TriS* recS;
    unsigned* counts;
    const unsigned* bins;
    unsigned long long* stats;       // [3]: overflows, saturations, nonfinite
    // estimate mode
    const float* targets;
    long long* R;                    // [pairs, G] per-pair group sums
    unsigned* K;                     // [G]
    int act_pos;                     // scatter vertex groups
    int act_cls[DRD_MAX_TEX];        // scatter texel groups of each class
    int any_act;                     // any group is scattered
    // loss mode: per (item, tile) partial sums
    double* partials;
    // render mode
    float* out_rgb;
    unsigned* out_id;
    float* out_uv;
};

struct FoldArgs {
    DScene sc;
    long long* R;                // [pairs, G], zeroed on the way out
    const uint32_t* bits;        // [pairs, words]
    int n_pairs;
    float eps[1 + DRD_MAX_TEX];
    long long* Q;
};

struct StepArgs {
    DScene sc;
    float eps[1 + DRD_MAX_TEX];
    float lr[1 + DRD_MAX_TEX];
    int averaging, n_pairs, kind, decode_only;
    float b1, omb1, b2, omb2, bc1, bc2, eps_hat;
    float* theta;
    float* m;
    float* v;
    long long* Q;
    unsigned* K;
    float* grad;                 // decode-only output
    unsigned long long* stats;
};

hipError_t launch_signs(hipStream_t st, unsigned long long seed, unsigned step, unsigned pair0, unsigned scene,
                        long long d, int words, int n_pairs, uint32_t* bits);
hipError_t launch_setup(hipStream_t st, const SetupArgs& a, int n_items);
hipError_t launch_tile(hipStream_t st, const TileArgs& a, int tile, int mode, int n_items, int max_tiles);
hipError_t launch_sum_tiles(hipStream_t st, const double* partials, int max_tiles, const DViews& views,
                            int n_views, double* out);
hipError_t launch_check_tri(hipStream_t st, const int* tri, long long n, int n_verts, unsigned long long* bad);
hipError_t launch_fold(hipStream_t st, const FoldArgs& a);
hipError_t launch_step(hipStream_t st, const StepArgs& a);
