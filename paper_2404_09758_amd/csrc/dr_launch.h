// dr_launch.h -- argument blocks and launchers of the estimator kernels
// (shared by the kernels and the host side of the C ABI).
#pragma once

#include "dr_device.h"

// Device counters (uint64 each).
#define ST_OVERFLOWS 0
#define ST_SATURATIONS 1
#define ST_NONFINITE 2
#define ST_BAD_INDEX 3
#define ST_MAX_BIN 4
#define ST_FULL_SCANS 5       // overflowing (tile, render) bins whose render's spill list was full
#define ST_COUNT 8

// Spill list of one render: entries (tile << 32 | triangle) of bins past
// their capacity, and two counters: [0] entries appended, [1] overflowing
// tiles not yet rasterised.  The last of those tiles empties the list.
#define SPILL_CAP 8192

// ------------------------------------------------------- single scene --

struct SetupArgs {
    DScene sc;
    DViews views;
    DPert pert;
    const float* theta;
    int n_views;            // views per pair (item -> pair = item / n_views)
    int item0;              // first item of this launch
    int nsign;              // 1 (render, loss) or 2 (+ and -)
    float sgn[2];
    int tile;               // tile size in pixels
    int cap;                // bin capacity
    int max_tiles;          // tile slots per (item, sign)
    TriR* recR;
    TriS* recS;
    unsigned* counts;
    unsigned* bins;
    unsigned* spn;                   // [slots, 2] spill counters, or null (no spill lists)
    unsigned long long* spill;       // [slots, SPILL_CAP]
    const float* fpos;      // subdivision surface: [pairs, nsign, n_verts, 3] positions, else null
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
    unsigned* spn;
    const unsigned long long* spill;
    unsigned long long* stats;
    // estimate mode
    const float* targets;            // target images, or dL/dI in the image form
    int img_grad;                    // image form: scatter <dL/dI, I+ - I->
    long long* R;                    // [pairs, G] per-pair group sums
    unsigned* K;                     // [G]
    int act_pos;                     // scatter vertex groups
    int act_cls[DRD_MAX_TEX];        // scatter texel groups of each class
    int any_act;                     // any group is scattered
    // loss mode: per (item, tile) partial sums
    double* partials;
    // full-image mode: per pair totals of the fixed-point differences
    long long* qtot;
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
    // full-image estimate
    const long long* qtot;       // [pairs]
    unsigned* K;
    int n_views;
};

struct OptimConst {
    int kind, averaging;
    float b1, omb1, b2, omb2, eps_hat;
};

struct StepArgs {
    DScene sc;
    float eps[1 + DRD_MAX_TEX];
    float lr[1 + DRD_MAX_TEX];
    int n_pairs, decode_only;
    OptimConst oc;
    float bc1, bc2;
    float* theta;
    float* m;
    float* v;
    long long* Q;
    unsigned* K;
    float* grad;                 // decode-only output
    unsigned long long* stats;
};

// ------------------------------------------------------------- batch --
//
// A batch runs one optimisation step of many independent scenes with one
// launch per kernel: one raster/scatter launch covers every (scene, pair,
// view) item's tiles.  All descriptors live in device memory and are fixed
// when the batch is created; the step number is read from a device counter,
// so the step can be captured once as a graph and replayed.

struct BScene {
    DScene sc;
    const float* theta;          // caller [d]
    float* m;
    float* v;
    long long* Q;                // caller [d]
    unsigned* K;                 // caller [G]
    uint32_t* bits;              // scratch [pairs, words]
    long long* R;                // scratch [pairs, G]
    const float* targets;        // caller: the scene's views, concatenated
    float eps[1 + DRD_MAX_TEX];
    float lr[1 + DRD_MAX_TEX];
    int act_pos, any_act;
    int act_cls[DRD_MAX_TEX];
    int n_views, view0;          // views [view0, view0 + n_views) of the view table
    int scene_index;             // counter word 3 of the signs
    long long sign_blk0;         // first block of this scene in the signs launch
    long long group_blk0;        // first block of this scene in the fold / step launches
};

struct BItem {
    int scene, pair, view;       // view: index in the batch view table
    int cap;                     // bin capacity
    long long rec_off;           // records of sign 0 (sign 1 at + n_tris)
    long long cnt_off;           // bin counters of sign 0 (sign 1 at + tiles)
    long long bin_off;           // bin entries of sign 0 (sign 1 at + tiles * cap)
    long long sp_off;            // spill list of sign 0 (sign 1 at + 1)
    long long setup_blk0;        // first block of this item in the setup launch
    long long tile0;             // first tile unit of this item in the tile launch
};

struct BatchArgs {
    const BScene* scenes;
    int n_scenes;
    const DView* views;
    const BItem* items;
    int n_items;
    int n_pairs;
    unsigned long long seed;
    const unsigned* step;        // device step counter (1-based)
    long long sign_blocks, setup_blocks, group_blocks, total_tiles;
    TriR* recR;
    TriS* recS;
    unsigned* counts;
    unsigned* bins;
    unsigned* spn;               // [2 items, 2] spill counters
    unsigned long long* spill;   // [2 items, SPILL_CAP]
    unsigned long long* stats;
    OptimConst oc;
    const float* bc1;            // Adam bias corrections by step, [n_bc]
    const float* bc2;
    int n_bc;
    int tile;
    int q_zero;                  // every scene's Q is known to be zero (the fused step skips reading it)
    long long unit0;             // setup and tile launches: the first block / tile unit of the launch
};

hipError_t launch_signs(hipStream_t st, unsigned long long seed, unsigned step, unsigned pair0, unsigned scene,
                        long long d, int words, int n_pairs, uint32_t* bits);
hipError_t launch_setup(hipStream_t st, const SetupArgs& a, int n_items);
hipError_t launch_subdiv(hipStream_t st, const DScene& sc, const DPert& pert, const float* theta, int n_pairs,
                         int nsign, float sgn0, float sgn1, float* fpos);
hipError_t launch_tile(hipStream_t st, const TileArgs& a, int tile, int mode, int n_items, int max_tiles);
hipError_t launch_sum_tiles(hipStream_t st, const double* partials, int max_tiles, const DViews& views,
                            int n_views, double* out);
hipError_t launch_check_tri(hipStream_t st, const int* tri, long long n, int n_verts, unsigned long long* bad);
hipError_t launch_fold(hipStream_t st, const FoldArgs& a);
hipError_t launch_broadcast(hipStream_t st, const FoldArgs& a);
hipError_t launch_zero64(hipStream_t st, long long* p, int n);
hipError_t launch_step(hipStream_t st, const StepArgs& a);

hipError_t launch_batch_signs(hipStream_t st, const BatchArgs& b);
// setup blocks [blk0, blk0 + nblk) of the batch's setup grid
struct BatchOne;
// setup blocks [blk0, blk0 + nblk); one: the batch's scene when it has one
hipError_t launch_batch_setup(hipStream_t st, const BatchArgs& b, const BatchOne* one, long long blk0,
                              long long nblk);
// A one-scene batch's scene constants and views, passed to the tile launch
// by value.
struct BatchOne {
    DScene sc;
    DView views[DRD_MAX_VIEWS];
    int n_views;
    // Tile units in pair-interleaved order: the launch walks (view, tile,
    // pair) while the units are numbered (pair, view, tile); tsum[v] is the
    // number of tiles of views 0 .. v-1.  il_pairs = 1 keeps unit order.
    int il_pairs;
    long long tsum[DRD_MAX_VIEWS + 1];
};

// one: non-null for a one-scene batch (the batch's view table is then the
// scene's views).
// tile units [w0, w0 + n) of the batch
hipError_t launch_batch_tile(hipStream_t st, const BatchArgs& b, const BatchOne* one, long long w0, long long n);
hipError_t launch_batch_fold(hipStream_t st, const BatchArgs& b);
hipError_t launch_batch_step(hipStream_t st, const BatchArgs& b);
// fold and step in one launch (at most 8 pairs)
hipError_t launch_batch_fold_step(hipStream_t st, const BatchArgs& b);
hipError_t launch_batch_end(hipStream_t st, const BatchArgs& b);
