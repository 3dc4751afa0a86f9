// dr_kernels.hip -- HIP kernels of the per-pixel stochastic gradient
// estimator for gfx950 (MI355X).
//
// Pipeline of one estimate (Sec. 4.3, Alg. 1 and 2, Eq. 8-9):
//   k_signs      Philox sign bits of every pair             (shader P)
//   k_setup_bin  per (item, sign, triangle): perturb the three vertices,
//                project, snap, build the raster record and append the
//                triangle to the bins of the tiles its bbox touches
//   k_tile       per (item, tile): rasterise the + and - scenes into LDS
//                depth|id keys (64-bit atomic min), shade both winners,
//                form the per-pixel loss difference and scatter it to the
//                union of the pixel's contribution groups    (R and G fused)
//   k_fold       Q_i += sum_n s_i^(n) R^(n)_g(i): the per-group sums of
//                each pair become per-parameter fixed-point sums
//   k_step       decode, per-parameter average, Adam / SGD   (shader D)
// An "item" is one (pair, view).  Triangle records, bins and the per-pair
// group sums R live in context scratch memory.
#include "dr_launch.h"

// ------------------------------------------------------------ k_signs --

__global__ void k_signs(unsigned long long seed, unsigned step, unsigned pair0, unsigned scene,
                        long long d, int words, uint32_t* __restrict__ bits) {
    long long blk = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int p = blockIdx.y;
    long long nblk = (d + 255) >> 8;
    if (blk >= nblk) return;
    unsigned long long r[4];
    philox4x64_10((unsigned long long)blk, (unsigned long long)(pair0 + p), step, scene, seed, 0ull, r);
    uint32_t* out = bits + (long long)p * words;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        long long word = blk * 8 + w;
        if (word < words) out[word] = (w & 1) ? (uint32_t)(r[w >> 1] >> 32) : (uint32_t)r[w >> 1];
    }
}

// -------------------------------------------------------- k_setup_bin --

__global__ void __launch_bounds__(256) k_setup_bin(SetupArgs a) {
    const DScene& sc = a.sc;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= sc.n_tris) return;
    int slot = blockIdx.y;                       // (local item, sign)
    int li = slot / a.nsign, s = slot % a.nsign;
    int item = a.item0 + li;
    int pair = item / a.n_views, view = item % a.n_views;
    const DView& vw = a.views.v[view];
    const uint32_t* pb = a.pert.bits ? a.pert.bits + (long long)pair * sc.words : nullptr;
    float sgn = a.sgn[s];
    float e0 = a.pert.eps[0];

    int vid[3];
    float p[9];
    Vtx v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        vid[k] = sc.tri[3 * (long long)t + k];
        long long base = 3 * (long long)vid[k];
        p[3 * k + 0] = pval(a.theta, base + 0, e0, pb, sgn);
        p[3 * k + 1] = pval(a.theta, base + 1, e0, pb, sgn);
        p[3 * k + 2] = pval(a.theta, base + 2, e0, pb, sgn);
        v[k] = xform(vw, p[3 * k + 0], p[3 * k + 1], p[3 * k + 2]);
    }
    TriR r;
    TriS sh;
    r.flags = 0u;
    r.pad[0] = 0; r.pad[1] = 0;
    long long rec = (long long)slot * sc.n_tris + t;
    bool ok = v[0].valid && v[1].valid && v[2].valid;
    long long area2 = 0;
    if (ok) {
        area2 = (long long)(v[1].X - v[0].X) * (long long)(v[2].Y - v[0].Y) -
                (long long)(v[1].Y - v[0].Y) * (long long)(v[2].X - v[0].X);
        ok = area2 != 0;
    }
    if (!ok) {
        r.flags = 0u;
        a.recR[rec] = r;
        return;
    }
    bool sw = area2 < 0;
    if (sw) {
        area2 = -area2;
        Vtx tmp = v[1]; v[1] = v[2]; v[2] = tmp;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { r.X[k] = v[k].X; r.Y[k] = v[k].Y; sh.iw[k] = v[k].iw; }
    r.area2 = area2;
    unsigned fl = TRI_VALID | (sw ? TRI_SWAPPED : 0u);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int ia = (k + 1) % 3, ib = (k + 2) % 3;
        int dx = r.X[ib] - r.X[ia], dy = r.Y[ib] - r.Y[ia];
        if ((dy < 0) || (dy == 0 && dx > 0)) fl |= (2u << k);
    }
    r.flags = fl;
    float d1 = v[1].z - v[0].z, d2 = v[2].z - v[0].z;
    float fX1 = (float)(r.X[1] - r.X[0]), fY1 = (float)(r.Y[1] - r.Y[0]);
    float fX2 = (float)(r.X[2] - r.X[0]), fY2 = (float)(r.Y[2] - r.Y[0]);
    float fa = (float)area2;
    r.z0 = v[0].z;
    r.zx = (d1 * fY2 - d2 * fY1) / fa;
    r.zy = (d2 * fX1 - d1 * fX2) / fa;
    int xmin = min(r.X[0], min(r.X[1], r.X[2])), xmax = max(r.X[0], max(r.X[1], r.X[2]));
    int ymin = min(r.Y[0], min(r.Y[1], r.Y[2])), ymax = max(r.Y[0], max(r.Y[1], r.Y[2]));
    // pixels whose centre 256 x + 128 lies in [min, max]
    int bx0 = max((xmin + 127) >> 8, 0), bx1 = min((xmax - 128) >> 8, vw.W - 1);
    int by0 = max((ymin + 127) >> 8, 0), by1 = min((ymax - 128) >> 8, vw.H - 1);
    if (bx0 > bx1 || by0 > by1) {               // no pixel centre in the bbox
        bx0 = 1; bx1 = 0; by0 = 1; by1 = 0;
    }
    r.bx0 = (short)bx0; r.bx1 = (short)bx1; r.by0 = (short)by0; r.by1 = (short)by1;
#pragma unroll
    for (int k = 0; k < 9; ++k) sh.p[k] = p[k];
    sh.vid[0] = vid[0]; sh.vid[1] = vid[1]; sh.vid[2] = vid[2];
    sh.pad = 0;
    a.recR[rec] = r;
    a.recS[rec] = sh;
    if (bx0 > bx1) return;
    int tx0 = bx0 / a.tile, tx1 = bx1 / a.tile, ty0 = by0 / a.tile, ty1 = by1 / a.tile;
    long long tbase = (long long)slot * a.max_tiles;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            long long tile = tbase + ty * vw.tiles_x + tx;
            unsigned k = atomicAdd(&a.counts[tile], 1u);
            if (k < (unsigned)a.cap) a.bins[tile * a.cap + k] = (unsigned)t;
        }
}

// ------------------------------------------------------------- k_tile --

// Map consecutive workgroups (which the dispatcher spreads round-robin over
// the 8 XCDs) to contiguous runs of tiles per XCD, so neighbouring tiles --
// sharing triangles, texels and accumulators -- meet in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    int x = bid & 7, k = bid >> 3;
    int q = nb >> 3, rem = nb & 7;
    return x * q + min(x, rem) + k;
}

template <int TILE>
__device__ __forceinline__ void raster_tri(const TriR& r, unsigned t, int px0, int py0, int lane,
                                           unsigned long long* key) {
    int x0 = max((int)r.bx0, px0), x1 = min((int)r.bx1, px0 + TILE - 1);
    int y0 = max((int)r.by0, py0), y1 = min((int)r.by1, py0 + TILE - 1);
    if (x0 > x1 || y0 > y1) return;
    int bw = x1 - x0 + 1;
    int n = bw * (y1 - y0 + 1);
    unsigned m = ((1u << 20) + (unsigned)bw - 1u) / (unsigned)bw;     // exact for bw <= 32, idx < 1024
    for (int base = 0; base < n; base += 64) {
        int idx = base + lane;
        if (idx < n) {
            int dy = (int)(((unsigned)idx * m) >> 20);
            int dx = idx - dy * bw;
            int x = x0 + dx, y = y0 + dy;
            int px = 256 * x + 128, py = 256 * y + 128;
            long long e0, e1, e2;
            if (inside(r, px, py, e0, e1, e2)) {
                float z = depth_at(r, px, py);
                unsigned long long k = ((unsigned long long)__float_as_uint(z) << 32) | t;
                atomicMin(&key[(y - py0) * TILE + (x - px0)], k);
            }
        }
    }
}

// ------------------------------------------------ tile-local aggregation --
//
// Contributions are summed per group inside the workgroup before they reach
// the global accumulators: an open-addressing table in LDS keyed by group
// (int64 sum + uint32 count per slot), flushed with one global atomic pair
// per distinct group of the tile.  Integer sums make the result identical
// to per-pixel global atomics.

#define HASH_EMPTY 0xFFFFFFFFu
#define HASH_PROBES 64

template <int LOG2T>
struct GroupTable {
    unsigned key[1 << LOG2T];
    unsigned long long sum[1 << LOG2T];
    unsigned cnt[1 << LOG2T];
};

__device__ __forceinline__ void global_add(long long* __restrict__ Rp, unsigned* __restrict__ K, long long g,
                                           long long q, unsigned c) {
    if (q != 0) atomicAdd((unsigned long long*)&Rp[g], (unsigned long long)q);
    atomicAdd(&K[g], c);
}

template <int LOG2T>
__device__ __forceinline__ void table_add(GroupTable<LOG2T>& tb, long long* __restrict__ Rp,
                                          unsigned* __restrict__ K, unsigned g, long long q, unsigned c) {
    constexpr unsigned MASK = (1u << LOG2T) - 1u;
    unsigned h = (g * 2654435761u) >> (32 - LOG2T);
    for (int probe = 0; probe < HASH_PROBES; ++probe) {
        unsigned k = __hip_atomic_load(&tb.key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == HASH_EMPTY) k = atomicCAS(&tb.key[h], HASH_EMPTY, g);
        if (k == HASH_EMPTY || k == g) {
            if (q != 0) atomicAdd(&tb.sum[h], (unsigned long long)q);
            atomicAdd(&tb.cnt[h], c);
            return;
        }
        h = (h + 1u) & MASK;
    }
    global_add(Rp, K, g, q, c);      // crowded table: go straight to memory
}

// Wave-level combine of the vertex contributions of pixels whose + and -
// renders show the same triangle: lanes with equal triangle ids are summed
// with a butterfly and one lane adds the three vertices.  Must be called by
// every lane of the wave.
template <int LOG2T>
__device__ __forceinline__ void wave_vertices(GroupTable<LOG2T>& tb, long long* __restrict__ Rp,
                                              unsigned* __restrict__ K, bool active, unsigned tri,
                                              int v0, int v1, int v2, long long q) {
    int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(active);
    while (pending) {
        int leader = __ffsll((unsigned long long)pending) - 1;
        unsigned lt = __shfl(tri, leader);
        bool mine = active && tri == lt;
        unsigned long long m = __ballot(mine);
        long long v = mine ? q : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == leader) {
            unsigned c = (unsigned)__popcll(m);
            table_add<LOG2T>(tb, Rp, K, (unsigned)v0, v, c);
            table_add<LOG2T>(tb, Rp, K, (unsigned)v1, v, c);
            table_add<LOG2T>(tb, Rp, K, (unsigned)v2, v, c);
        }
        if (mine) active = false;
        pending &= ~m;
    }
}

template <int TILE>
struct TileCfg {
    static constexpr int LOG2T = TILE == 8 ? 9 : (TILE == 16 ? 10 : 11);
};

// MODE: 0 estimate (both signs, scatter), 1 render (write rgb/id/uv),
// 2 loss (per-tile sum of the per-pixel L2 error f_{w,h}).
template <int TILE, int MODE>
__global__ void __launch_bounds__((TILE * TILE > 256) ? 256 : TILE * TILE) k_tile(TileArgs a) {
    constexpr bool RENDER = MODE != 0;
    constexpr int NPIX = TILE * TILE;
    constexpr int PPT = NPIX > 256 ? NPIX / 256 : 1;
    constexpr int TB = NPIX / PPT;
    constexpr int NW = TB / 64;
    constexpr int NS = RENDER ? 1 : 2;
    constexpr int LOG2T = TileCfg<TILE>::LOG2T;
    constexpr int TSIZE = 1 << LOG2T;
    __shared__ unsigned long long key[NS][NPIX];

    const DScene& sc = a.sc;
    int li = blockIdx.y;
    int item = a.item0 + li;
    int pair = item / a.n_views, view = item % a.n_views;
    const DView& vw = a.views.v[view];
    int ntiles = vw.tiles_x * vw.tiles_y;
    int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    int tx = tile % vw.tiles_x, ty = tile / vw.tiles_x;
    int px0 = tx * TILE, py0 = ty * TILE;
    int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    for (int j = tid; j < NS * NPIX; j += TB) (&key[0][0])[j] = ~0ull;
    __shared__ GroupTable<RENDER ? 1 : LOG2T> table;
    if constexpr (!RENDER) {
        for (int j = tid; j < TSIZE; j += TB) {
            table.key[j] = HASH_EMPTY;
            table.sum[j] = 0ull;
            table.cnt[j] = 0u;
        }
    }
    __syncthreads();

    unsigned cnt[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int slot = li * NS + s;
        long long tslot = (long long)slot * a.max_tiles + tile;
        cnt[s] = a.counts[tslot];
        const TriR* __restrict__ R = a.recR + (long long)slot * sc.n_tris;
        if (cnt[s] <= (unsigned)a.cap) {
            const unsigned* __restrict__ list = a.bins + tslot * a.cap;
            for (unsigned k = wave; k < cnt[s]; k += NW) {
                unsigned t = __builtin_amdgcn_readfirstlane(list[k]);
                TriR r = R[t];
                raster_tri<TILE>(r, t, px0, py0, lane, key[s]);
            }
        } else {
            // bin overflow: test every triangle against this tile
            for (int t = wave; t < sc.n_tris; t += NW) {
                TriR r = R[t];
                if (!(r.flags & TRI_VALID)) continue;
                raster_tri<TILE>(r, (unsigned)t, px0, py0, lane, key[s]);
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            long long tslot = (long long)(li * NS + s) * a.max_tiles + tile;
            a.counts[tslot] = 0u;                // leave the bin empty for the next use
            if (cnt[s] > (unsigned)a.cap) atomicAdd(&a.stats[0], 1ull);
        }
    }

    const uint32_t* pb = a.pert.bits ? a.pert.bits + (long long)pair * sc.words : nullptr;
    long long* Rp = RENDER ? nullptr : a.R + (long long)pair * sc.G;
    double loss_acc = 0.0;
    for (int j = 0; j < PPT; ++j) {
        int local = tid + j * TB;
        int lx = local % TILE, ly = local / TILE;
        int x = px0 + lx, y = py0 + ly;
        bool inpix = x < vw.W && y < vw.H;
        int px = 256 * x + 128, py = 256 * y + 128;
        unsigned id[NS];
        float rgb[NS][3], uv[NS][2];
        int vids[NS][3];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            unsigned long long k = inpix ? key[s][local] : ~0ull;
            id[s] = (k == ~0ull) ? DRD_BG : (unsigned)(k & 0xFFFFFFFFull);
            rgb[s][0] = 0.0f; rgb[s][1] = 0.0f; rgb[s][2] = 0.0f;
            uv[s][0] = 0.0f; uv[s][1] = 0.0f;
            vids[s][0] = vids[s][1] = vids[s][2] = -1;
            if (id[s] != DRD_BG) {
                long long rec = (long long)(li * NS + s) * sc.n_tris + id[s];
                TriR r = a.recR[rec];
                TriS sh = a.recS[rec];
                shade_pixel(sc, vw, a.theta, pb, a.pert.eps, a.sgn[s], r, sh, (int)id[s], px, py, rgb[s], uv[s]);
                vids[s][0] = sh.vid[0]; vids[s][1] = sh.vid[1]; vids[s][2] = sh.vid[2];
            }
        }
        long long pix = (long long)y * vw.W + x;
        if constexpr (MODE == 2) {
            if (inpix) {
                const float* tg = a.targets + vw.tgt_off + 3 * pix;
                float dr = rgb[0][0] - tg[0], dg = rgb[0][1] - tg[1], db = rgb[0][2] - tg[2];
                loss_acc += (double)((dr * dr + dg * dg) + db * db);
            }
        } else if constexpr (MODE == 1) {
            if (!inpix) continue;
            if (a.out_rgb) {
                a.out_rgb[3 * pix + 0] = rgb[0][0];
                a.out_rgb[3 * pix + 1] = rgb[0][1];
                a.out_rgb[3 * pix + 2] = rgb[0][2];
            }
            if (a.out_id) a.out_id[pix] = id[0];
            if (a.out_uv) {
                a.out_uv[2 * pix + 0] = uv[0][0];
                a.out_uv[2 * pix + 1] = uv[0][1];
            }
        } else {
            // an empty contribution set (background in both renders) adds nothing
            bool act = inpix && (id[0] != DRD_BG || id[1] != DRD_BG) && a.any_act;
            long long q = 0;
            if (act) {
                const float* tg = a.targets + vw.tgt_off + 3 * pix;
                float t0 = tg[0], t1 = tg[1], t2 = tg[2];
                float dr0 = rgb[0][0] - t0, dg0 = rgb[0][1] - t1, db0 = rgb[0][2] - t2;
                float dr1 = rgb[1][0] - t0, dg1 = rgb[1][1] - t1, db1 = rgb[1][2] - t2;
                float fp = (dr0 * dr0 + dg0 * dg0) + db0 * db0;
                float fm = (dr1 * dr1 + dg1 * dg1) + db1 * db1;
                int flag;
                q = quantize(fp - fm, flag);
                if (flag) atomicAdd(&a.stats[flag], 1ull);
            }
            if (a.act_pos) {
                // same triangle in both renders: combined per wave
                bool same = act && id[0] == id[1];
                wave_vertices<LOG2T>(table, Rp, a.K, same, id[0], vids[0][0], vids[0][1], vids[0][2], q);
                if (act && !same) {
                    // the union of the two triangles' vertices, each once
                    if (id[0] != DRD_BG) {
#pragma unroll
                        for (int k = 0; k < 3; ++k) table_add<LOG2T>(table, Rp, a.K, (unsigned)vids[0][k], q, 1u);
                    }
                    if (id[1] != DRD_BG) {
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            int g = vids[1][k];
                            bool dup = (g == vids[0][0]) || (g == vids[0][1]) || (g == vids[0][2]);
                            if (!dup) table_add<LOG2T>(table, Rp, a.K, (unsigned)g, q, 1u);
                        }
                    }
                }
            }
            if (act) {
                for (int c = 0; c < sc.n_cls; ++c) {
                    if (!a.act_cls[c]) continue;
                    int W = sc.cls_w[c], H = sc.cls_h[c];
                    long long base = sc.cls_goff[c];
                    long long gs[NS][4];
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        gs[s][0] = gs[s][1] = gs[s][2] = gs[s][3] = -1;
                        if (id[s] == DRD_BG) continue;
                        Foot f = footprint(uv[s][0], uv[s][1], W, H);
                        if (sc.tex_mode == 1) {
                            int xn = (f.fx >= 0.5f) ? f.xb : f.xa;
                            int yn = (f.fy >= 0.5f) ? f.yb : f.ya;
                            gs[s][0] = base + (long long)yn * W + xn;
                        } else {
                            gs[s][0] = base + (long long)f.ya * W + f.xa;
                            gs[s][1] = base + (long long)f.ya * W + f.xb;
                            gs[s][2] = base + (long long)f.yb * W + f.xa;
                            gs[s][3] = base + (long long)f.yb * W + f.xb;
                        }
                    }
#pragma unroll
                    for (int s = 0; s < NS; ++s)
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            long long g = gs[s][k];
                            if (g < 0) continue;
                            bool dup = false;
#pragma unroll
                            for (int j2 = 0; j2 < 4; ++j2)
                                if (j2 < k && gs[s][j2] == g) dup = true;
                            if (s == 1) {
#pragma unroll
                                for (int j2 = 0; j2 < 4; ++j2)
                                    if (gs[0][j2] == g) dup = true;
                            }
                            if (!dup) table_add<LOG2T>(table, Rp, a.K, (unsigned)g, q, 1u);
                        }
                }
            }
        }
    }
    if constexpr (MODE == 2) {
        // fixed-order tree reduction of the tile's per-pixel errors
        __shared__ double red[TB];
        red[tid] = loss_acc;
        __syncthreads();
        for (int w = TB / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] = red[tid] + red[tid + w];
            __syncthreads();
        }
        if (tid == 0) a.partials[(long long)li * a.max_tiles + tile] = red[0];
    }
    if constexpr (!RENDER) {
        __syncthreads();
        for (int j = tid; j < TSIZE; j += TB) {
            unsigned g = table.key[j];
            if (g != HASH_EMPTY) global_add(Rp, a.K, (long long)g, (long long)table.sum[j], table.cnt[j]);
        }
    }
}

template __global__ void k_tile<8, 0>(TileArgs);
template __global__ void k_tile<16, 0>(TileArgs);
template __global__ void k_tile<32, 0>(TileArgs);
template __global__ void k_tile<8, 1>(TileArgs);
template __global__ void k_tile<16, 1>(TileArgs);
template __global__ void k_tile<32, 1>(TileArgs);
template __global__ void k_tile<8, 2>(TileArgs);
template __global__ void k_tile<16, 2>(TileArgs);
template __global__ void k_tile<32, 2>(TileArgs);

// Per-view loss: the tiles' partial sums added in tile order (one block per
// view, fixed-order reduction), so the value is reproducible run to run.
__global__ void __launch_bounds__(256) k_sum_tiles(const double* __restrict__ partials, int max_tiles,
                                                   DViews views, double* __restrict__ out) {
    __shared__ double red[256];
    int v = blockIdx.x, tid = threadIdx.x;
    int n = views.v[v].tiles_x * views.v[v].tiles_y;
    double acc = 0.0;
    for (int t = tid; t < n; t += 256) acc += partials[(long long)v * max_tiles + t];
    red[tid] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] = red[tid] + red[tid + w];
        __syncthreads();
    }
    if (tid == 0) out[v] = red[0];
}

// ------------------------------------------------------------- k_fold --

// Parameters of group g: a vertex's x, y, z, or a texel's channels in
// every texture of its class.  Calls fn(param index, block).
template <typename Fn>
__device__ __forceinline__ void for_params(const DScene& sc, long long g, Fn fn) {
    if (g < sc.n_verts) {
        fn(3 * g + 0, 0);
        fn(3 * g + 1, 0);
        fn(3 * g + 2, 0);
        return;
    }
    for (int c = 0; c < sc.n_cls; ++c) {
        long long size = (long long)sc.cls_w[c] * sc.cls_h[c];
        long long texel = g - sc.cls_goff[c];
        if (texel < 0 || texel >= size) continue;
        for (int t = 0; t < sc.n_tex; ++t) {
            if (sc.tex_cls[t] != c) continue;
            int C = sc.tex_c[t];
            for (int ch = 0; ch < C; ++ch) fn(sc.tex_off[t] + texel * C + ch, 1 + t);
        }
    }
}

__global__ void __launch_bounds__(256) k_fold(FoldArgs a) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const DScene& sc = a.sc;
    if (g >= sc.G) return;
    for_params(sc, g, [&](long long i, int b) {
        if (a.eps[b] == 0.0f) return;
        long long acc = 0;
        for (int n = 0; n < a.n_pairs; ++n) {
            long long r = a.R[(long long)n * sc.G + g];
            acc += (sign_of(a.bits + (long long)n * sc.words, i) > 0) ? r : -r;
        }
        if (acc != 0) a.Q[i] += acc;
    });
    for (int n = 0; n < a.n_pairs; ++n) a.R[(long long)n * sc.G + g] = 0;
}

// ----------------------------------------------------- k_step / decode --

__global__ void __launch_bounds__(256) k_step(StepArgs a) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const DScene& sc = a.sc;
    if (g >= sc.G) return;
    unsigned kc = a.K[g];
    double D = (a.averaging == 0) ? (double)kc : (double)a.n_pairs;
    for_params(sc, g, [&](long long i, int b) {
        float e = a.eps[b];
        long long qv = a.Q[i];
        float gi = 0.0f;
        if (e != 0.0f && D != 0.0)
            gi = (float)(((double)qv * (1.0 / 4294967296.0)) / (2.0 * (double)e * D));
        if (a.decode_only) {
            a.grad[i] = gi;
            return;
        }
        a.Q[i] = 0;
        if (e == 0.0f) return;
        if (a.averaging == 0 && kc == 0u) return;
        if (!(fabsf(gi) <= 3.402823466e38f)) {
            atomicAdd(&a.stats[2], 1ull);
            return;
        }
        float lr = a.lr[b];
        if (a.kind == 1) {
            a.theta[i] = a.theta[i] - lr * gi;
        } else {
            float mi = a.b1 * a.m[i] + a.omb1 * gi;
            float vi = a.b2 * a.v[i] + a.omb2 * (gi * gi);
            a.m[i] = mi;
            a.v[i] = vi;
            float mh = mi / a.bc1;
            float vh = vi / a.bc2;
            a.theta[i] = a.theta[i] - lr * (mh / (sqrtf(vh) + a.eps_hat));
        }
    });
    if (!a.decode_only) a.K[g] = 0u;
}

// -------------------------------------------------------- k_check_tri --

// Counts vertex indices outside [0, n_verts): run once when a context is
// created, so no later kernel can index outside the vertex array.
__global__ void k_check_tri(const int* __restrict__ tri, long long n, int n_verts,
                            unsigned long long* __restrict__ bad) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int v = tri[i];
    if (v < 0 || v >= n_verts) atomicAdd(bad, 1ull);
}

// --------------------------------------------------------- launchers --

hipError_t launch_signs(hipStream_t st, unsigned long long seed, unsigned step, unsigned pair0, unsigned scene,
                        long long d, int words, int n_pairs, uint32_t* bits) {
    long long nblk = (d + 255) >> 8;
    dim3 grid((unsigned)((nblk + 255) / 256), (unsigned)n_pairs);
    hipLaunchKernelGGL(k_signs, grid, dim3(256), 0, st, seed, step, pair0, scene, d, words, bits);
    return hipGetLastError();
}

hipError_t launch_setup(hipStream_t st, const SetupArgs& a, int n_items) {
    dim3 grid((unsigned)((a.sc.n_tris + 255) / 256), (unsigned)(n_items * a.nsign));
    hipLaunchKernelGGL(k_setup_bin, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int TILE>
static void launch_tile_t(hipStream_t st, const TileArgs& a, int mode, dim3 grid) {
    dim3 block((TILE * TILE > 256) ? 256 : TILE * TILE);
    if (mode == 0) hipLaunchKernelGGL((k_tile<TILE, 0>), grid, block, 0, st, a);
    else if (mode == 1) hipLaunchKernelGGL((k_tile<TILE, 1>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_tile<TILE, 2>), grid, block, 0, st, a);
}

hipError_t launch_tile(hipStream_t st, const TileArgs& a, int tile, int mode, int n_items, int max_tiles) {
    dim3 grid((unsigned)max_tiles, (unsigned)n_items);
    if (tile == 8) launch_tile_t<8>(st, a, mode, grid);
    else if (tile == 16) launch_tile_t<16>(st, a, mode, grid);
    else launch_tile_t<32>(st, a, mode, grid);
    return hipGetLastError();
}

hipError_t launch_sum_tiles(hipStream_t st, const double* partials, int max_tiles, const DViews& views,
                            int n_views, double* out) {
    hipLaunchKernelGGL(k_sum_tiles, dim3((unsigned)n_views), dim3(256), 0, st, partials, max_tiles, views, out);
    return hipGetLastError();
}

hipError_t launch_check_tri(hipStream_t st, const int* tri, long long n, int n_verts, unsigned long long* bad) {
    dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_check_tri, grid, dim3(256), 0, st, tri, n, n_verts, bad);
    return hipGetLastError();
}

hipError_t launch_fold(hipStream_t st, const FoldArgs& a) {
    dim3 grid((unsigned)((a.sc.G + 255) / 256));
    hipLaunchKernelGGL(k_fold, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_step(hipStream_t st, const StepArgs& a) {
    dim3 grid((unsigned)((a.sc.G + 255) / 256));
    hipLaunchKernelGGL(k_step, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}
