// dr_kernels.hip -- HIP kernels of the per-pixel stochastic gradient
// estimator for gfx950 (MI355X).
//
// Pipeline of one estimate (Sec. 4.3, Alg. 1 and 2, Eq. 8-9):
//   signs      Philox sign bits of every pair                  (shader P)
//   subdiv     (subdivision surfaces only, Sec. 6.3) the tessellated
//              vertex positions of every (pair, sign)
//   setup      per (item, sign, triangle): perturb the three vertices,
//              project, snap, build the raster record and append the
//              triangle to the bins of the tiles its bbox touches
//   tile       per (item, tile): rasterise the + and - scenes into LDS
//              depth|id keys (64-bit atomic min; the L nearest keys for
//              semi-transparent scenes), shade (and composite), form the
//              per-pixel difference and scatter it to the union of the
//              pixel's contribution groups                  (R and G fused)
//   fold       Q_i += sum_n s_i^(n) R^(n)_g(i): the per-group sums of each
//              pair become per-parameter fixed-point sums
//   step       decode, per-parameter average, Adam / SGD    (shader D)
// An "item" is one (pair, view) of a scene.  The single-scene kernels take
// their descriptors as kernel arguments; the batch kernels read them from
// device memory and cover many scenes per launch (the tile launch of a
// one-scene batch takes the scene and its views as kernel arguments too).
// All share the bodies below, so they compute the same bits.
#include <type_traits>

#include "dr_launch.h"


// ---------------------------------------------------------------- signs --

// Philox block `blk` of pair `pair`: 256 signs, written as 8 uint32 words.
__device__ __forceinline__ void signs_block(unsigned long long seed, unsigned step, unsigned pair, unsigned scene,
                                            long long blk, int words, uint32_t* __restrict__ out) {
    unsigned long long r[4];
    philox4x64_10((unsigned long long)blk, (unsigned long long)pair, step, scene, seed, 0ull, r);
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        long long word = blk * 8 + w;
        if (word < words) out[word] = (w & 1) ? (uint32_t)(r[w >> 1] >> 32) : (uint32_t)r[w >> 1];
    }
}

__global__ void k_signs(unsigned long long seed, unsigned step, unsigned pair0, unsigned scene,
                        long long d, int words, uint32_t* __restrict__ bits) {
    long long blk = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int p = blockIdx.y;
    long long nblk = (d + 255) >> 8;
    if (blk >= nblk) return;
    signs_block(seed, step, pair0 + p, scene, blk, words, bits + (long long)p * words);
}

// ---------------------------------------------------------------- setup --

// Triangle t of one (item, sign): perturbed vertices, projection, snap,
// setup record, and its entries in the bins of the tiles it may cover.
// fpos: the perturbed tessellated vertex positions of this (pair, sign) of a
// subdivision surface, or null (positions are the perturbed parameters).
// The perturbed world positions of triangle t's corners (original order).
__device__ __forceinline__ void tri_positions(const DScene& sc, const float* __restrict__ theta,
                                              const uint32_t* __restrict__ pb, float e0, float sgn, int t,
                                              const float* __restrict__ fpos, float* p) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int vid = sc.tri[3 * (long long)t + k];
        long long base = 3 * (long long)vid;
        if (fpos) {
            p[3 * k + 0] = fpos[base + 0];
            p[3 * k + 1] = fpos[base + 1];
            p[3 * k + 2] = fpos[base + 2];
        } else {
            p[3 * k + 0] = pval(theta, base + 0, e0, pb, sgn);
            p[3 * k + 1] = pval(theta, base + 1, e0, pb, sgn);
            p[3 * k + 2] = pval(theta, base + 2, e0, pb, sgn);
        }
    }
}

// Setup and binning of triangle t in one view from its perturbed corners p.
__device__ __forceinline__ void setup_tri_at(const DView& vw, const float* p, int t,
                                             TriR* __restrict__ recR, TriS* __restrict__ recS,
                                             unsigned* __restrict__ counts,
                                             unsigned* __restrict__ bins, int tile_px, int cap,
                                             unsigned* __restrict__ spn, unsigned long long* __restrict__ spill) {
    Vtx v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = xform(vw, p[3 * k + 0], p[3 * k + 1], p[3 * k + 2]);
    TriR r;
    TriS sh;
    r.flags = 0u;
    r.ia = 0.0f;
    r.pad = 0;
    bool ok = v[0].valid && v[1].valid && v[2].valid;
    long long area2 = 0;
    if (ok) {
        area2 = (long long)(v[1].X - v[0].X) * (long long)(v[2].Y - v[0].Y) -
                (long long)(v[1].Y - v[0].Y) * (long long)(v[2].X - v[0].X);
        ok = area2 != 0;
    }
    if (!ok) {
        recR[t] = r;                 // flags 0: culled
        return;
    }
    bool sw = area2 < 0;
    if (sw) {
        area2 = -area2;
        Vtx tmp = v[1]; v[1] = v[2]; v[2] = tmp;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { r.X[k] = v[k].X; r.Y[k] = v[k].Y; sh.iw[k] = v[k].iw; }
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
    r.ia = 1.0f / fa;
    int xmin = min(r.X[0], min(r.X[1], r.X[2])), xmax = max(r.X[0], max(r.X[1], r.X[2]));
    int ymin = min(r.Y[0], min(r.Y[1], r.Y[2])), ymax = max(r.Y[0], max(r.Y[1], r.Y[2]));
    if (xmax - xmin < 32768 && ymax - ymin < 32768) r.flags |= TRI_SMALL;
    // pixels whose centre 256 x + 128 lies in [min, max]
    int bx0 = max((xmin + 127) >> 8, 0), bx1 = min((xmax - 128) >> 8, vw.W - 1);
    int by0 = max((ymin + 127) >> 8, 0), by1 = min((ymax - 128) >> 8, vw.H - 1);
    if (bx0 > bx1 || by0 > by1) {               // no pixel centre in the bbox
        bx0 = 1; bx1 = 0; by0 = 1; by1 = 0;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) sh.p[k] = p[k];
    recR[t] = r;
    recS[t] = sh;
    if (bx0 > bx1) return;
    // Bin entries, one per tile the bbox touches.  Neighbouring triangles
    // share tiles, so the wave's lanes bidding for one tile are grouped
    // first (ballots only), then each group's leader adds the group's size
    // to the tile's counter -- all leaders at once -- and each lane takes its
    // rank in its group: same-address atomics no longer queue at one L2
    // channel.  Only the order of a bin's entries depends on this.
    int tx0 = bx0 / tile_px, tx1 = bx1 / tile_px, ty0 = by0 / tile_px, ty1 = by1 / tile_px;
    int ntx = tx1 - tx0 + 1;
    int n = ntx * (ty1 - ty0 + 1);
    int lane = threadIdx.x & 63;
    unsigned long long below = (1ull << lane) - 1ull;
    for (int i = 0;; ++i) {
        bool has = i < n;
        unsigned long long pend = __ballot(has);
        if (pend == 0ull) break;
        int tile = -1;
        if (has) tile = (ty0 + i / ntx) * vw.tiles_x + tx0 + i % ntx;
        int my_leader = lane;
        unsigned rank = 0u, group = 0u;
        while (pend) {
            int leader = __ffsll(pend) - 1;
            int lt = __shfl(tile, leader);
            bool mine = has && tile == lt;
            unsigned long long m = __ballot(mine);
            if (mine) {
                my_leader = leader;
                rank = (unsigned)__popcll(m & below);
            }
            if (lane == leader) group = (unsigned)__popcll(m);
            pend &= ~m;
        }
        unsigned base = 0u;
        if (has && my_leader == lane) base = atomicAdd(&counts[tile], group);
        base = __shfl(base, my_leader);
        const unsigned k = base + rank;
        if (has && k < (unsigned)cap) bins[(long long)tile * cap + k] = (unsigned)t;
        // entries past the capacity go to the render's spill list (the
        // first of a tile also counts the tile as overflowing)
        const bool sp = has && k >= (unsigned)cap && spill != nullptr;
        const unsigned long long ms = __ballot(sp);
        if (ms) {
            const int first = __ffsll((long long)ms) - 1;
            unsigned j0 = 0u;
            if (lane == first) j0 = atomicAdd(&spn[0], (unsigned)__popcll(ms));
            j0 = __shfl(j0, first);
            if (sp) {
                const unsigned j = j0 + __builtin_amdgcn_mbcnt_hi((unsigned)(ms >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((unsigned)ms, 0u));
                if (j < SPILL_CAP) spill[j] = ((unsigned long long)(unsigned)tile << 32) | (unsigned)t;
                if (k == (unsigned)cap) atomicAdd(&spn[1], 1u);
            }
        }
    }
}

__device__ __forceinline__ void setup_tri(const DScene& sc, const DView& vw, const float* __restrict__ theta,
                                          const uint32_t* __restrict__ pb, float e0, float sgn, int t,
                                          TriR* __restrict__ recR, TriS* __restrict__ recS,
                                          unsigned* __restrict__ counts,
                                          unsigned* __restrict__ bins, int tile_px, int cap,
                                          unsigned* __restrict__ spn, unsigned long long* __restrict__ spill,
                                          const float* __restrict__ fpos) {
    float p[9];
    tri_positions(sc, theta, pb, e0, sgn, t, fpos, p);
    setup_tri_at(vw, p, t, recR, recS, counts, bins, tile_px, cap, spn, spill);
}

__global__ void __launch_bounds__(256) k_setup_bin(SetupArgs a) {
    const DScene& sc = a.sc;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= sc.n_tris) return;
    int slot = blockIdx.y;                       // (local item, sign)
    int li = slot / a.nsign, s = slot % a.nsign;
    int item = a.item0 + li;
    int pair = item / a.n_views, view = item % a.n_views;
    const uint32_t* pb = a.pert.bits ? a.pert.bits + (long long)pair * sc.words : nullptr;
    const float* fpos = a.fpos ? a.fpos + ((long long)pair * a.nsign + s) * 3 * sc.n_verts : nullptr;
    setup_tri(sc, a.views.v[view], a.theta, pb, a.pert.eps[0], a.sgn[s], t, a.recR + (long long)slot * sc.n_tris,
              a.recS + (long long)slot * sc.n_tris,
              a.counts + (long long)slot * a.max_tiles, a.bins + (long long)slot * a.max_tiles * a.cap, a.tile,
              a.cap, a.spn ? a.spn + 2ll * slot : nullptr, a.spill ? a.spill + (long long)slot * SPILL_CAP : nullptr,
              fpos);
}

// Tessellated vertex positions of a subdivision surface for every (pair,
// sign) of a call: vertex j, coordinate c = the row's weights times the
// perturbed control coordinates, added in row order from zero.
__global__ void __launch_bounds__(256) k_subdiv(DScene sc, DPert pert, const float* __restrict__ theta, int nsign,
                                                float sgn0, float sgn1, float* __restrict__ fpos) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= sc.n_verts) return;
    int slot = blockIdx.y;                       // (pair, sign)
    int pair = slot / nsign, s = slot % nsign;
    const uint32_t* pb = pert.bits ? pert.bits + (long long)pair * sc.words : nullptr;
    float sgn = s == 0 ? sgn0 : sgn1;
    float e0 = pert.eps[0];
    int k0 = sc.sub_rowptr[j], k1 = sc.sub_rowptr[j + 1];
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (int k = k0; k < k1; ++k) {
        float w = sc.sub_w[k];
        long long base = 3 * (long long)sc.sub_cols[k];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = acc[c] + w * pval(theta, base + c, e0, pb, sgn);
    }
    float* out = fpos + ((long long)slot * sc.n_verts + j) * 3;
    out[0] = acc[0];
    out[1] = acc[1];
    out[2] = acc[2];
}

// ----------------------------------------------------------------- tile --

// Map consecutive workgroups (which the dispatcher spreads round-robin over
// the 8 XCDs) to contiguous runs of tiles per XCD, so neighbouring tiles --
// sharing triangles, texels and accumulators -- meet in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    int x = bid & 7, k = bid >> 3;
    int q = nb >> 3, rem = nb & 7;
    return x * q + min(x, rem) + k;
}

// Rasterise triangle t over the tile: one lane per covered pixel.  Opaque
// (DEEP false): key[pixel] keeps the least depth|id (64-bit atomic min).
// Deep: key[pixel * DRD_MAX_LAYERS + l] keeps the L least keys in order,
// by an atomic-min cascade -- the key is offered to layer 0, and whichever
// of the offered and the resident key is larger moves on to the next layer
// (an empty slot ends the cascade).  Every layer thus ends with the least
// key that reached it, i.e. the l-th least key of the pixel, whatever the
// interleaving of the lanes and waves.
// Offer depth|id key k to pixel li of the tile.
template <bool DEEP>
__device__ __forceinline__ void insert_key(unsigned long long* key, int li, unsigned long long k, int L) {
    if constexpr (DEEP) {
        unsigned long long* list = key + li * DRD_MAX_LAYERS;
        for (int l = 0; l < L; ++l) {
            unsigned long long old = atomicMin(&list[l], k);
            if (old == ~0ull) break;
            k = old > k ? old : k;
        }
    } else {
        atomicMin(&key[li], k);
    }
}

// Coverage, depth and the depth|id resolve of triangle t at pixel (x, y) of
// the tile.
template <int TILE, bool DEEP>
__device__ __forceinline__ void raster_px(const TriR& r, unsigned t, int x, int y, int px0, int py0,
                                          unsigned long long* key, int L) {
    int px = 256 * x + 128, py = 256 * y + 128;
    bool cov;
    if (r.flags & TRI_SMALL) {
        cov = inside_small(r, px, py);
    } else {
        long long e0, e1, e2;
        cov = inside(r, px, py, e0, e1, e2);
    }
    if (!cov) return;
    float z = depth_at(r, px, py);
    insert_key<DEEP>(key, (y - py0) * TILE + (x - px0), ((unsigned long long)__float_as_uint(z) << 32) | t, L);
}

// (cx1, cy1): the tile's last pixel inside the view.
template <int TILE, bool DEEP>
__device__ __forceinline__ void raster_tri(const TriR& r, unsigned t, int px0, int py0, int cx1, int cy1,
                                           int lane, unsigned long long* key, int L) {
    int x0, x1, y0, y1;
    tri_box(r, px0, py0, cx1, cy1, x0, x1, y0, y1);
    if (x0 > x1 || y0 > y1) return;
    int bw = x1 - x0 + 1;
    int n = bw * (y1 - y0 + 1);
    unsigned m = ((1u << 20) + (unsigned)bw - 1u) / (unsigned)bw;     // exact for bw <= 32, idx < 1024
    for (int base = 0; base < n; base += 64) {
        int idx = base + lane;
        if (idx < n) {
            int dy = (int)(((unsigned)idx * m) >> 20);
            int dx = idx - dy * bw;
            raster_px<TILE, DEEP>(r, t, x0 + dx, y0 + dy, px0, py0, key, L);
        }
    }
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves: shifts
// by 1, 2, 4 and 8 within each row of 16 lanes (lanes shifted in from
// outside the row add 0), then row 0's total to row 1 and row 2's to row 3
// (row_bcast:15), then row 1's running total to rows 2 and 3 (row_bcast:31).
// Must be called by every lane of the wave.
__device__ __forceinline__ int wave_inclusive_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);     // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);     // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);     // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);     // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);     // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);     // row_bcast:31
    return v;
}

// Per-wave LDS staging of a batch of small triangles for the packed raster
// (80 B each): edge k as an integer plane over the triangle's clipped
// bounding box, e_k(dx, dy) = a_k dx + b_k dy + c_k at pixel (x0 + dx,
// y0 + dy), the depth plane's offsets and the key index of the box corner.
struct __align__(16) PTri {
    int b[3];            // 256 dX_k: change of edge k per pixel row
    int a[3];            // -256 dY_k: change of edge k per pixel column
    int c[3];            // edge k at the corner pixel, plus 1 on a top-left edge
    int dz[2];           // corner pixel centre minus vertex 0, in subpixels
    float z0, zx, zy;
    unsigned t;
    int off0;            // key index of the corner pixel
    int bw;              // box width
    unsigned m;          // ceil(2^20 / slots per row), slots of two pixels
    int pex;             // the triangle's first slot in the packed sequence
    int pad;
};

struct RasterStage {
    PTri tri[64];
    int mark[64];
};

// Lanes of one wave exchange data through the wave's stage: a release fence
// before the wave barrier and an acquire fence after it make each lane's LDS
// stores visible to the other lanes' later loads (the barrier itself
// declares no memory effects, so without the fences the compiler could
// forward a lane's own store to its load past the other lanes' writes).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

static_assert(sizeof(PTri) == 80, "PTri layout");

// Packed raster of a batch whose triangles are all TRI_SMALL, through the
// wave's LDS stage.  Each triangle's clipped box is cut into slots of
// RASTER_SLOT horizontally adjacent pixels (a row of w pixels gives
// ceil(w / RASTER_SLOT) slots), the batch's slots are laid end to end, and
// each pass gives one slot to every lane: one read of the staged record, one
// index computation and one pass marking then serve all the slot's pixels.  The non-empty triangles are stored
// by rank; each pass marks the slots where a triangle begins, and a lane's
// triangle is then the number of triangles begun up to its slot (a ballot
// and a lane-masked bit count) -- one LDS read of the staged record instead
// of a binary search and a shuffle per field.  Edge values are exact: for a
// TRI_SMALL triangle both products of an edge function are below 2^30 in
// magnitude at every pixel of the box, so the edge value (and its value
// plus 1) fits in 32 bits and the wrapped 32-bit sums a dx + b dy + c equal
// it, as do the slot's further pixels' values, each its left neighbour's
// plus a; e > 0 || (e == 0 && top-left) is e + [top-left] > 0.
// Slots of 4 pixels: measured on the paper-scale step against 2, 3, 6 and 8
// (2 -> 4: tile kernel -2 % at the start of an optimisation run, -9 % after
// 50 Adam steps, when the triangles have grown; 6 and 8 within 2 % of 4).
#define RASTER_SLOT 4
template <int TILE, bool DEEP>
__device__ __forceinline__ void raster_staged(RasterStage* st, const TriR& r, unsigned t, int x0, int y0, int bw,
                                              int bh, int px0, int py0, int lane, unsigned long long* key, int L) {
    constexpr int SL = RASTER_SLOT;                     // pixels per slot
    const int sw = (bw + SL - 1) / SL;                  // slots per row
    const int c = sw * bh;                              // slots of this lane's triangle (0: none)
    const int P = wave_inclusive_sum(c);
    const int N = __builtin_amdgcn_readlane(P, 63);
    const int pex = P - c;
    unsigned long long nz = __ballot(c > 0);
    if (c > 0) {
        int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(nz >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)nz, 0u));
        PTri q;
        int cx = 256 * x0 + 128, cy = 256 * y0 + 128;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int ia = (k + 1) % 3, ib = (k + 2) % 3;
            int dX = r.X[ib] - r.X[ia], dY = r.Y[ib] - r.Y[ia];
            q.b[k] = 256 * dX;
            q.a[k] = -256 * dY;
            q.c[k] = (__mul24(dX, cy - r.Y[ia]) - __mul24(dY, cx - r.X[ia])) + (int)((r.flags >> (k + 1)) & 1u);
        }
        q.dz[0] = cx - r.X[0];
        q.dz[1] = cy - r.Y[0];
        q.z0 = r.z0; q.zx = r.zx; q.zy = r.zy;
        q.t = t;
        q.off0 = (y0 - py0) * TILE + (x0 - px0);
        q.bw = bw;
        q.m = ((1u << 20) + (unsigned)sw - 1u) / (unsigned)sw;     // exact for sw <= 32, idx < 1024
        q.pex = pex;
        q.pad = 0;
        st->tri[rank] = q;
    }
    wave_sync();
    int base = 0;                                       // triangles begun before this pass
    for (int s0 = 0; s0 < N; s0 += 64) {
        st->mark[lane] = 0;
        wave_sync();
        if (c > 0 && pex >= s0 && pex < s0 + 64) st->mark[pex - s0] = 1;
        wave_sync();
        int f = st->mark[lane];
        unsigned long long M = __ballot(f != 0);
        int rr = base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(M >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((unsigned)M, 0u)) + f - 1;
        base += __popcll(M);
        int sl = s0 + lane;
        if (sl < N) {
            PTri q = st->tri[rr];
            int idx = sl - q.pex;
            int dy = (int)(((unsigned)idx * q.m) >> 20);
            int qsw = (q.bw + SL - 1) / SL;
            int dx = SL * (idx - dy * qsw);
            int e0 = (__mul24(q.a[0], dx) + __mul24(q.b[0], dy)) + q.c[0];
            int e1 = (__mul24(q.a[1], dx) + __mul24(q.b[1], dy)) + q.c[1];
            int e2 = (__mul24(q.a[2], dx) + __mul24(q.b[2], dy)) + q.c[2];
            const float zrow = (float)(256 * dy + q.dz[1]);
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                if ((k == 0 || dx + k < q.bw) && min(e0, min(e1, e2)) > 0) {
                    float z = (q.z0 + q.zx * (float)(256 * (dx + k) + q.dz[0])) + q.zy * zrow;
                    if (!(z > 0.0f)) z = 0.0f;
                    insert_key<DEEP>(key, q.off0 + dy * TILE + dx + k,
                                     ((unsigned long long)__float_as_uint(z) << 32) | q.t, L);
                }
                e0 += q.a[0];
                e1 += q.a[1];
                e2 += q.a[2];
            }
        }
        wave_sync();
    }
}

// Raster of up to 64 triangles held one per lane (mine: the triangle
// index, valid for lanes below n).  A batch of TRI_SMALL triangles goes
// through the wave's LDS stage (raster_staged) whenever there is one.
// Otherwise, lane-packed when that takes fewer passes: the triangles' clipped bounding boxes are laid end to end (a
// prefix sum of their pixel counts) and each pass gives one pixel of that
// sequence to every lane, which finds its triangle by binary search over
// the prefix sums and reads the triangle's data from its lane.  For small
// triangles this replaces one pass per triangle, mostly idle lanes, with a
// pass per 64 candidates; large triangles keep a pass per 64 pixels of each.
// A packed pass costs more, so packing is taken when it saves a quarter of
// the passes (measured against always and never packing on the mesh, the
// 64-scene batch and the triangle soups).
template <int TILE, bool DEEP>
__device__ __forceinline__ void raster_batch(const TriR* __restrict__ R, unsigned mine, unsigned n, int px0,
                                             int py0, int cx1, int cy1, int lane, unsigned long long* key, int L,
                                             RasterStage* stage) {
    TriR r{};
    int x0 = 0, y0 = 0, bw = 1, bh = 0, c = 0;
    if ((unsigned)lane < n) {
        r = gload(&R[mine]);
        int x1, y1;
        tri_box(r, px0, py0, cx1, cy1, x0, x1, y0, y1);
        if (x0 <= x1 && y0 <= y1) {
            bw = x1 - x0 + 1;
            bh = y1 - y0 + 1;
            c = bw * bh;
        }
    }
    // Packed, never more passes than one triangle at a time: the staged
    // form is taken whenever it applies.
    if (stage != nullptr && __ballot(c > 0 && !(r.flags & TRI_SMALL)) == 0ull) {
        raster_staged<TILE, DEEP>(stage, r, mine, x0, y0, bw, bh, px0, py0, lane, key, L);
        return;
    }
    int P = wave_inclusive_sum(c);                      // prefix sums of the pixel counts
    int N = __builtin_amdgcn_readlane(P, 63);
    int T = wave_inclusive_sum((c + 63) >> 6);          // passes of the per-triangle loop
    int passes_tri = __builtin_amdgcn_readlane(T, 63);
    int passes_packed = (N + 63) >> 6;
    if (4 * passes_packed >= 3 * passes_tri) {
        // one triangle at a time, its record read from the lane that holds it
        const int* mw = reinterpret_cast<const int*>(&r);
        for (unsigned j = 0; j < n; ++j) {
            TriR q;
            int* qw = reinterpret_cast<int*>(&q);
#pragma unroll
            for (int k = 0; k < (int)(sizeof(TriR) / 4); ++k) qw[k] = __builtin_amdgcn_readlane(mw[k], j);
            raster_tri<TILE, DEEP>(q, __builtin_amdgcn_readlane(mine, j), px0, py0, cx1, cy1, lane, key, L);
        }
        return;
    }
    int Pex = P - c;
    unsigned m = ((1u << 20) + (unsigned)bw - 1u) / (unsigned)bw;
    for (int s0 = 0; s0 < N; s0 += 64) {
        int sl = s0 + lane;
        int lo = 0, hi = 63;                            // first lane whose prefix exceeds sl
#pragma unroll
        for (int step = 0; step < 6; ++step) {
            int mid = (lo + hi) >> 1;
            int pm = __shfl(P, mid);
            if (pm > sl) hi = mid;
            else lo = mid + 1;
        }
        int j = lo;
        TriR q;
        q.X[0] = __shfl(r.X[0], j); q.X[1] = __shfl(r.X[1], j); q.X[2] = __shfl(r.X[2], j);
        q.Y[0] = __shfl(r.Y[0], j); q.Y[1] = __shfl(r.Y[1], j); q.Y[2] = __shfl(r.Y[2], j);
        q.z0 = __shfl(r.z0, j); q.zx = __shfl(r.zx, j); q.zy = __shfl(r.zy, j);
        q.flags = (unsigned)__shfl((int)r.flags, j);
        int qx0 = __shfl(x0, j), qy0 = __shfl(y0, j), qbw = __shfl(bw, j), qpex = __shfl(Pex, j);
        unsigned qm = (unsigned)__shfl((int)m, j);
        unsigned qt = (unsigned)__shfl((int)mine, j);
        if (sl < N) {
            int idx = sl - qpex;
            int dy = (int)(((unsigned)idx * qm) >> 20);
            int dx = idx - dy * qbw;
            raster_px<TILE, DEEP>(q, qt, qx0 + dx, qy0 + dy, px0, py0, key, L);
        }
    }
}

// Record the largest bin occupancy.  The value only grows, so a workgroup
// that reads a value at least as large (possibly a stale one) may skip the
// atomic: almost all do, and the single counter no longer serialises a
// launch of a hundred thousand workgroups on one L2 channel.
__device__ __forceinline__ void note_max_bin(unsigned long long* stats, unsigned c) {
    unsigned long long seen = stats[ST_MAX_BIN];
    if ((unsigned long long)c > seen) atomicMax(&stats[ST_MAX_BIN], (unsigned long long)c);
}

// A bin of c entries, capacity cap: its overflow and occupancy statistics.
__device__ __forceinline__ void note_bin(unsigned long long* stats, unsigned c, unsigned cap) {
    if (c > cap) atomicAdd(&stats[ST_OVERFLOWS], 1ull);
    note_max_bin(stats, c);
}

// A wave's batch of bin entries holding at least this many triangles goes
// through raster_batch (lane-packed when that saves passes); smaller batches
// take one triangle per pass.
#ifndef PACK_MIN_TRIS
#define PACK_MIN_TRIS 8u
#endif

// Rasterise the cnt triangles of a tile's bin.  Wave w takes entries
// w, w + nw, w + 2 nw, ...; it fetches 64 of them at once (one per lane),
// so only the record load remains per triangle.
// One wave's batch of n <= 64 triangles, triangle `mine` held by lane < n.
template <int TILE, bool DEEP>
__device__ __forceinline__ void raster_group(const TriR* __restrict__ R, unsigned mine, unsigned n, int px0,
                                             int py0, int cx1, int cy1, int lane, unsigned long long* key, int L,
                                             RasterStage* stage) {
    if (n >= PACK_MIN_TRIS) {
        raster_batch<TILE, DEEP>(R, mine, n, px0, py0, cx1, cy1, lane, key, L, stage);
        return;
    }
    for (unsigned j = 0; j < n; ++j) {
        unsigned t = __builtin_amdgcn_readlane(mine, j);
        TriR r = gload(&R[t]);
        raster_tri<TILE, DEEP>(r, t, px0, py0, cx1, cy1, lane, key, L);
    }
}

template <int TILE, bool DEEP>
__device__ __forceinline__ void raster_bin(const unsigned* __restrict__ list, unsigned cnt,
                                           const TriR* __restrict__ R, int wave, int nw, int lane, int px0,
                                           int py0, int cx1, int cy1, unsigned long long* key, int L,
                                           RasterStage* stage) {
    for (unsigned base = (unsigned)wave; base < cnt; base += 64u * (unsigned)nw) {
        unsigned k = base + (unsigned)lane * (unsigned)nw;
        unsigned mine = k < cnt ? gload(&list[k]) : 0u;
        unsigned n = (cnt - base + (unsigned)nw - 1u) / (unsigned)nw;
        if (n > 64u) n = 64u;
        raster_group<TILE, DEEP>(R, mine, n, px0, py0, cx1, cy1, lane, key, L, stage);
    }
}

// A tile whose bin overflowed while its render's spill list was full (or
// absent): every valid triangle of the render whose pixel box meets the
// tile, found 64 at a time (one record's flags and box
// per lane), packed to the low lanes and rasterised as one batch.  The cost
// is one coalesced pass over the render's records per overflowing tile,
// not one dependent record read per triangle.
template <int TILE, bool DEEP>
__device__ __forceinline__ void raster_scan(const TriR* __restrict__ R, int n_tris, int wave, int nw, int lane,
                                            int px0, int py0, int cx1, int cy1, unsigned long long* key, int L,
                                            RasterStage* stage) {
    for (int t0 = wave * 64; t0 < n_tris; t0 += 64 * nw) {
        int t = t0 + lane;
        bool hit = false;
        if (t < n_tris) {
            const TriR* q = &R[t];
            TriR b;                                          // corners and flags (the first 28 B)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                b.X[k] = gload(&q->X[k]);
                b.Y[k] = gload(&q->Y[k]);
            }
            unsigned fl = gload(&q->flags);
            int x0 = 1, x1 = 0, y0 = 1, y1 = 0;
            if (fl & TRI_VALID) tri_box(b, px0, py0, cx1, cy1, x0, x1, y0, y1);
            hit = x0 <= x1 && y0 <= y1;
        }
        unsigned long long m = __ballot(hit);
        if (m == 0ull) continue;
        int n = __popcll(m);
        int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        // a permutation of the lanes: the hits to the front, in lane order
        int dst = hit ? below : n + (lane - below);
        unsigned mine = (unsigned)__builtin_amdgcn_ds_permute(dst * 4, t);
        raster_group<TILE, DEEP>(R, mine, (unsigned)n, px0, py0, cx1, cy1, lane, key, L, stage);
    }
}

// The spill entries of an overflowing bin: the render's spill list read 64
// entries at a time, the triangles that name this tile packed to the low
// lanes and rasterised as one batch.
template <int TILE, bool DEEP>
__device__ __forceinline__ void raster_spill(const TriR* __restrict__ R, const unsigned long long* __restrict__ spill,
                                             unsigned ns, int tile, int wave, int nw, int lane, int px0, int py0,
                                             int cx1, int cy1, unsigned long long* key, int L, RasterStage* stage) {
    for (unsigned j0 = (unsigned)wave * 64u; j0 < ns; j0 += 64u * (unsigned)nw) {
        const unsigned j = j0 + (unsigned)lane;
        bool hit = false;
        unsigned t = 0u;
        if (j < ns) {
            const unsigned long long e = gload(&spill[j]);
            hit = (unsigned)(e >> 32) == (unsigned)tile;
            t = (unsigned)e;
        }
        unsigned long long m = __ballot(hit);
        if (m == 0ull) continue;
        int n = __popcll(m);
        int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        int dst = hit ? below : n + (lane - below);
        unsigned mine = (unsigned)__builtin_amdgcn_ds_permute(dst * 4, (int)t);
        raster_group<TILE, DEEP>(R, mine, (unsigned)n, px0, py0, cx1, cy1, lane, key, L, stage);
    }
}

// Every triangle of one render that may cover the tile: its bin of cnt
// entries; for a bin past its capacity the full bin and the tile's entries
// of the render's spill list, or, when that list ran out of room (or there
// is none), every triangle of the render.  `note`: this wave counts a
// full scan in the statistics.
template <int TILE, bool DEEP>
__device__ __forceinline__ void raster_render(const TriR* __restrict__ R, const unsigned* __restrict__ bin,
                                              unsigned cnt, unsigned cap, const unsigned* spn,
                                              const unsigned long long* __restrict__ spill, int n_tris, int tile,
                                              int wave, int nw, int lane, int px0, int py0, int cx1, int cy1,
                                              unsigned long long* key, int L, RasterStage* stage,
                                              unsigned long long* stats, bool note) {
    if (cnt <= cap) {
        raster_bin<TILE, DEEP>(bin, cnt, R, wave, nw, lane, px0, py0, cx1, cy1, key, L, stage);
        return;
    }
    const unsigned ns = spn ? gload(&spn[0]) : 0xFFFFFFFFu;
    if (ns <= SPILL_CAP) {
        raster_bin<TILE, DEEP>(bin, cap, R, wave, nw, lane, px0, py0, cx1, cy1, key, L, stage);
        raster_spill<TILE, DEEP>(R, spill, ns, tile, wave, nw, lane, px0, py0, cx1, cy1, key, L, stage);
    } else {
        if (note && lane == 0) atomicAdd(&stats[ST_FULL_SCANS], 1ull);
        raster_scan<TILE, DEEP>(R, n_tris, wave, nw, lane, px0, py0, cx1, cy1, key, L, stage);
    }
}

// After the tile's raster: leave its bin empty for the next use, and the
// last overflowing tile of the render empties the render's spill list.
__device__ __forceinline__ void release_bin(unsigned* counts, int tile, unsigned cap, unsigned* spn) {
    const unsigned c = counts[tile];
    counts[tile] = 0u;
    if (c > cap && spn != nullptr && atomicSub(&spn[1], 1u) == 1u) spn[0] = 0u;
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

// A slot packs the group's sum and count into one 64-bit word,
// sum * 2^12 + count, so one LDS atomic adds both: a tile has at most 1024
// pixels, so the count stays below 2^12, and |sum| <= 1024 * 2^37 keeps the
// packed word within int64.
#define PACK_SHIFT 12
#define PACK_MASK ((1ull << PACK_SHIFT) - 1ull)

template <int LOG2T>
struct GroupTable {
    unsigned key[1 << LOG2T];
    unsigned long long sum[1 << LOG2T];     // packed sum and count
};

__device__ __forceinline__ unsigned long long pack_sc(long long q, unsigned c) {
    return ((unsigned long long)q << PACK_SHIFT) + (unsigned long long)c;
}

__device__ __forceinline__ void unpack_sc(unsigned long long w, long long& q, unsigned& c) {
    c = (unsigned)(w & PACK_MASK);
    q = (long long)(w - c) >> PACK_SHIFT;
}

__device__ __forceinline__ void global_add(long long* __restrict__ Rp, unsigned* __restrict__ K, long long g,
                                           long long q, unsigned c) {
    if (q != 0)
        __hip_atomic_fetch_add((DRD_GLOBAL unsigned long long*)&Rp[g], (unsigned long long)q, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add((DRD_GLOBAL unsigned*)&K[g], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int LOG2T>
__device__ __forceinline__ void table_add(GroupTable<LOG2T>& tb, long long* __restrict__ Rp,
                                          unsigned* __restrict__ K, unsigned g, long long q, unsigned c) {
    constexpr unsigned MASK = (1u << LOG2T) - 1u;
    // multiplicative hash in 24-bit multiplies (full rate; the 32-bit one is
    // quarter rate), the high byte folded in first
    unsigned h = (__umul24(g ^ (g >> 24), 0x9E3779u) >> (24 - LOG2T)) & MASK;
    for (int probe = 0; probe < HASH_PROBES; ++probe) {
        unsigned k = __hip_atomic_load(&tb.key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == HASH_EMPTY) k = atomicCAS(&tb.key[h], HASH_EMPTY, g);
        if (k == HASH_EMPTY || k == g) {
            atomicAdd(&tb.sum[h], pack_sc(q, c));
            return;
        }
        h = (h + 1u) & MASK;
    }
    global_add(Rp, K, g, q, c);      // crowded table: go straight to memory
}

// Subdivision surface: pixels whose + and - renders show the same
// tessellated triangle are combined per wave -- lanes with equal triangle
// ids are summed with a butterfly -- and the wave's lanes then share the
// table adds of that triangle's control-vertex list.  Must be called by
// every lane of the wave.
template <int LOG2T>
__device__ __forceinline__ void wave_ctrl(GroupTable<LOG2T>& tb, long long* __restrict__ Rp,
                                          unsigned* __restrict__ K, const DScene& sc, bool active, unsigned tri,
                                          long long q) {
    int lane = threadIdx.x & 63;
    unsigned long long pending = __ballot(active);
    while (pending) {
        int leader = __ffsll((unsigned long long)pending) - 1;
        unsigned lt = __builtin_amdgcn_readfirstlane(__shfl(tri, leader));
        bool mine = active && tri == lt;
        unsigned long long m = __ballot(mine);
        long long v = mine ? q : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        unsigned c = (unsigned)__popcll(m);
        int b0 = sc.tri_rowptr[lt], b1 = sc.tri_rowptr[lt + 1];
        for (int j = b0 + lane; j < b1; j += 64) table_add<LOG2T>(tb, Rp, K, (unsigned)sc.tri_cols[j], v, c);
        if (mine) active = false;
        pending &= ~m;
    }
}

// The union of two tessellated triangles' control vertices (both lists
// ascending), each once, for one pixel.
template <int LOG2T>
__device__ __forceinline__ void ctrl_union_add(GroupTable<LOG2T>& tb, long long* __restrict__ Rp,
                                               unsigned* __restrict__ K, const DScene& sc, unsigned t0,
                                               unsigned t1, long long q) {
    int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    if (t0 != DRD_BG) { a0 = sc.tri_rowptr[t0]; a1 = sc.tri_rowptr[t0 + 1]; }
    if (t1 != DRD_BG) { b0 = sc.tri_rowptr[t1]; b1 = sc.tri_rowptr[t1 + 1]; }
    int i = a0, j = b0;
    while (i < a1 || j < b1) {
        int ga = i < a1 ? sc.tri_cols[i] : 0x7FFFFFFF;
        int gb = j < b1 ? sc.tri_cols[j] : 0x7FFFFFFF;
        int g = ga < gb ? ga : gb;
        if (ga == g) ++i;
        if (gb == g) ++j;
        table_add<LOG2T>(tb, Rp, K, (unsigned)g, q, 1u);
    }
}

// Opaque tile kernels of 8- and 16-pixel tiles are asked for 6 resident
// waves per SIMD (at most 80 VGPRs), which they meet without spilling
// (measured per paper-scale step: 3.35 ms at 5 waves, 3.04 ms at 6; 7 and
// 8 waves spill).  Larger tiles and deep buffers are held to fewer waves by
// their LDS anyway.
#define TILE_MIN_WAVES 6

template <int TILE>
struct TileCfg {
    static constexpr int LOG2T = TILE == 8 ? 9 : (TILE == 16 ? 10 : 11);
};


// Everything the tile body needs, resolved by the kernel's prologue.
struct TileJob {
    const DScene* sc;
    const DView* vw;
    const float* theta;
    const uint32_t* pb;                  // sign bits of the pair (null: unperturbed)
    const float* eps;                    // per block
    float sgn[2];
    const TriR* recR[2];                 // records of each sign (index = triangle)
    const TriS* recS[2];
    unsigned* counts[2];                 // bin counters of each sign (index = tile)
    const unsigned* bins[2];             // bin entries of each sign (tile * cap + k)
    unsigned* spn[2];                    // spill counters of each sign, or null
    const unsigned long long* spill[2];  // spill lists of each sign
    int cap;
    int tile;
    unsigned long long* stats;
    // estimate
    const float* targets;                // this view's target image (image form: dL/dI)
    int img;                             // image form of the per-pixel difference
    long long* Rp;                       // group sums of the pair
    unsigned* K;
    int act_pos, any_act;
    const int* act_cls;
    // render
    float* out_rgb;
    unsigned* out_id;
    float* out_uv;
    // loss
    double* partial;
    // full-image estimate: the pair's total of fixed-point differences
    long long* qtot;
};

// MODE: 0 estimate (both signs, scatter), 1 render (write rgb/id/uv),
// 2 loss (per-tile sum of the per-pixel L2 error f_{w,h}), 3 full-image
// estimate (both signs, per-tile sum of the fixed-point differences).
template <int TILE, int MODE>
struct TileShared {
    static constexpr int NPIX = TILE * TILE;
    static constexpr int PPT = NPIX > 256 ? NPIX / 256 : 1;
    static constexpr int TB = NPIX / PPT;
    static constexpr int NS = (MODE == 0 || MODE == 3) ? 2 : 1;
    static constexpr int LOG2T = MODE == 0 ? TileCfg<TILE>::LOG2T : 1;
    unsigned long long key[NS][NPIX];
    // the raster's per-wave stages, then (estimate) the group table
    union {
        RasterStage stage[TB / 64];
        GroupTable<LOG2T> table;
    } u;
    double red[MODE == 2 ? TB : 1];
    long long qred[MODE == 3 ? TB : 1];
    unsigned nfl;                        // occupied table slots (flush)
};

template <int TILE, int MODE>
__device__ __forceinline__ void tile_body(const TileJob& J, TileShared<TILE, MODE>& S) {
    using SH = TileShared<TILE, MODE>;
    constexpr int NPIX = SH::NPIX, PPT = SH::PPT, TB = SH::TB, NS = SH::NS;
    constexpr int NW = TB / 64;
    constexpr int LOG2T = SH::LOG2T;
    constexpr int TSIZE = 1 << LOG2T;
    const DScene& sc = *J.sc;
    const DView& vw = *J.vw;
    int tx = J.tile % vw.tiles_x, ty = J.tile / vw.tiles_x;
    int px0 = tx * TILE, py0 = ty * TILE;
    const int cx1 = min(px0 + TILE - 1, vw.W - 1), cy1 = min(py0 + TILE - 1, vw.H - 1);   // last pixel in view
    int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    if constexpr (MODE == 0 || MODE == 3) {
        // no triangle of either render touches the tile: every pixel is
        // background in both, so the tile adds nothing (its bins are empty)
        if ((J.counts[0][J.tile] | J.counts[NS - 1][J.tile]) == 0u) return;
    }
    for (int j = tid; j < NS * NPIX; j += TB) (&S.key[0][0])[j] = ~0ull;
    __syncthreads();

    // Both signs' bins: with two signs and several waves, half of the
    // waves take each sign, so the two chains of dependent reads (bin
    // counter, entries, records) run at once; one wave takes both in turn.
    {
        constexpr int SPLIT = (NS == 2 && NW >= 2) ? 2 : 1;
        constexpr int NWS = NW / SPLIT;                  // waves per sign
        const int s_lo = SPLIT == 2 ? wave / NWS : 0;
        const int s_hi = SPLIT == 2 ? s_lo + 1 : NS;
        const int wv = wave - s_lo * NWS;
        for (int s = s_lo; s < s_hi; ++s) {
            // the sign picked by selects: a run-time index into J's arrays
            // would move J to private memory
            const bool s1 = NS == 2 && s == 1;
            const TriR* __restrict__ R = s1 ? J.recR[NS - 1] : J.recR[0];
            const unsigned* bins = s1 ? J.bins[NS - 1] : J.bins[0];
            unsigned* counts = s1 ? J.counts[NS - 1] : J.counts[0];
            const unsigned* spn = s1 ? J.spn[NS - 1] : J.spn[0];
            const unsigned long long* spill = s1 ? J.spill[NS - 1] : J.spill[0];
            unsigned long long* key = s1 ? S.key[NS - 1] : S.key[0];
            unsigned cnt = counts[J.tile];
            if (wv == 0 && lane == 0) note_bin(J.stats, cnt, (unsigned)J.cap);
            raster_render<TILE, false>(R, bins + (long long)J.tile * J.cap, cnt, (unsigned)J.cap, spn, spill,
                                       sc.n_tris, J.tile, wv, NWS, lane, px0, py0, cx1, cy1, key, 1,
                                       &S.u.stage[wave], J.stats, wv == 0);
        }
    }
    __syncthreads();
    if (tid < NS) {                              // leave the bins empty for the next use
        const bool s1 = NS == 2 && tid == 1;
        release_bin(s1 ? J.counts[NS - 1] : J.counts[0], J.tile, (unsigned)J.cap, s1 ? J.spn[NS - 1] : J.spn[0]);
    }
    if constexpr (MODE == 0) {
        // the stages are done with: the group table takes their place
        if (tid == 0) S.nfl = 0u;
        for (int j = tid; j < TSIZE; j += TB) {
            S.u.table.key[j] = HASH_EMPTY;
            S.u.table.sum[j] = 0ull;
        }
    }

    double loss_acc = 0.0;
    long long qsum = 0;
    for (int j = 0; j < PPT; ++j) {
        int local = tid + j * TB;
        int lx = local % TILE, ly = local / TILE;
        int x = px0 + lx, y = py0 + ly;
        bool inpix = x < vw.W && y < vw.H;
        int px = 256 * x + 128, py = 256 * y + 128;
        unsigned id[NS];
        float rgb[NS][3], uv[NS][2];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            unsigned long long k = inpix ? S.key[s][local] : ~0ull;
            id[s] = (k == ~0ull) ? DRD_BG : (unsigned)(k & 0xFFFFFFFFull);
            rgb[s][0] = 0.0f; rgb[s][1] = 0.0f; rgb[s][2] = 0.0f;
            uv[s][0] = 0.0f; uv[s][1] = 0.0f;
            if (id[s] != DRD_BG) {
                TriR r = gload(&J.recR[s][id[s]]);
                TriS sh = gload(&J.recS[s][id[s]]);
                TriF fr;
                CornerUV cu = load_cuv(sc, id[s]);
                if (sc.shading != 0) face_frame(sc.shading, sh.p, cu, fr);
                float alpha;
                Foot f0;
                shade_pixel(sc, vw, J.theta, J.pb, J.eps, J.sgn[s], r, sh, fr, cu, px, py, rgb[s], uv[s], f0, alpha);
            }
        }
        long long pix = (long long)y * vw.W + x;
        if constexpr (MODE == 2) {
            if (inpix) {
                const float* tg = J.targets + 3 * pix;
                float dr = rgb[0][0] - tg[0], dg = rgb[0][1] - tg[1], db = rgb[0][2] - tg[2];
                loss_acc += (double)((dr * dr + dg * dg) + db * db);
            }
        } else if constexpr (MODE == 3) {
            if (inpix && (id[0] != DRD_BG || id[1] != DRD_BG)) {
                int flag;
                qsum += quantize(pixel_delta(rgb[0], rgb[1], J.targets + 3 * pix, J.img), flag);
                if (flag) atomicAdd(&J.stats[flag == 1 ? ST_SATURATIONS : ST_NONFINITE], 1ull);
            }
        } else if constexpr (MODE == 1) {
            if (!inpix) continue;
            if (J.out_rgb) {
                J.out_rgb[3 * pix + 0] = rgb[0][0];
                J.out_rgb[3 * pix + 1] = rgb[0][1];
                J.out_rgb[3 * pix + 2] = rgb[0][2];
            }
            if (J.out_id) J.out_id[pix] = id[0];
            if (J.out_uv) {
                J.out_uv[2 * pix + 0] = uv[0][0];
                J.out_uv[2 * pix + 1] = uv[0][1];
            }
        } else {
            // an empty contribution set (background in both renders) adds nothing
            bool act = inpix && (id[0] != DRD_BG || id[1] != DRD_BG) && J.any_act;
            long long q = 0;
            if (act) {
                int flag;
                q = quantize(pixel_delta(rgb[0], rgb[1], J.targets + 3 * pix, J.img), flag);
                if (flag) atomicAdd(&J.stats[flag == 1 ? ST_SATURATIONS : ST_NONFINITE], 1ull);
            }
            if (j == 0) __syncthreads();         // the group table is cleared
            if (J.act_pos && sc.n_ctrl > 0) {
                bool same = act && id[0] == id[1];
                wave_ctrl<LOG2T>(S.u.table, J.Rp, J.K, sc, same, id[0], q);
                if (act && !same) ctrl_union_add<LOG2T>(S.u.table, J.Rp, J.K, sc, id[0], id[1], q);
            } else if (J.act_pos && act) {
                // the union of the two renders' triangles' vertices, each once
                int v0[3] = {-1, -1, -1};
                if (id[0] != DRD_BG) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        v0[k] = gload(&sc.tri[3 * (long long)id[0] + k]);
                        table_add<LOG2T>(S.u.table, J.Rp, J.K, (unsigned)v0[k], q, 1u);
                    }
                }
                if (id[1] != DRD_BG && id[1] != id[0]) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        int g = gload(&sc.tri[3 * (long long)id[1] + k]);
                        bool dup = (g == v0[0]) || (g == v0[1]) || (g == v0[2]);
                        if (!dup) table_add<LOG2T>(S.u.table, J.Rp, J.K, (unsigned)g, q, 1u);
                    }
                }
            }
            if (act) {
                for (int c = 0; c < sc.n_cls; ++c) {
                    if (!J.act_cls[c]) continue;
                    int W = sc.cls_w[c], H = sc.cls_h[c];
                    unsigned base = (unsigned)sc.cls_goff[c];
                    unsigned gs[NS][4];
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        gs[s][0] = gs[s][1] = gs[s][2] = gs[s][3] = HASH_EMPTY;
                        if (id[s] == DRD_BG) continue;
                        Foot f = footprint(uv[s][0], uv[s][1], W, H);
                        if (sc.tex_mode == 1) {
                            int xn = (f.fx >= 0.5f) ? f.xb : f.xa;
                            int yn = (f.fy >= 0.5f) ? f.yb : f.ya;
                            gs[s][0] = base + (__umul24((unsigned)yn, (unsigned)W) + (unsigned)xn);
                        } else {
                            gs[s][0] = base + (__umul24((unsigned)f.ya, (unsigned)W) + (unsigned)f.xa);
                            gs[s][1] = base + (__umul24((unsigned)f.ya, (unsigned)W) + (unsigned)f.xb);
                            gs[s][2] = base + (__umul24((unsigned)f.yb, (unsigned)W) + (unsigned)f.xa);
                            gs[s][3] = base + (__umul24((unsigned)f.yb, (unsigned)W) + (unsigned)f.xb);
                        }
                    }
#pragma unroll
                    for (int s = 0; s < NS; ++s)
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            unsigned g = gs[s][k];
                            if (g == HASH_EMPTY) continue;
                            bool dup = false;
#pragma unroll
                            for (int j2 = 0; j2 < 4; ++j2)
                                if (j2 < k && gs[s][j2] == g) dup = true;
                            if (s == 1) {
#pragma unroll
                                for (int j2 = 0; j2 < 4; ++j2)
                                    if (gs[0][j2] == g) dup = true;
                            }
                            if (!dup) table_add<LOG2T>(S.u.table, J.Rp, J.K, g, q, 1u);
                        }
                }
            }
        }
    }
    if constexpr (MODE == 2) {
        // fixed-order tree reduction of the tile's per-pixel errors
        S.red[tid] = loss_acc;
        __syncthreads();
        for (int w = TB / 2; w > 0; w >>= 1) {
            if (tid < w) S.red[tid] = S.red[tid] + S.red[tid + w];
            __syncthreads();
        }
        if (tid == 0) *J.partial = S.red[0];
    }
    if constexpr (MODE == 3) {
        // integer sums: the order of the additions does not matter
        S.qred[tid] = qsum;
        __syncthreads();
        for (int w = TB / 2; w > 0; w >>= 1) {
            if (tid < w) S.qred[tid] = S.qred[tid] + S.qred[tid + w];
            __syncthreads();
        }
        if (tid == 0 && S.qred[0] != 0) atomicAdd((unsigned long long*)J.qtot, (unsigned long long)S.qred[0]);
    }
    if constexpr (MODE == 0) {
        __syncthreads();
        if constexpr (TILE >= 16) {
            // occupied slots first gathered into a dense list (in the key
            // buffers, free by now and large enough from 16-pixel tiles
            // on), so the global atomics go out in full waves
            unsigned* list = reinterpret_cast<unsigned*>(&S.key[0][0]);
            for (int j = tid; j < TSIZE; j += TB) {
                bool occ = S.u.table.key[j] != HASH_EMPTY;
                unsigned long long m = __ballot(occ);
                unsigned base = 0;
                if (lane == 0 && m) base = atomicAdd(&S.nfl, (unsigned)__popcll(m));
                base = __shfl(base, 0);
                if (occ) list[base + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))] = (unsigned)j;
            }
            __syncthreads();
            unsigned n = S.nfl;
            for (unsigned i = (unsigned)tid; i < n; i += TB) {
                unsigned j = list[i];
                long long q;
                unsigned c;
                unpack_sc(S.u.table.sum[j], q, c);
                global_add(J.Rp, J.K, (long long)S.u.table.key[j], q, c);
            }
        } else {
            for (int j = tid; j < TSIZE; j += TB) {
                unsigned g = S.u.table.key[j];
                if (g != HASH_EMPTY) {
                    long long q;
                    unsigned c;
                    unpack_sc(S.u.table.sum[j], q, c);
                    global_add(J.Rp, J.K, (long long)g, q, c);
                }
            }
        }
    }
}


// ------------------------------------------------- semi-transparent tile --
//
// Sec. 4.4 "Transparent geometry": the raster keeps, per pixel and sign,
// the L nearest fragments in front-to-back order (a deep ID buffer in LDS,
// built by the atomic-min cascade of raster_tri), the shading pass
// composites them over black, C = sum_l T_l alpha_l c_l with
// T_{l+1} = T_l (1 - alpha_l), and the scatter credits the union over both
// renders and all listed layers of the layers' vertices and footprint
// texels, each group once per pixel.  Tiles are 8 or 16 pixels (one pixel
// per lane).

template <int TILE, int MODE>
struct DeepShared {
    static constexpr int NPIX = TILE * TILE;
    static constexpr int TB = NPIX;
    static constexpr int NS = (MODE == 0 || MODE == 3) ? 2 : 1;
    static constexpr int LOG2T = MODE == 0 ? TileCfg<TILE>::LOG2T : 1;
    unsigned long long key[NS][NPIX * DRD_MAX_LAYERS];
    // the raster's per-wave stages, then (estimate) the group table
    union {
        RasterStage stage[TB / 64 > 0 ? TB / 64 : 1];
        GroupTable<LOG2T> table;
    } u;
    double red[MODE == 2 ? TB : 1];
    long long qred[MODE == 3 ? TB : 1];
};

// Texel groups of one fragment in class c: the bilinear footprint, or the
// nearest texel (the other entries HASH_EMPTY).
__device__ __forceinline__ void texel_groups(const DScene& sc, int c, float u, float v, unsigned* gs) {
    int W = sc.cls_w[c], H = sc.cls_h[c];
    unsigned base = (unsigned)sc.cls_goff[c];
    Foot f = footprint(u, v, W, H);
    if (sc.tex_mode == 1) {
        int xn = (f.fx >= 0.5f) ? f.xb : f.xa;
        int yn = (f.fy >= 0.5f) ? f.yb : f.ya;
        gs[0] = base + (__umul24((unsigned)yn, (unsigned)W) + (unsigned)xn);
        gs[1] = gs[2] = gs[3] = HASH_EMPTY;
    } else {
        gs[0] = base + (__umul24((unsigned)f.ya, (unsigned)W) + (unsigned)f.xa);
        gs[1] = base + (__umul24((unsigned)f.ya, (unsigned)W) + (unsigned)f.xb);
        gs[2] = base + (__umul24((unsigned)f.yb, (unsigned)W) + (unsigned)f.xa);
        gs[3] = base + (__umul24((unsigned)f.yb, (unsigned)W) + (unsigned)f.xb);
    }
}

template <int TILE, int MODE>
__device__ __forceinline__ void tile_body_deep(const TileJob& J, DeepShared<TILE, MODE>& S) {
    using SH = DeepShared<TILE, MODE>;
    constexpr int NPIX = SH::NPIX, TB = SH::TB, NS = SH::NS;
    constexpr int NW = TB / 64 > 0 ? TB / 64 : 1;
    constexpr int LOG2T = SH::LOG2T;
    constexpr int TSIZE = 1 << LOG2T;
    constexpr int LM = DRD_MAX_LAYERS;
    constexpr int NE = NS * LM;                    // fragment entries per pixel
    const DScene& sc = *J.sc;
    const DView& vw = *J.vw;
    const int L = sc.layers;
    int tx = J.tile % vw.tiles_x, ty = J.tile / vw.tiles_x;
    int px0 = tx * TILE, py0 = ty * TILE;
    const int cx1 = min(px0 + TILE - 1, vw.W - 1), cy1 = min(py0 + TILE - 1, vw.H - 1);   // last pixel in view
    int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    if constexpr (MODE == 0 || MODE == 3) {
        // no fragment in either render: the tile adds nothing
        if ((J.counts[0][J.tile] | J.counts[NS - 1][J.tile]) == 0u) return;
    }
    for (int j = tid; j < NS * NPIX * LM; j += TB) (&S.key[0][0])[j] = ~0ull;
    __syncthreads();

#pragma unroll
    for (int s = 0; s < NS; ++s) {
        unsigned cnt = J.counts[s][J.tile];
        if (tid == 0) note_bin(J.stats, cnt, (unsigned)J.cap);
        const TriR* __restrict__ R = J.recR[s];
        raster_render<TILE, true>(R, J.bins[s] + (long long)J.tile * J.cap, cnt, (unsigned)J.cap, J.spn[s],
                                  J.spill[s], sc.n_tris, J.tile, wave, NW, lane, px0, py0, cx1, cy1, S.key[s], L,
                                  &S.u.stage[wave], J.stats, wave == 0);
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) release_bin(J.counts[s], J.tile, (unsigned)J.cap, J.spn[s]);
    }
    if constexpr (MODE == 0) {
        // the stages are done with: the group table takes their place
        for (int j = tid; j < TSIZE; j += TB) {
            S.u.table.key[j] = HASH_EMPTY;
            S.u.table.sum[j] = 0ull;
        }
    }

    int local = tid;
    int lx = local % TILE, ly = local / TILE;
    int x = px0 + lx, y = py0 + ly;
    bool inpix = x < vw.W && y < vw.H;
    int px = 256 * x + 128, py = 256 * y + 128;
    long long pix = (long long)y * vw.W + x;
    // Lists fill from the front, so a list is empty when its first layer is.
    // The loops over layers stay rolled (the fragments are re-read from the
    // LDS list, their UVs recomputed where needed) so that nothing indexed
    // by layer has to live in registers.
    float rgb[NS][3];
    bool any = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        rgb[s][0] = 0.0f; rgb[s][1] = 0.0f; rgb[s][2] = 0.0f;
        float T = 1.0f;
        for (int l = 0; l < L; ++l) {
            unsigned long long k = inpix ? S.key[s][local * LM + l] : ~0ull;
            unsigned id = (k == ~0ull) ? DRD_BG : (unsigned)(k & 0xFFFFFFFFull);
            float uv[2] = {0.0f, 0.0f};
            if (id != DRD_BG) {
                any = true;
                TriR r = gload(&J.recR[s][id]);
                TriS sh = gload(&J.recS[s][id]);
                TriF fr;
                CornerUV cu = load_cuv(sc, id);
                if (sc.shading != 0) face_frame(sc.shading, sh.p, cu, fr);
                float c[3], al;
                Foot f0;
                shade_pixel(sc, vw, J.theta, J.pb, J.eps, J.sgn[s], r, sh, fr, cu, px, py, c, uv, f0, al);
                float wt = T * al;
                rgb[s][0] = rgb[s][0] + wt * c[0];
                rgb[s][1] = rgb[s][1] + wt * c[1];
                rgb[s][2] = rgb[s][2] + wt * c[2];
                T = T * (1.0f - al);
            }
            if constexpr (MODE == 1) {
                if (inpix) {
                    long long e = pix * L + l;
                    if (J.out_id) J.out_id[e] = id;
                    if (J.out_uv) {
                        J.out_uv[2 * e + 0] = uv[0];
                        J.out_uv[2 * e + 1] = uv[1];
                    }
                }
            }
        }
    }

    if constexpr (MODE == 1) {
        if (inpix && J.out_rgb) {
            J.out_rgb[3 * pix + 0] = rgb[0][0];
            J.out_rgb[3 * pix + 1] = rgb[0][1];
            J.out_rgb[3 * pix + 2] = rgb[0][2];
        }
        return;
    }
    if constexpr (MODE == 2) {
        double loss_acc = 0.0;
        if (inpix) {
            const float* tg = J.targets + 3 * pix;
            float dr = rgb[0][0] - tg[0], dg = rgb[0][1] - tg[1], db = rgb[0][2] - tg[2];
            loss_acc = (double)((dr * dr + dg * dg) + db * db);
        }
        S.red[tid] = loss_acc;
        __syncthreads();
        for (int w = TB / 2; w > 0; w >>= 1) {
            if (tid < w) S.red[tid] = S.red[tid] + S.red[tid + w];
            __syncthreads();
        }
        if (tid == 0) *J.partial = S.red[0];
        return;
    }
    if constexpr (MODE == 3) {
        long long qsum = 0;
        if (inpix && any) {
            int flag;
            qsum = quantize(pixel_delta(rgb[0], rgb[1], J.targets + 3 * pix, J.img), flag);
            if (flag) atomicAdd(&J.stats[flag == 1 ? ST_SATURATIONS : ST_NONFINITE], 1ull);
        }
        S.qred[tid] = qsum;
        __syncthreads();
        for (int w = TB / 2; w > 0; w >>= 1) {
            if (tid < w) S.qred[tid] = S.qred[tid] + S.qred[tid + w];
            __syncthreads();
        }
        if (tid == 0 && S.qred[0] != 0) atomicAdd((unsigned long long*)J.qtot, (unsigned long long)S.qred[0]);
        return;
    }
    if constexpr (MODE == 0) {
        __syncthreads();                             // the group table is cleared
        bool act = inpix && any && J.any_act;
        if (act) {
            int flag;
            long long q = quantize(pixel_delta(rgb[0], rgb[1], J.targets + 3 * pix, J.img), flag);
            if (flag) atomicAdd(&J.stats[flag == 1 ? ST_SATURATIONS : ST_NONFINITE], 1ull);
            // fragment e = s * L + l; each group is added by the first
            // fragment that holds it
            const int NF = NS * L;
            for (int e = 0; e < NF; ++e) {
                int s1 = e / L, l1 = e % L;
                unsigned long long k1 = (&S.key[0][0])[(s1 * NPIX + local) * LM + l1];
                if (k1 == ~0ull) continue;
                unsigned id1 = (unsigned)(k1 & 0xFFFFFFFFull);
                if (J.act_pos) {
                    int v1[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) v1[k] = gload(&sc.tri[3 * (long long)id1 + k]);
                    bool dup[3] = {false, false, false};
                    for (int e2 = 0; e2 < e; ++e2) {
                        unsigned long long k2 = (&S.key[0][0])[((e2 / L) * NPIX + local) * LM + e2 % L];
                        if (k2 == ~0ull) continue;
                        const int* t2 = sc.tri + 3 * (long long)(unsigned)(k2 & 0xFFFFFFFFull);
                        int v2[3] = {gload(&t2[0]), gload(&t2[1]), gload(&t2[2])};
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            dup[k] = dup[k] || v1[k] == v2[0] || v1[k] == v2[1] || v1[k] == v2[2];
                    }
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        if (!dup[k]) table_add<LOG2T>(S.u.table, J.Rp, J.K, (unsigned)v1[k], q, 1u);
                }
                if (J.any_act && sc.n_cls > 0) {
                    Attr a1 = frag_attr(sc, (s1 ? J.recR[1] : J.recR[0])[id1], (s1 ? J.recS[1] : J.recS[0])[id1],
                                        load_cuv(sc, id1), px, py);
                    for (int c = 0; c < sc.n_cls; ++c) {
                        if (!J.act_cls[c]) continue;
                        unsigned gs[4];
                        texel_groups(sc, c, a1.u, a1.v, gs);
                        bool dup[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            dup[k] = gs[k] == HASH_EMPTY;
#pragma unroll
                            for (int k2 = 0; k2 < 4; ++k2)
                                if (k2 < k && gs[k2] == gs[k]) dup[k] = true;
                        }
                        for (int e2 = 0; e2 < e; ++e2) {
                            unsigned long long k2 = (&S.key[0][0])[((e2 / L) * NPIX + local) * LM + e2 % L];
                            if (k2 == ~0ull) continue;
                            unsigned id2 = (unsigned)(k2 & 0xFFFFFFFFull);
                            Attr a2 = frag_attr(sc, (e2 >= L ? J.recR[1] : J.recR[0])[id2],
                                                (e2 >= L ? J.recS[1] : J.recS[0])[id2], load_cuv(sc, id2), px, py);
                            unsigned gs2[4];
                            texel_groups(sc, c, a2.u, a2.v, gs2);
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                dup[k] = dup[k] || gs[k] == gs2[0] || gs[k] == gs2[1] || gs[k] == gs2[2] ||
                                         gs[k] == gs2[3];
                        }
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            if (!dup[k]) table_add<LOG2T>(S.u.table, J.Rp, J.K, gs[k], q, 1u);
                    }
                }
            }
        }
        __syncthreads();
        for (int j = tid; j < TSIZE; j += TB) {
            unsigned g = S.u.table.key[j];
            if (g != HASH_EMPTY) {
                long long q;
                unsigned c;
                unpack_sc(S.u.table.sum[j], q, c);
                global_add(J.Rp, J.K, (long long)g, q, c);
            }
        }
    }
}

// One (item, tile) of a single-scene launch: opaque or semi-transparent
// body.  The job is built here, in the kernel itself, so that the argument
// block is read in place from the kernel-argument segment.
template <int TILE, int MODE, bool DEEP>
__global__ void __launch_bounds__((TILE * TILE > 256) ? 256 : TILE * TILE, (DEEP || TILE > 16) ? 1 : TILE_MIN_WAVES)
k_tile(TileArgs a) {
    using SH = std::conditional_t<DEEP, DeepShared<TILE, MODE>, TileShared<TILE, MODE>>;
    __shared__ SH S;
    constexpr int NS = SH::NS;
    const DScene& sc = a.sc;
    int li = blockIdx.y;
    int item = a.item0 + li;
    int pair = item / a.n_views, view = item % a.n_views;
    const DView& vw = a.views.v[view];
    int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= vw.tiles_x * vw.tiles_y) return;
    TileJob J;
    J.sc = &a.sc;
    J.vw = &vw;
    J.theta = a.theta;
    J.pb = a.pert.bits ? a.pert.bits + (long long)pair * sc.words : nullptr;
    J.eps = a.pert.eps;
    J.sgn[0] = a.sgn[0];
    J.sgn[1] = a.sgn[1];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        int slot = li * NS + (s < NS ? s : 0);
        J.recR[s] = a.recR + (long long)slot * sc.n_tris;
        J.recS[s] = a.recS + (long long)slot * sc.n_tris;
        J.counts[s] = a.counts + (long long)slot * a.max_tiles;
        J.bins[s] = a.bins + (long long)slot * a.max_tiles * a.cap;
        J.spn[s] = a.spn ? a.spn + 2ll * slot : nullptr;
        J.spill[s] = a.spill ? a.spill + (long long)slot * SPILL_CAP : nullptr;
    }
    J.cap = a.cap;
    J.tile = tile;
    J.stats = a.stats;
    J.targets = a.targets ? a.targets + vw.tgt_off : nullptr;
    J.img = a.img_grad;
    J.Rp = (MODE == 0) ? a.R + (long long)pair * sc.G : nullptr;
    J.K = a.K;
    J.act_pos = a.act_pos;
    J.any_act = a.any_act;
    J.act_cls = a.act_cls;
    J.out_rgb = a.out_rgb;
    J.out_id = a.out_id;
    J.out_uv = a.out_uv;
    J.partial = a.partials ? a.partials + (long long)li * a.max_tiles + tile : nullptr;
    J.qtot = (MODE == 3) ? a.qtot + pair : nullptr;
    if constexpr (DEEP) tile_body_deep<TILE, MODE>(J, S);
    else tile_body<TILE, MODE>(J, S);
}

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

// -------------------------------------------------------------- fold --

// Parameters of group g: a vertex's x, y, z, or a texel's channels in
// every texture of its class.  Calls fn(param index, block).
template <typename Fn>
__device__ __forceinline__ void for_params(const DScene& sc, long long g, Fn fn) {
    if (g < sc.n_vg) {
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

// Q_i += sum_n s_i^(n) R_g^(n) for the parameters of group g, then R_g = 0.
// Pairs are taken 8 at a time: the group's 8 sums are read once (not once
// per parameter), a chunk that is all zero (the group was not seen by those
// pairs) costs no sign reads, and only non-zero sums are cleared.
__device__ __forceinline__ void fold_group(const DScene& sc, long long g, long long* __restrict__ R,
                                           const uint32_t* __restrict__ bits, int n_pairs, const float* eps,
                                           long long* __restrict__ Q) {
    for (int n0 = 0; n0 < n_pairs; n0 += 8) {
        long long r[8];
        bool any = false;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            r[j] = (n0 + j < n_pairs) ? R[(long long)(n0 + j) * sc.G + g] : 0;
            any = any || r[j] != 0;
        }
        if (!any) continue;
        for_params(sc, g, [&](long long i, int b) {
            if (eps[b] == 0.0f) return;
            long long acc = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (r[j] == 0) continue;
                acc += (sign_of(bits + (long long)(n0 + j) * sc.words, i) > 0) ? r[j] : -r[j];
            }
            if (acc != 0) Q[i] += acc;
        });
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (r[j] != 0) R[(long long)(n0 + j) * sc.G + g] = 0;
    }
}

// Full-image estimate: every parameter of an active block gets
// s_i^(n) * T[n] for every pair n; every active group counts one
// contribution per (pair, view).  T is zeroed by k_zero64 before the call.
__global__ void __launch_bounds__(256) k_broadcast(FoldArgs a) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const DScene& sc = a.sc;
    if (g >= sc.G) return;
    bool active = false;
    if (g < sc.n_vg) {
        active = a.eps[0] != 0.0f;
    } else {
        for (int c = 0; c < sc.n_cls; ++c) {
            long long size = (long long)sc.cls_w[c] * sc.cls_h[c];
            long long texel = g - sc.cls_goff[c];
            if (texel >= 0 && texel < size)
                for (int t = 0; t < sc.n_tex; ++t)
                    if (sc.tex_cls[t] == c && a.eps[1 + t] != 0.0f) active = true;
        }
    }
    if (!active) return;
    for_params(sc, g, [&](long long i, int b) {
        if (a.eps[b] == 0.0f) return;
        long long acc = 0;
        for (int n = 0; n < a.n_pairs; ++n) {
            long long r = a.qtot[n];
            acc += (sign_of(a.bits + (long long)n * sc.words, i) > 0) ? r : -r;
        }
        if (acc != 0) a.Q[i] += acc;
    });
    a.K[g] += (unsigned)(a.n_pairs * a.n_views);
}

__global__ void k_zero64(long long* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void __launch_bounds__(256) k_fold(FoldArgs a) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.sc.G) return;
    fold_group(a.sc, g, a.R, a.bits, a.n_pairs, a.eps, a.Q);
}

// ------------------------------------------------------ step / decode --

__device__ __forceinline__ void step_group(const DScene& sc, long long g, const float* eps, const float* lr,
                                           int n_pairs, const OptimConst& oc, float bc1, float bc2,
                                           int decode_only, float* __restrict__ theta, float* __restrict__ m,
                                           float* __restrict__ v, long long* __restrict__ Q,
                                           unsigned* __restrict__ K, float* __restrict__ grad,
                                           unsigned long long* __restrict__ stats) {
    unsigned kc = K[g];
    double D = (oc.averaging == 0) ? (double)kc : (double)n_pairs;
    for_params(sc, g, [&](long long i, int b) {
        float e = eps[b];
        long long qv = Q[i];
        float gi = 0.0f;
        if (e != 0.0f && D != 0.0)
            gi = (float)(((double)qv * (1.0 / 4294967296.0)) / (2.0 * (double)e * D));
        if (decode_only) {
            grad[i] = gi;
            return;
        }
        Q[i] = 0;
        if (e == 0.0f) return;
        if (oc.averaging == 0 && kc == 0u) return;
        if (!(fabsf(gi) <= 3.402823466e38f)) {
            atomicAdd(&stats[ST_NONFINITE], 1ull);
            return;
        }
        float l = lr[b];
        if (oc.kind == 1) {
            theta[i] = theta[i] - l * gi;
        } else {
            float mi = oc.b1 * m[i] + oc.omb1 * gi;
            float vi = oc.b2 * v[i] + oc.omb2 * (gi * gi);
            m[i] = mi;
            v[i] = vi;
            float mh = mi / bc1;
            float vh = vi / bc2;
            theta[i] = theta[i] - l * (mh / (sqrtf(vh) + oc.eps_hat));
        }
    });
    if (!decode_only) K[g] = 0u;
}

__global__ void __launch_bounds__(256) k_step(StepArgs a) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.sc.G) return;
    step_group(a.sc, g, a.eps, a.lr, a.n_pairs, a.oc, a.bc1, a.bc2, a.decode_only, a.theta, a.m, a.v, a.Q, a.K,
               a.grad, a.stats);
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

// -------------------------------------------------------------- batch --

// Index of the last entry of a non-decreasing sequence (stride in bytes
// between entries, starting at `first`) that is <= x; n >= 1 entries.
__device__ __forceinline__ int last_le(const char* first, int stride, int n, long long x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        long long v = *(const long long*)(first + (long long)mid * stride);
        if (v <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_batch_end(unsigned* step) { *step = *step + 1u; }

// Signs of every (scene, pair): the blocks of a scene are contiguous and
// each (scene, pair) starts on a block boundary.
__global__ void __launch_bounds__(256) k_signs_b(BatchArgs b) {
    long long blk = blockIdx.x;
    int si = last_le((const char*)&b.scenes[0].sign_blk0, sizeof(BScene), b.n_scenes, blk);
    si = __builtin_amdgcn_readfirstlane(si);
    const BScene& S = b.scenes[si];
    long long nblk = (S.sc.d + 255) >> 8;
    long long per_pair = (nblk + 255) >> 8;               // blocks per pair
    long long local = blk - S.sign_blk0;
    int pair = (int)(local / per_pair);
    long long pblk = (local % per_pair) * 256 + threadIdx.x;
    if (pblk >= nblk) return;
    signs_block(b.seed, *b.step, (unsigned)pair, (unsigned)S.scene_index, pblk, S.sc.words,
                S.bits + (long long)pair * S.sc.words);
}

// Setup of every (item, sign, triangle): each (item, sign) starts on a
// block boundary.
__global__ void __launch_bounds__(256) k_setup_b(BatchArgs b) {
    long long blk = b.unit0 + blockIdx.x;
    int it = last_le((const char*)&b.items[0].setup_blk0, sizeof(BItem), b.n_items, blk);
    it = __builtin_amdgcn_readfirstlane(it);
    const BItem& I = b.items[it];
    const BScene& S = b.scenes[I.scene];
    const DScene& sc = S.sc;
    long long per_sign = ((long long)sc.n_tris + 255) >> 8;
    long long local = blk - I.setup_blk0;
    int s = (int)(local / per_sign);
    int t = (int)((local % per_sign) * 256 + threadIdx.x);
    if (t >= sc.n_tris) return;
    const DView& vw = b.views[I.view];
    int tiles = vw.tiles_x * vw.tiles_y;
    setup_tri(sc, vw, S.theta, S.bits + (long long)I.pair * sc.words, S.eps[0], s == 0 ? 1.0f : -1.0f, t,
              b.recR + I.rec_off + (long long)s * sc.n_tris, b.recS + I.rec_off + (long long)s * sc.n_tris,
              b.counts + I.cnt_off + (long long)s * tiles,
              b.bins + I.bin_off + (long long)s * tiles * I.cap, b.tile, I.cap, b.spn + 2 * (I.sp_off + s),
              b.spill + (I.sp_off + s) * SPILL_CAP, nullptr);
}

// Setup of a one-scene batch: a thread takes one (pair, sign, triangle)
// and sets the triangle up in every view, so the perturbed corners (index,
// parameter and sign reads) are formed once for all the views.  Items are
// numbered (pair, view).
__global__ void __launch_bounds__(256) k_setup_b1(BatchArgs b, BatchOne one) {
    const DScene& sc = one.sc;
    const BScene& S = b.scenes[0];
    const long long per_sign = ((long long)sc.n_tris + 255) >> 8;
    const long long blk = blockIdx.x;
    const int pair = (int)(blk / (2 * per_sign));
    const long long rem = blk - (long long)pair * 2 * per_sign;
    const int s = (int)(rem / per_sign);
    const int t = (int)((rem - s * per_sign) * 256 + threadIdx.x);
    if (t >= sc.n_tris) return;
    float p[9];
    tri_positions(sc, S.theta, S.bits + (long long)pair * sc.words, S.eps[0], s == 0 ? 1.0f : -1.0f, t, nullptr, p);
    for (int v = 0; v < one.n_views; ++v) {
        const BItem& I = b.items[pair * one.n_views + v];
        const DView& vw = one.views[v];
        const int tiles = vw.tiles_x * vw.tiles_y;
        setup_tri_at(vw, p, t, b.recR + I.rec_off + (long long)s * sc.n_tris,
                     b.recS + I.rec_off + (long long)s * sc.n_tris, b.counts + I.cnt_off + (long long)s * tiles,
                     b.bins + I.bin_off + (long long)s * tiles * I.cap, b.tile, I.cap, b.spn + 2 * (I.sp_off + s),
                     b.spill + (I.sp_off + s) * SPILL_CAP);
    }
}

// Raster / shade / scatter of every (scene, pair, view, tile) unit in one
// launch: one workgroup per unit, units in the XCD-aware order of
// xcd_tile(), items of the costliest scenes first.
// One tile unit of the batched launch: the job of item I (scene Sc, whose
// constants sc and view vw the caller resolves) and the tile body.
template <int TILE>
__device__ __forceinline__ void tile_b_unit(const BatchArgs& b, const BItem& I, const BScene& Sc, const DScene& sc,
                                            const DView& vw, long long w, TileShared<TILE, 0>& S) {
    int tiles = vw.tiles_x * vw.tiles_y;
    TileJob J;
    J.sc = &sc;
    J.vw = &vw;
    J.theta = Sc.theta;
    J.pb = Sc.bits + (long long)I.pair * sc.words;
    J.eps = Sc.eps;
    J.sgn[0] = 1.0f;
    J.sgn[1] = -1.0f;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        J.recR[s] = b.recR + I.rec_off + (long long)s * sc.n_tris;
        J.recS[s] = b.recS + I.rec_off + (long long)s * sc.n_tris;
        J.counts[s] = b.counts + I.cnt_off + (long long)s * tiles;
        J.bins[s] = b.bins + I.bin_off + (long long)s * tiles * I.cap;
        J.spn[s] = b.spn + 2 * (I.sp_off + s);
        J.spill[s] = b.spill + (I.sp_off + s) * SPILL_CAP;
    }
    J.cap = I.cap;
    J.tile = (int)(w - I.tile0);
    J.stats = b.stats;
    J.targets = Sc.targets + vw.tgt_off;
    J.img = 0;
    J.Rp = Sc.R + (long long)I.pair * sc.G;
    J.K = Sc.K;
    J.act_pos = Sc.act_pos;
    J.any_act = Sc.any_act;
    J.act_cls = Sc.act_cls;
    J.out_rgb = nullptr;
    J.out_id = nullptr;
    J.out_uv = nullptr;
    J.partial = nullptr;
    J.qtot = nullptr;
    tile_body<TILE, 0>(J, S);
}

// Item of tile unit w (uniform).
__device__ __forceinline__ int unit_item(const BatchArgs& b, long long w) {
    int it = last_le((const char*)&b.items[0].tile0, sizeof(BItem), b.n_items, w);
    return __builtin_amdgcn_readfirstlane(it);
}

template <int TILE>
__global__ void __launch_bounds__((TILE * TILE > 256) ? 256 : TILE * TILE, TILE > 16 ? 1 : TILE_MIN_WAVES) k_tile_b(BatchArgs b) {
    __shared__ TileShared<TILE, 0> S;
    long long w = b.unit0 + xcd_tile(blockIdx.x, gridDim.x);
    if (w >= b.total_tiles) return;
    const BItem& I = b.items[unit_item(b, w)];
    const BScene& Sc = b.scenes[I.scene];
    tile_b_unit<TILE>(b, I, Sc, Sc.sc, b.views[I.view], w, S);
}

// The same launch for a one-scene batch, with the scene's constants and
// views in the kernel arguments: the body reads them with scalar loads
// instead of vector loads that compete with the texel reads.
// Unit of position L of a one-scene launch in (view, tile, pair) order.
// The units of the pairs of one tile then follow each other, so they run
// at about the same time on one XCD and share its L2 for what they have in
// common: the texels and target pixels of the tile.
__device__ __forceinline__ long long pair_interleaved(const BatchOne& one, long long L) {
    const long long P = one.il_pairs;
    int v = 0;
    while (v + 1 < one.n_views && L >= P * one.tsum[v + 1]) ++v;
    const unsigned r = (unsigned)(L - P * one.tsum[v]);
    const unsigned t = r / (unsigned)P, p = r - t * (unsigned)P;
    return (long long)p * one.tsum[one.n_views] + one.tsum[v] + t;
}

template <int TILE>
__global__ void __launch_bounds__((TILE * TILE > 256) ? 256 : TILE * TILE, TILE > 16 ? 1 : TILE_MIN_WAVES) k_tile_b1(BatchArgs b, BatchOne one) {
    __shared__ TileShared<TILE, 0> S;
    long long w = b.unit0 + xcd_tile(blockIdx.x, gridDim.x);
    if (w >= b.total_tiles) return;
    if (one.il_pairs > 1) w = pair_interleaved(one, w);
    const BItem& I = b.items[unit_item(b, w)];
    const BScene& Sc = b.scenes[I.scene];
    tile_b_unit<TILE>(b, I, Sc, one.sc, one.views[I.view], w, S);
}

// Fold and step over the groups of every scene: each scene starts on a
// block boundary.
__global__ void __launch_bounds__(256) k_fold_b(BatchArgs b) {
    long long blk = blockIdx.x;
    int si = last_le((const char*)&b.scenes[0].group_blk0, sizeof(BScene), b.n_scenes, blk);
    si = __builtin_amdgcn_readfirstlane(si);
    const BScene& S = b.scenes[si];
    long long g = (blk - S.group_blk0) * 256 + threadIdx.x;
    if (g >= S.sc.G) return;
    fold_group(S.sc, g, S.R, S.bits, b.n_pairs, S.eps, S.Q);
}

__global__ void __launch_bounds__(256) k_step_b(BatchArgs b) {
    long long blk = blockIdx.x;
    int si = last_le((const char*)&b.scenes[0].group_blk0, sizeof(BScene), b.n_scenes, blk);
    si = __builtin_amdgcn_readfirstlane(si);
    const BScene& S = b.scenes[si];
    long long g = (blk - S.group_blk0) * 256 + threadIdx.x;
    if (g >= S.sc.G) return;
    unsigned t = *b.step;
    if (t < 1u) t = 1u;                      // Adam steps count from 1
    int ti = (int)min(t, (unsigned)b.n_bc) - 1;
    step_group(S.sc, g, S.eps, S.lr, b.n_pairs, b.oc, b.bc1[ti], b.bc2[ti], 0, (float*)S.theta, S.m, S.v, S.Q,
               S.K, nullptr, b.stats);
}

// Fold and step fused, for a descent over at most 8 pairs: each group's
// per-pair sums are read once and every parameter of the group goes from
// its sum straight to the update, so the fixed-point sums Q are not written
// and read back in between.  Q_i + sum_n s_i^(n) R_g^(n) is the value the
// fold would leave in Q; it is used as step_group uses Q, and Q, R and K are
// left zero as the two kernels leave them.
// q_zero: Q is known to be zero (not read).
__device__ __forceinline__ void fold_step_group(const DScene& sc, long long g, long long* __restrict__ R,
                                                const uint32_t* __restrict__ bits, int n_pairs, const float* eps,
                                                const float* lr, const OptimConst& oc, float bc1, float bc2,
                                                float* __restrict__ theta, float* __restrict__ m,
                                                float* __restrict__ v, long long* __restrict__ Q,
                                                unsigned* __restrict__ K, unsigned long long* __restrict__ stats,
                                                int q_zero) {
    long long r[8];
    bool any = false;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        r[j] = (j < n_pairs) ? R[(long long)j * sc.G + g] : 0;
        any = any || r[j] != 0;
    }
    unsigned kc = K[g];
    double D = (oc.averaging == 0) ? (double)kc : (double)n_pairs;
    for_params(sc, g, [&](long long i, int b) {
        float e = eps[b];
        long long q0 = q_zero ? 0ll : Q[i];
        long long acc = 0;
        if (any && e != 0.0f) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (r[j] == 0) continue;
                acc += (sign_of(bits + (long long)j * sc.words, i) > 0) ? r[j] : -r[j];
            }
        }
        long long qv = q0 + acc;
        float gi = 0.0f;
        if (e != 0.0f && D != 0.0)
            gi = (float)(((double)qv * (1.0 / 4294967296.0)) / (2.0 * (double)e * D));
        if (q0 != 0) Q[i] = 0;
        if (e == 0.0f) return;
        if (oc.averaging == 0 && kc == 0u) return;
        if (!(fabsf(gi) <= 3.402823466e38f)) {
            atomicAdd(&stats[ST_NONFINITE], 1ull);
            return;
        }
        float l = lr[b];
        if (oc.kind == 1) {
            theta[i] = theta[i] - l * gi;
        } else {
            float mi = oc.b1 * m[i] + oc.omb1 * gi;
            float vi = oc.b2 * v[i] + oc.omb2 * (gi * gi);
            m[i] = mi;
            v[i] = vi;
            float mh = mi / bc1;
            float vh = vi / bc2;
            theta[i] = theta[i] - l * (mh / (sqrtf(vh) + oc.eps_hat));
        }
    });
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (r[j] != 0) R[(long long)j * sc.G + g] = 0;
    K[g] = 0u;
}

__global__ void __launch_bounds__(256) k_fold_step_b(BatchArgs b) {
    long long blk = blockIdx.x;
    int si = last_le((const char*)&b.scenes[0].group_blk0, sizeof(BScene), b.n_scenes, blk);
    si = __builtin_amdgcn_readfirstlane(si);
    const BScene& S = b.scenes[si];
    long long g = (blk - S.group_blk0) * 256 + threadIdx.x;
    if (g >= S.sc.G) return;
    unsigned t = *b.step;
    if (t < 1u) t = 1u;                      // Adam steps count from 1
    int ti = (int)min(t, (unsigned)b.n_bc) - 1;
    fold_step_group(S.sc, g, S.R, S.bits, b.n_pairs, S.eps, S.lr, b.oc, b.bc1[ti], b.bc2[ti], (float*)S.theta,
                    S.m, S.v, S.Q, S.K, b.stats, b.q_zero);
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
    if (mode == 0) hipLaunchKernelGGL((k_tile<TILE, 0, false>), grid, block, 0, st, a);
    else if (mode == 1) hipLaunchKernelGGL((k_tile<TILE, 1, false>), grid, block, 0, st, a);
    else if (mode == 2) hipLaunchKernelGGL((k_tile<TILE, 2, false>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_tile<TILE, 3, false>), grid, block, 0, st, a);
}

template <int TILE>
static void launch_tile_deep_t(hipStream_t st, const TileArgs& a, int mode, dim3 grid) {
    dim3 block(TILE * TILE);
    if (mode == 0) hipLaunchKernelGGL((k_tile<TILE, 0, true>), grid, block, 0, st, a);
    else if (mode == 1) hipLaunchKernelGGL((k_tile<TILE, 1, true>), grid, block, 0, st, a);
    else if (mode == 2) hipLaunchKernelGGL((k_tile<TILE, 2, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_tile<TILE, 3, true>), grid, block, 0, st, a);
}

hipError_t launch_tile(hipStream_t st, const TileArgs& a, int tile, int mode, int n_items, int max_tiles) {
    dim3 grid((unsigned)max_tiles, (unsigned)n_items);
    if (a.sc.layers > 0) {
        if (tile == 8) launch_tile_deep_t<8>(st, a, mode, grid);
        else if (tile == 16) launch_tile_deep_t<16>(st, a, mode, grid);
        else return hipErrorInvalidValue;           // deep buffers fit LDS for tiles <= 16
        return hipGetLastError();
    }
    if (tile == 8) launch_tile_t<8>(st, a, mode, grid);
    else if (tile == 16) launch_tile_t<16>(st, a, mode, grid);
    else launch_tile_t<32>(st, a, mode, grid);
    return hipGetLastError();
}

hipError_t launch_subdiv(hipStream_t st, const DScene& sc, const DPert& pert, const float* theta, int n_pairs,
                         int nsign, float sgn0, float sgn1, float* fpos) {
    dim3 grid((unsigned)((sc.n_verts + 255) / 256), (unsigned)(n_pairs * nsign));
    hipLaunchKernelGGL(k_subdiv, grid, dim3(256), 0, st, sc, pert, theta, nsign, sgn0, sgn1, fpos);
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

hipError_t launch_broadcast(hipStream_t st, const FoldArgs& a) {
    dim3 grid((unsigned)((a.sc.G + 255) / 256));
    hipLaunchKernelGGL(k_broadcast, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_zero64(hipStream_t st, long long* p, int n) {
    hipLaunchKernelGGL(k_zero64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
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

hipError_t launch_batch_signs(hipStream_t st, const BatchArgs& b) {
    hipLaunchKernelGGL(k_signs_b, dim3((unsigned)b.sign_blocks), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_batch_setup(hipStream_t st, const BatchArgs& b, const BatchOne* one, long long blk0,
                              long long nblk) {
    if (nblk <= 0) return hipSuccess;
    if (one && blk0 == 0 && nblk == b.setup_blocks) {
        // the whole setup of a one-scene batch: a thread per (pair, sign, triangle)
        const long long blocks = (long long)b.n_pairs * 2 * (((long long)one->sc.n_tris + 255) >> 8);
        hipLaunchKernelGGL(k_setup_b1, dim3((unsigned)blocks), dim3(256), 0, st, b, *one);
        return hipGetLastError();
    }
    BatchArgs a = b;
    a.unit0 = blk0;
    hipLaunchKernelGGL(k_setup_b, dim3((unsigned)nblk), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_tile(hipStream_t st, const BatchArgs& b, const BatchOne* one, long long w0, long long n) {
    if (n <= 0) return hipSuccess;
    int tb = (b.tile * b.tile > 256) ? 256 : b.tile * b.tile;
    unsigned grid = (unsigned)n;
    BatchArgs a = b;
    a.unit0 = w0;
    if (one) {
        // the interleaved order is a permutation of all units: a launch of
        // part of them keeps unit order
        BatchOne o = *one;
        if (w0 != 0 || n != b.total_tiles) o.il_pairs = 1;
        if (a.tile == 8) hipLaunchKernelGGL(k_tile_b1<8>, dim3(grid), dim3(tb), 0, st, a, o);
        else if (a.tile == 16) hipLaunchKernelGGL(k_tile_b1<16>, dim3(grid), dim3(tb), 0, st, a, o);
        else hipLaunchKernelGGL(k_tile_b1<32>, dim3(grid), dim3(tb), 0, st, a, o);
    } else {
        if (a.tile == 8) hipLaunchKernelGGL(k_tile_b<8>, dim3(grid), dim3(tb), 0, st, a);
        else if (a.tile == 16) hipLaunchKernelGGL(k_tile_b<16>, dim3(grid), dim3(tb), 0, st, a);
        else hipLaunchKernelGGL(k_tile_b<32>, dim3(grid), dim3(tb), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_batch_fold(hipStream_t st, const BatchArgs& b) {
    hipLaunchKernelGGL(k_fold_b, dim3((unsigned)b.group_blocks), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_batch_fold_step(hipStream_t st, const BatchArgs& b) {
    hipLaunchKernelGGL(k_fold_step_b, dim3((unsigned)b.group_blocks), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_batch_step(hipStream_t st, const BatchArgs& b) {
    hipLaunchKernelGGL(k_step_b, dim3((unsigned)b.group_blocks), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_batch_end(hipStream_t st, const BatchArgs& b) {
    hipLaunchKernelGGL(k_batch_end, dim3(1), dim3(1), 0, st, (unsigned*)b.step);
    return hipGetLastError();
}
