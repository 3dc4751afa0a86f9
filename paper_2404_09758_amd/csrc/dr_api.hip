// dr_api.hip -- host side of the C ABI declared in include/dr.h.
//
// Owns the per-context scratch memory (sign bits, triangle records, bins,
// per-pair group sums), validates every argument on the host before
// launching, and orders the kernels of dr_kernels.hip on the context's
// stream.  Scratch buffers grow on demand and are reused; the bin counters
// and the per-pair sums are left zeroed by the kernels that consume them,
// so no clearing pass is needed between calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dr.h"
#include "dr_launch.h"

enum { K_SIGNS = 0, K_SETUP = 1, K_TILE = 2, K_FOLD = 3, K_STEP = 4 };

// Event pairs recorded around launches while enabled.
struct Timer {
    bool on = false;
    std::vector<hipEvent_t> free_;
    std::vector<hipEvent_t> pending[5][2];        // [kind][begin/end]

    hipEvent_t take() {
        if (!free_.empty()) {
            hipEvent_t e = free_.back();
            free_.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }

    // Runs one launch on stream st, bracketed by events when enabled.
    template <typename F>
    hipError_t run(hipStream_t st, int kind, F launch) {
        if (!on) return launch();
        hipEvent_t b = take(), e = take();
        if (!b || !e) return hipErrorOutOfMemory;
        hipError_t r = hipEventRecord(b, st);
        if (r != hipSuccess) return r;
        r = launch();
        if (r != hipSuccess) return r;
        r = hipEventRecord(e, st);
        pending[kind][0].push_back(b);
        pending[kind][1].push_back(e);
        return r;
    }

    // Sums the durations (the stream must be synchronised).
    hipError_t read(dr_timing_t* out, bool reset) {
        double ms[5] = {0, 0, 0, 0, 0};
        int64_t n[5] = {0, 0, 0, 0, 0};
        for (int k = 0; k < 5; ++k) {
            for (size_t i = 0; i < pending[k][0].size(); ++i) {
                float t = 0.0f;
                hipError_t r = hipEventElapsedTime(&t, pending[k][0][i], pending[k][1][i]);
                if (r != hipSuccess) return r;
                ms[k] += t;
                n[k] += 1;
            }
            if (reset)
                for (int j = 0; j < 2; ++j) {
                    for (hipEvent_t e : pending[k][j]) free_.push_back(e);
                    pending[k][j].clear();
                }
        }
        out->signs_ms = ms[K_SIGNS]; out->signs_launches = n[K_SIGNS];
        out->setup_ms = ms[K_SETUP]; out->setup_launches = n[K_SETUP];
        out->tile_ms = ms[K_TILE]; out->tile_launches = n[K_TILE];
        out->fold_ms = ms[K_FOLD]; out->fold_launches = n[K_FOLD];
        out->step_ms = ms[K_STEP]; out->step_launches = n[K_STEP];
        return hipSuccess;
    }

    void destroy() {
        for (int k = 0; k < 5; ++k)
            for (int j = 0; j < 2; ++j) {
                for (hipEvent_t e : pending[k][j]) (void)hipEventDestroy(e);
                pending[k][j].clear();
            }
        for (hipEvent_t e : free_) (void)hipEventDestroy(e);
        free_.clear();
    }
};

struct dr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    dr_scene hs{};
    DScene sc{};
    dr_tuning tune{16, 256, 1};
    uint32_t scene_index = 0;
    std::string err;
    TriR* recR = nullptr;
    TriS* recS = nullptr;
    long long rec_slots = 0;
    unsigned* counts = nullptr;
    unsigned* bins = nullptr;
    long long tile_slots = 0;       // slots * max_tiles allocated
    long long bin_entries = 0;      // tile_slots * cap allocated
    unsigned* spn = nullptr;        // [slots, 2] spill counters
    long long spn_words = 0;
    unsigned long long* spill = nullptr;   // [slots, SPILL_CAP] spill lists
    long long spill_entries = 0;
    long long* R = nullptr;
    long long R_pairs = 0;
    uint32_t* bits = nullptr;
    long long bits_words = 0;
    long long* qtot = nullptr;
    long long qtot_pairs = 0;
    double* partials = nullptr;
    long long partial_slots = 0;
    unsigned long long* stats = nullptr;
    int* tri_rowptr = nullptr;      // subdivision surface: control vertices per triangle
    int* tri_cols = nullptr;
    float* fpos = nullptr;          // tessellated positions per (pair, sign)
    long long fpos_slots = 0;
    // adaptive bin capacity: the largest bin of the last estimate, read back
    // asynchronously into pinned memory
    int adapt = 1;
    unsigned long long* h_seen = nullptr;
    hipEvent_t ev_seen = nullptr;
    bool seen_pending = false;
    Timer timer;
};

static dr_status fail(dr_ctx* c, dr_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

#define HIPCHK(c, expr)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail((c), DR_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

static bool finite_nonneg(float x) { return std::isfinite(x) && x >= 0.0f; }

static hipError_t scratch_lookup(int dev, void** out);

static dr_status device_guard(dr_ctx* c) {
    int cur = -1;
    HIPCHK(c, hipGetDevice(&cur));
    if (cur != c->device) HIPCHK(c, hipSetDevice(c->device));
    return DR_OK;
}

// ------------------------------------------------------------ scratch --

template <typename T>
static dr_status grow(dr_ctx* c, T** p, long long* have, long long need, size_t elem, bool zero) {
    if (need <= *have) return DR_OK;
    if (*p) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipFree(*p));
        *p = nullptr;
        *have = 0;
    }
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)need * elem) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, DR_E_OOM, "hipMalloc of " + std::to_string((size_t)need * elem) + " bytes failed");
    }
    if (zero) HIPCHK(c, hipMemsetAsync(q, 0, (size_t)need * elem, c->stream));
    *p = (T*)q;
    *have = need;
    return DR_OK;
}

static dr_status ensure_raster(dr_ctx* c, long long slots, int max_tiles) {
    long long have = c->rec_slots;
    dr_status s = grow(c, &c->recR, &have, slots * c->sc.n_tris, sizeof(TriR), false);
    if (s) return s;
    have = c->rec_slots;
    s = grow(c, &c->recS, &have, slots * c->sc.n_tris, sizeof(TriS), false);
    if (s) return s;
    if (slots * c->sc.n_tris > c->rec_slots) c->rec_slots = slots * c->sc.n_tris;
    s = grow(c, &c->counts, &c->tile_slots, slots * (long long)max_tiles, sizeof(unsigned), true);
    if (s) return s;
    s = grow(c, &c->spn, &c->spn_words, 2 * slots, sizeof(unsigned), true);
    if (s) return s;
    s = grow(c, &c->spill, &c->spill_entries, slots * (long long)SPILL_CAP, sizeof(unsigned long long), false);
    if (s) return s;
    return grow(c, &c->bins, &c->bin_entries, slots * (long long)max_tiles * c->tune.bin_capacity,
                sizeof(unsigned), false);
}

// ---------------------------------------------------------- validation --

static dr_status check_view(dr_ctx* c, const dr_view* v, int tile) {
    if (!v) return fail(c, DR_E_INVALID, "view is NULL");
    if (v->width < 1 || v->height < 1 || v->width > 16384 || v->height > 16384)
        return fail(c, DR_E_INVALID, "view size must be in [1, 16384]");
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(v->view_proj[i])) return fail(c, DR_E_INVALID, "view_proj is not finite");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(v->cam_pos[i])) return fail(c, DR_E_INVALID, "cam_pos is not finite");
    if (!std::isfinite(v->near_w)) return fail(c, DR_E_INVALID, "near_w is not finite");
    (void)tile;
    return DR_OK;
}

static DView make_dview(const dr_view& v, int tile, long long tgt_off) {
    DView d;
    d.W = v.width;
    d.H = v.height;
    std::memcpy(d.M, v.view_proj, sizeof(d.M));
    std::memcpy(d.cam, v.cam_pos, sizeof(d.cam));
    d.near_w = v.near_w;
    d.tiles_x = (v.width + tile - 1) / tile;
    d.tiles_y = (v.height + tile - 1) / tile;
    d.tgt_off = tgt_off;
    return d;
}

static dr_status check_eps(dr_ctx* c, const float* eps) {
    if (!eps) return fail(c, DR_E_INVALID, "eps is NULL");
    for (int b = 0; b < 1 + c->sc.n_tex; ++b)
        if (!finite_nonneg(eps[b])) return fail(c, DR_E_INVALID, "eps must be finite and >= 0");
    return DR_OK;
}

static dr_status check_tuning(dr_ctx* c, const dr_tuning* t) {
    if (t->tile_px != 8 && t->tile_px != 16 && t->tile_px != 32)
        return fail(c, DR_E_INVALID, "tile_px must be 8, 16 or 32");
    if (t->bin_capacity < 1 || t->bin_capacity > (1 << 20))
        return fail(c, DR_E_INVALID, "bin_capacity must be in [1, 2^20]");
    if (t->items_per_launch < 0) return fail(c, DR_E_INVALID, "items_per_launch must be >= 0");
    if (c->hs.layers > 0 && t->tile_px > 16)
        return fail(c, DR_E_UNSUPPORTED, "semi-transparent scenes need tile_px 8 or 16");
    return DR_OK;
}

// ------------------------------------------------------------- create --

// Subdivision surface: check the tessellation map and build, per
// tessellated triangle, the ascending list of control vertices its three
// corners combine (the vertex groups a pixel on it credits).
static dr_status setup_subdivision(dr_ctx* c, const dr_scene* s) {
    const long long nv = s->n_verts, nt = s->n_tris;
    std::vector<int> rowptr((size_t)nv + 1), tri((size_t)(3 * nt));
    HIPCHK(c, hipMemcpy(rowptr.data(), s->sub_rowptr, rowptr.size() * sizeof(int), hipMemcpyDeviceToHost));
    if (rowptr[0] != 0) return fail(c, DR_E_INVALID, "sub_rowptr[0] must be 0");
    for (long long j = 0; j < nv; ++j)
        if (rowptr[j + 1] < rowptr[j]) return fail(c, DR_E_INVALID, "sub_rowptr must not decrease");
    const long long nnz = rowptr[nv];
    std::vector<int> cols((size_t)(nnz > 0 ? nnz : 1));
    if (nnz > 0) HIPCHK(c, hipMemcpy(cols.data(), s->sub_cols, (size_t)nnz * sizeof(int), hipMemcpyDeviceToHost));
    for (long long k = 0; k < nnz; ++k)
        if (cols[k] < 0 || cols[k] >= s->n_ctrl) return fail(c, DR_E_INVALID, "sub_cols out of range");
    for (long long j = 0; j < nv; ++j)
        for (long long k = rowptr[j] + 1; k < rowptr[j + 1]; ++k)
            if (cols[k] <= cols[k - 1]) return fail(c, DR_E_INVALID, "sub_cols must ascend within a row");
    HIPCHK(c, hipMemcpy(tri.data(), s->tri, tri.size() * sizeof(int), hipMemcpyDeviceToHost));
    std::vector<int> trp(1, 0), tcols;
    std::vector<int> u;
    for (long long t = 0; t < nt; ++t) {
        u.clear();
        for (int k = 0; k < 3; ++k) {
            int v = tri[(size_t)(3 * t + k)];
            u.insert(u.end(), cols.begin() + rowptr[v], cols.begin() + rowptr[v + 1]);
        }
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        tcols.insert(tcols.end(), u.begin(), u.end());
        if (tcols.size() >= (size_t)0x7FFFFFFF) return fail(c, DR_E_UNSUPPORTED, "tessellation map too large");
        trp.push_back((int)tcols.size());
    }
    if (tcols.empty()) tcols.push_back(0);
    HIPCHK(c, hipMalloc(&c->tri_rowptr, trp.size() * sizeof(int)));
    HIPCHK(c, hipMalloc(&c->tri_cols, tcols.size() * sizeof(int)));
    HIPCHK(c, hipMemcpy(c->tri_rowptr, trp.data(), trp.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->tri_cols, tcols.data(), tcols.size() * sizeof(int), hipMemcpyHostToDevice));
    c->sc.tri_rowptr = c->tri_rowptr;
    c->sc.tri_cols = c->tri_cols;
    return DR_OK;
}

// Subdivision surface: tessellate theta (perturbed as dp says) for
// n_pairs x nsign (pair, sign) slots into fpos (room for n_pairs * nsign *
// n_verts * 3 floats); *out = null for a mesh whose vertices are the
// parameters.
static dr_status tessellate_into(dr_ctx* c, const float* theta, const DPert& dp, int n_pairs, int nsign,
                                 float sgn0, float sgn1, float* fpos, bool timed, const float** out) {
    *out = nullptr;
    if (c->sc.n_ctrl == 0) return DR_OK;
    auto go = [&] { return launch_subdiv(c->stream, c->sc, dp, theta, n_pairs, nsign, sgn0, sgn1, fpos); };
    if (timed) HIPCHK(c, c->timer.run(c->stream, K_SETUP, go));
    else HIPCHK(c, go());
    *out = fpos;
    return DR_OK;
}

// The same into the context's own buffer, grown as needed.
static dr_status tessellate(dr_ctx* c, const float* theta, const DPert& dp, int n_pairs, int nsign, float sgn0,
                            float sgn1, const float** out) {
    *out = nullptr;
    if (c->sc.n_ctrl == 0) return DR_OK;
    dr_status s = grow(c, &c->fpos, &c->fpos_slots, (long long)n_pairs * nsign,
                       (size_t)c->sc.n_verts * 3 * sizeof(float), false);
    if (s) return s;
    return tessellate_into(c, theta, dp, n_pairs, nsign, sgn0, sgn1, c->fpos, true, out);
}

extern "C" dr_status dr_create(dr_ctx** out, const dr_scene* s, const dr_tuning* tune, void* stream) {
    if (!out || !s) return DR_E_INVALID;
    *out = nullptr;
    if (s->n_verts < 1 || s->n_tris < 1) return DR_E_INVALID;
    if (!s->tri || !s->corner_uv) return DR_E_INVALID;
    if (s->n_tex < 0 || s->n_tex > DR_MAX_TEX) return DR_E_INVALID;
    if (s->shading < DR_UNLIT || s->shading > DR_GGX) return DR_E_INVALID;
    if (s->tex_mode != DR_TEX_FOOTPRINT && s->tex_mode != DR_TEX_NEAREST) return DR_E_INVALID;
    if (s->shading != DR_UNLIT && s->n_tex < 1) return DR_E_INVALID;
    if (s->layers < 0 || s->layers > DR_MAX_LAYERS) return DR_E_INVALID;
    if (s->layers > 0 && s->n_tex < 1) return DR_E_INVALID;
    if (s->n_ctrl < 0) return DR_E_INVALID;
    if (s->n_ctrl > 0 && (!s->sub_rowptr || !s->sub_cols || !s->sub_w)) return DR_E_INVALID;
    if (s->n_ctrl > 0 && s->layers > 0) return DR_E_UNSUPPORTED;
    const long long n_vg = s->n_ctrl > 0 ? s->n_ctrl : s->n_verts;     // position groups
    long long d = 3ll * n_vg;
    for (int t = 0; t < s->n_tex; ++t) {
        if (s->tex_w[t] < 1 || s->tex_h[t] < 1 || s->tex_w[t] > 32768 || s->tex_h[t] > 32768) return DR_E_INVALID;
        int want = (t == 2) ? 1 : (t == 0 && s->layers > 0 ? 4 : 3);
        if (s->tex_c[t] != want) return DR_E_INVALID;
        d += (long long)s->tex_w[t] * s->tex_h[t] * s->tex_c[t];
    }
    if (d >= (1ll << 36)) return DR_E_INVALID;
    // group indices are 32-bit keys in the tile-local aggregation tables
    long long groups = n_vg;
    for (int t = 0; t < s->n_tex; ++t) groups += (long long)s->tex_w[t] * s->tex_h[t];
    if (groups >= 0xFFFFFFFFll) return DR_E_UNSUPPORTED;
    dr_ctx* c = new (std::nothrow) dr_ctx();
    if (!c) return DR_E_OOM;
    c->hs = *s;
    c->stream = (hipStream_t)stream;
    if (tune) {
        if (check_tuning(c, tune)) {
            delete c;
            return DR_E_INVALID;
        }
        c->tune = *tune;
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return DR_E_HIP;
    }
    DScene& sc = c->sc;
    sc.n_verts = s->n_verts;
    sc.n_tris = s->n_tris;
    sc.tri = s->tri;
    sc.cuv = s->corner_uv;
    sc.n_tex = s->n_tex;
    sc.n_vg = (int)n_vg;
    sc.n_ctrl = s->n_ctrl;
    sc.sub_rowptr = s->sub_rowptr;
    sc.sub_cols = s->sub_cols;
    sc.sub_w = s->sub_w;
    sc.tri_rowptr = nullptr;
    sc.tri_cols = nullptr;
    long long off = 3ll * n_vg;
    long long goff = n_vg;
    sc.n_cls = 0;
    for (int t = 0; t < DRD_MAX_TEX; ++t) {
        sc.tex_w[t] = sc.tex_h[t] = sc.tex_c[t] = 0;
        sc.tex_off[t] = 0;
        sc.tex_cls[t] = -1;
        sc.cls_w[t] = sc.cls_h[t] = 0;
        sc.cls_goff[t] = 0;
    }
    for (int t = 0; t < s->n_tex; ++t) {
        sc.tex_w[t] = s->tex_w[t];
        sc.tex_h[t] = s->tex_h[t];
        sc.tex_c[t] = s->tex_c[t];
        sc.tex_off[t] = off;
        off += (long long)s->tex_w[t] * s->tex_h[t] * s->tex_c[t];
        int cls = -1;
        for (int k = 0; k < sc.n_cls; ++k)
            if (sc.cls_w[k] == s->tex_w[t] && sc.cls_h[k] == s->tex_h[t]) cls = k;
        if (cls < 0) {
            cls = sc.n_cls++;
            sc.cls_w[cls] = s->tex_w[t];
            sc.cls_h[cls] = s->tex_h[t];
            sc.cls_goff[cls] = goff;
            goff += (long long)s->tex_w[t] * s->tex_h[t];
        }
        sc.tex_cls[t] = cls;
    }
    sc.shading = s->shading;
    sc.tex_mode = s->tex_mode;
    sc.layers = s->layers;
    for (int i = 0; i < 3; ++i) {
        sc.light[i] = s->light_dir[i];
        sc.light_rgb[i] = s->light_rgb[i];
    }
    sc.ambient = s->ambient;
    sc.diffuse = s->diffuse;
    sc.d = off;
    sc.G = goff;
    sc.words = (int)((off + 31) / 32);
    if (hipMalloc(&c->stats, ST_COUNT * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->stats, 0, ST_COUNT * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        if (c->stats) (void)hipFree(c->stats);
        delete c;
        return DR_E_OOM;
    }
    // every vertex index must address the vertex array
    unsigned long long bad = 0;
    bool ok = launch_check_tri(c->stream, s->tri, 3ll * s->n_tris, s->n_verts, c->stats + ST_BAD_INDEX) ==
                  hipSuccess &&
              hipMemcpyAsync(&bad, c->stats + ST_BAD_INDEX, sizeof(bad), hipMemcpyDeviceToHost, c->stream) ==
                  hipSuccess &&
              hipStreamSynchronize(c->stream) == hipSuccess;
    if (!ok || bad != 0) {
        (void)hipGetLastError();
        (void)hipFree(c->stats);
        delete c;
        return ok ? DR_E_INVALID : DR_E_HIP;
    }
    if (s->n_ctrl > 0) {
        dr_status st = setup_subdivision(c, s);
        if (st) {
            (void)hipGetLastError();
            if (c->tri_rowptr) (void)hipFree(c->tri_rowptr);
            if (c->tri_cols) (void)hipFree(c->tri_cols);
            (void)hipFree(c->stats);
            delete c;
            return st;
        }
    }
    // the allocation-free estimate's scratch array on this device (its
    // address is needed by dr_estimate_grad_noalloc only; a failed lookup
    // is reported by that call)
    {
        void* p = nullptr;
        (void)scratch_lookup(c->device, &p);
    }
    *out = c;
    return DR_OK;
}

extern "C" dr_status dr_destroy(dr_ctx* c) {
    if (!c) return DR_E_INVALID;
    (void)hipStreamSynchronize(c->stream);
    if (c->h_seen) (void)hipHostFree(c->h_seen);
    if (c->ev_seen) (void)hipEventDestroy(c->ev_seen);
    void* ptrs[] = {c->recR, c->recS, c->counts, c->bins, c->spn, c->spill, c->R, c->bits, c->stats, c->partials,
                    c->qtot, c->tri_rowptr, c->tri_cols, c->fpos};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    c->timer.destroy();
    delete c;
    return DR_OK;
}

extern "C" dr_status dr_set_stream(dr_ctx* c, void* stream) {
    if (!c) return DR_E_INVALID;
    c->stream = (hipStream_t)stream;
    return DR_OK;
}

extern "C" dr_status dr_set_tuning(dr_ctx* c, const dr_tuning* t) {
    if (!c || !t) return fail(c, DR_E_INVALID, "NULL argument");
    dr_status s = check_tuning(c, t);
    if (s) return s;
    if (t->bin_capacity != c->tune.bin_capacity) {
        // the bin array is indexed with the capacity: reallocate on next use
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->bins) HIPCHK(c, hipFree(c->bins));
        c->bins = nullptr;
        c->bin_entries = 0;
    }
    c->tune = *t;
    return DR_OK;
}

extern "C" dr_status dr_set_scene_index(dr_ctx* c, uint32_t scene_index) {
    if (!c) return DR_E_INVALID;
    c->scene_index = scene_index;
    return DR_OK;
}

extern "C" int64_t dr_param_count(const dr_ctx* c) { return c ? c->sc.d : -1; }
extern "C" int64_t dr_group_count(const dr_ctx* c) { return c ? c->sc.G : -1; }

// -------------------------------------------------------------- signs --

// Sign bits of `pairs` pairs, plus a spare word that the texture sampling
// may read past the last pair's last word.
static dr_status ensure_bits(dr_ctx* c, long long pairs) {
    return grow(c, &c->bits, &c->bits_words, pairs * c->sc.words + 1, sizeof(uint32_t), false);
}

extern "C" dr_status dr_signs(dr_ctx* c, uint64_t seed, uint32_t step, uint32_t pair, uint32_t scene,
                              uint32_t* bits) {
    if (!c) return DR_E_INVALID;
    if (!bits) return fail(c, DR_E_INVALID, "bits is NULL");
    dr_status s = device_guard(c);
    if (s) return s;
    HIPCHK(c, c->timer.run(c->stream, K_SIGNS, [&] { return launch_signs(c->stream, seed, step, pair, scene, c->sc.d, c->sc.words, 1, bits); }));
    return DR_OK;
}

// ------------------------------------------------------------- render --

extern "C" dr_status dr_render(dr_ctx* c, const float* theta, const dr_view* view, const dr_perturb* pert,
                               float* rgb, uint32_t* id, float* uv) {
    if (!c) return DR_E_INVALID;
    if (!theta) return fail(c, DR_E_INVALID, "theta is NULL");
    int tile = c->tune.tile_px;
    dr_status s = check_view(c, view, tile);
    if (s) return s;
    if (pert) {
        if (pert->sign != 1 && pert->sign != -1) return fail(c, DR_E_INVALID, "pert->sign must be +1 or -1");
        s = check_eps(c, pert->eps);
        if (s) return s;
    }
    s = device_guard(c);
    if (s) return s;
    DView dv = make_dview(*view, tile, 0);
    int max_tiles = dv.tiles_x * dv.tiles_y;
    s = ensure_raster(c, 1, max_tiles);
    if (s) return s;
    DPert dp;
    dp.bits = nullptr;
    for (int b = 0; b <= DRD_MAX_TEX; ++b) dp.eps[b] = 0.0f;
    float sg = 1.0f;
    if (pert) {
        s = ensure_bits(c, 1);
        if (s) return s;
        HIPCHK(c, c->timer.run(c->stream, K_SIGNS, [&] {
            return launch_signs(c->stream, pert->seed, pert->step, pert->pair, pert->scene_index, c->sc.d,
                                c->sc.words, 1, c->bits);
        }));
        dp.bits = c->bits;
        for (int b = 0; b < 1 + c->sc.n_tex; ++b) dp.eps[b] = pert->eps[b];
        sg = (float)pert->sign;
    }
    SetupArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.sc = c->sc;
    sa.views.v[0] = dv;
    sa.pert = dp;
    sa.theta = theta;
    sa.n_views = 1;
    sa.item0 = 0;
    sa.nsign = 1;
    sa.sgn[0] = sg;
    sa.sgn[1] = sg;
    sa.tile = tile;
    sa.cap = c->tune.bin_capacity;
    sa.max_tiles = max_tiles;
    sa.recR = c->recR;
    sa.recS = c->recS;
    sa.counts = c->counts;
    sa.bins = c->bins;
    sa.spn = c->spn;
    sa.spill = c->spill;
    s = tessellate(c, theta, dp, 1, 1, sg, sg, &sa.fpos);
    if (s) return s;
    HIPCHK(c, c->timer.run(c->stream, K_SETUP, [&] { return launch_setup(c->stream, sa, 1); }));
    TileArgs ta;
    std::memset(&ta, 0, sizeof(ta));
    ta.sc = c->sc;
    ta.views.v[0] = dv;
    ta.pert = dp;
    ta.theta = theta;
    ta.n_views = 1;
    ta.item0 = 0;
    ta.nsign = 1;
    ta.sgn[0] = sg;
    ta.sgn[1] = sg;
    ta.cap = c->tune.bin_capacity;
    ta.max_tiles = max_tiles;
    ta.recR = c->recR;
    ta.recS = c->recS;
    ta.counts = c->counts;
    ta.bins = c->bins;
    ta.spn = c->spn;
    ta.spill = c->spill;
    ta.stats = c->stats;
    ta.out_rgb = rgb;
    ta.out_id = id;
    ta.out_uv = uv;
    HIPCHK(c, c->timer.run(c->stream, K_TILE, [&] { return launch_tile(c->stream, ta, tile, 1, 1, max_tiles); }));
    return DR_OK;
}

// ----------------------------------------------------------- estimate --

// Bins that overflowed in an earlier estimate: raise the capacity to the
// next power of two above 1.5x the largest bin seen.  The figure is read
// back asynchronously; if it has not arrived yet the check waits for the
// next call.  Results never depend on the capacity, only the speed does.
static dr_status adapt_capacity(dr_ctx* c) {
    if (!c->adapt || !c->seen_pending) return DR_OK;
    if (hipEventQuery(c->ev_seen) != hipSuccess) {
        (void)hipGetLastError();
        return DR_OK;
    }
    c->seen_pending = false;
    unsigned long long mb = *c->h_seen;
    if (mb <= (unsigned long long)c->tune.bin_capacity) return DR_OK;
    long long cap = 16;
    while (cap < (long long)(mb + mb / 2 + 1) && cap < (1ll << 16)) cap *= 2;
    if (cap <= c->tune.bin_capacity) return DR_OK;
    dr_tuning t = c->tune;
    t.bin_capacity = (int)cap;
    return dr_set_tuning(c, &t);
}

static dr_status note_bins(dr_ctx* c) {
    if (!c->adapt) return DR_OK;
    if (!c->h_seen) {
        HIPCHK(c, hipHostMalloc((void**)&c->h_seen, sizeof(unsigned long long), hipHostMallocDefault));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_seen, hipEventDisableTiming));
    }
    HIPCHK(c, hipMemcpyAsync(c->h_seen, c->stats + ST_MAX_BIN, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipEventRecord(c->ev_seen, c->stream));
    c->seen_pending = true;
    return DR_OK;
}

// Scratch of one estimate: where the sign bits, triangle records, bins,
// per-pair group sums (or full-image totals) and tessellated positions go,
// the bin capacity and the number of items per raster launch.
struct EstScratch {
    uint32_t* bits = nullptr;
    TriR* recR = nullptr;
    TriS* recS = nullptr;
    unsigned* counts = nullptr;
    unsigned* bins = nullptr;
    unsigned* spn = nullptr;
    unsigned long long* spill = nullptr;
    long long* R = nullptr;
    long long* qtot = nullptr;
    float* fpos = nullptr;
    int cap = 0;
    long long per = 1;
};

// Validated arguments of an estimate.
struct EstPlan {
    DViews dv;
    int max_tiles = 1;
    long long items = 0;
};

static dr_status estimate_check(dr_ctx* c, const float* theta, const dr_view* views, int32_t n_views,
                                const float* targets, int32_t n_pairs, const float* eps, int64_t* Q, uint32_t* K,
                                EstPlan& pl) {
    if (!c) return DR_E_INVALID;
    if (!theta || !targets || !Q || !K || !views) return fail(c, DR_E_INVALID, "NULL array argument");
    if (n_views < 1 || n_views > DR_MAX_VIEWS) return fail(c, DR_E_INVALID, "n_views must be in [1, 16]");
    if (n_pairs < 1 || n_pairs > 65535) return fail(c, DR_E_INVALID, "n_pairs must be in [1, 65535]");
    dr_status s = check_eps(c, eps);
    if (s) return s;
    int tile = c->tune.tile_px;
    std::memset(&pl.dv, 0, sizeof(pl.dv));
    long long tgt_off = 0;
    pl.max_tiles = 1;
    for (int v = 0; v < n_views; ++v) {
        s = check_view(c, &views[v], tile);
        if (s) return s;
        pl.dv.v[v] = make_dview(views[v], tile, tgt_off);
        tgt_off += 3ll * views[v].width * views[v].height;
        pl.max_tiles = std::max(pl.max_tiles, pl.dv.v[v].tiles_x * pl.dv.v[v].tiles_y);
    }
    pl.items = (long long)n_pairs * n_views;
    return DR_OK;
}

// Items per raster launch in the context's tuning (the grid y of the setup
// launch is 2 * items <= 65535).
static long long items_per_launch(const dr_ctx* c, long long items) {
    long long per = c->tune.items_per_launch == 0 ? items : std::min<long long>(items, c->tune.items_per_launch);
    return std::min<long long>(per, 32767);
}

// The context's own scratch, grown as needed.
static dr_status estimate_scratch_ctx(dr_ctx* c, const EstPlan& pl, int32_t n_pairs, bool full, EstScratch& x) {
    x.per = items_per_launch(c, pl.items);
    dr_status s = ensure_raster(c, 2 * x.per, pl.max_tiles);
    if (s) return s;
    s = ensure_bits(c, n_pairs);
    if (s) return s;
    if (full) {
        s = grow(c, &c->qtot, &c->qtot_pairs, n_pairs, sizeof(long long), false);
        if (s) return s;
    } else {
        s = grow(c, &c->R, &c->R_pairs, n_pairs, (size_t)c->sc.G * sizeof(long long), true);
        if (s) return s;
    }
    if (c->sc.n_ctrl > 0) {
        s = grow(c, &c->fpos, &c->fpos_slots, (long long)n_pairs * 2, (size_t)c->sc.n_verts * 3 * sizeof(float),
                 false);
        if (s) return s;
    }
    x.bits = c->bits;
    x.recR = c->recR;
    x.recS = c->recS;
    x.counts = c->counts;
    x.bins = c->bins;
    x.spn = c->spn;
    x.spill = c->spill;
    x.R = c->R;
    x.qtot = c->qtot;
    x.fpos = c->fpos;
    x.cap = c->tune.bin_capacity;
    return DR_OK;
}

// Signs, (tessellation,) setup and tile launches, then the fold or the
// full-image broadcast, on the scratch x.  timed: bracket the launches with
// the context's timing events.
static dr_status estimate_launch(dr_ctx* c, const EstPlan& pl, const float* theta, int32_t n_views,
                                 const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                                 const float* eps, int64_t* Q, uint32_t* K, bool full, bool image,
                                 const EstScratch& x, bool timed) {
    auto run = [&](int kind, auto launch) -> hipError_t {
        return timed ? c->timer.run(c->stream, kind, launch) : launch();
    };
    int tile = c->tune.tile_px;
    const int max_tiles = pl.max_tiles;
    const long long items = pl.items, per = x.per;
    DPert dp;
    dp.bits = x.bits;
    for (int b = 0; b <= DRD_MAX_TEX; ++b) dp.eps[b] = (b < 1 + c->sc.n_tex) ? eps[b] : 0.0f;
    HIPCHK(c, run(K_SIGNS, [&] {
        return launch_signs(c->stream, seed, step, 0u, c->scene_index, c->sc.d, c->sc.words, n_pairs, x.bits);
    }));

    SetupArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.sc = c->sc;
    sa.views = pl.dv;
    sa.pert = dp;
    sa.theta = theta;
    sa.n_views = n_views;
    sa.nsign = 2;
    sa.sgn[0] = 1.0f;
    sa.sgn[1] = -1.0f;
    sa.tile = tile;
    sa.cap = x.cap;
    sa.max_tiles = max_tiles;
    sa.recR = x.recR;
    sa.recS = x.recS;
    sa.counts = x.counts;
    sa.bins = x.bins;
    sa.spn = x.spn;
    sa.spill = x.spill;
    TileArgs ta;
    std::memset(&ta, 0, sizeof(ta));
    ta.sc = c->sc;
    ta.views = pl.dv;
    ta.pert = dp;
    ta.theta = theta;
    ta.n_views = n_views;
    ta.nsign = 2;
    ta.sgn[0] = 1.0f;
    ta.sgn[1] = -1.0f;
    ta.cap = x.cap;
    ta.max_tiles = max_tiles;
    ta.recR = x.recR;
    ta.recS = x.recS;
    ta.counts = x.counts;
    ta.bins = x.bins;
    ta.spn = x.spn;
    ta.spill = x.spill;
    ta.stats = c->stats;
    ta.targets = targets;
    ta.img_grad = image ? 1 : 0;
    ta.R = x.R;
    ta.qtot = x.qtot;
    ta.K = K;
    ta.act_pos = eps[0] != 0.0f;
    ta.any_act = ta.act_pos;
    for (int t = 0; t < c->sc.n_tex; ++t)
        if (eps[1 + t] != 0.0f) {
            ta.act_cls[c->sc.tex_cls[t]] = 1;
            ta.any_act = 1;
        }
    dr_status s = tessellate_into(c, theta, dp, n_pairs, 2, 1.0f, -1.0f, x.fpos, timed, &sa.fpos);
    if (s) return s;
    if (full) HIPCHK(c, launch_zero64(c->stream, x.qtot, n_pairs));
    for (long long i0 = 0; i0 < items; i0 += per) {
        int n = (int)std::min(per, items - i0);
        sa.item0 = (int)i0;
        ta.item0 = (int)i0;
        HIPCHK(c, run(K_SETUP, [&] { return launch_setup(c->stream, sa, n); }));
        HIPCHK(c, run(K_TILE, [&] { return launch_tile(c->stream, ta, tile, full ? 3 : 0, n, max_tiles); }));
    }
    FoldArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    fa.sc = c->sc;
    fa.R = x.R;
    fa.bits = x.bits;
    fa.n_pairs = n_pairs;
    for (int b = 0; b <= DRD_MAX_TEX; ++b) fa.eps[b] = dp.eps[b];
    fa.Q = (long long*)Q;
    fa.qtot = x.qtot;
    fa.K = K;
    fa.n_views = n_views;
    if (full) HIPCHK(c, run(K_FOLD, [&] { return launch_broadcast(c->stream, fa); }));
    else HIPCHK(c, run(K_FOLD, [&] { return launch_fold(c->stream, fa); }));
    return DR_OK;
}

static dr_status estimate_common(dr_ctx* c, const float* theta, const dr_view* views, int32_t n_views,
                                 const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                                 const float* eps, int64_t* Q, uint32_t* K, bool full, bool image) {
    EstPlan pl;
    dr_status s = estimate_check(c, theta, views, n_views, targets, n_pairs, eps, Q, K, pl);
    if (s) return s;
    s = device_guard(c);
    if (s) return s;
    s = adapt_capacity(c);
    if (s) return s;
    EstScratch x;
    s = estimate_scratch_ctx(c, pl, n_pairs, full, x);
    if (s) return s;
    s = estimate_launch(c, pl, theta, n_views, targets, seed, step, n_pairs, eps, Q, K, full, image, x, true);
    if (s) return s;
    return note_bins(c);
}

extern "C" dr_status dr_estimate_grad(dr_ctx* c, const float* theta, const dr_view* views, int32_t n_views,
                                      const float* targets, uint64_t seed, uint32_t step, int32_t n_pairs,
                                      const float* eps, int64_t* Q, uint32_t* K) {
    return estimate_common(c, theta, views, n_views, targets, seed, step, n_pairs, eps, Q, K, false, false);
}

extern "C" dr_status dr_estimate_grad_full(dr_ctx* c, const float* theta, const dr_view* views,
                                           int32_t n_views, const float* targets, uint64_t seed, uint32_t step,
                                           int32_t n_pairs, const float* eps, int64_t* Q, uint32_t* K) {
    return estimate_common(c, theta, views, n_views, targets, seed, step, n_pairs, eps, Q, K, true, false);
}

extern "C" dr_status dr_estimate_grad_image(dr_ctx* c, const float* theta, const dr_view* views,
                                            int32_t n_views, const float* grad_image, uint64_t seed, uint32_t step,
                                            int32_t n_pairs, const float* eps, int64_t* Q, uint32_t* K) {
    return estimate_common(c, theta, views, n_views, grad_image, seed, step, n_pairs, eps, Q, K, false, true);
}

// ------------------------------------------------ allocation-free estimate --
//
// dr_estimate_grad_noalloc takes all of its scratch from one file-scope
// device array instead of the context's buffers.  Every GPU the library is
// loaded on holds its own copy of the array until the process ends.  In
// host code the array's name stands for a host-side shadow, not for the
// device memory, so it is never passed to a kernel or a copy: its device
// address is looked up once per device (dr_create, with that device
// current) and kept in scratch_dev[].

static __device__ __align__(256) unsigned char scratch[DR_NOALLOC_SCRATCH_BYTES];

static std::mutex scratch_mu;
static constexpr int SCRATCH_MAX_DEVICES = 64;
static void* scratch_dev[SCRATCH_MAX_DEVICES];
static hipError_t scratch_err[SCRATCH_MAX_DEVICES];
static bool scratch_done[SCRATCH_MAX_DEVICES];

// Device address of `scratch` on the current device `dev` (looked up on the
// first call for that device).
static hipError_t scratch_lookup(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_done[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        scratch_dev[dev] = p;
        scratch_err[dev] = e;
        scratch_done[dev] = true;
    }
    *out = scratch_dev[dev];
    return scratch_err[dev];
}

static unsigned long long round256(unsigned long long b) { return (b + 255ull) & ~255ull; }

// Layout of the estimate's scratch in the static array, items per launch
// `per`: the bin counters and the per-pair group sums first (the part that
// must start at zero), then the sign bits, the records, the bins and the
// tessellated positions.  Returns the bytes needed; fills x when base is
// given.
static unsigned long long static_layout(const dr_ctx* c, const EstPlan& pl, int32_t n_pairs, long long per,
                                        unsigned char* base, EstScratch* x, unsigned long long* zero_bytes) {
    const DScene& sc = c->sc;
    const unsigned long long slots = 2ull * (unsigned long long)per;
    const unsigned long long cap = (unsigned long long)c->tune.bin_capacity;
    unsigned long long off = 0;
    auto take = [&](unsigned long long bytes) {
        unsigned long long o = off;
        off += round256(bytes);
        return o;
    };
    const unsigned long long bin_slots = slots * (unsigned long long)pl.max_tiles;
    unsigned long long o_counts = take(bin_slots * sizeof(unsigned));
    unsigned long long o_spn = take(slots * 2ull * sizeof(unsigned));
    unsigned long long o_R = take((unsigned long long)n_pairs * (unsigned long long)sc.G * sizeof(long long));
    if (zero_bytes) *zero_bytes = off;
    unsigned long long o_bits = take(((unsigned long long)n_pairs * (unsigned long long)sc.words + 1ull) * 4ull);
    unsigned long long o_recR = take(slots * (unsigned long long)sc.n_tris * sizeof(TriR));
    unsigned long long o_recS = take(slots * (unsigned long long)sc.n_tris * sizeof(TriS));
    unsigned long long o_bins = take(bin_slots * cap * sizeof(unsigned));
    unsigned long long o_spill = take(slots * (unsigned long long)SPILL_CAP * sizeof(unsigned long long));
    unsigned long long o_fpos = 0;
    if (sc.n_ctrl > 0) o_fpos = take((unsigned long long)n_pairs * 2ull * (unsigned long long)sc.n_verts * 12ull);
    if (base && x) {
        x->counts = (unsigned*)(base + o_counts);
        x->R = (long long*)(base + o_R);
        x->bits = (uint32_t*)(base + o_bits);
        x->recR = (TriR*)(base + o_recR);
        x->recS = (TriS*)(base + o_recS);
        x->bins = (unsigned*)(base + o_bins);
        x->spn = (unsigned*)(base + o_spn);
        x->spill = (unsigned long long*)(base + o_spill);
        x->fpos = sc.n_ctrl > 0 ? (float*)(base + o_fpos) : nullptr;
        x->qtot = nullptr;
        x->cap = (int)cap;
        x->per = per;
    }
    return off;
}

extern "C" dr_status dr_estimate_grad_noalloc(dr_ctx* c, const float* theta, const dr_view* views,
                                              int32_t n_views, const float* targets, uint64_t seed, uint32_t step,
                                              int32_t n_pairs, const float* eps, int64_t* Q, uint32_t* K) {
    EstPlan pl;
    dr_status s = estimate_check(c, theta, views, n_views, targets, n_pairs, eps, Q, K, pl);
    if (s) return s;
    s = device_guard(c);
    if (s) return s;
    void* base = nullptr;
    hipError_t e = scratch_lookup(c->device, &base);
    if (e != hipSuccess || !base)
        return fail(c, DR_E_HIP, std::string("device address of the static scratch array: ") + hipGetErrorString(e));
    // as many items per raster launch as the tuning asks for and the array
    // holds (the results do not depend on it); one at the least
    long long per = items_per_launch(c, pl.items);
    unsigned long long need = static_layout(c, pl, n_pairs, per, nullptr, nullptr, nullptr);
    while (need > DR_NOALLOC_SCRATCH_BYTES && per > 1) {
        per = (per + 1) / 2;
        need = static_layout(c, pl, n_pairs, per, nullptr, nullptr, nullptr);
    }
    if (need > DR_NOALLOC_SCRATCH_BYTES)
        return fail(c, DR_E_INVALID,
                    "dr_estimate_grad_noalloc needs " + std::to_string(need) + " bytes of scratch, more than its " +
                        std::to_string((unsigned long long)DR_NOALLOC_SCRATCH_BYTES) +
                        "-byte maximum (fewer pairs, fewer or smaller views, a smaller bin capacity, or "
                        "dr_estimate_grad)");
    EstScratch x;
    unsigned long long zero_bytes = 0;
    (void)static_layout(c, pl, n_pairs, per, (unsigned char*)base, &x, &zero_bytes);
    // the array keeps the last call's contents: clear the bin counters and
    // the group sums (a fill kernel, so the call can be captured in a graph)
    HIPCHK(c, launch_zero64(c->stream, (long long*)base, (int)(zero_bytes / 8ull)));
    return estimate_launch(c, pl, theta, n_views, targets, seed, step, n_pairs, eps, Q, K, false, false, x, false);
}


// --------------------------------------------------------------- loss --

extern "C" dr_status dr_loss(dr_ctx* c, const float* theta, const dr_view* views, int32_t n_views,
                             const float* targets, double* loss) {
    if (!c) return DR_E_INVALID;
    if (!theta || !targets || !loss || !views) return fail(c, DR_E_INVALID, "NULL array argument");
    if (n_views < 1 || n_views > DR_MAX_VIEWS) return fail(c, DR_E_INVALID, "n_views must be in [1, 16]");
    int tile = c->tune.tile_px;
    DViews dv;
    std::memset(&dv, 0, sizeof(dv));
    long long tgt_off = 0;
    int max_tiles = 1;
    for (int v = 0; v < n_views; ++v) {
        dr_status s = check_view(c, &views[v], tile);
        if (s) return s;
        dv.v[v] = make_dview(views[v], tile, tgt_off);
        tgt_off += 3ll * views[v].width * views[v].height;
        max_tiles = std::max(max_tiles, dv.v[v].tiles_x * dv.v[v].tiles_y);
    }
    dr_status s = device_guard(c);
    if (s) return s;
    s = ensure_raster(c, n_views, max_tiles);
    if (s) return s;
    s = grow(c, &c->partials, &c->partial_slots, (long long)n_views * max_tiles, sizeof(double), false);
    if (s) return s;
    DPert dp;
    dp.bits = nullptr;
    for (int b = 0; b <= DRD_MAX_TEX; ++b) dp.eps[b] = 0.0f;
    SetupArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.sc = c->sc;
    sa.views = dv;
    sa.pert = dp;
    sa.theta = theta;
    sa.n_views = n_views;
    sa.item0 = 0;
    sa.nsign = 1;
    sa.sgn[0] = sa.sgn[1] = 1.0f;
    sa.tile = tile;
    sa.cap = c->tune.bin_capacity;
    sa.max_tiles = max_tiles;
    sa.recR = c->recR;
    sa.recS = c->recS;
    sa.counts = c->counts;
    sa.bins = c->bins;
    sa.spn = c->spn;
    sa.spill = c->spill;
    s = tessellate(c, theta, dp, 1, 1, 1.0f, 1.0f, &sa.fpos);
    if (s) return s;
    HIPCHK(c, c->timer.run(c->stream, K_SETUP, [&] { return launch_setup(c->stream, sa, n_views); }));
    TileArgs ta;
    std::memset(&ta, 0, sizeof(ta));
    ta.sc = c->sc;
    ta.views = dv;
    ta.pert = dp;
    ta.theta = theta;
    ta.n_views = n_views;
    ta.item0 = 0;
    ta.nsign = 1;
    ta.sgn[0] = ta.sgn[1] = 1.0f;
    ta.cap = c->tune.bin_capacity;
    ta.max_tiles = max_tiles;
    ta.recR = c->recR;
    ta.recS = c->recS;
    ta.counts = c->counts;
    ta.bins = c->bins;
    ta.spn = c->spn;
    ta.spill = c->spill;
    ta.stats = c->stats;
    ta.targets = targets;
    ta.partials = c->partials;
    HIPCHK(c, c->timer.run(c->stream, K_TILE, [&] { return launch_tile(c->stream, ta, tile, 2, n_views, max_tiles); }));
    HIPCHK(c, launch_sum_tiles(c->stream, c->partials, max_tiles, dv, n_views, loss));
    return DR_OK;
}

// ------------------------------------------------------- decode / step --

// Adam constants, formed in double and rounded to float once.
static OptimConst optim_const(const dr_optim* o, int averaging) {
    OptimConst oc;
    oc.kind = o->kind;
    oc.averaging = averaging;
    oc.b1 = o->beta1;
    oc.b2 = o->beta2;
    oc.omb1 = (float)(1.0 - (double)o->beta1);
    oc.omb2 = (float)(1.0 - (double)o->beta2);
    oc.eps_hat = o->eps_hat;
    return oc;
}

static float bias_correction(float beta, uint32_t t) { return (float)(1.0 - std::pow((double)beta, (double)t)); }

static dr_status step_common(dr_ctx* c, float* theta, float* m, float* v, uint32_t t, int64_t* Q, uint32_t* K,
                             const float* eps, int32_t n_pairs, const dr_optim* o, int averaging, float* grad) {
    dr_status s = check_eps(c, eps);
    if (s) return s;
    if (averaging != DR_AVG_COUNT && averaging != DR_AVG_PAIRS) return fail(c, DR_E_INVALID, "bad averaging");
    if (averaging == DR_AVG_PAIRS && n_pairs < 1) return fail(c, DR_E_INVALID, "n_pairs must be >= 1");
    s = device_guard(c);
    if (s) return s;
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.sc = c->sc;
    for (int b = 0; b < 1 + c->sc.n_tex; ++b) a.eps[b] = eps[b];
    a.oc.averaging = averaging;
    a.n_pairs = n_pairs;
    a.Q = (long long*)Q;
    a.K = K;
    a.stats = c->stats;
    if (grad) {
        a.decode_only = 1;
        a.grad = grad;
    } else {
        a.oc = optim_const(o, averaging);
        for (int b = 0; b < 1 + c->sc.n_tex; ++b) a.lr[b] = o->lr[b];
        a.bc1 = bias_correction(o->beta1, t);
        a.bc2 = bias_correction(o->beta2, t);
        a.theta = theta;
        a.m = m;
        a.v = v;
    }
    HIPCHK(c, c->timer.run(c->stream, K_STEP, [&] { return launch_step(c->stream, a); }));
    return DR_OK;
}

extern "C" dr_status dr_decode_grad(dr_ctx* c, const int64_t* Q, const uint32_t* K, const float* eps,
                                    int32_t averaging, int32_t n_pairs, float* grad) {
    if (!c) return DR_E_INVALID;
    if (!Q || !K || !grad) return fail(c, DR_E_INVALID, "NULL array argument");
    return step_common(c, nullptr, nullptr, nullptr, 1, (int64_t*)Q, (uint32_t*)K, eps, n_pairs, nullptr,
                       averaging, grad);
}

extern "C" dr_status dr_step(dr_ctx* c, float* theta, float* m, float* v, uint32_t t, int64_t* Q, uint32_t* K,
                             const float* eps, int32_t n_pairs, const dr_optim* o) {
    if (!c) return DR_E_INVALID;
    if (!theta || !Q || !K || !o) return fail(c, DR_E_INVALID, "NULL argument");
    if (o->kind != DR_ADAM && o->kind != DR_SGD) return fail(c, DR_E_INVALID, "bad optimiser kind");
    if (o->kind == DR_ADAM) {
        if (!m || !v) return fail(c, DR_E_INVALID, "Adam needs m and v");
        if (t < 1) return fail(c, DR_E_INVALID, "Adam step t must be >= 1");
        if (!(o->beta1 >= 0.0f && o->beta1 < 1.0f && o->beta2 >= 0.0f && o->beta2 < 1.0f))
            return fail(c, DR_E_INVALID, "betas must be in [0, 1)");
        if (!finite_nonneg(o->eps_hat)) return fail(c, DR_E_INVALID, "eps_hat must be finite and >= 0");
    }
    for (int b = 0; b < 1 + c->sc.n_tex; ++b)
        if (!std::isfinite(o->lr[b])) return fail(c, DR_E_INVALID, "lr must be finite");
    return step_common(c, theta, m, v, t, Q, K, eps, n_pairs, o, o->averaging, nullptr);
}

// ------------------------------------------------------------- timing --

extern "C" dr_status dr_timing_enable(dr_ctx* c, int enable) {
    if (!c) return DR_E_INVALID;
    c->timer.on = enable != 0;
    return DR_OK;
}

extern "C" dr_status dr_timing_read(dr_ctx* c, dr_timing_t* out, int reset) {
    if (!c || !out) return fail(c, DR_E_INVALID, "NULL argument");
    dr_status s = device_guard(c);
    if (s) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, c->timer.read(out, reset != 0));
    return DR_OK;
}

// -------------------------------------------------------------- stats --

extern "C" dr_status dr_stats(dr_ctx* c, dr_stats_t* out) {
    if (!c || !out) return fail(c, DR_E_INVALID, "NULL argument");
    dr_status s = device_guard(c);
    if (s) return s;
    unsigned long long h[ST_COUNT];
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(h, c->stats, sizeof(h), hipMemcpyDeviceToHost));
    out->tile_overflows = h[ST_OVERFLOWS];
    out->saturations = h[ST_SATURATIONS];
    out->nonfinite = h[ST_NONFINITE];
    out->max_bin = h[ST_MAX_BIN];
    out->full_scans = h[ST_FULL_SCANS];
    return DR_OK;
}

extern "C" dr_status dr_set_adaptive_bins(dr_ctx* c, int32_t on) {
    if (!c) return DR_E_INVALID;
    c->adapt = on ? 1 : 0;
    c->seen_pending = false;
    return DR_OK;
}

extern "C" dr_status dr_get_tuning(const dr_ctx* c, dr_tuning* out) {
    if (!c || !out) return DR_E_INVALID;
    *out = c->tune;
    return DR_OK;
}

extern "C" dr_status dr_reset_stats(dr_ctx* c) {
    if (!c) return DR_E_INVALID;
    dr_status s = device_guard(c);
    if (s) return s;
    HIPCHK(c, hipMemsetAsync(c->stats, 0, ST_COUNT * sizeof(unsigned long long), c->stream));
    return DR_OK;
}

extern "C" const char* dr_status_str(dr_status s) {
    switch (s) {
        case DR_OK: return "ok";
        case DR_E_INVALID: return "invalid argument";
        case DR_E_OOM: return "out of device memory";
        case DR_E_HIP: return "HIP error";
        case DR_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" const char* dr_last_error(const dr_ctx* c) { return c ? c->err.c_str() : ""; }

// ============================================================== batch ==

// Item groups of a step of a batch of several scenes (see
// dr_batch::groups); a one-scene batch runs as one group.  Measured: the
// 64-scene batch 8.7 -> 7.4 ms per step with 4 groups; the one-scene paper
// step 2.19 -> 2.22 ms with 2 (its setup alone fills the chip).
#define BATCH_GROUPS 4

struct dr_batch {
    int device = 0;
    hipStream_t stream = nullptr;      // caller's stream
    hipStream_t gstream = nullptr;     // capture stream of the graph (replays go to the caller's stream)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
    BatchArgs args{};
    int n_scenes = 0;
    bool has_one = false;              // one scene: its constants go by value
    BatchOne one{};
    // device allocations
    std::vector<void*> allocs;
    unsigned long long* stats = nullptr;
    Timer timer;                       // direct launches only (not graph replays)
    bool q_dirty = true;               // Q may hold sums (set at creation and by dr_batch_estimate)
    // The step's items in groups of about equal tile counts: the setup of
    // groups 1.. runs on a second stream while the tile kernel works on the
    // groups before it, filling the chip while the many small scenes of a
    // batch leave it partly idle.
    struct Group {
        long long blk0, nblk;          // setup blocks
        long long w0, nw;              // tile units
    };
    std::vector<Group> groups;
    hipStream_t astream = nullptr;     // the setups of groups 1..
    hipEvent_t ev_signs = nullptr;
    std::vector<hipEvent_t> ev_setup;
};

static dr_status bfail(dr_batch* b, dr_status s, const std::string& msg) {
    if (b) b->err = msg;
    return s;
}

#define BHIPCHK(b, expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return bfail((b), DR_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

static void batch_free(dr_batch* b) {
    b->timer.destroy();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_signs) (void)hipEventDestroy(b->ev_signs);
    for (hipEvent_t e : b->ev_setup)
        if (e) (void)hipEventDestroy(e);
    if (b->astream) (void)hipStreamDestroy(b->astream);
    if (b->gstream) (void)hipStreamDestroy(b->gstream);
    for (void* p : b->allocs)
        if (p) (void)hipFree(p);
    b->allocs.clear();
}

template <typename T>
static dr_status balloc(dr_batch* b, T** p, size_t count, bool zero) {
    void* q = nullptr;
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&q, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, DR_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    b->allocs.push_back(q);
    if (zero && hipMemset(q, 0, bytes) != hipSuccess) return bfail(b, DR_E_HIP, "hipMemset failed");
    *p = (T*)q;
    return DR_OK;
}

extern "C" dr_status dr_batch_create(dr_batch** out, const dr_batch_scene* scenes, int32_t n_scenes,
                                     int32_t n_pairs, int32_t tile_px, const dr_optim* opt, uint64_t seed,
                                     uint32_t first_step, void* stream) {
    if (!out || !scenes || !opt) return DR_E_INVALID;
    *out = nullptr;
    if (n_scenes < 1 || n_scenes > (1 << 20)) return DR_E_INVALID;
    if (n_pairs < 1 || n_pairs > 65535) return DR_E_INVALID;
    if (tile_px != 8 && tile_px != 16 && tile_px != 32) return DR_E_INVALID;
    if (first_step < 1) return DR_E_INVALID;
    if (opt->kind != DR_ADAM && opt->kind != DR_SGD) return DR_E_INVALID;
    if (opt->averaging != DR_AVG_COUNT && opt->averaging != DR_AVG_PAIRS) return DR_E_INVALID;
    if (!(opt->beta1 >= 0.0f && opt->beta1 < 1.0f && opt->beta2 >= 0.0f && opt->beta2 < 1.0f) ||
        !finite_nonneg(opt->eps_hat))
        return DR_E_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DR_E_HIP;
    for (int i = 0; i < n_scenes; ++i) {
        const dr_batch_scene& s = scenes[i];
        if (!s.ctx || !s.views || !s.targets || !s.theta || !s.Q || !s.K) return DR_E_INVALID;
        if (s.ctx->device != dev) return DR_E_INVALID;
        if (s.ctx->sc.layers > 0) return DR_E_UNSUPPORTED;     // the batch raster is opaque only
        if (s.ctx->sc.n_ctrl > 0) return DR_E_UNSUPPORTED;     // and has no tessellation step
        if (opt->kind == DR_ADAM && (!s.m || !s.v)) return DR_E_INVALID;
        if (s.n_views < 1 || s.n_views > DR_MAX_VIEWS) return DR_E_INVALID;
        if (s.bin_capacity < 0 || s.bin_capacity > (1 << 20)) return DR_E_INVALID;
        for (int k = 0; k < 1 + s.ctx->sc.n_tex; ++k)
            if (!finite_nonneg(s.eps[k]) || !std::isfinite(s.lr[k])) return DR_E_INVALID;
        for (int v = 0; v < s.n_views; ++v)
            if (check_view(nullptr, &s.views[v], tile_px) != DR_OK) return DR_E_INVALID;
    }
    dr_batch* b = new (std::nothrow) dr_batch();
    if (!b) return DR_E_OOM;
    b->device = dev;
    b->stream = (hipStream_t)stream;
    b->n_scenes = n_scenes;
    BatchArgs& A = b->args;
    std::memset(&A, 0, sizeof(A));
    A.n_scenes = n_scenes;
    A.n_pairs = n_pairs;
    A.seed = seed;
    A.tile = tile_px;
    A.oc = optim_const(opt, opt->averaging);

    // host tables
    std::vector<BScene> hs(n_scenes);
    std::vector<DView> hv;
    std::vector<BItem> hi;
    std::vector<int> order(n_scenes);
    for (int i = 0; i < n_scenes; ++i) order[i] = i;
    // items of the costliest scenes first, so the launch ends on small units
    auto cost = [&](int i) {
        long long px = 0;
        for (int v = 0; v < scenes[i].n_views; ++v) px += (long long)scenes[i].views[v].width * scenes[i].views[v].height;
        return px;
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
    long long sign_blk = 0, group_blk = 0, rec = 0, cnt = 0, bin = 0, sp = 0, setup_blk = 0, tile0 = 0;
    std::vector<long long> bits_off(n_scenes), R_off(n_scenes);
    long long bits_total = 0, R_total = 0;
    for (int i = 0; i < n_scenes; ++i) {
        const dr_batch_scene& s = scenes[i];
        BScene& S = hs[i];
        std::memset(&S, 0, sizeof(S));
        S.sc = s.ctx->sc;
        S.theta = s.theta;
        S.m = s.m;
        S.v = s.v;
        S.Q = (long long*)s.Q;
        S.K = s.K;
        S.targets = s.targets;
        for (int k = 0; k <= DRD_MAX_TEX; ++k) {
            S.eps[k] = (k < 1 + S.sc.n_tex) ? s.eps[k] : 0.0f;
            S.lr[k] = (k < 1 + S.sc.n_tex) ? s.lr[k] : 0.0f;
        }
        S.act_pos = S.eps[0] != 0.0f;
        S.any_act = S.act_pos;
        for (int t = 0; t < S.sc.n_tex; ++t)
            if (S.eps[1 + t] != 0.0f) {
                S.act_cls[S.sc.tex_cls[t]] = 1;
                S.any_act = 1;
            }
        S.n_views = s.n_views;
        S.view0 = (int)hv.size();
        S.scene_index = i;
        long long tgt_off = 0;
        for (int v = 0; v < s.n_views; ++v) {
            hv.push_back(make_dview(s.views[v], tile_px, tgt_off));
            tgt_off += 3ll * s.views[v].width * s.views[v].height;
        }
        long long nblk = (S.sc.d + 255) >> 8;
        S.sign_blk0 = sign_blk;
        sign_blk += (long long)n_pairs * ((nblk + 255) >> 8);
        S.group_blk0 = group_blk;
        group_blk += (S.sc.G + 255) >> 8;
        bits_off[i] = bits_total;
        bits_total += (long long)n_pairs * S.sc.words;
        R_off[i] = R_total;
        R_total += (long long)n_pairs * S.sc.G;
    }
    for (int oi = 0; oi < n_scenes; ++oi) {
        int i = order[oi];
        const dr_batch_scene& s = scenes[i];
        const BScene& S = hs[i];
        int cap = s.bin_capacity > 0 ? s.bin_capacity : s.ctx->tune.bin_capacity;
        for (int n = 0; n < n_pairs; ++n)
            for (int v = 0; v < s.n_views; ++v) {
                const DView& dv = hv[S.view0 + v];
                long long tiles = (long long)dv.tiles_x * dv.tiles_y;
                BItem I;
                std::memset(&I, 0, sizeof(I));
                I.scene = i;
                I.pair = n;
                I.view = S.view0 + v;
                I.cap = cap;
                I.rec_off = rec;
                rec += 2ll * S.sc.n_tris;
                I.cnt_off = cnt;
                cnt += 2 * tiles;
                I.bin_off = bin;
                bin += 2 * tiles * cap;
                I.sp_off = sp;
                sp += 2;
                I.setup_blk0 = setup_blk;
                setup_blk += 2 * (((long long)S.sc.n_tris + 255) >> 8);
                I.tile0 = tile0;
                tile0 += tiles;
                hi.push_back(I);
            }
    }
    if (sign_blk > 0x7fffffffll || setup_blk > 0x7fffffffll || group_blk > 0x7fffffffll || tile0 > 0x7fffffffll) {
        batch_free(b);
        delete b;
        return DR_E_UNSUPPORTED;
    }
    A.n_items = (int)hi.size();
    A.sign_blocks = sign_blk;
    A.setup_blocks = setup_blk;
    A.group_blocks = group_blk;
    A.total_tiles = tile0;
    A.unit0 = 0;
    // items in BATCH_GROUPS groups of about equal tile counts (item order)
    {
        const int G = n_scenes == 1 ? 1 : (int)std::min<size_t>(BATCH_GROUPS, hi.size());
        size_t i = 0;
        for (int g = 0; g < G && i < hi.size(); ++g) {
            const long long cut = (g + 1 == G) ? tile0 : tile0 * (g + 1) / G;
            size_t j = i + 1;
            while (j < hi.size() && hi[j].tile0 < cut) ++j;
            if (g + 1 < G && j >= hi.size() && j > i + 1) --j;      // leave items for the later groups
            dr_batch::Group gr;
            gr.blk0 = hi[i].setup_blk0;
            gr.nblk = (j < hi.size() ? hi[j].setup_blk0 : setup_blk) - gr.blk0;
            gr.w0 = hi[i].tile0;
            gr.nw = (j < hi.size() ? hi[j].tile0 : tile0) - gr.w0;
            b->groups.push_back(gr);
            i = j;
        }
        if (b->groups.size() > 1) {
            bool ok2 = hipStreamCreateWithFlags(&b->astream, hipStreamNonBlocking) == hipSuccess &&
                       hipEventCreateWithFlags(&b->ev_signs, hipEventDisableTiming) == hipSuccess;
            b->ev_setup.assign(b->groups.size(), nullptr);
            for (size_t g = 1; ok2 && g < b->groups.size(); ++g)
                ok2 = hipEventCreateWithFlags(&b->ev_setup[g], hipEventDisableTiming) == hipSuccess;
            if (!ok2) {
                batch_free(b);
                delete b;
                return DR_E_HIP;
            }
        }
    }

    // Adam bias corrections by step, until both reach 1 in float
    std::vector<float> bc1, bc2;
    for (uint32_t t = 1; t <= (1u << 20); ++t) {
        bc1.push_back(bias_correction(opt->beta1, t));
        bc2.push_back(bias_correction(opt->beta2, t));
        if (bc1.back() == 1.0f && bc2.back() == 1.0f) break;
    }
    A.n_bc = (int)bc1.size();

    // device memory
    dr_status st = DR_OK;
    uint32_t* bits = nullptr;
    long long* R = nullptr;
    BScene* dsc = nullptr;
    DView* dvw = nullptr;
    BItem* dit = nullptr;
    float *dbc1 = nullptr, *dbc2 = nullptr;
    unsigned* dstep = nullptr;
    if ((st = balloc(b, &bits, (size_t)bits_total + 1, false)) || (st = balloc(b, &R, (size_t)R_total, true)) ||
        (st = balloc(b, &A.recR, (size_t)rec, false)) || (st = balloc(b, &A.recS, (size_t)rec, false)) ||
        (st = balloc(b, &A.counts, (size_t)cnt, true)) || (st = balloc(b, &A.bins, (size_t)bin, false)) ||
        (st = balloc(b, &A.spn, (size_t)sp * 2, true)) ||
        (st = balloc(b, &A.spill, (size_t)sp * SPILL_CAP, false)) ||
        (st = balloc(b, &dsc, hs.size(), false)) || (st = balloc(b, &dvw, hv.size(), false)) ||
        (st = balloc(b, &dit, hi.size(), false)) || (st = balloc(b, &dbc1, bc1.size(), false)) ||
        (st = balloc(b, &dbc2, bc2.size(), false)) || (st = balloc(b, &dstep, 1, false)) ||
        (st = balloc(b, &b->stats, ST_COUNT, true))) {
        batch_free(b);
        delete b;
        return st;
    }
    for (int i = 0; i < n_scenes; ++i) {
        hs[i].bits = bits + bits_off[i];
        hs[i].R = R + R_off[i];
    }
    bool ok = hipMemcpy(dsc, hs.data(), hs.size() * sizeof(BScene), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dvw, hv.data(), hv.size() * sizeof(DView), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dit, hi.data(), hi.size() * sizeof(BItem), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dbc1, bc1.data(), bc1.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dbc2, bc2.data(), bc2.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dstep, &first_step, sizeof(unsigned), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        batch_free(b);
        delete b;
        return DR_E_HIP;
    }
    A.scenes = dsc;
    A.views = dvw;
    A.items = dit;
    A.bc1 = dbc1;
    A.bc2 = dbc2;
    A.step = dstep;
    A.stats = b->stats;
    if (n_scenes == 1 && hv.size() <= (size_t)DRD_MAX_VIEWS) {
        b->has_one = true;
        b->one.sc = hs[0].sc;
        for (size_t v = 0; v < hv.size(); ++v) b->one.views[v] = hv[v];
        // items are numbered (pair, view): the tile launch walks them pair-interleaved
        b->one.n_views = (int)hv.size();
        b->one.il_pairs = n_pairs;
        b->one.tsum[0] = 0;
        for (size_t v = 0; v < hv.size(); ++v)
            b->one.tsum[v + 1] = b->one.tsum[v] + (long long)hv[v].tiles_x * hv[v].tiles_y;
    }
    *out = b;
    return DR_OK;
}

extern "C" dr_status dr_batch_destroy(dr_batch* b) {
    if (!b) return DR_E_INVALID;
    (void)hipStreamSynchronize(b->stream);
    if (b->gstream) (void)hipStreamSynchronize(b->gstream);
    if (b->astream) (void)hipStreamSynchronize(b->astream);
    batch_free(b);
    delete b;
    return DR_OK;
}

// Signs, then per group the setup and the tile launch, then the descent.
// Untimed, the setups of groups 1.. go to the second stream (ordered after
// the signs) and each group's tile launch waits for its setup; timed, every
// launch runs in order on st so that each is bracketed by its own events.
static hipError_t batch_enqueue(dr_batch* b, hipStream_t st, bool descend, bool timed) {
    const BatchArgs& A = b->args;
    Timer off;
    Timer& T = timed ? b->timer : off;
    hipError_t e;
    const BatchOne* one = b->has_one ? &b->one : nullptr;
    if ((e = T.run(st, K_SIGNS, [&] { return launch_batch_signs(st, A); })) != hipSuccess) return e;
    const size_t G = b->groups.size();
    if (!timed && G > 1) {
        if ((e = hipEventRecord(b->ev_signs, st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(b->astream, b->ev_signs, 0)) != hipSuccess) return e;
        for (size_t g = 1; g < G; ++g) {
            if ((e = launch_batch_setup(b->astream, A, one, b->groups[g].blk0, b->groups[g].nblk)) != hipSuccess) return e;
            if ((e = hipEventRecord(b->ev_setup[g], b->astream)) != hipSuccess) return e;
        }
        if ((e = launch_batch_setup(st, A, one, b->groups[0].blk0, b->groups[0].nblk)) != hipSuccess) return e;
        for (size_t g = 0; g < G; ++g) {
            if (g > 0 && (e = hipStreamWaitEvent(st, b->ev_setup[g], 0)) != hipSuccess) return e;
            if ((e = launch_batch_tile(st, A, one, b->groups[g].w0, b->groups[g].nw)) != hipSuccess) return e;
        }
    } else {
        for (size_t g = 0; g < G; ++g) {
            const auto& gr = b->groups[g];
            if ((e = T.run(st, K_SETUP, [&] { return launch_batch_setup(st, A, one, gr.blk0, gr.nblk); })) != hipSuccess)
                return e;
            if ((e = T.run(st, K_TILE, [&] { return launch_batch_tile(st, A, one, gr.w0, gr.nw); })) != hipSuccess)
                return e;
        }
    }
    if (descend && A.n_pairs <= 8) {
        // the fold's sums go straight into the update (timed as the step)
        if ((e = T.run(st, K_STEP, [&] { return launch_batch_fold_step(st, A); })) != hipSuccess) return e;
        return launch_batch_end(st, A);
    }
    if ((e = T.run(st, K_FOLD, [&] { return launch_batch_fold(st, A); })) != hipSuccess) return e;
    if (descend) {
        if ((e = T.run(st, K_STEP, [&] { return launch_batch_step(st, A); })) != hipSuccess) return e;
        if ((e = launch_batch_end(st, A)) != hipSuccess) return e;
    }
    return hipSuccess;
}

static dr_status batch_device(dr_batch* b) {
    int cur = -1;
    BHIPCHK(b, hipGetDevice(&cur));
    if (cur != b->device) BHIPCHK(b, hipSetDevice(b->device));
    return DR_OK;
}

extern "C" dr_status dr_batch_estimate(dr_batch* b) {
    if (!b) return DR_E_INVALID;
    dr_status s = batch_device(b);
    if (s) return s;
    BHIPCHK(b, batch_enqueue(b, b->stream, false, true));
    b->q_dirty = true;                   // Q now holds the estimate
    return DR_OK;
}

extern "C" dr_status dr_batch_step(dr_batch* b, int use_graph) {
    if (!b) return DR_E_INVALID;
    dr_status s = batch_device(b);
    if (s) return s;
    // A step reads Q only while it may hold sums (at creation, or after
    // dr_batch_estimate); a step leaves it zero.  The graph is captured
    // reading no Q, so a step with Q possibly non-zero runs directly.
    if (!use_graph || b->q_dirty) {
        b->args.q_zero = b->q_dirty ? 0 : 1;
        BHIPCHK(b, batch_enqueue(b, b->stream, true, true));
        b->q_dirty = false;
        return DR_OK;
    }
    if (!b->exec) {
        b->args.q_zero = 1;
        // captured on a stream of our own (the caller's may be the null
        // stream, which cannot be captured), with nothing pending on it
        BHIPCHK(b, hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking));
        BHIPCHK(b, hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal));
        hipError_t e = batch_enqueue(b, b->gstream, true, false);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->gstream, &g);
        if (e != hipSuccess || e2 != hipSuccess)
            return bfail(b, DR_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        b->graph = g;
        BHIPCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    // replayed on the caller's stream itself: no cross-stream waits between steps
    BHIPCHK(b, hipGraphLaunch(b->exec, b->stream));
    return DR_OK;
}

extern "C" dr_status dr_batch_set_step(dr_batch* b, uint32_t step) {
    if (!b) return DR_E_INVALID;
    if (step < 1) return bfail(b, DR_E_INVALID, "step must be >= 1");
    dr_status s = batch_device(b);
    if (s) return s;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    if (b->gstream) BHIPCHK(b, hipStreamSynchronize(b->gstream));
    BHIPCHK(b, hipMemcpy((void*)b->args.step, &step, sizeof(step), hipMemcpyHostToDevice));
    return DR_OK;
}

extern "C" dr_status dr_batch_get_step(dr_batch* b, uint32_t* step) {
    if (!b || !step) return DR_E_INVALID;
    dr_status s = batch_device(b);
    if (s) return s;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    if (b->gstream) BHIPCHK(b, hipStreamSynchronize(b->gstream));
    BHIPCHK(b, hipMemcpy(step, b->args.step, sizeof(*step), hipMemcpyDeviceToHost));
    return DR_OK;
}

extern "C" dr_status dr_batch_stats(dr_batch* b, dr_stats_t* out) {
    if (!b || !out) return DR_E_INVALID;
    dr_status s = batch_device(b);
    if (s) return s;
    unsigned long long h[ST_COUNT];
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    if (b->gstream) BHIPCHK(b, hipStreamSynchronize(b->gstream));
    BHIPCHK(b, hipMemcpy(h, b->stats, sizeof(h), hipMemcpyDeviceToHost));
    out->tile_overflows = h[ST_OVERFLOWS];
    out->saturations = h[ST_SATURATIONS];
    out->nonfinite = h[ST_NONFINITE];
    out->max_bin = h[ST_MAX_BIN];
    out->full_scans = h[ST_FULL_SCANS];
    return DR_OK;
}

extern "C" dr_status dr_batch_timing_enable(dr_batch* b, int enable) {
    if (!b) return DR_E_INVALID;
    b->timer.on = enable != 0;
    return DR_OK;
}

extern "C" dr_status dr_batch_timing_read(dr_batch* b, dr_timing_t* out, int reset) {
    if (!b || !out) return DR_E_INVALID;
    dr_status s = batch_device(b);
    if (s) return s;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    BHIPCHK(b, b->timer.read(out, reset != 0));
    return DR_OK;
}

extern "C" const char* dr_batch_last_error(const dr_batch* b) { return b ? b->err.c_str() : ""; }
