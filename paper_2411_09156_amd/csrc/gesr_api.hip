// C ABI of the GES rasterizer: argument validation, scratch layout and the
// launch sequence of each entry point.  Host code; device work is enqueued on
// the caller's stream and nothing is allocated here.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "gesr.h"
#include "gesr_device.h"
#include "gesr_kernels.h"

struct gesr_ctx {
    int device;
    std::string err;
};

namespace {

using namespace gesr;

gesr_status fail(gesr_ctx* ctx, gesr_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return s;
}

gesr_status hip_check(gesr_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return GESR_OK;
    return fail(ctx, GESR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define GESR_TRY(expr)                      \
    do {                                    \
        gesr_status _s = (expr);            \
        if (_s != GESR_OK) return _s;       \
    } while (0)

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

bool tile_supported(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 32 && th == 16) || (tw == 32 && th == 32);
}

gesr_status check_settings(gesr_ctx* ctx, const gesr_settings* st) {
    if (!st) return fail(ctx, GESR_ERR_INVALID, "settings is NULL");
    if (st->sh_degree < 0 || st->sh_degree > 3)
        return fail(ctx, GESR_ERR_INVALID, "sh_degree %d outside 0..3", st->sh_degree);
    if (!(st->kappa > 0.f) || !isfinite(st->kappa)) return fail(ctx, GESR_ERR_INVALID, "kappa must be > 0");
    if (!isfinite(st->rho)) return fail(ctx, GESR_ERR_INVALID, "rho must be finite");
    if (!(st->alpha_min > 0.f && st->alpha_min < st->alpha_max && st->alpha_max < 1.f))
        return fail(ctx, GESR_ERR_INVALID, "need 0 < alpha_min < alpha_max < 1");
    if (!(st->t_min > 0.f && st->t_min < 1.f)) return fail(ctx, GESR_ERR_INVALID, "need 0 < t_min < 1");
    if (!(st->blur >= 0.f) || !isfinite(st->blur)) return fail(ctx, GESR_ERR_INVALID, "blur must be >= 0");
    if (!(st->znear > 0.f) || !isfinite(st->znear)) return fail(ctx, GESR_ERR_INVALID, "znear must be > 0");
    if (!(st->clip_fac > 0.f) || !isfinite(st->clip_fac)) return fail(ctx, GESR_ERR_INVALID, "clip_fac must be > 0");
    for (int c = 0; c < 3; ++c)
        if (!isfinite(st->bg[c])) return fail(ctx, GESR_ERR_INVALID, "bg must be finite");
    if (st->tile_w <= 0 || st->tile_h <= 0) return fail(ctx, GESR_ERR_INVALID, "tile size must be positive");
    if (!tile_supported(st->tile_w, st->tile_h))
        return fail(ctx, GESR_ERR_UNSUPPORTED, "tile shape %dx%d not supported (16x16, 8x8, 32x16, 32x32)",
                    st->tile_w, st->tile_h);
    if (st->radix_bits < 4 || st->radix_bits > 8)
        return fail(ctx, GESR_ERR_INVALID, "radix_bits %d outside 4..8", st->radix_bits);
    if (st->batch != 0 && st->batch != 32 && st->batch != 64 && st->batch != 128)
        return fail(ctx, GESR_ERR_INVALID, "batch %d not in {0, 32, 64, 128}", st->batch);
    if (st->variant < 0 || st->variant > 1) return fail(ctx, GESR_ERR_INVALID, "variant must be 0 or 1");
    return GESR_OK;
}

struct Geometry {
    uint64_t total_tiles = 0, total_pixels = 0;
    uint64_t vn = 0;
    uint64_t total_rows = 0;  // tile rows over all views
};

gesr_status check_cams(gesr_ctx* ctx, const gesr_camera* cams, int V, int n, const gesr_settings* st, Geometry* g) {
    if (!cams) return fail(ctx, GESR_ERR_INVALID, "cams is NULL");
    if (V < 1 || V > GESR_MAX_VIEWS) return fail(ctx, GESR_ERR_INVALID, "V = %d outside 1..%d", V, GESR_MAX_VIEWS);
    if (n < 0) return fail(ctx, GESR_ERR_INVALID, "n = %d is negative", n);
    uint64_t tiles = 0, pix = 0;
    g->total_rows = 0;
    for (int v = 0; v < V; ++v) {
        const gesr_camera& c = cams[v];
        if (c.width < 1 || c.height < 1) return fail(ctx, GESR_ERR_INVALID, "view %d: width/height must be >= 1", v);
        if (!(c.fx > 0.f) || !(c.fy > 0.f) || !isfinite(c.fx) || !isfinite(c.fy) || !isfinite(c.cx) ||
            !isfinite(c.cy))
            return fail(ctx, GESR_ERR_INVALID, "view %d: focal lengths must be finite and > 0", v);
        for (int k = 0; k < 12; ++k)
            if (!isfinite(c.viewmat[k])) return fail(ctx, GESR_ERR_INVALID, "view %d: viewmat not finite", v);
        for (int k = 0; k < 3; ++k)
            if (!isfinite(c.campos[k])) return fail(ctx, GESR_ERR_INVALID, "view %d: campos not finite", v);
        const uint64_t tx = ((uint64_t)c.width + st->tile_w - 1) / st->tile_w;
        const uint64_t ty = ((uint64_t)c.height + st->tile_h - 1) / st->tile_h;
        if (tx > 0xFFFFu || ty > 0xFFFFu) return fail(ctx, GESR_ERR_INVALID, "view %d: too many tiles per axis", v);
        tiles += tx * ty;
        pix += (uint64_t)c.width * (uint64_t)c.height;
        g->total_rows += ty;
    }

    if (3 * pix >= (1ull << 32)) return fail(ctx, GESR_ERR_INVALID, "3 * total pixels must be < 2^32");
    if (tiles >= (1ull << 31)) return fail(ctx, GESR_ERR_INVALID, "too many tiles");
    const uint64_t vn = (uint64_t)V * (uint64_t)n;
    if (vn >= (1ull << 32)) return fail(ctx, GESR_ERR_INVALID, "V * n must be < 2^32");
    g->total_tiles = tiles;
    g->total_pixels = pix;
    g->vn = vn;
    return GESR_OK;
}

DevSettings dev_settings(const gesr_settings* s) {
    DevSettings d;
    d.kappa = s->kappa;
    d.neg_kappa_log2e = -s->kappa * 1.4426950408889634f;
    d.rho = s->rho;
    d.alpha_min = s->alpha_min;
    d.alpha_max = s->alpha_max;
    d.t_min = s->t_min;
    d.blur = s->blur;
    d.znear = s->znear;
    d.clip_fac = s->clip_fac;
    for (int c = 0; c < 3; ++c) d.bg[c] = s->bg[c];
    d.tile_w = s->tile_w;
    d.tile_h = s->tile_h;
    d.sh_degree = s->sh_degree;
    d.variant = s->variant;
    return d;
}

DevCams dev_cams(const gesr_camera* cams, int V, const gesr_settings* st) {
    DevCams d;
    memset(&d, 0, sizeof d);
    d.V = V;
    uint32_t tb = 0, pb = 0;
    for (int v = 0; v < V; ++v) {
        const gesr_camera& c = cams[v];
        DevView& w = d.v[v];
        w.W = c.width;
        w.H = c.height;
        w.fx = c.fx;
        w.fy = c.fy;
        w.cx = c.cx;
        w.cy = c.cy;
        for (int r = 0; r < 3; ++r) {
            for (int k = 0; k < 3; ++k) w.R[3 * r + k] = c.viewmat[4 * r + k];
            w.t[r] = c.viewmat[4 * r + 3];
            w.campos[r] = c.campos[r];
        }
        w.tiles_x = (c.width + st->tile_w - 1) / st->tile_w;
        w.tiles_y = (c.height + st->tile_h - 1) / st->tile_h;
        w.tile_base = tb;
        w.pix_base = pb;
        tb += (uint32_t)(w.tiles_x * w.tiles_y);
        pb += (uint32_t)(c.width * c.height);
    }
    return d;
}

// Layout of gesr_bins.scratch (256-byte aligned sub-buffers).
struct BinScratch {
    uint32_t *d_keys_a, *d_vals_a, *d_keys_b, *d_vals_b;  // (view, depth) sort, [V*n]
    uint32_t *rowlist, *rowcols;                          // row lists and their columns, [m_cap]
    uint2* srect;                                         // rectangles in (view, depth) order, [V*n]
    float4* sell;                                         // footprint ellipses in that order, [2 V*n]
    uint32_t *row_count, *row_start;                      // [total rows]
    uint32_t *seg_chunks, *chunk_off;                     // [segments + 1]
    uint32_t* mat;                                        // per-chunk bucket counts
    uint64_t mat_chunks;
    uint32_t* counters;                                   // [4]: row-list entries, overflow, listed
    uint32_t* chunk_total;                                // [1]
    uint32_t *w_keys_a, *w_vals_a, *w_keys_b;             // worklist sort, [T]
    uint32_t *tile_count, *tile_start;                    // [T]
    uint32_t *block_hist, *scan_partials;
    size_t bytes;
};

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

BinScratch carve(void* base, const Geometry& g, const DevCams& dc, int n, uint64_t m_cap) {
    BinScratch s;
    size_t off = 0;
    char* b = (char*)base;
    auto take = [&](uint64_t count) -> uint32_t* {
        uint32_t* p = b ? (uint32_t*)(b + off) : nullptr;
        off += ((count * 4 + 255) / 256) * 256;
        return p;
    };
    const uint64_t vn1 = g.vn > 0 ? g.vn : 1;
    const uint64_t T1 = g.total_tiles > 0 ? g.total_tiles : 1;
    const uint64_t nseg = std::max(is_segments(dc, 1), is_segments(dc, 2)) + 1;
    s.d_keys_a = take(vn1);
    s.d_vals_a = take(vn1);
    s.d_keys_b = take(vn1);
    s.d_vals_b = take(vn1);
    s.rowlist = take(m_cap);
    s.rowcols = take(m_cap);
    s.srect = reinterpret_cast<uint2*>(take(2 * vn1));
    s.sell = reinterpret_cast<float4*>(take(8 * vn1));
    s.row_count = take(g.total_rows + 1);
    s.row_start = take(g.total_rows + 1);
    s.seg_chunks = take(nseg);
    s.chunk_off = take(nseg);
    s.mat_chunks = std::max(is_chunk_bound(dc, 1, n, 0), is_chunk_bound(dc, 2, n, m_cap));
    s.mat = take(s.mat_chunks * is_window());
    s.counters = take(4);
    s.chunk_total = take(1);
    s.w_keys_a = take(T1);
    s.w_vals_a = take(T1);
    s.w_keys_b = take(T1);
    s.tile_count = take(T1);
    s.tile_start = take(T1);
    const uint64_t maxcount = std::max(vn1, T1);
    const uint64_t hist = 256ull * ceil_div(maxcount, SORT_TILE);
    s.block_hist = take(hist);
    const uint64_t scan_items = std::max(std::max(hist, vn1), std::max(T1, std::max(g.total_rows + 1, nseg)));
    s.scan_partials = take(ceil_div(scan_items, SCAN_TILE) + 64);
    s.bytes = off;
    return s;
}

// Layout of the backward workspace (256-byte aligned sub-buffers).
struct BwdWorkspace {
    uint32_t* visited;   // [ceil(m_cap / 32)] bit per instance slot
    float* grad2d;       // [V*n][GESR_GRAD2D_FLOATS]
    float* partials;     // [m_cap][kPartialStride]
    size_t bytes;
};

BwdWorkspace carve_bwd(void* base, uint64_t vn, uint64_t m_cap, uint64_t T) {
    BwdWorkspace w;
    size_t off = 0;
    char* b = (char*)base;
    auto take = [&](uint64_t bytes) -> char* {
        char* p = b ? b + off : nullptr;
        off += ((bytes + 255) / 256) * 256;
        return p;
    };
    w.visited = (uint32_t*)take(((m_cap + 31) / 32) * 4);
    w.grad2d = (float*)take((vn > 0 ? vn : 1) * GESR_GRAD2D_FLOATS * 4);
    w.partials = (float*)take(m_cap * kPartialStride * 4);
    w.bytes = off;
    return w;
}

int bits_for(uint64_t count) {
    int b = 0;
    while (b < 32 && (1ull << b) < count) ++b;
    return b;
}

gesr_status check_splats(gesr_ctx* ctx, const gesr_splats* sp, int sh_degree, bool need_all) {
    if (!sp) return fail(ctx, GESR_ERR_INVALID, "splats is NULL");
    if (sp->n < 0) return fail(ctx, GESR_ERR_INVALID, "splats->n is negative");
    if (sp->n == 0 && !need_all) return GESR_OK;
    const void* ptrs[6] = {sp->mean, sp->scale, sp->quat, sp->opacity, sp->beta, sp->sh};
    const char* names[6] = {"mean", "scale", "quat", "opacity", "beta", "sh"};
    for (int k = 0; k < 6; ++k) {
        if (!ptrs[k]) return fail(ctx, GESR_ERR_INVALID, "splats->%s is NULL", names[k]);
        if (!aligned16(ptrs[k])) return fail(ctx, GESR_ERR_INVALID, "splats->%s is not 16-byte aligned", names[k]);
    }
    (void)sh_degree;
    return GESR_OK;
}

gesr_status check_proj(gesr_ctx* ctx, const gesr_proj* p) {
    if (!p) return fail(ctx, GESR_ERR_INVALID, "proj is NULL");
    const void* ptrs[4] = {p->rec, p->tiles_touched, p->rect, p->depth_key};
    const char* names[4] = {"rec", "tiles_touched", "rect", "depth_key"};
    for (int k = 0; k < 4; ++k) {
        if (!ptrs[k]) return fail(ctx, GESR_ERR_INVALID, "proj->%s is NULL", names[k]);
        if (!aligned16(ptrs[k])) return fail(ctx, GESR_ERR_INVALID, "proj->%s is not 16-byte aligned", names[k]);
    }
    return GESR_OK;
}

gesr_status check_bins(gesr_ctx* ctx, const gesr_bins* b, bool need_scratch) {
    if (!b) return fail(ctx, GESR_ERR_INVALID, "bins is NULL");
    if (b->m_cap < 1 || b->m_cap >= (1ull << 32))
        return fail(ctx, GESR_ERR_INVALID, "m_cap must be in [1, 2^32)");
    const void* ptrs[5] = {b->val_sorted, b->ranges, b->worklist, b->inst_base, b->counters};
    const char* names[5] = {"val_sorted", "ranges", "worklist", "inst_base", "counters"};
    for (int k = 0; k < 5; ++k) {
        if (!ptrs[k]) return fail(ctx, GESR_ERR_INVALID, "bins->%s is NULL", names[k]);
        if (!aligned16(ptrs[k])) return fail(ctx, GESR_ERR_INVALID, "bins->%s is not 16-byte aligned", names[k]);
    }
    if (b->tile_sorted && !aligned16(b->tile_sorted))
        return fail(ctx, GESR_ERR_INVALID, "bins->tile_sorted is not 16-byte aligned");
    if (need_scratch && (!b->scratch || !aligned16(b->scratch)))
        return fail(ctx, GESR_ERR_INVALID, "bins->scratch is NULL or not 16-byte aligned");
    if (((uintptr_t)b->tile_work & 3u) != 0)
        return fail(ctx, GESR_ERR_INVALID, "bins->tile_work is not 4-byte aligned");
    return GESR_OK;
}

}  // namespace

extern "C" {

const char* gesr_status_string(gesr_status s) {
    switch (s) {
        case GESR_OK: return "ok";
        case GESR_ERR_INVALID: return "invalid argument";
        case GESR_ERR_CAPACITY: return "instance capacity exceeded";
        case GESR_ERR_HIP: return "HIP error";
        case GESR_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

gesr_status gesr_ctx_create(int device, gesr_ctx** out) {
    if (!out) return GESR_ERR_INVALID;
    if (device < 0) return GESR_ERR_INVALID;
    gesr_ctx* c = new gesr_ctx;
    c->device = device;
    *out = c;
    return GESR_OK;
}

void gesr_ctx_destroy(gesr_ctx* ctx) { delete ctx; }

const char* gesr_last_error(const gesr_ctx* ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

void gesr_default_settings(gesr_settings* s) {
    if (!s) return;
    memset(s, 0, sizeof *s);
    s->sh_degree = 0;
    s->kappa = 0.5f;
    s->rho = 0.1f;
    s->alpha_min = 1.0f / 255.0f;
    s->alpha_max = 0.99f;
    s->t_min = 1e-4f;
    s->blur = 0.3f;
    s->znear = 0.2f;
    s->clip_fac = 1.3f;
    s->tile_w = 16;
    s->tile_h = 16;
    s->batch = 0;
    s->radix_bits = 8;
}

gesr_status gesr_query_sizes(gesr_ctx* ctx, const gesr_camera* cams, int V, int n, const gesr_settings* st,
                             uint64_t m_cap, gesr_sizes* out) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!out) return fail(ctx, GESR_ERR_INVALID, "out is NULL");
    GESR_TRY(check_settings(ctx, st));
    Geometry g;
    GESR_TRY(check_cams(ctx, cams, V, n, st, &g));
    if (m_cap < 1 || m_cap >= (1ull << 32)) return fail(ctx, GESR_ERR_INVALID, "m_cap must be in [1, 2^32)");
    BinScratch s = carve(nullptr, g, dev_cams(cams, V, st), n, m_cap);
    out->total_tiles = g.total_tiles;
    out->total_pixels = g.total_pixels;
    out->bin_scratch_bytes = s.bytes;
    out->bwd_workspace_bytes = carve_bwd(nullptr, g.vn, m_cap, g.total_tiles).bytes;
    out->max_sort_blocks = ceil_div(std::max<uint64_t>(g.vn, g.total_tiles), SORT_TILE);
    ctx->err.clear();
    return GESR_OK;
}

gesr_status gesr_project(gesr_ctx* ctx, const gesr_splats* splats, const gesr_camera* cams, int V,
                         const gesr_settings* st, const gesr_proj* out, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    GESR_TRY(check_settings(ctx, st));
    GESR_TRY(check_splats(ctx, splats, st->sh_degree, false));
    Geometry g;
    GESR_TRY(check_cams(ctx, cams, V, splats->n, st, &g));
    GESR_TRY(check_proj(ctx, out));
    ProjectArgs a;
    a.n = splats->n;
    a.mean = splats->mean;
    a.scale = splats->scale;
    a.quat = splats->quat;
    a.opacity = splats->opacity;
    a.beta = splats->beta;
    a.sh = splats->sh;
    a.rec = out->rec;
    a.tiles_touched = out->tiles_touched;
    a.rect = out->rect;
    a.depth_key = out->depth_key;
    a.st = dev_settings(st);
    a.cams = dev_cams(cams, V, st);
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, launch_project(a, st->sh_degree, (hipStream_t)stream), "project launch"));
    ctx->err.clear();
    return GESR_OK;
}

}  // extern "C"

namespace {

// The binning pipeline of gesr_bin on a scratch buffer of `scratch_bytes` at
// `scratch` (checked against the layout's size).  Arguments are validated by
// the caller (g from check_cams); the device is current.
gesr_status bin_impl(gesr_ctx* ctx, const gesr_proj* proj, const gesr_camera* cams, int V, int n,
                     const gesr_settings* st, const gesr_bins* bins, const Geometry& g, void* scratch,
                     size_t scratch_bytes, int flags, uint64_t* m_out, void* stream) {
    if ((flags & GESR_BIN_WORK_ORDER) && !bins->tile_work)
        return fail(ctx, GESR_ERR_INVALID, "GESR_BIN_WORK_ORDER needs bins->tile_work");
    const DevCams dc = dev_cams(cams, V, st);
    BinScratch s = carve(scratch, g, dc, n, bins->m_cap);
    if (scratch_bytes < s.bytes)
        return fail(ctx, GESR_ERR_INVALID, "bins->scratch_bytes %zu < required %zu", scratch_bytes, s.bytes);
    hipStream_t strm = (hipStream_t)stream;
    const uint64_t T = g.total_tiles;

    // 1. (view, depth, pair) order of the (view, splat) pairs: LSD passes over
    //    the 32 depth bits and then the view bits, which the last pass or two
    //    take from the pair index (view = pair / n)
    SortBuffers db{s.d_keys_a, s.d_vals_a, s.d_keys_b, s.d_vals_b, s.block_hist, s.scan_partials};
    bool in_b = false;
    const int vbits = bits_for((uint64_t)V);
    GESR_TRY(hip_check(ctx,
                       radix_sort(proj->depth_key, nullptr, g.vn, nullptr, 32 + vbits, st->radix_bits, db, &in_b,
                                  strm, vbits > 0 ? (uint32_t)n : 0u),
                       "depth and view sort"));
    const uint32_t* order_vd = in_b ? s.d_vals_b : s.d_vals_a;
    // 2. instance slots: exclusive scan of tiles_touched in pair order; M -> counters[0]
    GESR_TRY(hip_check(ctx, scan_exclusive(proj->tiles_touched, bins->inst_base, g.vn, s.scan_partials,
                                           bins->counters, strm),
                       "instance slots"));
    GESR_TRY(hip_check(ctx, launch_set_counters(bins->counters, bins->m_cap, strm), "counters"));
    if (flags & GESR_BIN_SYNC) {
        uint32_t m = 0;
        GESR_TRY(hip_check(ctx, hipMemcpyAsync(&m, bins->counters, sizeof m, hipMemcpyDeviceToHost, strm), "M copy"));
        GESR_TRY(hip_check(ctx, hipStreamSynchronize(strm), "M sync"));
        if (m_out) *m_out = m;
        if ((uint64_t)m > bins->m_cap)
            return fail(ctx, GESR_ERR_CAPACITY, "M = %u instances exceed m_cap = %llu", m,
                        (unsigned long long)bins->m_cap);
    }
    // 3. row lists: every pair in the rows its rectangle covers (level 1), each
    //    entry with the columns its ellipse reaches in that row
    GESR_TRY(hip_check(ctx, launch_gather_rects(order_vd, proj->rec, g.vn, s.srect, s.sell, strm), "rectangles"));
    IsArgs ia;
    memset(&ia, 0, sizeof ia);
    ia.n = n;
    ia.vn = (uint32_t)g.vn;
    ia.chunk_off = s.chunk_off;
    ia.chunk_total = s.chunk_total;
    ia.mat = s.mat;
    ia.mat_chunks = s.mat_chunks;
    ia.cams = dc;
    IsArgs l1 = ia;
    l1.items = order_vd;
    l1.item_rect = s.srect;
    l1.out_cols = s.rowcols;
    l1.bucket_count = s.row_count;
    l1.bucket_start = s.row_start;
    l1.out_vals = s.rowlist;
    l1.out_cap = bins->m_cap;
    l1.item_ell = s.sell;  // each row entry carries its own row's columns
    l1.tile_w = st->tile_w;
    l1.tile_h = st->tile_h;
    GESR_TRY(hip_check(ctx,
                       launch_interval_scatter(l1, 1, (uint32_t)g.total_rows, s.counters, s.seg_chunks,
                                               s.scan_partials, strm),
                       "row lists"));
    GESR_TRY(hip_check(ctx, launch_set_counters(s.counters, bins->m_cap, strm), "row counters"));
    // 4. tile lists: every row-list entry in the tiles of its columns (level 2)
    IsArgs l2 = ia;
    l2.items = s.rowlist;
    l2.item_cols = s.rowcols;
    l2.items_listed = s.counters + 2;
    l2.row_start = s.row_start;
    l2.row_count = s.row_count;
    l2.bucket_count = s.tile_count;
    l2.bucket_start = s.tile_start;
    l2.out_vals = bins->val_sorted;
    l2.out_keys = bins->tile_sorted;
    l2.out_cap = bins->m_cap;
    GESR_TRY(hip_check(ctx,
                       launch_interval_scatter(l2, 2, (uint32_t)T, bins->counters + 3, s.seg_chunks, s.scan_partials,
                                               strm),
                       "tile lists"));
    GESR_TRY(hip_check(ctx, launch_ranges_from_counts(s.tile_count, s.tile_start, T, bins->counters + 2,
                                                      bins->ranges, strm),
                       "ranges"));
    // 5. worklist: tiles by decreasing list length, or by decreasing work of a
    //    previous forward (the positions each tile evaluated before terminating)
    const uint32_t* work = (flags & GESR_BIN_WORK_ORDER) ? bins->tile_work : nullptr;
    GESR_TRY(hip_check(ctx, launch_worklist_keys(bins->ranges, work, T, s.w_keys_b, strm), "worklist keys"));
    SortBuffers wb{s.w_keys_a, s.w_vals_a, s.w_keys_b, bins->worklist, s.block_hist, s.scan_partials};
    GESR_TRY(hip_check(ctx, radix_sort(s.w_keys_b, nullptr, T, nullptr, 16, 8, wb, &in_b, strm), "worklist sort"));
    ctx->err.clear();
    return GESR_OK;
}

}  // namespace

// Scratch of gesr_bin_static: one array per GPU, held until the process ends.
// Host code uses its device address from hipGetSymbolAddress (static_scratch),
// never the array's name.
static __device__ __align__(256) unsigned char scratch[GESR_BIN_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_address[kMaxDevices] = {};

// Device address of `scratch` on ctx's device (current), looked up once per device.
gesr_status static_scratch(gesr_ctx* ctx, void** out) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return fail(ctx, GESR_ERR_UNSUPPORTED, "device %d: the static scratch serves devices 0..%d", ctx->device,
                    kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_address[ctx->device]) {
        void* p = nullptr;
        GESR_TRY(hip_check(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
        if (!p) return fail(ctx, GESR_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_address[ctx->device] = p;
    }
    *out = g_scratch_address[ctx->device];
    return GESR_OK;
}

}  // namespace

extern "C" {

gesr_status gesr_bin(gesr_ctx* ctx, const gesr_proj* proj, const gesr_camera* cams, int V, int n,
                     const gesr_settings* st, const gesr_bins* bins, int flags, uint64_t* m_out, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    GESR_TRY(check_settings(ctx, st));
    Geometry g;
    GESR_TRY(check_cams(ctx, cams, V, n, st, &g));
    GESR_TRY(check_proj(ctx, proj));
    GESR_TRY(check_bins(ctx, bins, true));
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    return bin_impl(ctx, proj, cams, V, n, st, bins, g, bins->scratch, bins->scratch_bytes, flags, m_out, stream);
}

gesr_status gesr_bin_static(gesr_ctx* ctx, const gesr_proj* proj, const gesr_camera* cams, int V, int n,
                            const gesr_settings* st, const gesr_bins* bins, int flags, uint64_t* m_out,
                            void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    GESR_TRY(check_settings(ctx, st));
    Geometry g;
    GESR_TRY(check_cams(ctx, cams, V, n, st, &g));
    GESR_TRY(check_proj(ctx, proj));
    GESR_TRY(check_bins(ctx, bins, false));
    const size_t need = carve(nullptr, g, dev_cams(cams, V, st), n, bins->m_cap).bytes;
    if (need > (size_t)GESR_BIN_STATIC_SCRATCH_BYTES)
        return fail(ctx, GESR_ERR_CAPACITY, "gesr_bin_static: this binning needs %zu bytes of scratch; the static "
                    "scratch holds %zu", need, (size_t)GESR_BIN_STATIC_SCRATCH_BYTES);
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    void* base = nullptr;
    GESR_TRY(static_scratch(ctx, &base));
    return bin_impl(ctx, proj, cams, V, n, st, bins, g, base, (size_t)GESR_BIN_STATIC_SCRATCH_BYTES, flags,
                    m_out, stream);
}

// The extended channels run only in the one-wave 16x16 renderers.
static gesr_status check_channel_renderer(gesr_ctx* ctx, const gesr_settings* st) {
    if (st->tile_w != 16 || st->tile_h != 16 || st->variant != 0)
        return fail(ctx, GESR_ERR_UNSUPPORTED,
                    "depth/alpha channels need tile 16x16 and variant 0 (got %dx%d, variant %d)", st->tile_w,
                    st->tile_h, st->variant);
    return GESR_OK;
}

gesr_status gesr_render_fwd(gesr_ctx* ctx, const gesr_proj* proj, const gesr_bins* bins, const gesr_camera* cams,
                            int V, int n, const gesr_settings* st, float* image, float* final_T, uint32_t* n_contrib,
                            const gesr_fwd_counts* counts, void* stream) {
    return gesr_render_fwd_ext(ctx, proj, bins, cams, V, n, st, image, final_T, n_contrib, counts, nullptr, stream);
}

gesr_status gesr_render_fwd_ext(gesr_ctx* ctx, const gesr_proj* proj, const gesr_bins* bins,
                                const gesr_camera* cams, int V, int n, const gesr_settings* st, float* image,
                                float* final_T, uint32_t* n_contrib, const gesr_fwd_counts* counts,
                                const gesr_fwd_channels* channels, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    GESR_TRY(check_settings(ctx, st));
    Geometry g;
    GESR_TRY(check_cams(ctx, cams, V, n, st, &g));
    GESR_TRY(check_proj(ctx, proj));
    GESR_TRY(check_bins(ctx, bins, false));
    if (!image || !final_T || !n_contrib) return fail(ctx, GESR_ERR_INVALID, "image/final_T/n_contrib is NULL");
    if (counts && (!counts->n_listed || !counts->n_hit))
        return fail(ctx, GESR_ERR_INVALID, "counts given with a NULL array");
    const bool ext = channels && (channels->depth || channels->alpha);
    if (ext) GESR_TRY(check_channel_renderer(ctx, st));
    RenderArgs a;
    memset(&a, 0, sizeof a);
    a.n = n;
    a.rec = proj->rec;
    a.val_sorted = bins->val_sorted;
    a.ranges = bins->ranges;
    a.worklist = bins->worklist;
    a.inst_base = bins->inst_base;
    a.n_items = (uint32_t)g.total_tiles;
    a.batch = st->batch > 0 ? st->batch : 64;
    a.tile_work = bins->tile_work;
    a.image = image;
    a.final_T = final_T;
    a.n_contrib = n_contrib;
    a.n_listed = counts ? counts->n_listed : nullptr;
    a.n_hit = counts ? counts->n_hit : nullptr;
    a.out_depth = ext ? channels->depth : nullptr;
    a.out_alpha = ext ? channels->alpha : nullptr;
    a.st = dev_settings(st);
    a.cams = dev_cams(cams, V, st);
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, launch_render_fwd(a, st->tile_w, st->tile_h, counts != nullptr, (hipStream_t)stream),
                       "render_fwd launch"));
    ctx->err.clear();
    return GESR_OK;
}

gesr_status gesr_render_bwd_tiles(gesr_ctx* ctx, const gesr_proj* proj, const gesr_bins* bins,
                                  const gesr_camera* cams, int V, int n, const gesr_settings* st,
                                  const float* final_T, const uint32_t* n_contrib, const float* dL_dimage,
                                  void* workspace, void* stream) {
    return gesr_render_bwd_tiles_ext(ctx, proj, bins, cams, V, n, st, final_T, n_contrib, dL_dimage, nullptr,
                                     workspace, stream);
}

gesr_status gesr_render_bwd_tiles_ext(gesr_ctx* ctx, const gesr_proj* proj, const gesr_bins* bins,
                                      const gesr_camera* cams, int V, int n, const gesr_settings* st,
                                      const float* final_T, const uint32_t* n_contrib, const float* dL_dimage,
                                      const gesr_bwd_channels* channels, void* workspace, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    GESR_TRY(check_settings(ctx, st));
    Geometry g;
    GESR_TRY(check_cams(ctx, cams, V, n, st, &g));
    GESR_TRY(check_proj(ctx, proj));
    GESR_TRY(check_bins(ctx, bins, false));
    if (!final_T || !n_contrib || !dL_dimage) return fail(ctx, GESR_ERR_INVALID, "final_T/n_contrib/dL_dimage is NULL");
    if (!workspace || !aligned16(workspace)) return fail(ctx, GESR_ERR_INVALID, "workspace is NULL or misaligned");
    const bool ext = channels && (channels->dL_ddepth || channels->dL_dalpha);
    if (ext) GESR_TRY(check_channel_renderer(ctx, st));
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    const BwdWorkspace ws = carve_bwd(workspace, g.vn, bins->m_cap, g.total_tiles);
    RenderArgs a;
    memset(&a, 0, sizeof a);
    a.n = n;
    a.rec = proj->rec;
    a.val_sorted = bins->val_sorted;
    a.ranges = bins->ranges;
    a.worklist = bins->worklist;
    a.inst_base = bins->inst_base;
    a.n_items = (uint32_t)g.total_tiles;
    a.batch = st->batch > 0 ? st->batch : 64;
    a.final_T = const_cast<float*>(final_T);
    a.n_contrib = const_cast<uint32_t*>(n_contrib);
    a.dL_dimage = dL_dimage;
    a.dL_ddepth = ext ? channels->dL_ddepth : nullptr;
    a.dL_dalpha = ext ? channels->dL_dalpha : nullptr;
    a.partials = ws.partials;
    a.m_cap = (uint32_t)bins->m_cap;
    a.visited = ws.visited;
    a.st = dev_settings(st);
    a.cams = dev_cams(cams, V, st);
    const int batch = st->batch > 0 ? st->batch : 64;
    GESR_TRY(hip_check(ctx, launch_fill_u32(ws.visited, 0u, (bins->m_cap + 31) / 32, (hipStream_t)stream),
                       "visited bits"));
    GESR_TRY(hip_check(ctx, launch_render_bwd(a, st->tile_w, st->tile_h, batch, (hipStream_t)stream),
                       "render_bwd launch"));
    ctx->err.clear();
    return GESR_OK;
}

gesr_status gesr_project_bwd(gesr_ctx* ctx, const gesr_splats* splats, const gesr_proj* proj, const gesr_bins* bins,
                             const gesr_camera* cams, int V, const gesr_settings* st, void* workspace,
                             float* grad2d, const gesr_grads* out, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    GESR_TRY(check_settings(ctx, st));
    GESR_TRY(check_splats(ctx, splats, st->sh_degree, false));
    Geometry g;
    GESR_TRY(check_cams(ctx, cams, V, splats->n, st, &g));
    GESR_TRY(check_proj(ctx, proj));
    GESR_TRY(check_bins(ctx, bins, false));
    if (!workspace || !aligned16(workspace)) return fail(ctx, GESR_ERR_INVALID, "workspace is NULL or misaligned");
    if (grad2d && !aligned16(grad2d)) return fail(ctx, GESR_ERR_INVALID, "grad2d is misaligned");
    if (!out) return fail(ctx, GESR_ERR_INVALID, "out is NULL");
    if (splats->n > 0) {
        const void* ptrs[6] = {out->mean, out->scale, out->quat, out->opacity, out->beta, out->sh};
        for (int k = 0; k < 6; ++k)
            if (!ptrs[k] || !aligned16(ptrs[k])) return fail(ctx, GESR_ERR_INVALID, "gradient output %d invalid", k);
    }
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    const BwdWorkspace ws = carve_bwd(workspace, g.vn, bins->m_cap, g.total_tiles);
    const DevCams dc = dev_cams(cams, V, st);
    float* g2 = grad2d ? grad2d : ws.grad2d;
    SegReduceArgs r;
    r.vn = (uint32_t)g.vn;
    r.tiles_touched = proj->tiles_touched;
    r.inst_base = bins->inst_base;
    r.visited = ws.visited;
    r.partials = ws.partials;
    r.m_cap = bins->m_cap;
    r.grad2d = g2;
    GESR_TRY(hip_check(ctx, launch_seg_reduce(r, (hipStream_t)stream), "seg_reduce launch"));
    ProjectBwdArgs b;
    b.n = splats->n;
    b.mean = splats->mean;
    b.scale = splats->scale;
    b.quat = splats->quat;
    b.opacity = splats->opacity;
    b.beta = splats->beta;
    b.sh = splats->sh;
    b.tiles_touched = proj->tiles_touched;
    b.grad2d = g2;
    b.g_mean = out->mean;
    b.g_scale = out->scale;
    b.g_quat = out->quat;
    b.g_opacity = out->opacity;
    b.g_beta = out->beta;
    b.g_sh = out->sh;
    b.st = dev_settings(st);
    b.cams = dc;
    GESR_TRY(hip_check(ctx, launch_project_bwd(b, st->sh_degree, (hipStream_t)stream), "project_bwd launch"));
    ctx->err.clear();
    return GESR_OK;
}

gesr_status gesr_render_bwd(gesr_ctx* ctx, const gesr_splats* splats, const gesr_proj* proj, const gesr_bins* bins,
                            const gesr_camera* cams, int V, const gesr_settings* st, const float* final_T,
                            const uint32_t* n_contrib, const float* dL_dimage, void* workspace, float* grad2d,
                            const gesr_grads* out, void* stream) {
    return gesr_render_bwd_ext(ctx, splats, proj, bins, cams, V, st, final_T, n_contrib, dL_dimage, nullptr,
                               workspace, grad2d, out, stream);
}

gesr_status gesr_render_bwd_ext(gesr_ctx* ctx, const gesr_splats* splats, const gesr_proj* proj,
                                const gesr_bins* bins, const gesr_camera* cams, int V, const gesr_settings* st,
                                const float* final_T, const uint32_t* n_contrib, const float* dL_dimage,
                                const gesr_bwd_channels* channels, void* workspace, float* grad2d,
                                const gesr_grads* out, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!splats) return fail(ctx, GESR_ERR_INVALID, "splats is NULL");
    if (!out) return fail(ctx, GESR_ERR_INVALID, "out is NULL");
    GESR_TRY(gesr_render_bwd_tiles_ext(ctx, proj, bins, cams, V, splats->n, st, final_T, n_contrib, dL_dimage,
                                       channels, workspace, stream));
    return gesr_project_bwd(ctx, splats, proj, bins, cams, V, st, workspace, grad2d, out, stream);
}

gesr_status gesr_surface_points(gesr_ctx* ctx, const gesr_splats* splats, const gesr_proj* proj,
                                const gesr_bins* bins, const gesr_camera* cams, int V, const gesr_settings* st,
                                const gesr_surface_settings* ss, const float* depth, const float* alpha,
                                const uint32_t* pixels, uint32_t n_rays, float* points, float* normals,
                                uint32_t* dominant, uint32_t* n_candidates, void* workspace, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    GESR_TRY(check_settings(ctx, st));
    GESR_TRY(check_splats(ctx, splats, st->sh_degree, false));
    Geometry g;
    GESR_TRY(check_cams(ctx, cams, V, splats->n, st, &g));
    GESR_TRY(check_proj(ctx, proj));
    GESR_TRY(check_bins(ctx, bins, false));
    if (!ss) return fail(ctx, GESR_ERR_INVALID, "surface settings are NULL");
    if (ss->n_samples < 2 || ss->n_samples > GESR_SURFACE_MAX_SAMPLES)
        return fail(ctx, GESR_ERR_INVALID, "n_samples %d outside 2..%d", ss->n_samples, GESR_SURFACE_MAX_SAMPLES);
    if (!(ss->level > 0.f) || !(ss->span > 0.f) || !(ss->min_alpha >= 0.f))
        return fail(ctx, GESR_ERR_INVALID, "level and span must be > 0, min_alpha >= 0");
    if (n_rays == 0) {
        ctx->err.clear();
        return GESR_OK;
    }
    if (!depth || !alpha || !pixels || !points || !normals)
        return fail(ctx, GESR_ERR_INVALID, "depth/alpha/pixels/points/normals is NULL");
    if (!aligned16(points) || !aligned16(normals)) return fail(ctx, GESR_ERR_INVALID, "points/normals misaligned");
    if (splats->n > 0 && (!workspace || !aligned16(workspace)))
        return fail(ctx, GESR_ERR_INVALID, "workspace is NULL or misaligned");
    SurfaceArgs a;
    memset(&a, 0, sizeof a);
    a.n = splats->n;
    a.mean = splats->mean;
    a.scale = splats->scale;
    a.quat = splats->quat;
    a.opacity = splats->opacity;
    a.beta = splats->beta;
    a.rec = proj->rec;
    a.val_sorted = bins->val_sorted;
    a.ranges = bins->ranges;
    a.depth = depth;
    a.alpha = alpha;
    a.pixels = pixels;
    a.n_rays = n_rays;
    a.n_samples = ss->n_samples;
    a.level = ss->level;
    a.span = ss->span;
    a.min_alpha = ss->min_alpha;
    a.tile_w = st->tile_w;
    a.tile_h = st->tile_h;
    a.points = points;
    a.normals = normals;
    a.dominant = dominant;
    a.n_candidates = n_candidates;
    a.frames = (float*)workspace;
    a.st = dev_settings(st);
    a.cams = dev_cams(cams, V, st);
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, launch_surface_points(a, (hipStream_t)stream), "surface_points launch"));
    ctx->err.clear();
    return GESR_OK;
}

}  // extern "C"

namespace {

// Views and workspace layout of gesr_loss_eq8: 16 x 16 tiles per view; the
// three adjoint maps [3P] and the per-tile partial sums [T][2], 256-byte aligned.
struct LossLayout {
    bool ok;
    uint64_t pixels, tiles;
    size_t o_b, o_c, o_partial, bytes;
};

LossLayout loss_layout(const gesr_camera* cams, int V, gesr::LossArgs* a) {
    LossLayout L{false, 0, 0, 0, 0, 0, 0};
    if (!cams || V < 1 || V > GESR_MAX_VIEWS) return L;
    for (int v = 0; v < V; ++v) {
        const int W = cams[v].width, H = cams[v].height;
        if (W < 1 || H < 1 || W > 65535 || H > 65535) return L;
        if (a) {
            a->v[v].W = W;
            a->v[v].H = H;
            a->v[v].pix_base = (uint32_t)L.pixels;
            a->v[v].tile_base = (uint32_t)L.tiles;
            a->v[v].inv_n = (float)(1.0 / (3.0 * (double)W * (double)H));
        }
        L.pixels += (uint64_t)W * H;
        L.tiles += (uint64_t)((W + 15) / 16) * ((H + 15) / 16);
    }
    if (3 * L.pixels >= (1ull << 32)) return L;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t map = al(3 * L.pixels * sizeof(float));
    L.o_b = map;
    L.o_c = 2 * map;
    L.o_partial = 3 * map;
    L.bytes = 3 * map + al(2 * L.tiles * sizeof(float));
    L.ok = true;
    return L;
}

}  // namespace

extern "C" {

void gesr_default_loss_settings(gesr_loss_settings* s) {
    if (!s) return;
    s->lambda_dssim = 0.2f;
    s->c1 = 0.01f * 0.01f;
    s->c2 = 0.03f * 0.03f;
    s->sigma = 1.5f;
}

size_t gesr_loss_workspace_size(const gesr_camera* cams, int V) {
    const LossLayout L = loss_layout(cams, V, nullptr);
    return L.ok ? L.bytes : 0;
}

gesr_status gesr_loss_eq8(gesr_ctx* ctx, const gesr_camera* cams, int V, const gesr_loss_settings* ls,
                          const float* image, const float* target, float* grad, float* loss, void* workspace,
                          size_t workspace_bytes, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!ls) return fail(ctx, GESR_ERR_INVALID, "loss settings are NULL");
    if (!(ls->lambda_dssim >= 0.0f && ls->lambda_dssim <= 1.0f))
        return fail(ctx, GESR_ERR_INVALID, "lambda_dssim must be in [0, 1]");
    if (!(ls->c1 > 0.0f) || !(ls->c2 > 0.0f) || !isfinite(ls->c1) || !isfinite(ls->c2))
        return fail(ctx, GESR_ERR_INVALID, "c1 and c2 must be positive and finite");
    if (!(ls->sigma > 0.0f) || !isfinite(ls->sigma)) return fail(ctx, GESR_ERR_INVALID, "sigma must be positive");
    gesr::LossArgs a;
    memset(&a, 0, sizeof a);
    const LossLayout L = loss_layout(cams, V, &a);
    if (!L.ok) return fail(ctx, GESR_ERR_INVALID, "views: V in 1..%d, sizes 1..65535, 3 P < 2^32", GESR_MAX_VIEWS);
    const void* ptrs[4] = {image, target, grad, workspace};
    const char* names[4] = {"image", "target", "grad", "workspace"};
    for (int k = 0; k < 4; ++k) {
        if (!ptrs[k]) return fail(ctx, GESR_ERR_INVALID, "%s is NULL", names[k]);
        if (!aligned16(ptrs[k])) return fail(ctx, GESR_ERR_INVALID, "%s is not 16-byte aligned", names[k]);
    }
    if (grad == image || grad == target) return fail(ctx, GESR_ERR_INVALID, "grad aliases image or target");
    if (workspace_bytes < L.bytes)
        return fail(ctx, GESR_ERR_INVALID, "workspace_bytes %zu < required %zu", workspace_bytes, L.bytes);
    a.V = V;
    double wsum = 0.0, wd[2 * GESR_LOSS_RADIUS + 1];
    for (int k = -GESR_LOSS_RADIUS; k <= GESR_LOSS_RADIUS; ++k) {
        wd[k + GESR_LOSS_RADIUS] = exp(-(double)(k * k) / (2.0 * (double)ls->sigma * ls->sigma));
        wsum += wd[k + GESR_LOSS_RADIUS];
    }
    for (int k = 0; k <= 2 * GESR_LOSS_RADIUS; ++k) a.w[k] = (float)(wd[k] / wsum);
    a.lam = ls->lambda_dssim;
    a.c1 = ls->c1;
    a.c2 = ls->c2;
    a.image = image;
    a.target = target;
    char* ws = (char*)workspace;
    a.amap = (float*)ws;
    a.bmap = (float*)(ws + L.o_b);
    a.cmap = (float*)(ws + L.o_c);
    a.partial = (float*)(ws + L.o_partial);
    a.grad = grad;
    a.loss = loss;
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, gesr::launch_ssim_loss(a, (uint32_t)L.tiles, loss != nullptr, (hipStream_t)stream),
                       "loss launch"));
    ctx->err.clear();
    return GESR_OK;
}

size_t gesr_align_workspace_size(int n) { return n > 0 ? (size_t)((n + 255) / 256) * 2 * sizeof(float) + 256 : 0; }

gesr_status gesr_surface_align(gesr_ctx* ctx, const gesr_splats* splats, const float* normals, float w_scale,
                               float w_normal, const gesr_grads* grads, float* losses, void* workspace,
                               size_t workspace_bytes, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!splats || splats->n < 0) return fail(ctx, GESR_ERR_INVALID, "splats is NULL or n is negative");
    if (!isfinite(w_scale) || !isfinite(w_normal)) return fail(ctx, GESR_ERR_INVALID, "weights must be finite");
    const int n = splats->n;
    if (n == 0) {
        ctx->err.clear();
        return GESR_OK;
    }
    if (!grads) return fail(ctx, GESR_ERR_INVALID, "grads is NULL");
    const void* ptrs[5] = {splats->scale, splats->quat, normals, grads->scale, grads->quat};
    const char* names[5] = {"splats->scale", "splats->quat", "normals", "grads->scale", "grads->quat"};
    for (int k = 0; k < 5; ++k) {
        if (!ptrs[k]) return fail(ctx, GESR_ERR_INVALID, "%s is NULL", names[k]);
        if (!aligned16(ptrs[k])) return fail(ctx, GESR_ERR_INVALID, "%s is not 16-byte aligned", names[k]);
    }
    if (losses && (!workspace || workspace_bytes < gesr_align_workspace_size(n)))
        return fail(ctx, GESR_ERR_INVALID, "losses need a workspace of %zu bytes", gesr_align_workspace_size(n));
    gesr::AlignArgs a;
    a.n = n;
    a.scale = splats->scale;
    a.quat = splats->quat;
    a.normal = normals;
    a.w_scale_n = w_scale / (float)n;
    a.w_normal_n = w_normal / (float)n;
    a.g_scale = grads->scale;
    a.g_quat = grads->quat;
    a.partial = losses ? (float*)workspace : nullptr;
    a.losses = losses;
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, gesr::launch_surface_align(a, (hipStream_t)stream), "align launch"));
    ctx->err.clear();
    return GESR_OK;
}

gesr_status gesr_l1_grad(gesr_ctx* ctx, const float* image, const float* target, uint64_t count, float scale,
                         float* grad, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (count > 0 && (!image || !target || !grad)) return fail(ctx, GESR_ERR_INVALID, "NULL array");
    if (!isfinite(scale)) return fail(ctx, GESR_ERR_INVALID, "scale must be finite");
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, launch_l1_grad(image, target, count, scale, grad, (hipStream_t)stream), "l1 launch"));
    ctx->err.clear();
    return GESR_OK;
}

void gesr_default_adam_settings(gesr_adam_settings* s) {
    if (!s) return;
    memset(s, 0, sizeof *s);
    s->lr_mean = 1.6e-4f;
    s->lr_scale = 5e-3f;
    s->lr_quat = 1e-3f;
    s->lr_opacity = 0.05f;
    s->lr_beta = 1.5e-3f;
    s->lr_sh_dc = 2.5e-3f;
    s->lr_sh_rest = 2.5e-3f / 20.0f;
    s->beta1 = 0.9f;
    s->beta2 = 0.999f;
    s->eps = 1e-15f;
    s->entropy_weight = 0.0f;
    s->step = 1;
}

gesr_status gesr_adam_step(gesr_ctx* ctx, const gesr_params* p, const gesr_params* m, const gesr_params* v,
                           const gesr_grads* grads, const gesr_adam_settings* st, float* scale_out,
                           float* opacity_out, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!p || !m || !v || !grads || !st) return fail(ctx, GESR_ERR_INVALID, "NULL argument");
    if (p->n < 0) return fail(ctx, GESR_ERR_INVALID, "params->n is negative");
    if (p->sh_coeffs < 1 || p->sh_coeffs > 16) return fail(ctx, GESR_ERR_INVALID, "sh_coeffs %d outside 1..16",
                                                           p->sh_coeffs);
    if (m->n != p->n || v->n != p->n || m->sh_coeffs != p->sh_coeffs || v->sh_coeffs != p->sh_coeffs)
        return fail(ctx, GESR_ERR_INVALID, "params and moments differ in n or sh_coeffs");
    if (st->step < 1) return fail(ctx, GESR_ERR_INVALID, "step must be >= 1");
    const float lrs[7] = {st->lr_mean, st->lr_scale, st->lr_quat, st->lr_opacity, st->lr_beta, st->lr_sh_dc,
                          st->lr_sh_rest};
    for (float lr : lrs)
        if (!(lr >= 0.f) || !isfinite(lr)) return fail(ctx, GESR_ERR_INVALID, "learning rates must be finite and >= 0");
    if (!(st->beta1 >= 0.f && st->beta1 < 1.f) || !(st->beta2 >= 0.f && st->beta2 < 1.f))
        return fail(ctx, GESR_ERR_INVALID, "beta1 and beta2 must be in [0, 1)");
    if (!(st->eps > 0.f) || !isfinite(st->eps)) return fail(ctx, GESR_ERR_INVALID, "eps must be finite and > 0");
    if (!isfinite(st->entropy_weight)) return fail(ctx, GESR_ERR_INVALID, "entropy_weight must be finite");
    const int n = p->n;
    if (n > 0) {
        const gesr_params* sets[3] = {p, m, v};
        for (const gesr_params* q : sets) {
            const void* ptrs[6] = {q->mean, q->log_scale, q->quat, q->opacity_logit, q->beta, q->sh};
            for (const void* ptr : ptrs)
                if (!ptr || !aligned16(ptr))
                    return fail(ctx, GESR_ERR_INVALID, "parameter or moment array NULL or not 16-byte aligned");
        }
        const void* gp[8] = {grads->mean, grads->scale, grads->quat, grads->opacity, grads->beta, grads->sh,
                             scale_out, opacity_out};
        for (const void* ptr : gp)
            if (!ptr || !aligned16(ptr))
                return fail(ctx, GESR_ERR_INVALID, "gradient or output array NULL or not 16-byte aligned");
    }
    AdamArgs a{};
    a.n = n;
    a.p = *p;
    a.m = *m;
    a.v = *v;
    a.g_mean = grads->mean;
    a.g_scale = grads->scale;
    a.g_quat = grads->quat;
    a.g_opacity = grads->opacity;
    a.g_beta = grads->beta;
    a.g_sh = grads->sh;
    a.lr_mean = st->lr_mean;
    a.lr_scale = st->lr_scale;
    a.lr_quat = st->lr_quat;
    a.lr_opacity = st->lr_opacity;
    a.lr_beta = st->lr_beta;
    a.lr_sh_dc = st->lr_sh_dc;
    a.lr_sh_rest = st->lr_sh_rest;
    a.beta1 = st->beta1;
    a.beta2 = st->beta2;
    a.eps = st->eps;
    // bias corrections in double on the host, rounded once
    a.inv_c1 = (float)(1.0 / (1.0 - pow((double)st->beta1, (double)st->step)));
    a.inv_c2 = (float)(1.0 / (1.0 - pow((double)st->beta2, (double)st->step)));
    a.entropy_scale = n > 0 ? (float)((double)st->entropy_weight / (double)n) : 0.f;
    a.scale_out = scale_out;
    a.opacity_out = opacity_out;
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, launch_adam_step(a, 12 + 3 * p->sh_coeffs, (hipStream_t)stream), "adam launch"));
    ctx->err.clear();
    return GESR_OK;
}

size_t gesr_prune_workspace_size(int n) { return n < 0 ? 0 : prune_workspace_bytes(n); }

namespace {
// The six arrays of a gesr_params in the kernels' order, with their row counts.
void param_arrays(const gesr_params* q, float* out[6]) {
    out[0] = q->mean;
    out[1] = q->log_scale;
    out[2] = q->quat;
    out[3] = q->opacity_logit;
    out[4] = q->beta;
    out[5] = q->sh;
}
}  // namespace

gesr_status gesr_prune(gesr_ctx* ctx, const gesr_params* p, const gesr_params* m, const gesr_params* v,
                       const gesr_prune_settings* ps, const gesr_params* out_p, const gesr_params* out_m,
                       const gesr_params* out_v, float* scale_out, float* opacity_out, uint32_t* n_kept,
                       void* workspace, size_t workspace_bytes, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!p || !ps || !out_p || !n_kept) return fail(ctx, GESR_ERR_INVALID, "NULL argument");
    if ((m == nullptr) != (v == nullptr)) return fail(ctx, GESR_ERR_INVALID, "give both moments or neither");
    if (m && (!out_m || !out_v)) return fail(ctx, GESR_ERR_INVALID, "moment outputs missing");
    if (p->n < 0) return fail(ctx, GESR_ERR_INVALID, "params->n is negative");
    if (p->sh_coeffs < 1 || p->sh_coeffs > 16)
        return fail(ctx, GESR_ERR_INVALID, "sh_coeffs %d outside 1..16", p->sh_coeffs);
    if (m && (m->n != p->n || v->n != p->n || m->sh_coeffs != p->sh_coeffs || v->sh_coeffs != p->sh_coeffs))
        return fail(ctx, GESR_ERR_INVALID, "params and moments differ in n or sh_coeffs");
    if (!(ps->min_opacity >= 0.f && ps->min_opacity < 1.f))
        return fail(ctx, GESR_ERR_INVALID, "min_opacity must be in [0, 1)");
    if (!isfinite(ps->min_beta)) return fail(ctx, GESR_ERR_INVALID, "min_beta must be finite");
    if (!aligned16(n_kept)) return fail(ctx, GESR_ERR_INVALID, "n_kept is not 16-byte aligned");
    const int n = p->n;
    const size_t need = prune_workspace_bytes(n);
    if (!workspace || !aligned16(workspace) || workspace_bytes < need)
        return fail(ctx, GESR_ERR_INVALID, "workspace NULL, misaligned or smaller than %zu bytes", need);
    PruneArgs a{};
    a.n = n;
    const gesr_params* ins[3] = {p, m, v};
    const gesr_params* outs[3] = {out_p, out_m, out_v};
    for (int s = 0; s < 3; ++s) {
        if (!ins[s]) continue;
        float* in6[6];
        float* out6[6];
        param_arrays(ins[s], in6);
        param_arrays(outs[s], out6);
        for (int k = 0; k < 6; ++k) {
            if (n > 0 && (!in6[k] || !aligned16(in6[k]) || !out6[k] || !aligned16(out6[k])))
                return fail(ctx, GESR_ERR_INVALID, "parameter array NULL or not 16-byte aligned");
            if (s == 0) a.in_p[k] = in6[k], a.out_p[k] = out6[k];
            if (s == 1) a.in_m[k] = in6[k], a.out_m[k] = out6[k];
            if (s == 2) a.in_v[k] = in6[k], a.out_v[k] = out6[k];
        }
    }
    if (n > 0 && ((scale_out && !aligned16(scale_out)) || (opacity_out && !aligned16(opacity_out))))
        return fail(ctx, GESR_ERR_INVALID, "scale_out or opacity_out not 16-byte aligned");
    a.logit = p->opacity_logit;
    a.beta = p->beta;
    a.t_logit = ps->min_opacity > 0.f
                    ? (float)log((double)ps->min_opacity / (1.0 - (double)ps->min_opacity))
                    : -INFINITY;
    a.min_beta = ps->min_beta > 0.f ? ps->min_beta : -INFINITY;
    const uint32_t nb = prune_blocks(n);
    uint32_t* w = (uint32_t*)workspace;
    a.n_kept = n_kept;
    a.bits = w;
    a.counts = w + (size_t)nb * 32;
    a.offsets = a.counts + nb;
    uint32_t* partials = a.offsets + nb;
    a.scale_out = scale_out;
    a.opacity_out = opacity_out;
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, launch_prune(a, 12 + 3 * p->sh_coeffs, partials, (hipStream_t)stream), "prune launch"));
    ctx->err.clear();
    return GESR_OK;
}

gesr_status gesr_shape_reset(gesr_ctx* ctx, const gesr_params* p, const gesr_params* m, const gesr_params* v,
                             float value, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!p) return fail(ctx, GESR_ERR_INVALID, "params is NULL");
    if (p->n < 0) return fail(ctx, GESR_ERR_INVALID, "params->n is negative");
    if (!(value > 0.f) || !isfinite(value)) return fail(ctx, GESR_ERR_INVALID, "value must be finite and > 0");
    if (p->n > 0 && !p->beta) return fail(ctx, GESR_ERR_INVALID, "params->beta is NULL");
    if ((m && m->n != p->n) || (v && v->n != p->n)) return fail(ctx, GESR_ERR_INVALID, "moments differ in n");
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, launch_shape_reset(p->beta, m ? m->beta : nullptr, v ? v->beta : nullptr, p->n, value,
                                               (hipStream_t)stream),
                       "shape reset launch"));
    ctx->err.clear();
    return GESR_OK;
}

size_t gesr_knn_workspace_size(int n, int k) {
    if (n < 0 || k < 1 || k > GESR_KNN_MAX) return 0;
    return (size_t)knn_layout(n, k).words * 4 + 256;
}

gesr_status gesr_knn(gesr_ctx* ctx, const gesr_splats* splats, int k, uint32_t* knn, uint32_t* order,
                     uint32_t* inv_offsets, uint32_t* inv_entries, uint32_t* inv_slot, void* workspace,
                     size_t workspace_bytes, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!splats) return fail(ctx, GESR_ERR_INVALID, "splats is NULL");
    if (splats->n < 0) return fail(ctx, GESR_ERR_INVALID, "splats->n is negative");
    if (k < 1 || k > GESR_KNN_MAX) return fail(ctx, GESR_ERR_INVALID, "k = %d outside 1..%d", k, GESR_KNN_MAX);
    const int n = splats->n;
    if ((uint64_t)n * (uint64_t)k >= (1ull << 32)) return fail(ctx, GESR_ERR_INVALID, "n * k must be < 2^32");
    if (!inv_offsets || !aligned16(inv_offsets)) return fail(ctx, GESR_ERR_INVALID, "inv_offsets NULL or misaligned");
    if (n > 0) {
        const void* ptrs[5] = {splats->mean, knn, order, inv_entries, inv_slot};
        for (const void* ptr : ptrs)
            if (!ptr || !aligned16(ptr)) return fail(ctx, GESR_ERR_INVALID, "array NULL or not 16-byte aligned");
    }
    const size_t need = gesr_knn_workspace_size(n, k);
    if (!workspace || !aligned16(workspace) || workspace_bytes < need)
        return fail(ctx, GESR_ERR_INVALID, "workspace NULL, misaligned or smaller than %zu bytes", need);
    // 256-byte alignment of the sub-buffers
    uint32_t* ws = (uint32_t*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, launch_knn(splats->mean, n, k, knn, order, inv_offsets, inv_entries, inv_slot, ws,
                                       (hipStream_t)stream),
                       "knn launch"));
    ctx->err.clear();
    return GESR_OK;
}

size_t gesr_gsr_workspace_size(int n, int k, int with_grads) {
    if (n < 0 || k < 1 || k > GESR_KNN_MAX) return 0;
    const size_t n1 = (size_t)(n > 0 ? n : 1);
    const size_t nparts = (n1 + GSR_SUM_BLOCK - 1) / GSR_SUM_BLOCK;
    // frames, per-sample results and loss partials, rounded to 256 bytes
    size_t floats = (n1 * GSR_FRAME_FLOATS + n1 * 4 + 2 * nparts + 63) & ~(size_t)63;
    if (with_grads) floats += n1 * (size_t)k * GSR_PARTIAL_STRIDE;
    return floats * 4 + 256;
}

gesr_status gesr_gsr(gesr_ctx* ctx, const gesr_splats* splats, const gesr_settings* st, int k, const uint32_t* knn,
                     const uint32_t* order, const uint32_t* inv_offsets, const uint32_t* inv_slot, const float* xi,
                     const uint8_t* mask,
                     const gesr_gsr_settings* gs, float* sample_out, float* losses, const gesr_grads* grads,
                     void* workspace, size_t workspace_bytes, void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!splats || !st || !gs) return fail(ctx, GESR_ERR_INVALID, "NULL argument");
    GESR_TRY(check_settings(ctx, st));
    if (splats->n < 0) return fail(ctx, GESR_ERR_INVALID, "splats->n is negative");
    if (k < 1 || k > GESR_KNN_MAX) return fail(ctx, GESR_ERR_INVALID, "k = %d outside 1..%d", k, GESR_KNN_MAX);
    if (!isfinite(gs->w_sdf) || !isfinite(gs->w_nor)) return fail(ctx, GESR_ERR_INVALID, "weights must be finite");
    const int n = splats->n;
    if ((uint64_t)n * (uint64_t)k >= (1ull << 32)) return fail(ctx, GESR_ERR_INVALID, "n * k must be < 2^32");
    if (n > 0) {
        const void* ptrs[9] = {splats->mean, splats->scale, splats->quat, splats->opacity, splats->beta, knn,
                               order, xi, inv_offsets};
        for (const void* ptr : ptrs)
            if (!ptr || !aligned16(ptr)) return fail(ctx, GESR_ERR_INVALID, "array NULL or not 16-byte aligned");
        if (sample_out && !aligned16(sample_out)) return fail(ctx, GESR_ERR_INVALID, "sample_out not 16-byte aligned");
        if (grads) {
            const void* gp[6] = {grads->mean, grads->scale, grads->quat, grads->opacity, grads->beta, inv_slot};
            for (const void* ptr : gp)
                if (!ptr || !aligned16(ptr))
                    return fail(ctx, GESR_ERR_INVALID, "gradient or inverse-list array NULL or misaligned");
        }
    }
    if (losses && !aligned16(losses)) return fail(ctx, GESR_ERR_INVALID, "losses not 16-byte aligned");
    const size_t need = gesr_gsr_workspace_size(n, k, grads != nullptr);
    if (!workspace || !aligned16(workspace) || workspace_bytes < need)
        return fail(ctx, GESR_ERR_INVALID, "workspace NULL, misaligned or smaller than %zu bytes", need);
    float* ws = (float*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    const size_t n1 = (size_t)(n > 0 ? n : 1);
    GsrArgs a{};
    a.n = n;
    a.k = k;
    a.mean = splats->mean;
    a.scale = splats->scale;
    a.quat = splats->quat;
    a.opacity = splats->opacity;
    a.beta = splats->beta;
    a.knn = knn;
    a.order = order;
    a.inv_offsets = inv_offsets;
    a.inv_slot = inv_slot;
    a.xi = xi;
    a.mask = mask;
    a.kappa = st->kappa;
    a.rho = st->rho;
    a.w_sdf = gs->w_sdf;
    a.w_nor = gs->w_nor;
    a.frames = ws;
    a.sample_out = sample_out ? sample_out : ws + n1 * GSR_FRAME_FLOATS;
    const size_t nparts = (n1 + GSR_SUM_BLOCK - 1) / GSR_SUM_BLOCK;
    a.sum_parts = ws + n1 * GSR_FRAME_FLOATS + n1 * 4;
    // partial records start 256-byte aligned
    a.partials = grads ? ws + ((n1 * GSR_FRAME_FLOATS + n1 * 4 + 2 * nparts + 63) & ~(size_t)63) : nullptr;
    a.losses = losses;
    if (grads) {
        a.g_mean = grads->mean;
        a.g_scale = grads->scale;
        a.g_quat = grads->quat;
        a.g_opacity = grads->opacity;
        a.g_beta = grads->beta;
    }
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    GESR_TRY(hip_check(ctx, launch_gsr(a, (hipStream_t)stream), "gsr launch"));
    ctx->err.clear();
    return GESR_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ autotuner
namespace {

struct Candidate {
    int tw, th, variant, batch, radix;
};
// Renderer candidates (digit width 8), then digit widths for the best of them.
constexpr Candidate kRenderCands[] = {{16, 16, 0, 64, 8},  {16, 16, 0, 32, 8}, {16, 16, 1, 64, 8},
                                      {16, 16, 1, 128, 8}, {8, 8, 0, 64, 8},   {32, 16, 0, 64, 8},
                                      {32, 16, 0, 128, 8}, {32, 32, 0, 64, 8}};
constexpr int kNumRender = (int)(sizeof(kRenderCands) / sizeof(kRenderCands[0]));
constexpr int kRadixCands[] = {7, 6, 5};
constexpr int kNumCands = kNumRender + (int)(sizeof(kRadixCands) / sizeof(kRadixCands[0]));

// Device buffer owned by one trial.
struct DevBuf {
    void* p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    bool alloc(size_t bytes) {
        release();
        if (hipMalloc(&p, bytes > 256 ? bytes : 256) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return false;
        }
        return true;
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Milliseconds per forward + backward pipeline for settings `st`, or -1.
float autotune_trial(gesr_ctx* ctx, const gesr_splats* sp, const gesr_camera* cams, int V, const gesr_settings& st,
                     int reps, hipStream_t strm) {
    Geometry g;
    if (check_cams(ctx, cams, V, sp->n, &st, &g) != GESR_OK) return -1.f;
    const int n = sp->n;
    const uint64_t vn = g.vn, P = g.total_pixels, T = g.total_tiles;
    const uint64_t K = (uint64_t)(st.sh_degree + 1) * (uint64_t)(st.sh_degree + 1);
    DevBuf projbuf;
    const size_t o_tt = align256(vn * GESR_REC_FLOATS * 4), o_rect = o_tt + align256(vn * 4),
                 o_dk = o_rect + align256(vn * 8), proj_bytes = o_dk + align256(vn * 4);
    if (!projbuf.alloc(proj_bytes)) return -1.f;
    char* pb = projbuf.as<char>();
    gesr_proj proj;
    proj.rec = reinterpret_cast<float*>(pb);
    proj.tiles_touched = reinterpret_cast<uint32_t*>(pb + o_tt);
    proj.rect = reinterpret_cast<uint32_t*>(pb + o_rect);
    proj.depth_key = reinterpret_cast<uint32_t*>(pb + o_dk);
    if (gesr_project(ctx, sp, cams, V, &st, &proj, strm) != GESR_OK) return -1.f;

    // bins with capacity exactly M (as a capturable caller would size them)
    DevBuf binbuf;
    gesr_bins bins;
    auto alloc_bins = [&](uint64_t m_cap) -> bool {
        gesr_sizes sz;
        if (gesr_query_sizes(ctx, cams, V, n, &st, m_cap, &sz) != GESR_OK) return false;
        const size_t o_rng = align256(m_cap * 4), o_wl = o_rng + align256(T * 8), o_ib = o_wl + align256(T * 4),
                     o_cnt = o_ib + align256((vn > 0 ? vn : 1) * 4), o_scr = o_cnt + 256,
                     o_tw = o_scr + align256(sz.bin_scratch_bytes), bytes = o_tw + align256(T * 4);
        if (!binbuf.alloc(bytes)) return false;
        char* b = binbuf.as<char>();
        bins.m_cap = m_cap;
        bins.tile_sorted = nullptr;
        bins.val_sorted = reinterpret_cast<uint32_t*>(b);
        bins.ranges = reinterpret_cast<uint32_t*>(b + o_rng);
        bins.worklist = reinterpret_cast<uint32_t*>(b + o_wl);
        bins.inst_base = reinterpret_cast<uint32_t*>(b + o_ib);
        bins.counters = reinterpret_cast<uint32_t*>(b + o_cnt);
        bins.scratch = b + o_scr;
        bins.scratch_bytes = sz.bin_scratch_bytes;
        bins.tile_work = reinterpret_cast<uint32_t*>(b + o_tw);
        return true;
    };
    uint64_t m_cap = std::max<uint64_t>(4 * vn, 1024), M = 0;
    for (int attempt = 0;; ++attempt) {
        if (attempt == 3 || !alloc_bins(m_cap)) return -1.f;
        uint64_t m = 0;
        const gesr_status r = gesr_bin(ctx, &proj, cams, V, n, &st, &bins, GESR_BIN_SYNC, &m, strm);
        if (r == GESR_OK) {
            M = m;
            break;
        }
        if (r != GESR_ERR_CAPACITY) return -1.f;
        m_cap = m + 1;
    }
    if (std::max<uint64_t>(M, 1) != m_cap && !alloc_bins(std::max<uint64_t>(M, 1))) return -1.f;
    gesr_sizes sz;
    if (gesr_query_sizes(ctx, cams, V, n, &st, bins.m_cap, &sz) != GESR_OK) return -1.f;

    DevBuf outbuf, wsbuf, gradbuf;
    const size_t o_T = align256(3 * P * 4), o_nc = o_T + align256(P * 4), o_dL = o_nc + align256(P * 4),
                 out_bytes = o_dL + align256(3 * P * 4);
    if (!outbuf.alloc(out_bytes) || !wsbuf.alloc(sz.bwd_workspace_bytes)) return -1.f;
    char* ob = outbuf.as<char>();
    float* image = reinterpret_cast<float*>(ob);
    float* final_T = reinterpret_cast<float*>(ob + o_T);
    uint32_t* n_contrib = reinterpret_cast<uint32_t*>(ob + o_nc);
    float* dL = reinterpret_cast<float*>(ob + o_dL);
    const float unit = 1.0f / (float)(3 * (P > 0 ? P : 1));
    uint32_t unit_bits;
    memcpy(&unit_bits, &unit, 4);
    if (launch_fill_u32(reinterpret_cast<uint32_t*>(dL), unit_bits, 3 * P, strm) != hipSuccess) return -1.f;
    const uint64_t nn = (uint64_t)(n > 0 ? n : 1);
    const size_t gsz[6] = {3 * nn * 4, 3 * nn * 4, 4 * nn * 4, nn * 4, nn * 4, 3 * K * nn * 4};
    size_t goff[6], gbytes = 0;
    for (int k = 0; k < 6; ++k) {
        goff[k] = gbytes;
        gbytes += align256(gsz[k]);
    }
    if (!gradbuf.alloc(gbytes)) return -1.f;
    char* gb = gradbuf.as<char>();
    gesr_grads grads;
    grads.mean = reinterpret_cast<float*>(gb + goff[0]);
    grads.scale = reinterpret_cast<float*>(gb + goff[1]);
    grads.quat = reinterpret_cast<float*>(gb + goff[2]);
    grads.opacity = reinterpret_cast<float*>(gb + goff[3]);
    grads.beta = reinterpret_cast<float*>(gb + goff[4]);
    grads.sh = reinterpret_cast<float*>(gb + goff[5]);

    // the warm-up's forward measures each tile's work; the timed passes order
    // their worklists by it, as a steady-state caller would
    auto pipeline = [&](int bin_flags) -> bool {
        return gesr_project(ctx, sp, cams, V, &st, &proj, strm) == GESR_OK &&
               gesr_bin(ctx, &proj, cams, V, n, &st, &bins, bin_flags, nullptr, strm) == GESR_OK &&
               gesr_render_fwd(ctx, &proj, &bins, cams, V, n, &st, image, final_T, n_contrib, nullptr, strm) ==
                   GESR_OK &&
               gesr_render_bwd(ctx, sp, &proj, &bins, cams, V, &st, final_T, n_contrib, dL, wsbuf.p, nullptr,
                               &grads, strm) == GESR_OK;
    };
    if (!pipeline(0)) return -1.f;  // warm-up
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    float ms = -1.f;
    bool ok = hipEventRecord(e0, strm) == hipSuccess;
    for (int r = 0; ok && r < reps; ++r) ok = pipeline(GESR_BIN_WORK_ORDER);
    ok = ok && hipEventRecord(e1, strm) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok) return -1.f;
    // a capacity overflow would mean the timing covered truncated lists
    uint32_t cnt[2] = {0, 0};
    if (hipMemcpyAsync(cnt, bins.counters, sizeof cnt, hipMemcpyDeviceToHost, strm) != hipSuccess ||
        hipStreamSynchronize(strm) != hipSuccess || cnt[1] != 0)
        return -1.f;
    return ms / (float)reps;
}

void apply_candidate(const Candidate& c, gesr_settings* s) {
    s->tile_w = c.tw;
    s->tile_h = c.th;
    s->variant = c.variant;
    s->batch = c.batch;
    s->radix_bits = c.radix;
}

}  // namespace

extern "C" {

int gesr_autotune_candidate(int k, gesr_settings* out) {
    if (k == -1) return kNumCands;
    if (k < 0 || k >= kNumCands || !out) return -1;
    if (k < kNumRender) apply_candidate(kRenderCands[k], out);
    else out->radix_bits = kRadixCands[k - kNumRender];
    return 0;
}

gesr_status gesr_autotune(gesr_ctx* ctx, const gesr_splats* splats, const gesr_camera* cams, int V,
                          gesr_settings* inout, int reps, float* times_ms, int max_trials, int* n_trials,
                          void* stream) {
    if (!ctx) return GESR_ERR_INVALID;
    if (!inout) return fail(ctx, GESR_ERR_INVALID, "inout is NULL");
    if (reps < 1 || reps > 100) return fail(ctx, GESR_ERR_INVALID, "reps %d outside 1..100", reps);
    if (times_ms && max_trials < 0) return fail(ctx, GESR_ERR_INVALID, "max_trials is negative");
    GESR_TRY(check_settings(ctx, inout));
    GESR_TRY(check_splats(ctx, splats, inout->sh_degree, false));
    Geometry g;
    GESR_TRY(check_cams(ctx, cams, V, splats->n, inout, &g));
    if (n_trials) *n_trials = 0;
    if (splats->n == 0) {
        ctx->err.clear();
        return GESR_OK;
    }
    GESR_TRY(hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice"));
    hipStream_t strm = (hipStream_t)stream;
    int trials = 0, best = -1;
    float best_ms = 0.f;
    auto record = [&](float ms) {
        if (times_ms && trials < max_trials) times_ms[trials] = ms;
        ++trials;
    };
    for (int k = 0; k < kNumRender; ++k) {
        gesr_settings s = *inout;
        apply_candidate(kRenderCands[k], &s);
        const float ms = autotune_trial(ctx, splats, cams, V, s, reps, strm);
        record(ms);
        if (ms >= 0.f && (best < 0 || ms < best_ms)) {
            best = k;
            best_ms = ms;
        }
    }
    if (best < 0) return fail(ctx, GESR_ERR_HIP, "no autotuner candidate could run");
    gesr_settings chosen = *inout;
    apply_candidate(kRenderCands[best], &chosen);
    for (int k = 0; k < kNumCands - kNumRender; ++k) {
        gesr_settings s = chosen;
        s.radix_bits = kRadixCands[k];
        const float ms = autotune_trial(ctx, splats, cams, V, s, reps, strm);
        record(ms);
        if (ms >= 0.f && ms < best_ms) {
            best_ms = ms;
            chosen.radix_bits = s.radix_bits;
        }
    }
    *inout = chosen;
    if (n_trials) *n_trials = trials;
    ctx->err.clear();
    return GESR_OK;
}

}  // extern "C"

static_assert(sizeof(gesr::RenderArgs) < 4000, "kernel arguments too large");
static_assert(sizeof(gesr::ProjectArgs) < 4000, "kernel arguments too large");
static_assert(sizeof(gesr::ProjectBwdArgs) < 4000, "kernel arguments too large");
static_assert(sizeof(gesr::SegReduceArgs) < 4000, "kernel arguments too large");
