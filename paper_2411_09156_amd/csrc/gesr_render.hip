// Tile renderers of the GES rasterizer (gfx950).
//
// Forward: front-to-back alpha blending (Eq. 5 evaluated discretely) of the
// generalized-exponential falloff exp(-kappa q^(beta/2)) (Eq. 3 in screen
// space).  One workgroup per (view, tile) work item, taken in worklist order
// (most work first: the list length, or the positions a previous forward
// evaluated per tile, so the hardware dispatcher schedules greedily by
// load); each wave covers an 8x8 pixel block so lanes of a wave see similar
// footprints.  Splat records are staged through LDS in batches and every lane
// reads them by broadcast.
//
// Backward: the same tile mapping, traversing each pixel's list in reverse
// from its n_contrib and recovering transmittance by division from final_T
// (no per-fragment state is stored in the forward).  Per splat, each wave
// sums its pixels' 10 gradient terms with cross-lane reductions, the waves'
// sums are added in fixed order, and the tile writes one partial per
// instance: no atomics, bitwise reproducible.

#include "gesr_device.h"
#include "gesr_kernels.h"

namespace gesr {

namespace {

template <int TW, int TH>
struct TileMap {
    static constexpr int NT = TW * TH;
    static constexpr int NW = NT / 64;
    static constexpr int WX = TW / 8;
    // pixel offset inside the tile of thread `tid`
    __device__ static __forceinline__ void pixel(int tid, int& lx, int& ly) {
        const int w = tid >> 6, l = tid & 63;
        lx = (w % WX) * 8 + (l & 7);
        ly = (w / WX) * 8 + (l >> 3);
    }
};

struct TileInfo {
    int v;
    int x, y;       // pixel of this thread
    bool inside;
    uint32_t pix;   // index into per-pixel arrays
    uint32_t ch;    // channel stride of the view (H * W)
    uint32_t img;   // index of channel 0 in the image arrays
    uint32_t tx, ty;
    uint32_t r0, r1;  // list range
};

template <int TW, int TH>
__device__ __forceinline__ TileInfo tile_info(const RenderArgs& a, uint32_t t) {
    TileInfo ti;
    ti.v = view_of_tile(a.cams, t);
    const DevView& w = a.cams.v[ti.v];
    const uint32_t lt = t - w.tile_base;
    ti.tx = lt % (uint32_t)w.tiles_x;
    ti.ty = lt / (uint32_t)w.tiles_x;
    int lx, ly;
    TileMap<TW, TH>::pixel(threadIdx.x, lx, ly);
    ti.x = (int)ti.tx * TW + lx;
    ti.y = (int)ti.ty * TH + ly;
    ti.inside = ti.x < w.W && ti.y < w.H;
    const uint32_t local = (uint32_t)ti.y * (uint32_t)w.W + (uint32_t)ti.x;
    ti.pix = w.pix_base + local;
    ti.ch = (uint32_t)w.W * (uint32_t)w.H;
    ti.img = 3u * w.pix_base + local;
    const uint2 r = reinterpret_cast<const uint2*>(a.ranges)[t];
    ti.r0 = r.x;
    ti.r1 = r.y;
    return ti;
}

// Stage record `vi` into LDS as (u, v, L00, L10), (L11, o, beta/2, qmax),
// (r, g, b, -kappa beta); the last is the splat's factor of 2 dL/dq (below).
__device__ __forceinline__ void stage_record(const float* rec, uint32_t vi, float kappa, float4& sa, float4& sb,
                                             float4& sc) {
    const float4* r = reinterpret_cast<const float4*>(rec + (size_t)vi * GESR_REC_FLOATS);
    const float4 b = r[1], c = r[2];
    sa = r[0];
    sb = make_float4(b.x, b.y, 0.5f * b.z, b.w);
    sc = make_float4(c.x, c.y, c.z, -kappa * b.z);
}

// Adds the opacity, beta and footprint gradient terms of one composited
// fragment to gr (partial layout: d/du, d/dv, d/dL00, d/dL10, d/dL11, d/do,
// d/dbeta, d/dr, d/dg, d/db); dLda = dL/dalpha, c2 = -kappa ln2 / 2.  With
// G = exp(-kappa P), P = q^(beta/2):
//   dL/do    = dLda G                        (alpha = o G below the cap)
//   dL/dbeta = dLda o G P (-kappa/2) ln q    = X log2(q) c2,  X = dLda o G P
//   2 dL/dq  = dLda o G P (-kappa beta) / q  = X rc.w / q
// and q = t^2 + w^2 with t = L00 dx + L10 dy, w = L11 dy, (dx, dy) = pixel - (u, v).
__device__ __forceinline__ void add_fragment_grad(const Fragment& f, const float4& ra, const float4& rb,
                                                  float rcw, float dLda, float alpha_max, float c2,
                                                  float (&gr)[GESR_PARTIAL_FLOATS]) {
    if (f.oG > alpha_max) return;  // alpha clamped: no gradient to o, beta or the footprint
    gr[5] = fmaf(dLda, f.G, gr[5]);
    if (!(f.q > 1e-30f)) return;   // pixel at the centre: dq/d(geometry) = 0
    const float X = dLda * f.oG * f.P;
    gr[6] = fmaf(X * f.l2q, c2, gr[6]);
    const float d2 = X * rcw * hw_rcp(f.q);
    const float tq = d2 * f.t, wq = d2 * f.w;
    gr[0] = fmaf(-tq, ra.z, gr[0]);
    gr[1] = fmaf(-tq, ra.w, gr[1]);
    gr[1] = fmaf(-wq, rb.x, gr[1]);
    gr[2] = fmaf(tq, f.dx, gr[2]);
    gr[3] = fmaf(tq, f.dy, gr[3]);
    gr[4] = fmaf(wq, f.dy, gr[4]);
}

constexpr uint32_t kNoInstance = 0xFFFFFFFFu;

// Slot of the instance (splat vi, tile (tx, ty)) in the pair-major order: the
// splat's instance base plus the tile's row-major position in its rectangle.
// When the lists overflowed their capacity the ranges no longer match the
// truncated lists, so a listed splat may not cover the tile or its slot may lie
// beyond the capacity; kNoInstance then suppresses the partial write.
__device__ __forceinline__ uint32_t instance_index(const RenderArgs& a, uint2 r, uint32_t vi, uint32_t tx,
                                                   uint32_t ty) {
    const uint32_t tx0 = r.x & 0xFFFFu, ty0 = r.x >> 16, tx1 = r.y & 0xFFFFu, ty1 = r.y >> 16;
    const uint32_t inst = a.inst_base[vi] + (ty - ty0) * (tx1 - tx0 + 1u) + (tx - tx0);
    const bool inside = tx >= tx0 && tx <= tx1 && ty >= ty0 && ty <= ty1;
    return inside && inst < a.m_cap ? inst : kNoInstance;
}

// Partials of one instance (ten terms, dz with the extended channels, in a
// twelve-float slot): written, and its slot's bit set, unless all are zero
// (the segmented sum adding +-0 or skipping the slot gives the same float
// result, since its running sums start at +0).
template <bool EXT>
__device__ __forceinline__ void write_partial(const RenderArgs& a, uint32_t slot, const float* s) {
    constexpr int NT = EXT ? GESR_PARTIAL_FLOATS + 1 : GESR_PARTIAL_FLOATS;
    bool nz = false;
#pragma unroll
    for (int k = 0; k < NT; ++k) nz |= s[k] != 0.0f;
    if (!nz) return;
    float4* dst = reinterpret_cast<float4*>(a.partials + (size_t)slot * kPartialStride);
    dst[0] = make_float4(s[0], s[1], s[2], s[3]);
    dst[1] = make_float4(s[4], s[5], s[6], s[7]);
    dst[2] = make_float4(s[8], s[9], EXT ? s[10] : 0.0f, 0.0f);
    atomicOr(a.visited + (slot >> 5), 1u << (slot & 31u));
}

template <int TW, int TH, bool COUNT>
__global__ __launch_bounds__(TW * TH) void k_render_fwd(RenderArgs a) {
    constexpr int NT = TW * TH;
    __shared__ float4 sA[NT], sB[NT], sC[NT];
    const uint32_t t = a.worklist[blockIdx.x];
    const TileInfo ti = tile_info<TW, TH>(a, t);
    const DevSettings& st = a.st;
    const float amax = st.alpha_max;
    const float px = (float)ti.x + 0.5f, py = (float)ti.y + 0.5f;

    float T = 1.0f, cr = 0.f, cg = 0.f, cb = 0.f;
    uint32_t contrib = 0, listed = 0, hit = 0;
    bool done = !ti.inside;
    uint32_t stop = ti.r1;  // first list position not evaluated
    for (uint32_t base = ti.r0; base < ti.r1; base += NT) {
        if (__syncthreads_count(done) == NT) {
            stop = base;
            break;
        }
        const uint32_t pos = base + threadIdx.x;
        if (pos < ti.r1) stage_record(a.rec, a.val_sorted[pos], st.kappa, sA[threadIdx.x], sB[threadIdx.x], sC[threadIdx.x]);
        __syncthreads();
        const int cnt = (int)min<uint32_t>(NT, ti.r1 - base);
        if (!done) {
            for (int j = 0; j < cnt; ++j) {
                const float4 ra = sA[j];
                const float4 rb = sB[j];
                Fragment f;
                const float q = ges_q(ra, rb.x, px, py, f);
                if (COUNT) ++listed;
                if (q > rb.w) continue;  // beyond the alpha_min footprint
                ges_alpha(q, rb.z, rb.y, st, amax, f);
                if (f.alpha < st.alpha_min) continue;
                if (COUNT) ++hit;
                const float Tn = T * (1.0f - f.alpha);
                if (Tn < st.t_min) {
                    done = true;
                    break;
                }
                const float4 rc = sC[j];
                const float w = f.alpha * T;
                cr = fmaf(rc.x, w, cr);
                cg = fmaf(rc.y, w, cg);
                cb = fmaf(rc.z, w, cb);
                T = Tn;
                contrib = base + (uint32_t)j + 1u - ti.r0;
            }
        }
    }
    if (a.tile_work && threadIdx.x == 0) a.tile_work[t] = stop - ti.r0;
    if (ti.inside) {
        a.image[ti.img] = fmaf(T, st.bg[0], cr);
        a.image[ti.img + ti.ch] = fmaf(T, st.bg[1], cg);
        a.image[ti.img + 2 * ti.ch] = fmaf(T, st.bg[2], cb);
        a.final_T[ti.pix] = T;
        a.n_contrib[ti.pix] = contrib;
        if (COUNT) {
            a.n_listed[ti.pix] = listed;
            a.n_hit[ti.pix] = hit;
        }
    }
}

template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(TW * TH) void k_render_bwd(RenderArgs a) {
    // The gradient arithmetic may fuse multiply-adds; the alpha, threshold and
    // transmittance evaluation shared with the forward is written with explicit
    // fmaf (or has no multiply-add) and compiles identically in both kernels.
#pragma clang fp contract(fast)
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    constexpr int NP = GESR_PARTIAL_FLOATS;
    static_assert(BATCH <= NT, "batch larger than the workgroup");
    static_assert(NP == 10, "wave_sum10 reduces ten values");
    __shared__ float4 sA[BATCH], sB[BATCH], sC[BATCH];
    __shared__ uint32_t sInst[BATCH];
    __shared__ float sRed[NW][BATCH][NP];
    __shared__ uint32_t sMax[NW];

    const uint32_t t = a.worklist[blockIdx.x];
    const TileInfo ti = tile_info<TW, TH>(a, t);
    const DevSettings& st = a.st;
    const float amax = st.alpha_max;
    const float c2 = -0.5f * kLn2 * st.kappa;
    const float px = (float)ti.x + 0.5f, py = (float)ti.y + 0.5f;
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;

    float T = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    uint32_t nc = 0;
    if (ti.inside) {
        T = a.final_T[ti.pix];
        nc = a.n_contrib[ti.pix];
        g0 = a.dL_dimage[ti.img];
        g1 = a.dL_dimage[ti.img + ti.ch];
        g2 = a.dL_dimage[ti.img + 2 * ti.ch];
    }
    float Br = st.bg[0], Bg = st.bg[1], Bb = st.bg[2];  // colour behind, per unit transmittance

    // deepest list position any pixel of the tile composited
    const uint32_t wmax = wave_max_u32(nc);
    if (lane == 0) sMax[wave] = wmax;
    __syncthreads();
    uint32_t maxnc = 0;
    for (int w = 0; w < NW; ++w) maxnc = max(maxnc, sMax[w]);
    const uint32_t end = ti.r0 + maxnc;  // positions >= end contributed to no pixel
    const int slot = lane < 16 ? wave_sum10_slot(lane) : NP;  // value this lane writes after a reduction

    for (uint32_t hi = end; hi > ti.r0;) {
        const uint32_t lo = (hi - ti.r0 > (uint32_t)BATCH) ? hi - BATCH : ti.r0;
        const int cnt = (int)(hi - lo);
        if ((int)threadIdx.x < cnt) {
            const uint32_t pos = hi - 1u - threadIdx.x;
            const uint32_t vi = a.val_sorted[pos];
            stage_record(a.rec, vi, st.kappa, sA[threadIdx.x], sB[threadIdx.x], sC[threadIdx.x]);
            const float4 r3 = reinterpret_cast<const float4*>(a.rec + (size_t)vi * GESR_REC_FLOATS)[3];
            const uint2 r = make_uint2(__float_as_uint(r3.x), __float_as_uint(r3.y));  // the pair's rectangle
            sInst[threadIdx.x] = instance_index(a, r, vi, ti.tx, ti.ty);
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const uint32_t prel = hi - 1u - (uint32_t)j - ti.r0;  // 0-based list position
            float gr[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) gr[k] = opaque_zero();
            bool act = false;
            if (prel < nc) {
                const float4 ra = sA[j];
                const float4 rb = sB[j];
                Fragment f;
                const float q = ges_q(ra, rb.x, px, py, f);
                if (q <= rb.w) {
                    ges_alpha(q, rb.z, rb.y, st, amax, f);
                    if (f.alpha >= st.alpha_min) {
                        act = true;
                        const float4 rc = sC[j];
                        const float Tk = T * hw_rcp(1.0f - f.alpha);
                        const float aT = f.alpha * Tk;
                        gr[7] = aT * g0;
                        gr[8] = aT * g1;
                        gr[9] = aT * g2;
                        const float dLda = Tk * ((rc.x - Br) * g0 + (rc.y - Bg) * g1 + (rc.z - Bb) * g2);
                        Br = fmaf(f.alpha, rc.x - Br, Br);
                        Bg = fmaf(f.alpha, rc.y - Bg, Bg);
                        Bb = fmaf(f.alpha, rc.z - Bb, Bb);
                        T = Tk;
                        add_fragment_grad(f, ra, rb, rc.w, dLda, st.alpha_max, c2, gr);
                    }
                }
            }
            if (__ballot(act) != 0ull) {
                const float tot = wave_sum10(gr, lane);
                if (slot < NP) sRed[wave][j][slot] = tot;
            } else if ((int)lane < NP) {
                sRed[wave][j][lane] = 0.f;
            }
        }
        __syncthreads();
        for (int jj = threadIdx.x; jj < cnt; jj += NT) {
            if (sInst[jj] == kNoInstance) continue;
            float s[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) s[k] = sRed[0][jj][k];
            for (int w = 1; w < NW; ++w)
#pragma unroll
                for (int k = 0; k < NP; ++k) s[k] += sRed[w][jj][k];
            write_partial<false>(a, sInst[jj], s);
        }
        __syncthreads();
        hi = lo;
    }
}

// Forward, one wave per 16x16 tile with 4 pixels per lane (one per 8x8
// quadrant): a staged splat's LDS reads serve 256 pixels; the wave leaves the
// tile once all its pixels have terminated.
// EXT: also the extended channels (depth composited over zero, alpha = 1 - T).
template <bool COUNT, int B, bool EXT>
__global__ __launch_bounds__(64) void k_render_fwd_wave16(RenderArgs a) {
    static_assert(B >= 1 && B <= 64, "one staged record per lane");
    __shared__ float4 sA[B], sB[B], sC[B];
    const uint32_t t = a.worklist[blockIdx.x];
    const DevSettings& st = a.st;
    const float amax = st.alpha_max;
    const uint32_t lane = __lane_id();
    const int v = view_of_tile(a.cams, t);
    const DevView& w = a.cams.v[v];
    const uint32_t lt = t - w.tile_base;
    const uint32_t tx = lt % (uint32_t)w.tiles_x, ty = lt / (uint32_t)w.tiles_x;
    const uint2 rg = reinterpret_cast<const uint2*>(a.ranges)[t];
    const uint32_t r0 = rg.x, r1 = rg.y;

    float px[4], py[4], T[4], cr[4], cg[4], cb[4], cd[4];
    uint32_t contrib[4], listed[4], hit[4];
    bool done[4], inside[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = (int)tx * 16 + (q & 1) * 8 + (int)(lane & 7);
        const int y = (int)ty * 16 + (q >> 1) * 8 + (int)(lane >> 3);
        px[q] = (float)x + 0.5f;
        py[q] = (float)y + 0.5f;
        T[q] = 1.0f;
        cr[q] = cg[q] = cb[q] = cd[q] = 0.f;
        contrib[q] = listed[q] = hit[q] = 0;
        inside[q] = x < w.W && y < w.H;
        done[q] = !inside[q];
    }
    // the next batch's records are loaded into registers while the current
    // batch is rendered from LDS
    float4 na = make_float4(0.f, 0.f, 0.f, 0.f), nb = na, nc = na;
    auto fetch = [&](uint32_t b) {
        const uint32_t pos = b + lane;
        if ((int)lane < B && pos < r1) {
            const float4* r = reinterpret_cast<const float4*>(a.rec + (size_t)a.val_sorted[pos] * GESR_REC_FLOATS);
            na = r[0];
            nb = r[1];
            nc = r[2];
        }
    };
    fetch(r0);
    uint32_t stop = r1;  // first list position not evaluated
    for (uint32_t base = r0; base < r1; base += B) {
        const bool all_done = done[0] && done[1] && done[2] && done[3];
        if (__ballot(!all_done) == 0ull) {
            stop = base;
            break;
        }
        if ((int)lane < B && base + lane < r1) {
            sA[lane] = na;
            sB[lane] = make_float4(nb.x, nb.y, 0.5f * nb.z, nb.w);
            sC[lane] = nc;
        }
        __syncthreads();
        if (base + B < r1) fetch(base + B);
        const int cnt = (int)min<uint32_t>(B, r1 - base);
        for (int j = 0; j < cnt; ++j) {
            const float4 ra = sA[j];
            const float4 rb = sB[j];
            const float4 rc = sC[j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (done[q]) continue;
                Fragment f;
                const float qq = ges_q(ra, rb.x, px[q], py[q], f);
                if (COUNT) ++listed[q];
                if (qq > rb.w) continue;  // beyond the alpha_min footprint
                // Inside the footprint alpha almost never falls below alpha_min
                // and a pixel terminates once: both decisions are selects, the
                // state changing only where the fragment composites (a zero
                // weight leaves the sums as they are: colours and depths of
                // kept records are finite and non-negative).
                ges_alpha(qq, rb.z, rb.y, st, amax, f);
                const bool ok = !(f.alpha < st.alpha_min);
                if (COUNT) hit[q] += ok ? 1u : 0u;
                const float Tn = T[q] * (1.0f - f.alpha);
                const bool stop = ok && Tn < st.t_min;
                const bool acc = ok && !stop;
                done[q] = stop;
                const float wgt = acc ? f.alpha * T[q] : 0.0f;
                cr[q] = fmaf(rc.x, wgt, cr[q]);
                cg[q] = fmaf(rc.y, wgt, cg[q]);
                cb[q] = fmaf(rc.z, wgt, cb[q]);
                if (EXT) cd[q] = fmaf(rc.w, wgt, cd[q]);  // rc.w: the splat's depth
                T[q] = acc ? Tn : T[q];
                contrib[q] = acc ? base + (uint32_t)j + 1u - r0 : contrib[q];
            }
        }
        __syncthreads();
    }
    if (a.tile_work && lane == 0) a.tile_work[t] = stop - r0;
    const uint32_t ch = (uint32_t)w.W * (uint32_t)w.H;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!inside[q]) continue;
        const int x = (int)tx * 16 + (q & 1) * 8 + (int)(lane & 7);
        const int y = (int)ty * 16 + (q >> 1) * 8 + (int)(lane >> 3);
        const uint32_t local = (uint32_t)y * (uint32_t)w.W + (uint32_t)x;
        const uint32_t pix = w.pix_base + local, img = 3u * w.pix_base + local;
        a.image[img] = fmaf(T[q], st.bg[0], cr[q]);
        a.image[img + ch] = fmaf(T[q], st.bg[1], cg[q]);
        a.image[img + 2 * ch] = fmaf(T[q], st.bg[2], cb[q]);
        a.final_T[pix] = T[q];
        a.n_contrib[pix] = contrib[q];
        if (COUNT) {
            a.n_listed[pix] = listed[q];
            a.n_hit[pix] = hit[q];
        }
        if (EXT) {
            if (a.out_depth) a.out_depth[pix] = cd[q];
            if (a.out_alpha) a.out_alpha[pix] = 1.0f - T[q];
        }
    }
}

// Backward, one wave per 16x16 tile: lane l owns pixel (l & 7, l >> 3) of each
// 8x8 quadrant (4 pixels per lane), so a staged splat's LDS reads and its
// 10-value wave reduction serve 256 pixels, and no cross-wave reduction or
// workgroup barrier beyond the wave itself is needed.  EXT: the extended
// channels' upstream gradients too (depth and opacity as colour channels over
// a zero background; the depth term dz is the eleventh partial value).
template <int B, bool EXT>
__global__ __launch_bounds__(64) void k_render_bwd_wave16(RenderArgs a) {
    // The gradient arithmetic may fuse multiply-adds; the alpha, threshold and
    // transmittance evaluation shared with the forward is written with explicit
    // fmaf (or has no multiply-add) and compiles identically in both kernels.
#pragma clang fp contract(fast)
    static_assert(B >= 1 && B <= 64, "one staged record per lane");
    constexpr int NP = GESR_PARTIAL_FLOATS;
    static_assert(NP == 10, "wave_sum10 reduces ten values");
    __shared__ float4 sA[B], sB[B], sC[B];
    __shared__ uint32_t sInst[B];
    __shared__ float sRed[B][NP + 1];  // column NP: dz (extended channels)
    __shared__ float sZ[EXT ? B : 1];   // staged splat depths (extended channels)

    const uint32_t t = a.worklist[blockIdx.x];
    const DevSettings& st = a.st;
    const float amax = st.alpha_max;
    const float c2 = -0.5f * kLn2 * st.kappa;
    const uint32_t lane = __lane_id();
    const int v = view_of_tile(a.cams, t);
    const DevView& w = a.cams.v[v];
    const uint32_t lt = t - w.tile_base;
    const uint32_t tx = lt % (uint32_t)w.tiles_x, ty = lt / (uint32_t)w.tiles_x;
    const uint2 rg = reinterpret_cast<const uint2*>(a.ranges)[t];
    const uint32_t r0 = rg.x;
    const uint32_t ch = (uint32_t)w.W * (uint32_t)w.H;

    // pixel centres: quadrant q adds (q & 1) * 8 and (q >> 1) * 8 to the lane's base
    const float pxb = (float)(tx * 16 + (lane & 7)) + 0.5f, pyb = (float)(ty * 16 + (lane >> 3)) + 0.5f;
    float T[4], g0[4], g1[4], g2[4], Br[4], Bg[4], Bb[4];
    float gD[4], gA[4], BD[4], BA[4];  // extended channels: upstream gradients, depth and opacity behind
    uint32_t nc[4];
    uint32_t mymax = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = (int)tx * 16 + (q & 1) * 8 + (int)(lane & 7);
        const int y = (int)ty * 16 + (q >> 1) * 8 + (int)(lane >> 3);
        Br[q] = st.bg[0];
        Bg[q] = st.bg[1];
        Bb[q] = st.bg[2];
        T[q] = 0.f;
        g0[q] = g1[q] = g2[q] = 0.f;
        gD[q] = gA[q] = BD[q] = BA[q] = 0.f;
        nc[q] = 0;
        if (x < w.W && y < w.H) {
            const uint32_t local = (uint32_t)y * (uint32_t)w.W + (uint32_t)x;
            const uint32_t pix = w.pix_base + local, img = 3u * w.pix_base + local;
            T[q] = a.final_T[pix];
            nc[q] = a.n_contrib[pix];
            g0[q] = a.dL_dimage[img];
            g1[q] = a.dL_dimage[img + ch];
            g2[q] = a.dL_dimage[img + 2 * ch];
            if (EXT) {
                if (a.dL_ddepth) gD[q] = a.dL_ddepth[pix];
                if (a.dL_dalpha) gA[q] = a.dL_dalpha[pix];
            }
        }
        mymax = max(mymax, nc[q]);
    }
    const uint32_t maxnc = __builtin_amdgcn_readfirstlane(wave_max_u32(mymax));  // uniform: scalar loop control
    const uint32_t end = r0 + maxnc;  // positions >= end contributed to no pixel
    const int slot = lane < 16 ? wave_sum10_slot(lane) : NP;  // value this lane writes after a reduction

    for (uint32_t hi = end; hi > r0;) {
        const uint32_t lo = (hi - r0 > (uint32_t)B) ? hi - B : r0;
        const int cnt = (int)(hi - lo);
        if ((int)lane < cnt) {
            const uint32_t pos = hi - 1u - lane;
            const uint32_t vi = a.val_sorted[pos];
            stage_record(a.rec, vi, st.kappa, sA[lane], sB[lane], sC[lane]);
            if (EXT) sZ[lane] = a.rec[(size_t)vi * GESR_REC_FLOATS + 11];
            const float4 r3 = reinterpret_cast<const float4*>(a.rec + (size_t)vi * GESR_REC_FLOATS)[3];
            const uint2 r = make_uint2(__float_as_uint(r3.x), __float_as_uint(r3.y));  // the pair's rectangle
            sInst[lane] = instance_index(a, r, vi, tx, ty);
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const uint32_t prel = hi - 1u - (uint32_t)j - r0;  // 0-based list position
            const float4 ra = sA[j];
            const float4 rb = sB[j];
            const float4 rc = sC[j];
            const float z = EXT ? sZ[j] : 0.0f;
            float gr[NP], gz = 0.0f;
#pragma unroll
            for (int k = 0; k < NP; k += 2) opaque_zero2(gr[k], gr[k + 1]);
            if (EXT) gz = opaque_zero();
            bool act = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Fragment f;
                const float qq = ges_q(ra, rb.x, pxb + (float)((q & 1) * 8), pyb + (float)((q >> 1) * 8), f);
                if (prel >= nc[q] || qq > rb.w) continue;  // behind the pixel's last or beyond the footprint
                // Inside the footprint alpha almost never falls below alpha_min,
                // the alpha cap and a centred pixel are rarer still: those
                // decisions are selects (a zeroed term leaves the sums as they
                // are), so the wave takes one branch per quadrant.
                ges_alpha(qq, rb.z, rb.y, st, amax, f);
                const bool ok = !(f.alpha < st.alpha_min);
                act = act || ok;
                // a skipped fragment has alpha 0 here: it leaves T (rcp(1) = 1), the
                // colour behind and the sums as they are
                const float al = ok ? f.alpha : 0.0f;
                const float Tk = T[q] * hw_rcp(1.0f - al);
                const float aT = al * Tk;
                gr[7] += aT * g0[q];
                gr[8] += aT * g1[q];
                gr[9] += aT * g2[q];
                float dLda = Tk * ((rc.x - Br[q]) * g0[q] + (rc.y - Bg[q]) * g1[q] + (rc.z - Bb[q]) * g2[q]);
                Br[q] = fmaf(al, rc.x - Br[q], Br[q]);
                Bg[q] = fmaf(al, rc.y - Bg[q], Bg[q]);
                Bb[q] = fmaf(al, rc.z - Bb[q], Bb[q]);
                if (EXT) {
                    dLda += Tk * ((z - BD[q]) * gD[q] + (1.0f - BA[q]) * gA[q]);
                    gz += aT * gD[q];
                    BD[q] = fmaf(al, z - BD[q], BD[q]);
                    BA[q] = fmaf(al, 1.0f - BA[q], BA[q]);
                }
                T[q] = Tk;
                // add_fragment_grad with its two early exits as selects
                const bool live = ok && !(f.oG > st.alpha_max);
                const float dl = live ? dLda : 0.0f;
                gr[5] = fmaf(dl, f.G, gr[5]);
                const bool geo = live && f.q > 1e-30f;
                const float X = geo ? dl * f.oG * f.P : 0.0f;
                const float lq = geo ? f.l2q : 0.0f;
                gr[6] = fmaf(X * lq, c2, gr[6]);
                const float d2 = X * rc.w * hw_rcp(geo ? f.q : 1.0f);
                const float tq = d2 * f.t, wq = d2 * f.w;
                gr[0] = fmaf(-tq, ra.z, gr[0]);
                gr[1] = fmaf(-tq, ra.w, gr[1]);
                gr[1] = fmaf(-wq, rb.x, gr[1]);
                gr[2] = fmaf(tq, f.dx, gr[2]);
                gr[3] = fmaf(tq, f.dy, gr[3]);
                gr[4] = fmaf(wq, f.dy, gr[4]);
            }
            if (__ballot(act) != 0ull) {
                const float tot = wave_sum10(gr, lane);
                if (slot < NP) sRed[j][slot] = tot;
                if (EXT) {
                    const float tz = wave_sum(gz);
                    if (lane == 0) sRed[j][NP] = tz;
                }
            } else if ((int)lane < (EXT ? NP + 1 : NP)) {
                sRed[j][lane] = 0.f;
            }
        }
        __syncthreads();
        if ((int)lane < cnt && sInst[lane] != kNoInstance) write_partial<EXT>(a, sInst[lane], sRed[lane]);
        __syncthreads();
        hi = lo;
    }
}

template <int TW, int TH>
hipError_t fwd_shape(const RenderArgs& a, bool counts, hipStream_t s) {
    if (counts)
        hipLaunchKernelGGL((k_render_fwd<TW, TH, true>), dim3(a.n_items), dim3(TW * TH), 0, s, a);
    else
        hipLaunchKernelGGL((k_render_fwd<TW, TH, false>), dim3(a.n_items), dim3(TW * TH), 0, s, a);
    return hipGetLastError();
}

template <int TW, int TH, int BATCH>
hipError_t bwd_shape(const RenderArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_render_bwd<TW, TH, BATCH>), dim3(a.n_items), dim3(TW * TH), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_render_fwd(const RenderArgs& a, int tw, int th, bool counts, hipStream_t s) {
    if (a.n_items == 0) return hipSuccess;
    if (tw == 16 && th == 16) {
        if (a.st.variant == 1) return fwd_shape<16, 16>(a, counts, s);
        const bool small = a.batch == 32, ext = a.out_depth || a.out_alpha;
        const dim3 grid(a.n_items), block(64);
        if (ext) {
            if (counts) {
                if (small) hipLaunchKernelGGL((k_render_fwd_wave16<true, 32, true>), grid, block, 0, s, a);
                else hipLaunchKernelGGL((k_render_fwd_wave16<true, 64, true>), grid, block, 0, s, a);
            } else {
                if (small) hipLaunchKernelGGL((k_render_fwd_wave16<false, 32, true>), grid, block, 0, s, a);
                else hipLaunchKernelGGL((k_render_fwd_wave16<false, 64, true>), grid, block, 0, s, a);
            }
        } else if (counts) {
            if (small) hipLaunchKernelGGL((k_render_fwd_wave16<true, 32, false>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_render_fwd_wave16<true, 64, false>), grid, block, 0, s, a);
        } else {
            if (small) hipLaunchKernelGGL((k_render_fwd_wave16<false, 32, false>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_render_fwd_wave16<false, 64, false>), grid, block, 0, s, a);
        }
        return hipGetLastError();
    }
    if (tw == 8 && th == 8) return fwd_shape<8, 8>(a, counts, s);
    if (tw == 32 && th == 16) return fwd_shape<32, 16>(a, counts, s);
    if (tw == 32 && th == 32) return fwd_shape<32, 32>(a, counts, s);
    return hipErrorInvalidValue;
}

hipError_t launch_render_bwd(const RenderArgs& a, int tw, int th, int batch, hipStream_t s) {
    if (a.n_items == 0) return hipSuccess;
    if (tw == 16 && th == 16) {
        if (a.st.variant == 1)  // one workgroup of 4 waves per tile
            return batch >= 128 ? bwd_shape<16, 16, 128>(a, s) : bwd_shape<16, 16, 64>(a, s);
        const bool ext = a.dL_ddepth || a.dL_dalpha;
        const dim3 grid(a.n_items), block(64);
        if (ext) {
            if (batch == 32) hipLaunchKernelGGL((k_render_bwd_wave16<32, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_render_bwd_wave16<64, true>), grid, block, 0, s, a);
        } else {
            if (batch == 32) hipLaunchKernelGGL((k_render_bwd_wave16<32, false>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_render_bwd_wave16<64, false>), grid, block, 0, s, a);
        }
        return hipGetLastError();
    }
    if (tw == 8 && th == 8) return bwd_shape<8, 8, 64>(a, s);
    if (tw == 32 && th == 16) return batch >= 128 ? bwd_shape<32, 16, 128>(a, s) : bwd_shape<32, 16, 64>(a, s);
    if (tw == 32 && th == 32) return bwd_shape<32, 32, 64>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace gesr
