// Device-side definitions shared by the GES rasterizer kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gesr.h"

namespace gesr {

// Per-view constants, passed by value in kernel arguments.
struct DevView {
    int W, H;
    float fx, fy, cx, cy;
    float R[9];  // world -> camera rotation (row-major)
    float t[3];
    float campos[3];
    int tiles_x, tiles_y;
    uint32_t tile_base;  // first global tile id of the view
    uint32_t pix_base;   // first pixel of the view in the concatenated outputs
};

struct DevCams {
    int V;
    int pad[3];
    DevView v[GESR_MAX_VIEWS];
};

struct DevSettings {
    float kappa;
    float neg_kappa_log2e;  // -kappa * log2(e): G = exp2(neg_kappa_log2e * P)
    float rho;
    float alpha_min, alpha_max, t_min;
    float blur, znear, clip_fac;
    float bg[3];
    int tile_w, tile_h;
    int sh_degree;
    int variant;  // renderer variant for 16x16 tiles: 0 = one wave per tile, 1 = four waves per tile
};

constexpr float kLn2 = 0.693147180559945309f;

__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Index of the view that owns global tile `t` (views are few; linear scan).
__device__ __forceinline__ int view_of_tile(const DevCams& c, uint32_t t) {
    int v = 0;
    while (v + 1 < c.V && t >= c.v[v + 1].tile_base) ++v;
    return v;
}

// Screen-space record of one projected splat as staged by the renderers.
//   a = (u, v, L00, L10), b = (L11, opacity, beta / 2, qmax), c = (r, g, b, -)
// with the conic factored as q = (L00 dx + L10 dy)^2 + (L11 dy)^2.  The
// generalized-exponential falloff G = exp(-kappa q^(beta/2)) is evaluated by
// `ges_alpha`; the forward and the backward call the same functions so alpha
// is bit-identical in both.
struct Fragment {
    float dx, dy, t, w, q, l2q, P, G, oG, alpha;
};

__device__ __forceinline__ float ges_q(const float4& a, float L11, float px, float py, Fragment& f) {
    f.dx = px - a.x;
    f.dy = py - a.y;
    f.t = fmaf(a.w, f.dy, a.z * f.dx);
    f.w = L11 * f.dy;
    return fmaf(f.t, f.t, f.w * f.w);
}

__device__ __forceinline__ void ges_alpha(float q, float half_beta, float opacity, const DevSettings& st, Fragment& f) {
    f.q = q;
    f.l2q = hw_log2(q);                    // -inf at q = 0
    f.P = hw_exp2(half_beta * f.l2q);      // q^(beta/2); 0 at q = 0
    f.G = hw_exp2(st.neg_kappa_log2e * f.P);
    f.oG = opacity * f.G;
    f.alpha = fminf(st.alpha_max, f.oG);
}

// Wave-wide sum (64 lanes) by butterfly; every lane receives the total.
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// Wave-wide sum with DPP row operations (no LDS traffic); the total is valid
// in lane 63 only.  Fixed order: inclusive row sums by row_shr 1..8, then the
// row totals are chained with row_bcast 15 and row_bcast 31.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, BANK_MASK, true));
}
// Sum over each 16-lane row; the row total is valid in the row's lane 15.
__device__ __forceinline__ float row_sum_lane15(float x) {
    float s = x + dpp<0x111, 0xf, 0xf>(x);   // row_shr:1
    s = s + dpp<0x112, 0xf, 0xf>(x);         // row_shr:2
    s = s + dpp<0x113, 0xf, 0xf>(x);         // row_shr:3
    s = s + dpp<0x114, 0xf, 0xe>(s);         // row_shr:4, banks 1..3
    s = s + dpp<0x118, 0xf, 0xc>(s);         // row_shr:8, banks 2..3
    return s;
}

// Sum over each group of four lanes (quad_perm swaps); every lane of the quad
// holds the same total (the two orders agree by commutativity).
__device__ __forceinline__ float quad_sum(float x) {
    const float s = x + dpp<0xb1, 0xf, 0xf>(x);  // quad_perm [1, 0, 3, 2]
    return s + dpp<0x4e, 0xf, 0xf>(s);           // quad_perm [2, 3, 0, 1]
}

__device__ __forceinline__ float wave_sum_lane63(float x) {
    float s = x + dpp<0x111, 0xf, 0xf>(x);   // row_shr:1
    s = s + dpp<0x112, 0xf, 0xf>(x);         // row_shr:2
    s = s + dpp<0x113, 0xf, 0xf>(x);         // row_shr:3
    s = s + dpp<0x114, 0xf, 0xe>(s);         // row_shr:4, banks 1..3
    s = s + dpp<0x118, 0xf, 0xc>(s);         // row_shr:8, banks 2..3
    s = s + dpp<0x142, 0xa, 0xf>(s);         // row_bcast:15 into rows 1, 3
    s = s + dpp<0x143, 0xc, 0xf>(s);         // row_bcast:31 into rows 2, 3
    return s;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        uint32_t y = __shfl_xor(x, m, 64);
        x = x > y ? x : y;
    }
    return x;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t l = __lane_id();
    return l == 0 ? 0ull : ((~0ull) >> (64 - l));
}

}  // namespace gesr
