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

// alpha = min(opacity G, alpha_max) as one median-of-three: opacity G >= 0, so
// med3(opacity G, 0, alpha_max) is that minimum (and needs no NaN quieting of
// the kernel argument per fragment, as a min would).
__device__ __forceinline__ void ges_alpha(float q, float half_beta, float opacity, const DevSettings& st,
                                          float alpha_max, Fragment& f) {
    f.q = q;
    f.l2q = hw_log2(q);                    // -inf at q = 0
    f.P = hw_exp2(half_beta * f.l2q);      // q^(beta/2); 0 at q = 0
    f.G = hw_exp2(st.neg_kappa_log2e * f.P);
    f.oG = opacity * f.G;
    f.alpha = __builtin_amdgcn_fmed3f(f.oG, 0.0f, alpha_max);
}

// A zero the compiler cannot treat as a constant.  Accumulators that start
// from it are updated in place along nested branches; started from a literal
// 0 the compiler re-materialises the zeros on every skipped branch level.
__device__ __forceinline__ float opaque_zero() {
    float z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}
// Two such zeros from one 64-bit move.
__device__ __forceinline__ void opaque_zero2(float& a, float& b) {
    uint64_t z;
    asm volatile("v_mov_b64 %0, 0" : "=v"(z));
    a = __uint_as_float((uint32_t)z);
    b = __uint_as_float((uint32_t)(z >> 32));
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

// Stride of one instance partial in the backward workspace: the ten gradient
// terms padded to twelve floats so a partial is three aligned 16-byte
// accesses.
constexpr int kPartialStride = 12;

// Sum over each group of four lanes (quad_perm swaps); every lane of the quad
// holds the same total (the two orders agree by commutativity).
__device__ __forceinline__ float quad_sum(float x) {
    const float s = x + dpp<0xb1, 0xf, 0xf>(x);  // quad_perm [1, 0, 3, 2]
    return s + dpp<0x4e, 0xf, 0xf>(s);           // quad_perm [2, 3, 0, 1]
}

// Sum over each aligned group of L = 4, 8 or 16 lanes; every lane of the group
// holds the total (each step adds two equal-shaped partial sums, so partners
// agree by commutativity).
template <int L>
__device__ __forceinline__ float group_sum(float x) {
    static_assert(L == 4 || L == 8 || L == 16, "group of 4, 8 or 16 lanes");
    x = quad_sum(x);
    if (L >= 8) x += dpp<0x141, 0xf, 0xf>(x);  // row_half_mirror: the other quad of the 8
    if (L >= 16) x += dpp<0x128, 0xf, 0xf>(x); // row_ror:8: the other half of the row
    return x;
}

// Wave sums of ten per-lane values by a transposed butterfly: each step pairs
// lanes that differ in one bit of the lane index and lets each keep (and add
// its partner's copy of) half of the values it holds, so the work halves with
// the data: row_ror:8 (bit 3, 10 -> 5 values), row_half_mirror (bit 2, 5 -> 3),
// quad_perm swaps (bit 1, 3 -> 2; bit 0, 2 -> 1), then the four rows are added
// by two cross-row shuffles.  Every lane ends with the total of value
// wave_sum10_slot(lane) (>= 10: padding).  Fixed pattern, bitwise reproducible.
__device__ __forceinline__ int wave_sum10_slot(uint32_t lane) {
    const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
    int t = b0;                 // index after the bit-0 step into the bit-1 step's 2 values
    if (b1) t = t == 0 ? 2 : 3; // bit-1 lanes hold the third value (or padding)
    if (t > 2) return 16;
    int si = t;                 // index into the bit-2 step's 3 values
    if (b2) si = t < 2 ? t + 3 : 5;
    if (si > 4) return 16;
    return si + 5 * b3;
}

// The bit-3 and bit-2 steps need no selects: the half a lane keeps is the
// one whose DPP add writes the lane's bank (banks are lane bits 2-3 of a row),
// so each kept value is one masked v_add_f32_dpp of the value and its
// partner's copy.  Written as one asm block (the compiler's DPP intrinsics
// cannot express a bank-masked add whose unwritten lanes keep another add's
// result); the block opens with 5 wait states (EXEC or VGPR writes just
// before a DPP read), spaces each of its own DPP reads at least 2
// instructions after the write of that register, and closes with 2 wait
// states for DPP reads of its results.  In the bit-2 step the third value is
// added over all banks: the bit-2 lanes' copy is padding and never reaches a
// valid slot.
__device__ __forceinline__ float wave_sum10(const float (&v)[10], uint32_t lane) {
    const bool b0 = lane & 1, b1 = (lane >> 1) & 1;
    float s0, s1, s2, s3, s4, t[3];
    asm volatile(
        "s_nop 4\n"
        // lanes l and l ^ 8 (row_ror:8): banks 0-1 keep value p, banks 2-3 value p + 5
        "v_add_f32_dpp %[s0], %[v0], %[v0] row_ror:8 row_mask:0xf bank_mask:0x3\n"
        "v_add_f32_dpp %[s0], %[v5], %[v5] row_ror:8 row_mask:0xf bank_mask:0xc\n"
        "v_add_f32_dpp %[s1], %[v1], %[v1] row_ror:8 row_mask:0xf bank_mask:0x3\n"
        "v_add_f32_dpp %[s1], %[v6], %[v6] row_ror:8 row_mask:0xf bank_mask:0xc\n"
        "v_add_f32_dpp %[s2], %[v2], %[v2] row_ror:8 row_mask:0xf bank_mask:0x3\n"
        "v_add_f32_dpp %[s2], %[v7], %[v7] row_ror:8 row_mask:0xf bank_mask:0xc\n"
        "v_add_f32_dpp %[s3], %[v3], %[v3] row_ror:8 row_mask:0xf bank_mask:0x3\n"
        "v_add_f32_dpp %[s3], %[v8], %[v8] row_ror:8 row_mask:0xf bank_mask:0xc\n"
        "v_add_f32_dpp %[s4], %[v4], %[v4] row_ror:8 row_mask:0xf bank_mask:0x3\n"
        "v_add_f32_dpp %[s4], %[v9], %[v9] row_ror:8 row_mask:0xf bank_mask:0xc\n"
        // lanes l and l ^ 7 (row_half_mirror, bit 2 differs): banks 0 and 2 keep
        // value p, banks 1 and 3 value p + 3
        "v_add_f32_dpp %[t0], %[s0], %[s0] row_half_mirror row_mask:0xf bank_mask:0x5\n"
        "v_add_f32_dpp %[t0], %[s3], %[s3] row_half_mirror row_mask:0xf bank_mask:0xa\n"
        "v_add_f32_dpp %[t1], %[s1], %[s1] row_half_mirror row_mask:0xf bank_mask:0x5\n"
        "v_add_f32_dpp %[t1], %[s4], %[s4] row_half_mirror row_mask:0xf bank_mask:0xa\n"
        "v_add_f32_dpp %[t2], %[s2], %[s2] row_half_mirror row_mask:0xf bank_mask:0xf\n"
        "s_nop 1"
        : [s0] "=&v"(s0), [s1] "=&v"(s1), [s2] "=&v"(s2), [s3] "=&v"(s3), [s4] "=&v"(s4), [t0] "=&v"(t[0]),
          [t1] "=&v"(t[1]), [t2] "=&v"(t[2])
        : [v0] "v"(v[0]), [v1] "v"(v[1]), [v2] "v"(v[2]), [v3] "v"(v[3]), [v4] "v"(v[4]), [v5] "v"(v[5]),
          [v6] "v"(v[6]), [v7] "v"(v[7]), [v8] "v"(v[8]), [v9] "v"(v[9]));
    // lanes l and l ^ 2 (quad_perm [2, 3, 0, 1]): keep value 0 or 2; value 1 is
    // added on all lanes (the bit-1 lanes' copy is padding)
    float u[2];
    {
        const float keep = b1 ? t[2] : t[0], give = b1 ? t[0] : t[2];
        u[0] = keep + dpp<0x4e, 0xf, 0xf>(give);
        u[1] = t[1] + dpp<0x4e, 0xf, 0xf>(t[1]);
    }
    const float keep = b0 ? u[1] : u[0], give = b0 ? u[0] : u[1];
    float w = keep + dpp<0xb1, 0xf, 0xf>(give);  // quad_perm [1, 0, 3, 2]
    w += __shfl_xor(w, 16, 64);
    w += __shfl_xor(w, 32, 64);
    return w;
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
