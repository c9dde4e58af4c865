// Photometric loss of Eq. 8 (Sec. 3.2): L_v = (1 - lambda) mean|X - Y| +
// lambda (1 - mean SSIM) per view, and its gradient with respect to the
// rendered image X, for every view of the batch in one launch per kernel.
//
// SSIM (the paper names it, not its window): an 11 x 11 Gaussian window with
// zero padding, C1 and C2 as given.  With the window sums mu = G*X, m2 = G*X^2,
// mxy = G*(X Y):
//   S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
//   s_x^2 = m2x - mu_x^2, s_xy = mxy - mu_x mu_y.
// The gradient of sum_p S(p) is the window sum of the moments' adjoints:
//   dS/dX(q) = (G*a)(q) + 2 X(q) (G*b)(q) + Y(q) (G*c)(q)
// with a = dS/dmu_x, b = dS/dm2x, c = dS/dmxy per pixel (the window is
// symmetric, so the adjoint of a zero-padded window sum is the window sum).
//
// Both kernels work on 16 x 16 output tiles, one thread per pixel: the tile's
// 26 x 26 input patch (5 pixels of halo, zero outside the image) is staged in
// LDS, the 11 horizontal taps are summed per row, then the 11 vertical taps
// per pixel.  The forward writes a, b, c and per-tile partial sums of S and
// |X - Y| (fixed-order block reductions); a one-block-per-view kernel sums the
// partials in tile order; the backward adds the L1 term's sign.

#include "gesr_device.h"
#include "gesr_kernels.h"

namespace gesr {

namespace {

constexpr int kR = GESR_LOSS_RADIUS;  // window radius (11 taps)
constexpr int kTile = 16;
constexpr int kPatch = kTile + 2 * kR;  // 26
constexpr int kThreads = kTile * kTile;

__device__ __forceinline__ int view_of_loss_tile(const LossArgs& a, uint32_t t) {
    int v = 0;
    while (v + 1 < a.V && t >= a.v[v + 1].tile_base) ++v;
    return v;
}

// Fixed-order sum over the 256 threads of a block (wave butterflies, then the
// four wave totals in order); every thread receives the total.
__device__ __forceinline__ float block_sum(float x, float* lds4) {
    x = wave_sum(x);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds4[w] = x;
    __syncthreads();
    return ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
}

// Stages the patch of `src` around the tile (zero outside the view).
__device__ __forceinline__ void stage_patch(const float* src, const LossView& w, int tx0, int ty0,
                                            float (*dst)[kPatch + 1]) {
    for (int i = threadIdx.x; i < kPatch * kPatch; i += kThreads) {
        const int r = i / kPatch, q = i % kPatch;
        const int gy = ty0 + r - kR, gx = tx0 + q - kR;
        dst[r][q] = (gx >= 0 && gx < w.W && gy >= 0 && gy < w.H) ? src[(size_t)gy * w.W + gx] : 0.0f;
    }
}

__global__ __launch_bounds__(kThreads) void k_ssim_fwd(LossArgs a) {
    __shared__ float sx[kPatch][kPatch + 1], sy[kPatch][kPatch + 1];
    __shared__ float h[5][kPatch][kTile + 1];
    __shared__ float red[4];
    const uint32_t t = blockIdx.x;
    const int v = view_of_loss_tile(a, t);
    const LossView& w = a.v[v];
    const uint32_t lt = t - w.tile_base;
    const int tiles_x = (w.W + kTile - 1) / kTile;
    const int tx0 = (int)(lt % tiles_x) * kTile, ty0 = (int)(lt / tiles_x) * kTile;
    const int lx = threadIdx.x % kTile, ly = threadIdx.x / kTile;
    const int x = tx0 + lx, y = ty0 + ly;
    const bool inside = x < w.W && y < w.H;
    const size_t HW = (size_t)w.W * w.H;
    float s_sum = 0.0f, l1_sum = 0.0f;
    for (int ch = 0; ch < 3; ++ch) {
        const size_t base = 3 * (size_t)w.pix_base + ch * HW;
        __syncthreads();
        stage_patch(a.image + base, w, tx0, ty0, sx);
        stage_patch(a.target + base, w, tx0, ty0, sy);
        __syncthreads();
        for (int i = threadIdx.x; i < kPatch * kTile; i += kThreads) {
            const int r = i / kTile, q = i % kTile;
            float m1x = 0.f, m1y = 0.f, m2x = 0.f, m2y = 0.f, mxy = 0.f;
#pragma unroll
            for (int j = 0; j <= 2 * kR; ++j) {
                const float gx = a.w[j] * sx[r][q + j], yv = sy[r][q + j];
                const float gy = a.w[j] * yv;
                m1x += gx;
                m1y += gy;
                m2x = fmaf(gx, sx[r][q + j], m2x);
                m2y = fmaf(gy, yv, m2y);
                mxy = fmaf(gx, yv, mxy);
            }
            h[0][r][q] = m1x;
            h[1][r][q] = m1y;
            h[2][r][q] = m2x;
            h[3][r][q] = m2y;
            h[4][r][q] = mxy;
        }
        __syncthreads();
        float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i <= 2 * kR; ++i)
#pragma unroll
            for (int k = 0; k < 5; ++k) m[k] = fmaf(a.w[i], h[k][ly + i][lx], m[k]);
        if (inside) {
            const float mx = m[0], my = m[1];
            const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
            const float N1 = 2.f * mx * my + a.c1, N2 = 2.f * sxy + a.c2;
            const float D1 = mx * mx + my * my + a.c1, D2 = sxx + syy + a.c2;
            const float inv = 1.0f / (D1 * D2);
            const float S = N1 * N2 * inv;
            const float da = 2.f * my * N2 * inv - 2.f * mx * S / D1 + 2.f * mx * S / D2 - 2.f * my * N1 * inv;
            const size_t p = base + (size_t)y * w.W + x;
            a.amap[p] = da;
            a.bmap[p] = -S / D2;
            a.cmap[p] = 2.f * N1 * inv;
            s_sum += S;
            l1_sum += fabsf(sx[ly + kR][lx + kR] - sy[ly + kR][lx + kR]);
        }
    }
    const float ts = block_sum(s_sum, red);
    const float tl = block_sum(l1_sum, red);
    if (threadIdx.x == 0) {
        a.partial[2 * (size_t)t] = ts;
        a.partial[2 * (size_t)t + 1] = tl;
    }
}

// One block per view: the view's tile partials summed in tile order (each
// thread a fixed stride, then the block sum), then L_v.
__global__ __launch_bounds__(kThreads) void k_ssim_loss(LossArgs a) {
    __shared__ float red[4];
    const LossView& w = a.v[blockIdx.x];
    const uint32_t tiles = (uint32_t)(((w.W + kTile - 1) / kTile) * ((w.H + kTile - 1) / kTile));
    float s = 0.f, l = 0.f;
    for (uint32_t i = threadIdx.x; i < tiles; i += kThreads) {
        s += a.partial[2 * (size_t)(w.tile_base + i)];
        l += a.partial[2 * (size_t)(w.tile_base + i) + 1];
    }
    s = block_sum(s, red);
    l = block_sum(l, red);
    if (threadIdx.x == 0) a.loss[blockIdx.x] = (1.0f - a.lam) * l * w.inv_n + a.lam * (1.0f - s * w.inv_n);
}

__global__ __launch_bounds__(kThreads) void k_ssim_bwd(LossArgs a) {
    __shared__ float sp[3][kPatch][kPatch + 1];
    __shared__ float h[3][kPatch][kTile + 1];
    const uint32_t t = blockIdx.x;
    const int v = view_of_loss_tile(a, t);
    const LossView& w = a.v[v];
    const uint32_t lt = t - w.tile_base;
    const int tiles_x = (w.W + kTile - 1) / kTile;
    const int tx0 = (int)(lt % tiles_x) * kTile, ty0 = (int)(lt / tiles_x) * kTile;
    const int lx = threadIdx.x % kTile, ly = threadIdx.x / kTile;
    const int x = tx0 + lx, y = ty0 + ly;
    const bool inside = x < w.W && y < w.H;
    const size_t HW = (size_t)w.W * w.H;
    const float l1s = (1.0f - a.lam) * w.inv_n, ss = a.lam * w.inv_n;
    for (int ch = 0; ch < 3; ++ch) {
        const size_t base = 3 * (size_t)w.pix_base + ch * HW;
        __syncthreads();
        stage_patch(a.amap + base, w, tx0, ty0, sp[0]);
        stage_patch(a.bmap + base, w, tx0, ty0, sp[1]);
        stage_patch(a.cmap + base, w, tx0, ty0, sp[2]);
        __syncthreads();
        for (int i = threadIdx.x; i < kPatch * kTile; i += kThreads) {
            const int r = i / kTile, q = i % kTile;
            float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
            for (int j = 0; j <= 2 * kR; ++j) {
                s0 = fmaf(a.w[j], sp[0][r][q + j], s0);
                s1 = fmaf(a.w[j], sp[1][r][q + j], s1);
                s2 = fmaf(a.w[j], sp[2][r][q + j], s2);
            }
            h[0][r][q] = s0;
            h[1][r][q] = s1;
            h[2][r][q] = s2;
        }
        __syncthreads();
        float ga = 0.f, gb = 0.f, gc = 0.f;
#pragma unroll
        for (int i = 0; i <= 2 * kR; ++i) {
            ga = fmaf(a.w[i], h[0][ly + i][lx], ga);
            gb = fmaf(a.w[i], h[1][ly + i][lx], gb);
            gc = fmaf(a.w[i], h[2][ly + i][lx], gc);
        }
        if (inside) {
            const size_t p = base + (size_t)y * w.W + x;
            const float X = a.image[p], Y = a.target[p];
            const float d = X - Y;
            const float sgn = (d > 0.f) ? 1.f : ((d < 0.f) ? -1.f : 0.f);
            const float dS = ga + 2.f * X * gb + Y * gc;
            a.grad[p] = l1s * sgn - ss * dS;
        }
    }
}

}  // namespace

hipError_t launch_ssim_loss(const LossArgs& a, uint32_t n_tiles, bool want_loss, hipStream_t stream) {
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ssim_fwd, dim3(n_tiles), dim3(kThreads), 0, stream, a);
    if (want_loss) hipLaunchKernelGGL(k_ssim_loss, dim3(a.V), dim3(kThreads), 0, stream, a);
    hipLaunchKernelGGL(k_ssim_bwd, dim3(n_tiles), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace gesr

// --------------------------------------------------------------------------
// Surface-alignment regulariser of the flattened-splat workload: per splat,
// with k* the axis of the smallest scale (lowest index on ties), n = R(q) e_k*
// and m the true surface normal,
//   L = w_scale / N sum_i s_ik* + w_normal / N sum_i (1 - <n_i, m_i>^2);
// its gradient is added to the scale and quaternion gradients (one thread per
// splat: an HBM-bound pass) and its two sums are reduced in a fixed order.
namespace gesr {

namespace {

__global__ __launch_bounds__(256) void k_surface_align(AlignArgs a) {
    __shared__ float red[4];
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    const size_t n = (size_t)a.n;
    float ls = 0.f, ln = 0.f;
    if (i < (uint32_t)a.n) {
        const float s0 = a.scale[i], s1 = a.scale[n + i], s2 = a.scale[2 * n + i];
        const int k = (s0 <= s1 && s0 <= s2) ? 0 : (s1 <= s2 ? 1 : 2);
        const float qw0 = a.quat[i], qx0 = a.quat[n + i], qy0 = a.quat[2 * n + i], qz0 = a.quat[3 * n + i];
        const float inv = 1.0f / sqrtf(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
        const float w = qw0 * inv, x = qx0 * inv, y = qy0 * inv, z = qz0 * inv;
        // column k of R(q) and its derivative with respect to (w, x, y, z)
        float c[3], J[3][4];
        if (k == 0) {
            c[0] = 1.f - 2.f * (y * y + z * z); c[1] = 2.f * (x * y + w * z); c[2] = 2.f * (x * z - w * y);
            J[0][0] = 0.f;        J[0][1] = 0.f;       J[0][2] = -4.f * y;  J[0][3] = -4.f * z;
            J[1][0] = 2.f * z;    J[1][1] = 2.f * y;   J[1][2] = 2.f * x;   J[1][3] = 2.f * w;
            J[2][0] = -2.f * y;   J[2][1] = 2.f * z;   J[2][2] = -2.f * w;  J[2][3] = 2.f * x;
        } else if (k == 1) {
            c[0] = 2.f * (x * y - w * z); c[1] = 1.f - 2.f * (x * x + z * z); c[2] = 2.f * (y * z + w * x);
            J[0][0] = -2.f * z;   J[0][1] = 2.f * y;   J[0][2] = 2.f * x;   J[0][3] = -2.f * w;
            J[1][0] = 0.f;        J[1][1] = -4.f * x;  J[1][2] = 0.f;       J[1][3] = -4.f * z;
            J[2][0] = 2.f * x;    J[2][1] = 2.f * w;   J[2][2] = 2.f * z;   J[2][3] = 2.f * y;
        } else {
            c[0] = 2.f * (x * z + w * y); c[1] = 2.f * (y * z - w * x); c[2] = 1.f - 2.f * (x * x + y * y);
            J[0][0] = 2.f * y;    J[0][1] = 2.f * z;   J[0][2] = 2.f * w;   J[0][3] = 2.f * x;
            J[1][0] = -2.f * x;   J[1][1] = -2.f * w;  J[1][2] = 2.f * z;   J[1][3] = 2.f * y;
            J[2][0] = 0.f;        J[2][1] = -4.f * x;  J[2][2] = -4.f * y;  J[2][3] = 0.f;
        }
        const float m0 = a.normal[i], m1 = a.normal[n + i], m2 = a.normal[2 * n + i];
        const float d = c[0] * m0 + c[1] * m1 + c[2] * m2;
        ls = k == 0 ? s0 : (k == 1 ? s1 : s2);
        ln = 1.f - d * d;
        // dL/dn = -2 d w_normal / N m, then through the column and the normalisation
        const float gsc = -2.f * d * a.w_normal_n;
        const float gn[3] = {gsc * m0, gsc * m1, gsc * m2};
        float gq[4];
        for (int j = 0; j < 4; ++j) gq[j] = gn[0] * J[0][j] + gn[1] * J[1][j] + gn[2] * J[2][j];
        const float dot = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
        a.g_quat[i] += (gq[0] - dot * w) * inv;
        a.g_quat[n + i] += (gq[1] - dot * x) * inv;
        a.g_quat[2 * n + i] += (gq[2] - dot * y) * inv;
        a.g_quat[3 * n + i] += (gq[3] - dot * z) * inv;
        a.g_scale[(size_t)k * n + i] += a.w_scale_n;
    }
    const float ts = block_sum(ls, red);
    const float tn = block_sum(ln, red);
    if (a.partial && threadIdx.x == 0) {
        a.partial[2 * (size_t)blockIdx.x] = ts;
        a.partial[2 * (size_t)blockIdx.x + 1] = tn;
    }
}

// One block: the block partials summed in block order, scaled by the weights.
__global__ __launch_bounds__(256) void k_surface_align_sum(AlignArgs a, uint32_t blocks) {
    __shared__ float red[4];
    float s = 0.f, t = 0.f;
    for (uint32_t b = threadIdx.x; b < blocks; b += 256) {
        s += a.partial[2 * (size_t)b];
        t += a.partial[2 * (size_t)b + 1];
    }
    s = block_sum(s, red);
    t = block_sum(t, red);
    if (threadIdx.x == 0) {
        a.losses[0] = s * a.w_scale_n;
        a.losses[1] = t * a.w_normal_n;
    }
}

}  // namespace

hipError_t launch_surface_align(const AlignArgs& a, hipStream_t stream) {
    if (a.n <= 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)((a.n + 255) / 256);
    hipLaunchKernelGGL(k_surface_align, dim3(blocks), dim3(256), 0, stream, a);
    if (a.losses) hipLaunchKernelGGL(k_surface_align_sum, dim3(1), dim3(256), 0, stream, a, blocks);
    return hipGetLastError();
}

}  // namespace gesr
