// Projection of GES splats to screen-space conics and its adjoint (gfx950).
//
// Forward (Sec. 3.2): Sigma = R S S^T R^T (Eq. 4) with the shape-modulated
// scale S = diag(phi(beta) s) (Eq. 6-7, phi = 2 / (1 + exp(-rho (beta - 2)))),
// screen covariance Sigma' = J W Sigma W^T J^T + blur I, projected centre,
// SH colour, and the alpha_min footprint used for binning.  The conic
// Sigma'^-1 is stored as its Cholesky factor (q = (L00 dx + L10 dy)^2 +
// (L11 dy)^2): evaluating the quadratic form A dx^2 + 2B dx dy + C dy^2 in
// float32 loses most of its digits along the long axis of a thin footprint,
// the factored form does not.
// One thread per splat; the splat's parameters are read once (coalesced SoA
// loads) and every view is projected from registers.
//
// Adjoint: per (view, splat), a fixed-order sum of the per-instance partials
// written by the backward renderer (atomic-free, k_seg_reduce), then the chain
// rule through the projection, accumulated over views in ascending order.

#include "gesr_device.h"
#include "gesr_kernels.h"

namespace gesr {

namespace {

// Real spherical harmonics (Condon-Shortley phase, index l*l + l + m) as
// polynomials of the unit direction (x, y, z), degrees 0..3.
constexpr float SH_C0 = 0.28209479177387814f;
constexpr float SH_C1 = 0.4886025119029199f;
constexpr float SH_C2[5] = {1.0925484305920792f, -1.0925484305920792f, 0.31539156525252005f,
                            -1.0925484305920792f, 0.5462742152960396f};
constexpr float SH_C3[7] = {-0.5900435899266435f, 2.890611442640554f, -0.4570457994644658f, 0.3731763325901154f,
                            -0.4570457994644658f, 1.445305721320277f, -0.5900435899266435f};

template <int DEG>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float* Y) {
    Y[0] = SH_C0;
    if (DEG >= 1) {
        Y[1] = -SH_C1 * y;
        Y[2] = SH_C1 * z;
        Y[3] = -SH_C1 * x;
    }
    if (DEG >= 2) {
        float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = SH_C2[0] * (x * y);
        Y[5] = SH_C2[1] * (y * z);
        Y[6] = SH_C2[2] * (2.0f * zz - xx - yy);
        Y[7] = SH_C2[3] * (x * z);
        Y[8] = SH_C2[4] * (xx - yy);
        if (DEG >= 3) {
            Y[9] = SH_C3[0] * y * (3.0f * xx - yy);
            Y[10] = SH_C3[1] * (x * y) * z;
            Y[11] = SH_C3[2] * y * (4.0f * zz - xx - yy);
            Y[12] = SH_C3[3] * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = SH_C3[4] * x * (4.0f * zz - xx - yy);
            Y[14] = SH_C3[5] * z * (xx - yy);
            Y[15] = SH_C3[6] * x * (xx - 3.0f * yy);
        }
    }
}

// Gradient of sum_k Y_k(x, y, z) w_k with respect to (x, y, z) (polynomials
// taken off the sphere; the caller projects out the radial part).
template <int DEG>
__device__ __forceinline__ void sh_grad(float x, float y, float z, const float* w, float& gx, float& gy, float& gz) {
    gx = 0.f;
    gy = 0.f;
    gz = 0.f;
    if (DEG >= 1) {
        gy += -SH_C1 * w[1];
        gz += SH_C1 * w[2];
        gx += -SH_C1 * w[3];
    }
    if (DEG >= 2) {
        gx += SH_C2[0] * y * w[4];
        gy += SH_C2[0] * x * w[4];
        gy += SH_C2[1] * z * w[5];
        gz += SH_C2[1] * y * w[5];
        gx += -2.f * SH_C2[2] * x * w[6];
        gy += -2.f * SH_C2[2] * y * w[6];
        gz += 4.f * SH_C2[2] * z * w[6];
        gx += SH_C2[3] * z * w[7];
        gz += SH_C2[3] * x * w[7];
        gx += 2.f * SH_C2[4] * x * w[8];
        gy += -2.f * SH_C2[4] * y * w[8];
        if (DEG >= 3) {
            float xx = x * x, yy = y * y, zz = z * z;
            gx += 6.f * SH_C3[0] * x * y * w[9];
            gy += SH_C3[0] * (3.f * xx - 3.f * yy) * w[9];
            gx += SH_C3[1] * y * z * w[10];
            gy += SH_C3[1] * x * z * w[10];
            gz += SH_C3[1] * x * y * w[10];
            gx += -2.f * SH_C3[2] * x * y * w[11];
            gy += SH_C3[2] * (4.f * zz - xx - 3.f * yy) * w[11];
            gz += 8.f * SH_C3[2] * y * z * w[11];
            gx += -6.f * SH_C3[3] * x * z * w[12];
            gy += -6.f * SH_C3[3] * y * z * w[12];
            gz += SH_C3[3] * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
            gx += SH_C3[4] * (4.f * zz - 3.f * xx - yy) * w[13];
            gy += -2.f * SH_C3[4] * x * y * w[13];
            gz += 8.f * SH_C3[4] * x * z * w[13];
            gx += 2.f * SH_C3[5] * x * z * w[14];
            gy += -2.f * SH_C3[5] * y * z * w[14];
            gz += SH_C3[5] * (xx - yy) * w[14];
            gx += SH_C3[6] * (3.f * xx - 3.f * yy) * w[15];
            gy += -6.f * SH_C3[6] * x * y * w[15];
        }
    }
}

// Error-free transformations for the compensated depth dot product
// (Ogita, Rump and Oishi, "Accurate sum and dot product", 2005: TwoSum and
// TwoProduct via FMA), so the depth key is the float32 rounding of the exact
// camera depth except within rounding distance of a tie.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ float dot3_plus_compensated(const float* r, const float* m, float t) {
    float s = t, c = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float p = r[k] * m[k];
        float ep = fmaf(r[k], m[k], -p);
        float es;
        two_sum(s, p, s, es);
        c += ep + es;
    }
    return s + c;
}

// View-independent part of the projection: normalised quaternion, rotation,
// phi(beta) and the factor M of the 3-D covariance Sigma = M M^T.
struct SplatGeom {
    float qw, qx, qy, qz, qinv;  // normalised quaternion and 1 / |q|
    float R[9];
    float phi;
    float M[9];    // R diag(phi s)
    float ps[3];   // phi s
};

__device__ __forceinline__ void splat_geom(const float* s, const float* q, float beta, const DevSettings& st,
                                           SplatGeom& g) {
    float n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    g.qinv = 1.0f / sqrtf(n2);
    g.qw = q[0] * g.qinv;
    g.qx = q[1] * g.qinv;
    g.qy = q[2] * g.qinv;
    g.qz = q[3] * g.qinv;
    float w = g.qw, x = g.qx, y = g.qy, z = g.qz;
    g.R[0] = 1.f - 2.f * (y * y + z * z);
    g.R[1] = 2.f * (x * y - w * z);
    g.R[2] = 2.f * (x * z + w * y);
    g.R[3] = 2.f * (x * y + w * z);
    g.R[4] = 1.f - 2.f * (x * x + z * z);
    g.R[5] = 2.f * (y * z - w * x);
    g.R[6] = 2.f * (x * z - w * y);
    g.R[7] = 2.f * (y * z + w * x);
    g.R[8] = 1.f - 2.f * (x * x + y * y);
    g.phi = 2.0f / (1.0f + expf(-st.rho * (beta - 2.0f)));
    for (int b = 0; b < 3; ++b) g.ps[b] = g.phi * s[b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) g.M[3 * a + b] = g.R[3 * a + b] * g.ps[b];
}

// Per-view projection state (kept for the adjoint).
struct ViewProj {
    float p[3];        // camera-space centre (compensated dot products)
    float xt, yt;      // frustum-clamped x, y used by the Jacobian
    bool clx, cly;     // whether x / y were clamped
    float limx, limy;
    float T[6];        // J W (2 x 3)
    float U0[3], U1[3];  // rows of U = T M, so Sigma' = U U^T + blur I
    float a, b, c;     // Sigma' (with blur)
    float det;
    float L00, L10, L11;  // conic factor: q = (L00 dx + L10 dy)^2 + (L11 dy)^2
    float u, v;
    bool ok;           // survived near plane and determinant culls
};

__device__ __forceinline__ void project_view(const float* mean, const SplatGeom& g, const DevView& w,
                                             const DevSettings& st, ViewProj& vp) {
    vp.p[0] = dot3_plus_compensated(&w.R[0], mean, w.t[0]);
    vp.p[1] = dot3_plus_compensated(&w.R[3], mean, w.t[1]);
    vp.p[2] = dot3_plus_compensated(&w.R[6], mean, w.t[2]);
    vp.ok = vp.p[2] > st.znear;
    const float z = vp.p[2];
    const float iz = 1.0f / z;
    vp.limx = st.clip_fac * (float)w.W / (2.0f * w.fx);
    vp.limy = st.clip_fac * (float)w.H / (2.0f * w.fy);
    const float txz = vp.p[0] / z, tyz = vp.p[1] / z;
    vp.clx = fabsf(txz) > vp.limx;
    vp.cly = fabsf(tyz) > vp.limy;
    vp.xt = vp.clx ? copysignf(vp.limx, txz) * z : vp.p[0];
    vp.yt = vp.cly ? copysignf(vp.limy, tyz) * z : vp.p[1];
    const float J00 = w.fx * iz, J02 = -w.fx * vp.xt * iz * iz;
    const float J11 = w.fy * iz, J12 = -w.fy * vp.yt * iz * iz;
    for (int b = 0; b < 3; ++b) {
        vp.T[b] = J00 * w.R[b] + J02 * w.R[6 + b];
        vp.T[3 + b] = J11 * w.R[3 + b] + J12 * w.R[6 + b];
    }
    const float* T = vp.T;
    const float* M = g.M;
    for (int b = 0; b < 3; ++b) {
        vp.U0[b] = T[0] * M[b] + T[1] * M[3 + b] + T[2] * M[6 + b];
        vp.U1[b] = T[3] * M[b] + T[4] * M[3 + b] + T[5] * M[6 + b];
    }
    const float* U0 = vp.U0;
    const float* U1 = vp.U1;
    const float a0 = U0[0] * U0[0] + U0[1] * U0[1] + U0[2] * U0[2];
    const float c0 = U1[0] * U1[0] + U1[1] * U1[1] + U1[2] * U1[2];
    vp.b = U0[0] * U1[0] + U0[1] * U1[1] + U0[2] * U1[2];
    // det(U U^T + blur I) = |U0 x U1|^2 + blur (|U0|^2 + |U1|^2) + blur^2, a sum of
    // non-negative terms (no cancellation as in a c - b^2 for thin footprints).
    // With U0 = M^T T0, U1 = M^T T1:  U0 x U1 = det(M) M^-1 (T0 x T1), whose k-th
    // component is (prod_{j != k} phi s_j) (R^T (T0 x T1))_k -- exact in form even
    // for near-2-D splats seen edge-on.
    const float n0 = T[1] * T[5] - T[2] * T[4];
    const float n1 = T[2] * T[3] - T[0] * T[5];
    const float n2 = T[0] * T[4] - T[1] * T[3];
    const float* R = g.R;
    const float m0 = R[0] * n0 + R[3] * n1 + R[6] * n2;
    const float m1 = R[1] * n0 + R[4] * n1 + R[7] * n2;
    const float m2 = R[2] * n0 + R[5] * n1 + R[8] * n2;
    const float x0 = (g.ps[1] * g.ps[2]) * m0;
    const float x1 = (g.ps[0] * g.ps[2]) * m1;
    const float x2 = (g.ps[0] * g.ps[1]) * m2;
    vp.det = (x0 * x0 + x1 * x1 + x2 * x2) + st.blur * (a0 + c0) + st.blur * st.blur;
    vp.a = a0 + st.blur;
    vp.c = c0 + st.blur;
    vp.ok = vp.ok && vp.det > 0.0f && vp.c > 0.0f;
    // Cholesky factor of the conic Sigma'^-1: L11 = c^-1/2, L00 = (c / det)^1/2, L10 = -b (c det)^-1/2
    const float rs = 1.0f / sqrtf(vp.det);
    vp.L11 = 1.0f / sqrtf(vp.c);
    vp.L00 = sqrtf(vp.c) * rs;
    vp.L10 = -vp.b * vp.L11 * rs;
    vp.u = fmaf(w.fx, vp.p[0] / z, w.cx);
    vp.v = fmaf(w.fy, vp.p[1] / z, w.cy);
}

template <int DEG>
__device__ __forceinline__ void view_dir(const float* mean, const DevView& w, float& dx, float& dy, float& dz,
                                         float& inv) {
    float d0 = mean[0] - w.campos[0], d1 = mean[1] - w.campos[1], d2 = mean[2] - w.campos[2];
    inv = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
    dx = d0 * inv;
    dy = d1 * inv;
    dz = d2 * inv;
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project(ProjectArgs a) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int n = a.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float mean[3], s[3], q[4];
    for (int k = 0; k < 3; ++k) {
        mean[k] = a.mean[k * n + i];
        s[k] = a.scale[k * n + i];
    }
    for (int k = 0; k < 4; ++k) q[k] = a.quat[k * n + i];
    const float op = a.opacity[i];
    const float beta = a.beta[i];
    float sh[K * 3];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) sh[k] = a.sh[(size_t)k * n + i];

    const DevSettings& st = a.st;
    SplatGeom g;
    splat_geom(s, q, beta, st, g);
    // q_max = (ln(o / alpha_min) / kappa)^(2 / beta) (1 + 2^-10): alpha >= alpha_min only inside
    const float L = logf(op / st.alpha_min) / st.kappa;
    const float qmax = exp2f(log2f(L) * (2.0f / beta)) * (1.0f + 1.0f / 1024.0f);

    for (int v = 0; v < a.cams.V; ++v) {
        const DevView& w = a.cams.v[v];
        const size_t vi = (size_t)v * n + i;
        ViewProj vp;
        project_view(mean, g, w, st, vp);
        float dxn, dyn, dzn, dinv;
        view_dir<DEG>(mean, w, dxn, dyn, dzn, dinv);
        float Y[K];
        sh_eval<DEG>(dxn, dyn, dzn, Y);
        float rgb[3];
        for (int c = 0; c < 3; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) acc = fmaf(Y[k], sh[3 * k + c], acc);
            // clamp at 0; a NaN stays NaN (fmaxf would return 0) so the pair is culled below
            const float col = acc + 0.5f;
            rgb[c] = col < 0.0f ? 0.0f : col;
        }
        bool keep = vp.ok && op >= st.alpha_min;
        float rx = sqrtf(qmax * vp.a), ry = sqrtf(qmax * vp.c);
        float fx0 = ceilf(vp.u - rx - 0.5f), fx1 = floorf(vp.u + rx - 0.5f);
        float fy0 = ceilf(vp.v - ry - 0.5f), fy1 = floorf(vp.v + ry - 0.5f);
        fx0 = fmaxf(fx0, 0.f);
        fy0 = fmaxf(fy0, 0.f);
        fx1 = fminf(fx1, (float)(w.W - 1));
        fy1 = fminf(fy1, (float)(w.H - 1));
        keep = keep && fx0 <= fx1 && fy0 <= fy1;
        // non-finite parameters or results cull the pair
        float chk = vp.u + vp.v + vp.L00 + vp.L10 + vp.L11 + op + beta + rgb[0] + rgb[1] + rgb[2] + qmax + vp.a +
                    vp.c + vp.det;
        keep = keep && isfinite(chk);
        float4* rec = reinterpret_cast<float4*>(a.rec + vi * GESR_REC_FLOATS);
        if (keep) {
            int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
            int tx0 = x0 / st.tile_w, tx1 = x1 / st.tile_w, ty0 = y0 / st.tile_h, ty1 = y1 / st.tile_h;
            const uint2 rc = make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)tx1 | ((uint32_t)ty1 << 16));
            rec[0] = make_float4(vp.u, vp.v, vp.L00, vp.L10);
            rec[1] = make_float4(vp.L11, op, beta, qmax);
            rec[2] = make_float4(rgb[0], rgb[1], rgb[2], vp.p[2]);
            rec[3] = make_float4(__uint_as_float(rc.x), __uint_as_float(rc.y), 0.f, 0.f);
            a.tiles_touched[vi] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
            reinterpret_cast<uint2*>(a.rect)[vi] = rc;
            a.depth_key[vi] = __float_as_uint(vp.p[2]);
        } else {
            float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
            rec[0] = zero;
            rec[1] = zero;
            rec[2] = zero;
            rec[3] = make_float4(__uint_as_float(0xFFFFFFFFu), 0.f, 0.f, 0.f);
            a.tiles_touched[vi] = 0u;
            reinterpret_cast<uint2*>(a.rect)[vi] = make_uint2(0xFFFFFFFFu, 0u);  // culled: no rectangle
            a.depth_key[vi] = 0xFFFFFFFFu;
        }
    }
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd(ProjectBwdArgs a) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int n = a.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float mean[3], s[3], q[4];
    for (int k = 0; k < 3; ++k) {
        mean[k] = a.mean[k * n + i];
        s[k] = a.scale[k * n + i];
    }
    for (int k = 0; k < 4; ++k) q[k] = a.quat[k * n + i];
    const float beta = a.beta[i];
    float sh[K * 3];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) sh[k] = a.sh[(size_t)k * n + i];

    const DevSettings& st = a.st;
    SplatGeom g;
    splat_geom(s, q, beta, st, g);

    float gm[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
    float gop = 0.f, gbeta = 0.f;
    float gsh[K * 3];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) gsh[k] = 0.f;

    for (int v = 0; v < a.cams.V; ++v) {
        const size_t vi = (size_t)v * n + i;
        const uint32_t cnt = a.tiles_touched[vi];
        if (cnt == 0) continue;
        float g2[GESR_GRAD2D_FLOATS];
        const float4* src = reinterpret_cast<const float4*>(a.grad2d + vi * GESR_GRAD2D_FLOATS);
#pragma unroll
        for (int k = 0; k < GESR_GRAD2D_FLOATS / 4; ++k) {
            const float4 t4 = src[k];
            g2[4 * k] = t4.x;
            g2[4 * k + 1] = t4.y;
            g2[4 * k + 2] = t4.z;
            g2[4 * k + 3] = t4.w;
        }
        const float du = g2[0], dv = g2[1];

        const DevView& w = a.cams.v[v];
        ViewProj vp;
        project_view(mean, g, w, st, vp);

        // local (this view's) contributions, added to the accumulators at the end
        float lm[3] = {0.f, 0.f, 0.f};
        float lsh[K * 3];

        // ---- colour: rgb_c = max(sum_k Y_k sh_kc + 1/2, 0)
        float dxn, dyn, dzn, dinv;
        view_dir<DEG>(mean, w, dxn, dyn, dzn, dinv);
        float Y[K];
        sh_eval<DEG>(dxn, dyn, dzn, Y);
        float dcol[3];
        for (int c = 0; c < 3; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) acc = fmaf(Y[k], sh[3 * k + c], acc);
            dcol[c] = (acc + 0.5f < 0.0f) ? 0.0f : g2[7 + c];
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            for (int c = 0; c < 3; ++c) lsh[3 * k + c] = Y[k] * dcol[c];
        if (DEG > 0) {
            float wk[K];
#pragma unroll
            for (int k = 0; k < K; ++k) wk[k] = sh[3 * k] * dcol[0] + sh[3 * k + 1] * dcol[1] + sh[3 * k + 2] * dcol[2];
            float gx, gy, gz;
            sh_grad<DEG>(dxn, dyn, dzn, wk, gx, gy, gz);
            // d(dir)/d(mean) = (I - dir dir^T) / |mean - campos|
            float dd = gx * dxn + gy * dyn + gz * dzn;
            lm[0] += (gx - dd * dxn) * dinv;
            lm[1] += (gy - dd * dyn) * dinv;
            lm[2] += (gz - dd * dzn) * dinv;
        }

        // ---- conic factor (L00, L10, L11) -> Sigma' entries (a, b, c), det = a c - b^2
        const float dL00 = g2[2], dL10 = g2[3], dL11 = g2[4];
        const float ia = vp.a, ib = vp.b, ic = vp.c;
        const float idet = 1.0f / vp.det, icc = 1.0f / ic;
        const float da = -0.5f * ic * idet * (dL00 * vp.L00 + dL10 * vp.L10);
        const float db = (ib * dL00 - ia * dL10) * vp.L00 * idet;
        const float dc = dL00 * vp.L00 * 0.5f * (icc - ia * idet) - 0.5f * dL10 * vp.L10 * (icc + ia * idet) -
                         0.5f * dL11 * vp.L11 * icc;
        // Sigma' = U U^T + blur I with U = T M:  dU = 2 G' U, G' = [[da, db/2], [db/2, dc]]
        float dU0[3], dU1[3];
        for (int k = 0; k < 3; ++k) {
            dU0[k] = 2.f * da * vp.U0[k] + db * vp.U1[k];
            dU1[k] = db * vp.U0[k] + 2.f * dc * vp.U1[k];
        }
        const float* T = vp.T;
        // dT = dU M^T (2 x 3)
        float dT[6];
        for (int k = 0; k < 3; ++k) {
            dT[k] = dU0[0] * g.M[3 * k] + dU0[1] * g.M[3 * k + 1] + dU0[2] * g.M[3 * k + 2];
            dT[3 + k] = dU1[0] * g.M[3 * k] + dU1[1] * g.M[3 * k + 1] + dU1[2] * g.M[3 * k + 2];
        }
        // T = J W  ->  dJ = dT W^T (only J00, J02, J11, J12 vary)
        const float dJ00 = dT[0] * w.R[0] + dT[1] * w.R[1] + dT[2] * w.R[2];
        const float dJ02 = dT[0] * w.R[6] + dT[1] * w.R[7] + dT[2] * w.R[8];
        const float dJ11 = dT[3] * w.R[3] + dT[4] * w.R[4] + dT[5] * w.R[5];
        const float dJ12 = dT[3] * w.R[6] + dT[4] * w.R[7] + dT[5] * w.R[8];
        const float z = vp.p[2], iz = 1.0f / z, iz2 = iz * iz, iz3 = iz2 * iz;
        float dp[3] = {0.f, 0.f, 0.f};
        dp[2] += dJ00 * (-w.fx * iz2) + dJ02 * (2.f * w.fx * vp.xt * iz3) + dJ11 * (-w.fy * iz2) +
                 dJ12 * (2.f * w.fy * vp.yt * iz3);
        const float dxt = dJ02 * (-w.fx * iz2);
        const float dyt = dJ12 * (-w.fy * iz2);
        if (vp.clx) dp[2] += dxt * copysignf(vp.limx, vp.p[0] * iz);
        else dp[0] += dxt;
        if (vp.cly) dp[2] += dyt * copysignf(vp.limy, vp.p[1] * iz);
        else dp[1] += dyt;
        // projected centre
        dp[0] += du * w.fx * iz;
        dp[1] += dv * w.fy * iz;
        dp[2] += -(du * w.fx * vp.p[0] + dv * w.fy * vp.p[1]) * iz2;
        // depth of the centre (extended channels): z = p[2]
        dp[2] += g2[10];
        // p = W mean + t
        for (int k = 0; k < 3; ++k) lm[k] += w.R[k] * dp[0] + w.R[3 + k] * dp[1] + w.R[6 + k] * dp[2];

        // dM = T^T dU (3 x 3)
        float dM[9];
        for (int r = 0; r < 3; ++r)
            for (int c2 = 0; c2 < 3; ++c2) dM[3 * r + c2] = T[r] * dU0[c2] + T[3 + r] * dU1[c2];
        // ---- M = R diag(phi s)
        float ls[3], dphi = 0.f;
        float dR[9];
        for (int c2 = 0; c2 < 3; ++c2) {
            float acc = 0.f;
            for (int r = 0; r < 3; ++r) {
                dR[3 * r + c2] = dM[3 * r + c2] * (g.phi * s[c2]);
                acc += dM[3 * r + c2] * g.R[3 * r + c2];
            }
            ls[c2] = g.phi * acc;
            dphi += acc * s[c2];
        }
        // phi(beta) = 2 / (1 + exp(-rho (beta - 2)))  ->  dphi/dbeta = rho phi (1 - phi/2)
        const float lbeta = g2[6] + dphi * st.rho * g.phi * (1.f - 0.5f * g.phi);
        // rotation of the normalised quaternion
        const float w_ = g.qw, x = g.qx, y = g.qy, zq = g.qz;
        float dqn[4];
        dqn[0] = 2.f * (-zq * dR[1] + y * dR[2] + zq * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
        dqn[1] = 2.f * (y * dR[1] + zq * dR[2] + y * dR[3] - 2.f * x * dR[4] - w_ * dR[5] + zq * dR[6] + w_ * dR[7] -
                        2.f * x * dR[8]);
        dqn[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w_ * dR[2] + x * dR[3] + zq * dR[5] - w_ * dR[6] + zq * dR[7] -
                        2.f * y * dR[8]);
        dqn[3] = 2.f * (-2.f * zq * dR[0] - w_ * dR[1] + x * dR[2] + w_ * dR[3] - 2.f * zq * dR[4] + y * dR[5] +
                        x * dR[6] + y * dR[7]);
        const float qd = dqn[0] * w_ + dqn[1] * x + dqn[2] * y + dqn[3] * zq;
        const float qn[4] = {w_, x, y, zq};
        float lq[4];
        for (int k = 0; k < 4; ++k) lq[k] = (dqn[k] - qn[k] * qd) * g.qinv;

        // accumulate this view's contribution (fixed ascending view order)
        for (int k = 0; k < 3; ++k) gm[k] += lm[k];
        for (int k = 0; k < 3; ++k) gs[k] += ls[k];
        for (int k = 0; k < 4; ++k) gq[k] += lq[k];
        gop += g2[5];
        gbeta += lbeta;
#pragma unroll
        for (int k = 0; k < K * 3; ++k) gsh[k] += lsh[k];
    }
    for (int k = 0; k < 3; ++k) {
        a.g_mean[k * n + i] = gm[k];
        a.g_scale[k * n + i] = gs[k];
    }
    for (int k = 0; k < 4; ++k) a.g_quat[k * n + i] = gq[k];
    a.g_opacity[i] = gop;
    a.g_beta[i] = gbeta;
#pragma unroll
    for (int k = 0; k < K * 3; ++k) a.g_sh[(size_t)k * n + i] = gsh[k];
}

// Segmented sum of the visited partials per (view, splat).  The pair's
// instance slots are contiguous (inst_base[vi] + j) and are taken in blocks of
// 32 (one word of visited bits); within a block the set bits' partials are
// added in ascending slot order.  A pair of at most kSegSmall instances is
// summed by one lane (a sum per block, the two added at the end); a larger
// pair by an aligned group of kSegLanes lanes, lane l taking the blocks l,
// l + kSegLanes, ... in ascending order, then a fixed DPP tree over the group;
// a pair of more than kSegHuge instances likewise by the whole wave (a DPP
// tree per 16-lane row, then the four row totals in row order).  The order
// depends only on the pair's own instance count, so a batch of views and
// views rendered one at a time give identical sums.  One thread per pair: the
// small pairs (most of them) keep every lane busy, then each wave sums its
// huge pairs one at a time and hands the other large ones to its eight
// groups, eight at a time (the longest pairs, thousands of instances, would
// otherwise serialise hundreds of dependent loads on eight lanes).
constexpr uint32_t kSegLanes = 8;
constexpr uint32_t kSegSmall = 64;
constexpr uint32_t kSegHuge = 512;

// Adds block j0 .. j0 + 31 of the pair (first slot `base`, cnt slots) to acc.
template <int NP>
__device__ __forceinline__ void seg_block(const SegReduceArgs& a, uint64_t base, uint32_t cnt, uint32_t j0,
                                          uint64_t nwords, float (&acc)[NP]) {
    // visited bits of instances j0 .. j0 + 31 of this pair
    const uint64_t s0 = base + j0;
    const uint64_t wi = s0 >> 5;
    const uint32_t sh = (uint32_t)(s0 & 31u);
    const uint32_t w0 = wi < nwords ? a.visited[wi] : 0u;
    const uint32_t w1 = (sh != 0u && wi + 1 < nwords) ? a.visited[wi + 1] : 0u;
    uint32_t bits = sh != 0u ? (w0 >> sh) | (w1 << (32u - sh)) : w0;
    if (cnt - j0 < 32u) bits &= (1u << (cnt - j0)) - 1u;
    // up to four visited partials in flight, then added in ascending order
    while (bits != 0u) {
        float4 v[4][3];
        bool have[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            have[u] = bits != 0u;
            const uint32_t b = have[u] ? (uint32_t)__builtin_ctz(bits) : 0u;
            bits &= bits - 1u;
            const float4* src = reinterpret_cast<const float4*>(a.partials + (s0 + b) * kPartialStride);
#pragma unroll
            for (int k = 0; k < 3; ++k) v[u][k] = have[u] ? src[k] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (have[u]) {
                const float t[12] = {v[u][0].x, v[u][0].y, v[u][0].z, v[u][0].w, v[u][1].x, v[u][1].y,
                                     v[u][1].z, v[u][1].w, v[u][2].x, v[u][2].y, v[u][2].z, v[u][2].w};
#pragma unroll
                for (int k = 0; k < NP; ++k) acc[k] += t[k];
            }
    }
}

template <int NP>
__device__ __forceinline__ void seg_write(const SegReduceArgs& a, uint64_t vi, const float (&acc)[NP]) {
    float4* out = reinterpret_cast<float4*>(a.grad2d + (size_t)vi * GESR_GRAD2D_FLOATS);
    out[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    out[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
    out[2] = make_float4(acc[8], acc[9], acc[10], 0.0f);
}

__global__ __launch_bounds__(256) void k_seg_reduce(SegReduceArgs a) {
    constexpr int NP = GESR_PARTIAL_FLOATS + 1;  // the ten terms and dz
    constexpr uint32_t L = kSegLanes;
    const uint64_t vi = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const uint32_t lane = __lane_id();
    const bool valid = vi < a.vn;
    const uint32_t cnt = valid ? a.tiles_touched[vi] : 0u;
    const uint64_t base = valid ? a.inst_base[vi] : 0u;
    const uint64_t nwords = (a.m_cap + 31) / 32;
    const bool small = cnt <= kSegSmall;
    if (valid && small) {
        float acc0[NP], acc1[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) acc0[k] = acc1[k] = 0.f;
        if (cnt > 0) seg_block<NP>(a, base, cnt, 0u, nwords, acc0);
        if (cnt > 32) seg_block<NP>(a, base, cnt, 32u, nwords, acc1);
#pragma unroll
        for (int k = 0; k < NP; ++k) acc0[k] += acc1[k];
        seg_write<NP>(a, vi, acc0);
    }
    const uint64_t wave0 = vi - lane;
    // huge pairs of this wave, one at a time over all its lanes
    uint64_t huge = __ballot(valid && cnt > kSegHuge);
    while (huge != 0ull) {
        const uint32_t pick = (uint32_t)__builtin_ctzll(huge);
        const uint32_t c = (uint32_t)__shfl((int)cnt, (int)pick, 64);
        const uint64_t b0 = (uint64_t)(uint32_t)__shfl((int)(uint32_t)base, (int)pick, 64);
        float acc[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) acc[k] = 0.f;
        for (uint32_t j0 = lane * 32u; j0 < c; j0 += 64u * 32u) seg_block<NP>(a, b0, c, j0, nwords, acc);
        float tot[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int r = __float_as_int(group_sum<16>(acc[k]));
            tot[k] = ((__int_as_float(__builtin_amdgcn_readlane(r, 0)) + __int_as_float(__builtin_amdgcn_readlane(r, 16))) +
                      __int_as_float(__builtin_amdgcn_readlane(r, 32))) +
                     __int_as_float(__builtin_amdgcn_readlane(r, 48));
        }
        if (lane == 0) seg_write<NP>(a, wave0 + pick, tot);
        huge &= huge - 1u;
    }
    // the other large pairs, eight at a time (group g = lane / L takes the
    // g-th remaining one)
    uint64_t large = __ballot(valid && !small && cnt <= kSegHuge);
    const uint32_t g = lane / L, l = lane % L;
    while (large != 0ull) {
        uint64_t m = large;
        for (uint32_t k = 0; k < g; ++k) m &= m - 1u;
        const bool mine = m != 0ull;
        const uint32_t pick = mine ? (uint32_t)__builtin_ctzll(m) : 0u;
        const uint32_t c = (uint32_t)__shfl((int)cnt, (int)pick, 64);
        const uint64_t b0 = (uint64_t)(uint32_t)__shfl((int)(uint32_t)base, (int)pick, 64);
        float acc[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) acc[k] = 0.f;
        if (mine)
            for (uint32_t j0 = l * 32u; j0 < c; j0 += L * 32u) seg_block<NP>(a, b0, c, j0, nwords, acc);
#pragma unroll
        for (int k = 0; k < NP; ++k) acc[k] = group_sum<L>(acc[k]);
        if (mine && l == L - 1) seg_write<NP>(a, wave0 + pick, acc);
#pragma unroll
        for (uint32_t k = 0; k < 64u / L; ++k) large &= large - 1u;
    }
}

}  // namespace

hipError_t launch_project(const ProjectArgs& a, int sh_degree, hipStream_t stream) {
    if (a.n == 0) return hipSuccess;
    dim3 grid((a.n + 255) / 256), block(256);
    switch (sh_degree) {
        case 0: hipLaunchKernelGGL(k_project<0>, grid, block, 0, stream, a); break;
        case 1: hipLaunchKernelGGL(k_project<1>, grid, block, 0, stream, a); break;
        case 2: hipLaunchKernelGGL(k_project<2>, grid, block, 0, stream, a); break;
        default: hipLaunchKernelGGL(k_project<3>, grid, block, 0, stream, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_seg_reduce(const SegReduceArgs& a, hipStream_t stream) {
    if (a.vn == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_reduce, dim3((unsigned)(((uint64_t)a.vn + 255) / 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_project_bwd(const ProjectBwdArgs& a, int sh_degree, hipStream_t stream) {
    if (a.n == 0) return hipSuccess;
    dim3 grid((a.n + 255) / 256), block(256);
    switch (sh_degree) {
        case 0: hipLaunchKernelGGL(k_project_bwd<0>, grid, block, 0, stream, a); break;
        case 1: hipLaunchKernelGGL(k_project_bwd<1>, grid, block, 0, stream, a); break;
        case 2: hipLaunchKernelGGL(k_project_bwd<2>, grid, block, 0, stream, a); break;
        default: hipLaunchKernelGGL(k_project_bwd<3>, grid, block, 0, stream, a); break;
    }
    return hipGetLastError();
}

}  // namespace gesr
