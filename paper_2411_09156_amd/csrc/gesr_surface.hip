// Level-set surface points along depth-map rays (gfx950): the sampling step of
// the mesh extraction in Sec. 3.3.  For each requested pixel the ray from the
// camera centre through the pixel centre starts at the depth-map point
// (depth / alpha of the extended channels); the density of Eq. 9,
// d(x) = sum_i o_i exp(-kappa m_i(x)^beta_i) with m_i the 3-D Mahalanobis
// distance under Sigma_i = M_i M_i^T, M_i = R(q_i) diag(phi(beta_i) s_i)
// (Eq. 4, 6), is summed over the splats of the pixel's tile list whose screen
// footprint covers the pixel.  K samples spread over +-span sigma_g(w) around
// the depth-map point, g the splat with the largest term there (the dominating
// distribution of Eq. 10), sigma_g(w) = |M_g^T w|; the first sample pair with
// d_k < level <= d_{k+1} brackets the surface closest to the camera, t* by
// linear interpolation, and the normal is -grad d / |grad d| (the direction of
// grad f for the SDF of Eq. 11).
//
// Eight lanes per ray (eight rays per wave) stride over the tile list.  Along the ray each
// candidate's Mahalanobis vector is affine in the ray parameter, y(s) = a + s b
// (a = M^-1 (x0 - mu), b = M^-1 w, s = t - t0), so a sample costs two
// multiply-adds plus the falloff.  Each lane keeps its partial density of every
// sample in registers; the partials meet in LDS and are summed per sample in
// lane order (fixed order, reproducible).

#include "gesr_device.h"
#include "gesr_kernels.h"

namespace gesr {

namespace {

constexpr int kMaxSamples = GESR_SURFACE_MAX_SAMPLES;

// Rotation of the normalised quaternion (Eq. 4) and the shape-modulated scales
// phi(beta) s (Eq. 6) of splat i: M = R diag(ps).
__device__ __forceinline__ void splat_frame(const SurfaceArgs& A, uint32_t i, float R[9], float ps[3]) {
    const uint32_t n = (uint32_t)A.n;
    const float q[4] = {A.quat[i], A.quat[n + i], A.quat[2 * n + i], A.quat[3 * n + i]};
    const float qi = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float qw = q[0] * qi, qx = q[1] * qi, qy = q[2] * qi, qz = q[3] * qi;
    R[0] = 1.f - 2.f * (qy * qy + qz * qz);
    R[1] = 2.f * (qx * qy - qw * qz);
    R[2] = 2.f * (qx * qz + qw * qy);
    R[3] = 2.f * (qx * qy + qw * qz);
    R[4] = 1.f - 2.f * (qx * qx + qz * qz);
    R[5] = 2.f * (qy * qz - qw * qx);
    R[6] = 2.f * (qx * qz - qw * qy);
    R[7] = 2.f * (qy * qz + qw * qx);
    R[8] = 1.f - 2.f * (qx * qx + qy * qy);
    const float phi = 2.0f / (1.0f + expf(-A.st.rho * (A.beta[i] - 2.0f)));
#pragma unroll
    for (int c = 0; c < 3; ++c) ps[c] = phi * A.scale[c * n + i];
}

// Per splat (view independent), one 64-byte record: M^-1 = diag(1/ps) R^T row
// major (9), the mean (3), opacity and beta/2, so a candidate costs one cache
// line instead of ten scattered parameter loads and the frame arithmetic.
__global__ __launch_bounds__(256) void k_surface_frames(SurfaceArgs A) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= (uint32_t)A.n) return;
    const uint32_t n = (uint32_t)A.n;
    float R[9], ps[3];
    splat_frame(A, i, R, ps);
    float m[9];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float inv = 1.0f / ps[k];
        m[3 * k] = R[k] * inv;
        m[3 * k + 1] = R[3 + k] * inv;
        m[3 * k + 2] = R[6 + k] * inv;
    }
    float4* f = reinterpret_cast<float4*>(A.frames) + 4 * (size_t)i;
    f[0] = make_float4(m[0], m[1], m[2], m[3]);
    f[1] = make_float4(m[4], m[5], m[6], m[7]);
    f[2] = make_float4(m[8], A.mean[i], A.mean[n + i], A.mean[2 * n + i]);
    f[3] = make_float4(A.opacity[i], 0.5f * A.beta[i], 0.f, 0.f);
}

struct Frame {
    float m[9], mu[3], o, half_beta;
};

__device__ __forceinline__ void load_frame(const float* frames, uint32_t i, Frame& f) {
    const float4* p = reinterpret_cast<const float4*>(frames) + 4 * (size_t)i;
    const float4 f0 = p[0], f1 = p[1], f2 = p[2], f3 = p[3];
    f.m[0] = f0.x; f.m[1] = f0.y; f.m[2] = f0.z; f.m[3] = f0.w;
    f.m[4] = f1.x; f.m[5] = f1.y; f.m[6] = f1.z; f.m[7] = f1.w;
    f.m[8] = f2.x; f.mu[0] = f2.y; f.mu[1] = f2.z; f.mu[2] = f2.w;
    f.o = f3.x; f.half_beta = f3.y;
}

// a = M^-1 (x0 - mu), b = M^-1 w.
struct Affine {
    float a[3], b[3];
    float o, half_beta;
};

__device__ __forceinline__ void frame_affine(const Frame& fr, const float x0[3], const float w[3], Affine& f) {
    const float d[3] = {x0[0] - fr.mu[0], x0[1] - fr.mu[1], x0[2] - fr.mu[2]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        f.a[k] = fr.m[3 * k] * d[0] + fr.m[3 * k + 1] * d[1] + fr.m[3 * k + 2] * d[2];
        f.b[k] = fr.m[3 * k] * w[0] + fr.m[3 * k + 1] * w[1] + fr.m[3 * k + 2] * w[2];
    }
    f.o = fr.o;
    f.half_beta = fr.half_beta;
}

// o exp(-kappa (m^2)^(beta/2)) for m^2 = |a + s b|^2
__device__ __forceinline__ float affine_term(const Affine& f, float s, const DevSettings& st) {
    float m2 = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float y = fmaf(s, f.b[k], f.a[k]);
        m2 = fmaf(y, y, m2);
    }
    const float P = hw_exp2(f.half_beta * hw_log2(m2));  // 0 at m2 = 0
    return f.o * hw_exp2(st.neg_kappa_log2e * P);
}

// Calls body(frame, list position) for every candidate of pixel (px, py)
// among the list entries rg.x + u, + S, + 2S, ... (u: the lane's place among
// the S lanes of its ray): the splats whose screen footprint covers the pixel
// (q <= qmax, the renderers' test).  The next entry's splat id is loaded while
// the current entry is processed.
template <int S, class F>
__device__ __forceinline__ void for_candidates(const SurfaceArgs& A, uint2 rg, uint32_t u, float px, float py,
                                               F&& body) {
    uint32_t k = rg.x + u;
    uint32_t vi = k < rg.y ? A.val_sorted[k] : 0u;
    for (; k < rg.y; k += S) {
        const float4* r = reinterpret_cast<const float4*>(A.rec + (size_t)vi * GESR_REC_FLOATS);
        const float4 ra = r[0], rb = r[1];
        Frame fr;
        load_frame(A.frames, vi % (uint32_t)A.n, fr);
        const uint32_t kn = k + S;
        vi = kn < rg.y ? A.val_sorted[kn] : 0u;
        Fragment f;
        if (ges_q(ra, rb.x, px, py, f) <= rb.w) body(fr, k);
    }
}

// Sum over the L lanes of a ray's group (xor steps stay inside the group).
template <int L>
__device__ __forceinline__ float lane_group_sum(float x) {
#pragma unroll
    for (int m = L / 2; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// Eight rays per wave, eight lanes each.  Rays of the same tile (the caller
// passes pixels grouped by tile) traverse the same list in lockstep, so the
// lanes that load one entry for different rays hit the same addresses; rays of
// different tiles are simply handled side by side.
constexpr int kRaysPerWave = 8, kLanesPerRay = 64 / kRaysPerWave;

__global__ __launch_bounds__(64) void k_surface_points(SurfaceArgs A) {
    __shared__ float sPart[64][kMaxSamples + 1];
    __shared__ float sDen[kRaysPerWave][kMaxSamples];
    const uint32_t lane = __lane_id(), slot = lane / kLanesPerRay, u = lane % kLanesPerRay;
    const uint32_t ray = blockIdx.x * kRaysPerWave + slot;
    const bool has_ray = ray < A.n_rays;
    const DevSettings& st = A.st;
    const DevView* views = A.cams.v;
    const uint32_t pix = has_ray ? A.pixels[ray] : 0u;
    int v = 0;
    while (v + 1 < A.cams.V && views[v + 1].pix_base <= pix) ++v;
    const DevView& w = views[v];
    const uint32_t local = pix - w.pix_base;
    const int px = (int)(local % (uint32_t)w.W), py = (int)(local / (uint32_t)w.W);
    const float alpha = has_ray ? A.alpha[pix] : 0.f, depth = has_ray ? A.depth[pix] : 0.f;
    if (has_ray && u == 0) {
        reinterpret_cast<float4*>(A.points)[ray] = make_float4(0.f, 0.f, 0.f, 0.f);
        reinterpret_cast<float4*>(A.normals)[ray] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (A.dominant) A.dominant[ray] = 0xFFFFFFFFu;
        if (A.n_candidates) A.n_candidates[ray] = 0u;
    }
    bool live = has_ray && alpha >= A.min_alpha && alpha > 0.f;
    // ray: camera-space direction with unit z, rotated to world space by R^T
    const float dc[3] = {((float)px + 0.5f - w.cx) / w.fx, ((float)py + 0.5f - w.cy) / w.fy, 1.0f};
    const float nd = sqrtf(dc[0] * dc[0] + dc[1] * dc[1] + 1.0f);
    float wd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) wd[a] = (w.R[a] * dc[0] + w.R[3 + a] * dc[1] + w.R[6 + a] * dc[2]) / nd;
    const float t0 = live ? depth / alpha * nd : 0.f;
    const float x0[3] = {w.campos[0] + t0 * wd[0], w.campos[1] + t0 * wd[1], w.campos[2] + t0 * wd[2]};
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const uint32_t t = w.tile_base + (uint32_t)(py / A.tile_h) * (uint32_t)w.tiles_x + (uint32_t)(px / A.tile_w);
    uint2 rg = live ? reinterpret_cast<const uint2*>(A.ranges)[t] : make_uint2(0u, 0u);

    // pass 1: the dominating splat at x0 (largest term; ties to the earliest list position)
    float best = -1.0f;
    uint32_t best_pos = 0xFFFFFFFFu, ncand = 0;
    for_candidates<kLanesPerRay>(A, rg, u, fpx, fpy, [&](const Frame& fr, uint32_t k) {
        ++ncand;
        Affine f;
        frame_affine(fr, x0, wd, f);
        const float val = affine_term(f, 0.0f, st);
        if (val > best) {
            best = val;
            best_pos = k;
        }
    });
#pragma unroll
    for (int m = kLanesPerRay / 2; m >= 1; m >>= 1) {
        const float ob = __shfl_xor(best, m, 64);
        const uint32_t op = (uint32_t)__shfl_xor((int)best_pos, m, 64);
        if (ob > best || (ob == best && op < best_pos)) {
            best = ob;
            best_pos = op;
        }
    }
    const uint32_t tot = (uint32_t)lane_group_sum<kLanesPerRay>((float)ncand);  // exact below 2^24
    if (live && u == 0 && A.n_candidates) A.n_candidates[ray] = tot;
    live = live && best_pos != 0xFFFFFFFFu;
    const uint32_t g_vi = live ? A.val_sorted[best_pos] : 0u;
    if (live && u == 0 && A.dominant) A.dominant[ray] = g_vi;
    // sigma_g(w) = |M_g^T w| = |diag(ps) R^T w|
    float sg = 0.f;
    if (live) {
        float R[9], ps[3];
        splat_frame(A, g_vi % (uint32_t)A.n, R, ps);
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float e = ps[k] * (R[k] * wd[0] + R[3 + k] * wd[1] + R[6 + k] * wd[2]);
            acc = fmaf(e, e, acc);
        }
        sg = sqrtf(acc);
    }
    if (!live) rg = make_uint2(0u, 0u);
    const int K = A.n_samples;
    const float step = 2.0f * A.span * sg / (float)(K - 1), s0 = -A.span * sg;

    // pass 2: partial densities of the K samples
    float part[kMaxSamples];
#pragma unroll
    for (int k = 0; k < kMaxSamples; ++k) part[k] = 0.f;
    for_candidates<kLanesPerRay>(A, rg, u, fpx, fpy, [&](const Frame& fr, uint32_t) {
        Affine f;
        frame_affine(fr, x0, wd, f);
#pragma unroll
        for (int j = 0; j < kMaxSamples; ++j)
            if (j < K) part[j] += affine_term(f, fmaf((float)j, step, s0), st);
    });
#pragma unroll
    for (int j = 0; j < kMaxSamples; ++j) sPart[lane][j] = part[j];
    __syncthreads();
    // densities: sample j of the ray summed over its lanes in lane order
    for (int j = (int)u; j < K; j += kLanesPerRay) {
        float d = 0.f;
        for (int l = 0; l < kLanesPerRay; ++l) d += sPart[slot * kLanesPerRay + l][j];
        sDen[slot][j] = d;
    }
    __syncthreads();
    int kc = -1;
    if (live)
        for (int k = 0; k + 1 < K; ++k)
            if (sDen[slot][k] < A.level && sDen[slot][k + 1] >= A.level) {
                kc = k;
                break;
            }
    live = live && kc >= 0;
    float ss = 0.f;
    if (live) {
        const float d0 = sDen[slot][kc], d1 = sDen[slot][kc + 1];
        ss = fmaf((float)kc, step, s0) + (A.level - d0) / (d1 - d0) * step;
    }
    if (!live) rg = make_uint2(0u, 0u);

    // pass 3: density gradient at x0 + ss w
    float gd[3] = {0.f, 0.f, 0.f};
    const float xs[3] = {x0[0] + ss * wd[0], x0[1] + ss * wd[1], x0[2] + ss * wd[2]};
    for_candidates<kLanesPerRay>(A, rg, u, fpx, fpy, [&](const Frame& fr, uint32_t) {
        const float d[3] = {xs[0] - fr.mu[0], xs[1] - fr.mu[1], xs[2] - fr.mu[2]};
        float y[3], m2 = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            y[k] = fr.m[3 * k] * d[0] + fr.m[3 * k + 1] * d[1] + fr.m[3 * k + 2] * d[2];
            m2 = fmaf(y[k], y[k], m2);
        }
        if (!(m2 > 0.f)) return;  // at the centre the gradient vanishes
        const float l2 = hw_log2(m2);
        const float P = hw_exp2(fr.half_beta * l2);
        const float G = fr.o * hw_exp2(st.neg_kappa_log2e * P);
        // grad = -kappa beta (m^2)^(beta/2 - 1) G M^-T y
        const float coef = -st.kappa * 2.0f * fr.half_beta * hw_exp2((fr.half_beta - 1.0f) * l2) * G;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            gd[a] = fmaf(coef, fr.m[a] * y[0] + fr.m[3 + a] * y[1] + fr.m[6 + a] * y[2], gd[a]);
    });
#pragma unroll
    for (int a = 0; a < 3; ++a) gd[a] = lane_group_sum<kLanesPerRay>(gd[a]);
    const float gn = sqrtf(gd[0] * gd[0] + gd[1] * gd[1] + gd[2] * gd[2]);
    if (live && gn > 0.f && u == 0) {
        reinterpret_cast<float4*>(A.points)[ray] = make_float4(xs[0], xs[1], xs[2], 1.0f);
        reinterpret_cast<float4*>(A.normals)[ray] = make_float4(-gd[0] / gn, -gd[1] / gn, -gd[2] / gn, t0 + ss);
    }
}

}  // namespace

hipError_t launch_surface_points(const SurfaceArgs& a, hipStream_t stream) {
    if (a.n_rays == 0) return hipSuccess;
    if (a.n_samples < 2 || a.n_samples > kMaxSamples) return hipErrorInvalidValue;
    if (a.n > 0) hipLaunchKernelGGL(k_surface_frames, dim3((a.n + 255) / 256), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_surface_points, dim3((a.n_rays + kRaysPerWave - 1) / kRaysPerWave), dim3(64), 0, stream,
                       a);
    return hipGetLastError();
}

}  // namespace gesr
