// Fused optimiser step of the training schedule (Sec. 4.2): Adam on the raw
// parameters (mean, log scale, quaternion, opacity logit, beta, SH) with one
// learning rate per group, the chain rule from the activated parameters the
// renderer differentiates (scale = exp(log scale), opacity = sigmoid(logit)),
// the opacity-entropy term, and the activated scale and opacity written for
// the next forward.  One pass over every parameter element: HBM-bound.

#include <type_traits>

#include "gesr_device.h"
#include "gesr_kernels.h"

namespace gesr {

namespace {

struct Vec1 {
    float x[1];
};
struct Vec4 {
    float x[4];
};
template <int VEC>
using VecT = typename std::conditional<VEC == 4, Vec4, Vec1>::type;

template <int VEC>
__device__ __forceinline__ VecT<VEC> ld(const float* p) {
    VecT<VEC> r;
    if constexpr (VEC == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        r.x[0] = q.x; r.x[1] = q.y; r.x[2] = q.z; r.x[3] = q.w;
    } else {
        r.x[0] = *p;
    }
    return r;
}

template <int VEC>
__device__ __forceinline__ void st(float* p, const VecT<VEC>& r) {
    if constexpr (VEC == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(r.x[0], r.x[1], r.x[2], r.x[3]);
    } else {
        *p = r.x[0];
    }
}

// One thread updates VEC consecutive elements of one parameter row (VEC = 4
// needs n % 4 == 0 so that every row starts 16-byte aligned).
template <int VEC>
__global__ __launch_bounds__(256) void k_adam_step(AdamArgs a) {
    const uint32_t i = (blockIdx.x * 256u + threadIdx.x) * VEC;
    const uint32_t row = blockIdx.y;
    if (i >= (uint32_t)a.n) return;
    const size_t n = (size_t)a.n;
    // parameter group of this row: mean 0-2, log scale 3-5, quaternion 6-9,
    // logit 10, beta 11, SH 12.. (DC 12-14)
    float *p, *m, *v;
    const float* g;
    float lr;
    int kind = 0;  // 1: log scale, 2: logit
    size_t off;
    if (row < 3) {
        off = row * n; p = a.p.mean; m = a.m.mean; v = a.v.mean; g = a.g_mean; lr = a.lr_mean;
    } else if (row < 6) {
        off = (row - 3) * n; p = a.p.log_scale; m = a.m.log_scale; v = a.v.log_scale; g = a.g_scale;
        lr = a.lr_scale; kind = 1;
    } else if (row < 10) {
        off = (row - 6) * n; p = a.p.quat; m = a.m.quat; v = a.v.quat; g = a.g_quat; lr = a.lr_quat;
    } else if (row == 10) {
        off = 0; p = a.p.opacity_logit; m = a.m.opacity_logit; v = a.v.opacity_logit; g = a.g_opacity;
        lr = a.lr_opacity; kind = 2;
    } else if (row == 11) {
        off = 0; p = a.p.beta; m = a.m.beta; v = a.v.beta; g = a.g_beta; lr = a.lr_beta;
    } else {
        off = (row - 12) * n; p = a.p.sh; m = a.m.sh; v = a.v.sh; g = a.g_sh;
        lr = row < 15 ? a.lr_sh_dc : a.lr_sh_rest;
    }
    const size_t k = off + i;
    VecT<VEC> pk = ld<VEC>(p + k), gk = ld<VEC>(g + k), mk = ld<VEC>(m + k), vk = ld<VEC>(v + k), act;
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        const float x = pk.x[j];
        float gj = gk.x[j];
        if (kind == 1) {
            gj *= expf(x);  // d scale / d log scale
        } else if (kind == 2) {
            // o (1 - o) = e / (1 + e)^2 with e = exp(-|logit|): no cancellation in 1 - o
            const float e = expf(-fabsf(x));
            const float r = 1.0f / (1.0f + e);
            const float dodl = e * r * r;
            // entropy_weight * mean H(o): dH/dlogit = -logit o (1 - o)
            gj = fmaf(gj, dodl, a.entropy_scale * (-x) * dodl);
        }
        const float mj = fmaf(a.beta1, mk.x[j], (1.0f - a.beta1) * gj);
        const float vj = fmaf(a.beta2, vk.x[j], (1.0f - a.beta2) * gj * gj);
        const float pn = x - lr * (mj * a.inv_c1) / (sqrtf(vj * a.inv_c2) + a.eps);
        pk.x[j] = pn;
        mk.x[j] = mj;
        vk.x[j] = vj;
        act.x[j] = kind == 1 ? expf(pn) : 1.0f / (1.0f + expf(-pn));
    }
    st<VEC>(p + k, pk);
    st<VEC>(m + k, mk);
    st<VEC>(v + k, vk);
    if (kind == 1) st<VEC>(a.scale_out + k, act);
    else if (kind == 2) st<VEC>(a.opacity_out + i, act);
}

// ---------------------------------------------------------------- pruning
// Flags of PRUNE_BLOCK splats per block: one bit per splat (keep), and the
// block's count of kept splats.  Lane l of wave w evaluates splats
// base + j * 256 + w * 64 + l, so one ballot gives two consecutive words.
__global__ __launch_bounds__(256) void k_prune_flags(PruneArgs a) {
    const uint32_t b = blockIdx.x;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    __shared__ uint32_t s_cnt[16];
    for (int j = 0; j < 4; ++j) {
        const uint32_t i = b * PRUNE_BLOCK + j * 256u + wave * 64u + lane;
        bool keep = false;
        if (i < (uint32_t)a.n) keep = a.logit[i] >= a.t_logit && a.beta[i] >= a.min_beta;
        const uint64_t bal = __ballot(keep);
        const uint32_t word = (b * PRUNE_BLOCK + j * 256u + wave * 64u) >> 5;
        if (lane == 0) {
            a.bits[word] = (uint32_t)bal;
            a.bits[word + 1] = (uint32_t)(bal >> 32);
            s_cnt[j * 4 + wave] = (uint32_t)__popcll(bal);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0;
        for (int k = 0; k < 16; ++k) c += s_cnt[k];
        a.counts[b] = c;
    }
}

// Stable compaction of one parameter row (blockIdx.y) for PRUNE_BLOCK splats:
// kept splat i goes to column offsets[b] + (kept splats before it in the
// block); rows are packed with stride n_kept (read from the device).
__global__ __launch_bounds__(256) void k_prune_scatter(PruneArgs a) {
    const uint32_t b = blockIdx.x;
    const uint32_t row = blockIdx.y;
    __shared__ uint32_t s_bits[32], s_pre[32];
    if (threadIdx.x < 32) s_bits[threadIdx.x] = a.bits[b * 32u + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0;
        for (int k = 0; k < 32; ++k) {
            s_pre[k] = c;
            c += (uint32_t)__popc(s_bits[k]);
        }
    }
    __syncthreads();
    const size_t n = (size_t)a.n;
    const size_t nk = (size_t)*a.n_kept;
    const uint32_t base = a.offsets[b];
    // row -> (array, row within it) in the order of the Adam step
    int arr, rr;
    if (row < 3) { arr = 0; rr = row; }
    else if (row < 6) { arr = 1; rr = row - 3; }
    else if (row < 10) { arr = 2; rr = row - 6; }
    else if (row == 10) { arr = 3; rr = 0; }
    else if (row == 11) { arr = 4; rr = 0; }
    else { arr = 5; rr = row - 12; }
    const bool with_moments = a.in_m[0] != nullptr;
    for (int j = 0; j < 4; ++j) {
        const uint32_t loc = j * 256u + threadIdx.x;
        const uint32_t i = b * PRUNE_BLOCK + loc;
        if (i >= (uint32_t)a.n) break;
        const uint32_t w = s_bits[loc >> 5];
        if (!((w >> (loc & 31u)) & 1u)) continue;
        const size_t dst = (size_t)base + s_pre[loc >> 5] + (uint32_t)__popc(w & ((1u << (loc & 31u)) - 1u));
        const size_t src = (size_t)rr * n + i, dsto = (size_t)rr * nk + dst;
        const float x = a.in_p[arr][src];
        a.out_p[arr][dsto] = x;
        if (with_moments) {
            a.out_m[arr][dsto] = a.in_m[arr][src];
            a.out_v[arr][dsto] = a.in_v[arr][src];
        }
        if (arr == 1 && a.scale_out) a.scale_out[dsto] = expf(x);
        if (arr == 3 && a.opacity_out) a.opacity_out[dst] = 1.0f / (1.0f + expf(-x));
    }
}

__global__ __launch_bounds__(256) void k_shape_reset(float* beta, float* m, float* v, int n, float value) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= (uint32_t)n) return;
    beta[i] = value;
    if (m) m[i] = 0.0f;
    if (v) v[i] = 0.0f;
}

}  // namespace

uint32_t prune_blocks(int n) { return (uint32_t)(((uint64_t)n + PRUNE_BLOCK - 1) / PRUNE_BLOCK); }

size_t prune_workspace_bytes(int n) {
    const uint64_t nb = prune_blocks(n);
    const uint64_t partials = (nb + SCAN_TILE - 1) / SCAN_TILE;
    // bits (32 words per block), counts, offsets, scan partials, kept total
    return (size_t)(4 * (nb * 32 + 2 * nb + partials + 1) + 16);
}

hipError_t launch_prune(PruneArgs a, int rows, uint32_t* partials, hipStream_t stream) {
    const uint32_t nb = prune_blocks(a.n);
    if (nb == 0) {
        return launch_fill_u32(a.n_kept, 0u, 1, stream);
    }
    hipLaunchKernelGGL(k_prune_flags, dim3(nb), dim3(256), 0, stream, a);
    hipError_t e = scan_exclusive(a.counts, a.offsets, nb, partials, a.n_kept, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prune_scatter, dim3(nb, (unsigned)rows), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_shape_reset(float* beta, float* m, float* v, int n, float value, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shape_reset, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, beta, m, v, n, value);
    return hipGetLastError();
}

hipError_t launch_adam_step(const AdamArgs& a, int rows, hipStream_t stream) {
    if (a.n == 0) return hipSuccess;
    if (a.n % 4 == 0) {
        const unsigned quads = (unsigned)(a.n / 4);
        hipLaunchKernelGGL(k_adam_step<4>, dim3((quads + 255) / 256, (unsigned)rows), dim3(256), 0, stream, a);
    } else {
        hipLaunchKernelGGL(k_adam_step<1>, dim3((unsigned)((a.n + 255) / 256), (unsigned)rows), dim3(256), 0,
                           stream, a);
    }
    return hipGetLastError();
}

}  // namespace gesr
