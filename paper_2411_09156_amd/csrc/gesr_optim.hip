// Fused optimiser step of the training schedule (Sec. 4.2): Adam on the raw
// parameters (mean, log scale, quaternion, opacity logit, beta, SH) with one
// learning rate per group, the chain rule from the activated parameters the
// renderer differentiates (scale = exp(log scale), opacity = sigmoid(logit)),
// the opacity-entropy term, and the activated scale and opacity written for
// the next forward.  One pass over every parameter element: HBM-bound.

#include "gesr_device.h"
#include "gesr_kernels.h"

namespace gesr {

namespace {

__global__ __launch_bounds__(256) void k_adam_step(AdamArgs a) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
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
    const float pk = p[k];
    float gk = g[k];
    if (kind == 1) {
        gk *= expf(pk);  // d scale / d log scale
    } else if (kind == 2) {
        // o (1 - o) = e / (1 + e)^2 with e = exp(-|logit|): no cancellation in 1 - o
        const float e = expf(-fabsf(pk));
        const float r = 1.0f / (1.0f + e);
        const float dodl = e * r * r;
        // entropy_weight * mean H(o): dH/dlogit = -logit o (1 - o)
        gk = fmaf(gk, dodl, a.entropy_scale * (-pk) * dodl);
    }
    const float mk = fmaf(a.beta1, m[k], (1.0f - a.beta1) * gk);
    const float vk = fmaf(a.beta2, v[k], (1.0f - a.beta2) * gk * gk);
    const float pn = pk - lr * (mk * a.inv_c1) / (sqrtf(vk * a.inv_c2) + a.eps);
    p[k] = pn;
    m[k] = mk;
    v[k] = vk;
    if (kind == 1) a.scale_out[k] = expf(pn);
    else if (kind == 2) a.opacity_out[i] = 1.0f / (1.0f + expf(-pn));
}

}  // namespace

hipError_t launch_adam_step(const AdamArgs& a, int rows, hipStream_t stream) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam_step, dim3((unsigned)((a.n + 255) / 256), (unsigned)rows), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace gesr
