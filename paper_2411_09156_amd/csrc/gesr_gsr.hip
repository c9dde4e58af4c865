// Surface regulariser of Sec. 3.3 (Eq. 9-13) with the nearest-neighbour
// density of the training schedule (Sec. 4.2: 16 neighbours, lists refreshed
// periodically).
//
// Neighbour lists (knn[j][0] = j, then the k - 1 nearest other centres by
// squared distance, ties by index) come from a uniform grid over the centres'
// bounding box: the centres are radix-sorted by the Morton code of their
// cell, and each query (one
// thread, in cell order so that a wave's queries share cells) scans shells of
// cells around its own until the (k-1)-th distance is below the distance to
// any unscanned cell.  The cell order is kept: the regulariser runs its
// samples in it.  The inverse lists (for every splat, the entries p * k + s,
// p a position in the cell order, that name it) are a stable sort of the
// entries by neighbour.
//
// The loss runs one sample per splat: x_j = mu_j + R_j diag(phi s_j) xi_j.
// Pass 1 over the neighbours sums the terms o exp(-kappa q^(beta/2)) of Eq. 9
// and their gradient in x and picks g* (largest term); then the SDF terms of
// Eq. 10-13 and their adjoints (with respect to d, grad d and the g* frame).
// Pass 2 revisits the neighbours, takes every term's derivative with respect
// to its own splat and to x, adds the g* terms and, last, the dependence of x
// on the sampled splat, and writes one 12-float partial per (sample, slot) to
// that entry's position in the inverse lists.  A gather then adds each
// splat's contiguous records, in entry order, into the gradients:
// deterministic, no atomics.

#include <math.h>

#include <algorithm>

#include "gesr_device.h"
#include "gesr_kernels.h"

namespace gesr {

namespace {

constexpr float kGsrFloor = 1e-30f;

// ---------------------------------------------------------------- grid
// Per-block min / max of the centres.
__global__ __launch_bounds__(256) void k_knn_bounds(const float* mean, int n, float* part) {
    __shared__ float s[6][256];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < (uint32_t)n; i += gridDim.x * 256u)
        for (int a = 0; a < 3; ++a) {
            const float v = mean[(size_t)a * n + i];
            lo[a] = fminf(lo[a], v);
            hi[a] = fmaxf(hi[a], v);
        }
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w)
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + w]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// Grid over the box: cubic cells of side cs, about two centres per cell of
// the box's volume, at most 256 cells per axis and `cell_cap` cells in all.
__global__ void k_knn_grid(const float* part, int nparts, int n, uint32_t cell_cap, KnnGrid* g) {
    if (threadIdx.x != 0) return;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nparts; ++b)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], part[b * 6 + a]);
            hi[a] = fmaxf(hi[a], part[b * 6 + 3 + a]);
        }
    float ext[3], emax = 0.f;
    for (int a = 0; a < 3; ++a) {
        ext[a] = fmaxf(hi[a] - lo[a], 0.f);
        emax = fmaxf(emax, ext[a]);
    }
    if (!(emax > 0.f)) emax = 1.f;
    const float floor_e = emax / 256.f;
    float vol = 1.f;
    for (int a = 0; a < 3; ++a) vol *= fmaxf(ext[a], floor_e);
    float cs = fmaxf(cbrtf(vol / fmaxf(0.5f * (float)n, 1.f)), floor_e);
    int G[3];
    for (int it = 0; it < 64; ++it) {
        uint64_t total = 1;
        for (int a = 0; a < 3; ++a) {
            G[a] = (int)fminf(fmaxf(ceilf(ext[a] / cs), 1.f), 256.f);
            total *= (uint64_t)G[a];
        }
        if (total <= cell_cap) break;
        cs *= 1.25f;
    }
    for (int a = 0; a < 3; ++a) {
        g->lo[a] = lo[a];
        g->dim[a] = G[a];
    }
    g->cs = cs;
    g->inv_cs = 1.f / cs;
}

__device__ __forceinline__ int cell_coord(float v, float lo, float inv_cs, int G) {
    const int c = (int)floorf((v - lo) * inv_cs);
    return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

// Morton (Z-order) code of a cell, 8 bits per axis: cells close in space
// are close in the sort order, which the regulariser's gathers rely on.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0xFFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0xFFu;
    return v;
}

__global__ __launch_bounds__(256) void k_knn_cells(const float* mean, int n, const KnnGrid* g, uint32_t* keys) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= (uint32_t)n) return;
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = cell_coord(mean[(size_t)a * n + i], g->lo[a], g->inv_cs, g->dim[a]);
    keys[i] = spread3((uint32_t)c[0]) | (spread3((uint32_t)c[1]) << 1) | (spread3((uint32_t)c[2]) << 2);
}

// [start, end) of every cell (indexed x + X (y + Y z)) in the Morton-sorted
// order (cells start empty).
__global__ __launch_bounds__(256) void k_knn_ranges(const uint32_t* keys, int n, const KnnGrid* g, uint32_t* start,
                                                    uint32_t* end) {
    const uint32_t p = blockIdx.x * 256u + threadIdx.x;
    if (p >= (uint32_t)n) return;
    const uint32_t m = keys[p];
    const uint32_t c = compact3(m) + (uint32_t)g->dim[0] * (compact3(m >> 1) + (uint32_t)g->dim[1] * compact3(m >> 2));
    if (p == 0 || keys[p - 1] != m) start[c] = p;
    if (p + 1 == (uint32_t)n || keys[p + 1] != m) end[c] = p + 1;
}

// Centres in the sorted order, (x, y, z, index bits): a cell's centres are
// one contiguous run of 16-byte records.
__global__ __launch_bounds__(256) void k_knn_sorted_pos(const float* mean, int n, const uint32_t* order,
                                                        float4* pos) {
    const uint32_t p = blockIdx.x * 256u + threadIdx.x;
    if (p >= (uint32_t)n) return;
    const uint32_t i = order[p];
    pos[p] = make_float4(mean[i], mean[(size_t)n + i], mean[2 * (size_t)n + i], __uint_as_float(i));
}

// Scans one cell's centres into the sorted candidate list (d2, index) of
// WANT entries.
template <int WANT>
__device__ __forceinline__ void scan_cell(uint32_t c, const uint32_t* start, const uint32_t* end,
                                          const float4* pos, uint32_t self, float px, float py, float pz, float* bd,
                                          uint32_t* bi, int& have) {
    const uint32_t e = end[c];
    for (uint32_t q = start[c]; q < e; ++q) {
        const float4 v = pos[q];
        const uint32_t j = __float_as_uint(v.w);
        if (j == self) continue;
        const float dx = v.x - px, dy = v.y - py, dz = v.z - pz;
        const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        if (d2 > bd[WANT - 1] || (d2 == bd[WANT - 1] && j >= bi[WANT - 1])) continue;
        // insert (d2, j), shifting the larger entries up
        float cd = d2;
        uint32_t ci = j;
#pragma unroll
        for (int s = 0; s < WANT; ++s) {
            const bool less = cd < bd[s] || (cd == bd[s] && ci < bi[s]);
            const float td = bd[s];
            const uint32_t ti = bi[s];
            bd[s] = less ? cd : bd[s];
            bi[s] = less ? ci : bi[s];
            cd = less ? td : cd;
            ci = less ? ti : ci;
        }
        have = min(have + 1, WANT);
    }
}

// One query per thread, in cell order.  bd/bi hold the K - 1 nearest others
// sorted by (distance^2, index).
template <int K>
__global__ __launch_bounds__(256) void k_knn_query(const float4* pos, int n, const KnnGrid* gp,
                                                   const uint32_t* start, const uint32_t* end, uint32_t* knn) {
    const uint32_t p = blockIdx.x * 256u + threadIdx.x;
    if (p >= (uint32_t)n) return;
    const KnnGrid g = *gp;
    const float4 me = pos[p];
    const uint32_t i = __float_as_uint(me.w);
    const float px = me.x, py = me.y, pz = me.z;
    const int cx = cell_coord(px, g.lo[0], g.inv_cs, g.dim[0]);
    const int cy = cell_coord(py, g.lo[1], g.inv_cs, g.dim[1]);
    const int cz = cell_coord(pz, g.lo[2], g.inv_cs, g.dim[2]);
    constexpr int want = K - 1;
    float bd[want];
    uint32_t bi[want];
#pragma unroll
    for (int s = 0; s < want; ++s) {
        bd[s] = INFINITY;
        bi[s] = 0xFFFFFFFFu;
    }
    int have = 0;
    const int rmax = max(g.dim[0], max(g.dim[1], g.dim[2]));
    for (int r = 0; r <= rmax; ++r) {
        const int z0 = max(cz - r, 0), z1 = min(cz + r, g.dim[2] - 1);
        const int y0 = max(cy - r, 0), y1 = min(cy + r, g.dim[1] - 1);
        const int x0 = max(cx - r, 0), x1 = min(cx + r, g.dim[0] - 1);
        for (int z = z0; z <= z1; ++z)
            for (int y = y0; y <= y1; ++y) {
                const uint32_t row = (uint32_t)g.dim[0] * ((uint32_t)y + (uint32_t)g.dim[1] * (uint32_t)z);
                if (r == 0 || abs(z - cz) == r || abs(y - cy) == r) {
                    for (int x = x0; x <= x1; ++x)
                        scan_cell<want>(row + (uint32_t)x, start, end, pos, i, px, py, pz, bd, bi, have);
                } else {  // inner rows of the shell: its two end cells
                    if (cx - r >= 0)
                        scan_cell<want>(row + (uint32_t)(cx - r), start, end, pos, i, px, py, pz, bd, bi, have);
                    if (cx + r < g.dim[0])
                        scan_cell<want>(row + (uint32_t)(cx + r), start, end, pos, i, px, py, pz, bd, bi, have);
                }
            }
        // every unscanned centre lies outside the cube of cells within r
        float bound = INFINITY;
        if (cx - r > 0) bound = fminf(bound, px - (g.lo[0] + (float)(cx - r) * g.cs));
        if (cx + r < g.dim[0] - 1) bound = fminf(bound, g.lo[0] + (float)(cx + r + 1) * g.cs - px);
        if (cy - r > 0) bound = fminf(bound, py - (g.lo[1] + (float)(cy - r) * g.cs));
        if (cy + r < g.dim[1] - 1) bound = fminf(bound, g.lo[1] + (float)(cy + r + 1) * g.cs - py);
        if (cz - r > 0) bound = fminf(bound, pz - (g.lo[2] + (float)(cz - r) * g.cs));
        if (cz + r < g.dim[2] - 1) bound = fminf(bound, g.lo[2] + (float)(cz + r + 1) * g.cs - pz);
        if (bound == INFINITY) break;  // the whole grid is scanned
        // a centre's cell comes from a rounded (v - lo) / cs: keep a margin
        bound = fmaxf(bound - 1e-4f * g.cs, 0.f);
        if (have == want && bd[want - 1] < bound * bound) break;
    }
    uint32_t* out = knn + (size_t)i * K;
    out[0] = i;
#pragma unroll
    for (int s = 0; s < want; ++s) out[1 + s] = s < have ? bi[s] : 0xFFFFFFFFu;
}

// k = 1: the list is the splat itself.
__global__ __launch_bounds__(256) void k_knn_self(int n, uint32_t* knn) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < (uint32_t)n) knn[i] = i;
}

// Inverse-list keys in sample (cell) order: entry e = p * k + s is slot s of
// the list of splat order[p]; its key is the neighbour it names, n for padding.
__global__ __launch_bounds__(256) void k_inv_keys(const uint32_t* knn, const uint32_t* order, uint64_t total,
                                                  uint32_t k, uint32_t n, uint32_t* keys) {
    const uint64_t e = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (e >= total) return;
    const uint32_t e32 = (uint32_t)e;  // n * k < 2^32
    const uint32_t p = e32 / k, s = e32 - p * k;
    const uint32_t v = knn[(size_t)order[p] * k + s];
    keys[e] = v < n ? v : n;
}

__global__ __launch_bounds__(256) void k_inv_offsets(const uint32_t* keys, uint64_t total, uint32_t n,
                                                     uint32_t* offsets) {
    const uint64_t p = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (p > total) return;
    const uint32_t c = p < total ? keys[p] : n + 1;
    const uint32_t prev = p > 0 ? keys[p - 1] : 0xFFFFFFFFu;
    if (p == 0 || prev != c) {
        // every splat names itself, so consecutive keys differ by at most one
        // below n; offsets[n] marks the end of the valid entries
        const uint32_t from = p == 0 ? 0u : prev + 1;
        for (uint32_t id = from; id <= c && id <= n; ++id) offsets[id] = (uint32_t)p;
    }
}

// Position of every valid entry in the inverse order: the regulariser writes
// the partial of entry e to record inv_slot[e], so that each splat's records
// are contiguous for the gather.
__global__ __launch_bounds__(256) void k_inv_slots(const uint32_t* inv_entries, const uint32_t* inv_offsets,
                                                   uint32_t n, uint32_t* inv_slot) {
    const uint32_t pos = blockIdx.x * 256u + threadIdx.x;
    if (pos >= inv_offsets[n]) return;
    inv_slot[inv_entries[pos]] = pos;
}

// ---------------------------------------------------------------- loss
// Per-splat frame, one 64-byte record: normalised quaternion (4), mu (3),
// opacity, 1 / sigma (3) with sigma = phi s, beta, sigma (3), 1 / |q|.  The
// rotation, phi, 1 / beta and 1 / o are rebuilt from it where they are used,
// which halves the frames the regulariser gathers per neighbour.
struct GFrame {
    float R[9], sig[3], mu[3], o, beta, phi, qn[4], inv_q, isig[3], ibeta, io;
};

__global__ __launch_bounds__(256) void k_gsr_frames(GsrArgs a) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= (uint32_t)a.n) return;
    const size_t n = (size_t)a.n;
    float q[4];
    for (int c = 0; c < 4; ++c) q[c] = a.quat[c * n + i];
    const float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const float inv = 1.0f / sqrtf(qq);
    const float beta = a.beta[i];
    const float phi = 2.0f / (1.0f + expf(-a.rho * (beta - 2.0f)));
    float f[GSR_FRAME_FLOATS];
    for (int c = 0; c < 4; ++c) f[c] = q[c] * inv;
    for (int c = 0; c < 3; ++c) {
        f[4 + c] = a.mean[c * n + i];
        const float sg = phi * a.scale[c * n + i];
        f[8 + c] = 1.0f / sg;
        f[12 + c] = sg;
    }
    f[7] = a.opacity[i];
    f[11] = beta;
    f[15] = inv;
    float4* dst = reinterpret_cast<float4*>(a.frames + (size_t)i * GSR_FRAME_FLOATS);
    for (int c = 0; c < GSR_FRAME_FLOATS / 4; ++c)
        dst[c] = make_float4(f[4 * c], f[4 * c + 1], f[4 * c + 2], f[4 * c + 3]);
}

__device__ __forceinline__ GFrame load_gframe(const float* frames, uint32_t i, float rho) {
    const float4* s = reinterpret_cast<const float4*>(frames + (size_t)i * GSR_FRAME_FLOATS);
    float f[GSR_FRAME_FLOATS];
#pragma unroll
    for (int c = 0; c < GSR_FRAME_FLOATS / 4; ++c) {
        const float4 v = s[c];
        f[4 * c] = v.x; f[4 * c + 1] = v.y; f[4 * c + 2] = v.z; f[4 * c + 3] = v.w;
    }
    GFrame g;
    const float w = f[0], x = f[1], y = f[2], z = f[3];
    g.R[0] = 1.f - 2.f * (y * y + z * z); g.R[1] = 2.f * (x * y - w * z); g.R[2] = 2.f * (x * z + w * y);
    g.R[3] = 2.f * (x * y + w * z); g.R[4] = 1.f - 2.f * (x * x + z * z); g.R[5] = 2.f * (y * z - w * x);
    g.R[6] = 2.f * (x * z - w * y); g.R[7] = 2.f * (y * z + w * x); g.R[8] = 1.f - 2.f * (x * x + y * y);
#pragma unroll
    for (int c = 0; c < 4; ++c) g.qn[c] = f[c];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        g.mu[c] = f[4 + c];
        g.isig[c] = f[8 + c];
        g.sig[c] = f[12 + c];
    }
    g.o = f[7];
    g.beta = f[11];
    g.inv_q = f[15];
    g.phi = 2.0f / (1.0f + expf(-rho * (g.beta - 2.0f)));
    g.ibeta = __builtin_amdgcn_rcpf(g.beta);
    g.io = g.o > 0.f ? __builtin_amdgcn_rcpf(g.o) : 0.f;
    return g;
}

// One Eq. 9 term at x: the Mahalanobis vector a = diag(1/sig) R^T (x - mu),
// q = |a|^2, T = o exp(-kappa q^(beta/2)), c = dT/dq * 2 = -kappa beta q^(beta/2-1) T.
struct Term {
    float dx[3], a[3], q, iq, P, T, c, lq;
};

// x - mu is formed as (mu_0 - mu) + M_0 xi: rounding x itself to float32
// would cost a flat splat's thickness direction up to ulp(|mu|) / s_min.
__device__ __forceinline__ Term eval_term(const GFrame& f, const float mu0[3], const float d0[3], float kappa) {
    Term t;
    for (int c = 0; c < 3; ++c) t.dx[c] = (mu0[c] - f.mu[c]) + d0[c];
    for (int k = 0; k < 3; ++k)
        t.a[k] = (f.R[k] * t.dx[0] + f.R[3 + k] * t.dx[1] + f.R[6 + k] * t.dx[2]) * f.isig[k];
    t.q = t.a[0] * t.a[0] + t.a[1] * t.a[1] + t.a[2] * t.a[2];
    if (t.q > 0.f) {
        t.iq = __builtin_amdgcn_rcpf(t.q);
        t.lq = logf(t.q);
        t.P = expf(0.5f * f.beta * t.lq);
        t.T = f.o * expf(-kappa * t.P);
        t.c = -kappa * f.beta * t.P * t.iq * t.T;
    } else {
        t.iq = 0.f;
        t.lq = 0.f;
        t.P = 0.f;
        t.T = f.o;
        t.c = 0.f;
    }
    return t;
}

// d/dq of the normalised quaternion's rotation: G = dL/dR (row-major), returns
// dL/dq for the raw quaternion (through q / |q|).
__device__ __forceinline__ void rot_adjoint(const GFrame& f, const float G[9], float out[4]) {
    const float w = f.qn[0], x = f.qn[1], y = f.qn[2], z = f.qn[3];
    float g[4];
    g[0] = 2.f * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
    g[1] = 2.f * (y * G[1] + z * G[2] + y * G[3] - 2.f * x * G[4] - w * G[5] + z * G[6] + w * G[7] - 2.f * x * G[8]);
    g[2] = 2.f * (-2.f * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] - 2.f * y * G[8]);
    g[3] = 2.f * (-2.f * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.f * z * G[4] + y * G[5] + x * G[6] + y * G[7]);
    const float dot = g[0] * w + g[1] * x + g[2] * y + g[3] * z;
    out[0] = (g[0] - w * dot) * f.inv_q;
    out[1] = (g[1] - x * dot) * f.inv_q;
    out[2] = (g[2] - y * dot) * f.inv_q;
    out[3] = (g[3] - z * dot) * f.inv_q;
}

// Workgroups are dealt to the eight XCDs round robin; renumber them so that
// each XCD (with its own L2) takes one contiguous range of the work.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblocks) {
    const uint32_t per = (nblocks + 7u) / 8u;
    const uint32_t xcd = b % 8u, slot = b / 8u;
    const uint32_t full = nblocks % 8u == 0 ? 8u : nblocks % 8u;  // XCDs that get `per` blocks
    const uint32_t base = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1u);
    return base + slot;
}

// Samples run in the cell order of the neighbour lists, so that the
// neighbours a wave (and an XCD's L2) gathers overlap; partials are stored at
// the sample's position in that order (the inverse lists refer to these
// positions).  A sample's list is staged in LDS.
__global__ __launch_bounds__(128) void k_gsr_loss(GsrArgs a) {
    __shared__ uint32_t s_nb[GESR_KNN_MAX][128];
    __shared__ uint32_t s_slot[GESR_KNN_MAX][128];
    const uint32_t p = xcd_block(blockIdx.x, gridDim.x) * 128u + threadIdx.x;
    if (p >= (uint32_t)a.n) return;
    const uint32_t j = a.order[p];
    const int K = a.k;
    {
        const uint32_t* row = a.knn + (size_t)j * K;
        for (int s = 0; s < K; ++s) s_nb[s][threadIdx.x] = row[s];
        if (a.partials) {
            const uint32_t* srow = a.inv_slot + (size_t)p * K;
            for (int s = 0; s < K; ++s) s_slot[s][threadIdx.x] = srow[s];
        }
    }
    // each thread reads back only its own column: no barrier needed
    const uint32_t* nbl = &s_nb[0][threadIdx.x];
    const uint32_t* sll = &s_slot[0][threadIdx.x];
#define nb_at(s) nbl[(s) * 128]
    // the partial of slot s goes to record inv_slot[p * k + s]: each splat's
    // records end up contiguous, in inverse-list order
#define rec_at(s) (a.partials + (size_t)sll[(s) * 128] * GSR_PARTIAL_STRIDE)
    const bool with_part = a.partials != nullptr;
    const bool on = a.mask == nullptr || a.mask[j] != 0;
    if (!on) {
        if (with_part)
            for (int s = 0; s < K; ++s) {
                if (nb_at(s) >= (uint32_t)a.n) continue;  // padding slots have no record
                for (int c = 0; c < GSR_PARTIAL_STRIDE / 4; ++c)
                    reinterpret_cast<float4*>(rec_at(s))[c] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        a.sample_out[(size_t)j * 4 + 0] = 0.f;
        a.sample_out[(size_t)j * 4 + 1] = 0.f;
        a.sample_out[(size_t)j * 4 + 2] = -1.f;
        a.sample_out[(size_t)j * 4 + 3] = 0.f;
        return;
    }
    const float kappa = a.kappa;
    const GFrame f0 = load_gframe(a.frames, j, a.rho);
    float xi[3];
    for (int c = 0; c < 3; ++c) xi[c] = a.xi[(size_t)c * a.n + j];
    // the sample x = mu_0 + d0, d0 = R_0 diag(sig_0) xi, kept as the pair
    float d0[3];
    for (int r = 0; r < 3; ++r)
        d0[r] = f0.R[3 * r] * (f0.sig[0] * xi[0]) + f0.R[3 * r + 1] * (f0.sig[1] * xi[1]) +
                f0.R[3 * r + 2] * (f0.sig[2] * xi[2]);
    // pass 1: d, grad d, g*
    float d = 0.f, gd[3] = {0.f, 0.f, 0.f}, best = -1.f;
    int gs = 0;
    // the next neighbour's frame is loaded while this one is evaluated
    // (padding slots, n < k, load slot 0's frame and are skipped)
    GFrame fn = load_gframe(a.frames, j, a.rho);
    for (int s = 0; s < K; ++s) {
        const uint32_t i = nb_at(s);
        const GFrame f = fn;
        if (s + 1 < K) {
            const uint32_t i1 = nb_at(s + 1);
            fn = load_gframe(a.frames, i1 < (uint32_t)a.n ? i1 : j, a.rho);
        }
        if (i >= (uint32_t)a.n) continue;
        const Term t = eval_term(f, f0.mu, d0, kappa);
        d += t.T;
        const float as[3] = {t.a[0] * f.isig[0], t.a[1] * f.isig[1], t.a[2] * f.isig[2]};
        for (int r = 0; r < 3; ++r) gd[r] += t.c * (f.R[3 * r] * as[0] + f.R[3 * r + 1] * as[1] + f.R[3 * r + 2] * as[2]);
        if (t.T > best) {
            best = t.T;
            gs = s;
        }
    }
    // SDF terms of g* (Eq. 10-13)
    const GFrame fg = load_gframe(a.frames, nb_at(gs), a.rho);
    int ks = 0;
    if (fg.sig[1] < fg.sig[ks]) ks = 1;
    if (fg.sig[2] < fg.sig[ks]) ks = 2;
    // selects rather than a run-time index keep the frame in registers
    const float nrm[3] = {ks == 0 ? fg.R[0] : (ks == 1 ? fg.R[1] : fg.R[2]),
                          ks == 0 ? fg.R[3] : (ks == 1 ? fg.R[4] : fg.R[5]),
                          ks == 0 ? fg.R[6] : (ks == 1 ? fg.R[7] : fg.R[8])};
    const float smin = ks == 0 ? fg.sig[0] : (ks == 1 ? fg.sig[1] : fg.sig[2]);
    float xm[3];
    for (int c = 0; c < 3; ++c) xm[c] = (f0.mu[c] - fg.mu[c]) + d0[c];
    const float h = xm[0] * nrm[0] + xm[1] * nrm[1] + xm[2] * nrm[2];
    const float sg = h >= 0.f ? 1.f : -1.f;
    const float r = fabsf(h) / smin;
    const float lr = r > 0.f ? logf(r) : 0.f;
    const float A = r > 0.f ? expf(0.5f * fg.beta * lr) : 0.f;
    const bool floored = !(d > kGsrFloor);
    const float Ld = floored ? -logf(kGsrFloor) : -logf(d);
    const float B = Ld > 0.f ? sqrtf(Ld / kappa) : 0.f;
    const float diff = A - B;
    const float l_sdf = smin * fabsf(diff);
    // |grad d| scaled by its largest component, so that small densities do
    // not underflow the squares; the normal term needs d and |grad d| above
    // the floor
    const float gmax = fmaxf(fabsf(gd[0]), fmaxf(fabsf(gd[1]), fabsf(gd[2])));
    float l_nor = 0.f, gh[3] = {0.f, 0.f, 0.f}, gn_s = 0.f, inv_gmax = 0.f;
    bool with_nor = false;
    if (!floored && gmax > 0.f) {
        inv_gmax = 1.f / gmax;
        float gs3[3];
        for (int c = 0; c < 3; ++c) gs3[c] = gd[c] * inv_gmax;
        gn_s = sqrtf(gs3[0] * gs3[0] + gs3[1] * gs3[1] + gs3[2] * gs3[2]);
        with_nor = gmax * gn_s > kGsrFloor;
        if (with_nor)
            for (int c = 0; c < 3; ++c) {
                gh[c] = gs3[c] / gn_s;
                const float e = -sg * gh[c] - nrm[c];
                l_nor += e * e;
            }
    }
    a.sample_out[(size_t)j * 4 + 0] = l_sdf;
    a.sample_out[(size_t)j * 4 + 1] = l_nor;
    a.sample_out[(size_t)j * 4 + 2] = (float)gs;
    a.sample_out[(size_t)j * 4 + 3] = d;
    if (!with_part) return;

    // adjoints of the sample's loss w_sdf l_sdf + w_nor l_nor
    const float ws = a.w_sdf, wn = a.w_nor;
    const float e = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
    const float Lsd = ws * smin * e;                      // dl / dA = -dl / dB
    const float L_d = (!floored && Ld > 0.f && B > 0.f) ? Lsd / (2.f * kappa * d * B) : 0.f;
    // u = dl / d(grad d), kept scaled: u_s = u * gmax (bounded), and the
    // terms that multiply it take 1 / gmax instead
    float u[3] = {0.f, 0.f, 0.f};
    if (with_nor) {
        const float gdotn = gh[0] * nrm[0] + gh[1] * nrm[1] + gh[2] * nrm[2];
        for (int c = 0; c < 3; ++c) u[c] = 2.f * wn * sg * (nrm[c] - gdotn * gh[c]) / gn_s;
    }
    const float dAdr = r > 0.f ? 0.5f * fg.beta * A / r : 0.f;
    const float L_h = ws * e * sg * dAdr;
    const float L_smin = ws * (fabsf(diff) - e * r * dAdr);
    const float L_bg = Lsd * 0.5f * A * lr;                   // through A's exponent beta*/2
    float L_n[3];
    for (int c = 0; c < 3; ++c) L_n[c] = (with_nor ? 2.f * wn * (sg * gh[c] + nrm[c]) : 0.f) + L_h * xm[c];
    float gx[3] = {L_h * nrm[0], L_h * nrm[1], L_h * nrm[2]};  // dl / dx

    // pass 2, slot 0 last (it also carries the sample point's dependence)
    {
        const uint32_t il = nb_at(K - 1);
        fn = load_gframe(a.frames, il < (uint32_t)a.n ? il : j, a.rho);
    }
    for (int s = K - 1; s >= 0; --s) {
        const uint32_t i = nb_at(s);
        const GFrame f = fn;
        if (s > 0) {
            const uint32_t i1 = nb_at(s - 1);
            fn = load_gframe(a.frames, i1 < (uint32_t)a.n ? i1 : j, a.rho);
        }
        if (i >= (uint32_t)a.n) continue;  // padding slot: no record
        float* ps = rec_at(s);
        const Term t = eval_term(f, f0.mu, d0, kappa);
        // b = diag(1/sig) R^T u, scaled by gmax like u
        float b[3];
        for (int k = 0; k < 3; ++k) b[k] = (f.R[k] * u[0] + f.R[3 + k] * u[1] + f.R[6 + k] * u[2]) * f.isig[k];
        const float ab = t.a[0] * b[0] + t.a[1] * b[1] + t.a[2] * b[2];
        // S = L_d T + c (a . b); cg = c / gmax pairs with the scaled b
        const float cg = t.c * inv_gmax;
        float dcdq = 0.f, dTdb = 0.f, dcdb = 0.f;
        if (t.q > 0.f) {
            dcdq = ((0.5f * f.beta - 1.f) - kappa * 0.5f * f.beta * t.P) * t.iq;  // (dc/dq) / c
            dTdb = -0.5f * kappa * t.P * t.lq * t.T;
            dcdb = f.ibeta + 0.5f * t.lq - 0.5f * kappa * t.P * t.lq;           // (dc/dbeta) / c
        }
        float dSa[3], dSb[3];
        for (int k = 0; k < 3; ++k) {
            dSa[k] = L_d * t.c * t.a[k] + 2.f * ab * cg * dcdq * t.a[k] + cg * b[k];
            dSb[k] = cg * t.a[k];
        }
        float g_mu[3], g_sig[3], G[9];
        float sa[3], sb[3];
        for (int k = 0; k < 3; ++k) {
            sa[k] = dSa[k] * f.isig[k];
            sb[k] = dSb[k] * f.isig[k];
        }
        for (int r2 = 0; r2 < 3; ++r2) {
            const float v = f.R[3 * r2] * sa[0] + f.R[3 * r2 + 1] * sa[1] + f.R[3 * r2 + 2] * sa[2];
            gx[r2] += v;
            g_mu[r2] = -v;
        }
        for (int k = 0; k < 3; ++k) g_sig[k] = -(t.a[k] * sa[k] + b[k] * sb[k]);
        for (int r2 = 0; r2 < 3; ++r2)
            for (int k = 0; k < 3; ++k) G[3 * r2 + k] = sa[k] * t.dx[r2] + sb[k] * u[r2];
        float g_o = (L_d * t.T + cg * ab) * f.io;
        float g_beta = L_d * dTdb + ab * cg * dcdb;
        if (s == gs) {
            for (int c = 0; c < 3; ++c) {
                g_mu[c] -= L_h * nrm[c];
                for (int k = 0; k < 3; ++k) G[3 * c + k] += k == ks ? L_n[c] : 0.f;
            }
            for (int k = 0; k < 3; ++k) g_sig[k] += k == ks ? L_smin : 0.f;
            g_beta += L_bg;
        }
        if (s == 0) {
            // x = mu_0 + R_0 diag(sig_0) xi
            for (int c = 0; c < 3; ++c) g_mu[c] += gx[c];
            for (int k = 0; k < 3; ++k) {
                g_sig[k] += xi[k] * (f.R[k] * gx[0] + f.R[3 + k] * gx[1] + f.R[6 + k] * gx[2]);
                for (int r2 = 0; r2 < 3; ++r2) G[3 * r2 + k] += f.sig[k] * xi[k] * gx[r2];
            }
        }
        // sigma = phi(beta) s: ds = phi dsig; dbeta += phi'/phi sum sig dsig
        const float dphi = a.rho * (1.f - 0.5f * f.phi);  // phi' / phi
        g_beta += dphi * (f.sig[0] * g_sig[0] + f.sig[1] * g_sig[1] + f.sig[2] * g_sig[2]);
        float g_q[4];
        rot_adjoint(f, G, g_q);
        float4* o4 = reinterpret_cast<float4*>(ps);
        o4[0] = make_float4(g_mu[0], g_mu[1], g_mu[2], f.phi * g_sig[0]);
        o4[1] = make_float4(f.phi * g_sig[1], f.phi * g_sig[2], g_q[0], g_q[1]);
        o4[2] = make_float4(g_q[2], g_q[3], g_o, g_beta);
        // the whole 64-byte record, so that the cache takes the write without
        // reading the line first
        o4[3] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}
#undef nb_at
#undef rec_at

// Gradient of each splat: the sum of its records, which the loss kernel wrote
// contiguously in inverse-list order, added into the gradients.  Four
// records per step keep several loads in flight; the sum runs in order.
__global__ __launch_bounds__(256) void k_gsr_gather(GsrArgs a) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= (uint32_t)a.n) return;
    float acc[GSR_PARTIAL_FLOATS];
#pragma unroll
    for (int c = 0; c < GSR_PARTIAL_FLOATS; ++c) acc[c] = 0.f;
    const uint32_t e0 = a.inv_offsets[i], e1 = a.inv_offsets[i + 1];
    for (uint32_t e = e0; e < e1; e += 4) {
        float4 v[4][3];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (e + t < e1) {
                const float4* p = reinterpret_cast<const float4*>(a.partials + (size_t)(e + t) * GSR_PARTIAL_STRIDE);
                v[t][0] = p[0];
                v[t][1] = p[1];
                v[t][2] = p[2];
            } else {
                v[t][0] = v[t][1] = v[t][2] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            acc[0] += v[t][0].x; acc[1] += v[t][0].y; acc[2] += v[t][0].z; acc[3] += v[t][0].w;
            acc[4] += v[t][1].x; acc[5] += v[t][1].y; acc[6] += v[t][1].z; acc[7] += v[t][1].w;
            acc[8] += v[t][2].x; acc[9] += v[t][2].y; acc[10] += v[t][2].z; acc[11] += v[t][2].w;
        }
    }
    const size_t n = (size_t)a.n;
    for (int c = 0; c < 3; ++c) {
        a.g_mean[c * n + i] += acc[c];
        a.g_scale[c * n + i] += acc[3 + c];
    }
    for (int c = 0; c < 4; ++c) a.g_quat[c * n + i] += acc[6 + c];
    a.g_opacity[i] += acc[10];
    a.g_beta[i] += acc[11];
}

// Sums of the per-sample losses in a fixed order: each block adds
// GSR_SUM_BLOCK samples by a fixed tree, then one block adds the block sums.
__global__ __launch_bounds__(256) void k_gsr_sum_blocks(const float* sample_out, int n, float* parts) {
    __shared__ float s0[256], s1[256];
    const uint32_t base = blockIdx.x * (uint32_t)GSR_SUM_BLOCK;
    float a0 = 0.f, a1 = 0.f;
    for (uint32_t t = threadIdx.x; t < (uint32_t)GSR_SUM_BLOCK; t += 256u) {
        const uint32_t j = base + t;
        if (j < (uint32_t)n) {
            const float2 v = *reinterpret_cast<const float2*>(sample_out + (size_t)j * 4);
            a0 += v.x;
            a1 += v.y;
        }
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        parts[2 * blockIdx.x] = s0[0];
        parts[2 * blockIdx.x + 1] = s1[0];
    }
}

__global__ __launch_bounds__(1024) void k_gsr_sum(const float* parts, int nparts, float* losses) {
    __shared__ float s0[1024], s1[1024];
    float a0 = 0.f, a1 = 0.f;
    for (int b = threadIdx.x; b < nparts; b += 1024) {
        a0 += parts[2 * b];
        a1 += parts[2 * b + 1];
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        losses[0] = s0[0];
        losses[1] = s1[0];
    }
}

unsigned blocks(uint64_t count, unsigned per) { return (unsigned)((count + per - 1) / per); }

}  // namespace

KnnLayout knn_layout(int n, int k) {
    KnnLayout L{};
    const uint64_t n1 = n > 0 ? (uint64_t)n : 1;
    const uint64_t total = n1 * (uint64_t)k;
    L.bound_parts = (uint32_t)std::min<uint64_t>(blocks(n1, 256), 1024);
    L.cell_cap = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(4 * n1, 64), 1ull << 24);
    const uint64_t sort_n = std::max(n1, total);
    uint64_t off = 0;
    auto take = [&](uint64_t words) {
        const uint64_t o = off;
        off += (words + 63) & ~63ull;  // 256-byte aligned
        return o;
    };
    L.o_grid = take(sizeof(KnnGrid) / 4 + 1);
    L.o_parts = take(6ull * L.bound_parts);
    L.o_keys = take(sort_n);
    L.o_ka = take(sort_n);
    L.o_va = take(sort_n);
    L.o_kb = take(sort_n);
    L.o_vb = take(sort_n);
    L.o_hist = take(256ull * ((sort_n + SORT_TILE - 1) / SORT_TILE));
    const uint64_t hist_n = 256ull * ((sort_n + SORT_TILE - 1) / SORT_TILE);
    L.o_scan = take((std::max<uint64_t>(hist_n, sort_n) + SCAN_TILE - 1) / SCAN_TILE + 64);
    L.o_pos = take(4 * n1);
    L.o_start = take(L.cell_cap);
    L.o_end = take(L.cell_cap);
    L.words = off;
    return L;
}

static int bits_for(uint64_t v) {
    int b = 1;
    while (b < 32 && (1ull << b) <= v) ++b;
    return b;
}

hipError_t launch_knn(const float* mean, int n, int k, uint32_t* knn, uint32_t* order_out, uint32_t* inv_offsets,
                      uint32_t* inv_entries, uint32_t* inv_slot, uint32_t* ws, hipStream_t stream) {
    if (n == 0) return launch_fill_u32(inv_offsets, 0u, 1, stream);
    const KnnLayout L = knn_layout(n, k);
    KnnGrid* grid = reinterpret_cast<KnnGrid*>(ws + L.o_grid);
    float* parts = reinterpret_cast<float*>(ws + L.o_parts);
    hipLaunchKernelGGL(k_knn_bounds, dim3(L.bound_parts), dim3(256), 0, stream, mean, n, parts);
    hipLaunchKernelGGL(k_knn_grid, dim3(1), dim3(64), 0, stream, parts, (int)L.bound_parts, n, L.cell_cap, grid);
    hipLaunchKernelGGL(k_knn_cells, dim3(blocks(n, 256)), dim3(256), 0, stream, mean, n, grid, ws + L.o_keys);
    // three 8-bit passes over the 24-bit Morton keys end in the "a" buffers:
    // the sorted values land in order_out
    SortBuffers sb{ws + L.o_ka, order_out, ws + L.o_kb, ws + L.o_vb, ws + L.o_hist, ws + L.o_scan};
    bool in_b = false;
    hipError_t e = radix_sort(ws + L.o_keys, nullptr, (uint64_t)n, nullptr, 24, 8, sb, &in_b, stream);
    if (e != hipSuccess) return e;
    if (in_b) return hipErrorInvalidValue;  // not reached with an odd number of passes
    const uint32_t* skeys = sb.keys_a;
    const uint32_t* order = order_out;
    e = launch_fill_u32(ws + L.o_start, 0u, L.cell_cap, stream);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(ws + L.o_end, 0u, L.cell_cap, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_knn_ranges, dim3(blocks(n, 256)), dim3(256), 0, stream, skeys, n, grid, ws + L.o_start,
                       ws + L.o_end);
    const dim3 qg(blocks(n, 256)), qb(256);
    const uint32_t *cs0 = ws + L.o_start, *ce0 = ws + L.o_end;
    float4* pos = reinterpret_cast<float4*>(ws + L.o_pos);
    hipLaunchKernelGGL(k_knn_sorted_pos, qg, qb, 0, stream, mean, n, order, pos);
    switch (k) {
#define GESR_KNN_CASE(KK) \
    case KK: hipLaunchKernelGGL(k_knn_query<KK>, qg, qb, 0, stream, pos, n, grid, cs0, ce0, knn); break;
        GESR_KNN_CASE(2) GESR_KNN_CASE(3) GESR_KNN_CASE(4) GESR_KNN_CASE(5) GESR_KNN_CASE(6) GESR_KNN_CASE(7)
        GESR_KNN_CASE(8) GESR_KNN_CASE(9) GESR_KNN_CASE(10) GESR_KNN_CASE(11) GESR_KNN_CASE(12)
        GESR_KNN_CASE(13) GESR_KNN_CASE(14) GESR_KNN_CASE(15) GESR_KNN_CASE(16)
#undef GESR_KNN_CASE
        default: hipLaunchKernelGGL(k_knn_self, qg, qb, 0, stream, n, knn); break;
    }
    // inverse lists: stable sort of the entries by the neighbour they name
    const uint64_t total = (uint64_t)n * k;
    hipLaunchKernelGGL(k_inv_keys, dim3(blocks(total, 256)), dim3(256), 0, stream, knn, order, total, (uint32_t)k,
                       (uint32_t)n, ws + L.o_keys);
    SortBuffers ib{ws + L.o_ka, inv_entries, ws + L.o_kb, ws + L.o_vb, ws + L.o_hist, ws + L.o_scan};
    // an even number of passes leaves the result in (keys_b, vals_b): route the
    // values so that they end in inv_entries
    const int passes = radix_passes(bits_for((uint64_t)n), 8);
    if (passes % 2 == 0) ib = SortBuffers{ws + L.o_ka, ws + L.o_va, ws + L.o_kb, inv_entries, ws + L.o_hist, ws + L.o_scan};
    e = radix_sort(ws + L.o_keys, nullptr, total, nullptr, bits_for((uint64_t)n), 8, ib, &in_b, stream);
    if (e != hipSuccess) return e;
    const uint32_t* ikeys = in_b ? ib.keys_b : ib.keys_a;
    hipLaunchKernelGGL(k_inv_offsets, dim3(blocks(total + 1, 256)), dim3(256), 0, stream, ikeys, total, (uint32_t)n,
                       inv_offsets);
    hipLaunchKernelGGL(k_inv_slots, dim3(blocks(total, 256)), dim3(256), 0, stream, inv_entries, inv_offsets,
                       (uint32_t)n, inv_slot);
    return hipGetLastError();
}

hipError_t launch_gsr(GsrArgs a, hipStream_t stream) {
    if (a.n == 0) {
        if (a.losses) return launch_fill_u32(reinterpret_cast<uint32_t*>(a.losses), 0u, 2, stream);
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_gsr_frames, dim3(blocks(a.n, 256)), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_gsr_loss, dim3(blocks(a.n, 128)), dim3(128), 0, stream, a);
    if (a.partials) hipLaunchKernelGGL(k_gsr_gather, dim3(blocks(a.n, 256)), dim3(256), 0, stream, a);
    if (a.losses) {
        const unsigned nparts = blocks(a.n, GSR_SUM_BLOCK);
        hipLaunchKernelGGL(k_gsr_sum_blocks, dim3(nparts), dim3(256), 0, stream, a.sample_out, a.n, a.sum_parts);
        hipLaunchKernelGGL(k_gsr_sum, dim3(1), dim3(1024), 0, stream, a.sum_parts, (int)nparts, a.losses);
    }
    return hipGetLastError();
}

}  // namespace gesr
