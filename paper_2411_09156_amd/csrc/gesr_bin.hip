// Tile binning for the GES rasterizer (gfx950): prefix scans, a stable LSD
// radix sort, instance duplication, per-tile ranges and the render worklist.
//
// Every instance carries the 64-bit key (global tile id << 32 | depth bits).
// All instances of one (view, splat) share its depth, so the LSD passes over
// the 32 depth bits can run once per (view, splat) *before* duplication:
// splats are first sorted by depth, duplicated in that order, and only the
// tile-id bits are then sorted per instance.  Each pass is stable, so the
// result is exactly the stable sort of the full key.

#include "gesr_device.h"
#include "gesr_kernels.h"

namespace gesr {

namespace {

constexpr int WAVES = SORT_THREADS / 64;

// ------------------------------------------------------------------- scans
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d) x += y;
    }
    return x;
}

// Exclusive scan over a block of blockDim.x threads (multiple of 64); returns
// the thread's exclusive prefix and the block total in *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_wave, uint32_t* total) {
    const uint32_t lane = __lane_id(), wave = threadIdx.x / 64, nw = blockDim.x / 64;
    uint32_t inc = wave_inclusive_scan(x);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t w = 0; w < nw; ++w) {
            uint32_t c = s_wave[w];
            s_wave[w] = run;
            run += c;
        }
        s_wave[nw] = run;
    }
    __syncthreads();
    uint32_t r = s_wave[wave] + inc - x;
    *total = s_wave[nw];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* in, uint64_t count, uint32_t* partials) {
    __shared__ uint32_t s_wave[8];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < SCAN_TILE / 256; ++j) {
        uint64_t idx = base + (uint64_t)j * 256 + threadIdx.x;
        if (idx < count) acc += in[idx];
    }
    uint32_t tot;
    block_exclusive_scan(acc, s_wave, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// One block of 1024 threads scans up to SCAN_TOP_MAX partials in place.
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* partials, uint32_t nb, uint32_t* total) {
    __shared__ uint32_t s_wave[17];
    constexpr int PER = SCAN_TOP_MAX / 1024;
    const uint32_t t = threadIdx.x;
    uint32_t v[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        uint32_t idx = t * PER + k;
        v[k] = idx < nb ? partials[idx] : 0u;
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(sum, s_wave, &tot);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        uint32_t idx = t * PER + k;
        if (idx < nb) partials[idx] = run;
        run += v[k];
    }
    if (t == 0 && total) *total = tot;
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* in, uint32_t* out, uint64_t count,
                                                    const uint32_t* partials) {
    // striped (coalesced) loads into LDS, then each thread scans 16 consecutive items
    __shared__ uint32_t s[SCAN_TILE + SCAN_TILE / 16];
    __shared__ uint32_t s_wave[8];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int j = 0; j < SCAN_TILE / 256; ++j) {
        uint32_t L = j * 256 + threadIdx.x;
        uint64_t idx = base + L;
        s[L + L / 16] = idx < count ? in[idx] : 0u;
    }
    __syncthreads();
    uint32_t v[16], sum = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        v[k] = s[threadIdx.x * 17 + k];
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(sum, s_wave, &tot) + partials[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        s[threadIdx.x * 17 + k] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SCAN_TILE / 256; ++j) {
        uint32_t L = j * 256 + threadIdx.x;
        uint64_t idx = base + L;
        if (idx < count) out[idx] = s[L + L / 16];
    }
}

// -------------------------------------------------------------- radix sort
// Lanes of the wave holding the same digit (match by one ballot per bit).
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t digit, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const bool bit = (digit >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

__device__ __forceinline__ uint32_t count_of(const uint32_t* count_dev, uint64_t count_static) {
    return count_dev ? *count_dev : (uint32_t)count_static;
}

// Digit histogram of one block of SORT_TILE keys, stored digit-major:
// block_hist[digit * nblocks + block].  Counting needs no ranking, so LDS
// atomics (exact, order-independent) replace the ballot matching.
template <int BITS>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint32_t* keys, uint64_t count_static,
                                                             const uint32_t* count_dev, int shift,
                                                             uint32_t* block_hist, uint32_t nblocks) {
    constexpr int RADIX = 1 << BITS;
    __shared__ uint32_t hist[RADIX];
    for (int j = threadIdx.x; j < RADIX; j += SORT_THREADS) hist[j] = 0u;
    __syncthreads();
    const uint32_t n = count_of(count_dev, count_static);
    const uint64_t base = (uint64_t)blockIdx.x * SORT_TILE;
    if (base < n) {
        uint32_t k[SORT_ITEMS];
#pragma unroll
        for (int r = 0; r < SORT_ITEMS; ++r) {
            const uint64_t idx = base + (uint64_t)r * SORT_THREADS + threadIdx.x;
            k[r] = idx < n ? keys[idx] : 0u;
        }
#pragma unroll
        for (int r = 0; r < SORT_ITEMS; ++r) {
            const uint64_t idx = base + (uint64_t)r * SORT_THREADS + threadIdx.x;
            if (idx < n) atomicAdd(&hist[(k[r] >> shift) & (RADIX - 1)], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RADIX; d += SORT_THREADS) block_hist[(uint64_t)d * nblocks + blockIdx.x] = hist[d];
}

// Stable scatter of one block: ranks keys per digit in position order (wave
// ballots + per-wave running counts), stages the block in LDS in sorted
// order, then writes each digit run contiguously.
template <int BITS>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(const uint32_t* keys_in, const uint32_t* vals_in,
                                                                uint32_t* keys_out, uint32_t* vals_out,
                                                                uint64_t count_static, const uint32_t* count_dev,
                                                                int shift, const uint32_t* block_off,
                                                                uint32_t nblocks) {
    constexpr int RADIX = 1 << BITS;
    __shared__ uint32_t hist[WAVES][RADIX];
    __shared__ uint32_t digit_start[RADIX + 1];
    __shared__ uint32_t g_off[RADIX];
    __shared__ uint32_t s_keys[SORT_TILE];
    __shared__ uint32_t s_vals[SORT_TILE];
    __shared__ uint32_t s_wave[WAVES + 1];

    const uint32_t n = count_of(count_dev, count_static);
    const uint64_t block_start = (uint64_t)blockIdx.x * SORT_TILE;
    if (block_start >= n) return;  // uniform over the block
    for (int j = threadIdx.x; j < WAVES * RADIX; j += SORT_THREADS) (&hist[0][0])[j] = 0u;
    __syncthreads();

    const uint32_t lane = __lane_id(), wave = threadIdx.x / 64;
    const uint64_t base = block_start + wave * (64 * SORT_ITEMS);
    const uint64_t lt = lanemask_lt();
    uint32_t k[SORT_ITEMS], v[SORT_ITEMS], rank[SORT_ITEMS];
    // issue every load of the wave's chunk before any ranking work
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const uint64_t idx = base + r * 64 + lane;
        const bool valid = idx < n;
        k[r] = valid ? keys_in[idx] : 0xFFFFFFFFu;
        v[r] = valid ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
    }
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const uint64_t idx = base + r * 64 + lane;
        const bool valid = idx < n;
        const uint32_t digit = (k[r] >> shift) & (RADIX - 1);
        const uint64_t vmask = __ballot(valid);
        const uint64_t peers = match_digit<BITS>(digit, vmask);
        const uint32_t old = valid ? hist[wave][digit] : 0u;
        rank[r] = old + (uint32_t)__popcll(peers & lt);
        if (valid && lane == (uint32_t)__ffsll((unsigned long long)peers) - 1)
            hist[wave][digit] = old + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, and the block total
    uint32_t cnt = 0;
    if (threadIdx.x < RADIX) {
        const int d = threadIdx.x;
        for (int w = 0; w < WAVES; ++w) {
            uint32_t c = hist[w][d];
            hist[w][d] = cnt;
            cnt += c;
        }
        g_off[d] = block_off[(uint64_t)d * nblocks + blockIdx.x];
    }
    // exclusive scan of the block's digit counts (RADIX <= SORT_THREADS)
    uint32_t tot;
    const uint32_t ds = block_exclusive_scan(threadIdx.x < RADIX ? cnt : 0u, s_wave, &tot);
    if (threadIdx.x < RADIX) digit_start[threadIdx.x] = ds;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const uint64_t idx = base + r * 64 + lane;
        if (idx < n) {
            const uint32_t digit = (k[r] >> shift) & (RADIX - 1);
            const uint32_t lp = digit_start[digit] + hist[wave][digit] + rank[r];
            s_keys[lp] = k[r];
            s_vals[lp] = v[r];
        }
    }
    __syncthreads();
    const uint32_t in_block = (uint32_t)min<uint64_t>(SORT_TILE, n - block_start);
    for (uint32_t j = threadIdx.x; j < in_block; j += SORT_THREADS) {
        const uint32_t key = s_keys[j];
        const uint32_t digit = (key >> shift) & (RADIX - 1);
        const uint32_t pos = g_off[digit] + (j - digit_start[digit]);
        keys_out[pos] = key;
        vals_out[pos] = s_vals[j];
    }
}

template <int BITS>
hipError_t sort_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, uint64_t count_static,
                     const uint32_t* count_dev, int shift, const SortBuffers& b, hipStream_t stream) {
    const uint32_t nblocks = (uint32_t)((count_static + SORT_TILE - 1) / SORT_TILE);
    hipLaunchKernelGGL(k_radix_hist<BITS>, dim3(nblocks), dim3(SORT_THREADS), 0, stream, kin, count_static,
                       count_dev, shift, b.block_hist, nblocks);
    hipError_t e = scan_exclusive(b.block_hist, b.block_hist, (uint64_t)nblocks << BITS, b.scan_partials, nullptr,
                                  stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter<BITS>, dim3(nblocks), dim3(SORT_THREADS), 0, stream, kin, vin, kout, vout,
                       count_static, count_dev, shift, b.block_hist, nblocks);
    return hipGetLastError();
}

// ----------------------------------------------------------------- binning
__global__ __launch_bounds__(256) void k_gather_counts(const uint32_t* order, const uint32_t* tiles_touched,
                                                       uint32_t* out, uint64_t count) {
    const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < count) out[k] = tiles_touched[order[k]];
}

// Instance expansion, load-balanced: a block owns DUP_SPLATS consecutive
// (view, splat) pairs in depth order and writes their instances cooperatively
// (instance j finds its pair by binary search over the block's offsets in
// LDS), so every store is coalesced however large the rectangles are.
constexpr int DUP_SPLATS = 256;

__global__ __launch_bounds__(256) void k_duplicate(const uint32_t* order, const uint32_t* offsets, uint64_t count,
                                                   int n, const uint32_t* tiles_touched, const uint32_t* rect,
                                                   DevCams cams, uint64_t m_cap, const uint32_t* total,
                                                   uint32_t* keys, uint32_t* vals, uint32_t* inst_base) {
    __shared__ uint32_t s_off[DUP_SPLATS + 1];
    __shared__ uint32_t s_vi[DUP_SPLATS];
    __shared__ uint32_t s_r0[DUP_SPLATS];   // tx0 | ty0 << 16
    __shared__ uint32_t s_w[DUP_SPLATS];    // rectangle width in tiles
    __shared__ uint32_t s_row[DUP_SPLATS];  // tile_base of the view
    __shared__ uint32_t s_tx[DUP_SPLATS];   // tiles_x of the view
    const uint64_t k0 = (uint64_t)blockIdx.x * DUP_SPLATS;
    const uint64_t k = k0 + threadIdx.x;
    const uint32_t m_total = *total;
    if (k < count) {
        const uint32_t vi = order[k];
        const uint32_t off = offsets[k];
        inst_base[vi] = off;
        s_off[threadIdx.x] = off;
        s_vi[threadIdx.x] = vi;
        const uint2 r = reinterpret_cast<const uint2*>(rect)[vi];
        s_r0[threadIdx.x] = r.x;
        s_w[threadIdx.x] = (r.y & 0xFFFFu) - (r.x & 0xFFFFu) + 1u;
        const DevView& w = cams.v[vi / (uint32_t)n];
        s_row[threadIdx.x] = w.tile_base;
        s_tx[threadIdx.x] = (uint32_t)w.tiles_x;
    } else {
        s_off[threadIdx.x] = m_total;
    }
    if (threadIdx.x == 0) s_off[DUP_SPLATS] = (k0 + DUP_SPLATS < count) ? offsets[k0 + DUP_SPLATS] : m_total;
    __syncthreads();
    const uint64_t begin = s_off[0];
    const uint64_t end = min<uint64_t>(s_off[DUP_SPLATS], m_cap);
    for (uint64_t j = begin + threadIdx.x; j < end; j += 256) {
        // largest l with s_off[l] <= j (pairs with no instances are skipped over)
        int lo = 0, hi = DUP_SPLATS;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if ((uint64_t)s_off[mid] <= j) lo = mid;
            else hi = mid;
        }
        const uint32_t q = (uint32_t)(j - s_off[lo]);
        const uint32_t w = s_w[lo];
        const uint32_t r0 = s_r0[lo];
        const uint32_t ty = (r0 >> 16) + q / w, tx = (r0 & 0xFFFFu) + q % w;
        keys[j] = s_row[lo] + ty * s_tx[lo] + tx;
        vals[j] = s_vi[lo];
    }
}

// Per-tile instance counts from the rectangles: +1/-1 at the four corners of
// each rectangle in a per-view (tiles_y + 1) x (tiles_x + 1) difference grid,
// then a 2-D prefix sum.  Each block accumulates the corners of one chunk of
// CORNER_CHUNK splats of one view in an LDS copy of the grid (LDS atomics;
// integer sums, exact) and writes it out whole; k_tile_counts adds the
// chunks' grids in fixed order and takes the prefix sums.
constexpr int CORNER_CHUNK = 16384;
constexpr size_t MAX_CORNER_LDS = 64 * 1024;

__global__ __launch_bounds__(256) void k_rect_corners(const uint32_t* tiles_touched, const uint32_t* rect, int n,
                                                      DevCams cams, uint32_t chunks, int* partial_grids) {
    extern __shared__ int s_grid[];
    const int v = blockIdx.y;
    const uint32_t c = blockIdx.x;
    const DevView& w = cams.v[v];
    const uint32_t gx = (uint32_t)w.tiles_x + 1u;
    const uint32_t cells = gx * ((uint32_t)w.tiles_y + 1u);
    for (uint32_t k = threadIdx.x; k < cells; k += 256) s_grid[k] = 0;
    __syncthreads();
    const uint64_t i0 = (uint64_t)c * CORNER_CHUNK;
    const uint64_t i1 = min<uint64_t>(i0 + CORNER_CHUNK, (uint64_t)n);
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const uint64_t vi = (uint64_t)v * (uint64_t)n + i;
        if (tiles_touched[vi] == 0) continue;
        const uint2 r = reinterpret_cast<const uint2*>(rect)[vi];
        const uint32_t tx0 = r.x & 0xFFFFu, ty0 = r.x >> 16, tx1 = (r.y & 0xFFFFu) + 1u, ty1 = (r.y >> 16) + 1u;
        atomicAdd(&s_grid[ty0 * gx + tx0], 1);
        atomicAdd(&s_grid[ty0 * gx + tx1], -1);
        atomicAdd(&s_grid[ty1 * gx + tx0], -1);
        atomicAdd(&s_grid[ty1 * gx + tx1], 1);
    }
    __syncthreads();
    int* dst = partial_grids + (uint64_t)w.grid_base * chunks + (uint64_t)c * cells;
    for (uint32_t k = threadIdx.x; k < cells; k += 256) dst[k] = s_grid[k];
}

// Views whose grid does not fit in LDS: corners go straight to the global grid
// with global atomics (exact; slower under contention).
__global__ __launch_bounds__(256) void k_rect_corners_global(const uint32_t* tiles_touched, const uint32_t* rect,
                                                             uint64_t count, int n, DevCams cams, int* grid) {
    const uint64_t vi = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (vi >= count || tiles_touched[vi] == 0) return;
    const DevView& w = cams.v[(uint32_t)vi / (uint32_t)n];
    const uint32_t gx = (uint32_t)w.tiles_x + 1u;
    int* g = grid + w.grid_base;
    const uint2 r = reinterpret_cast<const uint2*>(rect)[vi];
    const uint32_t tx0 = r.x & 0xFFFFu, ty0 = r.x >> 16, tx1 = (r.y & 0xFFFFu) + 1u, ty1 = (r.y >> 16) + 1u;
    atomicAdd(&g[ty0 * gx + tx0], 1);
    atomicAdd(&g[ty0 * gx + tx1], -1);
    atomicAdd(&g[ty1 * gx + tx0], -1);
    atomicAdd(&g[ty1 * gx + tx1], 1);
}

// One block per view: sum the chunks' grids per cell (ascending chunk order;
// chunks == 0: the grid already holds the sums), then row and column prefix
// sums give each tile's instance count.
__global__ __launch_bounds__(256) void k_tile_counts(DevCams cams, uint32_t chunks, const int* partial_grids,
                                                     int* grid, uint32_t* counts) {
    const int v = blockIdx.x;
    const DevView& w = cams.v[v];
    const int gx = w.tiles_x + 1;
    const uint32_t cells = (uint32_t)gx * (uint32_t)(w.tiles_y + 1);
    int* g = grid + w.grid_base;
    const int* src = partial_grids + (uint64_t)w.grid_base * chunks;
    if (chunks > 0)
        for (uint32_t k = threadIdx.x; k < cells; k += 256) {
            int acc = 0;
            for (uint32_t c = 0; c < chunks; ++c) acc += src[(uint64_t)c * cells + k];
            g[k] = acc;
        }
    __syncthreads();
    for (int y = threadIdx.x; y < w.tiles_y; y += 256) {
        int run = 0;
        for (int x = 0; x < w.tiles_x; ++x) {
            run += g[y * gx + x];
            g[y * gx + x] = run;
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < w.tiles_x; x += 256) {
        int run = 0;
        for (int y = 0; y < w.tiles_y; ++y) {
            run += g[y * gx + x];
            counts[w.tile_base + (uint32_t)(y * w.tiles_x + x)] = (uint32_t)run;
        }
    }
}

// ranges[t] = [start, start + count), clamped to the instances actually listed
// (min(M, m_cap)); when the capacity overflowed the lists are incomplete and
// only memory safety is kept.
__global__ __launch_bounds__(256) void k_ranges_from_counts(const uint32_t* counts, const uint32_t* starts,
                                                            uint64_t total_tiles, const uint32_t* listed,
                                                            uint32_t* ranges) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total_tiles) return;
    const uint32_t m = *listed;
    const uint32_t c = counts[t];
    const uint32_t s0 = starts[t];
    const uint32_t s1 = s0 + c;
    // empty tiles get (0, 0)
    reinterpret_cast<uint2*>(ranges)[t] = c == 0 ? make_uint2(0u, 0u) : make_uint2(s0 < m ? s0 : m, s1 < m ? s1 : m);
}

__global__ void k_set_counters(uint32_t* c, uint64_t m_cap) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t m = c[0];
        c[1] = (uint64_t)m > m_cap ? 1u : 0u;
        c[2] = (uint32_t)((uint64_t)m > m_cap ? m_cap : m);
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint32_t value, uint64_t count) {
    const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < count) p[k] = value;
}

// Worklist key: longer lists first (descending length, ties by tile id).
__global__ __launch_bounds__(256) void k_worklist_keys(const uint32_t* ranges, uint64_t total_tiles, uint32_t* keys) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total_tiles) return;
    const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];  // list length as listed
    keys[t] = 0xFFFFu - (len < 0xFFFFu ? len : 0xFFFFu);
}

__global__ __launch_bounds__(256) void k_l1_grad(const float* image, const float* target, uint64_t count, float scale,
                                                 float* grad) {
    const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const float d = image[k] - target[k];
    grad[k] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
}

inline dim3 grid_for(uint64_t count) { return dim3((unsigned)((count + 255) / 256)); }

}  // namespace

hipError_t scan_exclusive(const uint32_t* in, uint32_t* out, uint64_t count, uint32_t* partials, uint32_t* total,
                          hipStream_t stream) {
    if (count == 0) {
        if (total) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, stream, total, 0u, (uint64_t)1);
        return hipGetLastError();
    }
    const uint64_t nb = (count + SCAN_TILE - 1) / SCAN_TILE;
    if (nb > (uint64_t)SCAN_TOP_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, stream, in, count, partials);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, stream, partials, (uint32_t)nb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, stream, in, out, count, partials);
    return hipGetLastError();
}

int radix_passes(int key_bits, int radix_bits) { return key_bits <= 0 ? 0 : (key_bits + radix_bits - 1) / radix_bits; }

hipError_t radix_sort(const uint32_t* keys_in, const uint32_t* vals_in, uint64_t count_static,
                      const uint32_t* count_dev, int key_bits, int radix_bits, const SortBuffers& b,
                      bool* result_in_b, hipStream_t stream) {
    const int passes = radix_passes(key_bits, radix_bits);
    const uint32_t* kin = keys_in;
    const uint32_t* vin = vals_in;
    bool in_b = false;
    if (count_static == 0) {
        *result_in_b = false;
        return hipSuccess;
    }
    for (int p = 0; p < passes; ++p) {
        // pass p writes to a if p is even, b if odd
        uint32_t* kout = (p & 1) ? b.keys_b : b.keys_a;
        uint32_t* vout = (p & 1) ? b.vals_b : b.vals_a;
        hipError_t e;
        switch (radix_bits) {
            case 4: e = sort_pass<4>(kin, vin, kout, vout, count_static, count_dev, p * 4, b, stream); break;
            case 5: e = sort_pass<5>(kin, vin, kout, vout, count_static, count_dev, p * 5, b, stream); break;
            case 6: e = sort_pass<6>(kin, vin, kout, vout, count_static, count_dev, p * 6, b, stream); break;
            case 7: e = sort_pass<7>(kin, vin, kout, vout, count_static, count_dev, p * 7, b, stream); break;
            default: e = sort_pass<8>(kin, vin, kout, vout, count_static, count_dev, p * 8, b, stream); break;
        }
        if (e != hipSuccess) return e;
        kin = kout;
        vin = vout;
        in_b = (p & 1);
    }
    *result_in_b = in_b;
    return hipSuccess;
}

hipError_t launch_gather_counts(const uint32_t* order, const uint32_t* tiles_touched, uint32_t* out, uint64_t count,
                                hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_counts, grid_for(count), dim3(256), 0, stream, order, tiles_touched, out, count);
    return hipGetLastError();
}

hipError_t launch_duplicate(const uint32_t* order, const uint32_t* offsets, uint64_t count, int n,
                            const uint32_t* tiles_touched, const uint32_t* rect, const DevCams& cams,
                            uint64_t m_cap, const uint32_t* total, uint32_t* keys, uint32_t* vals,
                            uint32_t* inst_base, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_duplicate, dim3((unsigned)((count + DUP_SPLATS - 1) / DUP_SPLATS)), dim3(256), 0, stream,
                       order, offsets, count, n, tiles_touched, rect, cams, m_cap, total, keys, vals, inst_base);
    return hipGetLastError();
}

uint32_t corner_chunks(int n) { return (uint32_t)((n + CORNER_CHUNK - 1) / CORNER_CHUNK); }

hipError_t launch_tile_counts(const uint32_t* tiles_touched, const uint32_t* rect, int n, const DevCams& cams,
                              int max_cells, int* partial_grids, int* grid, uint32_t* counts, hipStream_t stream) {
    if (n == 0) {  // no splats: every count is zero
        uint64_t total = 0;
        for (int v = 0; v < cams.V; ++v) total += (uint64_t)cams.v[v].tiles_x * cams.v[v].tiles_y;
        hipLaunchKernelGGL(k_fill_u32, grid_for(total), dim3(256), 0, stream, counts, 0u, total);
        return hipGetLastError();
    }
    uint32_t chunks = corner_chunks(n);
    const size_t lds = (size_t)max_cells * sizeof(int);
    if (lds <= MAX_CORNER_LDS) {
        hipLaunchKernelGGL(k_rect_corners, dim3(chunks, (unsigned)cams.V), dim3(256), lds, stream, tiles_touched, rect,
                           n, cams, chunks, partial_grids);
    } else {
        uint64_t cells = 0, vn = (uint64_t)cams.V * (uint64_t)n;
        for (int v = 0; v < cams.V; ++v) cells += (uint64_t)(cams.v[v].tiles_x + 1) * (cams.v[v].tiles_y + 1);
        hipLaunchKernelGGL(k_fill_u32, grid_for(cells), dim3(256), 0, stream, reinterpret_cast<uint32_t*>(grid), 0u,
                           cells);
        hipLaunchKernelGGL(k_rect_corners_global, grid_for(vn), dim3(256), 0, stream, tiles_touched, rect, vn, n, cams,
                           grid);
        chunks = 0;
    }
    hipLaunchKernelGGL(k_tile_counts, dim3((unsigned)cams.V), dim3(256), 0, stream, cams, chunks, partial_grids, grid,
                       counts);
    return hipGetLastError();
}

hipError_t launch_ranges_from_counts(const uint32_t* counts, const uint32_t* starts, uint64_t total_tiles,
                                     const uint32_t* listed, uint32_t* ranges, hipStream_t stream) {
    if (total_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ranges_from_counts, grid_for(total_tiles), dim3(256), 0, stream, counts, starts, total_tiles,
                       listed, ranges);
    return hipGetLastError();
}

hipError_t launch_set_counters(uint32_t* counters, uint64_t m_cap, hipStream_t stream) {
    hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, stream, counters, m_cap);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, grid_for(count), dim3(256), 0, stream, p, value, count);
    return hipGetLastError();
}

hipError_t launch_worklist_keys(const uint32_t* ranges, uint64_t total_tiles, uint32_t* keys, hipStream_t stream) {
    if (total_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_worklist_keys, grid_for(total_tiles), dim3(256), 0, stream, ranges, total_tiles, keys);
    return hipGetLastError();
}

hipError_t launch_l1_grad(const float* image, const float* target, uint64_t count, float scale, float* grad,
                          hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_l1_grad, grid_for(count), dim3(256), 0, stream, image, target, count, scale, grad);
    return hipGetLastError();
}

}  // namespace gesr
