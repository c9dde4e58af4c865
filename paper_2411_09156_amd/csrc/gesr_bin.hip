// Tile binning for the GES rasterizer (gfx950): prefix scans, a stable LSD
// radix sort, the two-level interval scatter that builds the tile lists,
// per-tile ranges and the render worklist.
//
// Every instance is ordered by the 64-bit key (global tile id << 32 | depth
// bits), ties by (view, splat) index.  All instances of one (view, splat)
// share its depth and its tiles form a rectangle, so no instance is ever
// sorted: the (view, splat) pairs are radix-sorted by depth and then stably
// by view; each pair is written, in that order, into the row lists of the
// tile rows its rectangle covers, and each row-list entry into the tile lists
// of the columns it covers.  Both writes are stable bucketings, so every tile
// list holds its instances in exactly the order of the stable key sort.

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

// One block of 1024 threads: exclusive scan of up to SCAN_TOP_MAX values
// (in may equal out), the total to *total (nullable).
__global__ __launch_bounds__(1024) void k_scan_single(const uint32_t* in, uint32_t* out, uint32_t count,
                                                      uint32_t* total) {
    __shared__ uint32_t s_wave[17];
    constexpr int PER = SCAN_TOP_MAX / 1024;
    const uint32_t t = threadIdx.x;
    uint32_t v[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t idx = t * PER + k;
        v[k] = idx < count ? in[idx] : 0u;
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(sum, s_wave, &tot);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t idx = t * PER + k;
        if (idx < count) out[idx] = run;
        run += v[k];
    }
    if (t == 0 && total) *total = tot;
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

// Digit of one key at bit `shift`.  With view_n != 0 the sorted key is the
// 64-bit (val / view_n) << 32 | key (the view of a pair val = view * n + splat
// above its 32-bit depth key), so a pass can take depth and view bits together.
template <int BITS, bool VIEW>
__device__ __forceinline__ uint32_t sort_digit(uint32_t key, uint32_t val, int shift, uint32_t view_n) {
    if (VIEW) {
        const uint64_t k64 = ((uint64_t)(val / view_n) << 32) | key;
        return (uint32_t)(k64 >> shift) & ((1u << BITS) - 1u);
    }
    return (key >> shift) & ((1u << BITS) - 1u);
}

// Digit histogram of one block of SORT_TILE keys, stored digit-major:
// block_hist[digit * nblocks + block].  Counting needs no ranking, so LDS
// atomics (exact, order-independent) replace the ballot matching.
template <int BITS, bool VIEW>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint32_t* keys, const uint32_t* vals,
                                                             uint64_t count_static, const uint32_t* count_dev,
                                                             int shift, uint32_t view_n, uint32_t* block_hist,
                                                             uint32_t nblocks) {
    constexpr int RADIX = 1 << BITS;
    __shared__ uint32_t hist[RADIX];
    for (int j = threadIdx.x; j < RADIX; j += SORT_THREADS) hist[j] = 0u;
    __syncthreads();
    const uint32_t n = count_of(count_dev, count_static);
    const uint64_t base = (uint64_t)blockIdx.x * SORT_TILE;
    if (base < n) {
        uint32_t k[SORT_ITEMS], v[SORT_ITEMS];
#pragma unroll
        for (int r = 0; r < SORT_ITEMS; ++r) {
            const uint64_t idx = base + (uint64_t)r * SORT_THREADS + threadIdx.x;
            k[r] = idx < n ? keys[idx] : 0u;
            v[r] = VIEW && idx < n ? (vals ? vals[idx] : (uint32_t)idx) : 0u;
        }
#pragma unroll
        for (int r = 0; r < SORT_ITEMS; ++r) {
            const uint64_t idx = base + (uint64_t)r * SORT_THREADS + threadIdx.x;
            if (idx < n) atomicAdd(&hist[sort_digit<BITS, VIEW>(k[r], v[r], shift, view_n)], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RADIX; d += SORT_THREADS) block_hist[(uint64_t)d * nblocks + blockIdx.x] = hist[d];
}

// Stable scatter of one block: ranks keys per digit in position order (wave
// ballots + per-wave running counts), stages the block in LDS in sorted
// order, then writes each digit run contiguously.
template <int BITS, bool VIEW>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(const uint32_t* keys_in, const uint32_t* vals_in,
                                                                uint32_t* keys_out, uint32_t* vals_out,
                                                                uint64_t count_static, const uint32_t* count_dev,
                                                                int shift, uint32_t view_n,
                                                                const uint32_t* block_off, uint32_t nblocks) {
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
        const uint32_t digit = sort_digit<BITS, VIEW>(k[r], v[r], shift, view_n);
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
            const uint32_t digit = sort_digit<BITS, VIEW>(k[r], v[r], shift, view_n);
            const uint32_t lp = digit_start[digit] + hist[wave][digit] + rank[r];
            s_keys[lp] = k[r];
            s_vals[lp] = v[r];
        }
    }
    __syncthreads();
    const uint32_t in_block = (uint32_t)min<uint64_t>(SORT_TILE, n - block_start);
    for (uint32_t j = threadIdx.x; j < in_block; j += SORT_THREADS) {
        const uint32_t key = s_keys[j], val = s_vals[j];
        const uint32_t digit = sort_digit<BITS, VIEW>(key, val, shift, view_n);
        const uint32_t pos = g_off[digit] + (j - digit_start[digit]);
        keys_out[pos] = key;
        vals_out[pos] = val;
    }
}

template <int BITS>
hipError_t sort_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, uint64_t count_static,
                     const uint32_t* count_dev, int shift, uint32_t view_n, const SortBuffers& b,
                     hipStream_t stream) {
    const uint32_t nblocks = (uint32_t)((count_static + SORT_TILE - 1) / SORT_TILE);
    if (view_n != 0u)
        hipLaunchKernelGGL((k_radix_hist<BITS, true>), dim3(nblocks), dim3(SORT_THREADS), 0, stream, kin, vin,
                           count_static, count_dev, shift, view_n, b.block_hist, nblocks);
    else
        hipLaunchKernelGGL((k_radix_hist<BITS, false>), dim3(nblocks), dim3(SORT_THREADS), 0, stream, kin, vin,
                           count_static, count_dev, shift, view_n, b.block_hist, nblocks);
    hipError_t e = scan_exclusive(b.block_hist, b.block_hist, (uint64_t)nblocks << BITS, b.scan_partials, nullptr,
                                  stream);
    if (e != hipSuccess) return e;
    if (view_n != 0u)
        hipLaunchKernelGGL((k_radix_scatter<BITS, true>), dim3(nblocks), dim3(SORT_THREADS), 0, stream, kin, vin,
                           kout, vout, count_static, count_dev, shift, view_n, b.block_hist, nblocks);
    else
        hipLaunchKernelGGL((k_radix_scatter<BITS, false>), dim3(nblocks), dim3(SORT_THREADS), 0, stream, kin, vin,
                           kout, vout, count_static, count_dev, shift, view_n, b.block_hist, nblocks);
    return hipGetLastError();
}

// ----------------------------------------------------------------- binning
// The footprint ellipse of a projected record, q = (L00 dx + L10 dy)^2 +
// (L11 dy)^2 <= Q, with Q its bound qmax widened by 2^-8 (so that float32
// rounding can only widen what follows), and the two row-independent
// quantities of its per-row extents: ym = sqrt(Q) / L11, the half-height, and
// dyr = -L10 sqrt(Q) / (L11 sqrt(L10^2 + L11^2)), the dy of its rightmost
// point (the leftmost is at -dyr).  Stored per item as (u, v, L00, L10),
// (L11, Q, ym, dyr).  Square roots (sqrtf) and quotients (__fdiv_rn) are
// correctly rounded, so the values are reproducible.
__device__ __forceinline__ void row_ellipse(const float* rec, uint32_t vi, float4& e0, float4& e1) {
    const float4* r = reinterpret_cast<const float4*>(rec + (size_t)vi * GESR_REC_FLOATS);
    const float4 a = r[0], b = r[1];
    const float l10 = a.w, l11 = b.x;
    const float Q = b.w + b.w * 0.00390625f;
    const float sq = sqrtf(Q);
    const float rr = sqrtf(l10 * l10 + l11 * l11);
    e0 = a;
    e1 = make_float4(l11, Q, __fdiv_rn(sq, l11), __fdiv_rn(-(l10 * sq), l11 * rr));
}

// Columns of tile row ty that the ellipse (e0, e1) can reach: the x-extent of
// the ellipse over the row's band [ty th, (ty + 1) th) (continuous, a superset
// of its pixel centres), as tile columns clamped to [tx0, tx1]; tx0 | tx1 << 16
// unchanged when a value is not finite, 1 | 0 << 16 (empty) when the band
// misses the ellipse.  Over a band the right end x_r(dy) = (-L10 dy +
// sqrt(Q - (L11 dy)^2)) / L00 is concave, so its maximum is at the ellipse's
// rightmost point clamped into the band (the left end mirrors it).
__device__ __forceinline__ uint32_t row_columns(const float4& e0, const float4& e1, int ty, int tw, int th, int tx0,
                                                int tx1) {
    const float u = e0.x, v = e0.y, l00 = e0.z, l10 = e0.w;
    const float l11 = e1.x, Q = e1.y, ym = e1.z, dyr = e1.w;
    const uint32_t full = (uint32_t)tx0 | ((uint32_t)tx1 << 16);
    const float d0 = (float)(ty * th) - v;
    const float d1 = (float)((ty + 1) * th) - v;
    const float lo = d0 > -ym ? d0 : -ym;
    const float hi = d1 < ym ? d1 : ym;
    if (!(lo <= hi)) return (lo > hi) ? 1u : full;  // empty band (NaN: keep the rectangle)
    const float tr = dyr < lo ? lo : (dyr > hi ? hi : dyr);
    const float tl = -dyr < lo ? lo : (-dyr > hi ? hi : -dyr);
    const float sr = Q - (l11 * tr) * (l11 * tr);
    const float sl = Q - (l11 * tl) * (l11 * tl);
    const float xr = __fdiv_rn(-(l10 * tr) + sqrtf(sr > 0.f ? sr : 0.f), l00);
    const float xl = __fdiv_rn(-(l10 * tl) - sqrtf(sl > 0.f ? sl : 0.f), l00);
    const float X0 = u + xl, X1 = u + xr;
    if (!(X0 <= X1) || !(X1 - X0 < 1e30f)) return full;
    const float inv = 1.0f / (float)tw;  // tile widths are powers of two: exact
    const float f0 = floorf(X0 * inv), f1 = floorf(X1 * inv);
    const int c0 = f0 < (float)tx0 ? tx0 : (f0 > (float)tx1 ? tx1 + 1 : (int)f0);
    const int c1 = f1 > (float)tx1 ? tx1 : (f1 < (float)tx0 ? tx0 - 1 : (int)f1);
    if (c0 > c1) return 1u;
    return (uint32_t)c0 | ((uint32_t)c1 << 16);
}

// The rectangle is read from the pair's record (its fourth 16-byte word), so a
// pair costs one gathered line: the ellipse terms sit in the same 64 bytes.
// Culled pairs carry the rectangle (0xFFFFFFFF, 0), which no rectangle has
// (its corners are tile indices below 2^16).
__global__ __launch_bounds__(256) void k_gather_rects(const uint32_t* order, const float* rec, uint64_t count,
                                                      uint2* out, float4* ell) {
    const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const uint32_t p = order[k];
    const float4 r3 = reinterpret_cast<const float4*>(rec + (size_t)p * GESR_REC_FLOATS)[3];
    const uint2 r = make_uint2(__float_as_uint(r3.x), __float_as_uint(r3.y));
    const bool touched = r.x != 0xFFFFFFFFu;
    out[k] = r;
    if (ell != nullptr) {
        float4 e0 = make_float4(0.f, 0.f, 0.f, 0.f), e1 = e0;
        if (touched) row_ellipse(rec, p, e0, e1);
        ell[2 * k] = e0;
        ell[2 * k + 1] = e1;
    }
}

// ------------------------------------------------- interval scatter (lists)
// A tile's list is every pair whose footprint reaches it, in (depth, pair)
// order: within its tile rectangle, a pair covers in each row one interval of
// columns (those its ellipse reaches over the row), so the lists are built in
// two stable bucketing levels without sorting instances:
//   level 1: pairs of a view, in depth order, go to the rows [ty0, ty1] they
//            cover (row lists, one entry per pair and row, carrying that
//            row's column interval);
//   level 2: a row list's pairs go to the columns of their interval (tile
//            lists, one entry per instance).
// Each level is split into segments: an ordered item list and a window of at
// most IS_W consecutive buckets (level 1: a view's rows 128k..128k+127; level
// 2: a row's tiles 128k..128k+127).  A segment's items are cut into chunks of
// IS_CHUNK (two items per lane of 16 waves; wave w holds items 128 w .. 128 w +
// 127, the second 64 in its second word).  Per-(chunk, bucket) counts are
// scanned over a segment's chunks, bucket totals over all buckets, and the
// scatter writes a chunk's entries of bucket b from b's start + the chunk
// prefix in chunk-item order, read off a (bucket, item) membership bitmap, so
// the order of equal buckets is the item order.  The bucketing arithmetic is
// integer and the result is unique, independent of scheduling.
constexpr int IS_W = 128;
constexpr int IS_IPL = 2;                            // items per lane
constexpr int IS_THREADS = 1024;
constexpr int IS_CHUNK = IS_IPL * IS_THREADS;        // items per chunk
constexpr int IS_WAVES = IS_THREADS / 64;

struct Seg {
    uint32_t begin, end;  // item range
    uint32_t bucket0;     // global bucket id of local bucket 0
    int lo_off;           // first row (level 1) / column (level 2) of the window
    int width;            // buckets in the window (1..IS_W)
};

// Segment s of a level: level 1 enumerates (view, row block), level 2
// (view, row, column block), both view-major.
template <int LEVEL>
__device__ __forceinline__ Seg locate_segment(const IsArgs& a, uint32_t s) {
    Seg g;
    uint32_t row_base = 0;
    for (int v = 0; v < a.cams.V; ++v) {
        const DevView& w = a.cams.v[v];
        if (LEVEL == 1) {
            const uint32_t nb = ((uint32_t)w.tiles_y + IS_W - 1) / IS_W;
            if (s < nb) {
                g.lo_off = (int)s * IS_W;
                g.width = min(IS_W, w.tiles_y - g.lo_off);
                g.bucket0 = row_base + (uint32_t)g.lo_off;
                g.begin = (uint32_t)v * (uint32_t)a.n;
                g.end = g.begin + (uint32_t)a.n;
                return g;
            }
            s -= nb;
        } else {
            const uint32_t nb = ((uint32_t)w.tiles_x + IS_W - 1) / IS_W;
            const uint32_t cnt = nb * (uint32_t)w.tiles_y;
            if (s < cnt) {
                const uint32_t ty = s / nb, k = s % nb;
                g.lo_off = (int)k * IS_W;
                g.width = min(IS_W, w.tiles_x - g.lo_off);
                g.bucket0 = w.tile_base + ty * (uint32_t)w.tiles_x + (uint32_t)g.lo_off;
                const uint32_t r = row_base + ty;
                const uint32_t listed = *a.items_listed;
                const uint32_t b0 = a.row_start[r], b1 = b0 + a.row_count[r];
                g.begin = b0 < listed ? b0 : listed;
                g.end = b1 < listed ? b1 : listed;
                return g;
            }
            s -= cnt;
        }
        row_base += (uint32_t)w.tiles_y;
    }
    g.begin = g.end = 0;
    g.bucket0 = 0;
    g.lo_off = 0;
    g.width = 0;
    return g;
}

// Item idx of a segment: its value and its bucket interval [a0, a1] (empty when
// a0 > a1) before windowing, and (level 1) the rectangle's columns.  Both
// inputs are read in item order (coalesced).
template <int LEVEL>
__device__ __forceinline__ void load_item(const IsArgs& a, uint32_t idx, uint32_t end, uint32_t& p, int& a0,
                                          int& a1, uint32_t& cols) {
    p = 0xFFFFFFFFu;
    a0 = 1;
    a1 = 0;
    cols = 0;
    if (idx >= end) return;
    p = a.items[idx];
    if (LEVEL == 1) {
        const uint2 r = a.item_rect[idx];
        if (r.x == 0xFFFFFFFFu) return;
        a0 = (int)(r.x >> 16);
        a1 = (int)(r.y >> 16);
        cols = (r.x & 0xFFFFu) | (r.y << 16);
    } else {
        const uint32_t c = a.item_cols[idx];
        a0 = (int)(c & 0xFFFFu);
        a1 = (int)(c >> 16);
    }
}

// Wave-wide integer reductions from one ballot per bit of x (x < 2^BITS):
// scalar and lane-count arithmetic only, no cross-lane data movement.
// Exclusive prefix of x over the lanes below this one; the wave total in *total.
template <int BITS>
__device__ __forceinline__ uint32_t wave_prefix_bits(uint32_t x, uint32_t* total) {
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < BITS; ++k) {
        const uint64_t b = __ballot((x >> k) & 1u);
        pre += __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u)) << k;
        tot += (uint32_t)__popcll(b) << k;
    }
    *total = tot;
    return pre;
}

// Maximum of x over the wave (wave-uniform).
template <int BITS>
__device__ __forceinline__ uint32_t wave_max_bits(uint32_t x) {
    uint64_t cand = __ballot(true);
    uint32_t m = 0;
#pragma unroll
    for (int k = BITS - 1; k >= 0; --k) {
        const uint64_t b = __ballot((x >> k) & 1u) & cand;
        if (b != 0ull) {
            m |= 1u << k;
            cand = b;
        }
    }
    return m;
}

// Chunk id -> segment: the largest s with chunk_off[s] <= cg.
__device__ __forceinline__ uint32_t chunk_segment(const uint32_t* chunk_off, uint32_t nseg, uint32_t cg) {
    uint32_t lo = 0, hi = nseg;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (chunk_off[mid] <= cg) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Number of chunks of every segment.
template <int LEVEL>
__global__ __launch_bounds__(256) void k_is_seg_chunks(IsArgs a, uint32_t* chunks) {
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= a.nseg) return;
    const Seg g = locate_segment<LEVEL>(a, s);
    chunks[s] = (g.end - g.begin + IS_CHUNK - 1) / IS_CHUNK;
}

// Inclusive prefix over the IS_W entries row[0..IS_W) by one wave (two per
// lane), for entries in [-OFF, 2^BITS / 2 - OFF): the lane sums (offset to be
// non-negative) are prefixed by one ballot per bit (no cross-lane shuffles).
template <int BITS, int OFF>
__device__ __forceinline__ void wave_prefix_row(int* row) {
    const uint32_t lane = __lane_id();
    const int x0 = row[2 * lane], x1 = row[2 * lane + 1];
    const uint32_t v = (uint32_t)(x0 + x1 + 2 * OFF);  // < 2^BITS
    uint32_t tot;
    const int ex = (int)(wave_prefix_bits<BITS>(v, &tot) - 2u * OFF * lane);
    row[2 * lane] = ex + x0;
    row[2 * lane + 1] = ex + x0 + x1;
}

// Count pass (MODE 0) and scatter pass (MODE 1) over the chunks; persistent
// blocks stride over the device-side chunk count.  The count pass takes
// per-wave bucket counts from difference arrays (+1 at lo, -1 at hi + 1;
// integer LDS atomics, order free).  The scatter marks membership in bitmaps,
// one bit per (bucket, chunk item): setting bits is order free (LDS OR
// atomics), and reading a bucket's bits in index order yields its entries in
// item order, so no ranks are computed.  Level 2 writes each bucket's entries
// from its bits (long runs through a per-wave stage); level 1, whose entries
// also get their row's columns (about 130 instructions each), first unpacks
// the bits into an LDS stage grouped by bucket (at most IS_STAGE entries at a
// time, bucket windows) and computes the columns over the window's entries
// with all threads of the block.
constexpr int IS_STAGE = 4096;
// Bitmap rows are padded to 65 words, so lanes setting bits of one item word in
// different buckets mostly fall in different banks.
constexpr int IS_BM_STRIDE = IS_CHUNK / 32 + 1;
// Level 2 writes a bucket's run straight from its bits when the run is short;
// a longer one (up to IS_WSTAGE entries) is unpacked into a per-wave LDS stage
// first and written coalesced (the direct writes scatter one value per lane
// over the run, as many stores as the fullest bitmap word has bits).
constexpr int IS_WSTAGE = 512;
constexpr int IS_WSTAGE_MIN = 96;

template <int LEVEL, int MODE>
__global__ __launch_bounds__(IS_THREADS) __attribute__((amdgpu_waves_per_eu(8))) void k_is_chunks(IsArgs a) {
    __shared__ int s_cnt[MODE == 0 ? IS_WAVES : 1][IS_W + 1];
    __shared__ uint32_t s_ls[IS_W + 1];  // chunk-local first entry of each bucket
    __shared__ uint32_t s_gb[IS_W];      // global position of that entry
    __shared__ uint32_t s_bm[MODE == 1 ? IS_W * IS_BM_STRIDE : 1];
    // level 2: a stage per wave for one bucket's run
    __shared__ uint32_t s_wst[LEVEL == 2 && MODE == 1 ? IS_WAVES * IS_WSTAGE : 1];
    // level 1: chunk-local item index | bucket << 11, grouped by bucket
    static_assert(IS_CHUNK <= 2048, "chunk-local item indices take 11 bits");
    __shared__ uint32_t s_stage[LEVEL == 1 && MODE == 1 ? IS_STAGE : 1];
    // the chunk's item values (level 1: and rectangle columns)
    __shared__ uint32_t s_item_p[MODE == 1 ? IS_CHUNK : 1];
    __shared__ uint32_t s_item_c[LEVEL == 1 && MODE == 1 ? IS_CHUNK : 1];
    const uint32_t lane = __lane_id(), wave = threadIdx.x / 64;
    const uint32_t item0 = wave * (64 * IS_IPL) + lane;  // chunk-local index of this lane's first item
    // a contiguous share of the chunks per block: the segment is looked up once
    // and the next chunk's items are loaded while the current one is processed
    const uint32_t total = min<uint64_t>(*a.chunk_total, a.mat_chunks);
    const uint32_t per = (total + gridDim.x - 1) / gridDim.x;
    const uint32_t cbeg = blockIdx.x * per, cend = min(cbeg + per, total);
    if (cbeg >= cend) return;
    uint32_t s = chunk_segment(a.chunk_off, a.nseg, cbeg);
    uint32_t s_first = a.chunk_off[s], s_next = a.chunk_off[s + 1];
    Seg g = locate_segment<LEVEL>(a, s);
    uint32_t idx = g.begin + (cbeg - s_first) * IS_CHUNK + item0;
    uint32_t p[IS_IPL], cols[IS_IPL];
    int a0[IS_IPL], a1[IS_IPL];
#pragma unroll
    for (int u = 0; u < IS_IPL; ++u) load_item<LEVEL>(a, idx + 64 * u, g.end, p[u], a0[u], a1[u], cols[u]);
    for (uint32_t cg = cbeg; cg < cend;) {
        // bucket bases of this chunk (scatter) are independent of the LDS work below
        uint32_t gb = 0;
        if (MODE == 1 && threadIdx.x < (uint32_t)g.width)
            gb = a.bucket_start[g.bucket0 + threadIdx.x] + a.mat[(uint64_t)cg * IS_W + threadIdx.x];
        int lo[IS_IPL], hi[IS_IPL];
        bool any[IS_IPL];
#pragma unroll
        for (int u = 0; u < IS_IPL; ++u) {
            lo[u] = max(a0[u] - g.lo_off, 0);
            hi[u] = min(a1[u] - g.lo_off, g.width - 1);
            any[u] = lo[u] <= hi[u];
        }
        const bool same = cg + 1 < cend && cg + 1 < s_next;
        const uint32_t idx_n = idx + IS_CHUNK;
        // the next chunk's items are loaded now, except by the level-1 scatter,
        // whose gathers in the copy-out need the registers (it loads them last)
        constexpr bool EARLY = !(LEVEL == 1 && MODE == 1);
        uint32_t p_n[IS_IPL], cols_n[IS_IPL];
        int a0_n[IS_IPL], a1_n[IS_IPL];
        if (EARLY) {
#pragma unroll
            for (int u = 0; u < IS_IPL; ++u)
                load_item<LEVEL>(a, idx_n + 64 * u, same ? g.end : 0u, p_n[u], a0_n[u], a1_n[u], cols_n[u]);
        }
        if constexpr (MODE == 0) {
            for (int j = threadIdx.x; j < IS_WAVES * (IS_W + 1); j += IS_THREADS) (&s_cnt[0][0])[j] = 0;
            __syncthreads();
#pragma unroll
            for (int u = 0; u < IS_IPL; ++u)
                if (any[u]) {
                    atomicAdd(&s_cnt[wave][lo[u]], 1);
                    atomicAdd(&s_cnt[wave][hi[u] + 1], -1);
                }
            __syncthreads();
            wave_prefix_row<10, 128>(s_cnt[wave]);  // s_cnt[w][b]: items of wave w covering bucket b
            __syncthreads();
            if (threadIdx.x < (uint32_t)g.width) {
                int acc = 0;
#pragma unroll
                for (int w = 0; w < IS_WAVES; ++w) acc += s_cnt[w][threadIdx.x];
                a.mat[(uint64_t)cg * IS_W + threadIdx.x] = (uint32_t)acc;
            }
        } else {
            for (int j = threadIdx.x; j < IS_W * IS_BM_STRIDE; j += IS_THREADS) s_bm[j] = 0u;
#pragma unroll
            for (int u = 0; u < IS_IPL; ++u) {
                s_item_p[item0 + 64 * u] = p[u];
                if (LEVEL == 1) s_item_c[item0 + 64 * u] = cols[u];
            }
            if (threadIdx.x < IS_W) s_gb[threadIdx.x] = gb;
            __syncthreads();
            // membership bits, lane-serial over the intervals (as long as the
            // wave's longest)
#pragma unroll
            for (int u = 0; u < IS_IPL; ++u) {
                const uint32_t item = item0 + 64u * (uint32_t)u;
                const uint32_t nn = any[u] ? (uint32_t)(hi[u] - lo[u] + 1) : 0u;  // <= IS_W
                const uint32_t mx = wave_max_bits<8>(nn);
                uint32_t* row = s_bm + (item >> 5) + (uint32_t)lo[u] * IS_BM_STRIDE;
                const uint32_t bit = 1u << (item & 31u);
                for (uint32_t k = 0; k < mx; ++k)
                    if (k < nn) atomicOr(row + k * IS_BM_STRIDE, bit);
            }
            __syncthreads();
            if constexpr (LEVEL == 2) {
                // a wave per bucket: lane l holds the bits of items 32 l .. 32 l + 31
                uint32_t* wst = s_wst + wave * IS_WSTAGE;
                for (int b = (int)wave; b < g.width; b += IS_WAVES) {
                    uint32_t bits = s_bm[b * IS_BM_STRIDE + lane];
                    uint32_t n_b;
                    const uint32_t pre = wave_prefix_bits<6>((uint32_t)__popc(bits), &n_b);
                    uint32_t pos = s_gb[b] + pre;
                    const uint32_t key = g.bucket0 + (uint32_t)b;
                    if (n_b > (uint32_t)IS_WSTAGE_MIN && n_b <= (uint32_t)IS_WSTAGE) {
                        // unpack into the wave's stage, then write the run coalesced
                        uint32_t q = pre;
                        while (bits != 0u) {
                            const uint32_t k = (uint32_t)__builtin_ctz(bits);
                            bits &= bits - 1u;
                            wst[q++] = s_item_p[lane * 32u + k];
                        }
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        const uint32_t dst = s_gb[b];
                        for (uint32_t j = lane; j < n_b; j += 64) {
                            if (dst + j < a.out_cap) {
                                a.out_vals[dst + j] = wst[j];
                                if (a.out_keys) a.out_keys[dst + j] = key;
                            }
                        }
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        continue;
                    }
                    while (bits != 0u) {
                        const uint32_t k = (uint32_t)__builtin_ctz(bits);
                        bits &= bits - 1u;
                        if (pos < a.out_cap) {
                            a.out_vals[pos] = s_item_p[lane * 32u + k];
                            if (a.out_keys) a.out_keys[pos] = key;
                        }
                        ++pos;
                    }
                }
            } else {
                // chunk-local bucket starts from the bitmap rows' populations
                for (int b = (int)wave; b < IS_W; b += IS_WAVES) {
                    const uint32_t c = b < g.width ? (uint32_t)__popc(s_bm[b * IS_BM_STRIDE + lane]) : 0u;
                    uint32_t t;
                    wave_prefix_bits<6>(c, &t);
                    if (lane == 0) s_ls[b + 1] = t;
                }
                if (threadIdx.x == 0) s_ls[0] = 0u;
                __syncthreads();
                if (wave == 0) wave_prefix_row<13, 0>(reinterpret_cast<int*>(s_ls + 1));
                __syncthreads();
                for (int b0 = 0; b0 < g.width;) {
                    // largest b1 with the window's entries fitting the stage (one
                    // bucket holds at most IS_CHUNK <= IS_STAGE entries)
                    int l = b0 + 1, h = g.width;
                    while (l < h) {
                        const int mid = (l + h + 1) >> 1;
                        if (s_ls[mid] - s_ls[b0] <= (uint32_t)IS_STAGE) l = mid;
                        else h = mid - 1;
                    }
                    const int b1 = l;
                    const uint32_t off0 = s_ls[b0];
                    for (int b = b0 + (int)wave; b < b1; b += IS_WAVES) {
                        uint32_t bits = s_bm[b * IS_BM_STRIDE + lane];
                        uint32_t n_b;
                        uint32_t q = s_ls[b] - off0 + wave_prefix_bits<6>((uint32_t)__popc(bits), &n_b);
                        while (bits != 0u) {
                            const uint32_t k = (uint32_t)__builtin_ctz(bits);
                            bits &= bits - 1u;
                            s_stage[q++] = (lane * 32u + k) | ((uint32_t)b << 11);
                        }
                    }
                    __syncthreads();
                    // the window's entries over all threads of the block, two per
                    // thread at a time so their ellipse gathers are in flight
                    // together; each gets the columns of its pair's rectangle that
                    // the ellipse reaches in the entry's row (view row g.lo_off + b)
                    const uint32_t wn = s_ls[b1] - off0;
                    const float4* ell = a.item_ell + 2 * (size_t)(idx - item0);
                    for (uint32_t i0 = threadIdx.x; i0 < wn; i0 += 2 * IS_THREADS) {
                        uint32_t w[2];
                        float4 e0[2], e1[2];
#pragma unroll
                        for (int r = 0; r < 2; ++r) {
                            const uint32_t i = i0 + (uint32_t)r * IS_THREADS;
                            w[r] = i < wn ? s_stage[i] : 0u;
                        }
#pragma unroll
                        for (int r = 0; r < 2; ++r) {
                            const uint32_t i = i0 + (uint32_t)r * IS_THREADS;
                            const uint32_t li = w[r] & (uint32_t)(IS_CHUNK - 1);
                            if (i < wn && a.item_ell != nullptr) {
                                e0[r] = ell[2 * li];
                                e1[r] = ell[2 * li + 1];
                            }
                        }
#pragma unroll
                        for (int r = 0; r < 2; ++r) {
                            const uint32_t i = i0 + (uint32_t)r * IS_THREADS;
                            if (i >= wn) continue;
                            const uint32_t li = w[r] & (uint32_t)(IS_CHUNK - 1), b = w[r] >> 11;
                            const uint32_t pos = s_gb[b] + (i + off0 - s_ls[b]);
                            if (pos < a.out_cap) {
                                uint32_t c = s_item_c[li];
                                if (a.item_ell != nullptr)
                                    c = row_columns(e0[r], e1[r], g.lo_off + (int)b, a.tile_w, a.tile_h,
                                                    (int)(c & 0xFFFFu), (int)(c >> 16));
                                a.out_vals[pos] = s_item_p[li];
                                a.out_cols[pos] = c;
                                if (a.out_keys) a.out_keys[pos] = g.bucket0 + b;
                            }
                        }
                    }
                    __syncthreads();
                    b0 = b1;
                }
            }
        }
        __syncthreads();
        ++cg;
        if (cg >= cend) break;
        if (same) {
            idx = idx_n;
            if (EARLY) {
#pragma unroll
                for (int u = 0; u < IS_IPL; ++u) {
                    p[u] = p_n[u];
                    cols[u] = cols_n[u];
                    a0[u] = a0_n[u];
                    a1[u] = a1_n[u];
                }
            } else {
#pragma unroll
                for (int u = 0; u < IS_IPL; ++u) load_item<LEVEL>(a, idx + 64 * u, g.end, p[u], a0[u], a1[u], cols[u]);
            }
        } else {
            while (cg >= s_next) {
                ++s;
                s_first = s_next;
                s_next = a.chunk_off[s + 1];
            }
            g = locate_segment<LEVEL>(a, s);
            idx = g.begin + (cg - s_first) * IS_CHUNK + item0;
#pragma unroll
            for (int u = 0; u < IS_IPL; ++u) load_item<LEVEL>(a, idx + 64 * u, g.end, p[u], a0[u], a1[u], cols[u]);
        }
    }
}

// Per (segment, bucket): exclusive scan of the chunk counts over the
// segment's chunks (in place) and the bucket total.  Eight threads per bucket
// each take a contiguous share of the chunks.
constexpr int IS_PARTS = 8;

template <int LEVEL>
__global__ __launch_bounds__(IS_W * IS_PARTS) void k_is_prefix(IsArgs a) {
    __shared__ uint32_t s_part[IS_PARTS][IS_W];
    const uint32_t s = blockIdx.x, b = threadIdx.x % IS_W, part = threadIdx.x / IS_W;
    const Seg g = locate_segment<LEVEL>(a, s);
    const uint32_t c0 = a.chunk_off[s];
    const uint32_t c1 = min<uint64_t>(a.chunk_off[s + 1], a.mat_chunks);
    const uint32_t nch = c1 > c0 ? c1 - c0 : 0u;
    const uint32_t per = (nch + IS_PARTS - 1) / IS_PARTS;
    const uint32_t r0 = c0 + min(part * per, nch), r1 = c0 + min((part + 1) * per, nch);
    const bool live = (int)b < g.width;
    uint32_t sum = 0;
    if (live)
        for (uint32_t c = r0; c < r1; ++c) sum += a.mat[(uint64_t)c * IS_W + b];
    s_part[part][b] = sum;
    __syncthreads();
    if (!live) return;
    uint32_t acc = 0;
    for (uint32_t q = 0; q < part; ++q) acc += s_part[q][b];
    for (uint32_t c = r0; c < r1; ++c) {
        const uint32_t x = a.mat[(uint64_t)c * IS_W + b];
        a.mat[(uint64_t)c * IS_W + b] = acc;
        acc += x;
    }
    if (part == IS_PARTS - 1) a.bucket_count[g.bucket0 + b] = acc;
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

// Worklist key: more work first (descending, ties by tile id); the work is the
// list length, or a previous forward's evaluated positions when given.
__global__ __launch_bounds__(256) void k_worklist_keys(const uint32_t* ranges, const uint32_t* work,
                                                       uint64_t total_tiles, uint32_t* keys) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total_tiles) return;
    const uint32_t len = work ? work[t] : ranges[2 * t + 1] - ranges[2 * t];
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
    if (count <= (uint64_t)SCAN_TOP_MAX) {  // one launch
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, stream, in, out, (uint32_t)count, total);
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
                      bool* result_in_b, hipStream_t stream, uint32_t view_n) {
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
        const int sh = p * radix_bits;
        // the view enters the digits of the passes reaching past the 32 key bits
        const uint32_t vn = sh + radix_bits > 32 ? view_n : 0u;
        switch (radix_bits) {
            case 4: e = sort_pass<4>(kin, vin, kout, vout, count_static, count_dev, sh, vn, b, stream); break;
            case 5: e = sort_pass<5>(kin, vin, kout, vout, count_static, count_dev, sh, vn, b, stream); break;
            case 6: e = sort_pass<6>(kin, vin, kout, vout, count_static, count_dev, sh, vn, b, stream); break;
            case 7: e = sort_pass<7>(kin, vin, kout, vout, count_static, count_dev, sh, vn, b, stream); break;
            default: e = sort_pass<8>(kin, vin, kout, vout, count_static, count_dev, sh, vn, b, stream); break;
        }
        if (e != hipSuccess) return e;
        kin = kout;
        vin = vout;
        in_b = (p & 1);
    }
    *result_in_b = in_b;
    return hipSuccess;
}

hipError_t launch_gather_rects(const uint32_t* order, const float* rec, uint64_t count, uint2* out, float4* ell,
                               hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rects, grid_for(count), dim3(256), 0, stream, order, rec, count, out, ell);
    return hipGetLastError();
}

uint32_t is_segments(const DevCams& cams, int level) {
    uint32_t s = 0;
    for (int v = 0; v < cams.V; ++v) {
        const DevView& w = cams.v[v];
        if (level == 1) s += ((uint32_t)w.tiles_y + IS_W - 1) / IS_W;
        else s += ((uint32_t)w.tiles_x + IS_W - 1) / IS_W * (uint32_t)w.tiles_y;
    }
    return s;
}

uint64_t is_chunk_bound(const DevCams& cams, int level, int n, uint64_t level2_items) {
    uint64_t c = 0;
    if (level == 1) {
        c = (uint64_t)is_segments(cams, 1) * (((uint64_t)n + IS_CHUNK - 1) / IS_CHUNK);
    } else {
        uint32_t nb_max = 1;
        for (int v = 0; v < cams.V; ++v) {
            const uint32_t nb = ((uint32_t)cams.v[v].tiles_x + IS_W - 1) / IS_W;
            if (nb > nb_max) nb_max = nb;
        }
        c = is_segments(cams, 2) + nb_max * ((level2_items + IS_CHUNK - 1) / IS_CHUNK);
    }
    return c > 0 ? c : 1;
}

uint32_t is_window() { return IS_W; }

hipError_t launch_interval_scatter(IsArgs a, int level, uint32_t n_buckets, uint32_t* bucket_total,
                                   uint32_t* seg_chunks, uint32_t* scan_partials, hipStream_t stream) {
    a.nseg = is_segments(a.cams, level);
    if (a.nseg == 0) return hipSuccess;
    const uint32_t grid = (uint32_t)(a.mat_chunks < 1024 ? a.mat_chunks : 1024);
    auto seg_k = level == 1 ? k_is_seg_chunks<1> : k_is_seg_chunks<2>;
    hipLaunchKernelGGL(seg_k, dim3((a.nseg + 255) / 256), dim3(256), 0, stream, a, seg_chunks);
    // chunk_off = exclusive scan of the chunk counts (nseg + 1 entries: the
    // last one, from a zero count, is the total)
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, stream, seg_chunks + a.nseg, 0u, (uint64_t)1);
    hipError_t e = scan_exclusive(seg_chunks, const_cast<uint32_t*>(a.chunk_off), (uint64_t)a.nseg + 1, scan_partials,
                                  const_cast<uint32_t*>(a.chunk_total), stream);
    if (e != hipSuccess) return e;
    auto count_k = level == 1 ? k_is_chunks<1, 0> : k_is_chunks<2, 0>;
    hipLaunchKernelGGL(count_k, dim3(grid), dim3(IS_THREADS), 0, stream, a);
    auto prefix_k = level == 1 ? k_is_prefix<1> : k_is_prefix<2>;
    hipLaunchKernelGGL(prefix_k, dim3(a.nseg), dim3(IS_W * IS_PARTS), 0, stream, a);
    e = scan_exclusive(a.bucket_count, const_cast<uint32_t*>(a.bucket_start), n_buckets, scan_partials, bucket_total,
                       stream);
    if (e != hipSuccess) return e;
    auto scatter_k = level == 1 ? k_is_chunks<1, 1> : k_is_chunks<2, 1>;
    hipLaunchKernelGGL(scatter_k, dim3(grid), dim3(IS_THREADS), 0, stream, a);
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

hipError_t launch_worklist_keys(const uint32_t* ranges, const uint32_t* work, uint64_t total_tiles, uint32_t* keys,
                                hipStream_t stream) {
    if (total_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_worklist_keys, grid_for(total_tiles), dim3(256), 0, stream, ranges, work, total_tiles, keys);
    return hipGetLastError();
}

hipError_t launch_l1_grad(const float* image, const float* target, uint64_t count, float scale, float* grad,
                          hipStream_t stream) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_l1_grad, grid_for(count), dim3(256), 0, stream, image, target, count, scale, grad);
    return hipGetLastError();
}

}  // namespace gesr
