// K2-K5: exclusive scan of tile counts, (tile, Gaussian) key emission, stable LSD radix sort
// of the keys, and per-tile list ranges.  Together they list, for every voxel tile of every
// grid, the Gaussians whose box overlaps it in ascending Gaussian id (the spatial query that
// stands in for the paper's block partition, Sec. 3.3.1).
#include "gm_internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;
constexpr unsigned SCAN_PREFIX_BLOCKS = 2048;   // final-pass blocks that sum their own prefix

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ __launch_bounds__(256) void k_copy_u32(const uint32_t* src, uint32_t* dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// block-wide exclusive scan of one int64 per thread; returns the block total in *total
__device__ int64_t block_exclusive_scan(int64_t v, int64_t* total)
{
    __shared__ int64_t s_wave[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / 64; ++w) {
        const int64_t x = s_wave[w];
        if (w < wave) before += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const int32_t* in, int64_t n,
                                                               int64_t* part)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * SCAN_THREADS + threadIdx.x;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// The chunk totals part[0..nb) replaced by their exclusive prefix sums, in place: one block
// walks them SCAN_CHUNK at a time with a running offset (used when the final pass has too many
// blocks to sum the totals before it one by one).
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_parts(int64_t* part, int64_t nb)
{
    int64_t running = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += SCAN_CHUNK) {
        const int64_t base = c0 + (int64_t)threadIdx.x * SCAN_ITEMS;
        int64_t v[SCAN_ITEMS];
        int64_t sum = 0;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            v[k] = base + k < nb ? part[base + k] : 0;
            sum += v[k];
        }
        int64_t tot;
        int64_t run = block_exclusive_scan(sum, &tot) + running;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            if (base + k < nb) part[base + k] = run;
            run += v[k];
        }
        running += tot;
    }
}

// prefixed: part holds the exclusive prefix sums of the chunk totals (k_scan_parts ran);
// otherwise each block sums the totals before it.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_final(const int32_t* in, int64_t n,
                                                              const int64_t* part,
                                                              int64_t* out, int prefixed)
{
    // each thread owns SCAN_ITEMS consecutive elements of the block's chunk, moved with
    // 16-byte loads and stores where the chunk is whole and the buffers are aligned
    static_assert(SCAN_ITEMS == 8, "vector path moves 8 elements per thread");
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    const bool vec = base + SCAN_ITEMS <= n && ((uintptr_t)in & 31u) == 0 &&
                     ((uintptr_t)out & 15u) == 0;
    int32_t v[SCAN_ITEMS];
    if (vec) {
        const int4 a = *reinterpret_cast<const int4*>(in + base);
        const int4 b = *reinterpret_cast<const int4*>(in + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            const int64_t i = base + k;
            v[k] = i < n ? in[i] : 0;
        }
    }
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
    // this block's offset: the sum of the chunk totals before it (read from L2; integer,
    // so the order of the sum does not matter), or its prefix when the totals were scanned
    int64_t before;
    if (prefixed) {
        before = part[blockIdx.x];
    } else {
        int64_t pre = 0;
        for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += SCAN_THREADS) pre += part[b];
        block_exclusive_scan(pre, &before);
    }
    int64_t tot;
    int64_t run = block_exclusive_scan(s, &tot) + before;
    int64_t r[SCAN_ITEMS];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        r[k] = run;
        run += v[k];
    }
    if (vec) {
        longlong2* o = reinterpret_cast<longlong2*>(out + base);
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS / 2; ++k) o[k] = make_longlong2(r[2 * k], r[2 * k + 1]);
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k)
            if (base + k < n) out[base + k] = r[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) out[n] = run;
}

// Thread per (grid, Gaussian): write its overlapped tiles (z, y, x order) at its offset.
__global__ __launch_bounds__(256) void k_emit(const EmitArgs a)
{
    const int64_t total = (int64_t)a.n_grids * a.n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const uint32_t* tb = a.tile_box + idx * 3;
    const uint32_t b0 = tb[0], b1 = tb[1], b2 = tb[2];
    const int lx = (int)(b0 & 0xffffu), ly = (int)(b0 >> 16), lz = (int)(b1 & 0xffffu);
    const int hx = (int)(b1 >> 16), hy = (int)(b2 & 0xffffu), hz = (int)(b2 >> 16);
    if (hx < lx || hy < ly || hz < lz) return;  // empty box: no tile
    const int k = (int)(idx / a.n);
    const uint32_t gid = (uint32_t)(idx - (int64_t)k * a.n);
    const GridConst& G = a.g[k];
    int64_t o = a.offsets[idx];
    // the emission runs before the host has checked the total against the capacity
    if (o + (int64_t)(hx - lx + 1) * (hy - ly + 1) * (hz - lz + 1) > a.capacity) return;
    // the first tile emitted holds the box's lower corner: its entry carries GM_HOME_BIT
    uint32_t home = GM_HOME_BIT;
    for (int tz = lz; tz <= hz; ++tz)
        for (int ty = ly; ty <= hy; ++ty)
            for (int tx = lx; tx <= hx; ++tx) {
                a.keys[o] = (uint32_t)(G.tile_base + ((int64_t)tz * G.nty + ty) * G.ntx + tx);
                a.vals[o] = gid | home;
                home = 0u;
                ++o;
            }
}

// ---- radix sort --------------------------------------------------------------------------
// The scatter's block holds 4096 keys (32 KB of LDS for keys and values): eight waves of
// eight 64-key rounds, so that a CU keeps 24 waves (three blocks) in flight through the load
// and store bursts.
constexpr int RS_THREADS = 512;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ROUNDS = 8;
constexpr int RS_WAVE_KEYS = 64 * RS_ROUNDS;
constexpr int RS_BLOCK_KEYS = RS_WAVE_KEYS * RS_WAVES;
constexpr int RS_HIST_THREADS = 256;  // one per digit
static_assert(RS_BLOCK_KEYS % (4 * RS_HIST_THREADS) == 0, "whole 16-byte loads per thread");
static_assert(RS_THREADS >= 256 && RS_THREADS % 256 == 0, "the digit phase uses the first 256 threads");

// Digit counts of one scatter block's keys.  Each wave counts into its own LDS histogram
// (fewer colliding atomics), full blocks read four keys per 16-byte load and add each run of
// equal digits among a load's four keys once (keys emitted for Gaussians close in space share
// tiles, so runs are common and fewer lanes collide), and the four histograms are summed per
// digit at the end.
__global__ __launch_bounds__(RS_HIST_THREADS) void k_rs_hist(const uint32_t* keys, int64_t n,
                                                              int shift, uint32_t mask,
                                                              int32_t* ghist, int64_t nblocks)
{
    constexpr int HW = RS_HIST_THREADS / 64;
    __shared__ uint32_t h[HW][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = lane; d < 256; d += 64) h[wave][d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_BLOCK_KEYS;
    const int64_t rem = n - base;
    const int nk = rem < RS_BLOCK_KEYS ? (int)rem : RS_BLOCK_KEYS;
    uint32_t* hw = h[wave];
    if (nk == RS_BLOCK_KEYS && (reinterpret_cast<uintptr_t>(keys) & 15u) == 0) {
        const uint4* k4 = reinterpret_cast<const uint4*>(keys + base);
        uint4 v[RS_BLOCK_KEYS / 4 / RS_HIST_THREADS];
#pragma unroll
        for (int j = 0; j < RS_BLOCK_KEYS / 4 / RS_HIST_THREADS; ++j)
            v[j] = k4[threadIdx.x + j * RS_HIST_THREADS];
#pragma unroll
        for (int j = 0; j < RS_BLOCK_KEYS / 4 / RS_HIST_THREADS; ++j) {
            const uint32_t d0 = (v[j].x >> shift) & mask, d1 = (v[j].y >> shift) & mask;
            const uint32_t d2 = (v[j].z >> shift) & mask, d3 = (v[j].w >> shift) & mask;
            // run lengths from each key to the end of its run of equal digits
            const uint32_t l3 = 1u;
            const uint32_t l2 = d3 == d2 ? l3 + 1u : 1u;
            const uint32_t l1 = d2 == d1 ? l2 + 1u : 1u;
            const uint32_t l0 = d1 == d0 ? l1 + 1u : 1u;
            // each run counted once, at its first key
            atomicAdd(&hw[d0], l0);
            if (d1 != d0) atomicAdd(&hw[d1], l1);
            if (d2 != d1) atomicAdd(&hw[d2], l2);
            if (d3 != d2) atomicAdd(&hw[d3], l3);
        }
    } else {
        for (int k = threadIdx.x; k < nk; k += RS_HIST_THREADS)
            atomicAdd(&hw[(keys[base + k] >> shift) & mask], 1u);
    }
    __syncthreads();
    const int d = threadIdx.x;
    if (d <= (int)mask) {  // the pass's digits only: rows of the digit-major histogram
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < HW; ++w) t += h[w][d];
        ghist[(int64_t)d * nblocks + blockIdx.x] = (int32_t)t;
    }
}

// Stable scatter.  Wave w of the block owns keys [base + w*512, base + (w+1)*512) and takes
// them in 8 rounds of 64 consecutive keys; lanes with equal digits are matched with ballots,
// so every key learns how many equal-digit keys precede it in the block.  The block's keys are
// first placed in LDS in digit order, then written out by consecutive threads, so that each
// digit's run leaves the block as one contiguous stretch of stores.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint32_t* kin,
                                                            const uint32_t* vin, uint32_t* kout,
                                                            uint32_t* vout, int64_t n, int shift,
                                                            int dbits, const int64_t* goff,
                                                            int64_t nblocks)
{
    __shared__ uint32_t wcnt[RS_WAVES][256];
    __shared__ uint32_t wsum[RS_WAVES];
    __shared__ uint32_t dstart[256];
    __shared__ int64_t obase[256];
    __shared__ uint32_t skey[RS_BLOCK_KEYS];
    __shared__ uint32_t sval[RS_BLOCK_KEYS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t mask = (1u << dbits) - 1u;
    for (int d = lane; d < 256; d += 64) wcnt[wave][d] = 0;
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t bbase = (int64_t)blockIdx.x * RS_BLOCK_KEYS;
    const int64_t wbase = bbase + (int64_t)wave * RS_WAVE_KEYS;
    uint32_t key[RS_ROUNDS], val[RS_ROUNDS], rank[RS_ROUNDS];
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        const bool ok = i < n;
        key[r] = ok ? kin[i] : 0u;
        val[r] = ok ? vin[i] : 0u;
        const uint32_t dg = (key[r] >> shift) & mask;
        uint64_t peers = __ballot(ok);
        for (int b = 0; b < dbits; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt);
        uint32_t base = 0;
        if (ok) base = wcnt[wave][dg];
        rank[r] = base + before;
        if (ok && before == 0) wcnt[wave][dg] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: offsets of the waves' runs, the digit's block total, and its block-local
    // start (exclusive scan over the 256 digits: within each wave with shuffles, then across
    // the four waves)
    // (thread d < 256 takes digit d; waves 0-3 are whole, so the shuffles see full waves)
    const int d = threadIdx.x;
    const bool dig = d < 256;
    uint32_t run = 0, incl = 0;
    if (dig) {
#pragma unroll
        for (int w = 0; w < RS_WAVES; ++w) {
            const uint32_t t = wcnt[w][d];
            wcnt[w][d] = run;
            run += t;
        }
        incl = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wsum[wave] = incl;
    }
    __syncthreads();
    if (dig) {
        uint32_t before_w = 0;
        for (int w = 0; w < wave; ++w) before_w += wsum[w];
        const uint32_t ds = before_w + incl - run;
        dstart[d] = ds;
        obase[d] = d <= (int)mask ? goff[(int64_t)d * nblocks + blockIdx.x] - (int64_t)ds : 0;
    }
    __syncthreads();
    // place the keys in digit order in LDS (positions < RS_BLOCK_KEYS by construction)
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t i = wbase + r * 64 + lane;
        if (i < n) {
            const uint32_t dg = (key[r] >> shift) & mask;
            const uint32_t lp = dstart[dg] + wcnt[wave][dg] + rank[r];
            skey[lp] = key[r];
            sval[lp] = val[r];
        }
    }
    __syncthreads();
    const int64_t rem = n - bbase;
    const int nkeys = rem < RS_BLOCK_KEYS ? (int)rem : RS_BLOCK_KEYS;
    for (int i = threadIdx.x; i < nkeys; i += RS_THREADS) {
        const uint32_t k = skey[i];
        const int64_t pos = obase[(k >> shift) & mask] + i;
        kout[pos] = k;
        vout[pos] = sval[i];
    }
}

__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t* keys, int64_t n,
                                                      int32_t* start, int64_t T)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > T) return;
    int64_t lo = 0, hi = n;  // first index with keys[idx] >= t
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < (uint32_t)t) lo = mid + 1;
        else hi = mid;
    }
    start[t] = (int32_t)lo;
}

// One thread per grid: copy the box-volume totals accumulated in the scratch report block
// to the caller's box_volume array, and each grid's first list entry (the scan of the tile
// counts at the grid's first Gaussian; emission is grid-major and the sort keeps grids apart)
// next to them, so that gm_bin reads everything it reports back in one device-to-host copy.
// With `host` (pinned host memory) the whole report is also written there, so that the host
// reads it after a stream synchronisation without a copy.
__global__ void k_bin_report(BinReport* rep, const int64_t* offsets, int64_t n,
                             int64_t* box_volume, int n_grids, BinReport* host)
{
    const int k = threadIdx.x;
    if (k < n_grids) box_volume[k] = (int64_t)rep->box_volume[k];
    const int64_t gs = k <= n_grids ? offsets[(int64_t)k * n] : 0;
    if (k <= n_grids) rep->grid_start[k] = gs;
    if (host) {
        if (k <= GM_MAX_GRIDS) host->grid_start[k] = gs;
        if (k < GM_MAX_GRIDS) host->box_volume[k] = k < n_grids ? rep->box_volume[k] : 0ull;
        if (k < 4) host->flags[k] = rep->flags[k];
    }
}

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    unsigned nb = grid_for(n, 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(nb), dim3(256), 0, s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_bin_report(BinReport* rep, const int64_t* offsets, int64_t n,
                             int64_t* box_volume, int n_grids, BinReport* host, hipStream_t s)
{
    static_assert(GM_MAX_GRIDS < 64, "one thread per grid");
    hipLaunchKernelGGL(k_bin_report, dim3(1), dim3(64), 0, s, rep, offsets, n, box_volume,
                       n_grids, host);
    return hipGetLastError();
}

hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    unsigned nb = grid_for(n, 256);
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_copy_u32, dim3(nb), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

size_t scan_workspace_bytes(int64_t n)
{
    return (size_t)(grid_for(n > 0 ? n : 1, SCAN_CHUNK)) * sizeof(int64_t) + 256;
}

hipError_t launch_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* ws,
                                  hipStream_t s)
{
    if (n <= 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, reinterpret_cast<uint32_t*>(out),
                           0u, (int64_t)2);
        return hipGetLastError();
    }
    const unsigned nb = grid_for(n, SCAN_CHUNK);
    int64_t* part = reinterpret_cast<int64_t*>(ws);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, part);
    // up to SCAN_PREFIX_BLOCKS blocks each sum the totals before them (a few L2 reads per
    // thread); beyond, one more pass scans the totals so that the final pass stays linear
    const int prefixed = nb > SCAN_PREFIX_BLOCKS ? 1 : 0;
    if (prefixed)
        hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(SCAN_THREADS), 0, s, part, (int64_t)nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, part, out,
                       prefixed);
    return hipGetLastError();
}

hipError_t launch_emit(const EmitArgs& a, hipStream_t s)
{
    const int64_t total = (int64_t)a.n_grids * a.n;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit, dim3(grid_for(total, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

size_t radix_workspace_bytes(int64_t n)
{
    const int64_t nb = (n + RS_BLOCK_KEYS - 1) / RS_BLOCK_KEYS;
    const int64_t hn = 256 * (nb > 0 ? nb : 1);
    // ghist (int32), offsets (int64, hn + 1), scan partials
    return (size_t)hn * 4 + 256 + (size_t)(hn + 1) * 8 + 256 + scan_workspace_bytes(hn) + 256;
}

hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                             uint32_t* vals_alt, int64_t n, int bits, void* ws,
                             int* result_in_alt, hipStream_t s)
{
    *result_in_alt = 0;
    if (n <= 1 || bits <= 0) return hipSuccess;
    const int passes = (bits + 7) / 8;
    const int dbits = (bits + passes - 1) / passes;
    const int64_t nb = (n + RS_BLOCK_KEYS - 1) / RS_BLOCK_KEYS;
    const int64_t hn = 256 * nb;
    char* w = reinterpret_cast<char*>(ws);
    int32_t* ghist = reinterpret_cast<int32_t*>(w);
    w += ((size_t)hn * 4 + 255) / 256 * 256 + 256;
    int64_t* goff = reinterpret_cast<int64_t*>(w);
    w += ((size_t)(hn + 1) * 8 + 255) / 256 * 256 + 256;
    void* sws = w;
    uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    hipError_t err = hipSuccess;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * dbits;
        const int db = (bits - shift) < dbits ? (bits - shift) : dbits;
        const uint32_t mask = (1u << db) - 1u;
        // the histogram holds the pass's 2^db digit rows of nb block counts each
        const int64_t hrows = (int64_t)nb << db;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(RS_HIST_THREADS), 0, s, ki, n, shift,
                           mask, ghist, nb);
        err = launch_scan_i32_to_i64(ghist, goff, hrows, sws, s);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(RS_THREADS), 0, s, ki, vi, ko,
                           vo, n, shift, db, goff, nb);
        uint32_t* t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    *result_in_alt = (passes & 1);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t* sorted_keys, int64_t n_pairs, int32_t* tile_start,
                              int64_t total_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_tile_ranges, dim3(grid_for(total_tiles + 1, 256)), dim3(256), 0, s,
                       sorted_keys, n_pairs, tile_start, total_tiles);
    return hipGetLastError();
}
