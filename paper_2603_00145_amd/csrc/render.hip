// K6: forward rendering of Magnetic Gaussians onto voxel tiles (Eq. 7; on stacks the
// Gaussian is pre-convolved with the slice profile, so the same formula applies with the
// record's amplitude and conic).
//
// One wavefront owns one GM_TX x GM_TY x GM_TZ tile and accumulates it in LDS.  It walks
// the tile's Gaussian list (ascending id) in batches of 64: each lane loads one record and
// prepares that Gaussian's piece (box intersect tile) in LDS; then, Gaussian after Gaussian,
// the lanes take the piece's voxels densely, evaluate amp * 2^(delta^T K delta) and add it
// into the tile accumulator.  Within one Gaussian every lane holds a different voxel, and
// Gaussians are taken one after another, so each voxel's sum is formed in ascending
// Gaussian order and the result is the same on every run.
#include "gm_internal.h"

namespace {

__device__ __forceinline__ int sgpr(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float sgprf(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Division by a per-Gaussian d in [1, 1024] of q in [0, 1024): floor(q / d) equals
// (q * M) >> 20 with M = ceil(2^20 / d), because q * d < 2^20.
__device__ __forceinline__ uint32_t magic20(uint32_t d) { return ((1u << 20) + d - 1u) / d; }
__device__ __forceinline__ uint32_t div20(uint32_t q, uint32_t M) { return __umul24(q, M) >> 20; }

// Per (Gaussian, tile) piece, prepared lane-parallel for a batch of 64 list entries:
// centre relative to the intersection origin, amplitude, base-2 conic, intersection size,
// magic divisors and the LDS offset of the intersection origin.
struct Piece {
    float ux, uy, uz, amp;
    float kxx, kyy, kzz, kxy;
    float kxz, kyz;
    int wx, wxy;
    int V, mx, mxy, base;
};

__global__ __launch_bounds__(64) void k_render(const RenderArgs a)
{
    __shared__ float acc[GM_TILE_VOX];
    __shared__ Piece pc[64];
    const int lane = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    int r = 0;
#pragma unroll 1
    while (r + 1 < a.n_render && blk >= a.rg[r + 1].first_block) ++r;
    const RenderGrid& G = a.rg[r];
    const int lt = blk - G.first_block;
    const int tx = lt % G.ntx, ty = (lt / G.ntx) % G.nty, tz = lt / (G.ntx * G.nty);
    const int t0x = tx * GM_TX, t0y = ty * GM_TY, t0z = tz * GM_TZ;
    const float* __restrict__ recbase = a.records + (size_t)G.grid_index * a.n_gauss * 16;
    const int* __restrict__ pg = a.pair_gauss;

#pragma unroll
    for (int i = lane; i < GM_TILE_VOX; i += 64) acc[i] = 0.0f;

    const int64_t bt = G.bin_tile_base + lt;
    const int s = sgpr(a.tile_start[bt]);
    const int e = sgpr(a.tile_start[bt + 1]);

#pragma unroll 1
    for (int b0 = s; b0 < e; b0 += 64) {
        const int nb = min(64, e - b0);
        __syncthreads();
        if (lane < nb) {
            const int gid = pg[b0 + lane];
            const float4* src = reinterpret_cast<const float4*>(recbase + (size_t)gid * 16);
            const float4 r0 = src[0], r1 = src[1], r2 = src[2], r3 = src[3];
            const int lox = __float_as_int(r2.z), loy = __float_as_int(r2.w);
            const int loz = __float_as_int(r3.x), hix = __float_as_int(r3.y);
            const int hiy = __float_as_int(r3.z), hiz = __float_as_int(r3.w);
            const int ix0 = max(lox, t0x), iy0 = max(loy, t0y), iz0 = max(loz, t0z);
            const int wx = min(hix, t0x + GM_TX - 1) - ix0 + 1;
            const int wy = min(hiy, t0y + GM_TY - 1) - iy0 + 1;
            const int wz = min(hiz, t0z + GM_TZ - 1) - iz0 + 1;
            const bool ok = wx > 0 && wy > 0 && wz > 0;  // always true for a listed tile
            Piece p;
            p.ux = r0.x - (float)(ix0 - lox);
            p.uy = r0.y - (float)(iy0 - loy);
            p.uz = r0.z - (float)(iz0 - loz);
            p.amp = r0.w;
            p.kxx = r1.x; p.kyy = r1.y; p.kzz = r1.z; p.kxy = r1.w;
            p.kxz = r2.x; p.kyz = r2.y;
            p.wx = ok ? wx : 1;
            p.wxy = ok ? wx * wy : 1;
            p.V = ok ? wx * wy * wz : 0;
            p.mx = (int)magic20((uint32_t)p.wx);
            p.mxy = (int)magic20((uint32_t)p.wxy);
            p.base = ((iz0 - t0z) * GM_TY + (iy0 - t0y)) * GM_TX + (ix0 - t0x);
            pc[lane] = p;
        }
        __syncthreads();
#pragma unroll 1
        for (int j = 0; j < nb; ++j) {
            const Piece p = pc[j];
            const int V = sgpr(p.V);
#pragma unroll 1
            for (int q0 = 0; q0 < V; q0 += 64) {
                const uint32_t q = (uint32_t)(q0 + lane);
                if (q < (uint32_t)V) {
                    const uint32_t z = div20(q, (uint32_t)p.mxy);
                    const uint32_t rm = q - __umul24(z, (uint32_t)p.wxy);
                    const uint32_t y = div20(rm, (uint32_t)p.mx);
                    const uint32_t x = rm - __umul24(y, (uint32_t)p.wx);
                    const float dx = (float)x - p.ux;
                    const float dy = (float)y - p.uy;
                    const float dz = (float)z - p.uz;
                    const float Q = dx * (p.kxx * dx + p.kxy * dy + p.kxz * dz) +
                                    dy * (p.kyy * dy + p.kyz * dz) + dz * (p.kzz * dz);
                    const float w = p.amp * __builtin_amdgcn_exp2f(Q);
                    // one wave owns the tile and the lanes of one Gaussian hold distinct
                    // voxels, so a plain read-add-write is race-free (and far faster than
                    // an LDS atomic)
                    static_assert(GM_TX == 16 && GM_TY == 16, "index shifts assume 16x16 tiles");
                    const int idx = p.base + (int)((z << 8) + (y << 4) + x);
                    acc[idx] += w;
                }
            }
        }
    }
    __syncthreads();
    float* out = G.out;
#pragma unroll
    for (int i = lane; i < GM_TILE_VOX; i += 64) {
        const int x = i % GM_TX, y = (i / GM_TX) % GM_TY, z = i / (GM_TX * GM_TY);
        const int gx = t0x + x, gy = t0y + y, gz = t0z + z;
        if (gx < G.nx && gy < G.ny && gz < G.nz)
            out[((size_t)gz * G.ny + gy) * G.nx + gx] = acc[i];
    }
}

}  // namespace

hipError_t launch_render(const RenderArgs& a, hipStream_t s)
{
    if (a.total_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_render, dim3((unsigned)a.total_blocks), dim3(64), 0, s, a);
    return hipGetLastError();
}
