// K6: forward rendering of Magnetic Gaussians onto voxel tiles (Eq. 7; on stacks the
// Gaussian is pre-convolved with the slice profile, so the same formula applies with the
// record's amplitude and conic).
//
// One wavefront owns one GM_TX x GM_TY x GM_TZ tile and accumulates it in LDS.  It walks
// the tile's Gaussian list (ascending id) in batches of 64 records staged in LDS; for each
// Gaussian the lanes take the voxels of (box intersect tile) densely, evaluate
// amp * 2^(delta^T K delta) and add it into the tile accumulator.  Within one Gaussian every
// lane holds a different voxel, and Gaussians are taken one after another, so each voxel's
// sum is formed in ascending Gaussian order and the result is the same on every run.
#include "gm_internal.h"

namespace {

__device__ __forceinline__ int sgpr(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float sgprf(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__global__ __launch_bounds__(64) void k_render(const RenderArgs a)
{
    __shared__ float acc[GM_TILE_VOX];
    __shared__ float4 rec[64 * 4];
    const int lane = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    int r = 0;
#pragma unroll 1
    while (r + 1 < a.n_render && blk >= a.rg[r + 1].first_block) ++r;
    const RenderGrid& G = a.rg[r];
    const int lt = blk - G.first_block;
    const int tx = lt % G.ntx, ty = (lt / G.ntx) % G.nty, tz = lt / (G.ntx * G.nty);
    const int t0x = tx * GM_TX, t0y = ty * GM_TY, t0z = tz * GM_TZ;

#pragma unroll
    for (int i = lane; i < GM_TILE_VOX; i += 64) acc[i] = 0.0f;

    const int64_t bt = G.bin_tile_base + lt;
    const int s = sgpr(a.tile_start[bt]);
    const int e = sgpr(a.tile_start[bt + 1]);
    const float* recbase = a.records + (size_t)G.grid_index * a.n_gauss * 16;

#pragma unroll 1
    for (int b0 = s; b0 < e; b0 += 64) {
        const int nb = min(64, e - b0);
        __syncthreads();
        if (lane < nb) {
            const int gid = a.pair_gauss[b0 + lane];
            const float4* src = reinterpret_cast<const float4*>(recbase + (size_t)gid * 16);
            rec[lane * 4 + 0] = src[0];
            rec[lane * 4 + 1] = src[1];
            rec[lane * 4 + 2] = src[2];
            rec[lane * 4 + 3] = src[3];
        }
        __syncthreads();
#pragma unroll 1
        for (int j = 0; j < nb; ++j) {
            const float4 r0 = rec[j * 4 + 0];
            const float4 r1 = rec[j * 4 + 1];
            const float4 r2 = rec[j * 4 + 2];
            const float4 r3 = rec[j * 4 + 3];
            const int lox = sgpr(__float_as_int(r2.z)), loy = sgpr(__float_as_int(r2.w));
            const int loz = sgpr(__float_as_int(r3.x));
            const int hix = sgpr(__float_as_int(r3.y)), hiy = sgpr(__float_as_int(r3.z));
            const int hiz = sgpr(__float_as_int(r3.w));
            const int ix0 = max(lox, t0x), iy0 = max(loy, t0y), iz0 = max(loz, t0z);
            const int wx = min(hix, t0x + GM_TX - 1) - ix0 + 1;
            const int wy = min(hiy, t0y + GM_TY - 1) - iy0 + 1;
            const int wz = min(hiz, t0z + GM_TZ - 1) - iz0 + 1;
            if (wx <= 0 || wy <= 0 || wz <= 0) continue;  // cannot happen for a listed tile
            const int wxy = wx * wy;
            const int V = wxy * wz;
            const float inv_wxy = __builtin_amdgcn_rcpf((float)wxy);
            const float inv_wx = __builtin_amdgcn_rcpf((float)wx);
            // offsets of the intersection from the box origin (for delta) and tile origin
            const int bx = ix0 - lox, by = iy0 - loy, bz = iz0 - loz;
            const int ox = ix0 - t0x, oy = iy0 - t0y, oz = iz0 - t0z;
            const float cx = sgprf(r0.x), cy = sgprf(r0.y), cz = sgprf(r0.z);
            const float amp = sgprf(r0.w);
            const float kxx = sgprf(r1.x), kyy = sgprf(r1.y), kzz = sgprf(r1.z);
            const float kxy = sgprf(r1.w), kxz = sgprf(r2.x), kyz = sgprf(r2.y);
#pragma unroll 1
            for (int q = lane; q < V; q += 64) {
                const int z = (int)(((float)q + 0.5f) * inv_wxy);
                const int rm = q - z * wxy;
                const int y = (int)(((float)rm + 0.5f) * inv_wx);
                const int x = rm - y * wx;
                const float dx = (float)(x + bx) - cx;
                const float dy = (float)(y + by) - cy;
                const float dz = (float)(z + bz) - cz;
                const float Q = dx * (kxx * dx + kxy * dy + kxz * dz) + dy * (kyy * dy + kyz * dz) +
                                dz * (kzz * dz);
                const float w = amp * __builtin_amdgcn_exp2f(Q);
                atomicAdd(&acc[((z + oz) * GM_TY + (y + oy)) * GM_TX + (x + ox)], w);
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
