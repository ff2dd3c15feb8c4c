// K13: devoxelization initialisation (Sec. 3.1: a uniform low-resolution grid of Gaussians
// initialised from the registered stacks; Fig. 1b).
//
// Gaussian i of a G^3 grid sits at the centre of cell (ix, iy, iz) of [-1,1]^3, with identity
// rotation and isotropic sigma = h/2 (h = 2/G).  Its intensity is the mean, over the stacks whose
// interpolation domain contains the centre, of the stack trilinearly sampled at the centre,
// scaled by h^3 / ((2 pi)^{3/2} sigma^3) so that the lattice of Gaussians sums back to the
// sampled intensity (partition of unity), clipped to [1e-3, 1 - 1e-3] and stored as a logit.
#include "gm_internal.h"

namespace {

__device__ float sample_trilinear(const float* __restrict__ v, int nx, int ny, int nz, float px,
                                  float py, float pz, bool* inside)
{
    *inside = px >= 0.0f && py >= 0.0f && pz >= 0.0f && px <= (float)(nx - 1) &&
              py <= (float)(ny - 1) && pz <= (float)(nz - 1);
    if (!*inside) return 0.0f;
    const int x0 = min((int)px, max(nx - 2, 0)), y0 = min((int)py, max(ny - 2, 0)),
              z0 = min((int)pz, max(nz - 2, 0));
    const int x1 = min(x0 + 1, nx - 1), y1 = min(y0 + 1, ny - 1), z1 = min(z0 + 1, nz - 1);
    const float fx = px - (float)x0, fy = py - (float)y0, fz = pz - (float)z0;
    auto at = [&](int x, int y, int z) { return v[((size_t)z * ny + y) * nx + x]; };
    const float c00 = at(x0, y0, z0) * (1.0f - fx) + at(x1, y0, z0) * fx;
    const float c10 = at(x0, y1, z0) * (1.0f - fx) + at(x1, y1, z0) * fx;
    const float c01 = at(x0, y0, z1) * (1.0f - fx) + at(x1, y0, z1) * fx;
    const float c11 = at(x0, y1, z1) * (1.0f - fx) + at(x1, y1, z1) * fx;
    const float c0 = c00 * (1.0f - fy) + c10 * fy;
    const float c1 = c01 * (1.0f - fy) + c11 * fy;
    return c0 * (1.0f - fz) + c1 * fz;
}

__global__ __launch_bounds__(256) void k_devox(const DevoxArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t G = a.g;
    if (i >= G * G * G) return;
    const int ix = (int)(i % G), iy = (int)((i / G) % G), iz = (int)(i / (G * G));
    const float h = 2.0f / (float)G;
    const float x = -1.0f + ((float)(2 * ix + 1)) / (float)G;
    const float y = -1.0f + ((float)(2 * iy + 1)) / (float)G;
    const float z = -1.0f + ((float)(2 * iz + 1)) / (float)G;
    float sum = 0.0f;
    int cnt = 0;
    for (int k = 0; k < a.n_stacks; ++k) {
        const GridConst& S = a.s[k];
        const float px = (float)(S.L[0] * x + S.L[1] * y + S.L[2] * z + S.t[0]);
        const float py = (float)(S.L[3] * x + S.L[4] * y + S.L[5] * z + S.t[1]);
        const float pz = (float)(S.L[6] * x + S.L[7] * y + S.L[8] * z + S.t[2]);
        bool in;
        const float v = sample_trilinear(a.data[k], S.nx, S.ny, S.nz, px, py, pz, &in);
        if (in) {
            sum += v;
            ++cnt;
        }
    }
    const float mean_v = cnt ? sum / (float)cnt : 0.0f;
    // h^3 / ((2 pi)^{3/2} (h/2)^3) = 8 / (2 pi)^{3/2}
    const float pu = 0.50794710f;
    const float alpha = fminf(fmaxf(mean_v * pu, 1e-3f), 1.0f - 1e-3f);
    a.mean[3 * i] = x;
    a.mean[3 * i + 1] = y;
    a.mean[3 * i + 2] = z;
    a.quat[4 * i] = 1.0f;
    a.quat[4 * i + 1] = 0.0f;
    a.quat[4 * i + 2] = 0.0f;
    a.quat[4 * i + 3] = 0.0f;
    const float ls = logf(0.5f * h);
    a.log_scale[3 * i] = ls;
    a.log_scale[3 * i + 1] = ls;
    a.log_scale[3 * i + 2] = ls;
    a.logit[i] = logf(alpha / (1.0f - alpha));
}

}  // namespace

hipError_t launch_devox(const DevoxArgs& a, hipStream_t s)
{
    const int64_t n = (int64_t)a.g * a.g * a.g;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_devox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}
