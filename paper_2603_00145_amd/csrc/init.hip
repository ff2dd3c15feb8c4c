// K13: devoxelization initialisation (Sec. 3.1: a uniform low-resolution grid of Gaussians
// initialised from the registered stacks; Fig. 1b), and the lattice resolution transition of
// progressive training (Sec. 4.1.3).
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

// Resolution transition of progressive training (Sec. 4.1.3): Gaussian j of the new
// g1^3 lattice sits at its cell centre; intensity (alpha) and scale are trilinear in the old
// g0^3 lattice sampled at that centre in old cell-index units (clamped to the old centres),
// the scale then multiplied by g0 / g1 (one lattice cell per Gaussian, as at initialisation);
// the rotation is the normalised weighted sum of the eight corners' normalised quaternions,
// each brought into the hemisphere of the heaviest corner (the first of equal weights).
// Binary64 throughout; one thread per new Gaussian, corners read through the cache.
__device__ __forceinline__ void lattice_axis(int i, int g0, int g1, int* i0, int* i1,
                                             double* w0, double* w1)
{
    const double c = -1.0 + (2.0 * (double)i + 1.0) / (double)g1;   // new cell centre
    double u = (c + 1.0) * (double)g0 / 2.0 - 0.5;                  // old cell-index units
    u = fmin(fmax(u, 0.0), (double)(g0 - 1));
    int k0 = (int)floor(u);
    k0 = min(k0, max(g0 - 2, 0));
    const double f = u - (double)k0;
    *i0 = k0;
    *i1 = min(k0 + 1, g0 - 1);
    *w0 = 1.0 - f;
    *w1 = f;
}

__global__ __launch_bounds__(256) void k_upsample(const UpsampleArgs a)
{
    const int64_t g1 = a.g_new, g0 = a.g_old;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g1 * g1 * g1) return;
    const int ix = (int)(j % g1), iy = (int)((j / g1) % g1), iz = (int)(j / (g1 * g1));
    int x[2], y[2], z[2];
    double wx[2], wy[2], wz[2];
    lattice_axis(ix, a.g_old, a.g_new, &x[0], &x[1], &wx[0], &wx[1]);
    lattice_axis(iy, a.g_old, a.g_new, &y[0], &y[1], &wy[0], &wy[1]);
    lattice_axis(iz, a.g_old, a.g_new, &z[0], &z[1], &wz[0], &wz[1]);
    double w[8];
    int64_t src[8];
    int ref = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int dz = k >> 2, dy = (k >> 1) & 1, dx = k & 1;
        w[k] = wz[dz] * wy[dy] * wx[dx];
        src[k] = ((int64_t)z[dz] * g0 + y[dy]) * g0 + x[dx];
        if (w[k] > w[ref]) ref = k;
    }
    double alpha = 0.0, sc[3] = {0.0, 0.0, 0.0}, qr[4], qs[4] = {0.0, 0.0, 0.0, 0.0};
    {
        const float* q = a.quat + 4 * src[ref];
        const double n = sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] +
                              (double)q[3] * q[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m) qr[m] = (double)q[m] / n;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t i = src[k];
        alpha += w[k] * (1.0 / (1.0 + exp(-(double)a.logit[i])));
#pragma unroll
        for (int m = 0; m < 3; ++m) sc[m] += w[k] * exp((double)a.log_scale[3 * i + m]);
        const float* q = a.quat + 4 * i;
        const double n = sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] +
                              (double)q[3] * q[3]);
        double qk[4], d = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            qk[m] = (double)q[m] / n;
            d += qk[m] * qr[m];
        }
        const double sg = d >= 0.0 ? w[k] : -w[k];
#pragma unroll
        for (int m = 0; m < 4; ++m) qs[m] += sg * qk[m];
    }
    const double nq = sqrt(qs[0] * qs[0] + qs[1] * qs[1] + qs[2] * qs[2] + qs[3] * qs[3]);
#pragma unroll
    for (int m = 0; m < 4; ++m)
        a.out_quat[4 * j + m] = (float)(nq > 0.0 ? qs[m] / nq : (m == 0 ? 1.0 : 0.0));
    const double ratio = (double)g0 / (double)g1;
#pragma unroll
    for (int m = 0; m < 3; ++m) a.out_log_scale[3 * j + m] = (float)log(sc[m] * ratio);
    alpha = fmin(fmax(alpha, 1e-6), 1.0 - 1e-6);
    a.out_logit[j] = (float)log(alpha / (1.0 - alpha));
    a.out_mean[3 * j] = (float)(-1.0 + (2.0 * ix + 1.0) / (double)g1);
    a.out_mean[3 * j + 1] = (float)(-1.0 + (2.0 * iy + 1.0) / (double)g1);
    a.out_mean[3 * j + 2] = (float)(-1.0 + (2.0 * iz + 1.0) / (double)g1);
}

}  // namespace

hipError_t launch_upsample(const UpsampleArgs& a, hipStream_t s)
{
    const int64_t n = (int64_t)a.g_new * a.g_new * a.g_new;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_upsample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_devox(const DevoxArgs& a, hipStream_t s)
{
    const int64_t n = (int64_t)a.g * a.g * a.g;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_devox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}
