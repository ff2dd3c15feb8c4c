// K1: per (grid, Gaussian) record, integer box and tile count.
//
// Built with -ffp-contract=off: the box is an integer decision made from floating point, so
// it follows one fixed IEEE binary64 recipe (no fused multiply-add, correctly rounded sqrt
// and division, the association written below) that gives the same boxes wherever it runs.
//
// Model (Sec. 3.2, Eq. 2-3): Sigma = R diag(e^{2s}) R^T with R from the normalised
// quaternion; alpha = sigmoid(logit).  On a grid with world->index affine [L | t] and
// slice-profile sigma sig (Sec. 3.3.2 with a Gaussian slice profile along index z):
//   c = L mu + t,  Sigma_idx = B B^T with B = L R diag(e^s),
//   Sigma_g = Sigma_idx + sig^2 e_z e_z^T,  C = Sigma_g^-1,
//   amp = alpha sqrt(det Sigma_idx / det Sigma_g)       (Gaussian (x) normalised profile).
// The box is +-cutoff marginal standard deviations sqrt((Sigma_g)_jj) around c, or, with a
// block radius, the paper's cell-neighbourhood query (Eqs. 4-6): exactly its voxels on
// axis-aligned grids, a box holding them on rotated grids (whose voxels the kernels test).
#include "gm_internal.h"

namespace {

// Cody-Waite reduction with a two-part ln 2 (the high part has 28 significant bits, so
// k * LN2_HI is exact), Taylor series of e^r to degree 13 in Horner form, ldexp by k.
__device__ double exp_cw(double s)
{
    const double LN2_HI = 0x1.62e42fe000000p-1;
    const double LN2_LO = 0x1.f473de6af278fp-30;
    const double INV_LN2 = 0x1.71547652b82fep+0;
    const double C[14] = {0x1.0000000000000p+0, 0x1.0000000000000p+0, 0x1.0000000000000p-1,
                          0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,
                          0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16,
                          0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26,
                          0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};
    const double k = rint(s * INV_LN2);
    const double r = (s - k * LN2_HI) - k * LN2_LO;
    double p = C[13];
#pragma unroll
    for (int i = 12; i >= 0; --i) p = p * r + C[i];
    const double kc = fmin(fmax(k, -2000.0), 2000.0);
    return ldexp(p, (int)kc);
}

__device__ __forceinline__ bool finite_d(double x) { return __builtin_isfinite(x); }

// Eq. 4 along one axis: floor((x + 1) res / 2), binary64, that association
__device__ __forceinline__ double cell_of(double x, double res) { return floor(((x + 1.0) * res) / 2.0); }

// The paper's block query (Eqs. 4-6) on index axis j of an axis-aligned grid: the voxels v with
// |cell(x(v)) - cm| <= r, x(v) = (v - t) / l the world coordinate along the mapped axis.  A
// candidate range from the real-number inverse, widened by two voxels, is narrowed by the
// exact predicate at both ends (the set is an interval: x(v) and the cell are monotone).
// Returns false when a bounded walk did not settle (never for finite grid scales).
__device__ bool block_interval(double l, double t, double cm, double r, double res, int dim,
                               int* lo, int* hi)
{
    const double CL = 1073741824.0;
    const double x0 = ((cm - r) * 2.0) / res - 1.0, x1 = ((cm + r + 1.0) * 2.0) / res - 1.0;
    const double va = x0 * l + t, vb = x1 * l + t;
    double a = floor(fmin(va, vb)) - 2.0, b = ceil(fmax(va, vb)) + 2.0;
    a = (a != a) ? CL : fmin(fmax(a, -CL), CL);
    b = (b != b) ? -CL : fmin(fmax(b, -CL), CL);
    int v0 = (int)a, v1 = (int)b;
    v0 = v0 < 0 ? 0 : v0;
    v1 = v1 > dim - 1 ? dim - 1 : v1;
    auto in = [&](int v) { return fabs(cell_of(((double)v - t) / l, res) - cm) <= r; };
    int steps = 0;
    while (v0 <= v1 && !in(v0) && steps < 16) {
        ++v0;
        ++steps;
    }
    steps = 0;
    while (v1 >= v0 && !in(v1) && steps < 16) {
        --v1;
        ++steps;
    }
    *lo = v0;
    *hi = v1;
    return v0 > v1 || (in(v0) && in(v1));
}

// BLOCK: the block query (a.block_radius > 0); the sigma box otherwise.  Two kernels, so that
// the sigma-box kernel carries none of the block rule's registers (and fits five wavefronts per
// SIMD).
template <bool BLOCK>
__device__ __forceinline__ void preprocess_body(const PreprocessArgs& a)
{
    __shared__ unsigned long long s_vol[GM_MAX_GRIDS];
    if (threadIdx.x < GM_MAX_GRIDS) s_vol[threadIdx.x] = 0ull;
    __syncthreads();

    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.n) {
        const double mu0 = a.mean[3 * i], mu1 = a.mean[3 * i + 1], mu2 = a.mean[3 * i + 2];
        const double qw = a.quat[4 * i], qx = a.quat[4 * i + 1], qy = a.quat[4 * i + 2],
                     qz = a.quat[4 * i + 3];
        const double s0 = a.log_scale[3 * i], s1 = a.log_scale[3 * i + 1],
                     s2 = a.log_scale[3 * i + 2];
        const double lg = a.logit[i];

        // step 1: validity and normalisation
        const double n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
        bool valid = finite_d(mu0) && finite_d(mu1) && finite_d(mu2) && finite_d(qw) &&
                     finite_d(qx) && finite_d(qy) && finite_d(qz) && finite_d(s0) &&
                     finite_d(s1) && finite_d(s2) && finite_d(lg) && n2 > 0.0 && finite_d(n2);
        const double nq = sqrt(valid ? n2 : 1.0);
        const double w = qw / nq, x = qx / nq, y = qy / nq, z = qz / nq;
        // step 2: rotation (Hamilton), fixed association
        double R[9];
        R[0] = 1.0 - 2.0 * ((y * y) + (z * z));
        R[1] = 2.0 * ((x * y) - (w * z));
        R[2] = 2.0 * ((x * z) + (w * y));
        R[3] = 2.0 * ((x * y) + (w * z));
        R[4] = 1.0 - 2.0 * ((x * x) + (z * z));
        R[5] = 2.0 * ((y * z) - (w * x));
        R[6] = 2.0 * ((x * z) - (w * y));
        R[7] = 2.0 * ((y * z) + (w * x));
        R[8] = 1.0 - 2.0 * ((x * x) + (y * y));
        // step 3: scales
        const double e[3] = {exp_cw(valid ? s0 : 0.0), exp_cw(valid ? s1 : 0.0),
                             exp_cw(valid ? s2 : 0.0)};
        valid = valid && finite_d(e[0]) && finite_d(e[1]) && finite_d(e[2]) && e[0] > 0.0 &&
                e[1] > 0.0 && e[2] > 0.0;
        if (!valid) atomicOr(a.flags, 1u);
        const double alpha = 1.0 / (1.0 + exp(-lg));
        // block query: the mean's cell on each world axis (Eq. 4), clamped to [-2^30, 2^30],
        // kept for the kernels that test voxels of rotated grids
        double cmw[3] = {0.0, 0.0, 0.0};
        if (BLOCK) {
            const double res = (double)a.cell_res, CC = 1073741824.0;
            const double mus[3] = {mu0, mu1, mu2};
#pragma unroll
            for (int w_ = 0; w_ < 3; ++w_)
                cmw[w_] = valid ? fmin(fmax(cell_of(mus[w_], res), -CC), CC) : 0.0;
            a.cells[i] = make_int4((int)cmw[0], (int)cmw[1], (int)cmw[2], 0);
        }

        for (int k = 0; k < a.n_grids; ++k) {
            const GridConst& G = a.g[k];
            const double* L = G.L;
            // step 4: B = (L R) diag(e)
            double B[9];
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    B[3 * j + m] = ((L[3 * j] * R[m] + L[3 * j + 1] * R[3 + m]) +
                                    L[3 * j + 2] * R[6 + m]) * e[m];
            // step 5: marginal variances, slice profile on z, half-widths
            double D[3];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                D[j] = (B[3 * j] * B[3 * j] + B[3 * j + 1] * B[3 * j + 1]) +
                       B[3 * j + 2] * B[3 * j + 2];
            D[2] = D[2] + G.sig * G.sig;
            // step 6: centre
            const double c[3] = {((L[0] * mu0 + L[1] * mu1) + L[2] * mu2) + G.t[0],
                                 ((L[3] * mu0 + L[4] * mu1) + L[5] * mu2) + G.t[1],
                                 ((L[6] * mu0 + L[7] * mu1) + L[8] * mu2) + G.t[2]};
            // step 7: integer box, clipped
            const int dims[3] = {G.nx, G.ny, G.nz};
            int lo[3], hi[3];
            bool nonempty = valid;
            const double CL = 1073741824.0;
            if (BLOCK && G.waxis[0] < 0) {
                // rotated grid: the block's world box (Eq. 5 solved for x), widened by 1e-9
                // (relative), mapped to index space (the bounds of a linear map over a box),
                // widened by 1e-6 (relative) and rounded outwards.  It holds every voxel whose
                // cell test passes; the kernels test each voxel of it.
                const double res = (double)a.cell_res, r = (double)a.block_radius;
                double x0[3], x1[3];
#pragma unroll
                for (int w_ = 0; w_ < 3; ++w_) {
                    const double u0 = ((cmw[w_] - r) * 2.0) / res - 1.0;
                    const double u1 = ((cmw[w_] + r + 1.0) * 2.0) / res - 1.0;
                    x0[w_] = u0 - 1e-9 * (1.0 + fabs(u0));
                    x1[w_] = u1 + 1e-9 * (1.0 + fabs(u1));
                }
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double vmin = G.t[j], vmax = G.t[j];
#pragma unroll
                    for (int w_ = 0; w_ < 3; ++w_) {
                        const double p = G.L[3 * j + w_] * x0[w_], q = G.L[3 * j + w_] * x1[w_];
                        vmin = vmin + fmin(p, q);
                        vmax = vmax + fmax(p, q);
                    }
                    double l = ceil(vmin - 1e-6 * (1.0 + fabs(vmin)));
                    double h = floor(vmax + 1e-6 * (1.0 + fabs(vmax)));
                    l = (l != l) ? CL : fmin(fmax(l, -CL), CL);
                    h = (h != h) ? -CL : fmin(fmax(h, -CL), CL);
                    int li = (int)l, hj = (int)h;
                    li = li < 0 ? 0 : li;
                    hj = hj > dims[j] - 1 ? dims[j] - 1 : hj;
                    lo[j] = li;
                    hi[j] = hj;
                    nonempty = nonempty && (li <= hj);
                }
            } else if (BLOCK) {
                const double mus[3] = {mu0, mu1, mu2};
                const double res = (double)a.cell_res, r = (double)a.block_radius;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int wa = G.waxis[j];
                    const double cm = cell_of(valid ? mus[wa] : 0.0, res);
                    if (!block_interval(G.L[3 * j + wa], G.t[j], cm, r, res, dims[j], &lo[j], &hi[j]))
                        atomicOr(a.flags, 2u);
                    nonempty = nonempty && (lo[j] <= hi[j]);
                }
            } else {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double rho = a.cutoff * sqrt(D[j]);
                double l = ceil(c[j] - rho), h = floor(c[j] + rho);
                l = (l != l) ? CL : fmin(fmax(l, -CL), CL);
                h = (h != h) ? -CL : fmin(fmax(h, -CL), CL);
                int li = (int)l, hj = (int)h;
                li = li < 0 ? 0 : li;
                hj = hj > dims[j] - 1 ? dims[j] - 1 : hj;
                lo[j] = li;
                hi[j] = hj;
                nonempty = nonempty && (li <= hj);
            }
            }
            // record: c - lo, amp, base-2 conic, box
            double Si[6];  // Sigma_idx = B B^T: xx yy zz xy xz yz
            Si[0] = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
            Si[1] = B[3] * B[3] + B[4] * B[4] + B[5] * B[5];
            Si[2] = B[6] * B[6] + B[7] * B[7] + B[8] * B[8];
            Si[3] = B[0] * B[3] + B[1] * B[4] + B[2] * B[5];
            Si[4] = B[0] * B[6] + B[1] * B[7] + B[2] * B[8];
            Si[5] = B[3] * B[6] + B[4] * B[7] + B[5] * B[8];
            const double gxx = Si[0], gyy = Si[1], gzz = Si[2] + G.sig * G.sig;
            const double gxy = Si[3], gxz = Si[4], gyz = Si[5];
            const double axx = gyy * gzz - gyz * gyz, ayy = gxx * gzz - gxz * gxz,
                         azz = gxx * gyy - gxy * gxy, axy = gxz * gyz - gxy * gzz,
                         axz = gxy * gyz - gxz * gyy, ayz = gxy * gxz - gxx * gyz;
            const double detG = gxx * axx + gxy * axy + gxz * axz;
            const double detB = B[0] * (B[4] * B[8] - B[5] * B[7]) -
                                B[1] * (B[3] * B[8] - B[5] * B[6]) +
                                B[2] * (B[3] * B[7] - B[4] * B[6]);
            const double detI = detB * detB;
            const double amp = alpha * sqrt(detI / detG);
            const double kd = GM_KAPPA / detG;

            float4 r0, r1, r2, r3;
            r0.x = (float)(c[0] - lo[0]);
            r0.y = (float)(c[1] - lo[1]);
            r0.z = (float)(c[2] - lo[2]);
            r0.w = nonempty ? (float)amp : 0.0f;
            r1.x = (float)(kd * axx);
            r1.y = (float)(kd * ayy);
            r1.z = (float)(kd * azz);
            r1.w = (float)(2.0 * kd * axy);
            r2.x = (float)(2.0 * kd * axz);
            r2.y = (float)(2.0 * kd * ayz);
            r2.z = __int_as_float(nonempty ? lo[0] : 0);
            r2.w = __int_as_float(nonempty ? lo[1] : 0);
            r3.x = __int_as_float(nonempty ? lo[2] : 0);
            r3.y = __int_as_float(nonempty ? hi[0] : -1);
            r3.z = __int_as_float(nonempty ? hi[1] : -1);
            r3.w = __int_as_float(nonempty ? hi[2] : -1);
            float4* rec = reinterpret_cast<float4*>(a.records + ((size_t)k * a.n + i) * 16);
            rec[0] = r0;
            rec[1] = r1;
            rec[2] = r2;
            rec[3] = r3;

            int cnt = 0;
            unsigned long long vol = 0ull;
            if (nonempty) {
                cnt = (hi[0] / GM_TX - lo[0] / GM_TX + 1) * (hi[1] / GM_TY - lo[1] / GM_TY + 1) *
                      (hi[2] / GM_TZ - lo[2] / GM_TZ + 1);
                vol = (unsigned long long)(hi[0] - lo[0] + 1) * (unsigned long long)(hi[1] - lo[1] + 1) *
                      (unsigned long long)(hi[2] - lo[2] + 1);
            }
            a.tile_count[(size_t)k * a.n + i] = cnt;
            {
                // the tile range alone, for the pair emission (which then need not read
                // the 64-byte records); tile indices fit 16 bits for grids of <= 32768
                uint32_t* tb = a.tile_box + ((size_t)k * a.n + i) * 3;
                const uint32_t tlx = nonempty ? (uint32_t)(lo[0] / GM_TX) : 1u;
                const uint32_t tly = nonempty ? (uint32_t)(lo[1] / GM_TY) : 1u;
                const uint32_t tlz = nonempty ? (uint32_t)(lo[2] / GM_TZ) : 1u;
                const uint32_t thx = nonempty ? (uint32_t)(hi[0] / GM_TX) : 0u;
                const uint32_t thy = nonempty ? (uint32_t)(hi[1] / GM_TY) : 0u;
                const uint32_t thz = nonempty ? (uint32_t)(hi[2] / GM_TZ) : 0u;
                tb[0] = tlx | (tly << 16);
                tb[1] = tlz | (thx << 16);
                tb[2] = thy | (thz << 16);
            }
            if (vol) atomicAdd(&s_vol[k], vol);
            // the backward visits only Gaussians listed in some tile: the grid-frame
            // partials of an empty box are its zeros, written here
            if (!nonempty && a.grid_grads) {
                float2* o = reinterpret_cast<float2*>(a.grid_grads + ((size_t)k * a.n + i) * 10);
#pragma unroll
                for (int t = 0; t < 5; ++t) o[t] = make_float2(0.0f, 0.0f);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < a.n_grids && s_vol[threadIdx.x])
        atomicAdd(&a.box_volume[threadIdx.x], s_vol[threadIdx.x]);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_preprocess(
    const PreprocessArgs a)
{
    preprocess_body<false>(a);
}

__global__ __launch_bounds__(256) void k_preprocess_block(const PreprocessArgs a)
{
    preprocess_body<true>(a);
}

}  // namespace

hipError_t launch_preprocess(const PreprocessArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    const int64_t blocks = (a.n + 255) / 256;
    if (a.block_radius > 0)
        hipLaunchKernelGGL(k_preprocess_block, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_preprocess, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}
