// K9 smooth-L1 data term (Eq. 11) with its per-voxel gradient, the anisotropy regulariser
// value (Eq. 13), the mean squared error behind PSNR (Sec. 4.1.3) and K10 Adam (Sec. 4.1.4).
// Reductions are two-pass (fixed block partials in FP64, then one block in fixed order), so
// every value is the same on every run.
#include "gm_internal.h"

namespace {

constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 1024;  // partials fit GM_REDUCE_WORKSPACE_BYTES (8 KB of doubles)

__device__ double block_sum(double v)
{
    __shared__ double s[RED_THREADS];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = RED_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(RED_THREADS) void k_finish(const double* part, int nb, double scale,
                                                         float* out)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += RED_THREADS) v += part[i];
    v = block_sum(v);
    if (threadIdx.x == 0) *out = (float)(v * scale);
}

__global__ __launch_bounds__(RED_THREADS) void k_smooth_l1(const LossArgs a, double inv_n,
                                                            double* part)
{
    double acc = 0.0;
    const float g_scale = (float)inv_n;
    for (int k = 0; k < a.n_stacks; ++k) {
        const int64_t n = a.begin[k + 1] - a.begin[k];
        const float* p = a.pred[k];
        const float* y = a.target[k];
        float* dl = a.dl[k];
        for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * RED_THREADS) {
            const float d = p[i] - y[i];
            const float ad = fabsf(d);
            acc += ad < 1.0f ? 0.5 * (double)d * (double)d : (double)ad - 0.5;
            dl[i] = fminf(fmaxf(d, -1.0f), 1.0f) * g_scale;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(RED_THREADS) void k_aniso(const float* ls, int64_t n, float lam,
                                                        double* part)
{
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * RED_THREADS) {
        const float a0 = ls[3 * i], a1 = ls[3 * i + 1], a2 = ls[3 * i + 2];
        const double mx = fmaxf(a0, fmaxf(a1, a2)), mn = fminf(a0, fminf(a1, a2));
        const double r = exp(mx - mn) - (double)lam;
        acc += r > 0.0 ? r : 0.0;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(RED_THREADS) void k_sqdiff(const float* a, const float* b, int64_t n,
                                                         double* part)
{
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * RED_THREADS) {
        const double d = (double)a[i] - (double)b[i];
        acc += d * d;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                               float* __restrict__ m, float* __restrict__ v,
                                               int64_t n, const AdamScalars c)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float pi = p[i], mi = m[i], vi = v[i];
        adam_elem(pi, mi, vi, g[i], c);
        m[i] = mi;
        v[i] = vi;
        p[i] = pi;
    }
}

unsigned red_blocks(int64_t n)
{
    int64_t b = (n + RED_THREADS - 1) / RED_THREADS;
    if (b < 1) b = 1;
    if (b > RED_BLOCKS) b = RED_BLOCKS;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_smooth_l1(const LossArgs& a, float* loss, void* ws, hipStream_t s)
{
    double* part = reinterpret_cast<double*>(ws);
    const unsigned nb = red_blocks(a.total);
    const double inv_n = a.total > 0 ? 1.0 / (double)a.total : 0.0;
    hipLaunchKernelGGL(k_smooth_l1, dim3(nb), dim3(RED_THREADS), 0, s, a, inv_n, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(RED_THREADS), 0, s, part, (int)nb, inv_n, loss);
    return hipGetLastError();
}

hipError_t launch_aniso(const float* log_scale, int64_t n, float lambda_r, float* value,
                        void* ws, hipStream_t s)
{
    double* part = reinterpret_cast<double*>(ws);
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_aniso, dim3(nb), dim3(RED_THREADS), 0, s, log_scale, n, lambda_r, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(RED_THREADS), 0, s, part, (int)nb,
                       n > 0 ? 1.0 / (double)n : 0.0, value);
    return hipGetLastError();
}

hipError_t launch_mse(const float* a, const float* b, int64_t n, float* mse, void* ws,
                      hipStream_t s)
{
    double* part = reinterpret_cast<double*>(ws);
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_sqdiff, dim3(nb), dim3(RED_THREADS), 0, s, a, b, n, part);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(RED_THREADS), 0, s, part, (int)nb,
                       n > 0 ? 1.0 / (double)n : 0.0, mse);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n,
                       const AdamScalars& c, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)nb), dim3(256), 0, s, p, g, m, v, n, c);
    return hipGetLastError();
}

AdamScalars adam_scalars(double lr, double beta1, double beta2, double eps, int32_t step)
{
    const double bc1 = 1.0 - pow(beta1, (double)step);
    const double bc2 = 1.0 - pow(beta2, (double)step);
    AdamScalars c;
    c.b1 = (float)beta1;
    c.omb1 = (float)(1.0 - beta1);
    c.b2 = (float)beta2;
    c.omb2 = (float)(1.0 - beta2);
    c.eps = (float)eps;
    c.step_size = (float)(lr / bc1);
    c.bc2_sqrt = (float)sqrt(bc2);
    return c;
}
