// SSIM term of the reconstruction loss (Sec. 3.5.2, Eq. 10) on whole stack slices, with its
// gradient, fused in one kernel over 32 x 32 pixel tiles of the slices.
//
// Every z-slice of a stack is a 2D image.  The SSIM map uses an 11 x 11 Gaussian window (the
// outer product of 11 taps g, sigma 1.5), zero padding outside the slice, C1 = 0.01^2 and
// C2 = 0.03^2.  L = 1 - mean of the map over every stack voxel, and with the window sums
// (mu_x, m_xx, m_xy) taken as the variables,
//     dL/dx_q = -(1/N) sum_p w(q - p) [S_mu + 2 x_q S_xx + y_q S_xy](p).
//
// The statistics and the map's partial derivatives are formed in FP64: the variances are
// differences of window sums (m - mu^2), whose cancellation would cost FP32 about four of its
// seven digits, and gfx950 issues FP64 FMAs at its FP32 (unpacked) rate.  Per tile of TY x TX
// output pixels (R = 5, the window's half width):
//   1. stage the (TY + 4R) x (TX + 4R) input region of x (prediction) and y (target), FP32;
//   2. vertical window pass of x, y, x^2, y^2, x y -> (TY + 2R) x (TX + 4R), FP64;
//   3. horizontal pass -> the five statistics at the (TY + 2R) x (TX + 2R) map positions whose
//      windows reach the tile; there S and its partials (zero outside the slice); S summed over
//      the tile's own positions;
//   4. vertical then horizontal adjoint passes of the three partials -> TY x TX;
//      dl[q] += -(lambda / N) (A_mu + 2 x_q A_xx + y_q A_xy).
// The window passes stream along their axis (each thread slides over a short run of outputs),
// so every staged value is read once per run rather than once per tap.  Each map position is
// summed by one tile and each pixel written by one tile; per-block FP64 sums are added in a
// fixed order, so loss and gradient are the same on every run.
#include "gm_internal.h"

namespace {

constexpr int R = 5, WN = 2 * R + 1;
constexpr int TY = 32, TX = 32;
constexpr int IR = TY + 4 * R, IC = TX + 4 * R;   // staged input region 52 x 52
constexpr int VR = TY + 2 * R;                    // rows after the vertical pass: 42
constexpr int MC = TX + 2 * R;                    // map columns: 42
constexpr int NT = 1024;
constexpr int SSIM_BLOCKS = 1024;                 // block partials fit the reduction workspace

// stage 2: (column, run of V_SEG rows); stage 3: (row, run of H_SEG columns)
constexpr int V_SEG = 3, V_RUNS = (VR + V_SEG - 1) / V_SEG;     // 14 runs x 52 columns
constexpr int H_SEG = 3, H_RUNS = MC / H_SEG;                   // 14 runs x 42 rows
constexpr int A_SEG = 4, A_RUNS = TY / A_SEG;                   // 8 runs x 42 columns x 3 maps
static_assert(V_RUNS * IC <= NT, "stage 2 runs exceed the block");
static_assert(MC % H_SEG == 0, "stage 3 runs must tile the map row");
static_assert(VR * H_RUNS <= NT, "stage 3 runs exceed the block");
static_assert(A_RUNS * MC * 3 <= NT, "stage 4 runs exceed the block");
static_assert(TY * TX == NT, "stage 4b: one output per thread");

constexpr int V_SIZE = VR * IC;    // one vertical-pass plane
constexpr int P_SIZE = VR * MC;    // one partial-derivative plane
constexpr int U_SIZE = TY * MC;    // one vertical-adjoint plane
static_assert(3 * P_SIZE + 3 * U_SIZE <= 5 * V_SIZE, "partials and adjoint rows alias the sums");

struct Lds {
    float x[IR][IC];
    float y[IR][IC];
    double buf[5 * V_SIZE];     // vertical sums; then partials [3][VR][MC] + adjoint [3][TY][MC]
    double red[NT / 64];
};

// 1/d from the hardware reciprocal refined by two Newton steps (error ~1 ulp); here
// d = b1 b2 lies in [C1 C2, 4.1]
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}

__device__ double block_sum(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

struct TileGeom {
    int k, nx, ny, y0, x0;
    int64_t slice;     // offset of the tile's slice in its stack
};

__device__ TileGeom tile_geom(const SsimArgs& a, int64_t t)
{
    TileGeom g;
    int k = 0;
    while (t >= a.tile_begin[k + 1]) ++k;
    g.k = k;
    g.nx = a.nx[k];
    g.ny = a.ny[k];
    const int64_t local = t - a.tile_begin[k];
    const int64_t per_slice = (int64_t)a.tiles_x[k] * a.tiles_y[k];
    const int z = (int)(local / per_slice);
    const int rem = (int)(local - (int64_t)z * per_slice);
    g.y0 = (rem / a.tiles_x[k]) * TY;
    g.x0 = (rem % a.tiles_x[k]) * TX;
    g.slice = (int64_t)z * g.ny * g.nx;
    return g;
}

constexpr int LOAD_ITERS = (IR * IC + NT - 1) / NT;   // input elements per thread

// the thread's share of a tile's input region (zero outside the slice), into registers
__device__ __forceinline__ void load_region(const SsimArgs& a, const TileGeom& g, int tid,
                                            float (&vx)[LOAD_ITERS], float (&vy)[LOAD_ITERS])
{
    const float* px = a.pred[g.k] + g.slice;
    const float* py = a.target[g.k] + g.slice;
#pragma unroll
    for (int i = 0; i < LOAD_ITERS; ++i) {
        const int e = tid + i * NT;
        const int r = e / IC, c = e - r * IC;
        const int Y = g.y0 - 2 * R + r, X = g.x0 - 2 * R + c;
        const bool in = e < IR * IC && Y >= 0 && Y < g.ny && X >= 0 && X < g.nx;
        const int64_t o = (int64_t)Y * g.nx + X;
        vx[i] = in ? px[o] : 0.0f;
        vy[i] = in ? py[o] : 0.0f;
    }
}

// one 1024-thread block per CU (107 KB of LDS): four waves per SIMD
__global__ __launch_bounds__(NT) void k_ssim(const SsimArgs a, double* part)
{
    __shared__ Lds s;
    const int64_t total = a.tile_begin[a.n_stacks];
    double ssum = 0.0;
    // the next tile's input region is fetched into registers while the current one is
    // processed, so its latency is hidden behind the window passes
    float nxv[LOAD_ITERS], nyv[LOAD_ITERS];
    if ((int64_t)blockIdx.x < total) load_region(a, tile_geom(a, blockIdx.x), threadIdx.x, nxv, nyv);
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        // the thread's roles are recomputed per tile: kept out of the loop they would hold
        // dozens of registers for the whole kernel
        int tid = threadIdx.x;
        __asm__ __volatile__("" : "+v"(tid));
        const TileGeom geo = tile_geom(a, t);
        const int k = geo.k, nx = geo.nx, ny = geo.ny, y0 = geo.y0, x0 = geo.x0;
        const int64_t slice = geo.slice;

        // 1. input region (prefetched), then the fetch of the next tile's
#pragma unroll
        for (int i = 0; i < LOAD_ITERS; ++i) {
            const int e = tid + i * NT;
            if (e < IR * IC) {
                const int r = e / IC, c = e - r * IC;
                s.x[r][c] = nxv[i];
                s.y[r][c] = nyv[i];
            }
        }
        __syncthreads();
        if (t + gridDim.x < total) load_region(a, tile_geom(a, t + gridDim.x), tid, nxv, nyv);

        // 2. vertical pass: V[q][r][c] = sum_i g_i f_q(in[r + i][c])
        if (tid < V_RUNS * IC) {
            const int c = tid % IC, r0 = (tid / IC) * V_SEG;
            double acc[V_SEG][5];
#pragma unroll
            for (int j = 0; j < V_SEG; ++j)
#pragma unroll
                for (int q = 0; q < 5; ++q) acc[j][q] = 0.0;
#pragma unroll
            for (int ii = 0; ii < V_SEG + WN - 1; ++ii) {
                const int ri = r0 + ii;
                const double xv = ri < IR ? (double)s.x[ri][c] : 0.0;
                const double yv = ri < IR ? (double)s.y[ri][c] : 0.0;
                const double f[5] = {xv, yv, xv * xv, yv * yv, xv * yv};
#pragma unroll
                for (int j = 0; j < V_SEG; ++j) {
                    const int tap = ii - j;
                    if (tap >= 0 && tap < WN) {
#pragma unroll
                        for (int q = 0; q < 5; ++q) acc[j][q] = fma(a.g[tap], f[q], acc[j][q]);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < V_SEG; ++j)
                if (r0 + j < VR) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) s.buf[q * V_SIZE + (r0 + j) * IC + c] = acc[j][q];
                }
        }
        __syncthreads();

        // 3. horizontal pass, SSIM and its partials at the map positions
        double pd[H_SEG][3];
        const bool h_on = tid < VR * H_RUNS;
        const int hr = tid / H_RUNS, hc0 = (tid % H_RUNS) * H_SEG;
        if (h_on) {
            double m[H_SEG][5];
#pragma unroll
            for (int j = 0; j < H_SEG; ++j)
#pragma unroll
                for (int q = 0; q < 5; ++q) m[j][q] = 0.0;
#pragma unroll
            for (int jj = 0; jj < H_SEG + WN - 1; ++jj) {
                double v[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) v[q] = s.buf[q * V_SIZE + hr * IC + hc0 + jj];
#pragma unroll
                for (int j = 0; j < H_SEG; ++j) {
                    const int tap = jj - j;
                    if (tap >= 0 && tap < WN) {
#pragma unroll
                        for (int q = 0; q < 5; ++q) m[j][q] = fma(a.g[tap], v[q], m[j][q]);
                    }
                }
            }
            const int Y = y0 - R + hr;
#pragma unroll
            for (int j = 0; j < H_SEG; ++j) {
                const int c = hc0 + j, X = x0 - R + c;
                const double mx = m[j][0], my = m[j][1];
                const double vx = m[j][2] - mx * mx, vy = m[j][3] - my * my;
                const double cxy = m[j][4] - mx * my;
                const double a1 = 2.0 * mx * my + GM_SSIM_C1, a2 = 2.0 * cxy + GM_SSIM_C2;
                const double b1 = mx * mx + my * my + GM_SSIM_C1, b2 = vx + vy + GM_SSIM_C2;
                const double rb = recip(b1 * b2), r1 = b2 * rb, r2 = b1 * rb;   // 1/b1, 1/b2
                const double sv = a1 * a2 * rb;
                const bool in = Y >= 0 && Y < ny && X >= 0 && X < nx;
                const bool own = in && hr >= R && hr < R + TY && c >= R && c < R + TX;
                if (own) ssum += sv;
                pd[j][0] = in ? 2.0 * my * (a2 - a1) * rb + 2.0 * mx * sv * (r2 - r1) : 0.0;
                pd[j][1] = in ? -sv * r2 : 0.0;
                pd[j][2] = in ? 2.0 * a1 * rb : 0.0;
            }
        }
        __syncthreads();   // the partials overwrite the vertical sums
        if (h_on) {
#pragma unroll
            for (int j = 0; j < H_SEG; ++j)
#pragma unroll
                for (int q = 0; q < 3; ++q) s.buf[q * P_SIZE + hr * MC + hc0 + j] = pd[j][q];
        }
        __syncthreads();

        // 4a. vertical adjoint: U[t][o][c] = sum_i g[2R - i] P[t][o + i][c]
        double* U = s.buf + 3 * P_SIZE;
        if (tid < A_RUNS * MC * 3) {
            const int c = tid % MC, rest = tid / MC;
            const int tm = rest % 3, o0 = (rest / 3) * A_SEG;
            const double* P = s.buf + tm * P_SIZE;
            double acc[A_SEG];
#pragma unroll
            for (int j = 0; j < A_SEG; ++j) acc[j] = 0.0;
#pragma unroll
            for (int ii = 0; ii < A_SEG + WN - 1; ++ii) {
                const double v = P[(o0 + ii) * MC + c];
#pragma unroll
                for (int j = 0; j < A_SEG; ++j) {
                    const int i = ii - j;
                    if (i >= 0 && i < WN) acc[j] = fma(a.g[2 * R - i], v, acc[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < A_SEG; ++j) U[tm * U_SIZE + (o0 + j) * MC + c] = acc[j];
        }
        __syncthreads();

        // 4b. horizontal adjoint and the gradient, one output pixel per thread
        {
            const int o = tid / TX, oc = tid % TX;
            double gsum[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int tm = 0; tm < 3; ++tm)
                    gsum[tm] = fma(a.g[2 * R - j], U[tm * U_SIZE + o * MC + oc + j], gsum[tm]);
            const int Y = y0 + o, X = x0 + oc;
            if (Y < ny && X < nx) {
                const double xq = s.x[o + 2 * R][oc + 2 * R], yq = s.y[o + 2 * R][oc + 2 * R];
                const double gq = a.grad_scale * (gsum[0] + 2.0 * xq * gsum[1] + yq * gsum[2]);
                float* d = a.dl[k] + slice + (int64_t)Y * nx + X;
                *d += (float)gq;
            }
        }
        __syncthreads();   // the next tile restages the region and the buffer
    }
    const double tot = block_sum(ssum, s.red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_ssim_finish(const double* part, int nb, double inv_n,
                                                     float* loss)
{
    __shared__ double sh[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) v += part[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = inv_n > 0.0 ? (float)(1.0 - sh[0] * inv_n) : 0.0f;
}

}  // namespace

void ssim_tiles(int nx, int ny, int* tiles_x, int* tiles_y)
{
    *tiles_x = (nx + TX - 1) / TX;
    *tiles_y = (ny + TY - 1) / TY;
}

hipError_t launch_ssim(const SsimArgs& a, int64_t n_voxels, float* loss, void* ws,
                       hipStream_t s)
{
    double* part = reinterpret_cast<double*>(ws);
    const int64_t total = a.tile_begin[a.n_stacks];
    const int nb = (int)(total < SSIM_BLOCKS ? total : SSIM_BLOCKS);
    if (nb > 0) hipLaunchKernelGGL(k_ssim, dim3((unsigned)nb), dim3(NT), 0, s, a, part);
    hipLaunchKernelGGL(k_ssim_finish, dim3(1), dim3(256), 0, s, part, nb,
                       n_voxels > 0 ? 1.0 / (double)n_voxels : 0.0, loss);
    return hipGetLastError();
}
