// K11: neural residual field (Sec. 3.4, Eq. 8) on MFMA: BF16 weights and activations,
// FP32 accumulation.
//
// r(x) = out_scale tanh(w_out . a_D + b_out),  a_l = SiLU(W_l a_{l-1} + b_l),
// a_0 = gamma(x) = (x, sin(2^k pi x), cos(2^k pi x), k < n_freq), zero-padded to in_pad.
//
// Layout trick: each layer is computed transposed, Z^T = W X^T, with gfx950's 16x16x32 BF16
// MFMA (A = 16 output features x 32 input features of W, B = 32 input features x 16 points).
// The result holds, per lane, 4 consecutive output features of one point; two such tiles are
// exactly the B operand of one 32-wide K step of the next layer (the weights are staged with
// the same K order), so activations never leave registers inside a layer stack.  The encoding
// is computed directly in that layout.
//
// Backward (for a list of sampled voxels): recompute, then per layer dZ_l = dA_l * SiLU'(Z_l),
// dA_{l-1} = W_l^T dZ_l (MFMA); dZ_l and A_{l-1} are written feature-major (BF16) and the
// weight gradients dW_l = dZ_l A_{l-1}^T are formed by a split-K MFMA GEMM over the points.
// The forward alone (k_nrf_forward) is in nrf_fwd.hip.
#include "nrf_core.h"

namespace {

using namespace nrfcore;

// Recompute a tile and write, feature-major with point stride P: DZO (f32, per point), and
// for each layer l (1..D) dZ_l [W][P] and A_{l-1} [in_l][P] (BF16), plus A_D [W][P].
template <int KT, int DEPTH>
__global__ __launch_bounds__(256) void k_nrf_chain(const NrfArgs a, NrfWork w)
{
    __shared__ LdsChain<KT, DEPTH> s;
    load_weights<KT, DEPTH>(a, s.f, s.w_hid_t);
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
    v4s wo[4];
    load_wout(a, wo);
    const int64_t P = w.P;
    const int64_t ntiles = w.np / 16;
    // the output layer's gradient over this wavefront's points: gwo[4 o + j] for feature
    // 16 o + 4 g + j (sum of dzo a_D), gbo the sum of dzo (lanes of group 0)
    float gwo[16], gbo = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) gwo[i] = 0.0f;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles;
         tile += (int64_t)gridDim.x * 4) {
        const int64_t p = tile * 16 + row;
        const bool valid = p < a.n_points;
        int vx = 0, vy = 0, vz = 0;
        if (valid) point_xyz(a, p, &vx, &vy, &vz);
        const float x[3] = {world_coord(a.m, vx, vy, vz), world_coord(a.m + 4, vx, vy, vz),
                            world_coord(a.m + 8, vx, vy, vz)};
        Tile<KT, DEPTH> T;
        tile_forward<KT, DEPTH>(a, s.f, x, T, &w, w.p0 + p);
        // z_o of the lane's point, from lane group 0 to all four
        const float zo = __shfl(tile_output<KT, DEPTH>(a, T, wo), row, 64);
        float dl = 0.0f;
        if (valid) dl = a.dl_dr[((int64_t)vz * a.ny + vy) * a.nx + vx];
        const float th = tanhf(zo);
        const float dzo = valid ? dl * a.scale * a.out_scale * (1.0f - th * th) : 0.0f;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const v4s h = T.act[DEPTH - 1][o];
            gwo[4 * o + 0] += dzo * from_bf16((uint16_t)h.x);
            gwo[4 * o + 1] += dzo * from_bf16((uint16_t)h.y);
            gwo[4 * o + 2] += dzo * from_bf16((uint16_t)h.z);
            gwo[4 * o + 3] += dzo * from_bf16((uint16_t)h.w);
        }
        if (g == 0) gbo += dzo;
        // dA_D = dzo w_out, then back through the layers
        v4f da[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int f = 16 * o + 4 * g;
            da[o].x = dzo * from_bf16(a.w_out[f]);
            da[o].y = dzo * from_bf16(a.w_out[f + 1]);
            da[o].z = dzo * from_bf16(a.w_out[f + 2]);
            da[o].w = dzo * from_bf16(a.w_out[f + 3]);
        }
#pragma unroll
        for (int l = DEPTH - 1; l >= 0; --l) {
            v4s dz[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const v4f z = T.z[l][o];
                const v4f d = da[o];
                dz[o] = pack4(d.x * dsilu(z.x), d.y * dsilu(z.y), d.z * dsilu(z.z), d.w * dsilu(z.w));
                store_fm(w.dz[l], 16 * o + 4 * g, P, w.p0 + p, dz[o]);
            }
            if (l == 0) break;
            // dA_{l-1} = W_l^T dZ_l
            const v4s* Wt = s.w_hid_t + (l - 1) * 16 * 64;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int o = 0; o < 4; o += 2)
                    acc = mfma2(Wt[(i * 4 + o) * 64 + lane], Wt[(i * 4 + o + 1) * 64 + lane], dz[o],
                                dz[o + 1], acc);
                da[i] = acc;
            }
        }
    }
    // sum over the 16 points of each lane group, then one partial per wavefront:
    // part[wave][64] for w_out, then part[nwaves * 64 + wave] for b_out (waves counted over
    // every grid of the call)
#pragma unroll
    for (int i = 0; i < 16; ++i)
        for (int o = 1; o < 16; o <<= 1) gwo[i] += __shfl_xor(gwo[i], o, 64);
    for (int o = 1; o < 16; o <<= 1) gbo += __shfl_xor(gbo, o, 64);
    const int64_t nwaves = w.nwaves_total;
    const int64_t wid = w.wave0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row == 0) {
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int j = 0; j < 4; ++j) w.part[wid * W + 16 * o + 4 * g + j] = gwo[4 * o + j];
        if (g == 0) w.part[nwaves * W + wid] = gbo;
    }
}

// Split-K GEMM over points: part[blk][m][n] = sum over block blk's points p of L[m][p] R[n][p],
// L [64][P] and R [N][P] BF16 (N = 16 NT, P a multiple of 16), FP32 accumulation on MFMA.  Each
// block owns a contiguous range of GPB points and every output tile: per round it stages 64
// points of all 64 + N rows in LDS (each row's 128 bytes read as one coalesced segment), laid
// out so that every MFMA operand is 512 contiguous bytes, and wavefront w multiplies output
// rows 16 w .. 16 w + 15 against all N columns, its A operand loaded once per 16 points.  With
// rowpart the block also writes the row sums of L over its points (rowpart[blk][64]).
constexpr int GPB = 1024;   // points per block
constexpr int GK = 64;      // points per LDS round

template <int NT>
__global__ __launch_bounds__(256) void k_gemm_nt_rows(const uint16_t* __restrict__ L,
                                                      const uint16_t* __restrict__ R, int64_t P,
                                                      float* __restrict__ part,
                                                      float* __restrict__ rowpart)
{
    constexpr int ROWS = 64 + 16 * NT;
    constexpr int PER = ROWS * 16 / 256;   // 8-byte segments each thread stages per round
    static_assert(ROWS * 16 % 256 == 0, "rounds split evenly over the block");
    __shared__ v4s sl[4 * 4 * 64];     // [row block][16-point step][lane]
    __shared__ v4s sr[NT * 4 * 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v4f acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t p0 = (int64_t)blockIdx.x * GPB;
    const int64_t p1 = min(p0 + (int64_t)GPB, P);
    // the next round's segments are fetched into registers while this round multiplies
    v4s nxt[PER];
    auto fetch = [&](int64_t q0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = (int)threadIdx.x + i * 256;
            const int r = e >> 4, c = e & 15;
            const int64_t q = q0 + 4 * c;
            const bool isl = r < 64;
            const uint16_t* src = (isl ? L : R) + (int64_t)(isl ? r : r - 64) * P;
            nxt[i] = q < p1 ? *reinterpret_cast<const v4s*>(src + q) : v4s{0, 0, 0, 0};
        }
    };
    if (p0 < p1) fetch(p0);
    float rsum = 0.0f;
    for (int64_t q0 = p0; q0 < p1; q0 += GK) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = (int)threadIdx.x + i * 256;
            const int r = e >> 4, c = e & 15;
            const bool isl = r < 64;
            const int rr = isl ? r : r - 64;
            const int slot = ((rr >> 4) * 4 + (c >> 2)) * 64 + (rr & 15) + 16 * (c & 3);
            if (isl)
                sl[slot] = nxt[i];
            else
                sr[slot] = nxt[i];
        }
        __syncthreads();
        if (q0 + GK < p1) fetch(q0 + GK);
#pragma unroll
        for (int st = 0; st < 4; st += 2) {
            const v4s a0 = sl[(w * 4 + st) * 64 + lane];
            const v4s a1 = sl[(w * 4 + st + 1) * 64 + lane];
            rsum += (from_bf16((uint16_t)a0.x) + from_bf16((uint16_t)a0.y)) +
                    (from_bf16((uint16_t)a0.z) + from_bf16((uint16_t)a0.w));
            rsum += (from_bf16((uint16_t)a1.x) + from_bf16((uint16_t)a1.y)) +
                    (from_bf16((uint16_t)a1.z) + from_bf16((uint16_t)a1.w));
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[t] = mfma2(a0, a1, sr[(t * 4 + st) * 64 + lane], sr[(t * 4 + st + 1) * 64 + lane],
                               acc[t]);
        }
    }
    // row sums of L (the bias gradient when L = dZ): lane (row, g) holds a quarter of row
    // 16 w + row; the four quarters are added across g
    rsum += __shfl_xor(rsum, 16, 64);
    rsum += __shfl_xor(rsum, 32, 64);
    if (rowpart && lane < 16) rowpart[(int64_t)blockIdx.x * 64 + 16 * w + lane] = rsum;
    // acc[t] holds output rows 16 w + 4 g + j, column 16 t + (lane & 15)
    const int g = lane >> 4, col = lane & 15;
    float* out = part + (int64_t)blockIdx.x * 64 * (16 * NT);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        out[(16 * w + 4 * g + 0) * (16 * NT) + 16 * t + col] = acc[t].x;
        out[(16 * w + 4 * g + 1) * (16 * NT) + 16 * t + col] = acc[t].y;
        out[(16 * w + 4 * g + 2) * (16 * NT) + 16 * t + col] = acc[t].z;
        out[(16 * w + 4 * g + 3) * (16 * NT) + 16 * t + col] = acc[t].w;
    }
}

// out[e] += sum_c part[c][e] in a fixed order: 64 elements per block, wavefront w summing
// chunks w, w + 4, ..., then the four sums added in order
// Sum over the nchunk partials of element e: SUM_WAVES wavefronts of the block share the
// chunks (chunk c to wavefront c mod SUM_WAVES), each with four independent accumulators so
// that its loads are in flight together, then the wavefronts' sums are added in a fixed order.
constexpr int SUM_WAVES = 16;
constexpr int SUM_THREADS = 64 * SUM_WAVES;

__device__ __forceinline__ float sum_chunks(const float* __restrict__ part, int64_t nchunk,
                                            int64_t n, int64_t e)
{
    __shared__ float sh[SUM_WAVES][64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    if (e < n) {
        int64_t c = w;
        for (; c + 3 * SUM_WAVES < nchunk; c += 4 * SUM_WAVES) {
            a0 += part[c * n + e];
            a1 += part[(c + SUM_WAVES) * n + e];
            a2 += part[(c + 2 * SUM_WAVES) * n + e];
            a3 += part[(c + 3 * SUM_WAVES) * n + e];
        }
        for (; c < nchunk; c += SUM_WAVES) a0 += part[c * n + e];
    }
    sh[w][l] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    float t = 0.0f;
#pragma unroll
    for (int i = 0; i < SUM_WAVES; ++i) t += sh[i][l];
    return t;
}

__global__ __launch_bounds__(SUM_THREADS) void k_sum_parts(const float* __restrict__ part,
                                                           int64_t nchunk, int64_t n,
                                                           float* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    const float s = sum_chunks(part, nchunk, n, e);
    if (threadIdx.x < 64 && e < n) out[e] += s;
}

// The same for the first layer's weights, whose K dimension the GPU holds in its own encoding
// order: out[m][natural_feature(i)] += sum_c part[c][m][i]; padding slots are dropped.
template <int KT>
__global__ __launch_bounds__(SUM_THREADS) void k_sum_parts_in(const float* __restrict__ part,
                                                      int64_t nchunk, int n_freq,
                                                      float* __restrict__ out)
{
    constexpr int N = 16 * KT;
    const int e = blockIdx.x * 64 + (threadIdx.x & 63);
    const float s = sum_chunks(part, nchunk, W * N, e);
    if (threadIdx.x >= 64 || e >= W * N) return;
    const int m = e / N, nf = natural_feature<KT>(e % N, n_freq);
    if (nf < 0) return;
    out[m * N + nf] += s;
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ in,
                                                 uint16_t* __restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = to_bf16(in[i]);
}

}  // namespace

template <int KT, int DEPTH>
void chain_blocks_t(const NrfArgs& a, int64_t np, unsigned* nb)
{
    (void)a;
    *nb = nrfcore::blocks_for_tiles(k_nrf_chain<KT, DEPTH>, np / 16);
}

template <int KT, int DEPTH>
void launch_chain_t(const NrfArgs& a, const NrfWork& w, unsigned nb, hipStream_t s)
{
    hipLaunchKernelGGL((k_nrf_chain<KT, DEPTH>), dim3(nb), dim3(256), 0, s, a, w);
}

int nrf_max_bands(int in_pad) { return in_pad == 64 ? max_bands<4>() : max_bands<8>(); }

size_t nrf_part_floats(int64_t P, int in_pad)
{
    const int64_t gemm = ((P + GPB - 1) / GPB) * W * ((in_pad > W ? in_pad : W) + 1);
    // the chain kernel's output-layer partials: W + 1 per wavefront, at most np/16 + 3 of them
    // for each grid of a call
    const int64_t rows = (int64_t)(W + 1) * (P / 16 + 4 * GM_MAX_GRIDS);
    return (size_t)(gemm > rows ? gemm : rows);
}

unsigned nrf_chain_blocks(const NrfArgs& a, int64_t np)
{
    unsigned nb = 0;
    switch ((a.in_pad >> 4) * 8 + a.depth) {
    case 4 * 8 + 1: chain_blocks_t<4, 1>(a, np, &nb); break;
    case 4 * 8 + 2: chain_blocks_t<4, 2>(a, np, &nb); break;
    case 4 * 8 + 3: chain_blocks_t<4, 3>(a, np, &nb); break;
    case 4 * 8 + 4: chain_blocks_t<4, 4>(a, np, &nb); break;
    case 8 * 8 + 1: chain_blocks_t<8, 1>(a, np, &nb); break;
    case 8 * 8 + 2: chain_blocks_t<8, 2>(a, np, &nb); break;
    case 8 * 8 + 3: chain_blocks_t<8, 3>(a, np, &nb); break;
    case 8 * 8 + 4: chain_blocks_t<8, 4>(a, np, &nb); break;
    default: break;
    }
    return nb;
}

// One chain launch per grid, each writing its points' columns of the shared workspace and its
// wavefronts' output-layer partials; then the output layer's sums and, once over all the
// points, the layers' weight-gradient GEMMs and sums.
hipError_t launch_nrf_backward_grids(const NrfArgs* as, int n, const NrfWork& w, hipStream_t s)
{
    const NrfArgs& a = as[0];
    unsigned nb[GM_MAX_GRIDS];
    int64_t np[GM_MAX_GRIDS], totw = 0;
    for (int k = 0; k < n; ++k) {
        np[k] = ((as[k].n_points + 15) / 16) * 16;
        nb[k] = np[k] > 0 ? nrf_chain_blocks(as[k], np[k]) : 0;
        if (np[k] > 0 && nb[k] == 0) return hipErrorInvalidValue;
        totw += (int64_t)nb[k] * 4;
    }
    if (totw == 0) return hipSuccess;
    int64_t p0 = 0, wave0 = 0;
    for (int k = 0; k < n; ++k) {
        if (np[k] == 0) continue;
        NrfWork wk = w;
        wk.p0 = p0;
        wk.np = np[k];
        wk.wave0 = wave0;
        wk.nwaves_total = totw;
        const NrfArgs& ak = as[k];
        GM_NRF_DISPATCH(launch_chain_t, ak, wk, nb[k], s)
        p0 += np[k];
        wave0 += (int64_t)nb[k] * 4;
    }
    // the output layer's gradient from the chain kernels' per-wavefront partials (the layer
    // GEMMs below reuse the partial buffer after these sums)
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(SUM_THREADS), 0, s, w.part, totw, (int64_t)W,
                       a.g_w_out);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(SUM_THREADS), 0, s, w.part + totw * W, totw,
                       (int64_t)1, a.g_b_out);
    const int64_t nchunk = (w.P + GPB - 1) / GPB;
    for (int l = 0; l < a.depth; ++l) {
        const int N = l == 0 ? a.in_pad : W;
        float* dst = l == 0 ? a.g_w_in : a.g_w_hid + (int64_t)(l - 1) * W * W;
        float* dbias = l == 0 ? a.g_b_in : a.g_b_hid + (int64_t)(l - 1) * W;
        // block row sums of dZ_l (the bias gradient) after the GEMM partials
        float* rowpart = w.part + nchunk * W * N;
        if (N == 128)
            hipLaunchKernelGGL(k_gemm_nt_rows<8>, dim3((unsigned)nchunk), dim3(256), 0, s, w.dz[l],
                               w.a[l], w.P, w.part, rowpart);
        else
            hipLaunchKernelGGL(k_gemm_nt_rows<4>, dim3((unsigned)nchunk), dim3(256), 0, s, w.dz[l],
                               w.a[l], w.P, w.part, rowpart);
        const int64_t ne = (int64_t)W * N;
        const dim3 grid((unsigned)((ne + 63) / 64));
        if (l > 0)
            hipLaunchKernelGGL(k_sum_parts, grid, dim3(SUM_THREADS), 0, s, w.part, nchunk, ne, dst);
        else if (N == 64)
            hipLaunchKernelGGL(k_sum_parts_in<4>, grid, dim3(SUM_THREADS), 0, s, w.part, nchunk,
                               a.n_freq, dst);
        else
            hipLaunchKernelGGL(k_sum_parts_in<8>, grid, dim3(SUM_THREADS), 0, s, w.part, nchunk,
                               a.n_freq, dst);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(SUM_THREADS), 0, s, rowpart, nchunk, (int64_t)W,
                           dbias);
    }
    return hipGetLastError();
}

hipError_t launch_nrf_backward(const NrfArgs& a, const NrfWork& w, hipStream_t s)
{
    if (a.n_points <= 0) return hipSuccess;
    return launch_nrf_backward_grids(&a, 1, w, s);
}

hipError_t launch_to_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)b), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
