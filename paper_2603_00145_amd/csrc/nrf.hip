// K11: neural residual field (Sec. 3.4, Eq. 8) on MFMA: BF16 weights and activations,
// FP32 accumulation.
//
// r(x) = out_scale tanh(w_out . a_D + b_out),  a_l = SiLU(W_l a_{l-1} + b_l),
// a_0 = gamma(x) = (x, sin(2^k pi x), cos(2^k pi x), k < n_freq), zero-padded to in_pad.
//
// Layout trick: each layer is computed transposed, Z^T = W X^T, with the 16x16x16 BF16 MFMA
// (A = 16 output features x 16 input features of W, B = 16 input features x 16 points).  The
// MFMA result holds, per lane, 4 consecutive output features of one point - exactly the B
// operand layout of the next layer - so activations never leave registers inside a layer
// stack.  The encoding is computed directly in that layout.
//
// Backward (for a list of sampled voxels): recompute, then per layer dZ_l = dA_l * SiLU'(Z_l),
// dA_{l-1} = W_l^T dZ_l (MFMA); dZ_l and A_{l-1} are written feature-major (BF16) and the
// weight gradients dW_l = dZ_l A_{l-1}^T are formed by a split-K MFMA GEMM over the points.
#include "gm_internal.h"

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int W = 64;          // hidden width (fixed)
constexpr int MAX_IN = 128;    // in_pad <= 128
constexpr int MAX_DEPTH = 4;   // depth <= 4, in_pad in {64, 128}

// float -> bfloat16 bits, round to nearest even (gfx950's v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

// four floats -> BF16 bits, round to nearest even, two per v_cvt_pk_bf16_f32
__device__ __forceinline__ v4s pack4(float a, float b, float c, float d)
{
    const uint32_t lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{a, b}, v2bf));
    const uint32_t hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{c, d}, v2bf));
    return __builtin_bit_cast(v4s, (uint64_t)lo | ((uint64_t)hi << 32));
}

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// sigmoid with the hardware reciprocal (1 ulp; the field runs in BF16): exp(-z) overflows to
// +inf for very negative z, whose reciprocal is 0, the right limit
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

// World coordinate of voxel (vx, vy, vz): binary64 without contraction (hipcc fuses a * b + c
// by default, the pragma stops it here), rounded once to binary32.
__device__ __forceinline__ float world_coord(const double* M, int vx, int vy, int vz)
{
#pragma clang fp contract(off)
    double s = M[0] * (double)vx;
    s = s + M[1] * (double)vy;
    s = s + M[2] * (double)vz;
    s = s + M[3];
    return (float)s;
}

// Order of the encoding along the first layer's K dimension on the GPU.  The MFMA B operand of
// K-tile t gives lane group g = lane / 16 the features 16 t + 4 g + j, j < 4; call c = 4 t + j
// the column of that slot.  The last column holds the raw coordinates (x[g] for g < 3, else
// padding); column c = 6 q + m holds frequency band 4 q + g of kind m (sin of axis m for m < 3,
// cos of axis m - 3).  Kind, axis and band offset are compile-time constants of the unrolled
// encoding loop and the lane group only shifts the band, so nothing per slot has to be looked
// up or kept in registers.  The first layer's weights are permuted into this order when they
// are staged and its weight gradient is permuted back.  Bands: up to 8 with 4 K-tiles, 20 with 8.
template <int KT>
__host__ __device__ constexpr int max_bands() { return 4 * ((4 * KT - 1) / 6); }

// natural feature index (x_a: a; sin(2^k pi x_a): 3 + 6 k + a; cos: 6 + 6 k + a) of GPU slot
// i = 16 t + 4 g + j, or -1 for padding
template <int KT>
__device__ __forceinline__ int natural_feature(int i, int n_freq)
{
    const int t = i >> 4, g = (i >> 2) & 3, j = i & 3, c = 4 * t + j;
    if (c == 4 * KT - 1) return g < 3 ? g : -1;
    const int q = c / 6, m = c - 6 * q, band = 4 * q + g;
    return band < n_freq ? 3 + 6 * band + m : -1;
}

// The encoding of the lane's point, in the B operand layout of the K-tiles.
template <int KT>
__device__ __forceinline__ void encode(const float x[3], int n_freq, v4s b0[KT])
{
    const int g = (threadIdx.x >> 4) & 3;
    const float xg = g == 0 ? x[0] : (g == 1 ? x[1] : x[2]);
    const int nb = n_freq - g;          // band 4 q + g exists for 4 q < nb
#pragma unroll
    for (int t = 0; t < KT; ++t) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * t + j;
            if (c == 4 * KT - 1) {
                v[j] = g < 3 ? xg : 0.0f;
            } else {
                const int q = c / 6, m = c % 6;
                const float phi = ldexpf(x[m % 3], 4 * q - 1 + g);   // exact power-of-two scaling
                const float frac = phi - rintf(phi);                  // exact
                // v_sin_f32 / v_cos_f32 take their argument in revolutions
                const float sc = m < 3 ? __builtin_amdgcn_sinf(frac) : __builtin_amdgcn_cosf(frac);
                v[j] = 4 * q < nb ? sc : 0.0f;
            }
        }
        b0[t] = pack4(v[0], v[1], v[2], v[3]);
    }
}

// Weights staged in LDS in MFMA A-operand order: operand (o, t) of a layer is 64 lanes x 4 BF16,
// lane (g, row) holding W[16 o + row][16 t + 4 g + j], so that a wavefront reads an operand as
// 512 contiguous bytes (one ds_read_b64 per lane, free of bank conflicts).
struct Lds {
    v4s w_in[4 * (MAX_IN / 16) * 64];              // [o][t][lane], K in the GPU encoding order
    v4s w_hid[(MAX_DEPTH - 1) * 16 * 64];          // [l][o][t][lane]
};
// the backward also needs W_l^T as A operand: [l][i][o][lane], lane (g, row) holding
// W_l[16 o + 4 g + j][16 i + row]
struct LdsChain {
    Lds f;
    v4s w_hid_t[(MAX_DEPTH - 1) * 16 * 64];
};

template <int KT>
__device__ void load_weights(const NrfArgs& a, Lds& s, v4s* w_hid_t = nullptr)
{
    for (int e = threadIdx.x; e < 4 * KT * 64; e += blockDim.x) {
        const int lane = e & 63, t = (e >> 6) % KT, o = (e >> 6) / KT;
        const int g = lane >> 4, row = lane & 15;
        const uint16_t* src = a.w_in + (16 * o + row) * (16 * KT);
        short v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int nf = natural_feature<KT>(16 * t + 4 * g + j, a.n_freq);
            v[j] = nf >= 0 ? (short)src[nf] : (short)0;
        }
        s.w_in[e] = v4s{v[0], v[1], v[2], v[3]};
    }
    const int nh = (a.depth - 1) * 16 * 64;
    for (int e = threadIdx.x; e < nh; e += blockDim.x) {
        const int lane = e & 63, t = (e >> 6) & 3, o = (e >> 8) & 3, l = e >> 10;
        const int g = lane >> 4, row = lane & 15;
        const uint16_t* Wl = a.w_hid + l * W * W;
        short v[4], vt[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = (short)Wl[(16 * o + row) * W + 16 * t + 4 * g + j];
            vt[j] = (short)Wl[(16 * t + 4 * g + j) * W + 16 * o + row];
        }
        s.w_hid[e] = v4s{v[0], v[1], v[2], v[3]};
        if (w_hid_t) w_hid_t[e] = v4s{vt[0], vt[1], vt[2], vt[3]};
    }
    __syncthreads();
}

// voxel (x, y, z) of point p (grids hold < 2^31 voxels, so 32-bit division suffices)
__device__ __forceinline__ void point_xyz(const NrfArgs& a, int64_t p, int* vx, int* vy, int* vz)
{
    uint32_t v = a.idx ? (uint32_t)a.idx[p] : (uint32_t)p;
    const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
    const uint32_t q = v / nx;
    *vx = (int)(v - q * nx);
    const uint32_t r = q / ny;
    *vy = (int)(q - r * ny);
    *vz = (int)r;
}

// Forward for the 16 points of a tile: Z (pre-activations) and the BF16 activations A
// (register layout: o-tile x 4 features of point lane&15).
template <int KT, int DEPTH>
struct Tile {
    v4f z[DEPTH][4];
    v4s act[DEPTH][4];
};

// Store a register tile (4 features x point p) feature-major into dst [features][P].
__device__ __forceinline__ void store_fm(uint16_t* dst, int f, int64_t P, int64_t p, v4s v)
{
    dst[(int64_t)(f + 0) * P + p] = (uint16_t)v.x;
    dst[(int64_t)(f + 1) * P + p] = (uint16_t)v.y;
    dst[(int64_t)(f + 2) * P + p] = (uint16_t)v.z;
    dst[(int64_t)(f + 3) * P + p] = (uint16_t)v.w;
}

// With a workspace (w != NULL) the encoding (in the GPU order) and each layer's BF16
// activations are written out feature-major as soon as they are formed (the backward needs
// them for dW), so they need not stay live in registers.
template <int KT, int DEPTH>
__device__ __forceinline__ void tile_forward(const NrfArgs& a, const Lds& s, const float x[3],
                                             Tile<KT, DEPTH>& T, const NrfWork* w = nullptr,
                                             int64_t p = 0)
{
    const int lane = threadIdx.x & 63, g = lane >> 4;
    v4s b0[KT];
    encode<KT>(x, a.n_freq, b0);
    if (w) {
#pragma unroll
        for (int t = 0; t < KT; ++t) store_fm(w->a[0], 16 * t + 4 * g, w->P, p, b0[t]);
    }
    // layer 1
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int f = 16 * o + 4 * g;
        v4f acc = {a.b_in[f], a.b_in[f + 1], a.b_in[f + 2], a.b_in[f + 3]};   // bias as C
#pragma unroll
        for (int t = 0; t < KT; ++t) acc = mfma(s.w_in[(o * KT + t) * 64 + lane], b0[t], acc);
        T.z[0][o] = acc;
        T.act[0][o] = pack4(silu(acc.x), silu(acc.y), silu(acc.z), silu(acc.w));
        if (w && DEPTH > 1) store_fm(w->a[1], f, w->P, p, T.act[0][o]);
    }
    // hidden layers
#pragma unroll
    for (int l = 1; l < DEPTH; ++l) {
        const v4s* Wl = s.w_hid + (l - 1) * 16 * 64;
        const float* bl = a.b_hid + (l - 1) * W;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int f = 16 * o + 4 * g;
            v4f acc = {bl[f], bl[f + 1], bl[f + 2], bl[f + 3]};
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = mfma(Wl[(o * 4 + t) * 64 + lane], T.act[l - 1][t], acc);
            T.z[l][o] = acc;
            T.act[l][o] = pack4(silu(acc.x), silu(acc.y), silu(acc.z), silu(acc.w));
            if (w && l + 1 < DEPTH) store_fm(w->a[l + 1], f, w->P, p, T.act[l][o]);
        }
    }
}

// output pre-activation z_o of the tile's point from the BF16 activations of the last layer
// (all 4 lane groups end with the total)
template <int KT, int DEPTH>
__device__ __forceinline__ float tile_output(const NrfArgs& a, const Tile<KT, DEPTH>& T)
{
    const int lane = threadIdx.x & 63, g = lane >> 4;
    float sacc = 0.0f;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const v4s h = T.act[DEPTH - 1][o];
        const int f = 16 * o + 4 * g;
        sacc += from_bf16(a.w_out[f]) * from_bf16((uint16_t)h.x) +
                from_bf16(a.w_out[f + 1]) * from_bf16((uint16_t)h.y) +
                from_bf16(a.w_out[f + 2]) * from_bf16((uint16_t)h.z) +
                from_bf16(a.w_out[f + 3]) * from_bf16((uint16_t)h.w);
    }
    sacc += __shfl_xor(sacc, 16, 64);
    sacc += __shfl_xor(sacc, 32, 64);
    return sacc + a.b_out[0];
}

template <int KT, int DEPTH>
__global__ __launch_bounds__(256) void k_nrf_forward(const NrfArgs a)
{
    __shared__ Lds s;
    load_weights<KT>(a, s);
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
    const int64_t ntiles = (a.n_points + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles;
         tile += (int64_t)gridDim.x * 4) {
        const int64_t p = tile * 16 + row;
        const bool valid = p < a.n_points;
        int vx = 0, vy = 0, vz = 0;
        if (valid) point_xyz(a, p, &vx, &vy, &vz);
        const float x[3] = {world_coord(a.m, vx, vy, vz), world_coord(a.m + 4, vx, vy, vz),
                            world_coord(a.m + 8, vx, vy, vz)};
        Tile<KT, DEPTH> T;
        tile_forward<KT, DEPTH>(a, s, x, T);
        const float zo = tile_output<KT, DEPTH>(a, T);
        if (valid && g == 0) {
            const int64_t v = ((int64_t)vz * a.ny + vy) * a.nx + vx;
            a.out[v] += a.out_scale * tanhf(zo);
        }
    }
}

// Recompute a tile and write, feature-major with point stride P: DZO (f32, per point), and
// for each layer l (1..D) dZ_l [W][P] and A_{l-1} [in_l][P] (BF16), plus A_D [W][P].
template <int KT, int DEPTH>
__global__ __launch_bounds__(256) void k_nrf_chain(const NrfArgs a, NrfWork w)
{
    __shared__ LdsChain s;
    load_weights<KT>(a, s.f, s.w_hid_t);
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
    const int64_t P = w.P;
    const int64_t ntiles = P / 16;
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
        tile_forward<KT, DEPTH>(a, s.f, x, T, &w, p);
        const float zo = tile_output<KT, DEPTH>(a, T);
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
                store_fm(w.dz[l], 16 * o + 4 * g, P, p, dz[o]);
            }
            if (l == 0) break;
            // dA_{l-1} = W_l^T dZ_l
            const v4s* Wt = s.w_hid_t + (l - 1) * 16 * 64;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int o = 0; o < 4; ++o) acc = mfma(Wt[(i * 4 + o) * 64 + lane], dz[o], acc);
                da[i] = acc;
            }
        }
    }
    // sum over the 16 points of each lane group, then one partial per wavefront:
    // part[wave][64] for w_out, then part[nwaves * 64 + wave] for b_out
#pragma unroll
    for (int i = 0; i < 16; ++i)
        for (int o = 1; o < 16; o <<= 1) gwo[i] += __shfl_xor(gwo[i], o, 64);
    for (int o = 1; o < 16; o <<= 1) gbo += __shfl_xor(gbo, o, 64);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
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
        for (int st = 0; st < 4; ++st) {
            const v4s a = sl[(w * 4 + st) * 64 + lane];
            rsum += (from_bf16((uint16_t)a.x) + from_bf16((uint16_t)a.y)) +
                    (from_bf16((uint16_t)a.z) + from_bf16((uint16_t)a.w));
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = mfma(a, sr[(t * 4 + st) * 64 + lane], acc[t]);
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

// Grid of a tile loop: every block resident at once (the blocks then take equal shares of the
// tiles, with no partial last wave of blocks), capped by the work.
template <typename K>
unsigned blocks_for_tiles(K kernel, int64_t ntiles)
{
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0);
    int64_t full = (int64_t)(cus > 0 ? cus : 256) * (per_cu > 0 ? per_cu : 1);
    int64_t b = (ntiles + 3) / 4;
    if (b > full) b = full;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

template <int KT, int DEPTH>
void launch_fwd_t(const NrfArgs& a, hipStream_t s)
{
    const unsigned nb = blocks_for_tiles(k_nrf_forward<KT, DEPTH>, (a.n_points + 15) / 16);
    hipLaunchKernelGGL((k_nrf_forward<KT, DEPTH>), dim3(nb), dim3(256), 0, s, a);
}

template <int KT, int DEPTH>
void launch_chain_t(const NrfArgs& a, const NrfWork& w, hipStream_t s, int64_t* nwaves)
{
    const unsigned nb = blocks_for_tiles(k_nrf_chain<KT, DEPTH>, w.P / 16);
    *nwaves = (int64_t)nb * 4;
    hipLaunchKernelGGL((k_nrf_chain<KT, DEPTH>), dim3(nb), dim3(256), 0, s, a, w);
}

// supported shapes: in_pad 64 or 128 (4 or 8 K-tiles; at most max_bands<KT>() bands), depth 1..4
#define GM_NRF_DISPATCH(FN, ...)                                                           \
    switch ((a.in_pad >> 4) * 8 + a.depth) {                                               \
    case 4 * 8 + 1: FN<4, 1>(__VA_ARGS__); break;                                          \
    case 4 * 8 + 2: FN<4, 2>(__VA_ARGS__); break;                                          \
    case 4 * 8 + 3: FN<4, 3>(__VA_ARGS__); break;                                          \
    case 4 * 8 + 4: FN<4, 4>(__VA_ARGS__); break;                                          \
    case 8 * 8 + 1: FN<8, 1>(__VA_ARGS__); break;                                          \
    case 8 * 8 + 2: FN<8, 2>(__VA_ARGS__); break;                                          \
    case 8 * 8 + 3: FN<8, 3>(__VA_ARGS__); break;                                          \
    case 8 * 8 + 4: FN<8, 4>(__VA_ARGS__); break;                                          \
    default: return hipErrorInvalidValue;                                                  \
    }

int nrf_max_bands(int in_pad) { return in_pad == 64 ? max_bands<4>() : max_bands<8>(); }

hipError_t launch_nrf_forward(const NrfArgs& a, hipStream_t s)
{
    if (a.n_points <= 0) return hipSuccess;
    GM_NRF_DISPATCH(launch_fwd_t, a, s)
    return hipGetLastError();
}

size_t nrf_part_floats(int64_t P, int in_pad)
{
    const int64_t gemm = ((P + GPB - 1) / GPB) * W * ((in_pad > W ? in_pad : W) + 1);
    // the chain kernel's output-layer partials: W + 1 per wavefront, at most P/16 + 3 of them
    const int64_t rows = (int64_t)(W + 1) * (P / 16 + 4);
    return (size_t)(gemm > rows ? gemm : rows);
}

hipError_t launch_nrf_backward(const NrfArgs& a, const NrfWork& w, hipStream_t s)
{
    if (a.n_points <= 0) return hipSuccess;
    int64_t nwaves = 0;
    GM_NRF_DISPATCH(launch_chain_t, a, w, s, &nwaves)
    // the output layer's gradient from the chain kernel's per-wavefront partials (the layer
    // GEMMs below reuse the partial buffer after these sums)
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(SUM_THREADS), 0, s, w.part, nwaves, (int64_t)W,
                       a.g_w_out);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(SUM_THREADS), 0, s, w.part + nwaves * W, nwaves,
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
        const int64_t n = (int64_t)W * N;
        const dim3 grid((unsigned)((n + 63) / 64));
        if (l > 0)
            hipLaunchKernelGGL(k_sum_parts, grid, dim3(SUM_THREADS), 0, s, w.part, nchunk, n, dst);
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

hipError_t launch_to_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)b), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
