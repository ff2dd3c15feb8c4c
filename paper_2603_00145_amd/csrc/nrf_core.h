// Device code of the neural residual field (Sec. 3.4, Eq. 8) shared by the field's own kernels
// and by the renderer's fused epilogue: BF16 operands on gfx950's 16x16x32 MFMA with FP32
// accumulation, the sinusoidal encoding computed in the MFMA operand layout, weights staged in
// LDS in operand order, and the forward of one 16-point tile kept in registers.
#ifndef GM_NRF_CORE_H
#define GM_NRF_CORE_H
#include "gm_internal.h"

namespace nrfcore {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int W = 64;          // hidden width (fixed); in_pad is 64 or 128, depth 1..4

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

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// gfx950's 16x16x32 BF16 MFMA on two 16-wide K halves: lane group g supplies, in A and in B
// alike, slots 4 g + j of the first half (a0, b0) and of the second (a1, b1), so the sum runs
// over all 32 slots whatever order the hardware gives them.  A 16x16x16 operand tile of each
// half is used unchanged, and the result has the 16x16x16 layout (lane group g: rows 4 g + j).
__device__ __forceinline__ v4f mfma2(v4s a0, v4s a1, v4s b0, v4s b1, v4f c)
{
    const v8bf a = __builtin_bit_cast(v8bf, __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7));
    const v8bf b = __builtin_bit_cast(v8bf, __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7));
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
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
// 512 contiguous bytes (one ds_read_b64 per lane, free of bank conflicts).  Sized for KT K-tiles
// of the first layer and DEPTH - 1 hidden layers.
template <int KT, int DEPTH>
struct Lds {
    v4s w_in[4 * KT * 64];                                 // [o][t][lane], GPU encoding order
    v4s w_hid[(DEPTH > 1 ? DEPTH - 1 : 1) * 16 * 64];      // [l][o][t][lane]
};
// the backward also needs W_l^T as A operand: [l][i][o][lane], lane (g, row) holding
// W_l[16 o + 4 g + j][16 i + row]
template <int KT, int DEPTH>
struct LdsChain {
    Lds<KT, DEPTH> f;
    v4s w_hid_t[(DEPTH > 1 ? DEPTH - 1 : 1) * 16 * 64];
};

// Stages the weights (every thread of the block takes part; ends with a block barrier).
template <int KT, int DEPTH>
__device__ void load_weights(const NrfArgs& a, Lds<KT, DEPTH>& s, v4s* w_hid_t = nullptr)
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
    const int nh = (DEPTH - 1) * 16 * 64;
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

// Where tile_forward takes the layers' MFMA A operands from: the LDS stage, read at each use,
// or the wavefront's registers (each lane its quad of every operand, 4 KT + 16 (DEPTH - 1)
// quads, copied once from the stage; the per-tile LDS reads of the weights, 512 bytes per lane,
// then disappear).
template <int KT, int DEPTH>
struct WeightsLds {
    const Lds<KT, DEPTH>& s;
    int lane;
    __device__ v4s in(int o, int t) const { return s.w_in[(o * KT + t) * 64 + lane]; }
    __device__ v4s hid(int l, int o, int t) const
    {
        return s.w_hid[((l - 1) * 16 + o * 4 + t) * 64 + lane];
    }
};
template <int KT, int DEPTH>
struct WeightsReg {
    v4s w_in[4 * KT];
    v4s w_hid[(DEPTH > 1 ? DEPTH - 1 : 1) * 16];
    __device__ void load(const Lds<KT, DEPTH>& s, int lane)
    {
#pragma unroll
        for (int i = 0; i < 4 * KT; ++i) w_in[i] = s.w_in[i * 64 + lane];
#pragma unroll
        for (int i = 0; i < (DEPTH - 1) * 16; ++i) w_hid[i] = s.w_hid[i * 64 + lane];
    }
    __device__ v4s in(int o, int t) const { return w_in[o * KT + t]; }
    __device__ v4s hid(int l, int o, int t) const { return w_hid[(l - 1) * 16 + o * 4 + t]; }
};

// With a workspace (w != NULL) the encoding (in the GPU order) and each layer's BF16
// activations are written out feature-major as soon as they are formed (the backward needs
// them for dW), so they need not stay live in registers.
template <int KT, int DEPTH, typename WS>
__device__ __forceinline__ void tile_forward_w(const NrfArgs& a, const WS& ws, const float x[3],
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
        for (int t = 0; t < KT; t += 2)
            acc = mfma2(ws.in(o, t), ws.in(o, t + 1), b0[t], b0[t + 1], acc);
        T.z[0][o] = acc;
        T.act[0][o] = pack4(silu(acc.x), silu(acc.y), silu(acc.z), silu(acc.w));
        if (w && DEPTH > 1) store_fm(w->a[1], f, w->P, p, T.act[0][o]);
    }
    // hidden layers
#pragma unroll
    for (int l = 1; l < DEPTH; ++l) {
        const float* bl = a.b_hid + (l - 1) * W;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int f = 16 * o + 4 * g;
            v4f acc = {bl[f], bl[f + 1], bl[f + 2], bl[f + 3]};
#pragma unroll
            for (int t = 0; t < 4; t += 2)
                acc = mfma2(ws.hid(l, o, t), ws.hid(l, o, t + 1), T.act[l - 1][t],
                            T.act[l - 1][t + 1], acc);
            T.z[l][o] = acc;
            T.act[l][o] = pack4(silu(acc.x), silu(acc.y), silu(acc.z), silu(acc.w));
            if (w && l + 1 < DEPTH) store_fm(w->a[l + 1], f, w->P, p, T.act[l][o]);
        }
    }
}

// tile_forward_w with the weights read from the LDS stage at each use
template <int KT, int DEPTH>
__device__ __forceinline__ void tile_forward(const NrfArgs& a, const Lds<KT, DEPTH>& s, const float x[3],
                                             Tile<KT, DEPTH>& T, const NrfWork* w = nullptr,
                                             int64_t p = 0)
{
    const WeightsLds<KT, DEPTH> ws{s, (int)(threadIdx.x & 63)};
    tile_forward_w<KT, DEPTH>(a, ws, x, T, w, p);
}

// The output layer as a 16-row MFMA A operand whose row 0 is w_out and the other rows zero:
// lane (g, 0) holds w_out[16 t + 4 g + j] of K-tile t.  Loaded once per wavefront.
__device__ __forceinline__ void load_wout(const NrfArgs& a, v4s (&wo)[4])
{
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const v4s v = *reinterpret_cast<const v4s*>(a.w_out + 16 * t + 4 * g);
        wo[t] = row == 0 ? v : v4s{0, 0, 0, 0};
    }
}

// output pre-activation z_o of the tile's point from the BF16 activations of the last layer,
// on the matrix cores (wo from load_wout): row 0 of the product, held by lane group 0, is
// w_out . a_D for the lane's point.  Valid in lane group 0 only (the other groups get b_out).
template <int KT, int DEPTH>
__device__ __forceinline__ float tile_output(const NrfArgs& a, const Tile<KT, DEPTH>& T,
                                             const v4s (&wo)[4])
{
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = mfma2(wo[0], wo[1], T.act[DEPTH - 1][0], T.act[DEPTH - 1][1], acc);
    acc = mfma2(wo[2], wo[3], T.act[DEPTH - 1][2], T.act[DEPTH - 1][3], acc);
    return acc.x + a.b_out[0];
}

// Grid of a tile loop: every block resident at once (the blocks then take equal shares of the
// tiles, with no partial last wave of blocks), capped by the work.
template <typename K>
inline unsigned blocks_for_tiles(K kernel, int64_t ntiles)
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

}  // namespace nrfcore

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

#endif
