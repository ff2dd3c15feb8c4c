// K12: warm-start network - per Gaussian a 3-channel 8^3 patch of the registered stacks
// through four 3D convolutions (width 32, BF16 weights and activations, FP32 accumulation on
// MFMA) and a linear head that predicts residuals (d log-scale 3, d quaternion 4, d logit 1)
// on top of the devoxelization initialisation.  Training backward (dX and dW) on MFMA.
//
// Every convolution is an implicit GEMM on the 16x16x16 BF16 MFMA with one operand gathered
// on the fly (no im2col buffer):
//   forward      Z[o][(b,p_out)]   = sum_{(c,tap)} W[o][(c,tap)] X[b][c][p_in(p_out,tap)]
//   backward-X   dX[c][(b,p_in)]   = sum_{(o,tap)} W[o][(c,tap)] dZ[b][o][p_out(p_in,tap)]
//   backward-W   dW[o][(c,tap)]    = sum_{(b,p_out)} dZ[b][o][p_out] X[b][c][p_in(p_out,tap)]
// Activations are stored [sample][channel][position] (BF16, pre-activations FP32).
#include "gm_internal.h"

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (gfx950's v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// sigmoid with the hardware reciprocal (1 ulp; the network runs in BF16): exp(-z) overflows
// to +inf for very negative z, whose reciprocal is 0, the right limit
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// gfx950's 16x16x32 BF16 MFMA over two 16-wide K halves: lane group g supplies, in A and in B
// alike, slots 4 g + j of the first half (a0, b0) and of the second (a1, b1), so the product
// sums all 32 slots whatever order the hardware gives them.  The result has the 16x16x16
// layout (lane group g: rows 4 g + j of column lane & 15).
__device__ __forceinline__ v4f mfma2(v4s a0, v4s a1, v4s b0, v4s b1, v4f c)
{
    const v8bf a = __builtin_bit_cast(v8bf, __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7));
    const v8bf b = __builtin_bit_cast(v8bf, __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7));
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int CO = 32;

// layer geometry: CI input channels, K^3 taps, stride ST, padding PD, DI^3 -> DO^3
template <int CI_, int K_, int ST_, int PD_, int DI_, int DO_>
struct Geo {
    static constexpr int CI = CI_, K = K_, ST = ST_, PD = PD_, DI = DI_, DO = DO_;
    static constexpr int KV = K * K * K;
    static constexpr int PI = DI * DI * DI, PO = DO * DO * DO;
    static constexpr int KREAL = CI * KV;
    static constexpr int KPAD = (KREAL + 15) / 16 * 16;
};
using G1 = Geo<3, 3, 1, 1, 8, 8>;
using G2 = Geo<32, 3, 2, 1, 8, 4>;
using G3 = Geo<32, 3, 2, 1, 4, 2>;
using G4 = Geo<32, 2, 1, 0, 2, 1>;

// ---- forward ------------------------------------------------------------------------------
// C tile = 16 output channels x 16 columns (sample, output position); one wavefront per tile.
template <class G>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ W,
                                                  const float* __restrict__ bias,
                                                  const uint16_t* __restrict__ X, int64_t B,
                                                  float* __restrict__ Z, uint16_t* __restrict__ A)
{
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
    const int64_t ncol = B * G::PO;
    const int64_t ntile = ncol / 16;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= ntile) return;
    const int m0 = 16 * blockIdx.y;
    const int64_t n = tile * 16 + row;                 // this lane's column
    const int64_t b = n / G::PO;
    const int p = (int)(n - b * G::PO);
    const int oz = p / (G::DO * G::DO), oy = (p / G::DO) % G::DO, ox = p % G::DO;
    const uint16_t* xb = X + b * G::CI * G::PI;
    static_assert(G::KPAD % 32 == 0, "whole 32-wide K steps");
    // the A and B fragments of the 16-wide K block at k0
    auto frag = [&](int k0, v4s& Af, v4s& Bf) {
        Af = *reinterpret_cast<const v4s*>(W + (m0 + row) * G::KPAD + k0 + 4 * g);
        short bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + 4 * g + j;
            const int c = k / G::KV, t = k - c * G::KV;
            const int kz = t / (G::K * G::K), ky = (t / G::K) % G::K, kx = t % G::K;
            const int iz = G::ST * oz - G::PD + kz, iy = G::ST * oy - G::PD + ky,
                      ix = G::ST * ox - G::PD + kx;
            const bool ok = k < G::KREAL && iz >= 0 && iz < G::DI && iy >= 0 && iy < G::DI &&
                            ix >= 0 && ix < G::DI;
            const int idx = ok ? c * G::PI + (iz * G::DI + iy) * G::DI + ix : 0;  // always valid
            const short v = (short)xb[idx];
            bv[j] = ok ? v : (short)0;
        }
        Bf = v4s{bv[0], bv[1], bv[2], bv[3]};
    };
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < G::KPAD; k0 += 32) {
        v4s A0, B0, A1, B1;
        frag(k0, A0, B0);
        frag(k0 + 16, A1, B1);
        acc = mfma2(A0, A1, B0, B1, acc);
    }
    const float av[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = m0 + 4 * g + j;
        const float z = av[j] + bias[m];
        const int64_t o = (b * CO + m) * G::PO + p;
        if (Z) Z[o] = z;  // the pre-activation is kept for the backward only
        A[o] = to_bf16(silu(z));
    }
}

// Forward for the layers whose sample has a multiple of 16 output positions: one block per
// sample.  The sample's input is staged in LDS, zero-padded as far as the windows reach past
// it (PD below, up to PD above), with a table
// of each K index's offset in it (channel, kz, ky, kx), so that a B-fragment element costs a
// table entry (four per 16-byte read) and one LDS read, with no index arithmetic or bounds
// check; K indices past the real taps read as zero.  The wavefronts share the sample's
// (output-channel tile, column tile) pairs.
template <class G>
__global__ __launch_bounds__(256) void k_conv_fwd_lds(const uint16_t* __restrict__ W,
                                                      const float* __restrict__ bias,
                                                      const uint16_t* __restrict__ X,
                                                      float* __restrict__ Z,
                                                      uint16_t* __restrict__ A)
{
    static_assert(G::PO % 16 == 0, "whole column tiles per sample");
    // padding: PD below; above, only as far as the last window reaches past the input
    constexpr int REACH = G::ST * (G::DO - 1) - G::PD + G::K;   // one past the last index read
    constexpr int PH = REACH > G::DI ? REACH - G::DI : 0;
    constexpr int DP = G::PD + G::DI + PH, PP = DP * DP * DP;
    static_assert(G::CI * PP * 2 + G::KPAD * 4 <= 65536, "staged input and table fit 64 KB");
    constexpr int NCT = G::PO / 16;            // column tiles per sample
    __shared__ uint16_t xin[G::CI * PP];
    __shared__ __align__(16) int koff[G::KPAD];
    const int64_t b = blockIdx.x;
    for (int k = threadIdx.x; k < G::KPAD; k += 256) {
        int o = -1;
        if (k < G::KREAL) {
            const int c = k / G::KV, t = k - c * G::KV;
            const int kz = t / (G::K * G::K), ky = (t / G::K) % G::K, kx = t % G::K;
            o = c * PP + (kz * DP + ky) * DP + kx;
        }
        koff[k] = o;
    }
    for (int i = threadIdx.x; i < G::CI * PP; i += 256) xin[i] = 0;
    __syncthreads();
    const uint16_t* xb = X + b * G::CI * G::PI;
    for (int i = threadIdx.x; i < G::CI * G::PI; i += 256) {
        const int c = i / G::PI, r = i - c * G::PI;
        const int z = r / (G::DI * G::DI), y = (r / G::DI) % G::DI, x = r % G::DI;
        xin[c * PP + ((z + G::PD) * DP + (y + G::PD)) * DP + (x + G::PD)] = xb[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
    for (int tI = threadIdx.x >> 6; tI < 2 * NCT; tI += 4) {
        const int m0 = 16 * (tI / NCT);
        const int p = (tI % NCT) * 16 + row;  // this lane's output position
        const int oz = p / (G::DO * G::DO), oy = (p / G::DO) % G::DO, ox = p % G::DO;
        const int base = ((G::ST * oz) * DP + G::ST * oy) * DP + G::ST * ox;
        auto frag = [&](int k0, v4s& Af, v4s& Bf) {
            Af = *reinterpret_cast<const v4s*>(W + (m0 + row) * G::KPAD + k0 + 4 * g);
            const int4 ko = *reinterpret_cast<const int4*>(koff + k0 + 4 * g);
            short bv[4];
            const int kk[4] = {ko.x, ko.y, ko.z, ko.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if constexpr (G::KPAD != G::KREAL) {
                    const short v = (short)xin[base + max(kk[j], 0)];
                    bv[j] = kk[j] < 0 ? (short)0 : v;
                } else {
                    bv[j] = (short)xin[base + kk[j]];
                }
            }
            Bf = v4s{bv[0], bv[1], bv[2], bv[3]};
        };
        static_assert(G::KPAD % 32 == 0, "whole 32-wide K steps");
        v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 3
        for (int k0 = 0; k0 < G::KPAD; k0 += 32) {
            v4s A0, B0, A1, B1;
            frag(k0, A0, B0);
            frag(k0 + 16, A1, B1);
            acc = mfma2(A0, A1, B0, B1, acc);
        }
        const float av[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + 4 * g + j;
            const float z = av[j] + bias[m];
            const int64_t o = (b * CO + m) * G::PO + p;
            if (Z) Z[o] = z;
            A[o] = to_bf16(silu(z));
        }
    }
}

// ---- backward through the input: dZ_prev = (W^T dZ) * SiLU'(Z_prev) -----------------------
// C tile = 16 input channels x 16 columns (sample, input position).
template <class G>
__global__ __launch_bounds__(256) void k_conv_bwd_x(const uint16_t* __restrict__ W,
                                                    const uint16_t* __restrict__ dZ, int64_t B,
                                                    const float* __restrict__ Zprev,
                                                    uint16_t* __restrict__ dZprev)
{
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
    const int64_t ncol = B * G::PI;
    const int64_t ntile = ncol / 16;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= ntile) return;
    const int m0 = 16 * blockIdx.y;                    // input channel tile
    const int64_t n = tile * 16 + row;
    const int64_t b = n / G::PI;
    const int p = (int)(n - b * G::PI);
    const int iz = p / (G::DI * G::DI), iy = (p / G::DI) % G::DI, ix = p % G::DI;
    const uint16_t* dzb = dZ + b * CO * G::PO;
    constexpr int KT = CO * G::KV;                     // reduction over (o, tap)
    static_assert(KT % 32 == 0, "whole 32-wide K steps");
    auto frag = [&](int k0, v4s& Af, v4s& Bf) {
        short av[4], bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // A[c = m0 + row][k] = W[o][c * KV + tap]
            const int ka = k0 + 4 * g + j;
            const int oa = ka / G::KV, ta = ka - oa * G::KV;
            av[j] = (short)W[oa * G::KPAD + (m0 + row) * G::KV + ta];
            // B[k][n] = dZ[b][o][p_out] with p_in = ST p_out - PD + tap on each axis
            const int o = ka / G::KV, t = ka - o * G::KV;
            const int kz = t / (G::K * G::K), ky = (t / G::K) % G::K, kx = t % G::K;
            const int tz = iz + G::PD - kz, ty = iy + G::PD - ky, tx = ix + G::PD - kx;
            const bool ok = tz >= 0 && ty >= 0 && tx >= 0 && tz % G::ST == 0 && ty % G::ST == 0 &&
                            tx % G::ST == 0 && tz / G::ST < G::DO && ty / G::ST < G::DO &&
                            tx / G::ST < G::DO;
            const int idx = ok ? o * G::PO + ((tz / G::ST) * G::DO + ty / G::ST) * G::DO + tx / G::ST : 0;
            const short v = (short)dzb[idx];
            bv[j] = ok ? v : (short)0;
        }
        Af = v4s{av[0], av[1], av[2], av[3]};
        Bf = v4s{bv[0], bv[1], bv[2], bv[3]};
    };
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < KT; k0 += 32) {
        v4s A0, B0, A1, B1;
        frag(k0, A0, B0);
        frag(k0 + 16, A1, B1);
        acc = mfma2(A0, A1, B0, B1, acc);
    }
    const float r[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = m0 + 4 * g + j;
        const int64_t o = (b * G::CI + c) * G::PI + p;
        dZprev[o] = to_bf16(r[j] * dsilu(Zprev[o]));
    }
}

// Backward through the input of a stride-2, 3-tap, pad-1 layer by parity class.  Along an axis,
// input position i = 2a + p receives tap 1 from output a when p = 0, and taps 0 and 2 from
// outputs a + 1 and a when p = 1 (output DO counts as zero).  The 8 classes of positions by
// (z, y, x) parity are then dense GEMMs over their own taps only (2^popcount(class) per
// channel, 1/8 of the 27) instead of over all taps with zeros.  One block per sample: dZ staged
// in LDS with a zero plane past the last output on each axis, and tables of each class's K
// entries (output channel o major, then the taps): their offsets in the staged dZ and in W.
template <class G>
__global__ __launch_bounds__(256) void k_conv_bwd_x_par(const uint16_t* __restrict__ W,
                                                        const uint16_t* __restrict__ dZ,
                                                        const float* __restrict__ Zprev,
                                                        uint16_t* __restrict__ dZprev)
{
    static_assert(G::ST == 2 && G::K == 3 && G::PD == 1 && G::DI == 2 * G::DO,
                  "stride-2, 3-tap, pad-1 layer");
    constexpr int H = G::DO;                  // positions per axis within a class
    constexpr int NPC = H * H * H;            // positions per class
    static_assert(NPC % 16 == 0, "whole column tiles per class");
    constexpr int NCT = NPC / 16;
    constexpr int DQ = G::DO + 1, QQ = DQ * DQ * DQ;
    constexpr int KTOT = CO * 27;             // the classes' K entries together
    __shared__ uint16_t dzs[CO * QQ];
    __shared__ int boff[KTOT];
    __shared__ int aoff[KTOT];
    const int64_t b = blockIdx.x;
    // tables; class c = pz << 2 | py << 1 | px, entry k of class c at kbase(c) + k
    for (int e = threadIdx.x; e < KTOT; e += 256) {
        int c = 0, base = 0;
        while (base + CO * (1 << __popc(c)) <= e) {
            base += CO * (1 << __popc(c));
            ++c;
        }
        const int nc = 1 << __popc(c);
        const int k = e - base, o = k / nc;
        int bits = k % nc, tap = 0, d = 0;
        // axes x, y, z; an odd-parity axis takes one bit of the tap number
        const int wt[3] = {1, G::K, G::K * G::K}, wd[3] = {1, DQ, DQ * DQ};
        for (int ax = 0; ax < 3; ++ax) {
            int kx = 1, dx = 0;
            if ((c >> ax) & 1) {
                const int pick = bits & 1;
                bits >>= 1;
                kx = pick ? 2 : 0;
                dx = pick ? 0 : 1;
            }
            tap += kx * wt[ax];
            d += dx * wd[ax];
        }
        boff[e] = o * QQ + d;
        aoff[e] = o * G::KPAD + tap;
    }
    for (int i = threadIdx.x; i < CO * QQ; i += 256) dzs[i] = 0;
    __syncthreads();
    const uint16_t* dzb = dZ + b * CO * G::PO;
    for (int i = threadIdx.x; i < CO * G::PO; i += 256) {
        const int o = i / G::PO, r = i - o * G::PO;
        const int z = r / (G::DO * G::DO), y = (r / G::DO) % G::DO, x = r % G::DO;
        dzs[o * QQ + (z * DQ + y) * DQ + x] = dzb[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
    for (int tI = threadIdx.x >> 6; tI < 8 * 2 * NCT; tI += 4) {
        const int c = tI / (2 * NCT), rem = tI - c * 2 * NCT;
        const int m0 = 16 * (rem / NCT), ct = rem % NCT;
        int kb = 0;
        for (int d = 0; d < c; ++d) kb += CO * (1 << __popc(d));
        const int kc = CO * (1 << __popc(c));
        const int q = ct * 16 + row;         // this lane's position within the class
        const int az = q / (H * H), ay = (q / H) % H, ax = q % H;
        const int colbase = (az * DQ + ay) * DQ + ax;
        // kc = CO 2^popcount(class) is a multiple of 32
        auto frag = [&](int k0, v4s& Af, v4s& Bf) {
            const int e0 = kb + k0 + 4 * g;
            short av[4], bv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                av[j] = (short)W[aoff[e0 + j] + (m0 + row) * G::KV];
                bv[j] = (short)dzs[colbase + boff[e0 + j]];
            }
            Af = v4s{av[0], av[1], av[2], av[3]};
            Bf = v4s{bv[0], bv[1], bv[2], bv[3]};
        };
        static_assert(CO % 32 == 0, "whole 32-wide K steps per class");
        v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int k0 = 0; k0 < kc; k0 += 32) {
            v4s A0, B0, A1, B1;
            frag(k0, A0, B0);
            frag(k0 + 16, A1, B1);
            acc = mfma2(A0, A1, B0, B1, acc);
        }
        const int iz = 2 * az + ((c >> 2) & 1), iy = 2 * ay + ((c >> 1) & 1), ix = 2 * ax + (c & 1);
        const int pin = (iz * G::DI + iy) * G::DI + ix;
        const float r[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cc = m0 + 4 * g + j;
            const int64_t o = (b * G::CI + cc) * G::PI + pin;
            dZprev[o] = to_bf16(r[j] * dsilu(Zprev[o]));
        }
    }
}

// ---- backward to the weights: split over chunks of 256 columns (sample, output position) ---
// C tile = 16 output channels x 16 (c, tap); partial[chunk][o][k].
template <class G>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const uint16_t* __restrict__ dZ,
                                                    const uint16_t* __restrict__ X, int64_t B,
                                                    float* __restrict__ part)
{
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
    constexpr int NT = G::KPAD / 16;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= 2 * NT) return;
    const int m0 = 16 * (tile / NT), n0 = 16 * (tile % NT);
    const int64_t R = B * G::PO;
    const int64_t r_begin = (int64_t)blockIdx.y * 256;
    const int64_t r_end = r_begin + 256 < R ? r_begin + 256 : R;
    // this lane's B column (c, tap)
    const int kn = n0 + row;
    const int c = kn / G::KV, t = kn - c * G::KV;
    const int kz = t / (G::K * G::K), ky = (t / G::K) % G::K, kx = t % G::K;
    const bool kvalid = kn < G::KREAL;
    auto frag = [&](int64_t r0, v4s& Af, v4s& Bf) {
        short av[4], bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t r = r0 + 4 * g + j;
            const int64_t b = r / G::PO;
            const int p = (int)(r - b * G::PO);
            av[j] = (short)dZ[(b * CO + m0 + row) * G::PO + p];
            const int oz = p / (G::DO * G::DO), oy = (p / G::DO) % G::DO, ox = p % G::DO;
            const int iz = G::ST * oz - G::PD + kz, iy = G::ST * oy - G::PD + ky,
                      ix = G::ST * ox - G::PD + kx;
            const bool ok = kvalid && iz >= 0 && iz < G::DI && iy >= 0 && iy < G::DI && ix >= 0 &&
                            ix < G::DI;
            const int64_t idx = ok ? (b * G::CI + c) * G::PI + (iz * G::DI + iy) * G::DI + ix : 0;
            const short v = (short)X[idx];
            bv[j] = ok ? v : (short)0;
        }
        Af = v4s{av[0], av[1], av[2], av[3]};
        Bf = v4s{bv[0], bv[1], bv[2], bv[3]};
    };
    // the chunk holds a multiple of 16 rows (B is); an odd 16-row block at its end pairs with
    // zeros
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t r0 = r_begin; r0 < r_end; r0 += 32) {
        v4s A0, B0, A1 = v4s{0, 0, 0, 0}, B1 = v4s{0, 0, 0, 0};
        frag(r0, A0, B0);
        if (r0 + 16 < r_end) frag(r0 + 16, A1, B1);
        acc = mfma2(A0, A1, B0, B1, acc);
    }
    float* out = part + (int64_t)blockIdx.y * CO * G::KPAD;
    const float r[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) out[(m0 + 4 * g + j) * G::KPAD + n0 + row] = r[j];
}

// out[e] += sum_c part[c][e]
// out[e] += sum over the nchunk partials part[c][e]: SUM_WAVES wavefronts share the chunks
// (chunk c to wavefront c mod SUM_WAVES), four independent accumulators each so that the loads
// are in flight together; the wavefronts' sums are added in a fixed order.
constexpr int SUM_WAVES = 16;
constexpr int SUM_THREADS = 64 * SUM_WAVES;

__global__ __launch_bounds__(SUM_THREADS) void k_sum_parts_ws(const float* __restrict__ part,
                                                              int64_t nchunk, int64_t n,
                                                              float* __restrict__ out)
{
    __shared__ float sh[SUM_WAVES][64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 64 + l;
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
    if (w != 0 || e >= n) return;
    float t = 0.0f;
#pragma unroll
    for (int i = 0; i < SUM_WAVES; ++i) t += sh[i][l];
    out[e] += t;
}

// Bias gradient partials: part[split][o] = sum over the split's share of the (sample,
// position) pairs of dZ[b][o][p]; grid (CO, BIAS_SPLIT), added in a fixed order afterwards.
constexpr int BIAS_SPLIT = 64;
static_assert(BIAS_SPLIT <= 256, "the bias partials fit the smallest weight-partial buffer");

__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t* __restrict__ dZ, int64_t B,
                                                   int P, float* __restrict__ part)
{
    __shared__ float sh[256];
    const int o = blockIdx.x;
    const int64_t total = B * P;
    const int64_t per = (total + BIAS_SPLIT - 1) / BIAS_SPLIT;
    const int64_t i0 = (int64_t)blockIdx.y * per, i1 = min(i0 + per, total);
    float acc = 0.0f;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const int64_t b = i / P;
        const int p = (int)(i - b * P);
        acc += from_bf16(dZ[(b * CO + o) * P + p]);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * CO + o] = sh[0];
}

// ---- patch gather -------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ws_gather(const WsGatherArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n * 3 * 512) return;
    const int64_t b = i / (3 * 512);
    const int rem = (int)(i - b * 3 * 512);
    const int k = rem / 512, v = rem % 512;
    const int z = v / 64, y = (v / 8) % 8, x = v % 8;
    const float wx = a.means[3 * b] + ((float)x - 3.5f) * a.spacing;
    const float wy = a.means[3 * b + 1] + ((float)y - 3.5f) * a.spacing;
    const float wz = a.means[3 * b + 2] + ((float)z - 3.5f) * a.spacing;
    const GridConst& S = a.s[k];
    const float px = (float)(S.L[0] * wx + S.L[1] * wy + S.L[2] * wz + S.t[0]);
    const float py = (float)(S.L[3] * wx + S.L[4] * wy + S.L[5] * wz + S.t[1]);
    const float pz = (float)(S.L[6] * wx + S.L[7] * wy + S.L[8] * wz + S.t[2]);
    float val = 0.0f;
    if (px >= 0.0f && py >= 0.0f && pz >= 0.0f && px <= (float)(S.nx - 1) &&
        py <= (float)(S.ny - 1) && pz <= (float)(S.nz - 1)) {
        const int x0 = min((int)px, max(S.nx - 2, 0)), y0 = min((int)py, max(S.ny - 2, 0)),
                  z0 = min((int)pz, max(S.nz - 2, 0));
        const int x1 = min(x0 + 1, S.nx - 1), y1 = min(y0 + 1, S.ny - 1), z1 = min(z0 + 1, S.nz - 1);
        const float fx = px - (float)x0, fy = py - (float)y0, fz = pz - (float)z0;
        const float* d = a.data[k];
        auto at = [&](int xx, int yy, int zz) { return d[((size_t)zz * S.ny + yy) * S.nx + xx]; };
        const float c00 = at(x0, y0, z0) * (1.0f - fx) + at(x1, y0, z0) * fx;
        const float c10 = at(x0, y1, z0) * (1.0f - fx) + at(x1, y1, z0) * fx;
        const float c01 = at(x0, y0, z1) * (1.0f - fx) + at(x1, y0, z1) * fx;
        const float c11 = at(x0, y1, z1) * (1.0f - fx) + at(x1, y1, z1) * fx;
        val = ((c00 * (1.0f - fy) + c10 * fy) * (1.0f - fz) + (c01 * (1.0f - fy) + c11 * fy) * fz);
    }
    a.patches[i] = to_bf16(val);
}

// ---- head: linear 32 -> 8, residual assembly, loss and its gradient -------------------------
__device__ void rot_from_q(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__global__ __launch_bounds__(256) void k_ws_head(const WsHeadArgs a)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.n) return;
    float a4[CO];
#pragma unroll
    for (int c = 0; c < CO; ++c) a4[c] = silu(a.z4[b * CO + c]);
    float out[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float s = a.bl[j];
#pragma unroll
        for (int c = 0; c < CO; ++c) s += a.wl[j * CO + c] * a4[c];
        out[j] = s;
    }
    const double s_[3] = {(double)a.s0[3 * b] + out[0], (double)a.s0[3 * b + 1] + out[1],
                          (double)a.s0[3 * b + 2] + out[2]};
    const double q_[4] = {1.0 + out[3], (double)out[4], (double)out[5], (double)out[6]};
    const double lg = (double)a.logit0[b] + out[7];
    if (a.s_out) {
#pragma unroll
        for (int m = 0; m < 3; ++m) a.s_out[3 * b + m] = (float)s_[m];
#pragma unroll
        for (int m = 0; m < 4; ++m) a.q_out[4 * b + m] = (float)q_[m];
        a.logit_out[b] = (float)lg;
    }
    if (!a.sig_t) return;
    // loss: |Sigma - Sigma*|_F^2 / |Sigma*|_F^2 + (logit - logit*)^2, mean over samples
    const double qn = sqrt(q_[0] * q_[0] + q_[1] * q_[1] + q_[2] * q_[2] + q_[3] * q_[3]);
    const double qh[4] = {q_[0] / qn, q_[1] / qn, q_[2] / qn, q_[3] / qn};
    double R[9];
    rot_from_q(qh, R);
    const double S2[3] = {exp(2.0 * s_[0]), exp(2.0 * s_[1]), exp(2.0 * s_[2])};
    const float* st = a.sig_t + 6 * b;  // xx yy zz xy xz yz
    const double T[9] = {st[0], st[3], st[4], st[3], st[1], st[5], st[4], st[5], st[2]};
    double S[9], num = 0.0, den = 0.0;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            S[3 * p + q] = R[3 * p] * S2[0] * R[3 * q] + R[3 * p + 1] * S2[1] * R[3 * q + 1] +
                           R[3 * p + 2] * S2[2] * R[3 * q + 2];
            num += (S[3 * p + q] - T[3 * p + q]) * (S[3 * p + q] - T[3 * p + q]);
            den += T[3 * p + q] * T[3 * p + q];
        }
    const double dlg_ = lg - (double)a.logit_t[b];
    a.loss_each[b] = (float)(num / den + dlg_ * dlg_);
    const double inv = 1.0 / (double)a.n;
    double G[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) G[t] = 2.0 * (S[t] - T[t]) / den * inv;
    // Sigma = R diag(S2) R^T
    double GR[9], RtGR[9];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q)
            GR[3 * p + q] = G[3 * p] * R[q] + G[3 * p + 1] * R[3 + q] + G[3 * p + 2] * R[6 + q];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q)
            RtGR[3 * p + q] = R[p] * GR[q] + R[3 + p] * GR[3 + q] + R[6 + p] * GR[6 + q];
    double g[9];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) g[3 * p + q] = 2.0 * GR[3 * p + q] * S2[q];
    double dout[8];
    dout[0] = 2.0 * S2[0] * RtGR[0];
    dout[1] = 2.0 * S2[1] * RtGR[4];
    dout[2] = 2.0 * S2[2] * RtGR[8];
    const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    double dq[4];
    dq[0] = 2.0 * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
    dq[1] = 2.0 * (y * g[1] + z * g[2] + y * g[3] - 2.0 * x * g[4] - w * g[5] + z * g[6] + w * g[7] -
                   2.0 * x * g[8]);
    dq[2] = 2.0 * (-2.0 * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] + z * g[7] -
                   2.0 * y * g[8]);
    dq[3] = 2.0 * (-2.0 * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2.0 * z * g[4] + y * g[5] +
                   x * g[6] + y * g[7]);
    const double dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
#pragma unroll
    for (int m = 0; m < 4; ++m) dout[3 + m] = (dq[m] - qh[m] * dot) / qn;
    dout[7] = 2.0 * dlg_ * inv;
#pragma unroll
    for (int j = 0; j < 8; ++j) a.dout[8 * b + j] = (float)dout[j];
#pragma unroll
    for (int c = 0; c < CO; ++c) {
        a.a4[b * CO + c] = a4[c];
        float da = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) da += a.wl[j * CO + c] * (float)dout[j];
        a.dz4[b * CO + c] = to_bf16(da * dsilu(a.z4[b * CO + c]));
    }
}

// Training targets: Sigma = R(q/|q|) diag(e^{2 s}) R^T per Gaussian in FP64, stored as
// (xx, yy, zz, xy, xz, yz).
__global__ __launch_bounds__(256) void k_ws_targets(const float* __restrict__ ls,
                                                    const float* __restrict__ quat, int64_t n,
                                                    float* __restrict__ sig6)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double q[4] = {quat[4 * i], quat[4 * i + 1], quat[4 * i + 2], quat[4 * i + 3]};
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double qh[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
    double R[9];
    rot_from_q(qh, R);
    const double S2[3] = {exp(2.0 * (double)ls[3 * i]), exp(2.0 * (double)ls[3 * i + 1]),
                          exp(2.0 * (double)ls[3 * i + 2])};
    auto sig = [&](int p, int r) {
        return R[3 * p] * S2[0] * R[3 * r] + R[3 * p + 1] * S2[1] * R[3 * r + 1] +
               R[3 * p + 2] * S2[2] * R[3 * r + 2];
    };
    float* o = sig6 + 6 * i;
    o[0] = (float)sig(0, 0);
    o[1] = (float)sig(1, 1);
    o[2] = (float)sig(2, 2);
    o[3] = (float)sig(0, 1);
    o[4] = (float)sig(0, 2);
    o[5] = (float)sig(1, 2);
}

// head weight gradients: dWl[j][c] += sum_b dout[b][j] a4[b][c]; dbl[j] += sum_b dout[b][j]
// Head weight/bias gradient partials over HG_SPLIT ranges of samples: part[split][j][c] =
// sum of dout[b][j] a4[b][c], then part[HG_SPLIT * 256 + split * 8 + j] = sum of dout[b][j];
// the ranges are added in a fixed order afterwards.
constexpr int HG_SPLIT = 64;
static_assert(8 * CO == 256, "one thread per head weight");

__global__ __launch_bounds__(256) void k_ws_head_grad(const float* __restrict__ dout,
                                                      const float* __restrict__ a4, int64_t n,
                                                      float* __restrict__ part)
{
    const int t = threadIdx.x;  // 256 = 8 x 32
    const int j = t / CO, c = t % CO;
    const int64_t per = (n + HG_SPLIT - 1) / HG_SPLIT;
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(b0 + per, n);
    float s = 0.0f, sb = 0.0f;
    for (int64_t b = b0; b < b1; ++b) {
        s += dout[8 * b + j] * a4[b * CO + c];
        if (c == 0) sb += dout[8 * b + j];
    }
    part[(int64_t)blockIdx.x * 256 + t] = s;
    if (c == 0) part[(int64_t)HG_SPLIT * 256 + blockIdx.x * 8 + j] = sb;
}

__global__ __launch_bounds__(256) void k_mean(const float* __restrict__ v, int64_t n,
                                              float* __restrict__ out)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += v[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(sh[0] / (double)(n > 0 ? n : 1));
}

template <class G>
void conv_fwd(const uint16_t* W, const float* b, const uint16_t* X, int64_t B, float* Z,
              uint16_t* A, hipStream_t s)
{
    const int64_t ntile = B * G::PO / 16;
    if constexpr (G::PO % 16 == 0 && G::PD > 0) {
        hipLaunchKernelGGL(k_conv_fwd_lds<G>, dim3((unsigned)B), dim3(256), 0, s, W, b, X, Z, A);
        return;
    }
    hipLaunchKernelGGL(k_conv_fwd<G>, dim3((unsigned)((ntile + 3) / 4), 2), dim3(256), 0, s, W, b,
                       X, B, Z, A);
}

template <class G>
void conv_bwd_x(const uint16_t* W, const uint16_t* dZ, int64_t B, const float* Zprev,
                uint16_t* dZprev, hipStream_t s)
{
    if constexpr (G::ST == 2 && G::K == 3 && G::PD == 1 && G::DI == 2 * G::DO &&
                  (G::DO * G::DO * G::DO) % 16 == 0 && G::CI == 32) {
        hipLaunchKernelGGL(k_conv_bwd_x_par<G>, dim3((unsigned)B), dim3(256), 0, s, W, dZ, Zprev,
                           dZprev);
        return;
    }
    const int64_t ntile = B * G::PI / 16;
    hipLaunchKernelGGL(k_conv_bwd_x<G>, dim3((unsigned)((ntile + 3) / 4), 2), dim3(256), 0, s, W,
                       dZ, B, Zprev, dZprev);
}

template <class G>
void conv_bwd_w(const uint16_t* dZ, const uint16_t* X, int64_t B, float* part, float* dW,
                float* db, hipStream_t s)
{
    constexpr int NT = G::KPAD / 16;
    const int64_t R = B * G::PO;
    const int64_t nchunk = (R + 255) / 256;
    hipLaunchKernelGGL(k_conv_bwd_w<G>, dim3((unsigned)((2 * NT + 3) / 4), (unsigned)nchunk),
                       dim3(256), 0, s, dZ, X, B, part);
    const int64_t n = (int64_t)CO * G::KPAD;
    hipLaunchKernelGGL(k_sum_parts_ws, dim3((unsigned)((n + 63) / 64)), dim3(SUM_THREADS), 0, s,
                       part, nchunk, n, dW);
    // the weight partials have been consumed: their buffer takes the bias partials
    hipLaunchKernelGGL(k_bias_grad, dim3(CO, BIAS_SPLIT), dim3(256), 0, s, dZ, B, G::PO, part);
    hipLaunchKernelGGL(k_sum_parts_ws, dim3((CO + 63) / 64), dim3(SUM_THREADS), 0, s, part,
                       (int64_t)BIAS_SPLIT, (int64_t)CO, db);
}

}  // namespace

int ws_kpad(int layer)
{
    switch (layer) {
    case 1: return G1::KPAD;
    case 2: return G2::KPAD;
    case 3: return G3::KPAD;
    default: return G4::KPAD;
    }
}

size_t ws_part_floats(int64_t B)
{
    // largest split-K partial buffer over the four layers
    const int64_t c1 = (B * G1::PO + 255) / 256 * CO * G1::KPAD;
    const int64_t c2 = (B * G2::PO + 255) / 256 * CO * G2::KPAD;
    const int64_t c3 = (B * G3::PO + 255) / 256 * CO * G3::KPAD;
    const int64_t c4 = (B * G4::PO + 255) / 256 * CO * G4::KPAD;
    int64_t m = c1 > c2 ? c1 : c2;
    m = m > c3 ? m : c3;
    m = m > c4 ? m : c4;
    return (size_t)m;
}

hipError_t launch_ws_gather(const WsGatherArgs& a, hipStream_t s)
{
    const int64_t n = a.n * 3 * 512;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ws_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ws_forward(const WsNet& net, const uint16_t* X0, int64_t B, const WsActs& w,
                             const WsHeadArgs& head, hipStream_t s)
{
    conv_fwd<G1>(net.w[0], net.b[0], X0, B, w.z[0], w.a[0], s);
    conv_fwd<G2>(net.w[1], net.b[1], w.a[0], B, w.z[1], w.a[1], s);
    conv_fwd<G3>(net.w[2], net.b[2], w.a[1], B, w.z[2], w.a[2], s);
    conv_fwd<G4>(net.w[3], net.b[3], w.a[2], B, w.z[3], w.a[3], s);
    hipLaunchKernelGGL(k_ws_head, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, head);
    return hipGetLastError();
}

hipError_t launch_ws_backward(const WsNet& net, const uint16_t* X0, int64_t B, const WsActs& w,
                              const WsHeadArgs& head, const WsGrads& g, float* loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, s, head.loss_each, B, loss);
    hipLaunchKernelGGL(k_ws_head_grad, dim3(HG_SPLIT), dim3(256), 0, s, head.dout, head.a4, B,
                       w.part);
    hipLaunchKernelGGL(k_sum_parts_ws, dim3(4), dim3(SUM_THREADS), 0, s, w.part,
                       (int64_t)HG_SPLIT, (int64_t)256, g.wl);
    hipLaunchKernelGGL(k_sum_parts_ws, dim3(1), dim3(SUM_THREADS), 0, s,
                       w.part + (int64_t)HG_SPLIT * 256, (int64_t)HG_SPLIT, (int64_t)8, g.bl);
    // layer 4 (dZ4 written by the head)
    conv_bwd_w<G4>(w.dz[3], w.a[2], B, w.part, g.w[3], g.b[3], s);
    conv_bwd_x<G4>(net.w[3], w.dz[3], B, w.z[2], w.dz[2], s);
    conv_bwd_w<G3>(w.dz[2], w.a[1], B, w.part, g.w[2], g.b[2], s);
    conv_bwd_x<G3>(net.w[2], w.dz[2], B, w.z[1], w.dz[1], s);
    conv_bwd_w<G2>(w.dz[1], w.a[0], B, w.part, g.w[1], g.b[1], s);
    conv_bwd_x<G2>(net.w[1], w.dz[1], B, w.z[0], w.dz[0], s);
    conv_bwd_w<G1>(w.dz[0], X0, B, w.part, g.w[0], g.b[0], s);
    return hipGetLastError();
}

hipError_t launch_ws_targets(const float* ls, const float* quat, int64_t n, float* sig6,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ws_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ls,
                       quat, n, sig6);
    return hipGetLastError();
}
