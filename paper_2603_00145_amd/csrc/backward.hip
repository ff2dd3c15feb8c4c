// K7 + K8: gradients of L = sum_k sum_v dL/dI_k[v] I_k[v] (+ lambda_aniso * L_aniso,
// Eq. 12-13) with respect to every Gaussian parameter, boxes held fixed.
//
// K7 (grid-frame partials): eight lanes per Gaussian gather g = dL/dI over the voxels of the
// Gaussian's box on each listed grid, recomputing E = 2^Q (no per-voxel contributions are
// stored).  With delta = v - c, Q = delta^T K delta (K the record's base-2 conic as a
// symmetric matrix) and w = amp E, the ten grid-frame partials are
//     d amp = sum g E,   d c = -2 amp ln2 K m,   d K_ab = amp ln2 m_ab
// with the weighted moments m = sum g E delta and m_ab = sum g E delta_a delta_b.  A lane
// owns one (x, z) column of the box at a time and walks it along y, summing g E, g E dy and
// g E dy^2; the column's share of the ten moments follows from those three sums and its
// (dx, dz).  The moments are reduced across the eight lanes with DPP and turned into the
// partials once per (grid, Gaussian).  No global atomics are needed.  With the paper's block
// query on a rotated grid (k_partials<true>) every Gaussian of that grid takes the global-memory
// path and each voxel of its box is also tested against its cell block (Eqs. 4-6): the sums
// run over the voxels that pass.
//
// K8 (chain rule, FP64): thread per Gaussian.  The partials of every grid are pulled back
// through c = L mu + t, C = Sigma_g^-1, amp = alpha sqrt(det Sigma_idx / det Sigma_g),
// Sigma_idx = L Sigma L^T, Sigma = R diag(e^{2s}) R^T (Eq. 3), R(q/|q|) and
// alpha = sigmoid(logit), summed over grids, and added (+=) to the gradient buffers.
#include "gm_internal.h"

namespace {

__device__ __forceinline__ int sgpr(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum of v over each aligned group of G lanes (G = 8 or 16; every lane of the group ends with
// it): DPP adds across lane xor 1, xor 2, the half-row mirror and, for 16, the row mirror.
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    static_assert(G == 8 || G == 16, "groups of 8 or 16 lanes");
    int xi;
    xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false);  // xor 1
    v += __int_as_float(xi);
    xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false);  // xor 2
    v += __int_as_float(xi);
    xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false); // half mirror
    v += __int_as_float(xi);
    if (G == 16) {
        xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false); // mirror
        v += __int_as_float(xi);
    }
    return v;
}

// Largest / smallest value of v over the lanes 0, G, 2G, ... (one per group).
template <int G>
__device__ __forceinline__ int group_max(int v)
{
    int m = __builtin_amdgcn_readlane(v, 0);
#pragma unroll
    for (int r = 1; r < 64 / G; ++r) m = max(m, __builtin_amdgcn_readlane(v, r * G));
    return m;
}
template <int G>
__device__ __forceinline__ int group_min(int v)
{
    int m = __builtin_amdgcn_readlane(v, 0);
#pragma unroll
    for (int r = 1; r < 64 / G; ++r) m = min(m, __builtin_amdgcn_readlane(v, r * G));
    return m;
}

// dL/dI region a block stages in LDS: its tile plus a halo of 8 voxels on the upper side in x
// and y and 6 in z (a home Gaussian's box starts inside the tile; thick-slice boxes are short
// in z).  The z planes are RZS floats apart, RZS = 8 (mod 32), so the up-to-four z rows a lane
// row reads at one step sit in different LDS banks.
constexpr int RX = GM_TX + 8, RY = GM_TY + 8, RZ = GM_TZ + 6;
constexpr int RZS = RX * RY + 8;
constexpr int BWD_G = 8;   // lanes per Gaussian in the backward
constexpr int WINB = 1024; // list entries a block sorts at a time
constexpr int EPT = WINB / 256;  // ... per thread
// sort keys of home entries: boxes inside the staged region by (column chunks, y length), both
// capped, 8 x 16 keys; then one key for boxes reaching past the region
constexpr int NKEY = 8 * 16 + 1;
static_assert(RZS % 32 == 8, "z-plane stride must be 8 mod 32 banks");

// Column sums s0 = sum ge, s1 = sum k ge, s2 = sum k^2 ge (ge = g 2^Q_k) over the first NK
// rows of a column whose rows are RX floats apart in the staged region.  Rows 0..7 of a home
// box lie inside the region (the box starts in the tile, the region reaches 8 rows past it),
// so all NK reads are issued at immediate offsets before the first use; rows past the column
// (k >= ncol) are masked where they are used.  NK is the wavefront's longest column (up to 8),
// a compile-time constant, so the steps carry no branches.
template <int NK, bool MASK>
__device__ __forceinline__ void lds_column(const float* __restrict__ region, uint32_t off,
                                           int ncol, float A, float B, float kyy, float& s0,
                                           float& s1, float& s2)
{
    float gv[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) gv[k] = region[off + k * RX];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const float Q = k == 0 ? A : fmaf((float)k, fmaf((float)k, kyy, B), A);
        // without MASK every active column of the wavefront is at least NK long
        const float gk = (k == 0 || !MASK) ? gv[k] : (k < ncol ? gv[k] : 0.0f);
        const float ge = gk * __builtin_amdgcn_exp2f(Q);
        s0 += ge;
        if (k > 0) {
            s1 = fmaf((float)k, ge, s1);
            s2 = fmaf((float)(k * k), ge, s2);
        }
    }
}

// 64/G Gaussians of one grid at a time, one per group of G lanes: the ten moments of each,
// turned into the grid-frame partials and stored.  A group maps its lanes onto chunks of G
// (x, z) columns of its Gaussian's box and walks each column along y (for thick-slice stacks the box
// is longest in-plane, so this gives the fewest chunks and the longest walks).  With FROM_LDS
// every box lies inside the block's staged region and dL/dI is read from LDS; otherwise from
// global memory.  All of a column's values are read first; step k then costs
// Q_k = A + k (B + k kyy) (two FMAs), one exp2, one multiply and three adds for the column sums
// of g E, k g E and k^2 g E (k a compile-time constant in the unrolled loop).  Past a shorter
// box, a row's reads are clamped and zeroed.
// A Gaussian's 64-byte render record on one grid, as the group loads it (zeros when invalid).
struct Rec {
    float4 r0, r1, r2, r3;
};

// (an invalid lane group passes mine = 0 and gets Gaussian 0's record: finite values whose
// box group_of_gaussians never walks)
__device__ __forceinline__ Rec load_record(const BackwardArgs& a, int gi, uint32_t mine)
{
    const int64_t gid = min((int64_t)(mine & GM_ID_MASK), a.n - 1);
    const float4* rp = reinterpret_cast<const float4*>(a.records + ((size_t)gi * a.n + gid) * 16);
    Rec r;
    r.r0 = rp[0];
    r.r1 = rp[1];
    r.r2 = rp[2];
    r.r3 = rp[3];
    return r;
}

template <int G, bool FROM_LDS, bool MASK = false>
__device__ __forceinline__ void group_of_gaussians(const BackwardArgs& a, int kk, uint32_t mine,
                                                   bool gvalid, const Rec& rec,
                                                   const float* __restrict__ region,
                                                   int t0x, int t0y, int t0z, bool mk = false)
{
    static_assert(!(MASK && FROM_LDS), "masked grids read dL/dI from global memory");
    const int ql = threadIdx.x & (G - 1);
    const int gi = a.grid_index[kk];
    const int nx = a.nx[kk], ny = a.ny[kk];
    const float* __restrict__ g = a.dl_di[kk];
    const int64_t gid = min((int64_t)(mine & GM_ID_MASK), a.n - 1);
    const float4 r0 = rec.r0, r1 = rec.r1, r2 = rec.r2, r3 = rec.r3;
    // masked grid: the Gaussian's cell and the grid's index -> world affine
    const int4 cm = (MASK && mk) ? a.bq.cells[gid] : make_int4(0, 0, 0, 0);
    const double* mw = a.m[kk];
    const int lox = __float_as_int(r2.z), loy = __float_as_int(r2.w), loz = __float_as_int(r3.x);
    const int hix = __float_as_int(r3.y), hiy = __float_as_int(r3.z), hiz = __float_as_int(r3.w);
    // a listed Gaussian's box is never empty; an invalid lane group (past the round's end)
    // holds a finite record (Gaussian 0's) and takes no steps: its box counts as empty
    const bool nonempty = gvalid && lox <= hix && loy <= hiy && loz <= hiz;
    const int wx = nonempty ? hix - lox + 1 : 1;
    const int wy = nonempty ? hiy - loy + 1 : 0;
    const int wz = nonempty ? hiz - loz + 1 : 0;
    const float cx = r0.x, cy = r0.y, cz = r0.z;
    const float kxx = r1.x, kyy = r1.y, kzz = r1.z, kxy = r1.w;
    const float kxz = r2.x, kyz = r2.y;
    const int fp = wx * wz;                       // (x, z) footprint of the box
    const int chunks = (fp + G - 1) / G;
    const int max_chunks = group_max<G>(chunks);
    const int max_wy = group_max<G>(wy);
    // y steps every active column of the wavefront takes (no mask needed below it)
    const int min_wy = group_min<G>(nonempty ? wy : 64);
    // column f -> (x, z) = (f mod wx, f div wx), with fh = f + 1/2: z = floor(fh / wx) (the
    // fraction stays at least 1/(2 wx) away from an integer, far beyond the hardware
    // reciprocal's error for any f < 2^20) and x + 1/2 = fh - z wx, exact in float
    const float wxf = (float)wx;
    const float inv_wx = __builtin_amdgcn_rcpf(wxf);
    const float dy0 = -cy;                        // dy = dy0 + k at step k of a column
    const float B0 = 2.0f * kyy * dy0;
    // Q along a column at (dx, dz): A = qxz + dy0 (kxy dx + kyz dz + kyy dy0) regrouped as
    // dx (kxx dx + kxz dz + dy0 kxy) + dz (kzz dz + dy0 kyz) + kyy dy0^2
    const float g1 = dy0 * kxy, g2 = dy0 * kyz, A0 = kyy * dy0 * dy0;
    const float cxh = cx + 0.5f;
    // staged-region index of the box's voxel (x, 0, z) minus 1/2, as a float: zf RZS + (x + 1/2)
    // + obase, exact (the region holds fewer than 2^13 floats); in the grid, integer arithmetic
    const int ystride = FROM_LDS ? RX : nx;       // between consecutive y steps
    const float obase = (float)((loz - t0z) * RZS + (loy - t0y) * RX + (lox - t0x)) - 0.5f;
    const float qlh = (float)ql + 0.5f;
    // weighted moments: m0 = sum gE, m1 = sum gE delta, m2 = sum gE delta delta^T
    float m0 = 0.0f, mx = 0.0f, mz = 0.0f, mxx = 0.0f, mzz = 0.0f, mxz = 0.0f;
    // ... and in the column step index k: k1 = sum k gE, k2 = sum k^2 gE, k1x = sum k gE dx,
    // k1z = sum k gE dz
    float k1 = 0.0f, k2 = 0.0f, k1x = 0.0f, k1z = 0.0f;
#pragma unroll 1
    for (int c = 0; c < max_chunks; ++c) {
        const float fh = fmaf((float)c, (float)G, qlh);
        const bool act = fh < (float)fp;
        const float zf = floorf(fh * inv_wx);
        const float xh = fmaf(-zf, wxf, fh);
        const float dx = xh - cxh, dz = zf - cz;
        // Q along the column: Q_k = A + k (B + k kyy).  A lane outside the footprint reads
        // the first voxel of the region (or grid) at every step and gets A = -inf, so its
        // every term is exactly zero.
        const float Aq = fmaf(dx, fmaf(kxx, dx, fmaf(kxz, dz, g1)), fmaf(dz, fmaf(kzz, dz, g2), A0));
        const float A = act ? Aq : -__builtin_inff();
        const float B = fmaf(kxy, dx, fmaf(kyz, dz, B0));
        // the global-memory path's centred form: Q = qxz + dy (by + kyy dy)
        const float by = fmaf(kxy, dx, kyz * dz);
        const float qxz = act ? fmaf(dx, fmaf(kxx, dx, kxz * dz), kzz * dz * dz)
                              : -__builtin_inff();
        uint32_t off = 0u;
        if (act) {
            off = FROM_LDS ? (uint32_t)fmaf(zf, (float)RZS, xh + obase)
                           : (uint32_t)(((loz + (int)zf) * ny + loy) * nx + (lox + (int)xh));
        }
        const int ncol = act ? wy : 1;             // steps whose voxel lies in the box
        // s0 = sum ge, s1 = sum k ge, s2 = sum k^2 ge over the column (ge = g 2^Q)
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
        if (FROM_LDS) {
            const int nk = max_wy < 8 ? max_wy : 8;
            if (min_wy >= nk) {
                switch (nk) {
                case 1: lds_column<1, false>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 2: lds_column<2, false>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 3: lds_column<3, false>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 4: lds_column<4, false>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 5: lds_column<5, false>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 6: lds_column<6, false>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 7: lds_column<7, false>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                default: lds_column<8, false>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                }
            } else {
                switch (nk) {
                case 1: lds_column<1, true>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 2: lds_column<2, true>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 3: lds_column<3, true>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 4: lds_column<4, true>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 5: lds_column<5, true>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 6: lds_column<6, true>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                case 7: lds_column<7, true>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                default: lds_column<8, true>(region, off, ncol, A, B, kyy, s0, s1, s2); break;
                }
            }
        } else {
            // masked grid: the column's voxel (vx, loy + k, vz)
            const int vx = lox + (int)xh, vz = loz + (int)zf;
            float gv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (k < max_wy) {
                    if (k < min_wy) {
                        gv[k] = (g + (size_t)k * nx)[off];
                    } else {
                        const int kc = min(k, ncol - 1);
                        const float t = (g + (size_t)kc * nx)[off];
                        gv[k] = k < ncol ? t : 0.0f;
                    }
                }
            }
            if (MASK && mk) {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (k < max_wy &&
                        !voxel_in_block(mw, a.bq.res, a.bq.radius, vx, loy + k, vz, cm))
                        gv[k] = 0.0f;
            }
            // centred in y: Q = qxz + dy (by + kyy dy) with dy = dy0 + k, and the column sums
            // in dy itself (s1 = sum dy gE, s2 = sum dy^2 gE), so that a box much wider than
            // its Gaussian (the block query) adds no large terms that cancel
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (k < max_wy) {
                    const float dy = dy0 + (float)k;
                    const float Q = fmaf(dy, fmaf(kyy, dy, by), qxz);
                    const float ge = gv[k] * __builtin_amdgcn_exp2f(Q);
                    s0 += ge;
                    s1 = fmaf(dy, ge, s1);
                    s2 = fmaf(dy * dy, ge, s2);
                }
            }
        }
#pragma unroll 1
        for (int k = 8; k < max_wy; ++k) {  // boxes longer than 8 voxels in y
            const int kc = min(k, ncol - 1);
            const float t = FROM_LDS ? region[off + kc * RX] : g[(size_t)kc * ystride + off];
            float gk = k < ncol ? t : 0.0f;
            if (MASK && mk &&
                !voxel_in_block(mw, a.bq.res, a.bq.radius, lox + (int)xh, loy + k, loz + (int)zf,
                                cm))
                gk = 0.0f;
            const float fk = (float)k;
            if (FROM_LDS) {
                const float ge = gk * __builtin_amdgcn_exp2f(A + fk * (B + fk * kyy));
                s0 += ge;
                s1 += fk * ge;
                s2 += fk * fk * ge;
            } else {
                const float dy = dy0 + fk;
                const float ge = gk * __builtin_amdgcn_exp2f(fmaf(dy, fmaf(kyy, dy, by), qxz));
                s0 += ge;
                s1 = fmaf(dy, ge, s1);
                s2 = fmaf(dy * dy, ge, s2);
            }
        }
        // the column's share in the step index k (moments in dy = dy0 + k follow below)
        const float ax = s0 * dx, az = s0 * dz;
        m0 += s0;
        mx += ax;
        mz += az;
        mxx = fmaf(ax, dx, mxx);
        mzz = fmaf(az, dz, mzz);
        mxz = fmaf(ax, dz, mxz);
        k1 += s1;
        k2 += s2;
        k1x = fmaf(s1, dx, k1x);
        k1z = fmaf(s1, dz, k1z);
    }
    // from sums over the step index k to moments in dy = dy0 + k (dy0 is the Gaussian's):
    // sum (dy0 + k) gE = k1 + dy0 m0, sum (dy0 + k)^2 gE = k2 + dy0 (2 k1 + dy0 m0), and
    // the products with dx and dz likewise
    // (the global-memory path summed in dy already: k1, k2, k1x, k1z are the moments)
    float my = FROM_LDS ? fmaf(dy0, m0, k1) : k1;
    float myy = FROM_LDS ? fmaf(dy0, fmaf(2.0f, k1, dy0 * m0), k2) : k2;
    float mxy = FROM_LDS ? fmaf(dy0, mx, k1x) : k1x;
    float myz = FROM_LDS ? fmaf(dy0, mz, k1z) : k1z;
    m0 = group_sum<G>(m0);
    mx = group_sum<G>(mx);
    my = group_sum<G>(my);
    mz = group_sum<G>(mz);
    mxx = group_sum<G>(mxx);
    myy = group_sum<G>(myy);
    mzz = group_sum<G>(mzz);
    mxy = group_sum<G>(mxy);
    mxz = group_sum<G>(mxz);
    myz = group_sum<G>(myz);
    if (ql == 0 && gvalid) {
        // K as a full symmetric matrix has off-diagonal entries kxy/2, kxz/2, kyz/2
        const float Al = r0.w * GM_LN2F;   // amp ln2
        const float hxy = 0.5f * kxy, hxz = 0.5f * kxz, hyz = 0.5f * kyz;
        const float tx = kxx * mx + hxy * my + hxz * mz;
        const float ty = hxy * mx + kyy * my + hyz * mz;
        const float tz = hxz * mx + hyz * my + kzz * mz;
        float2* o = reinterpret_cast<float2*>(a.grid_grads + ((size_t)gi * a.n + gid) * 10);
        o[0] = make_float2(m0, -2.0f * Al * tx);
        o[1] = make_float2(-2.0f * Al * ty, -2.0f * Al * tz);
        o[2] = make_float2(Al * mxx, Al * myy);
        o[3] = make_float2(Al * mzz, Al * mxy);
        o[4] = make_float2(Al * mxz, Al * myz);
    }
}

// Exclusive prefix sums of hist[0..NKEY) in place and the total in hist[NKEY], by one
// wavefront (three keys per lane).
__device__ __forceinline__ void scan_keys(int* hist, int lane)
{
    static_assert(NKEY <= 3 * 64, "three keys per lane");
    int c[3], sum = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int k = 3 * lane + i;
        c[i] = k < NKEY ? hist[k] : 0;
        sum += c[i];
    }
    int incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    int off = incl - sum;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int k = 3 * lane + i;
        if (k < NKEY) hist[k] = off;
        off += c[i];
    }
    if (lane == 63) hist[NKEY] = incl;
}

// One block (four wavefronts) per tile of a listed grid.  The block stages the tile's dL/dI
// region in LDS (coalesced rows), then sorts the home Gaussians of the tile's list (the tile
// holding the box's lower corner: every Gaussian of the grid exactly once), WINB list entries
// at a time, by the loop trips of their boxes: a counting sort over (column chunks, y length)
// with LDS atomics.  The sorted Gaussians are taken eight at a time (a round), rounds dealt to
// the wavefronts in turn, so that the eight Gaussians of a wavefront have similar loop trips
// and the wavefronts of the block similar work.  Each Gaussian is read from LDS when its box
// lies inside the region (the common case) and from global memory otherwise.  A Gaussian's
// partials come from its own eight lanes only and do not depend on which others share its
// round, so the order the atomics give within a key does not change any result bit.
// Gaussians with an empty box are in no list; gm_bin wrote their zeros.
template <bool MASK>
__global__ __launch_bounds__(256) void k_partials(const BackwardArgs a)
{
    __shared__ float region[RZ * RZS];
    __shared__ uint32_t order[WINB];
    __shared__ int hist[NKEY + 1];
    __shared__ int zext;
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    int kk = 0;                                            // listed grid of this block
#pragma unroll 1
    while (kk + 1 < a.n_ids && lin >= a.block_start[kk + 1]) ++kk;
    const int t = lin - a.block_start[kk];
    const int ntx = a.ntx[kk], nty = a.nty[kk];
    const int t0x = (t % ntx) * GM_TX, t0y = ((t / ntx) % nty) * GM_TY, t0z = (t / (ntx * nty)) * GM_TZ;
    const int64_t T = a.tile_base[kk] + t;
    const int e0 = __builtin_amdgcn_readfirstlane(a.tile_start[T]);
    const int e1 = __builtin_amdgcn_readfirstlane(a.tile_start[T + 1]);
    if (e0 == e1) return;  // block-uniform
    const int nx = a.nx[kk], ny = a.ny[kk], nz = a.nz[kk];
    const float* __restrict__ g = a.dl_di[kk];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int gi = a.grid_index[kk];
    const bool mk = MASK && a.masked[kk];   // block query on a rotated grid

    // list entry -> its sort key (-1: not a home entry) and the z planes its box reaches in
    // the region (0 when it reaches past the region; always on a masked grid, whose voxels
    // are tested in the global-memory path)
    auto classify = [&](int entry, uint32_t& v, int& zreach) -> int {
        zreach = 0;
        v = entry < e1 ? a.pair_gauss[entry] : 0u;
        if (entry >= e1 || !(v & GM_HOME_BIT)) return -1;
        if (mk) return NKEY - 1;
        const int4* rc = reinterpret_cast<const int4*>(
            a.records + ((size_t)gi * a.n + min((int64_t)(v & GM_ID_MASK), a.n - 1)) * 16);
        const int4 r2 = rc[2], r3 = rc[3];     // (kxz, kyz, lox, loy), (loz, hix, hiy, hiz)
        const int lx = r2.z, ly = r2.w, lz = r3.x, hx = r3.y, hy = r3.z, hz = r3.w;
        if (!(hx - t0x < RX && hy - t0y < RY && hz - t0z < RZ)) return NKEY - 1;
        if (a.block_query) {
            // a box much wider in y than its Gaussian (|kyy| wy^2 > 64; a 3-sigma box stays
            // below about 50) takes the global-memory path, whose walk is centred
            const float kyy = __int_as_float(rc[1].y);
            const float wyf = (float)(hy - ly + 1);
            if (fabsf(kyy) * wyf * wyf > 64.0f) return NKEY - 1;
        }
        zreach = hz - t0z + 1;
        const int chunks = ((hx - lx + 1) * (hz - lz + 1) + BWD_G - 1) / BWD_G;
        return (min(chunks, 8) - 1) * 16 + (min(hy - ly + 1, 16) - 1);
    };
    uint32_t v[EPT];
    int key[EPT], rank[EPT];
    // counts the keys of entries [w0, w0 + WINB) into hist (zeroed before); a thread's rank
    // within its key is the count the atomic returns
    auto count_keys = [&](int w0, int& zmax) {
#pragma unroll
        for (int h = 0; h < EPT; ++h) {
            int zr;
            key[h] = classify(w0 + h * 256 + tid, v[h], zr);
            zmax = max(zmax, zr);
            rank[h] = key[h] >= 0 ? atomicAdd(&hist[key[h]], 1) : 0;
        }
    };
    auto scatter = [&]() {
#pragma unroll
        for (int h = 0; h < EPT; ++h)
            if (key[h] >= 0) order[hist[key[h]] + rank[h]] = v[h];
    };
    // the rounds of one sorted window: n_lds Gaussians from LDS, then the rest from global
    // memory; round r (order entries 8 r .. 8 r + 7) goes to wavefront r mod 4, and the next
    // round's records are in flight while a round is processed
    constexpr int PER_ROUND = 64 / BWD_G;
    const int grp = lane / BWD_G;
    auto rounds = [&](int n_lds, int n_all) {
        const int nr = (n_lds + PER_ROUND - 1) / PER_ROUND;
        // two record buffers used in turn (no copy between rounds)
        uint32_t ma = 0u, mb = 0u;
        bool va = false, vb = false;
        Rec ra, rb;
        auto fetch = [&](int r, Rec& rec, uint32_t& m, bool& v) {
            const int ix = r * PER_ROUND + grp;
            v = ix < n_lds;
            m = v ? order[ix] : 0u;
            rec = load_record(a, gi, m);
        };
        if (wv < nr) fetch(wv, ra, ma, va);
#pragma unroll 1
        for (int r = wv; r < nr; r += 8) {
            if (r + 4 < nr) fetch(r + 4, rb, mb, vb);
            group_of_gaussians<BWD_G, true>(a, kk, ma, va, ra, region, t0x, t0y, t0z);
            if (r + 4 >= nr) break;
            if (r + 8 < nr) fetch(r + 8, ra, ma, va);
            group_of_gaussians<BWD_G, true>(a, kk, mb, vb, rb, region, t0x, t0y, t0z);
        }
        const int ng = (n_all - n_lds + PER_ROUND - 1) / PER_ROUND;
#pragma unroll 1
        for (int r = wv; r < ng; r += 4) {
            const int ix = n_lds + r * PER_ROUND + grp;
            const bool valid = ix < n_all;
            const uint32_t mine = valid ? order[ix] : 0u;
            const Rec rec = load_record(a, gi, mine);
            group_of_gaussians<BWD_G, false, MASK>(a, kk, mine, valid, rec, region, t0x, t0y,
                                                   t0z, mk);
        }
    };

    // first window: keys counted while the z planes the home boxes reach (those that fit
    // the region) are found over the whole list; only those planes are staged
    if (tid == 0) zext = 0;
    for (int i = tid; i < NKEY; i += 256) hist[i] = 0;
    __syncthreads();
    int zmax = 0;
    count_keys(e0, zmax);
    for (int i = e0 + WINB + tid; i < e1; i += 256) {
        uint32_t vi;
        int zr;
        classify(i, vi, zr);
        zmax = max(zmax, zr);
    }
    if (zmax > 0) atomicMax(&zext, zmax);
    __syncthreads();
    if (wv == 0) scan_keys(hist, lane);
    const int nzr = min(zext, nz - t0z);
    // rows of RX voxels along x: thread -> (x, y) of a plane, then the planes
    for (int i = tid; i < RX * RY; i += 256) {
        const int y = i / RX, x = i - y * RX;
        const int gx = t0x + x, gy = t0y + y;
        const bool in = gx < nx && gy < ny;
        const float* src = g + ((size_t)t0z * ny + gy) * nx + gx;
        float* dst = region + y * RX + x;
        for (int z = 0; z < nzr; ++z) {
            dst[z * RZS] = in ? src[0] : 0.0f;
            src += (size_t)nx * ny;
        }
    }
    __syncthreads();
    scatter();
    __syncthreads();
    rounds(hist[NKEY - 1], hist[NKEY]);
    // further windows (lists longer than WINB entries)
#pragma unroll 1
    for (int w0 = e0 + WINB; w0 < e1; w0 += WINB) {
        __syncthreads();                       // order and hist are free again
        for (int i = tid; i < NKEY; i += 256) hist[i] = 0;
        __syncthreads();
        int zr = 0;
        count_keys(w0, zr);
        __syncthreads();
        if (wv == 0) scan_keys(hist, lane);
        __syncthreads();
        scatter();
        __syncthreads();
        rounds(hist[NKEY - 1], hist[NKEY]);
    }
}

// symmetric 3x3 stored full, row-major
__device__ __forceinline__ void mm3(const double* A, const double* B, double* C)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

__device__ __forceinline__ double inv3(const double* A, double* Ai)
{
    const double c00 = A[4] * A[8] - A[5] * A[7];
    const double c01 = A[5] * A[6] - A[3] * A[8];
    const double c02 = A[3] * A[7] - A[4] * A[6];
    const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    const double id = 1.0 / det;
    Ai[0] = c00 * id;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    Ai[3] = c01 * id;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    Ai[6] = c02 * id;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return det;
}

// One Gaussian on one grid: from its grid-frame partials pg (d amp, d c, d K) and its world
// covariance Sig, the derivative Gi = dL/dSigma_idx (C = Sigma_g^-1 gives dL/dSigma_g =
// -C G_C C; amp = alpha sqrt(det Sigma_idx / det Sigma_g) adds -1/2 d_amp amp C and
// +1/2 d_amp amp Sigma_idx^-1), the centre partial dc, and amp.
__device__ __forceinline__ double sigma_idx_grad(const GridConst& G, const double* Sig,
                                                 double alpha, const float* pg, double* dc,
                                                 double* Gi)
{
    const double damp = pg[0];
    dc[0] = pg[1];
    dc[1] = pg[2];
    dc[2] = pg[3];
    // full-matrix dL/dC from the base-2 conic partials: C-entry = K-entry * KAPPA
    const double GC[9] = {GM_KAPPA * pg[4], GM_KAPPA * pg[7], GM_KAPPA * pg[8],
                          GM_KAPPA * pg[7], GM_KAPPA * pg[5], GM_KAPPA * pg[9],
                          GM_KAPPA * pg[8], GM_KAPPA * pg[9], GM_KAPPA * pg[6]};
    const double* L = G.L;
    double T[9], SI[9];
    mm3(L, Sig, T);
    const double Lt[9] = {L[0], L[3], L[6], L[1], L[4], L[7], L[2], L[5], L[8]};
    mm3(T, Lt, SI);  // Sigma_idx
    double SG[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) SG[t] = SI[t];
    SG[8] += G.sig * G.sig;
    double C[9], SIi[9];
    const double detG = inv3(SG, C);
    const double detI = inv3(SI, SIi);
    const double amp = alpha * sqrt(detI / detG);
    double CG[9], CGC[9];
    mm3(C, GC, CG);
    mm3(CG, C, CGC);
    const double ha = 0.5 * damp * amp;
#pragma unroll
    for (int t = 0; t < 9; ++t) Gi[t] = -CGC[t] - ha * C[t] + ha * SIi[t];
    return amp;
}

// Normalised quaternion (w, x, y, z), its rotation R (Hamilton) and Sigma = R diag(S2) R^T.
__device__ __forceinline__ void world_covariance(const float* quat, const float* log_scale,
                                                 int64_t i, double* qh, double* qn, double* R,
                                                 double* S2, double* Sig)
{
    const double qw = quat[4 * i], qx = quat[4 * i + 1], qy = quat[4 * i + 2],
                 qz = quat[4 * i + 3];
    *qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const double w = qw / *qn, x = qx / *qn, y = qy / *qn, z = qz / *qn;
    qh[0] = w;
    qh[1] = x;
    qh[2] = y;
    qh[3] = z;
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
#pragma unroll
    for (int m = 0; m < 3; ++m) S2[m] = exp(2.0 * (double)log_scale[3 * i + m]);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q)
            Sig[3 * p + q] = R[3 * p] * S2[0] * R[3 * q] + R[3 * p + 1] * S2[1] * R[3 * q + 1] +
                             R[3 * p + 2] * S2[2] * R[3 * q + 2];
}

// three waves per SIMD (at most 168 VGPRs): a few registers more drop it to two, 25% slower
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3))) void k_chain(const ChainArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    double qh[4], qn, R[9], S2[3], Sig[9];
    world_covariance(a.quat, a.log_scale, i, qh, &qn, R, S2, Sig);
    const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    const double ls[3] = {a.log_scale[3 * i], a.log_scale[3 * i + 1], a.log_scale[3 * i + 2]};
    const double alpha = 1.0 / (1.0 + exp(-(double)a.logit[i]));

    double dmu[3] = {0, 0, 0}, GS[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dalpha = 0.0;
#pragma unroll 1
    for (int k = 0; k < a.n_ids; ++k) {
        const GridConst& G = a.g[k];
        const int gi = a.grid_index[k];
        const float* pg = a.grid_grads + ((size_t)gi * a.n + i) * 10;
        if (a.tile_count[(size_t)gi * a.n + i] == 0) continue;  // empty box
        double dc[3], Gi[9];
        const double amp = sigma_idx_grad(G, Sig, alpha, pg, dc, Gi);
        const double* L = G.L;
        // mu
#pragma unroll
        for (int m = 0; m < 3; ++m) dmu[m] += L[m] * dc[0] + L[3 + m] * dc[1] + L[6 + m] * dc[2];
        // Sigma = L^T Gi L
        const double Lt[9] = {L[0], L[3], L[6], L[1], L[4], L[7], L[2], L[5], L[8]};
        double U[9], V9[9];
        mm3(Lt, Gi, U);
        mm3(U, L, V9);
#pragma unroll
        for (int t = 0; t < 9; ++t) GS[t] += V9[t];
        dalpha += (double)pg[0] * amp / alpha;
    }
    // Sigma = R diag(S2) R^T
    double GR[9], RtGR[9], GRR[9];
    mm3(GS, R, GR);  // G R
    double Rt[9] = {R[0], R[3], R[6], R[1], R[4], R[7], R[2], R[5], R[8]};
    mm3(Rt, GR, RtGR);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) GRR[3 * p + q] = 2.0 * GR[3 * p + q] * S2[q];  // dL/dR
    double ds[3] = {2.0 * S2[0] * RtGR[0], 2.0 * S2[1] * RtGR[4], 2.0 * S2[2] * RtGR[8]};
    const double* g = GRR;
    double dq[4];
    dq[0] = 2.0 * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
    dq[1] = 2.0 * (y * g[1] + z * g[2] + y * g[3] - 2.0 * x * g[4] - w * g[5] + z * g[6] +
                   w * g[7] - 2.0 * x * g[8]);
    dq[2] = 2.0 * (-2.0 * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] +
                   z * g[7] - 2.0 * y * g[8]);
    dq[3] = 2.0 * (-2.0 * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2.0 * z * g[4] + y * g[5] +
                   x * g[6] + y * g[7]);
    const double dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    // anisotropy regulariser (Eq. 13 on the actual scales)
    if (a.lambda_aniso != 0.0f) {
        int im = 0, in = 0;
#pragma unroll
        for (int m = 1; m < 3; ++m) {
            if (a.log_scale[3 * i + m] > a.log_scale[3 * i + im]) im = m;
            if (a.log_scale[3 * i + m] < a.log_scale[3 * i + in]) in = m;
        }
        const double ratio = exp(ls[im] - ls[in]);
        if (ratio > (double)a.lambda_r) {
            const double gr = (double)a.lambda_aniso * ratio / (double)a.n;
            ds[im] += gr;
            ds[in] -= gr;
        }
    }
    float gr[11];  // the gradient as float: mean (3), quat (4), log_scale (3), logit (1)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        gr[m] = (float)dmu[m];
        gr[7 + m] = (float)ds[m];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) gr[3 + m] = (float)((dq[m] - qh[m] * dot) / qn);
    gr[10] = (float)(dalpha * alpha * (1.0 - alpha));
    if (!a.adam) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            a.g_mean[3 * i + m] += gr[m];
            a.g_log_scale[3 * i + m] += gr[7 + m];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) a.g_quat[4 * i + m] += gr[3 + m];
        a.g_logit[i] += gr[10];
        return;
    }
    // fused Adam: the value a zeroed gradient buffer would hold (0 + g), applied at once to
    // the parameter and its moments, group by group
    constexpr int width[4] = {3, 4, 3, 1}, first[4] = {0, 3, 7, 10};
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
#pragma unroll
        for (int m = 0; m < width[grp]; ++m) {
            const int64_t e = width[grp] * i + m;
            float pv = a.prm[grp][e], mv = a.m1[grp][e], vv = a.m2[grp][e];
            adam_elem(pv, mv, vv, 0.0f + gr[first[grp] + m], a.adam_s[grp]);
            a.m1[grp][e] = mv;
            a.m2[grp][e] = vv;
            a.prm[grp][e] = pv;
        }
    }
}

// Gradient with respect to each listed grid's world->index affine [L | t] (boxes fixed): per
// Gaussian, c = L mu + t contributes dc mu^T to dL/dL and dc to dL/dt, and Sigma_idx =
// L Sigma L^T contributes 2 Gi L Sigma.  One pass over the Gaussians per grid; FP64 block sums
// part[block][grid][12] (row-major 3x4), added in a fixed order by k_pose_sum.
constexpr int POSE_BLOCKS = 256, POSE_THREADS = 256;
static_assert(GM_POSE_WORKSPACE_BYTES(1) == (size_t)POSE_BLOCKS * 12 * sizeof(double),
              "the header's workspace size follows the block count");

__global__ __launch_bounds__(POSE_THREADS) void k_pose(const ChainArgs a, double* part)
{
    __shared__ double red[POSE_THREADS / 64][12];
    for (int k = 0; k < a.n_ids; ++k) {
        const GridConst& G = a.g[k];
        const int gi = a.grid_index[k];
        double acc[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j] = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * POSE_THREADS + threadIdx.x; i < a.n;
             i += (int64_t)gridDim.x * POSE_THREADS) {
            if (a.tile_count[(size_t)gi * a.n + i] == 0) continue;  // empty box
            double qh[4], qn, R[9], S2[3], Sig[9];
            world_covariance(a.quat, a.log_scale, i, qh, &qn, R, S2, Sig);
            const double alpha = 1.0 / (1.0 + exp(-(double)a.logit[i]));
            const float* pg = a.grid_grads + ((size_t)gi * a.n + i) * 10;
            double dc[3], Gi[9];
            sigma_idx_grad(G, Sig, alpha, pg, dc, Gi);
            double GL[9], GLS[9];
            mm3(Gi, G.L, GL);
            mm3(GL, Sig, GLS);
            const double mu[3] = {a.mean[3 * i], a.mean[3 * i + 1], a.mean[3 * i + 2]};
#pragma unroll
            for (int r = 0; r < 3; ++r) {
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[4 * r + c] += dc[r] * mu[c] + 2.0 * GLS[3 * r + c];
                acc[4 * r + 3] += dc[r];
            }
        }
        // block sum: wavefront butterflies, then the four wavefronts in order
#pragma unroll
        for (int j = 0; j < 12; ++j)
            for (int o = 32; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o, 64);
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int j = 0; j < 12; ++j) red[threadIdx.x >> 6][j] = acc[j];
        __syncthreads();
        if (threadIdx.x < 12) {
            double v = 0.0;
            for (int w = 0; w < POSE_THREADS / 64; ++w) v += red[w][threadIdx.x];
            part[((size_t)blockIdx.x * a.n_ids + k) * 12 + threadIdx.x] = v;
        }
        __syncthreads();
    }
}

// one block per (grid, entry): the block partials added by a fixed tree in LDS
__global__ __launch_bounds__(POSE_BLOCKS) void k_pose_sum(const double* part, int nb, int n_ids,
                                                          double* out)
{
    __shared__ double sh[POSE_BLOCKS];
    const int e = blockIdx.x;   // (grid, entry)
    sh[threadIdx.x] = (int)threadIdx.x < nb ? part[(size_t)threadIdx.x * n_ids * 12 + e] : 0.0;
    __syncthreads();
    for (int o = POSE_BLOCKS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = sh[0];
}

}  // namespace

hipError_t launch_backward_partials(const BackwardArgs& a, hipStream_t s)
{
    if (a.n == 0 || a.n_ids == 0) return hipSuccess;
    const int32_t blocks = a.block_start[a.n_ids];   // one per tile of the listed grids
    if (blocks <= 0) return hipSuccess;
    bool masked = false;
    for (int k = 0; k < a.n_ids; ++k) masked = masked || a.masked[k];
    if (masked)
        hipLaunchKernelGGL(k_partials<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_partials<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_chain(const ChainArgs& a, hipStream_t s)
{
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_chain, dim3((unsigned)((a.n + 127) / 128)), dim3(128), 0, s, a);
    return hipGetLastError();
}

size_t pose_workspace_bytes(int n_ids) { return (size_t)POSE_BLOCKS * n_ids * 12 * sizeof(double); }

hipError_t launch_pose(const ChainArgs& a, double* out, void* ws, hipStream_t s)
{
    if (a.n_ids == 0) return hipSuccess;
    int64_t nb = (a.n + POSE_THREADS - 1) / POSE_THREADS;
    if (nb > POSE_BLOCKS) nb = POSE_BLOCKS;
    if (nb < 1) nb = 1;
    double* part = reinterpret_cast<double*>(ws);
    hipLaunchKernelGGL(k_pose, dim3((unsigned)nb), dim3(POSE_THREADS), 0, s, a, part);
    hipLaunchKernelGGL(k_pose_sum, dim3((unsigned)(a.n_ids * 12)), dim3(POSE_BLOCKS), 0, s, part,
                       (int)nb, a.n_ids, out);
    return hipGetLastError();
}
