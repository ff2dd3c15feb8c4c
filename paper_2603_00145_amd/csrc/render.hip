// K6: forward rendering of Magnetic Gaussians onto voxel tiles (Eq. 7; on stacks the
// Gaussian is pre-convolved with the slice profile, so the same formula applies with the
// record's amplitude and conic).
//
// One wavefront owns one GM_TX x GM_TY x GM_TZ tile and accumulates it in LDS.  It walks
// the tile's Gaussian list (ascending id) in batches of 32: a lane loads one record and
// prepares that Gaussian's piece (box intersect tile) in LDS.  Then the pieces are taken in
// list order.  A lane holds one (x, y) column of a piece's footprint and walks the piece's
// z-range, so the in-plane part of the exponent is formed once per column and each voxel
// costs two FMAs, one exp2 and one accumulate.  Two consecutive pieces whose footprints sum to
// at most 64 columns share the wave (the first piece's columns on the low lanes); the first
// piece's lanes add into the tile before the second's, so every voxel's sum is still formed
// in ascending Gaussian order and the result is the same on every run.
//
// With the paper's block query on a rotated grid (k_render_block, and k_render_field's MASK
// form) a Gaussian's voxels are not its box: each evaluated voxel of the box is also tested
// against the Gaussian's cell block (Eqs. 4-6) and gets zero when it fails (k_render_block
// forms the tile's voxel cells once per tile in LDS; the field kernel, short of LDS, forms
// them per voxel).
#include "nrf_core.h"

namespace {

__device__ __forceinline__ int sgpr(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Per (Gaussian, tile) piece, prepared lane-parallel for a batch of list entries, in the
// frame of the piece's intersection origin (the box clipped to the tile): the centre's x offset
// plus 1/2 and its y offset, the base-2 conic (off-diagonals doubled), the z-walk constants of
// the column formula below (F0, E, g1 = d0 kxz, g2 = d0 kyz), the footprint width (as a float
// and its reciprocal) and area, and the LDS index of the origin minus 1/2.
struct Piece {
    float uxh, uy, F0, E;
    float kxx, kyy, kzz, kxy;
    float kxz, kyz, g1, g2;
    float inv_wx, wxf, Ff, basef;
};

// Keeps the compiler from moving or merging LDS accesses across this point.  The two groups of
// lanes of a wave that hold two different Gaussians may touch the same voxel; their
// read-add-writes must stay two separate, ordered sequences.
__device__ __forceinline__ void lds_order() { __asm__ __volatile__("" ::: "memory"); }

// Column f of piece p, passed as fh = f + 1/2: its voxel values w[k] = amp 2^Q_k for the
// z-steps k < KM, and the LDS index of its voxel at k = 0.  The column is (x, y) = (f mod wx,
// f div wx), found as y = floor(fh / wx) (the fraction (x + 1/2) / wx stays at least 1/(2 wx)
// from an integer, far beyond the reciprocal's error) and x + 1/2 = fh - y wx, all exact in
// float.  With dz = k + d0 (d0 = minus the centre's z offset), Q_k = qxy + dz (bz + kzz dz),
// qxy = dx (kxx dx + kxy dy) + kyy dy^2 and bz = kxz dx + kyz dy, is expanded in k as
// A + k (B + k kzz) with A = dx (kxx dx + kxy dy + d0 kxz) + dy (kyy dy + d0 kyz) + F0 and
// B = bz + E: the per-piece parts (F0 = log2 amp + kzz d0^2, E = 2 kzz d0, d0 kxz, d0 kyz) are
// formed once, and amp enters as log2 amp in the exponent.
template <int KM>
__device__ __forceinline__ void eval_column(const Piece& p, float fh, float (&w)[KM], int& idx)
{
    const float yf = floorf(fh * p.inv_wx);
    const float xh = fmaf(-yf, p.wxf, fh);
    const float dx = xh - p.uxh;
    const float dy = yf - p.uy;
    const float A = fmaf(dx, fmaf(p.kxx, dx, fmaf(p.kxy, dy, p.g1)),
                         fmaf(dy, fmaf(p.kyy, dy, p.g2), p.F0));
    static_assert(GM_TX == 16 && GM_TY == 16, "index arithmetic assumes 16x16 tiles");
    idx = (int)fmaf(yf, (float)GM_TX, xh + p.basef);     // an exact small integer
    w[0] = __builtin_amdgcn_exp2f(A);
    if (KM > 1) {
        const float B = fmaf(p.kxz, dx, fmaf(p.kyz, dy, p.E));
#pragma unroll
        for (int k = 1; k < KM; ++k)
            w[k] = __builtin_amdgcn_exp2f(fmaf((float)k, fmaf((float)k, p.kzz, B), A));
    }
}

// The block query on a masked grid (Sec. 3.3.1, Eqs. 4-6): per piece of the batch, its first
// voxel in grid coordinates and its Gaussian's cell; per tile, the grid's index -> world affine
// and the query's resolution and radius.
struct PieceCell {
    int ix0, iy0, iz0, pad;
    int4 cm;
};
struct MaskCtx {
    bool on;                // the tile's grid is masked
    const PieceCell* pcc;   // the wavefront's batch
    const double* m;
    double res;
    int radius;
    const int* vc;          // the tile's voxel cells [3][GM_TILE_VOX] (x, y, z planes), or NULL
};

// w[k] = 0 for the voxels of column fh of piece p (as eval_column maps it, LDS index idx at
// k = 0) outside the block: from the tile's voxel cells when they are staged, else formed here
template <int KM>
__device__ __forceinline__ void mask_column(const Piece& p, const PieceCell& q, const MaskCtx& mc,
                                            float fh, int idx, float (&w)[KM])
{
    if (mc.vc) {
        const long long r = mc.radius;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            // a lane past its piece (or a z step past the tile) reads some voxel's cells and
            // stores nothing
            const int vi = min(max(idx + k * GM_TX * GM_TY, 0), GM_TILE_VOX - 1);
            const long long dx = (long long)mc.vc[vi] - q.cm.x;
            const long long dy = (long long)mc.vc[GM_TILE_VOX + vi] - q.cm.y;
            const long long dz = (long long)mc.vc[2 * GM_TILE_VOX + vi] - q.cm.z;
            const bool in = dx >= -r && dx <= r && dy >= -r && dy <= r && dz >= -r && dz <= r;
            if (!in) w[k] = 0.0f;
        }
        return;
    }
    const float yf = floorf(fh * p.inv_wx);
    const float xh = fmaf(-yf, p.wxf, fh);        // x + 1/2 within the piece
    const int x = q.ix0 + (int)xh, y = q.iy0 + (int)yf;
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (!voxel_in_block(mc.m, mc.res, mc.radius, x, y, q.iz0 + k, q.cm)) w[k] = 0.0f;
}

// acc[column voxel at z-step k] += w[k] for k < KZ (the piece's exact z extent; KZ <= the
// length of w).  The z-steps are distinct voxels, so all reads are issued before the writes.
template <int KZ, int KM>
__device__ __forceinline__ void add_column(float* acc, int idx, const float (&w)[KM])
{
    static_assert(KZ <= KM, "z extent within the evaluated steps");
    float old[KZ];
#pragma unroll
    for (int k = 0; k < KZ; ++k) old[k] = acc[idx + k * GM_TX * GM_TY];
#pragma unroll
    for (int k = 0; k < KZ; ++k) acc[idx + k * GM_TX * GM_TY] = old[k] + w[k];
}

// One piece on the whole wave: columns f0 + lane, KM z-steps each (lane_fh = lane + 1/2).
// MASK: mc (mc.on on a masked grid) and the piece's batch slot jq.
template <int KM, bool MASK>
__device__ __forceinline__ void single_piece(const Piece& p, float* acc, int F, float lane_fh,
                                             const MaskCtx& mc, int jq)
{
    float fh = lane_fh;
#pragma unroll 1
    for (int f0 = 0; f0 < F; f0 += 64) {
        float w[KM];
        int idx;
        eval_column<KM>(p, fh, w, idx);
        if (MASK && mc.on) mask_column<KM>(p, mc.pcc[jq], mc, fh, idx, w);
        if (fh < p.Ff) add_column<KM, KM>(acc, idx, w);
        fh += 64.0f;
    }
}

// Two pieces side by side in the wave (lane's piece p, column fh - 1/2) with z extents ZA
// and ZB, evaluated over the larger of the two.  The first piece's read-add-writes complete
// before the second piece's are issued.  Both extents are template parameters, so a pass
// dispatches once on the pair and its two add phases carry no branches of their own.
template <int ZA, int ZB, bool MASK>
__device__ __forceinline__ void paired_pieces(const Piece& p, float* acc, bool act, bool first,
                                              float fh, const MaskCtx& mc, int jq)
{
    constexpr int KM = ZA > ZB ? ZA : ZB;
    // every lane evaluates (a lane past its piece's footprint computes values it never
    // stores), so no lane mask is needed around the evaluation
    float w[KM];
    int idx;
    eval_column<KM>(p, fh, w, idx);
    if (MASK && mc.on) mask_column<KM>(p, mc.pcc[jq], mc, fh, idx, w);
    lds_order();
    if (act && first) add_column<ZA, KM>(acc, idx, w);
    lds_order();
    if (act && !first) add_column<ZB, KM>(acc, idx, w);
    lds_order();
}

// paired_pieces for uniform z extents wza, wzb in [1, GM_TZ]
template <bool MASK>
__device__ __forceinline__ void paired_pieces_kz(const Piece& p, float* acc, bool act,
                                                 bool first, float fh, int wza, int wzb,
                                                 const MaskCtx& mc, int jq)
{
    static_assert(GM_TZ == 4, "z extents 1..4 are dispatched below");
#define GM_PAIR_CASE(A, B) \
    case (A - 1) * 4 + (B - 1): paired_pieces<A, B, MASK>(p, acc, act, first, fh, mc, jq); break;
    switch ((wza - 1) * 4 + (wzb - 1)) {
    GM_PAIR_CASE(1, 1) GM_PAIR_CASE(1, 2) GM_PAIR_CASE(1, 3) GM_PAIR_CASE(1, 4)
    GM_PAIR_CASE(2, 1) GM_PAIR_CASE(2, 2) GM_PAIR_CASE(2, 3) GM_PAIR_CASE(2, 4)
    GM_PAIR_CASE(3, 1) GM_PAIR_CASE(3, 2) GM_PAIR_CASE(3, 3) GM_PAIR_CASE(3, 4)
    GM_PAIR_CASE(4, 1) GM_PAIR_CASE(4, 2) GM_PAIR_CASE(4, 3)
    default: paired_pieces<4, 4, MASK>(p, acc, act, first, fh, mc, jq); break;
    }
#undef GM_PAIR_CASE
}

// List entries prepared per batch; 32 keeps the LDS of a wavefront at 6 KB so that six
// wavefronts fit per SIMD.
constexpr int RB = 32;

// Barrier before LDS written by some lanes is read by others.  BLOCK: the workgroup is this
// one wavefront (a block barrier); otherwise the other wavefronts of the block run their own
// tiles, so only this wavefront's LDS accesses are ordered (a workgroup-scope fence waits for
// them; the wavefront's lanes run in lockstep).
template <bool BLOCK>
__device__ __forceinline__ void tile_sync()
{
    if constexpr (BLOCK) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

// Origin and grid of flattened tile t of a launch (t < a.total_blocks).
struct TilePos {
    const RenderGrid* G;
    int lt;                 // tile within its grid
    int t0x, t0y, t0z;      // first voxel
};

__device__ __forceinline__ TilePos tile_pos(const RenderArgs& a, int t)
{
    int r = 0;
#pragma unroll 1
    while (r + 1 < a.n_render && t >= a.rg[r + 1].first_block) ++r;
    TilePos p;
    p.G = &a.rg[r];
    p.lt = t - p.G->first_block;
    const int tx = p.lt % p.G->ntx, ty = (p.lt / p.G->ntx) % p.G->nty;
    const int tz = p.lt / (p.G->ntx * p.G->nty);
    p.t0x = tx * GM_TX;
    p.t0y = ty * GM_TY;
    p.t0z = tz * GM_TZ;
    return p;
}

constexpr int VPL = GM_TILE_VOX / 64;   // tile voxels per lane in the epilogues

// loss mode: the tile's data values, loaded before the Gaussian list is walked so that their
// latency is hidden behind the accumulation
__device__ __forceinline__ void load_targets(const TilePos& P, int lane, float (&tv)[VPL])
{
    const RenderGrid& G = *P.G;
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        const int i = j * 64 + lane;
        const int x = i % GM_TX, y = (i / GM_TX) % GM_TY, z = i / (GM_TX * GM_TY);
        const int gx = P.t0x + x, gy = P.t0y + y, gz = P.t0z + z;
        // outside the grid: a valid address (voxel 0) whose value goes unused
        const bool in = (gx < G.nx) & (gy < G.ny) & (gz < G.nz);
        const size_t v = in ? ((size_t)gz * G.ny + gy) * G.nx + gx : 0;
        tv[j] = __builtin_nontemporal_load(G.target + v);
    }
}

// acc (the tile's voxels, LDS) = the sum over the tile's list of Gaussians, in list order.
// Ends with a tile_sync, so every lane may read any voxel afterwards.  MASK: on a masked grid
// every voxel is also tested against its Gaussian's cell block (pcc: the batch's PieceCells;
// vcell, when given: LDS for the tile's voxel cells, formed once per tile).
template <bool BLOCK, bool MASK>
__device__ __forceinline__ void accumulate_tile(const RenderArgs& a, const TilePos& P, float* acc,
                                                Piece* pc, int lane, PieceCell* pcc,
                                                int* vcell = nullptr)
{
    const RenderGrid& G = *P.G;
    const int t0x = P.t0x, t0y = P.t0y, t0z = P.t0z;
    const float* __restrict__ recbase = a.records + (size_t)G.grid_index * a.n_gauss * 16;
    const int* __restrict__ pg = a.pair_gauss;
    const float lane_fh = (float)lane + 0.5f;

#pragma unroll
    for (int j = 0; j < GM_TILE_VOX / 64; ++j) acc[j * 64 + lane] = 0.0f;

    const int64_t bt = G.bin_tile_base + P.lt;
    const int s = sgpr(a.tile_start[bt]);
    const int e = sgpr(a.tile_start[bt + 1]);

    // Software pipeline over batches: while a batch's pieces are evaluated, the next batch's
    // records and the list entries of the batch after it are in flight (lane i of a batch
    // holds entry b0 + i).  Out-of-range lanes load nothing and keep zeros.
    // (the id's home bit is cleared only when the record is loaded, so that no wait for the
    // entry is placed right after its load)
    auto load_id = [&](int b) -> int {
        return (lane < RB && b + lane < e) ? pg[b + lane] : -1;
    };
    float4 n0 = make_float4(0, 0, 0, 0), n1 = n0, n2 = n0, n3 = n0;   // next batch's records
    auto load_rec = [&](int entry) {
        if (entry != -1) {
            const uint32_t gid = (uint32_t)entry & GM_ID_MASK;
            const float4* src = reinterpret_cast<const float4*>(recbase + (size_t)gid * 16);
            n0 = src[0];
            n1 = src[1];
            n2 = src[2];
            n3 = src[3];
        }
    };
    int id_rec = load_id(s);     // the entry whose record is in n0..n3
    load_rec(id_rec);
    int id_next = load_id(s + RB);
    MaskCtx mcv;
    mcv.pcc = pcc;
    mcv.m = G.index_to_world;
    mcv.res = a.bq.res;
    mcv.radius = a.bq.radius;
    mcv.vc = vcell;
    mcv.on = MASK && G.masked;
    const MaskCtx& mc = mcv;
    if (MASK && mc.on && vcell) {
        // the cells of the tile's voxels (the tile_sync at the first batch orders these
        // stores before their reads), clamped to [-2^30, 2^30] as the means' cells are
#pragma unroll 1
        for (int j = 0; j < GM_TILE_VOX / 64; ++j) {
            const int i = j * 64 + lane;
            double c[3];
            voxel_cells(G.index_to_world, a.bq.res, t0x + i % GM_TX, t0y + (i / GM_TX) % GM_TY,
                        t0z + i / (GM_TX * GM_TY), c);
#pragma unroll
            for (int u = 0; u < 3; ++u)
                vcell[u * GM_TILE_VOX + i] = (int)fmin(fmax(c[u], -1073741824.0), 1073741824.0);
        }
    }

#pragma unroll 1
    for (int b0 = s; b0 < e; b0 += RB) {
        const int nb = min(RB, e - b0);
        const float4 r0 = n0, r1 = n1, r2 = n2, r3 = n3;
        const int my_entry = id_rec;
        load_rec(id_next);
        id_rec = id_next;
        id_next = load_id(b0 + 2 * RB);
        tile_sync<BLOCK>();
        int myF = 0, myWz = 0;  // this lane's piece: footprint area and z extent
        if (lane < nb) {
            const int lox = __float_as_int(r2.z), loy = __float_as_int(r2.w);
            const int loz = __float_as_int(r3.x), hix = __float_as_int(r3.y);
            const int hiy = __float_as_int(r3.z), hiz = __float_as_int(r3.w);
            const int ix0 = max(lox, t0x), iy0 = max(loy, t0y), iz0 = max(loz, t0z);
            const int wx = min(hix, t0x + GM_TX - 1) - ix0 + 1;
            const int wy = min(hiy, t0y + GM_TY - 1) - iy0 + 1;
            const int wz = min(hiz, t0z + GM_TZ - 1) - iz0 + 1;
            const bool ok = wx > 0 && wy > 0 && wz > 0;  // always true for a listed tile
            const float d0 = (float)(iz0 - loz) - r0.z;
            const int wxe = ok ? wx : 1;
            Piece p;
            p.uxh = (r0.x - (float)(ix0 - lox)) + 0.5f;
            p.uy = r0.y - (float)(iy0 - loy);
            p.kxx = r1.x; p.kyy = r1.y; p.kzz = r1.z; p.kxy = r1.w;
            p.kxz = r2.x; p.kyz = r2.y;
            // amp >= 0 (0 for an empty box, never listed): log2 0 = -inf gives zeros
            p.F0 = log2f(r0.w) + p.kzz * d0 * d0;
            p.E = 2.0f * p.kzz * d0;
            p.g1 = d0 * p.kxz;
            p.g2 = d0 * p.kyz;
            p.wxf = (float)wxe;
            p.inv_wx = __builtin_amdgcn_rcpf(p.wxf);
            myF = ok ? wx * wy : 0;
            myWz = ok ? wz : 0;
            p.Ff = (float)myF;
            p.basef = (float)(((iz0 - t0z) * GM_TY + (iy0 - t0y)) * GM_TX + (ix0 - t0x)) - 0.5f;
            pc[lane] = p;
            if (MASK && mc.on) {
                PieceCell q;
                q.ix0 = ix0;
                q.iy0 = iy0;
                q.iz0 = iz0;
                q.pad = 0;
                q.cm = a.bq.cells[(uint32_t)my_entry & GM_ID_MASK];
                pcc[lane] = q;
            }
        }
        // bit j: pieces j and j + 1 fit side by side in the wave (footprints summing to <= 64)
        const int nextF = __shfl_down(myF, 1, 64);
        const uint64_t pm = __ballot(lane + 1 < nb && myF + nextF <= 64);
        // lane j: (F_j << 6) | (wz_{j+1} << 3) | wz_j, so that one read gives a pass its
        // footprint and both z extents (F <= 256, wz <= 4)
        const int pk = (myF << 6) | (__shfl_down(myWz, 1, 64) << 3) | myWz;
        tile_sync<BLOCK>();
        int j = 0;
#pragma unroll 1
        while (j < nb) {
            const int k = __builtin_amdgcn_readlane(pk, j);
            if ((pm >> j) & 1u) {
                // pieces j and j+1 side by side: lanes [0, Fa) take piece j, the next Fb piece j+1
                const int Fa = k >> 6, wza = k & 7, wzb = (k >> 3) & 7;
                const bool first = lane < Fa;
                const Piece p = *reinterpret_cast<const Piece*>(
                    reinterpret_cast<const char*>(pc + j) + (first ? 0 : (int)sizeof(Piece)));
                const float fh = lane_fh - (first ? 0.0f : (float)Fa);
                const bool act = fh < p.Ff;
                paired_pieces_kz<MASK>(p, acc, act, first, fh, wza, wzb, mc, first ? j : j + 1);
                j += 2;
            } else {
                const Piece p = pc[j];
                const int F = k >> 6, wz = k & 7;
                switch (wz) {
                case 0: break;
                case 1: single_piece<1, MASK>(p, acc, F, lane_fh, mc, j); break;
                case 2: single_piece<2, MASK>(p, acc, F, lane_fh, mc, j); break;
                case 3: single_piece<3, MASK>(p, acc, F, lane_fh, mc, j); break;
                default: single_piece<GM_TZ, MASK>(p, acc, F, lane_fh, mc, j); break;
                }
                j += 1;
            }
        }
    }
    tile_sync<BLOCK>();
}

// Writes the finished tile (plain mode), or (loss mode) the smooth-L1 data term on it (Eq. 11,
// beta = 1): dL/dI = clamp(I - y, -1, 1) / N, the rendering when G.out is set, and the tile's
// FP64 sum of smoothL1(I - y) to a.loss_part[part].
__device__ __forceinline__ void finish_tile(const RenderArgs& a, const TilePos& P,
                                            const float* acc, const float (&tv)[VPL], int lane,
                                            int part)
{
    const RenderGrid& G = *P.G;
    float* out = G.out;
    if (!a.loss_part) {
#pragma unroll
        for (int j = 0; j < GM_TILE_VOX / 64; ++j) {
            const int i = j * 64 + lane;
            const int x = i % GM_TX, y = (i / GM_TX) % GM_TY, z = i / (GM_TX * GM_TY);
            const int gx = P.t0x + x, gy = P.t0y + y, gz = P.t0z + z;
            if ((gx < G.nx) & (gy < G.ny) & (gz < G.nz))
                out[((size_t)gz * G.ny + gy) * G.nx + gx] = acc[i];
        }
        return;
    }
    const float g_scale = (float)a.inv_n;
    double lsum = 0.0;
#pragma unroll
    for (int j = 0; j < GM_TILE_VOX / 64; ++j) {
        const int i = j * 64 + lane;
        const int x = i % GM_TX, y = (i / GM_TX) % GM_TY, z = i / (GM_TX * GM_TY);
        const int gx = P.t0x + x, gy = P.t0y + y, gz = P.t0z + z;
        if ((gx < G.nx) & (gy < G.ny) & (gz < G.nz)) {
            const size_t v = ((size_t)gz * G.ny + gy) * G.nx + gx;
            const float val = acc[i];
            if (out) out[v] = val;
            const float d = val - tv[j];
            const float ad = fabsf(d);
            lsum += ad < 1.0f ? 0.5 * (double)d * (double)d : (double)ad - 0.5;
            G.dl[v] = fminf(fmaxf(d, -1.0f), 1.0f) * g_scale;
        }
    }
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
    if (lane == 0) a.loss_part[part] = lsum;
}

__global__ __launch_bounds__(64) void k_render(const RenderArgs a)
{
    __shared__ float acc[GM_TILE_VOX];
    __shared__ Piece pc[RB];
    const int lane = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const TilePos P = tile_pos(a, blk);
    float tv[VPL];
    if (a.loss_part) load_targets(P, lane, tv);
    accumulate_tile<true, false>(a, P, acc, pc, lane, nullptr);
    finish_tile(a, P, acc, tv, lane, blk);
}

// k_render for launches that hold a masked grid (the block query on a rotated grid)
__global__ __launch_bounds__(64) void k_render_block(const RenderArgs a)
{
    __shared__ float acc[GM_TILE_VOX];
    __shared__ Piece pc[RB];
    __shared__ PieceCell pcc[RB];
    __shared__ int vcell[3 * GM_TILE_VOX];
    const int lane = threadIdx.x;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const TilePos P = tile_pos(a, blk);
    float tv[VPL];
    if (a.loss_part) load_targets(P, lane, tv);
    accumulate_tile<true, true>(a, P, acc, pc, lane, pcc, vcell);
    finish_tile(a, P, acc, tv, lane, blk);
}

// Render + residual field (Sec. 3.4, Eq. 8: I_final = I + r) in one pass.  Blocks of FW
// wavefronts share the field's weights, staged once in LDS; each wavefront takes whole tiles
// (the tiles of the launch are split into eight contiguous ranges, one per XCD, whose blocks
// deal them to their wavefronts), renders a tile into its LDS accumulator exactly as k_render
// does, then evaluates the field on the tile's voxels in 64 groups of 16 (one x row each) and
// adds out_scale tanh(z_out) to each voxel before the store or loss epilogue.  Each point's
// field value is the same arithmetic as the field's own forward kernel, so the result is bit
// for bit the render followed by gm_nrf_forward (and the loss the same terms).
constexpr int FW = 8;

template <int KT, int DEPTH, bool MASK>
__global__ __launch_bounds__(64 * FW) void k_render_field(const RenderArgs a, const NrfArgs f)
{
    __shared__ nrfcore::Lds<KT, DEPTH> sw;
    __shared__ float accs[FW][GM_TILE_VOX];
    __shared__ Piece pcs[FW][RB];
    __shared__ PieceCell pccs[MASK ? FW : 1][RB];
    nrfcore::load_weights<KT, DEPTH>(f, sw);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, row = lane & 15;
    nrfcore::v4s wo[4];
    nrfcore::load_wout(f, wo);
    float* acc = accs[w];
    Piece* pc = pcs[w];
    const int xcd = blockIdx.x & 7;
    const int nbx = (int)(gridDim.x >> 3);     // the launch has a multiple of 8 blocks
    const int T = a.total_blocks;
    const int lo = (int)((int64_t)T * xcd / 8), hi = (int)((int64_t)T * (xcd + 1) / 8);
#pragma unroll 1
    for (int t = lo + (int)(blockIdx.x >> 3) * FW + w; t < hi; t += nbx * FW) {
        const TilePos P = tile_pos(a, t);
        const RenderGrid& G = *P.G;
        float tv[VPL];
        if (a.loss_part) load_targets(P, lane, tv);
        accumulate_tile<false, MASK>(a, P, acc, pc, lane, pccs[MASK ? w : 0]);
#pragma unroll 1
        for (int q = 0; q < GM_TILE_VOX / 16; ++q) {
            const int vy = P.t0y + (q % GM_TY), vz = P.t0z + q / GM_TY, vx = P.t0x + row;
            if (vy >= G.ny || vz >= G.nz) continue;     // uniform over the wavefront
            const float x[3] = {nrfcore::world_coord(G.index_to_world, vx, vy, vz),
                                nrfcore::world_coord(G.index_to_world + 4, vx, vy, vz),
                                nrfcore::world_coord(G.index_to_world + 8, vx, vy, vz)};
            nrfcore::Tile<KT, DEPTH> Tl;
            nrfcore::tile_forward<KT, DEPTH>(f, sw, x, Tl);
            const float zo = nrfcore::tile_output<KT, DEPTH>(f, Tl, wo);   // lane group 0
            if (g == 0 && vx < G.nx) acc[q * 16 + row] += f.out_scale * tanhf(zo);
        }
        tile_sync<false>();
        finish_tile(a, P, acc, tv, lane, t);
        tile_sync<false>();
    }
}

// loss = inv_n * sum of the per-block sums, in a fixed order.  Each thread takes four
// partials per round (all four loads in flight), then a tree over the block.
constexpr int FIN_THREADS = 1024;

__global__ __launch_bounds__(FIN_THREADS) void k_render_loss_finish(const double* part, int nb,
                                                                    double inv_n, float* loss)
{
    __shared__ double sh[FIN_THREADS];
    const int t = threadIdx.x;
    double v = 0.0;
    for (int i = t; i < nb; i += 4 * FIN_THREADS) {
        double q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = i + u * FIN_THREADS;
            q[u] = k < nb ? part[k] : 0.0;
        }
        v += (q[0] + q[1]) + (q[2] + q[3]);
    }
    sh[t] = v;
    __syncthreads();
    for (int o = FIN_THREADS / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    if (t == 0) *loss = (float)(sh[0] * inv_n);
}

}  // namespace

hipError_t launch_render(const RenderArgs& a, hipStream_t s)
{
    if (a.total_blocks == 0) return hipSuccess;
    bool masked = false;
    for (int k = 0; k < a.n_render; ++k) masked = masked || a.rg[k].masked;
    if (masked)
        hipLaunchKernelGGL(k_render_block, dim3((unsigned)a.total_blocks), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL(k_render, dim3((unsigned)a.total_blocks), dim3(64), 0, s, a);
    if (a.loss_part)
        hipLaunchKernelGGL(k_render_loss_finish, dim3(1), dim3(FIN_THREADS), 0, s, a.loss_part,
                           a.total_blocks, a.inv_n, a.loss);
    return hipGetLastError();
}

template <int KT, int DEPTH, bool MASK>
static void launch_field_mt(const RenderArgs& a, const NrfArgs& f, hipStream_t s)
{
    // every block resident at once, a multiple of 8 (one share per XCD), capped by the tiles
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_render_field<KT, DEPTH, MASK>,
                                                       64 * FW, 0);
    int64_t full = (int64_t)(cus > 0 ? cus : 256) * (per_cu > 0 ? per_cu : 1);
    int64_t need = ((int64_t)a.total_blocks + FW - 1) / FW;
    int64_t nb = need < full ? need : full;
    nb = (nb + 7) / 8 * 8;
    hipLaunchKernelGGL((k_render_field<KT, DEPTH, MASK>), dim3((unsigned)nb), dim3(64 * FW), 0, s,
                       a, f);
}

template <int KT, int DEPTH>
static void launch_field_t(const RenderArgs& a, const NrfArgs& f, hipStream_t s)
{
    bool masked = false;
    for (int k = 0; k < a.n_render; ++k) masked = masked || a.rg[k].masked;
    if (masked)
        launch_field_mt<KT, DEPTH, true>(a, f, s);
    else
        launch_field_mt<KT, DEPTH, false>(a, f, s);
}

hipError_t launch_render_field(const RenderArgs& a, const NrfArgs& f, hipStream_t s)
{
    if (a.total_blocks == 0) return hipSuccess;
    switch ((f.in_pad >> 4) * 8 + f.depth) {
    case 4 * 8 + 1: launch_field_t<4, 1>(a, f, s); break;
    case 4 * 8 + 2: launch_field_t<4, 2>(a, f, s); break;
    case 4 * 8 + 3: launch_field_t<4, 3>(a, f, s); break;
    case 4 * 8 + 4: launch_field_t<4, 4>(a, f, s); break;
    case 8 * 8 + 1: launch_field_t<8, 1>(a, f, s); break;
    case 8 * 8 + 2: launch_field_t<8, 2>(a, f, s); break;
    case 8 * 8 + 3: launch_field_t<8, 3>(a, f, s); break;
    case 8 * 8 + 4: launch_field_t<8, 4>(a, f, s); break;
    default: return hipErrorInvalidValue;
    }
    if (a.loss_part)
        hipLaunchKernelGGL(k_render_loss_finish, dim3(1), dim3(FIN_THREADS), 0, s, a.loss_part,
                           a.total_blocks, a.inv_n, a.loss);
    return hipGetLastError();
}
