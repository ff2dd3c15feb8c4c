// Internal declarations shared by the HIP translation units of libgm (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gm.h"

// Tile of the forward render: one wavefront owns one tile and accumulates it in LDS.
#define GM_TX 16
#define GM_TY 16
#define GM_TZ 4
#define GM_TILE_VOX (GM_TX * GM_TY * GM_TZ)
// Set on the one entry of each (grid, Gaussian) in the tile lists whose tile holds the box's
// lower corner; the id is the low 31 bits.
#define GM_HOME_BIT 0x80000000u
#define GM_ID_MASK 0x7fffffffu

// -1/2 log2(e): folds the Gaussian's -1/2 and the change to base 2 into the conic.
#define GM_KAPPA (-0.72134752044448170368)
#define GM_LN2F 0.69314718055994530942f

struct GridConst {
    int32_t nx, ny, nz;
    int32_t ntx, nty, ntz;   // tiles per axis
    int64_t tile_base;       // global id of the grid's first tile
    double L[9];             // world -> index linear part, row-major
    double t[3];
    double sig;              // slice-profile sigma along index z
    int32_t waxis[3];        // world axis of each index axis (axis-aligned grids), else -1
};

// The paper's cell-neighbourhood query (Sec. 3.3.1, Eqs. 4-6) on a grid that is not
// axis-aligned: a voxel takes a Gaussian when, on every world axis, the Eq. 4 cell of the
// voxel's world position lies within the block radius of the cell of the Gaussian's mean.
// Such a voxel set is not a box, so the binning gives each Gaussian a box that contains it and
// the kernels test every voxel of that box.
struct BlockQuery {
    const int4* cells;   // [n]: each Gaussian's cell (x, y, z, 0), clamped to [-2^30, 2^30]
    double res;          // cells per axis of [-1, 1]
    int32_t radius;      // block radius (> 0)
};

// The voxel's world position ((m_a0 x + m_a1 y) + m_a2 z) + m_a3 per world axis a (m the
// grid's index -> world affine, row-major 3x4) and its cell floor(((w + 1) res) / 2), in
// binary64 without contraction.
__device__ __forceinline__ void voxel_cells(const double* m, double res, int x, int y, int z,
                                            double (&cell)[3])
{
#pragma clang fp contract(off)
    const double xd = (double)x, yd = (double)y, zd = (double)z;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double w = ((m[4 * a] * xd + m[4 * a + 1] * yd) + m[4 * a + 2] * zd) + m[4 * a + 3];
        cell[a] = floor(((w + 1.0) * res) / 2.0);
    }
}

// true when every axis of the voxel's cell is within radius of cm
__device__ __forceinline__ bool voxel_in_block(const double* m, double res, int radius, int x,
                                               int y, int z, int4 cm)
{
    double cell[3];
    voxel_cells(m, res, x, y, z, cell);
    const double r = (double)radius;
    return cell[0] >= (double)cm.x - r && cell[0] <= (double)cm.x + r &&
           cell[1] >= (double)cm.y - r && cell[1] <= (double)cm.y + r &&
           cell[2] >= (double)cm.z - r && cell[2] <= (double)cm.z + r;
}

// ---- launchers (one per kernel family) --------------------------------------------------
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);

// What gm_bin reads back after its one synchronisation: device-detected conditions (bit 0:
// a non-finite parameter or zero quaternion), per-grid contributing-pair totals (summed by
// the preprocess kernel) and the (tile, Gaussian) pair total from the scan.
struct BinReport {
    uint32_t flags[4];
    unsigned long long box_volume[GM_MAX_GRIDS];
    int64_t grid_start[GM_MAX_GRIDS + 1];  // first list entry of each grid; [n_grids] = total
};
hipError_t launch_bin_report(BinReport* rep, const int64_t* offsets, int64_t n,
                             int64_t* box_volume, int n_grids, BinReport* host, hipStream_t s);

struct PreprocessArgs {
    int64_t n;
    int32_t n_grids;
    double cutoff;
    int32_t block_radius;    // > 0: the cell-neighbourhood query of Eqs. 4-6 instead
    int32_t cell_res;
    const float* mean;
    const float* quat;
    const float* log_scale;
    const float* logit;
    float* records;          // [n_grids][n][16]
    int32_t* tile_count;     // [n_grids][n]
    unsigned long long* box_volume;  // [n_grids]
    uint32_t* flags;         // bit 0: invalid parameter seen; bit 1: block box not settled
    float* grid_grads;       // [n_grids][n][10] or NULL: zeroed for empty boxes
    uint32_t* tile_box;      // [n_grids][n][3]: the box's tile range (lo, hi) as 16-bit
                             // fields x | y << 16, z | X << 16, Y | Z << 16 (lo > hi: empty)
    int4* cells;             // block query: each Gaussian's cell (written once per Gaussian)
    GridConst g[GM_MAX_GRIDS];
};
hipError_t launch_preprocess(const PreprocessArgs& a, hipStream_t s);

// exclusive scan of int32 counts into int64 offsets; total at out[n]
size_t scan_workspace_bytes(int64_t n);
hipError_t launch_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* ws,
                                  hipStream_t s);

struct EmitArgs {
    int64_t n;
    int32_t n_grids;
    const uint32_t* tile_box;  // [n_grids * n][3], as written by the preprocess
    const int64_t* offsets;  // [n_grids * n + 1]
    int64_t capacity;        // pairs the key/value buffers hold: a Gaussian past it emits none
    uint32_t* keys;
    uint32_t* vals;
    GridConst g[GM_MAX_GRIDS];
};
hipError_t launch_emit(const EmitArgs& a, hipStream_t s);

// stable LSD radix sort of (key, value) pairs on the low `bits` key bits.
size_t radix_workspace_bytes(int64_t n);
hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                             uint32_t* vals_alt, int64_t n, int bits, void* ws,
                             int* result_in_alt, hipStream_t s);

hipError_t launch_tile_ranges(const uint32_t* sorted_keys, int64_t n_pairs, int32_t* tile_start,
                              int64_t total_tiles, hipStream_t s);
hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, int64_t n, hipStream_t s);

struct RenderGrid {
    int32_t nx, ny, nz, ntx, nty, ntz;
    int32_t grid_index;      // index into the binned grids (records)
    int32_t first_block;     // first flattened tile of this grid in the launch
    int64_t bin_tile_base;   // global tile id of the grid's first tile in the binning
    float* out;              // rendered values, or NULL (loss mode only)
    const float* target;     // loss mode: the stack's data
    float* dl;               // loss mode: dL/dI of the smooth-L1 term
    double index_to_world[12]; // with a residual field or a masked grid: index -> world
    int32_t masked;          // the block query on a rotated grid: test every voxel
};
struct RenderArgs {
    int32_t n_render;
    int32_t total_blocks;
    int64_t n_gauss;
    const float* records;
    const int32_t* tile_start;
    const int32_t* pair_gauss;
    double* loss_part;       // loss mode (non-NULL): per-block smooth-L1 sums [total_blocks]
    float* loss;             // loss mode: the mean, written by the finishing kernel
    double inv_n;            // loss mode: 1 / voxels of the listed grids
    BlockQuery bq;           // read on masked grids
    RenderGrid rg[GM_MAX_GRIDS];
};
hipError_t launch_render(const RenderArgs& a, hipStream_t s);
struct NrfArgs;
// the render with the residual field added to every voxel in the same pass (f's grid fields
// unused: each grid's index -> world affine comes from its RenderGrid)
hipError_t launch_render_field(const RenderArgs& a, const NrfArgs& f, hipStream_t s);

struct BackwardArgs {
    int64_t n;
    int32_t n_ids;
    const float* records;
    float* grid_grads;
    int32_t grid_index[GM_MAX_GRIDS];
    int32_t nx[GM_MAX_GRIDS], ny[GM_MAX_GRIDS], nz[GM_MAX_GRIDS];
    const float* dl_di[GM_MAX_GRIDS];
    const uint32_t* pair_gauss;         // tile-sorted entries, GM_HOME_BIT on home entries
    const int32_t* tile_start;          // CSR rows of the tile lists
    int64_t tile_base[GM_MAX_GRIDS];    // global id of each listed grid's first tile
    int32_t ntx[GM_MAX_GRIDS], nty[GM_MAX_GRIDS];
    int32_t block_start[GM_MAX_GRIDS + 1];  // first block (= tile) of each listed grid
    BlockQuery bq;                      // read on masked grids
    int32_t block_query;                // the bins come from the block query (any grid)
    int32_t masked[GM_MAX_GRIDS];       // the block query on a rotated grid
    double m[GM_MAX_GRIDS][12];         // masked grids: index -> world affine
};
hipError_t launch_backward_partials(const BackwardArgs& a, hipStream_t s);

// Adam's per-group scalars, rounded once to float from double hyperparameters
struct AdamScalars {
    float b1, omb1, b2, omb2, eps, step_size, bc2_sqrt;
};
AdamScalars adam_scalars(double lr, double beta1, double beta2, double eps, int32_t step);

// One Adam element update (PyTorch arrangement).  No multiply-add is contracted here (division
// and square root are correctly rounded), so that each kernel that calls it (the plain step and
// the fused chain step) gives the same bits.
__device__ __forceinline__ void adam_elem(float& p, float& m, float& v, float g,
                                          const AdamScalars& c)
{
#pragma clang fp contract(off)
    const float mi = c.b1 * m + c.omb1 * g;
    const float vi = c.b2 * v + c.omb2 * g * g;
    m = mi;
    v = vi;
    p = p - c.step_size * mi / (sqrtf(vi) / c.bc2_sqrt + c.eps);
}

struct ChainArgs {
    int64_t n;
    int32_t n_ids;
    float lambda_aniso, lambda_r;
    const float* mean;
    const float* quat;
    const float* log_scale;
    const float* logit;
    const int32_t* tile_count;  // [grids][n]: 0 exactly for an empty box
    const float* grid_grads;
    float* g_mean;
    float* g_quat;
    float* g_log_scale;
    float* g_logit;
    // fused Adam (adam != 0): the gradient is applied to the parameters (prm, the same arrays
    // as mean..logit) and the moments m1, m2 of groups mean, quat, log_scale, logit instead of
    // being added to g_*
    int32_t adam;
    float* prm[4];
    float* m1[4];
    float* m2[4];
    AdamScalars adam_s[4];
    int32_t grid_index[GM_MAX_GRIDS];
    GridConst g[GM_MAX_GRIDS];
};
hipError_t launch_chain(const ChainArgs& a, hipStream_t s);
// gradient with respect to the listed grids' affines: out [n_ids][12] doubles
size_t pose_workspace_bytes(int n_ids);
hipError_t launch_pose(const ChainArgs& a, double* out, void* ws, hipStream_t s);

struct LossArgs {
    int32_t n_stacks;
    int64_t total;
    int64_t begin[GM_MAX_GRIDS + 1];
    const float* pred[GM_MAX_GRIDS];
    const float* target[GM_MAX_GRIDS];
    float* dl[GM_MAX_GRIDS];
};
hipError_t launch_smooth_l1(const LossArgs& a, float* loss, void* ws, hipStream_t s);

// SSIM term on whole stack slices (Eq. 10): every z-slice is a 2D image; 16 x 32 pixel tiles
constexpr double GM_SSIM_C1 = 0.01 * 0.01, GM_SSIM_C2 = 0.03 * 0.03;
struct SsimArgs {
    int32_t n_stacks;
    int32_t nx[GM_MAX_GRIDS], ny[GM_MAX_GRIDS];
    int32_t tiles_x[GM_MAX_GRIDS], tiles_y[GM_MAX_GRIDS];
    int64_t tile_begin[GM_MAX_GRIDS + 1];   // prefix of nz * tiles_y * tiles_x
    const float* pred[GM_MAX_GRIDS];
    const float* target[GM_MAX_GRIDS];
    float* dl[GM_MAX_GRIDS];
    double g[11];                           // 1D window taps, sum 1
    double grad_scale;                      // -lambda / N
};
void ssim_tiles(int nx, int ny, int* tiles_x, int* tiles_y);
hipError_t launch_ssim(const SsimArgs& a, int64_t n_voxels, float* loss, void* ws, hipStream_t s);
hipError_t launch_aniso(const float* log_scale, int64_t n, float lambda_r, float* value,
                        void* ws, hipStream_t s);
hipError_t launch_mse(const float* a, const float* b, int64_t n, float* mse, void* ws,
                      hipStream_t s);
// scalars formed in double on the host and rounded once: 1 - beta, lr / (1 - beta1^t),
// sqrt(1 - beta2^t)
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n,
                       const AdamScalars& c, hipStream_t s);

struct DevoxArgs {
    int32_t g;
    int32_t n_stacks;
    const float* data[GM_MAX_GRIDS];
    GridConst s[GM_MAX_GRIDS];
    float* mean;
    float* quat;
    float* log_scale;
    float* logit;
};
hipError_t launch_devox(const DevoxArgs& a, hipStream_t s);

struct UpsampleArgs {
    int32_t g_old, g_new;
    const float* quat;         // old lattice [g_old^3][4]
    const float* log_scale;    // [g_old^3][3]
    const float* logit;        // [g_old^3]
    float* out_mean;           // new lattice [g_new^3][3]
    float* out_quat;
    float* out_log_scale;
    float* out_logit;
};
hipError_t launch_upsample(const UpsampleArgs& a, hipStream_t s);

struct NrfArgs {
    int32_t n_freq, depth, in_pad;
    float out_scale;
    const uint16_t* w_in;
    const float* b_in;
    const uint16_t* w_hid;
    const float* b_hid;
    const uint16_t* w_out;
    const float* b_out;
    int32_t nx, ny, nz;
    int64_t n_points;
    const int32_t* idx;      // voxel linear indices, or NULL for every voxel in order
    double m[12];            // index -> world affine
    float* out;              // forward: out[v] += r
    const float* dl_dr;      // backward: per-voxel dL/dr of the grid
    float scale;
    float* g_w_in;
    float* g_b_in;
    float* g_w_hid;
    float* g_b_hid;
    float* g_w_out;
    float* g_b_out;
};
struct NrfWork {
    int64_t P;               // workspace points (every grid's, each rounded up to 16)
    float* dzo;              // [P]
    uint16_t* dz[4];         // [64][P] per layer
    uint16_t* a[5];          // a[0] [in_pad][P], a[l] [64][P]
    float* part;             // split-K partials
    // the chain kernel's grid: its points sit at workspace columns p0 .. p0 + np (np its point
    // count rounded up to 16), its wavefronts' output-layer partials at rows wave0 .. of
    // nwaves_total
    int64_t p0, np, wave0, nwaves_total;
};
// most frequency bands the kernels encode with in_pad 64 / 128 input features
int nrf_max_bands(int in_pad);
hipError_t launch_nrf_forward(const NrfArgs& a, hipStream_t s);
// floats of split-K / row-sum partials gm_nrf_backward needs for P points
size_t nrf_part_floats(int64_t P, int in_pad);
hipError_t launch_nrf_backward(const NrfArgs& a, const NrfWork& w, hipStream_t s);
// the backward summed over n grids' point lists (a[k]: grid k's arguments, the weights and
// gradients the same in all), into one workspace of w.P = sum of the rounded point counts
hipError_t launch_nrf_backward_grids(const NrfArgs* a, int n, const NrfWork& w, hipStream_t s);
// chain kernel blocks (4 wavefronts each) for np points
unsigned nrf_chain_blocks(const NrfArgs& a, int64_t np);
hipError_t launch_to_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s);

struct WsGatherArgs {
    int64_t n;
    float spacing;
    const float* means;
    uint16_t* patches;
    const float* data[3];
    GridConst s[3];
};
struct WsNet {
    const uint16_t* w[4];
    const float* b[4];
    const float* wl;
    const float* bl;
};
struct WsActs {
    float* z[4];
    uint16_t* a[4];
    uint16_t* dz[4];
    float* part;
};
struct WsHeadArgs {
    int64_t n;
    const float* z4;
    const float* wl;
    const float* bl;
    const float* s0;
    const float* logit0;
    float* s_out;
    float* q_out;
    float* logit_out;
    const float* sig_t;      // NULL: inference only
    const float* logit_t;
    float* loss_each;
    float* dout;
    float* a4;
    uint16_t* dz4;
};
struct WsGrads {
    float* w[4];
    float* b[4];
    float* wl;
    float* bl;
};
int ws_kpad(int layer);
size_t ws_part_floats(int64_t B);
hipError_t launch_ws_gather(const WsGatherArgs& a, hipStream_t s);
hipError_t launch_ws_targets(const float* ls, const float* quat, int64_t n, float* sig6,
                             hipStream_t s);
hipError_t launch_ws_forward(const WsNet& net, const uint16_t* X0, int64_t B, const WsActs& w,
                             const WsHeadArgs& head, hipStream_t s);
hipError_t launch_ws_backward(const WsNet& net, const uint16_t* X0, int64_t B, const WsActs& w,
                              const WsHeadArgs& head, const WsGrads& g, float* loss, hipStream_t s);

// ---- device helpers ---------------------------------------------------------------------
#ifdef __HIPCC__
// Sum of v over the 64 lanes of the wavefront, returned in every lane (DPP adds within each
// row of 16, row broadcasts across rows, then lane 63 read back).
__device__ __forceinline__ float wave_sum(float v)
{
    int xi;
    xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false); // quad xor 1
    v += __int_as_float(xi);
    xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false); // quad xor 2
    v += __int_as_float(xi);
    xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false); // half mirror
    v += __int_as_float(xi);
    xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false); // mirror
    v += __int_as_float(xi);
    xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false); // bcast15
    v += __int_as_float(xi);
    xi = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false); // bcast31
    v += __int_as_float(xi);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Bijective blockIdx -> work-item map that gives each XCD (workgroups are dealt to the 8 XCDs
// round robin) a contiguous range of work items, so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int xcd = b & 7, k = b >> 3;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
}
#endif
