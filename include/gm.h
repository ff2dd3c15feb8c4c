/* gm.h - C ABI of the Magnetic-Gaussian voxel-evaluation library (libgm.so, gfx950).
 *
 * The library evaluates the paper's Magnetic Gaussian primitives (M-Gaussian, arXiv
 * 2603.00145, Sec. 3.2, Eq. 2-3) onto voxel grids - the thick-slice stacks a
 * reconstruction is fitted to (Sec. 3.3.2, Eq. 7, with a Gaussian slice profile along each
 * stack's slice normal) and the isotropic target volume (Sec. 3.1, inference) - and runs
 * the matching backward pass, the losses of Sec. 3.5.2 and the Adam update of Sec. 4.1.4.
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless marked [host].  The caller allocates and frees
 *     every buffer; the library allocates no device memory and keeps no pointer after a
 *     call returns (the one exception, a static per-device array loaded with the library,
 *     serves gm_render_loss_smooth_l1_noalloc).  Buffers must be 16-byte aligned (PyTorch
 *     allocations are).
 *   - Every call enqueues its kernels on `stream` (a hipStream_t; NULL = default stream)
 *     and returns without synchronising, except gm_bin (one synchronisation, see there).
 *   - Every call returns a gm_status.  Arguments are validated on the host before anything
 *     is enqueued; on error nothing is enqueued and gm_last_error() describes the problem.
 *     An asynchronous device fault surfaces as GM_ERR_HIP from a later call.
 *   - Gaussian parameters (Eq. 2-3), float32, row-major:
 *       mean[n][3]       centre in normalised world coordinates ([-1,1]^3 is the volume)
 *       quat[n][4]       rotation quaternion (w, x, y, z), unnormalised; normalised before
 *                        use (Sec. 3.2)
 *       log_scale[n][3]  log of the world-space standard deviations (S = diag(exp s))
 *       logit[n]         intensity alpha = 1 / (1 + exp(-logit)), so alpha is in [0, 1]
 *   - Voxel arrays are float32 [nz][ny][nx] (x fastest).  Voxel v of a grid sits at the
 *     integer index v of that grid's index frame.
 *   - Reentrant.  The only global state is the thread-local error string, and the static
 *     scratch array of gm_render_loss_smooth_l1_noalloc (see there: its calls race when
 *     they overlap on one GPU).
 */
#ifndef GM_H
#define GM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GM_ABI_VERSION 5
#define GM_MAX_GRIDS 8
#define GM_RECORD_FLOATS 16       /* floats per (grid, Gaussian) record                */
#define GM_GRID_GRAD_FLOATS 10    /* floats per (grid, Gaussian) backward partial      */
#define GM_REDUCE_WORKSPACE_BYTES 16384 /* workspace for the reductions below           */
#define GM_NOALLOC_MAX_TILES 131072     /* tiles gm_render_loss_smooth_l1_noalloc takes    */

typedef void* gm_stream; /* hipStream_t */

typedef enum gm_status {
    GM_OK = 0,
    GM_ERR_INVALID_ARGUMENT = 1, /* bad size, NULL or misaligned pointer, bad descriptor */
    GM_ERR_CAPACITY = 2,         /* pair buffer too small; *n_pairs holds the need        */
    GM_ERR_NONFINITE = 3,        /* NaN/Inf parameter, zero quaternion or exp overflow    */
    GM_ERR_HIP = 4,              /* HIP runtime error (launch failure, device fault)      */
    GM_ERR_UNSUPPORTED = 5
} gm_status;

/* Gaussian parameters (read only) and their gradients (accumulated with +=). */
typedef struct gm_gaussians {
    int64_t n;
    const float* mean;
    const float* quat;
    const float* log_scale;
    const float* logit;
} gm_gaussians;

typedef struct gm_gaussian_grads {
    int64_t n;
    float* mean;
    float* quat;
    float* log_scale;
    float* logit;
} gm_gaussian_grads;

/* [host] A voxel grid.  world_to_index is the row-major 3x4 affine [L | t] taking normalised
 * world coordinates to this grid's voxel indices; for a stack it folds in the stack's rigid
 * placement T_k (Sec. 3.3.2).  psf_sigma_z is the standard deviation, in index units along
 * index z (the slice normal), of the Gaussian slice profile the stack was acquired with;
 * 0 means point sampling (Eq. 7 exactly, used for the target volume). */
typedef struct gm_grid {
    int32_t nx, ny, nz, reserved;
    double world_to_index[12];
    double psf_sigma_z;
} gm_grid;

/* [host] Binning options.  cutoff_sigma: a Gaussian is evaluated on the voxels of the
 * axis-aligned box of +-cutoff_sigma marginal standard deviations around its centre in the
 * grid's index frame (3 = the 3-sigma box); it stands in for the paper's cell-neighbourhood
 * query (Sec. 3.3.1, Eq. 4-6). */
typedef struct gm_bin_opts {
    double cutoff_sigma;
    /* > 0: the paper's own query (Sec. 3.3.1, Eqs. 4-6) instead of the sigma box: [-1, 1]^3
     * is cut into cell_resolution^3 cells (Eq. 4, cell = floor((x + 1) res / 2) per axis, in
     * binary64) and voxel v takes Gaussian i when on every world axis the cell of v's world
     * position lies within block_radius of the cell of mu_i.  On an axis-aligned grid (each row
     * of L one non-zero entry, in distinct columns) a voxel's world coordinate along world axis
     * a is (v_j - t_j) / L[j][a] for the index axis j mapped to it, and the voxels form a box.
     * On any other grid (rotated stacks) it is ((m_a0 x + m_a1 y) + m_a2 z) + m_a3 with m the
     * index->world affine of gm_index_to_world (binary64, that association), the voxels do not
     * form a box: the record carries a box that contains them (from the block's world box,
     * widened by 1e-9 world and 1e-6 index units) and every kernel tests each voxel of it, and
     * the pair counts (box_volume, box_pairs) count that box.  The means' cells are clamped to
     * [-2^30, 2^30].  0: the sigma box. */
    int32_t block_radius;
    int32_t cell_resolution;
} gm_bin_opts;

/* Binning state: caller-allocated device buffers (sizes from gm_bin_query) plus host fields
 * that gm_bin fills in and later calls read.
 *   records     [n_grids][n_gauss][16] float: per (grid, Gaussian)
 *               c_rel(3) = centre - lo, amp, K(6) = -1/2 log2(e) x conic with the three
 *               off-diagonal terms doubled (xx, yy, zz, xy, xz, yz), lo(3), hi(3) (int32
 *               bit patterns, inclusive voxel box; lo > hi means empty)
 *   tile_count  [n_grids][n_gauss] int32: tiles the box overlaps
 *   box_volume  [n_grids] int64: sum of box volumes = contributing (Gaussian, voxel) pairs
 *   tile_start  [total_tiles + 1] int32: CSR row starts of the per-tile lists
 *   pair_gauss  [capacity_pairs] uint32: Gaussian ids (low 31 bits) grouped by tile,
 *               ascending per tile; bit 31 is set on the one entry of each (grid,
 *               Gaussian) whose tile holds the box's lower corner (its "home" tile)
 *   grid_grads  [n_grids][n_gauss][10] float: written by gm_backward / gm_grid_partials
 *               (grid-frame partials d amp, d c(3), d K(6))
 *   scratch     scratch_bytes of device memory for sorting; with the block query it also
 *               holds each Gaussian's cell, which the renders and the backward read on
 *               rotated grids until the next gm_bin                                       */
typedef struct gm_bins {
    int32_t n_grids;
    int32_t reserved;
    int64_t n_gauss;
    int64_t capacity_pairs;
    float* records;
    int32_t* tile_count;
    int64_t* box_volume;
    int32_t* tile_start;
    int32_t* pair_gauss;
    float* grid_grads;
    void* scratch;
    size_t scratch_bytes;
    /* [host] filled by gm_bin */
    gm_grid grids[GM_MAX_GRIDS];
    int64_t tile_base[GM_MAX_GRIDS + 1]; /* global tile id of each grid's first tile */
    int64_t n_pairs;                     /* (tile, Gaussian) pairs of the last gm_bin;
                                            set it < 0 when allocating: calls that read
                                            the tile lists refuse bins without them      */
    int64_t box_pairs[GM_MAX_GRIDS];     /* contributing (Gaussian, voxel) pairs per grid
                                            of the last gm_bin (= box_volume)            */
    int64_t list_start[GM_MAX_GRIDS + 1]; /* pair_gauss entries of grid k are
                                            [list_start[k], list_start[k + 1])           */
    double cutoff_sigma;
    int32_t block_radius;                /* the gm_bin_opts of the last gm_bin (0: sigma box) */
    int32_t cell_resolution;
} gm_bins;

/* Library identity. */
int32_t gm_abi_version(void);
/* Thread-local description of the last error; valid until the next gm_* call. */
const char* gm_last_error(void);
/* [host out] tile edge lengths (x, y, z) in voxels used by the binning. */
void gm_tile_dims(int32_t out_xyz[3]);

/* Sizes of the buffers a gm_bins needs for n Gaussians on the given grids with a pair
 * capacity of capacity_pairs.  All outputs [host]; any may be NULL. */
gm_status gm_bin_query(int64_t n, const gm_grid* grids, int32_t n_grids,
                       int64_t capacity_pairs, size_t* records_bytes,
                       int64_t* total_tiles, size_t* scratch_bytes);

/* Spatial query (stands in for Sec. 3.3.1): per (grid, Gaussian) compute the record and
 * the box, then list for every tile of every grid the Gaussians whose box overlaps it, in
 * ascending Gaussian id (a stable device radix sort of (tile, Gaussian) keys).
 * Waits once on the host for the pair total (an event recorded after the count; the pair
 * emission is already enqueued behind it); *n_pairs [host] receives it.
 * GM_ERR_CAPACITY if it exceeds bins->capacity_pairs (records, counts and box volumes are
 * still valid; lists are not).  GM_ERR_NONFINITE if any parameter is non-finite, a
 * quaternion is zero or exp(log_scale) overflows (those Gaussians get empty boxes; the
 * rest of the binning is complete and valid).  bins->n_grids / n_gauss / capacity_pairs /
 * buffers must be set by the caller; the host fields are filled in. */
gm_status gm_bin(const gm_gaussians* g, const gm_grid* grids, int32_t n_grids,
                 const gm_bin_opts* opts, gm_bins* bins, int64_t* n_pairs, gm_stream stream);

/* Forward rendering (Eq. 7 with the slice profile): for each listed grid (indices into the
 * binned grids) write out[k][v] = sum over Gaussians i whose box contains v of
 * amp_i exp(-1/2 (v - c_i)^T C_i (v - c_i)).  outs [host] array of n_ids device pointers,
 * each [nz][ny][nx].  Overwrites.  Bit-deterministic run to run. */
gm_status gm_render_stacks(const gm_bins* bins, const int32_t* grid_ids, int32_t n_ids,
                           float* const* outs, gm_stream stream);

/* Forward rendering fused with the smooth-L1 data term (Eq. 7 and Eq. 11, beta = 1): the
 * listed grids are rendered as by gm_render_stacks and, while each tile is still on chip,
 *   dl_di[k][v] = clamp(I_k[v] - targets[k][v], -1, 1) / N   (overwritten),
 *   *loss (device float) = (1/N) sum over every voxel of smoothL1(I_k[v] - targets[k][v]),
 * N = voxels of the listed grids; dl_di is bit-identical to gm_render_stacks followed by
 * gm_loss_smooth_l1, the loss equal up to the order of its FP64 sum.  outs may be NULL (the
 * rendered stacks are then not stored) or an array whose entries are NULL or [nz][ny][nx]
 * device buffers that receive the rendering.  targets / dl_di: [host] arrays of n_ids (>= 1)
 * device pointers to [nz][ny][nx] float32.  workspace: device bytes >= 8 x the tiles of the
 * listed grids (one FP64 partial per tile).  Bit-deterministic run to run. */
gm_status gm_render_loss_smooth_l1(const gm_bins* bins, const int32_t* grid_ids, int32_t n_ids,
                                   const float* const* targets, float* const* outs,
                                   float* const* dl_di, float* loss, void* workspace,
                                   size_t workspace_bytes, gm_stream stream);

/* gm_render_loss_smooth_l1 for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the per-tile FP64
 * partials go to a static array of the library, GM_NOALLOC_MAX_TILES doubles (1 MiB) on each
 * GPU the library runs on, held until the process ends, instead of a workspace argument.  Same
 * kernels, so the same results bit for bit.  The listed grids may hold at most
 * GM_NOALLOC_MAX_TILES tiles of the size gm_tile_dims reports (the three 256x256x64 stacks of a
 * 256^3 reconstruction hold 12288, five 320x320x80 stacks 40000); more is GM_ERR_CAPACITY and
 * nothing is enqueued.  The call allocates nothing; its first call on a device looks the
 * array's device address up (hipGetSymbolAddress) with that device current.  Every call on one
 * GPU shares that GPU's array: calls that may overlap on one GPU (two streams, two host
 * threads) race and must be ordered by the caller.  The array needs no clearing: every tile of
 * a call writes its partial before the final sum reads it. */
gm_status gm_render_loss_smooth_l1_noalloc(const gm_bins* bins, const int32_t* grid_ids,
                                           int32_t n_ids, const float* const* targets,
                                           float* const* outs, float* const* dl_di, float* loss,
                                           gm_stream stream);

/* Neural residual field parameters for the fused volume epilogue (Eq. 8).  Weights are
 * bf16 stored as uint16 bit patterns, row-major [out][in]; biases float32.
 * n_freq frequency bands: input features (x, sin(2^k pi x), cos(2^k pi x)), k < n_freq,
 * dimension 3 + 6 n_freq, zero-padded to in_pad: 64 (n_freq <= 8) or 128 (n_freq <= 20;
 * the kernels group the bands in fours, which is why 9 or 10 bands need in_pad 128 although
 * 3 + 6 n_freq <= 64).  Feature order: x_a at a, sin(2^k pi x_a) at 3 + 6 k + a, cos(2^k pi x_a)
 * at 6 + 6 k + a (a < 3); padded columns of w_in are ignored.  depth hidden layers of
 * width (SiLU), then a linear output; r = out_scale * tanh(output). */
typedef struct gm_nrf {
    int32_t n_freq, depth, width, in_pad;
    float out_scale;
    int32_t reserved;
    const uint16_t* w_in;    /* [width][in_pad]              */
    const float* b_in;       /* [width]                      */
    const uint16_t* w_hid;   /* [depth - 1][width][width]    */
    const float* b_hid;      /* [depth - 1][width]           */
    const uint16_t* w_out;   /* [width]                      */
    const float* b_out;      /* [1]                          */
} gm_nrf;

/* Inference (Sec. 3.1): render binned grid grid_id into out [nz][ny][nx]; when nrf is not
 * NULL add the residual r(x) at each voxel's world coordinate (Eq. 8, I_final = I + r) in the
 * same pass: each tile is rendered in LDS, the field is evaluated on its voxels with the
 * weights staged once per block, and the sum is stored once.  Bit-identical to the render
 * without the field followed by gm_nrf_forward on the same grid. */
gm_status gm_render_volume(const gm_bins* bins, int32_t grid_id, const gm_nrf* nrf,
                           float* out, gm_stream stream);

/* gm_render_loss_smooth_l1 with the residual field (Sec. 3.4, Eq. 8) added to every voxel of
 * the listed stacks before the data term (Eq. 11) is formed, all in one pass: the prediction is
 * I_k[v] + r(x_v) at the voxel's world coordinate x_v.  dl_di and the stored renderings (outs,
 * as there; they hold I + r) are bit-identical to gm_render_stacks, gm_nrf_forward on each
 * stack and gm_loss_smooth_l1, the loss equal up to the order of its FP64 sum.  dl_di is also dL/dr, the input gm_nrf_backward takes.  nrf must not be NULL;
 * other arguments as for gm_render_loss_smooth_l1. */
gm_status gm_render_nrf_loss_smooth_l1(const gm_bins* bins, const int32_t* grid_ids,
                                       int32_t n_ids, const gm_nrf* nrf,
                                       const float* const* targets, float* const* outs,
                                       float* const* dl_di, float* loss, void* workspace,
                                       size_t workspace_bytes, gm_stream stream);

/* [host out] The index->world affine (row-major 3x4, binary64) of a grid: the inverse of its
 * world_to_index.  The residual field encodes the world coordinate of voxel v as, per row a,
 * float32(((M[a][0] vx + M[a][1] vy) + M[a][2] vz) + M[a][3]) evaluated in binary64 without
 * contraction. */
gm_status gm_index_to_world(const gm_grid* grid, double out[12]);

/* Neural residual field forward (Sec. 3.4, Eq. 8) on every voxel of grid: out[v] += r(x_v).
 * Requires width 64, 1 <= depth <= 4, in_pad and n_freq as for gm_nrf.  MFMA BF16 x BF16 ->
 * FP32 for the layers; encoding, bias, SiLU and tanh in FP32, activations (the last layer's
 * too, which feeds the output layer) rounded to BF16. */
gm_status gm_nrf_forward(const gm_nrf* nrf, const gm_grid* grid, float* out, gm_stream stream);

/* Weight gradients (FP32) of the field, accumulated (+=); same shapes as gm_nrf's weights. */
typedef struct gm_nrf_grads {
    float* w_in;   /* [width][in_pad]           */
    float* b_in;   /* [width]                   */
    float* w_hid;  /* [depth - 1][width][width] */
    float* b_hid;  /* [depth - 1][width]        */
    float* w_out;  /* [width]                   */
    float* b_out;  /* [1]                       */
} gm_nrf_grads;

/* [host out] device workspace bytes gm_nrf_backward needs for n_points points. */
gm_status gm_nrf_workspace(const gm_nrf* nrf, int64_t n_points, size_t* bytes);

/* Backward of scale * sum_{k < n_points} dl_dr[v_k] r(x_{v_k}) over the voxels v_k = idx[k]
 * (linear indices into grid; idx NULL = every voxel in order, n_points then the grid's voxels
 * or 0) with respect to every weight
 * and bias of the field; accumulates into grads.  dl_dr is grid-sized [nz][ny][nx].  With a
 * random subset of n voxels and scale = (grid voxels) / n this is an unbiased estimate of the
 * full gradient (the paper trains on sampled points).  Recomputes the forward, writes the
 * per-layer dZ and activations in BF16 to the workspace, forms dA = W^T dZ and
 * dW = dZ A^T on MFMA (split over points, partial sums added in fixed order). */
gm_status gm_nrf_backward(const gm_nrf* nrf, const gm_grid* grid, const int32_t* idx,
                          int64_t n_points, const float* dl_dr, float scale,
                          gm_nrf_grads* grads, void* workspace, size_t workspace_bytes,
                          gm_stream stream);

/* [host out] device workspace bytes gm_nrf_backward_grids needs for n_grids point lists of
 * n_points[k] points (each rounded up to a multiple of 16 in the workspace). */
gm_status gm_nrf_workspace_grids(const gm_nrf* nrf, int32_t n_grids, const int64_t* n_points,
                                 size_t* bytes);

/* The backward of gm_nrf_backward summed over several grids in one pass: the gradient of
 * sum_k scales[k] sum_{j < n_points[k]} dl_dr[k][v_kj] r(x_{v_kj}), v_kj = idx[k][j] (idx[k]
 * NULL = every voxel of grids[k]), accumulated into grads.  Equal to the n_grids calls of
 * gm_nrf_backward up to the order of the FP32 sums: the chain kernel runs once per grid into
 * one workspace, then the weight-gradient GEMMs and their sums run once over all the points
 * (the paper's sampled training points of every stack, Sec. 3.4).  grids, idx, n_points,
 * dl_dr, scales: [host] arrays of n_grids (1 <= n_grids <= GM_MAX_GRIDS); idx[k] and dl_dr[k]
 * device pointers; other arguments and errors as for gm_nrf_backward, with workspace_bytes at
 * least what gm_nrf_workspace_grids gives. */
gm_status gm_nrf_backward_grids(const gm_nrf* nrf, int32_t n_grids, const gm_grid* grids,
                                const int32_t* const* idx, const int64_t* n_points,
                                const float* const* dl_dr, const float* scales,
                                gm_nrf_grads* grads, void* workspace, size_t workspace_bytes,
                                gm_stream stream);

/* out[i] = bfloat16(in[i]) (round to nearest even), as uint16 bit patterns. */
gm_status gm_f32_to_bf16(const float* in, uint16_t* out, int64_t n, gm_stream stream);

/* smooth-L1 data term (Eq. 11, beta = 1) averaged over every voxel of the listed stacks:
 * *loss (device float) = mean smoothL1(pred - target); dl_di[k][v] = clamp(pred - target,
 * -1, 1) / N_total (overwritten).  preds/targets/dl_di: [host] arrays of device pointers;
 * sizes [host] voxel counts.  workspace: GM_REDUCE_WORKSPACE_BYTES device bytes. */
gm_status gm_loss_smooth_l1(int32_t n_stacks, const float* const* preds,
                            const float* const* targets, const int64_t* sizes,
                            float* const* dl_di, float* loss, void* workspace,
                            gm_stream stream);

/* SSIM term of the reconstruction loss (Sec. 3.5.2, Eq. 10: L_recon = L_L1 + lambda_SSIM L_SSIM;
 * lambda_SSIM = 0.5 in Sec. 4.1.4).  The paper names the term without window or constants; read
 * as textbook SSIM on whole slices: every z-slice of stack k is a 2D image of nx x ny pixels,
 * 11 x 11 Gaussian window (sigma 1.5, normalised), zero padding outside the slice,
 * C1 = 0.01^2, C2 = 0.03^2 (intensities in [0, 1]).
 *   *loss (device float) = L_SSIM = 1 - mean of the SSIM map over every voxel of the listed
 *                          stacks (0 when they hold no voxel);
 *   dl_di[k][v] += lambda * dL_SSIM / d pred_k[v]  (accumulated, so that it adds onto the
 *                          smooth-L1 gradient written by gm_loss_smooth_l1).
 * preds/targets/dl_di: [host] arrays of device pointers to [nz][ny][nx] float32 stacks;
 * dims: [host] n_stacks x (nx, ny, nz), each >= 0.  Statistics and derivatives in FP64.
 * workspace: GM_REDUCE_WORKSPACE_BYTES device bytes.  Bit-reproducible run to run.  A stack
 * must not alias another's dl_di. */
gm_status gm_loss_ssim(int32_t n_stacks, const float* const* preds, const float* const* targets,
                       const int32_t* dims, float lambda, float* const* dl_di, float* loss,
                       void* workspace, gm_stream stream);

/* Anisotropy regulariser (Eq. 13, reading the ratio as exp(max s - min s), the ratio of the
 * actual scales): *value (device float) = mean_i max(0, exp(max s_i - min s_i) - lambda_r). */
gm_status gm_aniso_reg(const gm_gaussians* g, float lambda_r, float* value, void* workspace,
                       gm_stream stream);

/* Backward of sum_k sum_v dl_di[k][v] I_k[v] (+ lambda_aniso * aniso) with respect to every
 * Gaussian parameter, boxes held fixed (Sec. 3.5).  Recomputes each Gaussian's values
 * instead of storing per-voxel contributions.  Writes bins->grid_grads for the listed
 * grids, then ACCUMULATES (+=) into grad (caller zeroes it).  g must be the parameters
 * bins was built from, by a gm_bin that returned GM_OK or GM_ERR_NONFINITE (the tile lists
 * are walked to take the Gaussians in spatial order).  dl_di [host] array of n_ids device
 * pointers.  Bit-reproducible. */
gm_status gm_backward(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                      int32_t n_ids, const float* const* dl_di, float lambda_aniso,
                      float lambda_r, gm_gaussian_grads* grad, gm_stream stream);

/* First stage of gm_backward alone (Sec. 3.5): for every Gaussian and listed grid, the ten
 * sums over its box of the derivatives of sum_v dl_di[k][v] I_k[v] with respect to the
 * record's amplitude (1), centre (3) and the six distinct entries of its conic K as a
 * symmetric matrix (xx yy zz xy xz yz), written (overwritten) to
 * bins->grid_grads[grid][i][10] (a Gaussian whose box is empty on a grid has zeros there,
 * written by gm_bin).  Needs the tile lists, as gm_backward does.  These per-grid quantities
 * are also where an update of the stacks' rigid placements would start from. */
gm_status gm_grid_partials(const gm_gaussians* g, const gm_bins* bins,
                           const int32_t* grid_ids, int32_t n_ids, const float* const* dl_di,
                           gm_stream stream);

/* Second stage of gm_backward alone: pulls bins->grid_grads of the listed grids (as written
 * by gm_grid_partials for the same grid_ids) back to (mean, quat, log_scale, logit) in FP64,
 * sums over grids, adds lambda_aniso times the anisotropy gradient (Eq. 13) and ACCUMULATES
 * (+=) into grad.  gm_grid_partials followed by gm_chain is exactly gm_backward. */
gm_status gm_chain(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                   int32_t n_ids, float lambda_aniso, float lambda_r, gm_gaussian_grads* grad,
                   gm_stream stream);

/* Workspace gm_grid_pose_grads needs: GM_POSE_WORKSPACE_BYTES(n_ids) device bytes. */
#define GM_POSE_WORKSPACE_BYTES(n_ids) ((size_t)256 * (size_t)(n_ids) * 12 * sizeof(double))

/* Gradient with respect to each listed grid's world->index affine A = [L | t] (row-major
 * 3x4), boxes held fixed, of the objective whose per-voxel derivatives produced the grid-frame
 * partials in bins->grid_grads (a gm_backward or gm_grid_partials call on the same bins and
 * parameters): out[k][12] (device, binary64, overwritten) = dL/dA of grid grid_ids[k].
 * This is what the joint optimisation of the stacks' rigid transforms T_k (Sec. 3.3.2)
 * chains through: with A = A0 o T_k^-1, a rigid increment of T_k changes A linearly.
 *   c = L mu + t          -> dL/dL += d_c mu^T,  dL/dt += d_c
 *   Sigma_idx = L Sigma L^T -> dL/dL += 2 (dL/dSigma_idx) L Sigma
 * summed over the Gaussians with non-empty boxes, in FP64 and a fixed order (reproducible).
 * workspace: GM_POSE_WORKSPACE_BYTES(n_ids) device bytes. */
gm_status gm_grid_pose_grads(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                             int32_t n_ids, double* out, void* workspace, size_t workspace_bytes,
                             gm_stream stream);

/* Hyperparameters of the fused chain-rule + Adam step: one learning rate per parameter group
 * (Sec. 4.1.4; groups mean, quat, log_scale, logit in that order), shared betas and eps. */
typedef struct gm_adam_opts {
    double lr[4];
    double beta1, beta2, eps;
    int32_t step;  /* >= 1 */
} gm_adam_opts;

/* gm_chain into a zeroed gradient followed by gm_adam_step on each of the four parameter groups
 * (with opts->lr[0..3]), in one pass: each Gaussian's gradient is formed in FP64, rounded to
 * float as gm_chain stores it, and applied at once, so it never goes to memory.  The result is
 * bit-identical to that three-step sequence.  g's four parameter arrays are updated IN PLACE
 * (they must be writable device memory, whatever the const of gm_gaussians says) and must be
 * the parameters bins->grid_grads was computed for by gm_grid_partials with the same grid_ids;
 * m and v are the first and second moments, laid out as the parameters (device, updated in
 * place).  The Adam scalars are formed as gm_adam_step forms them. */
gm_status gm_chain_adam(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                        int32_t n_ids, float lambda_aniso, float lambda_r,
                        const gm_adam_opts* opts, gm_gaussian_grads* m, gm_gaussian_grads* v,
                        gm_stream stream);

/* Adam (Sec. 4.1.4; PyTorch arrangement, no weight decay) on n float32 elements in place:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= (lr / (1 - b1^step)) m / (sqrt(v) / sqrt(1 - b2^step) + eps).  step >= 1.
 * The scalars (1 - b1), (1 - b2), lr / (1 - b1^step) and sqrt(1 - b2^step) are formed in
 * double from the double hyperparameters and rounded once to float. */
gm_status gm_adam_step(float* param, const float* grad, float* m, float* v, int64_t n,
                       double lr, double beta1, double beta2, double eps, int32_t step,
                       gm_stream stream);

/* Devoxelization initialisation (Sec. 3.1; Fig. 1b): fill n = g^3 Gaussians (g >= 1) laid on
 * the cell centres of a uniform g^3 grid over [-1,1]^3 (Gaussian i = (iz g + iy) g + ix), with
 * identity rotation, isotropic log-scale ln(h/2) (h = 2/g) and intensity
 * alpha = clip(mean over the stacks containing the centre of the stack sampled trilinearly at
 * the centre, times 8 / (2 pi)^{3/2}, 1e-3, 1 - 1e-3) (the factor makes the lattice of
 * Gaussians sum back to the sampled intensity); logit = log(alpha / (1 - alpha)).
 * stacks [host] n_stacks descriptors; stack_data [host] array of device pointers [nz][ny][nx].
 * Outputs: mean [n][3], quat [n][4], log_scale [n][3], logit [n] (overwritten). */
gm_status gm_devox_init(int32_t g, const gm_grid* stacks, int32_t n_stacks,
                        const float* const* stack_data, float* mean, float* quat,
                        float* log_scale, float* logit, gm_stream stream);

/* Resolution transition of multi-resolution progressive training (Sec. 4.1.3): the Gaussians
 * of a g_old^3 lattice (Gaussian (ix, iy, iz) at index (iz g + iy) g + ix, as gm_devox_init lays
 * them out) are replaced by a g_new^3 lattice interpolated from them.  The paper names
 * trilinear interpolation for intensity and scale and normalised linear interpolation for the
 * rotation; readings: new Gaussians at the new cell centres; the old lattice sampled there in
 * its cell-index units, clamped to its centres; alpha = sigmoid(logit) and exp(log_scale)
 * interpolated, the scale multiplied by g_old / g_new (one cell per Gaussian, which keeps the
 * rendered intensity), alpha clipped to [1e-6, 1 - 1e-6]; quaternions normalised, aligned to
 * the hemisphere of the heaviest corner (the first of equal weights in (z, y, x) corner
 * order), summed with the weights and normalised.  Binary64 arithmetic.
 * old: device parameters of g_old^3 Gaussians (mean unused); outputs: device arrays for g_new^3
 * Gaussians ([n][3], [n][4], [n][3], [n]), overwritten, not aliasing the inputs. */
gm_status gm_upsample_lattice(int32_t g_old, const gm_gaussians* old, int32_t g_new,
                              float* mean, float* quat, float* log_scale, float* logit,
                              gm_stream stream);

/* ---- warm-start network ------------------------------------------------------------------
 * Predicts, for each Gaussian of a devoxelization initialisation, residuals of its log-scale,
 * rotation and intensity from a 3-channel 8^3 patch of the registered stacks around its centre
 * (initialisation stage of Sec. 3.1 / Fig. 1b, learned):
 *   conv 3->32 (3^3, stride 1, pad 1), SiLU        8^3
 *   conv 32->32 (3^3, stride 2, pad 1), SiLU       4^3
 *   conv 32->32 (3^3, stride 2, pad 1), SiLU       2^3
 *   conv 32->32 (2^3, valid), SiLU                 1
 *   linear 32->8  ->  (d log_scale 3, d quat 4, d logit 1)
 *   log_scale = s0 + d, quat = (1,0,0,0) + d, logit = logit0 + d.
 * Conv weights are BF16 [32][K_pad] with K = c*k^3 + (kz*k + ky)*k + kx, zero-padded to K_pad
 * = 96, 864, 864, 256; biases FP32 [32]; head FP32 wl [8][32], bl [8].  Batches n must be
 * multiples of 16.  Convolutions run on MFMA (BF16 x BF16 -> FP32). */
typedef struct gm_ws_net {
    const uint16_t* w[4];
    const float* b[4];
    const float* wl;
    const float* bl;
} gm_ws_net;
typedef struct gm_ws_grads { /* FP32, same shapes; accumulated (+=) */
    float* w[4];
    float* b[4];
    float* wl;
    float* bl;
} gm_ws_grads;

/* patches [n][3][8][8][8] BF16: channel k = stack k (n_stacks = 3) sampled trilinearly (zero
 * outside its index domain) at world points means[i] + ((x, y, z) - 3.5) * spacing. */
gm_status gm_ws_gather(const gm_grid* stacks, int32_t n_stacks, const float* const* stack_data,
                       const float* means, int64_t n, float spacing, uint16_t* patches,
                       gm_stream stream);
/* Training targets from a reconstruction's parameters: sigma_target[i] = the covariance
 * R(q_i/|q_i|) diag(e^{2 log_scale_i}) R^T (Eq. 3) as (xx, yy, zz, xy, xz, yz), FP64 inside,
 * rounded to float.  log_scale [n][3], quat [n][4]. */
gm_status gm_ws_targets(const float* log_scale, const float* quat, int64_t n,
                        float* sigma_target, gm_stream stream);
/* [host out] workspace bytes for a batch of n. */
gm_status gm_ws_workspace(int64_t n, size_t* bytes);
/* Inference: log_scale_out [n][3], quat_out [n][4], logit_out [n]. */
gm_status gm_ws_forward(const gm_ws_net* net, const uint16_t* patches, int64_t n,
                        const float* s0, const float* logit0, float* log_scale_out,
                        float* quat_out, float* logit_out, void* workspace,
                        size_t workspace_bytes, gm_stream stream);
/* Training step gradients: loss = mean_i |Sigma_i - Sigma*_i|_F^2 / |Sigma*_i|_F^2
 * + (logit_i - logit*_i)^2 with Sigma_i = R(q_i) diag(e^{2 s_i}) R(q_i)^T; sigma_target
 * [n][6] (xx, yy, zz, xy, xz, yz), logit_target [n]; *loss (device float); grads += . */
gm_status gm_ws_backward(const gm_ws_net* net, const uint16_t* patches, int64_t n,
                         const float* s0, const float* logit0, const float* sigma_target,
                         const float* logit_target, float* loss, gm_ws_grads* grads,
                         void* workspace, size_t workspace_bytes, gm_stream stream);

/* Mean squared error of vol against ref over n voxels into *mse (device float);
 * PSNR = 10 log10(1 / mse) for intensities in [0, 1] (Sec. 4.1.3). */
gm_status gm_mse(const float* vol, const float* ref, int64_t n, float* mse, void* workspace,
                 gm_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* GM_H */
