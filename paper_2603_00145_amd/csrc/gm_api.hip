// Host side of the C ABI declared in include/gm.h: argument validation, workspace layout,
// launch configuration and status codes.  Nothing here allocates device memory; the one
// library-held buffer is the static array behind gm_render_loss_smooth_l1_noalloc.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "gm_internal.h"

namespace {

thread_local std::string g_err;

gm_status fail(gm_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
gm_status fail(gm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

gm_status hip_fail(hipError_t e, const char* where)
{
    return fail(GM_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define GM_HIP(call, where)                                  \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, where);    \
    } while (0)

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

#define REQ_PTR(p, name)                                                                   \
    do {                                                                                   \
        if ((p) == nullptr) return fail(GM_ERR_INVALID_ARGUMENT, "%s is NULL", name);     \
        if (!aligned16(p)) return fail(GM_ERR_INVALID_ARGUMENT, "%s is not 16-byte aligned", name); \
    } while (0)

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

gm_status check_grid(const gm_grid& g, int k)
{
    if (g.nx <= 0 || g.ny <= 0 || g.nz <= 0 || g.nx > 32768 || g.ny > 32768 || g.nz > 32768)
        return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: dims (%d, %d, %d) outside [1, 32768]", k,
                    g.nx, g.ny, g.nz);
    if ((int64_t)g.nx * g.ny * g.nz >= 0x7fffffffLL)
        return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: more than 2^31 - 1 voxels", k);
    for (int i = 0; i < 12; ++i)
        if (!isfinite(g.world_to_index[i]))
            return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: non-finite world_to_index", k);
    if (!(g.psf_sigma_z >= 0.0) || !isfinite(g.psf_sigma_z))
        return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: psf_sigma_z must be finite and >= 0", k);
    const double* A = g.world_to_index;
    const double det = A[0] * (A[5] * A[10] - A[6] * A[9]) - A[1] * (A[4] * A[10] - A[6] * A[8]) +
                       A[2] * (A[4] * A[9] - A[5] * A[8]);
    if (!(fabs(det) > 0.0) || !isfinite(det))
        return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: world_to_index is singular", k);
    return GM_OK;
}

GridConst make_const(const gm_grid& g, int64_t tile_base)
{
    GridConst c;
    c.nx = g.nx;
    c.ny = g.ny;
    c.nz = g.nz;
    c.ntx = (int32_t)cdiv(g.nx, GM_TX);
    c.nty = (int32_t)cdiv(g.ny, GM_TY);
    c.ntz = (int32_t)cdiv(g.nz, GM_TZ);
    c.tile_base = tile_base;
    for (int r = 0; r < 3; ++r) {
        for (int j = 0; j < 3; ++j) c.L[3 * r + j] = g.world_to_index[4 * r + j];
        c.t[r] = g.world_to_index[4 * r + 3];
    }
    c.sig = g.psf_sigma_z;
    // world axis of each index axis when [L] is a scaled permutation
    bool aligned = true;
    for (int r = 0; r < 3; ++r) {
        int nzc = 0, col = -1;
        for (int j = 0; j < 3; ++j)
            if (c.L[3 * r + j] != 0.0) {
                ++nzc;
                col = j;
            }
        c.waxis[r] = nzc == 1 ? col : -1;
        aligned = aligned && nzc == 1;
    }
    if (!aligned || c.waxis[0] == c.waxis[1] || c.waxis[0] == c.waxis[2] || c.waxis[1] == c.waxis[2])
        c.waxis[0] = c.waxis[1] = c.waxis[2] = -1;
    return c;
}

int64_t grid_tiles(const gm_grid& g)
{
    return cdiv(g.nx, GM_TX) * cdiv(g.ny, GM_TY) * cdiv(g.nz, GM_TZ);
}

// scratch layout of gm_bins
struct BinScratch {
    int64_t* offsets;   // [n_grids * n + 1]
    void* scan_ws;
    uint32_t* keys0;
    uint32_t* keys1;
    uint32_t* vals0;
    void* radix_ws;
    BinReport* report;
    uint32_t* tile_box;  // [n_grids * n][3]
    int4* cells;         // [n]: the Gaussians' cells (block query)
    size_t bytes;
};

BinScratch scratch_layout(char* base, int64_t n, int32_t n_grids, int64_t cap)
{
    BinScratch s;
    size_t o = 0;
    const int64_t m = (int64_t)n_grids * n;
    auto take = [&](size_t b) { char* p = base ? base + o : nullptr; o += align256(b); return p; };
    s.offsets = reinterpret_cast<int64_t*>(take((size_t)(m + 1) * 8));
    s.scan_ws = take(scan_workspace_bytes(m));
    const int64_t c = cap > 0 ? cap : 1;
    s.keys0 = reinterpret_cast<uint32_t*>(take((size_t)c * 4));
    s.keys1 = reinterpret_cast<uint32_t*>(take((size_t)c * 4));
    s.vals0 = reinterpret_cast<uint32_t*>(take((size_t)c * 4));
    s.radix_ws = take(radix_workspace_bytes(c));
    s.report = reinterpret_cast<BinReport*>(take(sizeof(BinReport)));
    s.tile_box = reinterpret_cast<uint32_t*>(take((size_t)(m > 0 ? m : 1) * 12));
    s.cells = reinterpret_cast<int4*>(take((size_t)(n > 0 ? n : 1) * 16));
    s.bytes = o;
    return s;
}

gm_status check_gauss(const gm_gaussians* g)
{
    if (!g) return fail(GM_ERR_INVALID_ARGUMENT, "gaussians is NULL");
    if (g->n < 0 || g->n > 0x7fffffffLL)
        return fail(GM_ERR_INVALID_ARGUMENT, "n = %lld outside [0, 2^31)", (long long)g->n);
    if (g->n > 0) {
        REQ_PTR(g->mean, "mean");
        REQ_PTR(g->quat, "quat");
        REQ_PTR(g->log_scale, "log_scale");
        REQ_PTR(g->logit, "logit");
    }
    return GM_OK;
}

// The block query's state in the bins (the cells live in the binning scratch)
BlockQuery block_query(const gm_bins* b)
{
    BlockQuery q;
    q.cells = scratch_layout(reinterpret_cast<char*>(b->scratch), b->n_gauss, b->n_grids,
                             b->capacity_pairs).cells;
    q.res = (double)b->cell_resolution;
    q.radius = b->block_radius;
    return q;
}

gm_status check_bins(const gm_bins* b, bool need_lists)
{
    if (!b) return fail(GM_ERR_INVALID_ARGUMENT, "bins is NULL");
    if (b->n_grids < 1 || b->n_grids > GM_MAX_GRIDS)
        return fail(GM_ERR_INVALID_ARGUMENT, "bins->n_grids = %d outside [1, %d]", b->n_grids,
                    GM_MAX_GRIDS);
    if (need_lists && (b->n_pairs < 0 || b->n_pairs > b->capacity_pairs))
        return fail(GM_ERR_INVALID_ARGUMENT,
                    "bins hold no valid tile lists (last gm_bin needed %lld pairs, capacity %lld)",
                    (long long)b->n_pairs, (long long)b->capacity_pairs);
    return GM_OK;
}

// The block query on a grid that is not axis-aligned: its kernels test every voxel
bool grid_masked(const gm_bins* b, int id)
{
    return b->block_radius > 0 && make_const(b->grids[id], 0).waxis[0] < 0;
}

gm_status check_ids(const gm_bins* b, const int32_t* ids, int32_t n_ids)
{
    if (n_ids < 0 || n_ids > GM_MAX_GRIDS)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_ids = %d outside [0, %d]", n_ids, GM_MAX_GRIDS);
    if (n_ids > 0 && !ids) return fail(GM_ERR_INVALID_ARGUMENT, "grid_ids is NULL");
    for (int k = 0; k < n_ids; ++k) {
        if (ids[k] < 0 || ids[k] >= b->n_grids)
            return fail(GM_ERR_INVALID_ARGUMENT, "grid id %d outside [0, %d)", ids[k], b->n_grids);
        for (int j = 0; j < k; ++j)
            if (ids[j] == ids[k])
                return fail(GM_ERR_INVALID_ARGUMENT, "grid id %d listed twice", ids[k]);
    }
    return GM_OK;
}

bool index_to_world(const gm_grid& g, double* M)
{
    const double* A = g.world_to_index;
    const double a = A[0], b = A[1], c = A[2], d = A[4], e = A[5], f = A[6], h = A[8], i = A[9],
                 j = A[10];
    const double c00 = e * j - f * i, c01 = f * h - d * j, c02 = d * i - e * h;
    const double det = a * c00 + b * c01 + c * c02;
    if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
    const double L[9] = {c00 / det, (c * i - b * j) / det, (b * f - c * e) / det,
                         c01 / det, (a * j - c * h) / det, (c * d - a * f) / det,
                         c02 / det, (b * h - a * i) / det, (a * e - b * d) / det};
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) M[4 * r + k] = L[3 * r + k];
        M[4 * r + 3] = -(L[3 * r] * A[3] + L[3 * r + 1] * A[7] + L[3 * r + 2] * A[11]);
    }
    return true;
}

gm_status check_nrf(const gm_nrf* n)
{
    if (!n) return fail(GM_ERR_INVALID_ARGUMENT, "nrf is NULL");
    if (n->width != 64) return fail(GM_ERR_UNSUPPORTED, "nrf width must be 64");
    if (n->depth < 1 || n->depth > 4) return fail(GM_ERR_UNSUPPORTED, "nrf depth outside [1, 4]");
    if (n->in_pad != 64 && n->in_pad != 128)
        return fail(GM_ERR_UNSUPPORTED, "nrf in_pad must be 64 or 128");
    if (n->n_freq < 0 || n->n_freq > nrf_max_bands(n->in_pad))
        return fail(GM_ERR_INVALID_ARGUMENT,
                    "nrf n_freq outside [0, 8] (in_pad 64) or [0, 20] (in_pad 128)");
    if (!isfinite(n->out_scale)) return fail(GM_ERR_INVALID_ARGUMENT, "nrf out_scale not finite");
    if (!n->w_in || !n->b_in || !n->w_out || !n->b_out || (n->depth > 1 && (!n->w_hid || !n->b_hid)))
        return fail(GM_ERR_INVALID_ARGUMENT, "nrf weight pointer is NULL");
    if (((uintptr_t)n->w_in & 7u) || (n->w_hid && ((uintptr_t)n->w_hid & 7u)))
        return fail(GM_ERR_INVALID_ARGUMENT, "nrf weights must be 8-byte aligned");
    return GM_OK;
}

NrfArgs nrf_args(const gm_nrf* n, const gm_grid& g, const double* M)
{
    NrfArgs a;
    memset(&a, 0, sizeof a);
    a.n_freq = n->n_freq;
    a.depth = n->depth;
    a.in_pad = n->in_pad;
    a.out_scale = n->out_scale;
    a.w_in = n->w_in;
    a.b_in = n->b_in;
    a.w_hid = n->w_hid;
    a.b_hid = n->b_hid;
    a.w_out = n->w_out;
    a.b_out = n->b_out;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    for (int k = 0; k < 12; ++k) a.m[k] = M[k];
    return a;
}

struct NrfLayout {
    size_t bytes;
    size_t off_dzo, off_dz[4], off_a[5], off_part;
    int64_t P;
};

NrfLayout nrf_layout(const gm_nrf* n, int64_t npts)
{
    NrfLayout L;
    memset(&L, 0, sizeof L);
    L.P = ((npts + 15) / 16) * 16;
    size_t o = 0;
    auto take = [&](size_t b) { const size_t r = o; o += align256(b); return r; };
    L.off_dzo = take((size_t)L.P * 4);
    for (int l = 0; l < n->depth; ++l) L.off_dz[l] = take((size_t)64 * L.P * 2);
    L.off_a[0] = take((size_t)n->in_pad * L.P * 2);
    for (int l = 1; l <= n->depth; ++l) L.off_a[l] = take((size_t)64 * L.P * 2);
    L.off_part = take(nrf_part_floats(L.P, n->in_pad) * 4);
    L.bytes = o;
    return L;
}

struct WsLayout {
    size_t bytes, off_z[4], off_a[4], off_dz[4], off_part, off_loss, off_dout, off_a4;
};

WsLayout ws_layout(int64_t B)
{
    static const int PO[4] = {512, 64, 8, 1};
    WsLayout L;
    memset(&L, 0, sizeof L);
    size_t o = 0;
    auto take = [&](size_t b) { const size_t r = o; o += align256(b); return r; };
    for (int l = 0; l < 4; ++l) {
        L.off_z[l] = take((size_t)B * 32 * PO[l] * 4);
        L.off_a[l] = take((size_t)B * 32 * PO[l] * 2);
        L.off_dz[l] = take((size_t)B * 32 * PO[l] * 2);
    }
    L.off_part = take(ws_part_floats(B) * 4);
    L.off_loss = take((size_t)B * 4);
    L.off_dout = take((size_t)B * 8 * 4);
    L.off_a4 = take((size_t)B * 32 * 4);
    L.bytes = o;
    return L;
}

gm_status check_ws_net(const gm_ws_net* n)
{
    if (!n) return fail(GM_ERR_INVALID_ARGUMENT, "net is NULL");
    for (int l = 0; l < 4; ++l) {
        if (!n->w[l] || !n->b[l] || ((uintptr_t)n->w[l] & 7u))
            return fail(GM_ERR_INVALID_ARGUMENT, "conv %d weights NULL or not 8-byte aligned", l + 1);
    }
    if (!n->wl || !n->bl) return fail(GM_ERR_INVALID_ARGUMENT, "head weights NULL");
    return GM_OK;
}

WsNet ws_net(const gm_ws_net* n)
{
    WsNet w;
    for (int l = 0; l < 4; ++l) {
        w.w[l] = n->w[l];
        w.b[l] = n->b[l];
    }
    w.wl = n->wl;
    w.bl = n->bl;
    return w;
}

WsActs ws_acts(char* base, const WsLayout& L)
{
    WsActs w;
    for (int l = 0; l < 4; ++l) {
        w.z[l] = reinterpret_cast<float*>(base + L.off_z[l]);
        w.a[l] = reinterpret_cast<uint16_t*>(base + L.off_a[l]);
        w.dz[l] = reinterpret_cast<uint16_t*>(base + L.off_dz[l]);
    }
    w.part = reinterpret_cast<float*>(base + L.off_part);
    return w;
}

}  // namespace

extern "C" {

int32_t gm_abi_version(void) { return GM_ABI_VERSION; }

const char* gm_last_error(void) { return g_err.c_str(); }

void gm_tile_dims(int32_t out_xyz[3])
{
    if (!out_xyz) return;
    out_xyz[0] = GM_TX;
    out_xyz[1] = GM_TY;
    out_xyz[2] = GM_TZ;
}

gm_status gm_bin_query(int64_t n, const gm_grid* grids, int32_t n_grids, int64_t capacity_pairs,
                       size_t* records_bytes, int64_t* total_tiles, size_t* scratch_bytes)
{
    g_err.clear();
    if (n < 0 || n > 0x7fffffffLL) return fail(GM_ERR_INVALID_ARGUMENT, "n outside [0, 2^31)");
    if (n_grids < 1 || n_grids > GM_MAX_GRIDS || !grids)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_grids must be in [1, %d] with grids != NULL",
                    GM_MAX_GRIDS);
    if (capacity_pairs < 0 || capacity_pairs > 0x7fffffffLL)
        return fail(GM_ERR_INVALID_ARGUMENT, "capacity_pairs outside [0, 2^31)");
    int64_t T = 0;
    for (int k = 0; k < n_grids; ++k) {
        gm_status st = check_grid(grids[k], k);
        if (st != GM_OK) return st;
        T += grid_tiles(grids[k]);
    }
    if (T >= 0x7fffffffLL) return fail(GM_ERR_INVALID_ARGUMENT, "too many tiles");
    if (records_bytes) *records_bytes = (size_t)n_grids * (size_t)n * 16 * sizeof(float);
    if (total_tiles) *total_tiles = T;
    if (scratch_bytes) *scratch_bytes = scratch_layout(nullptr, n, n_grids, capacity_pairs).bytes;
    return GM_OK;
}

gm_status gm_bin(const gm_gaussians* g, const gm_grid* grids, int32_t n_grids,
                 const gm_bin_opts* opts, gm_bins* bins, int64_t* n_pairs, gm_stream stream)
{
    g_err.clear();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    gm_status st = check_gauss(g);
    if (st != GM_OK) return st;
    if (!bins || !n_pairs) return fail(GM_ERR_INVALID_ARGUMENT, "bins / n_pairs is NULL");
    int64_t T = 0;
    size_t need_scratch = 0;
    st = gm_bin_query(g->n, grids, n_grids, bins->capacity_pairs, nullptr, &T, &need_scratch);
    if (st != GM_OK) return st;
    if (bins->n_grids != n_grids || bins->n_gauss != g->n)
        return fail(GM_ERR_INVALID_ARGUMENT, "bins sized for %d grids x %lld Gaussians, got %d x %lld",
                    bins->n_grids, (long long)bins->n_gauss, n_grids, (long long)g->n);
    const double cutoff = opts ? opts->cutoff_sigma : 3.0;
    if (!(cutoff > 0.0) || !isfinite(cutoff))
        return fail(GM_ERR_INVALID_ARGUMENT, "cutoff_sigma must be finite and > 0");
    const int32_t block_radius = opts ? opts->block_radius : 0;
    const int32_t cell_res = opts ? opts->cell_resolution : 0;
    if (block_radius < 0 || (block_radius > 0 && (cell_res < 1 || cell_res > (1 << 20))))
        return fail(GM_ERR_INVALID_ARGUMENT, "block query needs block_radius >= 0 and "
                                             "cell_resolution in [1, 2^20]");
    REQ_PTR(bins->tile_start, "bins->tile_start");
    REQ_PTR(bins->box_volume, "bins->box_volume");
    REQ_PTR(bins->scratch, "bins->scratch");
    if (g->n > 0) {
        REQ_PTR(bins->records, "bins->records");
        REQ_PTR(bins->tile_count, "bins->tile_count");
    }
    if (bins->capacity_pairs > 0) REQ_PTR(bins->pair_gauss, "bins->pair_gauss");
    if (bins->scratch_bytes < need_scratch)
        return fail(GM_ERR_INVALID_ARGUMENT, "scratch_bytes %zu < required %zu",
                    bins->scratch_bytes, need_scratch);

    // host fields
    int64_t base = 0;
    PreprocessArgs pa;
    memset(&pa, 0, sizeof pa);
    for (int k = 0; k < n_grids; ++k) {
        bins->grids[k] = grids[k];
        bins->tile_base[k] = base;
        pa.g[k] = make_const(grids[k], base);
        base += grid_tiles(grids[k]);
    }
    bins->tile_base[n_grids] = base;
    bins->cutoff_sigma = cutoff;
    bins->block_radius = block_radius;
    bins->cell_resolution = block_radius > 0 ? cell_res : 0;
    bins->n_pairs = -1;

    const int64_t n = g->n;
    const int64_t m = (int64_t)n_grids * n;
    BinScratch sc = scratch_layout(reinterpret_cast<char*>(bins->scratch), n, n_grids,
                                   bins->capacity_pairs);
    static_assert(sizeof(BinReport) % 4 == 0, "report block is cleared as u32 words");
    GM_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(sc.report), 0u, sizeof(BinReport) / 4, s),
           "clear report");
    pa.n = n;
    pa.n_grids = n_grids;
    pa.cutoff = cutoff;
    pa.block_radius = block_radius;
    pa.cell_res = cell_res;
    pa.cells = sc.cells;
    pa.mean = g->mean;
    pa.quat = g->quat;
    pa.log_scale = g->log_scale;
    pa.logit = g->logit;
    pa.records = bins->records;
    pa.tile_count = bins->tile_count;
    pa.box_volume = sc.report->box_volume;
    pa.flags = sc.report->flags;
    pa.grid_grads = bins->grid_grads;
    pa.tile_box = sc.tile_box;
    GM_HIP(launch_preprocess(pa, s), "preprocess");
    GM_HIP(launch_scan_i32_to_i64(bins->tile_count, sc.offsets, m, sc.scan_ws, s), "scan");

    // the report lands in a pinned host block of this thread (allocated once, kept for the
    // life of the process), written by the report kernel itself
    static thread_local BinReport* t_report = nullptr;
    if (!t_report) {
        void* hp = nullptr;
        GM_HIP(hipHostMalloc(&hp, sizeof(BinReport), hipHostMallocDefault), "pinned report block");
        t_report = static_cast<BinReport*>(hp);
    }
    GM_HIP(launch_bin_report(sc.report, sc.offsets, n, bins->box_volume, n_grids, t_report, s),
           "report");
    // The host waits for the report only (an event after it, one per device and thread); the
    // pair emission is enqueued first, sized by the Gaussians and guarded by the capacity on
    // the device, so that the GPU emits while the host wakes up.
    static thread_local hipEvent_t t_done[64] = {};
    int dev = 0;
    if (s) {
        hipDevice_t sd = 0;
        GM_HIP(hipStreamGetDevice(s, &sd), "stream device");
        dev = (int)sd;
    } else {
        GM_HIP(hipGetDevice(&dev), "current device");
    }
    if (dev < 0 || dev >= 64) return fail(GM_ERR_UNSUPPORTED, "device index %d >= 64", dev);
    if (!t_done[dev]) {
        // the event belongs to the stream's device: create it with that device current
        int cur = 0;
        GM_HIP(hipGetDevice(&cur), "current device");
        if (cur != dev) GM_HIP(hipSetDevice(dev), "select stream device");
        const hipError_t ce = hipEventCreateWithFlags(&t_done[dev], hipEventDisableTiming);
        if (cur != dev) GM_HIP(hipSetDevice(cur), "restore device");
        GM_HIP(ce, "report event");
    }
    GM_HIP(hipEventRecord(t_done[dev], s), "record report event");

    int bits = 0;
    while ((int64_t(1) << bits) < T) ++bits;
    const int passes = (bits + 7) / 8;
    uint32_t* pg = reinterpret_cast<uint32_t*>(bins->pair_gauss);
    // arrange the ping-pong buffers so the last pass lands in pair_gauss
    uint32_t *k_in = sc.keys0, *k_alt = sc.keys1;
    uint32_t *v_in = (passes & 1) ? sc.vals0 : pg, *v_alt = (passes & 1) ? pg : sc.vals0;
    {
        EmitArgs ea;
        memset(&ea, 0, sizeof ea);
        ea.n = n;
        ea.n_grids = n_grids;
        ea.tile_box = sc.tile_box;
        ea.offsets = sc.offsets;
        ea.capacity = bins->capacity_pairs;
        ea.keys = k_in;
        ea.vals = v_in;
        for (int k = 0; k < n_grids; ++k) ea.g[k] = pa.g[k];
        GM_HIP(launch_emit(ea, s), "emit");
    }
    GM_HIP(hipEventSynchronize(t_done[dev]), "synchronise");
    const BinReport rep = *t_report;
    const int64_t total = rep.grid_start[n_grids];
    const uint32_t flags = rep.flags[0];
    *n_pairs = total;
    bins->n_pairs = total;
    for (int k = 0; k < GM_MAX_GRIDS; ++k) bins->box_pairs[k] = k < n_grids ? (int64_t)rep.box_volume[k] : 0;
    for (int k = 0; k <= GM_MAX_GRIDS; ++k)
        bins->list_start[k] = rep.grid_start[k < n_grids ? k : n_grids];
    if (total > bins->capacity_pairs) {
        fail(GM_ERR_CAPACITY, "%lld (tile, Gaussian) pairs exceed capacity %lld", (long long)total,
             (long long)bins->capacity_pairs);
        return GM_ERR_CAPACITY;
    }

    if (total > 0) {
        int in_alt = 0;
        GM_HIP(launch_radix_sort(k_in, v_in, k_alt, v_alt, total, bits, sc.radix_ws, &in_alt, s),
               "radix sort");
        GM_HIP(launch_tile_ranges(in_alt ? k_alt : k_in, total, bins->tile_start, T, s),
               "tile ranges");
    } else {
        GM_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(bins->tile_start), 0u, T + 1, s),
               "zero tile starts");
    }
    if (flags & 1u)
        return fail(GM_ERR_NONFINITE,
                    "non-finite parameter, zero quaternion or overflowing scale (empty boxes)");
    if (flags & 2u)
        return fail(GM_ERR_UNSUPPORTED, "a block-query box did not settle (grid scale too extreme)");
    return GM_OK;
}

// The loss fields (targets, dl, loss) are NULL for a plain render; with them the render also
// writes the smooth-L1 gradient and loss, and outs (the array or an entry) may be NULL.
struct RenderLoss {
    const float* const* targets;
    float* const* dl;
    float* loss;
    void* ws;
    size_t ws_bytes;
};

// nrf (optional): add the residual field to every rendered voxel in the same pass.
static gm_status render_impl(const gm_bins* bins, const int32_t* ids, int32_t n_ids,
                             float* const* outs, const RenderLoss* lo, hipStream_t s,
                             const gm_nrf* nrf = nullptr)
{
    if (nrf) {
        gm_status sn = check_nrf(nrf);
        if (sn != GM_OK) return sn;
    }
    gm_status st = check_bins(bins, true);
    if (st != GM_OK) return st;
    st = check_ids(bins, ids, n_ids);
    if (st != GM_OK) return st;
    if (n_ids > 0 && !outs && !lo) return fail(GM_ERR_INVALID_ARGUMENT, "outs is NULL");
    if (lo) {
        if (n_ids < 1) return fail(GM_ERR_INVALID_ARGUMENT, "n_ids must be >= 1");
        if (!lo->targets || !lo->dl) return fail(GM_ERR_INVALID_ARGUMENT, "NULL array argument");
        REQ_PTR(lo->loss, "loss");
    }
    RenderArgs ra;
    memset(&ra, 0, sizeof ra);
    int64_t blocks = 0, voxels = 0;
    for (int k = 0; k < n_ids; ++k) {
        const gm_grid& g = bins->grids[ids[k]];
        if (lo) {
            if (grid_tiles(g) > 0) {
                REQ_PTR(lo->targets[k], "targets[k]");
                REQ_PTR(lo->dl[k], "dl_di[k]");
            }
            ra.rg[k].target = lo->targets[k];
            ra.rg[k].dl = lo->dl[k];
            voxels += (int64_t)g.nx * g.ny * g.nz;
        } else {
            REQ_PTR(outs[k], "outs[k]");
        }
        RenderGrid& r = ra.rg[k];
        r.nx = g.nx;
        r.ny = g.ny;
        r.nz = g.nz;
        r.ntx = (int32_t)cdiv(g.nx, GM_TX);
        r.nty = (int32_t)cdiv(g.ny, GM_TY);
        r.ntz = (int32_t)cdiv(g.nz, GM_TZ);
        r.grid_index = ids[k];
        r.first_block = (int32_t)blocks;
        r.bin_tile_base = bins->tile_base[ids[k]];
        r.out = outs ? outs[k] : nullptr;
        r.masked = grid_masked(bins, ids[k]) ? 1 : 0;
        if ((nrf || r.masked) && !index_to_world(g, r.index_to_world))
            return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: singular affine", ids[k]);
        if (r.masked && !ra.bq.cells) {
            REQ_PTR(bins->scratch, "bins->scratch");
            ra.bq = block_query(bins);
        }
        blocks += grid_tiles(g);
    }
    if (blocks >= 0x7fffffffLL) return fail(GM_ERR_INVALID_ARGUMENT, "too many tiles");
    if (lo) {
        if (lo->ws_bytes < (size_t)blocks * sizeof(double))
            return fail(GM_ERR_INVALID_ARGUMENT, "workspace_bytes %zu < %lld (8 per tile)",
                        lo->ws_bytes, (long long)blocks * (long long)sizeof(double));
        if (blocks > 0) REQ_PTR(lo->ws, "workspace");
        ra.loss_part = reinterpret_cast<double*>(lo->ws);
        ra.loss = lo->loss;
        ra.inv_n = voxels > 0 ? 1.0 / (double)voxels : 0.0;
        if (blocks == 0) {
            GM_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(lo->loss), 0u, 1, s), "zero loss");
            return GM_OK;
        }
    }
    if (blocks == 0) return GM_OK;
    if (bins->n_gauss > 0) REQ_PTR(bins->records, "bins->records");
    REQ_PTR(bins->tile_start, "bins->tile_start");
    ra.n_render = n_ids;
    ra.total_blocks = (int32_t)blocks;
    ra.n_gauss = bins->n_gauss;
    ra.records = bins->records;
    ra.tile_start = bins->tile_start;
    ra.pair_gauss = bins->pair_gauss;
    if (nrf) {
        const NrfArgs f = nrf_args(nrf, bins->grids[ids[0]], ra.rg[0].index_to_world);
        GM_HIP(launch_render_field(ra, f, s), "render + field");
    } else {
        GM_HIP(launch_render(ra, s), "render");
    }
    return GM_OK;
}

gm_status gm_render_stacks(const gm_bins* bins, const int32_t* grid_ids, int32_t n_ids,
                           float* const* outs, gm_stream stream)
{
    g_err.clear();
    return render_impl(bins, grid_ids, n_ids, outs, nullptr, reinterpret_cast<hipStream_t>(stream));
}

gm_status gm_render_loss_smooth_l1(const gm_bins* bins, const int32_t* grid_ids, int32_t n_ids,
                                   const float* const* targets, float* const* outs,
                                   float* const* dl_di, float* loss, void* workspace,
                                   size_t workspace_bytes, gm_stream stream)
{
    g_err.clear();
    const RenderLoss lo{targets, dl_di, loss, workspace, workspace_bytes};
    return render_impl(bins, grid_ids, n_ids, outs, &lo, reinterpret_cast<hipStream_t>(stream));
}

// Per-tile FP64 loss partials of gm_render_loss_smooth_l1_noalloc.  Each GPU the library runs
// on holds its own copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name is not a device address
// in host code).
static __device__ __align__(256) double scratch[GM_NOALLOC_MAX_TILES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
}  // namespace

// The scratch array's address on the current device, looked up once per device.
static gm_status scratch_for_current_device(void** ptr)
{
    int dev = -1;
    GM_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(GM_ERR_UNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        GM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(GM_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return GM_OK;
}

gm_status gm_render_loss_smooth_l1_noalloc(const gm_bins* bins, const int32_t* grid_ids,
                                           int32_t n_ids, const float* const* targets,
                                           float* const* outs, float* const* dl_di, float* loss,
                                           gm_stream stream)
{
    g_err.clear();
    // the tile count is checked here, before the lookup, so that an oversized call fails with
    // a clear message; render_impl checks the buffer size again against the same figure
    gm_status st = check_bins(bins, true);
    if (st != GM_OK) return st;
    st = check_ids(bins, grid_ids, n_ids);
    if (st != GM_OK) return st;
    int64_t tiles = 0;
    for (int k = 0; k < n_ids; ++k) tiles += grid_tiles(bins->grids[grid_ids[k]]);
    if (tiles > GM_NOALLOC_MAX_TILES)
        return fail(GM_ERR_CAPACITY, "%lld tiles exceed the %d the static scratch holds",
                    (long long)tiles, GM_NOALLOC_MAX_TILES);
    void* ws = nullptr;
    st = scratch_for_current_device(&ws);
    if (st != GM_OK) return st;
    const RenderLoss lo{targets, dl_di, loss, ws, (size_t)GM_NOALLOC_MAX_TILES * sizeof(double)};
    return render_impl(bins, grid_ids, n_ids, outs, &lo, reinterpret_cast<hipStream_t>(stream));
}

gm_status gm_render_volume(const gm_bins* bins, int32_t grid_id, const gm_nrf* nrf, float* out,
                           gm_stream stream)
{
    g_err.clear();
    float* outs[1] = {out};
    return render_impl(bins, &grid_id, 1, outs, nullptr, reinterpret_cast<hipStream_t>(stream),
                       nrf);
}

gm_status gm_render_nrf_loss_smooth_l1(const gm_bins* bins, const int32_t* grid_ids,
                                       int32_t n_ids, const gm_nrf* nrf,
                                       const float* const* targets, float* const* outs,
                                       float* const* dl_di, float* loss, void* workspace,
                                       size_t workspace_bytes, gm_stream stream)
{
    g_err.clear();
    if (!nrf) return fail(GM_ERR_INVALID_ARGUMENT, "nrf is NULL");
    const RenderLoss lo{targets, dl_di, loss, workspace, workspace_bytes};
    return render_impl(bins, grid_ids, n_ids, outs, &lo, reinterpret_cast<hipStream_t>(stream),
                       nrf);
}

gm_status gm_index_to_world(const gm_grid* grid, double out[12])
{
    g_err.clear();
    if (!grid || !out) return fail(GM_ERR_INVALID_ARGUMENT, "NULL argument");
    gm_status st = check_grid(*grid, 0);
    if (st != GM_OK) return st;
    if (!index_to_world(*grid, out)) return fail(GM_ERR_INVALID_ARGUMENT, "singular grid affine");
    return GM_OK;
}

gm_status gm_nrf_forward(const gm_nrf* nrf, const gm_grid* grid, float* out, gm_stream stream)
{
    g_err.clear();
    gm_status st = check_nrf(nrf);
    if (st != GM_OK) return st;
    if (!grid) return fail(GM_ERR_INVALID_ARGUMENT, "grid is NULL");
    st = check_grid(*grid, 0);
    if (st != GM_OK) return st;
    REQ_PTR(out, "out");
    double M[12];
    if (!index_to_world(*grid, M)) return fail(GM_ERR_INVALID_ARGUMENT, "singular grid affine");
    NrfArgs a = nrf_args(nrf, *grid, M);
    a.n_points = (int64_t)grid->nx * grid->ny * grid->nz;
    a.out = out;
    GM_HIP(launch_nrf_forward(a, reinterpret_cast<hipStream_t>(stream)), "nrf forward");
    return GM_OK;
}

gm_status gm_nrf_workspace(const gm_nrf* nrf, int64_t n_points, size_t* bytes)
{
    g_err.clear();
    gm_status st = check_nrf(nrf);
    if (st != GM_OK) return st;
    if (n_points < 0 || n_points > 0x7fffffffLL || !bytes)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_points outside [0, 2^31) or bytes NULL");
    *bytes = nrf_layout(nrf, n_points).bytes;
    return GM_OK;
}

namespace {

// the workspace views of a layout over P points
NrfWork nrf_work(const gm_nrf* nrf, const NrfLayout& L, void* workspace)
{
    char* base = reinterpret_cast<char*>(workspace);
    NrfWork w;
    memset(&w, 0, sizeof w);
    w.P = L.P;
    w.dzo = reinterpret_cast<float*>(base + L.off_dzo);
    for (int l = 0; l < nrf->depth; ++l) w.dz[l] = reinterpret_cast<uint16_t*>(base + L.off_dz[l]);
    for (int l = 0; l <= nrf->depth; ++l) w.a[l] = reinterpret_cast<uint16_t*>(base + L.off_a[l]);
    w.part = reinterpret_cast<float*>(base + L.off_part);
    return w;
}

gm_status check_nrf_grads(const gm_nrf* nrf, const gm_nrf_grads* grads)
{
    if (!grads) return fail(GM_ERR_INVALID_ARGUMENT, "grads is NULL");
    REQ_PTR(grads->w_in, "grads->w_in");
    REQ_PTR(grads->b_in, "grads->b_in");
    REQ_PTR(grads->w_out, "grads->w_out");
    REQ_PTR(grads->b_out, "grads->b_out");
    if (nrf->depth > 1) {
        REQ_PTR(grads->w_hid, "grads->w_hid");
        REQ_PTR(grads->b_hid, "grads->b_hid");
    }
    return GM_OK;
}

// one grid's point list of a backward call, checked
gm_status nrf_backward_grid(const gm_nrf* nrf, int k, const gm_grid& grid, const int32_t* idx,
                            int64_t n_points, const float* dl_dr, float scale,
                            const gm_nrf_grads* grads, NrfArgs* out)
{
    gm_status st = check_grid(grid, k);
    if (st != GM_OK) return st;
    if (n_points < 0 || n_points > 0x7fffffffLL)
        return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: n_points outside [0, 2^31)", k);
    if (!idx && n_points != 0 && n_points != (int64_t)grid.nx * grid.ny * grid.nz)
        return fail(GM_ERR_INVALID_ARGUMENT,
                    "grid %d: idx NULL requires n_points = 0 or the grid's voxels", k);
    if (!isfinite(scale)) return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: scale not finite", k);
    if (n_points > 0) REQ_PTR(dl_dr, "dl_dr");
    double M[12];
    if (!index_to_world(grid, M))
        return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: singular grid affine", k);
    NrfArgs a = nrf_args(nrf, grid, M);
    a.n_points = n_points;
    a.idx = idx;
    a.dl_dr = dl_dr;
    a.scale = scale;
    a.g_w_in = grads->w_in;
    a.g_b_in = grads->b_in;
    a.g_w_hid = grads->w_hid;
    a.g_b_hid = grads->b_hid;
    a.g_w_out = grads->w_out;
    a.g_b_out = grads->b_out;
    *out = a;
    return GM_OK;
}

int64_t rounded_points(int32_t n_grids, const int64_t* n_points)
{
    int64_t P = 0;
    for (int k = 0; k < n_grids; ++k) P += ((n_points[k] + 15) / 16) * 16;
    return P;
}

}  // namespace

gm_status gm_nrf_backward(const gm_nrf* nrf, const gm_grid* grid, const int32_t* idx,
                          int64_t n_points, const float* dl_dr, float scale, gm_nrf_grads* grads,
                          void* workspace, size_t workspace_bytes, gm_stream stream)
{
    g_err.clear();
    gm_status st = check_nrf(nrf);
    if (st != GM_OK) return st;
    if (!grid || !grads) return fail(GM_ERR_INVALID_ARGUMENT, "grid / grads is NULL");
    NrfArgs a;
    st = nrf_backward_grid(nrf, 0, *grid, idx, n_points, dl_dr, scale, grads, &a);
    if (st != GM_OK) return st;
    if (n_points == 0) return GM_OK;
    REQ_PTR(workspace, "workspace");
    st = check_nrf_grads(nrf, grads);
    if (st != GM_OK) return st;
    const NrfLayout L = nrf_layout(nrf, n_points);
    if (workspace_bytes < L.bytes)
        return fail(GM_ERR_INVALID_ARGUMENT, "workspace %zu bytes < required %zu", workspace_bytes,
                    L.bytes);
    const NrfWork w = nrf_work(nrf, L, workspace);
    GM_HIP(launch_nrf_backward(a, w, reinterpret_cast<hipStream_t>(stream)), "nrf backward");
    return GM_OK;
}

gm_status gm_nrf_workspace_grids(const gm_nrf* nrf, int32_t n_grids, const int64_t* n_points,
                                 size_t* bytes)
{
    g_err.clear();
    gm_status st = check_nrf(nrf);
    if (st != GM_OK) return st;
    if (n_grids < 1 || n_grids > GM_MAX_GRIDS || !n_points || !bytes)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_grids outside [1, %d], or n_points / bytes NULL",
                    GM_MAX_GRIDS);
    for (int k = 0; k < n_grids; ++k)
        if (n_points[k] < 0 || n_points[k] > 0x7fffffffLL)
            return fail(GM_ERR_INVALID_ARGUMENT, "n_points[%d] outside [0, 2^31)", k);
    const int64_t P = rounded_points(n_grids, n_points);
    if (P > 0x7fffffffLL) return fail(GM_ERR_INVALID_ARGUMENT, "more than 2^31 points in all");
    *bytes = nrf_layout(nrf, P).bytes;
    return GM_OK;
}

gm_status gm_nrf_backward_grids(const gm_nrf* nrf, int32_t n_grids, const gm_grid* grids,
                                const int32_t* const* idx, const int64_t* n_points,
                                const float* const* dl_dr, const float* scales,
                                gm_nrf_grads* grads, void* workspace, size_t workspace_bytes,
                                gm_stream stream)
{
    g_err.clear();
    gm_status st = check_nrf(nrf);
    if (st != GM_OK) return st;
    if (n_grids < 1 || n_grids > GM_MAX_GRIDS)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_grids outside [1, %d]", GM_MAX_GRIDS);
    if (!grids || !idx || !n_points || !dl_dr || !scales || !grads)
        return fail(GM_ERR_INVALID_ARGUMENT, "grids / idx / n_points / dl_dr / scales / grads NULL");
    NrfArgs as[GM_MAX_GRIDS];
    for (int k = 0; k < n_grids; ++k) {
        st = nrf_backward_grid(nrf, k, grids[k], idx[k], n_points[k], dl_dr[k], scales[k], grads,
                               &as[k]);
        if (st != GM_OK) return st;
    }
    const int64_t P = rounded_points(n_grids, n_points);
    if (P == 0) return GM_OK;
    if (P > 0x7fffffffLL) return fail(GM_ERR_INVALID_ARGUMENT, "more than 2^31 points in all");
    REQ_PTR(workspace, "workspace");
    st = check_nrf_grads(nrf, grads);
    if (st != GM_OK) return st;
    const NrfLayout L = nrf_layout(nrf, P);
    if (workspace_bytes < L.bytes)
        return fail(GM_ERR_INVALID_ARGUMENT, "workspace %zu bytes < required %zu", workspace_bytes,
                    L.bytes);
    const NrfWork w = nrf_work(nrf, L, workspace);
    GM_HIP(launch_nrf_backward_grids(as, n_grids, w, reinterpret_cast<hipStream_t>(stream)),
           "nrf backward over grids");
    return GM_OK;
}

gm_status gm_f32_to_bf16(const float* in, uint16_t* out, int64_t n, gm_stream stream)
{
    g_err.clear();
    if (n < 0) return fail(GM_ERR_INVALID_ARGUMENT, "n < 0");
    if (n == 0) return GM_OK;
    if (!in || !out) return fail(GM_ERR_INVALID_ARGUMENT, "NULL pointer");
    GM_HIP(launch_to_bf16(in, out, n, reinterpret_cast<hipStream_t>(stream)), "to bf16");
    return GM_OK;
}

namespace {

// Shared body of gm_backward (both stages), gm_grid_partials (K7 only) and gm_chain (K8
// only).
// the fused chain + Adam step: moments and per-group scalars
struct AdamFuse {
    gm_gaussian_grads* m;
    gm_gaussian_grads* v;
    AdamScalars c[4];
};

gm_status backward_impl(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                        int32_t n_ids, const float* const* dl_di, float lambda_aniso,
                        float lambda_r, gm_gaussian_grads* grad, hipStream_t s, bool partials,
                        bool chain, const AdamFuse* fuse = nullptr)
{
    gm_status st = check_gauss(g);
    if (st != GM_OK) return st;
    st = check_bins(bins, partials);  // the partials walk the tile lists
    if (st != GM_OK) return st;
    st = check_ids(bins, grid_ids, n_ids);
    if (st != GM_OK) return st;
    if (bins->n_gauss != g->n)
        return fail(GM_ERR_INVALID_ARGUMENT, "bins were built for %lld Gaussians, got %lld",
                    (long long)bins->n_gauss, (long long)g->n);
    if (chain) {
        if (fuse) {
            if (!fuse->m || !fuse->v || fuse->m->n != g->n || fuse->v->n != g->n)
                return fail(GM_ERR_INVALID_ARGUMENT, "Adam moments missing or wrong n");
        } else if (!grad || grad->n != g->n) {
            return fail(GM_ERR_INVALID_ARGUMENT, "grad missing or wrong n");
        }
        if (!isfinite(lambda_aniso) || !isfinite(lambda_r))
            return fail(GM_ERR_INVALID_ARGUMENT, "non-finite lambda");
    }
    if (partials && n_ids > 0 && !dl_di) return fail(GM_ERR_INVALID_ARGUMENT, "dl_di is NULL");
    if (g->n == 0) return GM_OK;
    if (chain && !fuse) {
        REQ_PTR(grad->mean, "grad->mean");
        REQ_PTR(grad->quat, "grad->quat");
        REQ_PTR(grad->log_scale, "grad->log_scale");
        REQ_PTR(grad->logit, "grad->logit");
    }
    if (fuse) {
        for (const gm_gaussian_grads* t : {fuse->m, fuse->v}) {
            REQ_PTR(t->mean, "moment mean");
            REQ_PTR(t->quat, "moment quat");
            REQ_PTR(t->log_scale, "moment log_scale");
            REQ_PTR(t->logit, "moment logit");
        }
    }
    REQ_PTR(bins->records, "bins->records");
    REQ_PTR(bins->tile_count, "bins->tile_count");
    if (n_ids > 0) REQ_PTR(bins->grid_grads, "bins->grid_grads");
    if (partials && bins->n_pairs > 0) {
        REQ_PTR(bins->pair_gauss, "bins->pair_gauss");
        REQ_PTR(bins->tile_start, "bins->tile_start");
    }
    BackwardArgs ba;
    memset(&ba, 0, sizeof ba);
    ChainArgs ca;
    memset(&ca, 0, sizeof ca);
    ba.n = g->n;
    ba.n_ids = n_ids;
    ba.records = bins->records;
    ba.grid_grads = bins->grid_grads;
    ba.pair_gauss = reinterpret_cast<const uint32_t*>(bins->pair_gauss);
    ba.tile_start = bins->tile_start;
    ba.block_query = bins->block_radius > 0 ? 1 : 0;
    for (int k = 0; k < n_ids; ++k) {
        const gm_grid& gr = bins->grids[grid_ids[k]];
        if (partials) {
            REQ_PTR(dl_di[k], "dl_di[k]");
            ba.dl_di[k] = dl_di[k];
        }
        ba.grid_index[k] = grid_ids[k];
        {
            const GridConst c = make_const(gr, bins->tile_base[grid_ids[k]]);
            ba.tile_base[k] = c.tile_base;
            ba.ntx[k] = c.ntx;
            ba.nty[k] = c.nty;
            ba.block_start[k + 1] = ba.block_start[k] + (int32_t)(grid_tiles(gr));
        }
        ba.nx[k] = gr.nx;
        ba.ny[k] = gr.ny;
        ba.nz[k] = gr.nz;
        if (partials && grid_masked(bins, grid_ids[k])) {
            ba.masked[k] = 1;
            if (!index_to_world(gr, ba.m[k]))
                return fail(GM_ERR_INVALID_ARGUMENT, "grid %d: singular affine", grid_ids[k]);
            if (!ba.bq.cells) {
                REQ_PTR(bins->scratch, "bins->scratch");
                ba.bq = block_query(bins);
            }
        }
        ca.grid_index[k] = grid_ids[k];
        ca.g[k] = make_const(gr, bins->tile_base[grid_ids[k]]);
    }
    if (partials) GM_HIP(launch_backward_partials(ba, s), "backward partials");
    if (!chain) return GM_OK;
    ca.n = g->n;
    ca.n_ids = n_ids;
    ca.lambda_aniso = lambda_aniso;
    ca.lambda_r = lambda_r;
    ca.mean = g->mean;
    ca.quat = g->quat;
    ca.log_scale = g->log_scale;
    ca.logit = g->logit;
    ca.tile_count = bins->tile_count;
    ca.grid_grads = bins->grid_grads;
    if (fuse) {
        // the parameters are updated in place
        ca.adam = 1;
        ca.prm[0] = const_cast<float*>(g->mean);
        ca.prm[1] = const_cast<float*>(g->quat);
        ca.prm[2] = const_cast<float*>(g->log_scale);
        ca.prm[3] = const_cast<float*>(g->logit);
        const gm_gaussian_grads* mv[2] = {fuse->m, fuse->v};
        float** dst[2] = {ca.m1, ca.m2};
        for (int t = 0; t < 2; ++t) {
            dst[t][0] = mv[t]->mean;
            dst[t][1] = mv[t]->quat;
            dst[t][2] = mv[t]->log_scale;
            dst[t][3] = mv[t]->logit;
        }
        for (int k = 0; k < 4; ++k) ca.adam_s[k] = fuse->c[k];
    } else {
        ca.g_mean = grad->mean;
        ca.g_quat = grad->quat;
        ca.g_log_scale = grad->log_scale;
        ca.g_logit = grad->logit;
    }
    GM_HIP(launch_chain(ca, s), "chain rule");
    return GM_OK;
}

}  // namespace

gm_status gm_backward(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                      int32_t n_ids, const float* const* dl_di, float lambda_aniso, float lambda_r,
                      gm_gaussian_grads* grad, gm_stream stream)
{
    g_err.clear();
    return backward_impl(g, bins, grid_ids, n_ids, dl_di, lambda_aniso, lambda_r, grad,
                         reinterpret_cast<hipStream_t>(stream), true, true);
}

gm_status gm_grid_partials(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                           int32_t n_ids, const float* const* dl_di, gm_stream stream)
{
    g_err.clear();
    return backward_impl(g, bins, grid_ids, n_ids, dl_di, 0.0f, 0.0f, nullptr,
                         reinterpret_cast<hipStream_t>(stream), true, false);
}

gm_status gm_grid_pose_grads(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                             int32_t n_ids, double* out, void* workspace, size_t workspace_bytes,
                             gm_stream stream)
{
    g_err.clear();
    gm_status st = check_gauss(g);
    if (st != GM_OK) return st;
    st = check_bins(bins, false);
    if (st != GM_OK) return st;
    st = check_ids(bins, grid_ids, n_ids);
    if (st != GM_OK) return st;
    if (bins->n_gauss != g->n)
        return fail(GM_ERR_INVALID_ARGUMENT, "bins were built for %lld Gaussians, got %lld",
                    (long long)bins->n_gauss, (long long)g->n);
    if (n_ids == 0) return GM_OK;
    REQ_PTR(out, "out");
    REQ_PTR(workspace, "workspace");
    if (workspace_bytes < pose_workspace_bytes(n_ids))
        return fail(GM_ERR_INVALID_ARGUMENT, "workspace needs %zu bytes",
                    pose_workspace_bytes(n_ids));
    if (g->n > 0) {
        REQ_PTR(bins->tile_count, "bins->tile_count");
        REQ_PTR(bins->grid_grads, "bins->grid_grads");
    }
    ChainArgs ca;
    memset(&ca, 0, sizeof ca);
    ca.n = g->n;
    ca.n_ids = n_ids;
    ca.mean = g->mean;
    ca.quat = g->quat;
    ca.log_scale = g->log_scale;
    ca.logit = g->logit;
    ca.tile_count = bins->tile_count;
    ca.grid_grads = bins->grid_grads;
    for (int k = 0; k < n_ids; ++k) {
        ca.grid_index[k] = grid_ids[k];
        ca.g[k] = make_const(bins->grids[grid_ids[k]], bins->tile_base[grid_ids[k]]);
    }
    GM_HIP(launch_pose(ca, out, workspace, reinterpret_cast<hipStream_t>(stream)), "pose gradient");
    return GM_OK;
}

gm_status gm_chain(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                   int32_t n_ids, float lambda_aniso, float lambda_r, gm_gaussian_grads* grad,
                   gm_stream stream)
{
    g_err.clear();
    return backward_impl(g, bins, grid_ids, n_ids, nullptr, lambda_aniso, lambda_r, grad,
                         reinterpret_cast<hipStream_t>(stream), false, true);
}

gm_status gm_chain_adam(const gm_gaussians* g, const gm_bins* bins, const int32_t* grid_ids,
                        int32_t n_ids, float lambda_aniso, float lambda_r,
                        const gm_adam_opts* opts, gm_gaussian_grads* m, gm_gaussian_grads* v,
                        gm_stream stream)
{
    g_err.clear();
    if (!opts) return fail(GM_ERR_INVALID_ARGUMENT, "opts is NULL");
    if (opts->step < 1) return fail(GM_ERR_INVALID_ARGUMENT, "step must be >= 1");
    if (!(opts->beta1 >= 0.0 && opts->beta1 < 1.0 && opts->beta2 >= 0.0 && opts->beta2 < 1.0) ||
        !(opts->eps >= 0.0) || !isfinite(opts->eps))
        return fail(GM_ERR_INVALID_ARGUMENT, "bad Adam hyperparameters");
    AdamFuse fuse;
    fuse.m = m;
    fuse.v = v;
    for (int k = 0; k < 4; ++k) {
        if (!isfinite(opts->lr[k])) return fail(GM_ERR_INVALID_ARGUMENT, "non-finite learning rate");
        fuse.c[k] = adam_scalars(opts->lr[k], opts->beta1, opts->beta2, opts->eps, opts->step);
    }
    if (!m || !v) return fail(GM_ERR_INVALID_ARGUMENT, "Adam moments missing");
    return backward_impl(g, bins, grid_ids, n_ids, nullptr, lambda_aniso, lambda_r, nullptr,
                         reinterpret_cast<hipStream_t>(stream), false, true, &fuse);
}

gm_status gm_loss_smooth_l1(int32_t n_stacks, const float* const* preds,
                            const float* const* targets, const int64_t* sizes, float* const* dl_di,
                            float* loss, void* workspace, gm_stream stream)
{
    g_err.clear();
    if (n_stacks < 1 || n_stacks > GM_MAX_GRIDS)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_stacks outside [1, %d]", GM_MAX_GRIDS);
    if (!preds || !targets || !sizes || !dl_di)
        return fail(GM_ERR_INVALID_ARGUMENT, "NULL array argument");
    REQ_PTR(loss, "loss");
    REQ_PTR(workspace, "workspace");
    LossArgs la;
    memset(&la, 0, sizeof la);
    la.n_stacks = n_stacks;
    int64_t tot = 0;
    for (int k = 0; k < n_stacks; ++k) {
        if (sizes[k] < 0) return fail(GM_ERR_INVALID_ARGUMENT, "negative size");
        if (sizes[k] > 0) {
            REQ_PTR(preds[k], "preds[k]");
            REQ_PTR(targets[k], "targets[k]");
            REQ_PTR(dl_di[k], "dl_di[k]");
        }
        la.begin[k] = tot;
        la.pred[k] = preds[k];
        la.target[k] = targets[k];
        la.dl[k] = dl_di[k];
        tot += sizes[k];
    }
    la.begin[n_stacks] = tot;
    la.total = tot;
    GM_HIP(launch_smooth_l1(la, loss, workspace, reinterpret_cast<hipStream_t>(stream)), "smooth-L1");
    return GM_OK;
}

gm_status gm_loss_ssim(int32_t n_stacks, const float* const* preds, const float* const* targets,
                       const int32_t* dims, float lambda, float* const* dl_di, float* loss,
                       void* workspace, gm_stream stream)
{
    g_err.clear();
    if (n_stacks < 1 || n_stacks > GM_MAX_GRIDS)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_stacks outside [1, %d]", GM_MAX_GRIDS);
    if (!preds || !targets || !dims || !dl_di)
        return fail(GM_ERR_INVALID_ARGUMENT, "NULL array argument");
    REQ_PTR(loss, "loss");
    REQ_PTR(workspace, "workspace");
    if (!isfinite(lambda)) return fail(GM_ERR_INVALID_ARGUMENT, "lambda not finite");
    SsimArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.n_stacks = n_stacks;
    int64_t tiles = 0, vox = 0;
    for (int k = 0; k < n_stacks; ++k) {
        const int32_t nx = dims[3 * k], ny = dims[3 * k + 1], nz = dims[3 * k + 2];
        if (nx < 0 || ny < 0 || nz < 0) return fail(GM_ERR_INVALID_ARGUMENT, "negative dims");
        const int64_t n = (int64_t)nx * ny * nz;
        if (n > 0) {
            REQ_PTR(preds[k], "preds[k]");
            REQ_PTR(targets[k], "targets[k]");
            REQ_PTR(dl_di[k], "dl_di[k]");
        }
        sa.nx[k] = nx;
        sa.ny[k] = ny;
        ssim_tiles(nx, ny, &sa.tiles_x[k], &sa.tiles_y[k]);
        sa.tile_begin[k] = tiles;
        if (n > 0) tiles += (int64_t)nz * sa.tiles_x[k] * sa.tiles_y[k];
        sa.pred[k] = preds[k];
        sa.target[k] = targets[k];
        sa.dl[k] = dl_di[k];
        vox += n;
    }
    sa.tile_begin[n_stacks] = tiles;
    // 1D Gaussian taps, sigma 1.5, normalised
    double gs = 0.0;
    for (int i = 0; i < 11; ++i) {
        const double d = (double)(i - 5);
        sa.g[i] = exp(-d * d / (2.0 * 1.5 * 1.5));
        gs += sa.g[i];
    }
    for (int i = 0; i < 11; ++i) sa.g[i] /= gs;
    sa.grad_scale = vox > 0 ? -(double)lambda / (double)vox : 0.0;
    GM_HIP(launch_ssim(sa, vox, loss, workspace, reinterpret_cast<hipStream_t>(stream)), "SSIM");
    return GM_OK;
}

gm_status gm_aniso_reg(const gm_gaussians* g, float lambda_r, float* value, void* workspace,
                       gm_stream stream)
{
    g_err.clear();
    gm_status st = check_gauss(g);
    if (st != GM_OK) return st;
    REQ_PTR(value, "value");
    REQ_PTR(workspace, "workspace");
    GM_HIP(launch_aniso(g->log_scale, g->n, lambda_r, value, workspace,
                        reinterpret_cast<hipStream_t>(stream)), "aniso");
    return GM_OK;
}

gm_status gm_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, double lr,
                       double beta1, double beta2, double eps, int32_t step, gm_stream stream)
{
    g_err.clear();
    if (n < 0) return fail(GM_ERR_INVALID_ARGUMENT, "n < 0");
    if (step < 1) return fail(GM_ERR_INVALID_ARGUMENT, "step must be >= 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0) || !(eps >= 0.0) ||
        !isfinite(lr) || !isfinite(eps))
        return fail(GM_ERR_INVALID_ARGUMENT, "bad Adam hyperparameters");
    if (n == 0) return GM_OK;
    REQ_PTR(param, "param");
    REQ_PTR(grad, "grad");
    REQ_PTR(m, "m");
    REQ_PTR(v, "v");
    GM_HIP(launch_adam(param, grad, m, v, n, adam_scalars(lr, beta1, beta2, eps, step),
                       reinterpret_cast<hipStream_t>(stream)), "adam");
    return GM_OK;
}

gm_status gm_upsample_lattice(int32_t g_old, const gm_gaussians* old, int32_t g_new,
                              float* mean, float* quat, float* log_scale, float* logit,
                              gm_stream stream)
{
    g_err.clear();
    if (g_old < 1 || g_new < 1 || g_old > 2048 || g_new > 2048)
        return fail(GM_ERR_INVALID_ARGUMENT, "lattice sizes outside [1, 2048]");
    gm_status st = check_gauss(old);
    if (st != GM_OK) return st;
    if (old->n != (int64_t)g_old * g_old * g_old)
        return fail(GM_ERR_INVALID_ARGUMENT, "old holds %lld Gaussians, not g_old^3",
                    (long long)old->n);
    REQ_PTR(mean, "mean");
    REQ_PTR(quat, "quat");
    REQ_PTR(log_scale, "log_scale");
    REQ_PTR(logit, "logit");
    UpsampleArgs ua;
    ua.g_old = g_old;
    ua.g_new = g_new;
    ua.quat = old->quat;
    ua.log_scale = old->log_scale;
    ua.logit = old->logit;
    ua.out_mean = mean;
    ua.out_quat = quat;
    ua.out_log_scale = log_scale;
    ua.out_logit = logit;
    GM_HIP(launch_upsample(ua, reinterpret_cast<hipStream_t>(stream)), "lattice upsample");
    return GM_OK;
}

gm_status gm_devox_init(int32_t g, const gm_grid* stacks, int32_t n_stacks,
                        const float* const* stack_data, float* mean, float* quat,
                        float* log_scale, float* logit, gm_stream stream)
{
    g_err.clear();
    if (g < 1 || g > 1290) return fail(GM_ERR_INVALID_ARGUMENT, "g outside [1, 1290]");
    if (n_stacks < 1 || n_stacks > GM_MAX_GRIDS || !stacks || !stack_data)
        return fail(GM_ERR_INVALID_ARGUMENT, "n_stacks outside [1, %d] or NULL arrays", GM_MAX_GRIDS);
    REQ_PTR(mean, "mean");
    REQ_PTR(quat, "quat");
    REQ_PTR(log_scale, "log_scale");
    REQ_PTR(logit, "logit");
    DevoxArgs da;
    memset(&da, 0, sizeof da);
    da.g = g;
    da.n_stacks = n_stacks;
    for (int k = 0; k < n_stacks; ++k) {
        gm_status st = check_grid(stacks[k], k);
        if (st != GM_OK) return st;
        REQ_PTR(stack_data[k], "stack_data[k]");
        da.s[k] = make_const(stacks[k], 0);
        da.data[k] = stack_data[k];
    }
    da.mean = mean;
    da.quat = quat;
    da.log_scale = log_scale;
    da.logit = logit;
    GM_HIP(launch_devox(da, reinterpret_cast<hipStream_t>(stream)), "devox init");
    return GM_OK;
}

gm_status gm_ws_gather(const gm_grid* stacks, int32_t n_stacks, const float* const* stack_data,
                       const float* means, int64_t n, float spacing, uint16_t* patches,
                       gm_stream stream)
{
    g_err.clear();
    if (n_stacks != 3 || !stacks || !stack_data)
        return fail(GM_ERR_INVALID_ARGUMENT, "the warm-start network takes exactly 3 stacks");
    if (n < 0 || !isfinite(spacing) || !(spacing > 0.0f))
        return fail(GM_ERR_INVALID_ARGUMENT, "n < 0 or bad spacing");
    if (n == 0) return GM_OK;
    REQ_PTR(means, "means");
    REQ_PTR(patches, "patches");
    WsGatherArgs a;
    memset(&a, 0, sizeof a);
    a.n = n;
    a.spacing = spacing;
    a.means = means;
    a.patches = patches;
    for (int k = 0; k < 3; ++k) {
        gm_status st = check_grid(stacks[k], k);
        if (st != GM_OK) return st;
        REQ_PTR(stack_data[k], "stack_data[k]");
        a.data[k] = stack_data[k];
        a.s[k] = make_const(stacks[k], 0);
    }
    GM_HIP(launch_ws_gather(a, reinterpret_cast<hipStream_t>(stream)), "ws gather");
    return GM_OK;
}

gm_status gm_ws_targets(const float* log_scale, const float* quat, int64_t n,
                        float* sigma_target, gm_stream stream)
{
    g_err.clear();
    if (n < 0) return fail(GM_ERR_INVALID_ARGUMENT, "n < 0");
    if (n == 0) return GM_OK;
    REQ_PTR(log_scale, "log_scale");
    REQ_PTR(quat, "quat");
    REQ_PTR(sigma_target, "sigma_target");
    GM_HIP(launch_ws_targets(log_scale, quat, n, sigma_target,
                             reinterpret_cast<hipStream_t>(stream)), "ws targets");
    return GM_OK;
}

gm_status gm_ws_workspace(int64_t n, size_t* bytes)
{
    g_err.clear();
    if (n < 0 || n % 16 != 0 || !bytes)
        return fail(GM_ERR_INVALID_ARGUMENT, "n must be a non-negative multiple of 16");
    *bytes = ws_layout(n).bytes;
    return GM_OK;
}

static gm_status ws_common(const gm_ws_net* net, const uint16_t* patches, int64_t n,
                           const float* s0, const float* logit0, void* ws, size_t ws_bytes,
                           WsLayout* L)
{
    gm_status st = check_ws_net(net);
    if (st != GM_OK) return st;
    if (n <= 0 || n % 16 != 0) return fail(GM_ERR_INVALID_ARGUMENT, "n must be a positive multiple of 16");
    REQ_PTR(patches, "patches");
    REQ_PTR(s0, "s0");
    REQ_PTR(logit0, "logit0");
    REQ_PTR(ws, "workspace");
    *L = ws_layout(n);
    if (ws_bytes < L->bytes)
        return fail(GM_ERR_INVALID_ARGUMENT, "workspace %zu bytes < required %zu", ws_bytes, L->bytes);
    return GM_OK;
}

gm_status gm_ws_forward(const gm_ws_net* net, const uint16_t* patches, int64_t n,
                        const float* s0, const float* logit0, float* log_scale_out,
                        float* quat_out, float* logit_out, void* workspace,
                        size_t workspace_bytes, gm_stream stream)
{
    g_err.clear();
    WsLayout L;
    gm_status st = ws_common(net, patches, n, s0, logit0, workspace, workspace_bytes, &L);
    if (st != GM_OK) return st;
    REQ_PTR(log_scale_out, "log_scale_out");
    REQ_PTR(quat_out, "quat_out");
    REQ_PTR(logit_out, "logit_out");
    char* base = reinterpret_cast<char*>(workspace);
    WsActs w = ws_acts(base, L);
    // inference: only the last layer's pre-activation (read by the head) is stored
    for (int l = 0; l < 3; ++l) w.z[l] = nullptr;
    WsHeadArgs h;
    memset(&h, 0, sizeof h);
    h.n = n;
    h.z4 = w.z[3];
    h.wl = net->wl;
    h.bl = net->bl;
    h.s0 = s0;
    h.logit0 = logit0;
    h.s_out = log_scale_out;
    h.q_out = quat_out;
    h.logit_out = logit_out;
    GM_HIP(launch_ws_forward(ws_net(net), patches, n, w, h, reinterpret_cast<hipStream_t>(stream)),
           "ws forward");
    return GM_OK;
}

gm_status gm_ws_backward(const gm_ws_net* net, const uint16_t* patches, int64_t n,
                         const float* s0, const float* logit0, const float* sigma_target,
                         const float* logit_target, float* loss, gm_ws_grads* grads,
                         void* workspace, size_t workspace_bytes, gm_stream stream)
{
    g_err.clear();
    WsLayout L;
    gm_status st = ws_common(net, patches, n, s0, logit0, workspace, workspace_bytes, &L);
    if (st != GM_OK) return st;
    REQ_PTR(sigma_target, "sigma_target");
    REQ_PTR(logit_target, "logit_target");
    REQ_PTR(loss, "loss");
    if (!grads) return fail(GM_ERR_INVALID_ARGUMENT, "grads is NULL");
    WsGrads g;
    for (int l = 0; l < 4; ++l) {
        REQ_PTR(grads->w[l], "grads->w[l]");
        REQ_PTR(grads->b[l], "grads->b[l]");
        g.w[l] = grads->w[l];
        g.b[l] = grads->b[l];
    }
    REQ_PTR(grads->wl, "grads->wl");
    REQ_PTR(grads->bl, "grads->bl");
    g.wl = grads->wl;
    g.bl = grads->bl;
    char* base = reinterpret_cast<char*>(workspace);
    WsActs w = ws_acts(base, L);
    WsHeadArgs h;
    memset(&h, 0, sizeof h);
    h.n = n;
    h.z4 = w.z[3];
    h.wl = net->wl;
    h.bl = net->bl;
    h.s0 = s0;
    h.logit0 = logit0;
    h.sig_t = sigma_target;
    h.logit_t = logit_target;
    h.loss_each = reinterpret_cast<float*>(base + L.off_loss);
    h.dout = reinterpret_cast<float*>(base + L.off_dout);
    h.a4 = reinterpret_cast<float*>(base + L.off_a4);
    h.dz4 = w.dz[3];
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    GM_HIP(launch_ws_forward(ws_net(net), patches, n, w, h, s), "ws forward");
    GM_HIP(launch_ws_backward(ws_net(net), patches, n, w, h, g, loss, s), "ws backward");
    return GM_OK;
}

gm_status gm_mse(const float* vol, const float* ref, int64_t n, float* mse, void* workspace,
                 gm_stream stream)
{
    g_err.clear();
    if (n < 0) return fail(GM_ERR_INVALID_ARGUMENT, "n < 0");
    if (n > 0) {
        REQ_PTR(vol, "vol");
        REQ_PTR(ref, "ref");
    }
    REQ_PTR(mse, "mse");
    REQ_PTR(workspace, "workspace");
    GM_HIP(launch_mse(vol, ref, n, mse, workspace, reinterpret_cast<hipStream_t>(stream)), "mse");
    return GM_OK;
}

}  // extern "C"
