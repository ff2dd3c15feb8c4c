// K11 forward alone: the neural residual field (Sec. 3.4, Eq. 8) added to a volume or a list
// of voxels, r(x) = out_scale tanh(w_out . a_D + b_out) with the layer stack of nrf_core.h.
// A wavefront takes 16 points at a time and keeps the weights in registers for all of them
// (they are staged once per block in LDS to build the MFMA operand layout).  Its own source
// file because it is built with the MFMA results in ordinary VGPRs (every accumulator is read
// back for the activation), which the backward's chain kernel is not.
#include "nrf_core.h"

namespace {

using namespace nrfcore;

template <int KT, int DEPTH>
__global__ __launch_bounds__(256) void k_nrf_forward(const NrfArgs a)
{
    __shared__ Lds<KT, DEPTH> s;
    load_weights<KT, DEPTH>(a, s);
    const int lane = threadIdx.x & 63, g = lane >> 4, row = lane & 15;
    v4s wo[4];
    load_wout(a, wo);
    WeightsReg<KT, DEPTH> wr;     // the weights stay in registers for every tile
    wr.load(s, lane);
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
        tile_forward_w<KT, DEPTH>(a, wr, x, T);
        const float zo = tile_output<KT, DEPTH>(a, T, wo);     // lane group 0
        if (valid && g == 0) {
            const int64_t v = ((int64_t)vz * a.ny + vy) * a.nx + vx;
            a.out[v] += a.out_scale * tanhf(zo);
        }
    }
}

}  // namespace

template <int KT, int DEPTH>
void launch_fwd_t(const NrfArgs& a, hipStream_t s)
{
    const unsigned nb =
        nrfcore::blocks_for_tiles(k_nrf_forward<KT, DEPTH>, (a.n_points + 15) / 16);
    hipLaunchKernelGGL((k_nrf_forward<KT, DEPTH>), dim3(nb), dim3(256), 0, s, a);
}

hipError_t launch_nrf_forward(const NrfArgs& a, hipStream_t s)
{
    if (a.n_points <= 0) return hipSuccess;
    GM_NRF_DISPATCH(launch_fwd_t, a, s)
    return hipGetLastError();
}
