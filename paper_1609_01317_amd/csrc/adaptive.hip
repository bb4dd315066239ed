// Adaptive sampling (Section 5.2: detail-poor regions are sampled at a lower
// rate).  A sample in an 8^3 brick whose value range is at most adapt_range
// advances its ray by adapt steps, any other by one; each sample's opacity
// is corrected to the distance it stands for.  The sample positions depend
// on the bricks met along each ray, so there is no lattice shared by the
// rays; shaded renders still march a tile's rays together in chunks of ray
// parameter with LDS-staged boxes (adaptive.h).  Arithmetic per sample is
// the volume mode's (march.h).  The per-tile march (adaptive_tile) is
// shared with the persistent batched kernel.
#include "adaptive.h"

namespace rc {

// One wave per tile, three waves per SIMD and a 12 KiB box, as the
// fixed-step shaded kernel.
template <typename VT, int OP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void raycast_adaptive(
    RenderParams P) {
    __shared__ __align__(16) unsigned char lds[kWaveLdsBytes];
    const ViewParams& V = P.view;
    int tile = tile_of_block(blockIdx.x, V.tiles_x, V.n_tiles / V.tiles_x);
    if (tile < 0) return;
    adaptive_tile<VT, OP>(P, V, tile, threadIdx.x, lds, kWaveLdsBytes);
}

template <typename VT>
static void launch_adaptive_t(const RenderParams& P, int op, hipStream_t st) {
    const ViewParams& V = P.view;
    dim3 grid((unsigned)group_grid_blocks(V.tiles_x, V.n_tiles / V.tiles_x)), block(64);
    if (op == RC_GRAD_CENTRAL)
        hipLaunchKernelGGL((raycast_adaptive<VT, RC_GRAD_CENTRAL>), grid, block, 0, st, P);
    else if (op == RC_GRAD_SOBEL3D)
        hipLaunchKernelGGL((raycast_adaptive<VT, RC_GRAD_SOBEL3D>), grid, block, 0, st, P);
    else
        hipLaunchKernelGGL((raycast_adaptive<VT, RC_GRAD_ZUCKER_HUMMEL>), grid, block, 0, st, P);
}

rc_status launch_adaptive(const RenderParams& P, rc_dtype dt, int op, hipStream_t st) {
    if (dt == RC_U8) launch_adaptive_t<uint8_t>(P, op, st);
    else if (dt == RC_U16) launch_adaptive_t<uint16_t>(P, op, st);
    else launch_adaptive_t<float>(P, op, st);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

}  // namespace rc
