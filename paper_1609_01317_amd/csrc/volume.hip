// Volume handles: ingest into the brick-tiled layout, per-brick value
// ranges for empty-space skipping, error reporting.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "march.h"      // RC_IDX: index checks of the bounds-checked build

namespace rc {

static thread_local std::string g_last_error;

rc_status fail(rc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

rc_status hip_fail(hipError_t e, const char* what) {
    // the error is reported here: clear the runtime's last-error state so a
    // later launch check does not see it again (after a failed allocation
    // the library stays usable)
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory)
        return fail(RC_E_OOM, "%s: %s", what, hipGetErrorString(e));
    return fail(RC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- kernels
// One workgroup per run of kTileRun bricks along x: the run's voxels (rows
// of up to kBrick * kTileRun voxels, contiguous along x in the source) are
// read row by row at clamped coordinates, so the padding replicates the
// edge (Section 2.1: the grid is a 3D array of samples), staged in LDS, and
// written out brick by brick in Morton order: the run's bricks are
// consecutive in the bricked array, so both the reads and the writes are
// contiguous runs.  With `range` set the block also takes the one-voxel
// high apron (one more row, plane and column) and writes each brick's value
// range from LDS, as brick_minmax defines it.  The staging rows and planes
// are padded (kRunRow, kRunPlane) so the 64 voxels a wave reads back in
// Morton order fall in distinct LDS banks.
constexpr int kTileRun = 8;
// 8 voxels of a Morton group, stored with one (16-byte for u16) vector write
template <typename T> struct alignas(8 * sizeof(T)) Group {
    T v[8];
};
// 4 consecutive voxels of a source row, read with one vector load
template <typename T> struct alignas(4 * sizeof(T)) Quad {
    T v[4];
};
constexpr int kRunRow = kBrick * kTileRun + 4;
constexpr int kRunPlane = (kBrick + 1) * kRunRow + 12;
template <typename T>
__global__ __launch_bounds__(256) void brick_tile(const T* __restrict__ src, T* __restrict__ dst,
                                                  float2* __restrict__ range, int nx, int ny,
                                                  int nz, int nbx, int nby, long long n_runs,
                                                  unsigned int* dbg) {
    // voxel (x, y, z) of the run (apron included) at z, y, x strides
    __shared__ __align__(16) T run[(kBrick + 1) * kRunPlane];
    const long long r = blockIdx.x;
    if (r >= n_runs) return;
    const int runs_x = (nbx + kTileRun - 1) / kTileRun;
    const int rx = (int)(r % runs_x);
    const long long rest = r / runs_x;
    const int by = (int)(rest % nby), bz = (int)(rest / nby);
    const int bx0 = rx * kTileRun, nb = min(kTileRun, nbx - bx0);
    const int x0 = bx0 * kBrick, y0 = by * kBrick, z0 = bz * kBrick;
    const long long n_src = (long long)nx * ny * nz;
    const long long n_bricks = (long long)nbx * nby * ((nz + kBrick - 1) / kBrick);
    constexpr int n_lds = (kBrick + 1) * kRunPlane;
    const int apron = range ? 1 : 0;
    const int ncol = kBrick * nb + apron, nyr = kBrick + apron, nrow = nyr * (kBrick + apron);
    // Rows whose voxels sit 4-aligned in the source (an aligned base, nx a
    // multiple of 4; x0 is a multiple of 64) are read 4 voxels per load where
    // all 4 lie inside the row; the rest, and other sources, voxel by voxel.
    constexpr int kQuads = kBrick * kTileRun / 4 + 1;       // 16 quads + the apron column
    const bool quads = (nx & 3) == 0 && ((uintptr_t)src & (4 * sizeof(T) - 1)) == 0;
    const int per_row = quads ? kQuads : kBrick * kTileRun + 1;
    for (int i = threadIdx.x; i < nrow * per_row; i += blockDim.x) {
        const int c = i % per_row, row = i / per_row;
        const int yl = row % nyr, zl = row / nyr;
        const int y = min(y0 + yl, ny - 1), z = min(z0 + zl, nz - 1);
        const long long line = ((long long)z * ny + y) * nx;
        const int l = zl * kRunPlane + yl * kRunRow;
        const int xl = quads ? min(4 * c, kBrick * kTileRun) : c;
        if (xl >= ncol) continue;
        if (quads && c < kQuads - 1 && x0 + xl + 3 < nx) {
            *(Quad<T>*)&run[RC_IDX(dbg, l + xl, n_lds - 3)] =
                *(const Quad<T>*)&src[RC_IDX(dbg, line + x0 + xl, n_src - 3)];
        } else {
            const int n = (quads && c < kQuads - 1) ? 4 : 1;
            for (int d = 0; d < n; ++d)
                run[RC_IDX(dbg, l + xl + d, n_lds)] =
                    src[RC_IDX(dbg, line + min(x0 + xl + d, nx - 1), n_src)];
        }
    }
    __syncthreads();
    // one 2x2x2 Morton group (8 consecutive voxels of the bricked array) per
    // thread and step, written with one vector store
    const long long first = (((long long)bz * nby + by) * nbx + bx0) * kBrickVox;
    for (int grp = threadIdx.x; grp < (kBrickVox / 8) * nb; grp += blockDim.x) {
        const uint32_t m = (uint32_t)(grp & (kBrickVox / 8 - 1)) << 3;
        const int l0 = (int)compact3(m >> 2) * kRunPlane + (int)compact3(m >> 1) * kRunRow +
                       (grp / (kBrickVox / 8)) * kBrick + (int)compact3(m);
        Group<T> g;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            g.v[q] = run[RC_IDX(dbg, l0 + (q >> 2) * kRunPlane + ((q >> 1) & 1) * kRunRow + (q & 1),
                                n_lds)];
        *(Group<T>*)(dst + RC_IDX(dbg, first + 8ll * grp, n_bricks * kBrickVox - 7)) = g;
    }
    if (!range) return;
    // one wave per brick of the run: min and max over its 9^3 voxels
    const int lane = threadIdx.x & 63;
    for (int j = threadIdx.x >> 6; j < nb; j += blockDim.x >> 6) {
        float lo = INFINITY, hi = -INFINITY;
        for (int q = lane; q < 729; q += 64) {
            const int dx = q % 9, dy = (q / 9) % 9, dz = q / 81;
            const float v =
                (float)run[RC_IDX(dbg, dz * kRunPlane + dy * kRunRow + j * kBrick + dx, n_lds)];
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
        for (int o = 32; o > 0; o >>= 1) {
            lo = fminf(lo, __shfl_xor(lo, o));
            hi = fmaxf(hi, __shfl_xor(hi, o));
        }
        if (lane == 0)
            range[RC_IDX(dbg, ((long long)bz * nby + by) * nbx + bx0 + j, n_bricks)] =
                make_float2(lo, hi);
    }
}

// One wave per brick: min and max over voxels [b0, b0+8] per axis (the
// brick plus its one-voxel high apron, clamped to the grid), which is every
// voxel a trilinear sample inside the brick's cells can touch.
template <typename T>
__global__ __launch_bounds__(64) void brick_minmax(const T* __restrict__ vox, float2* __restrict__ out,
                                                   int nx, int ny, int nz, int nbx, int nby,
                                                   int sy, int sz, long long nbricks,
                                                   unsigned int* dbg) {
    long long b = blockIdx.x;
    if (b >= nbricks) return;
    int bx = (int)(b % nbx);
    long long rest = b / nbx;
    int by = (int)(rest % nby);
    int bz = (int)(rest / nby);
    float lo = INFINITY, hi = -INFINITY;
    for (int q = threadIdx.x; q < 729; q += 64) {
        int dx = q % 9, dy = (q / 9) % 9, dz = q / 81;
        int x = min(bx * kBrick + dx, nx - 1);
        int y = min(by * kBrick + dy, ny - 1);
        int z = min(bz * kBrick + dz, nz - 1);
        float v = (float)vox[RC_IDX(dbg, off_x(x) + off_y(y, sy) + off_z(z, sz),
                                    nbricks * kBrickVox)];
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o));
        hi = fmaxf(hi, __shfl_xor(hi, o));
    }
    if (threadIdx.x == 0) out[RC_IDX(dbg, b, nbricks)] = make_float2(lo, hi);
}

static int elem_size(rc_dtype dt) { return dt == RC_U8 ? 1 : dt == RC_U16 ? 2 : 4; }

// range: the brick ranges to rebuild in the same pass, or null
static rc_status launch_tile(rc_volume* v, const void* src, float2* range, hipStream_t st) {
    const long long total = (long long)((v->nbx + kTileRun - 1) / kTileRun) * v->nby * v->nbz;
    const unsigned grid = (unsigned)total;
    switch (v->dtype) {
        case RC_U8:
            hipLaunchKernelGGL(brick_tile<uint8_t>, dim3(grid), dim3(256), 0, st,
                               (const uint8_t*)src, (uint8_t*)v->bricked, range, v->nx, v->ny,
                               v->nz, v->nbx, v->nby, total, debug_counter());
            break;
        case RC_U16:
            hipLaunchKernelGGL(brick_tile<uint16_t>, dim3(grid), dim3(256), 0, st,
                               (const uint16_t*)src, (uint16_t*)v->bricked, range, v->nx, v->ny,
                               v->nz, v->nbx, v->nby, total, debug_counter());
            break;
        default:
            hipLaunchKernelGGL(brick_tile<float>, dim3(grid), dim3(256), 0, st,
                               (const float*)src, (float*)v->bricked, range, v->nx, v->ny, v->nz,
                               v->nbx, v->nby, total, debug_counter());
    }
    RC_HIP(hipGetLastError());
    return RC_OK;
}

static rc_status launch_minmax(rc_volume* v, hipStream_t st) {
    int sy = v->nbx * kBrickVox, sz = v->nbx * v->nby * kBrickVox;
    dim3 grid((unsigned)v->nbricks), block(64);
    switch (v->dtype) {
        case RC_U8:
            hipLaunchKernelGGL(brick_minmax<uint8_t>, grid, block, 0, st,
                               (const uint8_t*)v->bricked, v->brick_range, v->nx, v->ny, v->nz,
                               v->nbx, v->nby, sy, sz, v->nbricks, debug_counter());
            break;
        case RC_U16:
            hipLaunchKernelGGL(brick_minmax<uint16_t>, grid, block, 0, st,
                               (const uint16_t*)v->bricked, v->brick_range, v->nx, v->ny, v->nz,
                               v->nbx, v->nby, sy, sz, v->nbricks, debug_counter());
            break;
        default:
            hipLaunchKernelGGL(brick_minmax<float>, grid, block, 0, st, (const float*)v->bricked,
                               v->brick_range, v->nx, v->ny, v->nz, v->nbx, v->nby, sy, sz,
                               v->nbricks, debug_counter());
    }
    RC_HIP(hipGetLastError());
    return RC_OK;
}

}  // namespace rc

using namespace rc;

extern "C" const char* rc_last_error(void) { return g_last_error.c_str(); }

extern "C" rc_status rc_create_volume(const void* src_dev, int nx, int ny, int nz,
                                      int32_t dtype_in, const double spacing[3], float vmin,
                                      float vmax, void* stream, rc_volume** out) {
    if (!out) return fail(RC_E_INVALID, "rc_create_volume: out is NULL");
    *out = nullptr;
    if (!src_dev) return fail(RC_E_INVALID, "rc_create_volume: src_dev is NULL");
    if (!spacing) return fail(RC_E_INVALID, "rc_create_volume: spacing is NULL");
    if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
        return fail(RC_E_INVALID, "rc_create_volume: dims %d x %d x %d outside 1..4096", nx, ny, nz);
    // an int on the ABI: an out-of-range value must not be held in the enum
    if (dtype_in != RC_U8 && dtype_in != RC_U16 && dtype_in != RC_F32)
        return fail(RC_E_INVALID, "rc_create_volume: unknown dtype %d", (int)dtype_in);
    const rc_dtype dtype = (rc_dtype)dtype_in;
    for (int a = 0; a < 3; ++a)
        if (!(std::isfinite(spacing[a]) && spacing[a] > 0.0))
            return fail(RC_E_INVALID, "rc_create_volume: spacing[%d] must be finite and > 0", a);
    if (!(std::isfinite(vmin) && std::isfinite(vmax) && vmax > vmin))
        return fail(RC_E_INVALID, "rc_create_volume: need finite vmin < vmax");
    int nbx = (nx + 7) / 8, nby = (ny + 7) / 8, nbz = (nz + 7) / 8;
    long long nbricks = (long long)nbx * nby * nbz;
    if (nbricks * kBrickVox >= (1LL << 31))
        return fail(RC_E_INVALID, "rc_create_volume: padded volume exceeds 2^31 voxels");
    rc_volume* v = new (std::nothrow) rc_volume();
    if (!v) return fail(RC_E_OOM, "rc_create_volume: host allocation failed");
    v->nx = nx; v->ny = ny; v->nz = nz;
    v->dtype = dtype;
    v->elem_bytes = elem_size(dtype);
    for (int a = 0; a < 3; ++a) v->spacing[a] = spacing[a];
    v->vmin = vmin; v->vmax = vmax;
    v->nbx = nbx; v->nby = nby; v->nbz = nbz;
    v->nbricks = nbricks;
    v->brick_range = nullptr;
    v->nsx = (nbx + 3) / 4; v->nsy = (nby + 3) / 4; v->nsz = (nbz + 3) / 4;
    v->nsuper = (long long)v->nsx * v->nsy * v->nsz;
    hipError_t e = hipGetDevice(&v->device);
    if (e != hipSuccess) { delete v; return hip_fail(e, "hipGetDevice"); }
    e = hipMalloc(&v->bricked, (size_t)nbricks * kBrickVox * v->elem_bytes);
    if (e != hipSuccess) { delete v; return hip_fail(e, "hipMalloc(bricked volume)"); }
    rc_status st = launch_tile(v, src_dev, nullptr, (hipStream_t)stream);
    if (st != RC_OK) { (void)hipFree(v->bricked); delete v; return st; }
    *out = v;
    return RC_OK;
}

extern "C" rc_status rc_update_volume(rc_volume* v, const void* src_dev, void* stream) {
    if (!v) return fail(RC_E_INVALID, "rc_update_volume: volume is NULL");
    if (!src_dev) return fail(RC_E_INVALID, "rc_update_volume: src_dev is NULL");
    // existing brick ranges are rebuilt from the same staged voxels
    return launch_tile(v, src_dev, v->brick_range, (hipStream_t)stream);
}

extern "C" rc_status rc_build_bricks(rc_volume* v, int brick_edge, void* stream) {
    if (!v) return fail(RC_E_INVALID, "rc_build_bricks: volume is NULL");
    if (brick_edge != kBrick)
        return fail(RC_E_UNSUPPORTED, "rc_build_bricks: brick edge %d (only 8 is built)", brick_edge);
    if (!v->brick_range) {
        hipError_t e = hipMalloc((void**)&v->brick_range, (size_t)v->nbricks * sizeof(float2));
        if (e != hipSuccess) { v->brick_range = nullptr; return hip_fail(e, "hipMalloc(brick ranges)"); }
    }
    return launch_minmax(v, (hipStream_t)stream);
}

// The handle is not tied to one stream (renders may read it on several),
// so its memory is released after the volume's device has finished all
// work (hipFree waits for that device as well); the wait is on the
// volume's own device, made current for the call.
extern "C" void rc_destroy_volume(rc_volume* v) {
    if (!v) return;
    int cur = -1;
    const bool other = hipGetDevice(&cur) == hipSuccess && cur != v->device;
    if (other) (void)hipSetDevice(v->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(v->bricked);
    if (v->brick_range) (void)hipFree(v->brick_range);
    if (other) (void)hipSetDevice(cur);
    delete v;
}
