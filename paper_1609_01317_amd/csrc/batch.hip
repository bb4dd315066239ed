// Batched rendering: many images of many volumes in one persistent launch.
// Each item is the argument set of one rc_render call.  Resident waves pull
// (item, tile) work units from per-XCD work queues until all are empty
// (persist.h); the per-item empty-brick and super-brick masks are built by
// three batched kernels; the whole sequence can be captured into a HIP graph
// and replayed.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <map>
#include <numeric>
#include <tuple>
#include <string>
#include <vector>

#include "persist.h"

namespace rc {

struct MaskJob {
    const float2* range;
    const float4* tf;
    int M;
    float vmin, inv_range, Mm1;
    long long nbricks;
    long long brick_off;        // offset into the concatenated mask array
    long long prefix_off;       // offset into the concatenated prefix array
    int nbx, nby, nbz, nsx, nsy;
    long long nsuper;
    long long super_off;        // offset into the concatenated super mask array
    float adapt_range;          // detail-poor bound of adaptive items, NaN otherwise
};

// ---------------------------------------------------------------- kernels
// the kQueues work-queue counters of a launch
__global__ void batch_reset(int* counters) {
    if (threadIdx.x < kQueues) counters[threadIdx.x * kQueueStride] = 0;
}

// one workgroup per mask job: prefix counts of non-zero table opacities
__global__ __launch_bounds__(256) void batch_prefix(const MaskJob* __restrict__ jobs,
                                                    int* __restrict__ prefix_all) {
    __shared__ int part[256];
    const MaskJob& J = jobs[blockIdx.x];
    int* prefix = prefix_all + J.prefix_off;
    int M = J.M;
    int chunk = (M + 255) / 256;
    int lo = threadIdx.x * chunk, hi = min(lo + chunk, M);
    int cnt = 0;
    for (int i = lo; i < hi; ++i) cnt += J.tf[i].w != 0.0f;
    part[threadIdx.x] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int t = 0; t < 256; ++t) {
            int c = part[t];
            part[t] = acc;
            acc += c;
        }
        prefix[M] = acc;
    }
    __syncthreads();
    int acc = part[threadIdx.x];
    for (int i = lo; i < hi; ++i) {
        prefix[i] = acc;
        acc += J.tf[i].w != 0.0f;
    }
}

// one thread per brick of every mask job (same rule as empty_mask)
__global__ __launch_bounds__(256) void batch_mask(const MaskJob* __restrict__ jobs, int njobs,
                                                  long long total, const int* __restrict__ prefix_all,
                                                  uint8_t* __restrict__ mask_all) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (jobs[mid].brick_off <= g) lo = mid; else hi = mid;
    }
    const MaskJob& J = jobs[lo];
    long long b = g - J.brick_off;
    if (b < 0 || b >= J.nbricks) return;
    const int* prefix = prefix_all + J.prefix_off;
    float2 r = J.range[b];
    float ulo = fminf(fmaxf((r.x - J.vmin) * J.inv_range, 0.0f), 1.0f) * J.Mm1;
    float uhi = fminf(fmaxf((r.y - J.vmin) * J.inv_range, 0.0f), 1.0f) * J.Mm1;
    int ilo = max((int)ulo - 1, 0);
    int ihi = min((int)uhi + 2, J.M - 1);
    mask_all[g] = (prefix[ihi + 1] - prefix[ilo]) == 0;
}

// one thread per super-brick of every mask job (same flags as the
// single-render super mask)
__global__ __launch_bounds__(256) void batch_super(const MaskJob* __restrict__ jobs, int njobs,
                                                   long long total,
                                                   const uint8_t* __restrict__ mask_all,
                                                   uint8_t* __restrict__ super_all) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (jobs[mid].super_off <= g) lo = mid; else hi = mid;
    }
    const MaskJob& J = jobs[lo];
    long long sidx = g - J.super_off;
    if (sidx < 0 || sidx >= J.nsuper) return;
    const uint8_t* mask = mask_all + J.brick_off;
    int sx = (int)(sidx % J.nsx);
    long long rest = sidx / J.nsx;
    int sy = (int)(rest % J.nsy), sz = (int)(rest / J.nsy);
    const bool adaptive = !isnan(J.adapt_range);      // else no brick range is read
    bool all = true, all_poor = adaptive, no_poor = true;
    for (int bz = sz * 4; bz < min(sz * 4 + 4, J.nbz); ++bz)
        for (int by = sy * 4; by < min(sy * 4 + 4, J.nby); ++by)
            for (int bx = sx * 4; bx < min(sx * 4 + 4, J.nbx); ++bx) {
                const long long b = ((long long)bz * J.nby + by) * J.nbx + bx;
                all = all && mask[b] != 0;
                const bool poor = adaptive && brick_poor(J.range[b], J.adapt_range);
                all_poor = all_poor && poor;
                no_poor = no_poor && !poor;
            }
    super_all[g] = (all ? kSuperEmpty : 0) | (all_poor ? kSuperPoor : 0) |
                   (no_poor ? kSuperRich : 0);
}

}  // namespace rc

using namespace rc;

struct rc_batch {
    int n;
    int device;
    rc_batch_config cfg;
    int total_tiles;
    int n_jobs;
    long long total_bricks;
    long long total_super;
    int grid;
    int lds_bytes;              // LDS box budget per wave
    const PersistKernel* kernel;    // the instantiation for the items' kinds
    void* dmem;                 // one allocation holding everything below
    RenderParams* d_items;
    int* d_kinds;
    int* d_tile_off;
    int* d_order;
    int* d_counter;             // kQueues work-queue counters
    MaskJob* d_jobs;
    int* d_prefix;
    uint8_t* d_mask;
    uint8_t* d_super;
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool captured;
};

static bool box_ok(int b) { return b == 0 || (b >= 2048 && b <= 32768 && b % 1024 == 0); }

static rc_status check_config(const rc_batch_config& c) {
    if (c.tile_w != 4 && c.tile_w != 8 && c.tile_w != 16 && c.tile_w != 32)
        return fail(RC_E_INVALID, "batch config: tile_w must be 4, 8, 16 or 32");
    if (c.waves_per_wg != 1 && c.waves_per_wg != 2 && c.waves_per_wg != 4)
        return fail(RC_E_INVALID, "batch config: waves_per_wg must be 1, 2 or 4");
    if (c.wg_per_cu < 1 || c.wg_per_cu > 32)
        return fail(RC_E_INVALID, "batch config: wg_per_cu must be 1..32");
    if (c.order != 0 && c.order != 1) return fail(RC_E_INVALID, "batch config: order must be 0/1");
    if (!box_ok(c.box_bytes_grad) || !box_ok(c.box_bytes_cd))
        return fail(RC_E_INVALID,
                    "batch config: box budgets must be 0 or a multiple of 1024 in 2048..32768");
    if (c.chunk_len != 0 && (c.chunk_len < 4 || c.chunk_len > 64))
        return fail(RC_E_INVALID, "batch config: chunk_len must be 0 or 4..64");
    return RC_OK;
}

static rc_batch_config default_config() { return rc_batch_config{8, 1, 8, 1, 0, 0, 0}; }

// The box budget of an item: FP32 boxes for the 64-voxel stencils, boxes of
// the volume's type for central differences, nothing for unshaded items
// (they read the bricked volume directly).
static int item_box_bytes(const rc_batch_item& it, const rc_batch_config& c) {
    if (it.sh.model == RC_SHADE_NONE) return 16;
    if (it.opt.gradient_op == RC_GRAD_CENTRAL)
        return c.box_bytes_cd ? c.box_bytes_cd : kBatchWaveLdsBytes;
    return c.box_bytes_grad ? c.box_bytes_grad : kWaveLdsBytes;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" rc_status rc_batch_create(const rc_batch_item* items, int n, const rc_batch_config* cfg,
                                     void* stream, rc_batch** out) {
    if (!out) return fail(RC_E_INVALID, "rc_batch_create: out is NULL");
    *out = nullptr;
    if (!items || n < 1 || n > 65536) return fail(RC_E_INVALID, "rc_batch_create: need 1..65536 items");
    rc_batch_config c = cfg ? *cfg : default_config();
    rc_status st = check_config(c);
    if (st != RC_OK) return st;
    std::vector<RenderParams> P(n);
    std::vector<int> kinds(n), tiles(n);
    std::vector<MaskJob> jobs;
    // items of one volume and table (and, for adaptive items, one detail-poor
    // bound) share a mask
    std::vector<int> job_of(n, -1);
    std::map<std::tuple<const void*, const void*, int, uint32_t>, int> job_index;
    long long total_bricks = 0, total_prefix = 0, total_super = 0;
    for (int i = 0; i < n; ++i) {
        const rc_batch_item& it = items[i];
        st = check_render_args(it.vol, &it.cam, it.tf_rgba_dev, it.tf_len, &it.sh, &it.opt);
        if (st != RC_OK) return fail(st, "item %d: %s", i, rc_last_error());
        if (!it.out_rgba_dev) return fail(RC_E_INVALID, "item %d: out_rgba_dev is NULL", i);
        if (it.reserved != 0) return fail(RC_E_INVALID, "item %d: reserved field must be 0", i);
        fill_render_params(P[i], it.vol, &it.cam, it.tf_rgba_dev, it.tf_len, &it.sh, &it.opt);
        set_tiling(P[i].view, c.tile_w);
        P[i].box_bytes = item_box_bytes(it, c);
        P[i].chunk_init = c.chunk_len ? c.chunk_len : kChunkInit;
        P[i].view.out = (float4*)it.out_rgba_dev;
        P[i].view.aux = it.aux_dev;
        kinds[i] = item_kind(it.vol, &it.sh, &it.opt);
        tiles[i] = P[i].view.n_tiles;
        if (it.opt.skip_empty) {
            const float adapt_range = it.opt.adapt_factor > 1 ? it.opt.adapt_range : NAN;
            uint32_t adapt_bits;
            std::memcpy(&adapt_bits, &adapt_range, sizeof(adapt_bits));
            const auto key = std::make_tuple((const void*)it.vol, (const void*)it.tf_rgba_dev,
                                             it.tf_len, adapt_bits);
            const auto found = job_index.find(key);
            if (found != job_index.end()) {
                job_of[i] = found->second;
                continue;
            }
            job_of[i] = (int)jobs.size();
            job_index.emplace(key, job_of[i]);
            MaskJob J;
            J.range = it.vol->brick_range;
            J.tf = (const float4*)it.tf_rgba_dev;
            J.M = it.tf_len;
            J.vmin = it.vol->vmin;
            J.inv_range = (float)(1.0 / ((double)it.vol->vmax - (double)it.vol->vmin));
            J.Mm1 = (float)(it.tf_len - 1);
            J.nbricks = it.vol->nbricks;
            J.brick_off = total_bricks;
            J.prefix_off = total_prefix;
            J.nbx = it.vol->nbx;
            J.nby = it.vol->nby;
            J.nbz = it.vol->nbz;
            J.nsx = it.vol->nsx;
            J.nsy = it.vol->nsy;
            J.nsuper = it.vol->nsuper;
            J.super_off = total_super;
            J.adapt_range = adapt_range;
            total_bricks += J.nbricks;
            total_prefix += it.tf_len + 1;
            total_super += J.nsuper;
            jobs.push_back(J);
        }
    }
    // every wave holds the largest box budget its items use
    int lds_bytes = 16;
    for (int i = 0; i < n; ++i) lds_bytes = std::max(lds_bytes, P[i].box_bytes);
    if ((long long)lds_bytes * c.waves_per_wg > 65536)
        return fail(RC_E_INVALID, "rc_batch_create: %d waves x %d LDS bytes exceed 64 KiB",
                    c.waves_per_wg, lds_bytes);
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    if (c.order == 1)
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return tiles[a] > tiles[b]; });
    std::vector<int> tile_off(n + 1, 0);
    long long total = 0;
    for (int q = 0; q < n; ++q) {
        tile_off[q] = (int)total;
        total += tiles[order[q]];
    }
    tile_off[n] = (int)total;
    if (total >= (1LL << 31)) return fail(RC_E_INVALID, "rc_batch_create: too many tiles");

    size_t o_items = 0;
    size_t o_kinds = align256(o_items + sizeof(RenderParams) * n);
    size_t o_toff = align256(o_kinds + sizeof(int) * n);
    size_t o_order = align256(o_toff + sizeof(int) * (n + 1));
    size_t o_counter = align256(o_order + sizeof(int) * n);
    size_t o_jobs = align256(o_counter + sizeof(int) * kQueues * kQueueStride);
    size_t o_prefix = align256(o_jobs + sizeof(MaskJob) * std::max<size_t>(jobs.size(), 1));
    size_t o_mask = align256(o_prefix + sizeof(int) * std::max<long long>(total_prefix, 1));
    size_t o_super = align256(o_mask + std::max<long long>(total_bricks, 1));
    size_t bytes = align256(o_super + std::max<long long>(total_super, 1));

    rc_batch* b = new (std::nothrow) rc_batch();
    if (!b) return fail(RC_E_OOM, "rc_batch_create: host allocation failed");
    b->n = n;
    b->cfg = c;
    b->total_tiles = (int)total;
    b->n_jobs = (int)jobs.size();
    b->total_bricks = total_bricks;
    b->total_super = total_super;
    b->captured = false;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipMalloc(&b->dmem, bytes);
    if (e != hipSuccess) { delete b; return hip_fail(e, "rc_batch_create: hipMalloc"); }
    char* base = (char*)b->dmem;
    b->d_items = (RenderParams*)(base + o_items);
    b->d_kinds = (int*)(base + o_kinds);
    b->d_tile_off = (int*)(base + o_toff);
    b->d_order = (int*)(base + o_order);
    b->d_counter = (int*)(base + o_counter);
    b->d_jobs = (MaskJob*)(base + o_jobs);
    b->d_prefix = (int*)(base + o_prefix);
    b->d_mask = (uint8_t*)(base + o_mask);
    b->d_super = (uint8_t*)(base + o_super);
    for (int i = 0; i < n; ++i)
        if (job_of[i] >= 0) {
            P[i].empty = b->d_mask + jobs[job_of[i]].brick_off;
            P[i].super_empty = b->d_super + jobs[job_of[i]].super_off;
        }
    hipStream_t s = (hipStream_t)stream;
    e = hipMemcpyAsync(b->d_items, P.data(), sizeof(RenderParams) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_kinds, kinds.data(), sizeof(int) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_tile_off, tile_off.data(), sizeof(int) * (n + 1),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_order, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !jobs.empty())
        e = hipMemcpyAsync(b->d_jobs, jobs.data(), sizeof(MaskJob) * jobs.size(),
                           hipMemcpyHostToDevice, s);
    // the host vectors go out of scope: wait for the copies
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(b->dmem);
        delete b;
        return hip_fail(e, "rc_batch_create: upload");
    }
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e != hipSuccess || cus < 1) cus = 256;
    b->grid = cus * c.wg_per_cu;
    b->lds_bytes = lds_bytes;
    unsigned mask = 0;
    for (int i = 0; i < n; ++i) mask |= 1u << kinds[i];
    b->kernel = &persist_kernel(mask);
    *out = b;
    return RC_OK;
}

static rc_status enqueue_batch(rc_batch* b, hipStream_t s) {
    hipLaunchKernelGGL(batch_reset, dim3(1), dim3(64), 0, s, b->d_counter);
    if (b->n_jobs > 0) {
        hipLaunchKernelGGL(batch_prefix, dim3(b->n_jobs), dim3(256), 0, s, b->d_jobs, b->d_prefix);
        unsigned g = (unsigned)((b->total_bricks + 255) / 256);
        hipLaunchKernelGGL(batch_mask, dim3(g), dim3(256), 0, s, b->d_jobs, b->n_jobs,
                           b->total_bricks, b->d_prefix, b->d_mask);
        g = (unsigned)((b->total_super + 255) / 256);
        hipLaunchKernelGGL(batch_super, dim3(g), dim3(256), 0, s, b->d_jobs, b->n_jobs,
                           b->total_super, b->d_mask, b->d_super);
    }
    hipLaunchKernelGGL(b->kernel->fn, dim3(b->grid), dim3(64 * b->cfg.waves_per_wg),
                       (size_t)b->lds_bytes * b->cfg.waves_per_wg, s,
                       b->d_items, b->d_kinds, b->d_tile_off, b->d_order, b->n, b->total_tiles,
                       b->d_counter, b->lds_bytes);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

// Items already in device memory (built there by the caller's own kernel):
// the queue reset and the persistent launch, one wave per workgroup and as
// many resident per SIMD as the chosen instantiation targets.
rc_status rc::launch_batch_items(const RenderParams* items, const int* kinds, const int* tile_off,
                             const int* order, int n, int total, int* counter, int lds_bytes,
                             unsigned kind_mask, hipStream_t s) {
    // compute units per device, looked up once (threads may race to store
    // the same value)
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int n_cu = cus[dev].load(std::memory_order_relaxed);
    if (n_cu == 0) {
        if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n_cu < 1)
            n_cu = 256;
        cus[dev].store(n_cu, std::memory_order_relaxed);
    }
    const PersistKernel& k = persist_kernel(kind_mask);
    hipLaunchKernelGGL(batch_reset, dim3(1), dim3(64), 0, s, counter);
    hipLaunchKernelGGL(k.fn, dim3((unsigned)(n_cu * 4 * k.waves)), dim3(64), (size_t)lds_bytes,
                       s, items, kinds, tile_off, order, n, total, counter, lds_bytes);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

extern "C" rc_status rc_batch_render(rc_batch* b, int use_graph, void* stream) {
    if (!b) return fail(RC_E_INVALID, "rc_batch_render: batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) return enqueue_batch(b, s);
    if (!s) return fail(RC_E_INVALID, "rc_batch_render: graph mode needs a non-NULL stream");
    if (!b->captured) {
        RC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        rc_status st = enqueue_batch(b, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != RC_OK) { if (g) (void)hipGraphDestroy(g); return st; }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e, "hipGraphInstantiate"); }
        b->graph = g;
        b->captured = true;
    }
    RC_HIP(hipGraphLaunch(b->exec, s));
    return RC_OK;
}

// As rc_destroy_volume: the batch may have been rendered on several
// streams, so its memory is released once its device is idle.
extern "C" void rc_batch_destroy(rc_batch* b) {
    if (!b) return;
    int cur = -1;
    const bool other = hipGetDevice(&cur) == hipSuccess && cur != b->device;
    if (other) (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->captured) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
    }
    (void)hipFree(b->dmem);
    if (other) (void)hipSetDevice(cur);
    delete b;
}

extern "C" rc_status rc_render_batch(const rc_batch_item* items, int n, const rc_batch_config* cfg,
                                     void* stream) {
    rc_batch* b = nullptr;
    rc_status st = rc_batch_create(items, n, cfg, stream, &b);
    if (st != RC_OK) return st;
    st = rc_batch_render(b, 0, stream);
    rc_batch_destroy(b);
    return st;
}

// ---------------------------------------------------------------- autotuner
static unsigned long long fnv1a(const std::string& s) {
    unsigned long long h = 1469598103934665603ULL;
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 1099511628211ULL;
    }
    return h;
}

static std::string batch_key(const rc_batch_item* items, int n) {
    std::string k = "v2;n=" + std::to_string(n) + ";";
    for (int i = 0; i < n; ++i) {
        const rc_batch_item& it = items[i];
        k += std::to_string(it.vol->nx) + "x" + std::to_string(it.vol->ny) + "x" +
             std::to_string(it.vol->nz) + ":" + std::to_string((int)it.vol->dtype) + ":" +
             std::to_string(it.cam.width) + "x" + std::to_string(it.cam.height) + ":" +
             std::to_string(it.opt.gradient_op) + ":" + std::to_string(it.sh.model) + ":" +
             std::to_string(it.opt.skip_empty) + ":" + std::to_string(it.opt.sampling) + ":" +
             std::to_string(it.opt.opacity_ref_step > 0.0f) + ";";
    }
    char buf[32];
    snprintf(buf, sizeof buf, "%016llx", fnv1a(k));
    return buf;
}

static bool read_int(const char* line, const char* name, int* v) {
    std::string pat = std::string("\"") + name + "\":";
    const char* p = strstr(line, pat.c_str());
    return p && sscanf(p + pat.size(), " %d", v) == 1;
}

static bool cache_lookup(const char* path, const std::string& key, rc_batch_config* out) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[768];
    bool found = false;
    std::string needle = "\"key\": \"" + key + "\"";
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, needle.c_str())) continue;
        rc_batch_config c;
        if (read_int(line, "tile_w", &c.tile_w) && read_int(line, "waves_per_wg", &c.waves_per_wg) &&
            read_int(line, "wg_per_cu", &c.wg_per_cu) && read_int(line, "order", &c.order) &&
            read_int(line, "box_bytes_grad", &c.box_bytes_grad) &&
            read_int(line, "box_bytes_cd", &c.box_bytes_cd) &&
            read_int(line, "chunk_len", &c.chunk_len) && check_config(c) == RC_OK) {
            *out = c;
            found = true;
        }
    }
    fclose(f);
    return found;
}

// Time one configuration: a warm-up render, then three timed renders.
static rc_status time_config(const rc_batch_item* items, int n, const rc_batch_config& c,
                             hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* ms) {
    rc_batch* b = nullptr;
    rc_status st = rc_batch_create(items, n, &c, s, &b);
    if (st != RC_OK) return st;
    st = enqueue_batch(b, s);
    if (st == RC_OK && hipEventRecord(e0, s) != hipSuccess) st = RC_E_DEVICE;
    for (int r = 0; r < 3 && st == RC_OK; ++r) st = enqueue_batch(b, s);
    if (st == RC_OK && hipEventRecord(e1, s) != hipSuccess) st = RC_E_DEVICE;
    if (st == RC_OK && hipEventSynchronize(e1) != hipSuccess) st = RC_E_DEVICE;
    if (st == RC_OK && hipEventElapsedTime(ms, e0, e1) != hipSuccess) st = RC_E_DEVICE;
    rc_batch_destroy(b);
    if (st != RC_OK) return fail(st, "rc_batch_autotune: timing failed");
    return RC_OK;
}

extern "C" rc_status rc_batch_autotune(const rc_batch_item* items, int n, const char* cache_path,
                                       void* stream, rc_batch_config* out) {
    if (!out) return fail(RC_E_INVALID, "rc_batch_autotune: out is NULL");
    if (!items || n < 1) return fail(RC_E_INVALID, "rc_batch_autotune: no items");
    for (int i = 0; i < n; ++i)
        if (!items[i].vol) return fail(RC_E_INVALID, "item %d: volume is NULL", i);
    std::string key = batch_key(items, n);
    if (cache_path && cache_lookup(cache_path, key, out)) return RC_OK;
    hipStream_t s = (hipStream_t)stream;
    bool has_grad = false, has_cd = false;
    for (int i = 0; i < n; ++i) {
        if (items[i].sh.model == RC_SHADE_NONE) continue;
        if (items[i].opt.gradient_op == RC_GRAD_CENTRAL) has_cd = true;
        else has_grad = true;
    }
    rc_batch_config best = default_config();
    float best_ms = INFINITY;
    hipEvent_t e0, e1;
    RC_HIP(hipEventCreate(&e0));
    RC_HIP(hipEventCreate(&e1));
    rc_status st = RC_OK;
    auto trial = [&](const rc_batch_config& c) -> rc_status {
        float ms = 0.0f;
        rc_status r = time_config(items, n, c, s, e0, e1, &ms);
        if (r == RC_OK && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        return r;
    };
    // stage 1: launch shape, default boxes
    const int tws[] = {8, 16, 4};
    const int wpw[] = {1, 4};
    const int wpc[] = {4, 8, 16};
    const int ords[] = {1, 0};
    for (int tw : tws)
        for (int w : wpw)
            for (int pc : wpc)
                for (int od : ords)
                    if (st == RC_OK) st = trial(rc_batch_config{tw, w, std::max(1, pc / w), od, 0, 0, 0});
    // stage 2: box budgets of the kinds present (a budget too large for the
    // shape's waves per workgroup is skipped)
    if (st == RC_OK) {
        const rc_batch_config shape = best;
        const int grads[] = {8192, 12288, 16384, 20480};
        const int cds[] = {4096, 8192, 12288};
        for (int g : grads) {
            if (!has_grad && g != grads[0]) break;
            for (int d : cds) {
                if (!has_cd && d != cds[0]) break;
                rc_batch_config c = shape;
                c.box_bytes_grad = has_grad ? g : 0;
                c.box_bytes_cd = has_cd ? d : 0;
                if ((long long)std::max(g, d) * c.waves_per_wg > 65536) continue;
                if (st == RC_OK) st = trial(c);
            }
        }
    }
    // stage 3: first chunk length
    if (st == RC_OK && (has_grad || has_cd)) {
        const rc_batch_config boxes = best;
        for (int len : {8, 32}) {
            rc_batch_config c = boxes;
            c.chunk_len = len;
            if (st == RC_OK) st = trial(c);
        }
    }
    if (st != RC_OK) goto done;
    *out = best;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (!f) { st = fail(RC_E_INVALID, "rc_batch_autotune: cannot write %s", cache_path); goto done; }
        fprintf(f,
                "{\"key\": \"%s\", \"tile_w\": %d, \"waves_per_wg\": %d, \"wg_per_cu\": %d, "
                "\"order\": %d, \"box_bytes_grad\": %d, \"box_bytes_cd\": %d, "
                "\"chunk_len\": %d, \"ms_per_batch\": %.4f, \"items\": %d}\n",
                key.c_str(), best.tile_w, best.waves_per_wg, best.wg_per_cu, best.order,
                best.box_bytes_grad, best.box_bytes_cd, best.chunk_len, best_ms / 3.0f, n);
        fclose(f);
    }
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
