// The persistent batched kernel: resident waves pull (item, tile) work units
// from device work queues until every queue is empty and render each with
// the instantiation its item's kind selects (Section 3.10: rays are
// independent, so rays of different images can share one launch).
//
// Work queues: one per XCD.  The launch's units (items in queue order, each
// item's tiles row by row) are cut into groups of kQueueGroup consecutive
// tiles, dealt round-robin to the kQueues queues: queue q holds groups q,
// q + kQueues, ..., so an XCD renders strips of neighbouring tiles (neighbouring
// rays read the same voxels through that XCD's L2).  A wave takes units from
// the queue of its own XCD (the hardware XCC id), one atomic add per unit,
// and when that queue is empty from the others in turn; it leaves when all
// of them are empty.  Every unit is handed out once; the counters only grow,
// so every wave leaves after at most (units + kQueues) fetches in all, and a
// counter compared unsigned makes a stale or negative start an empty queue
// instead of a loop.  The counters sit kQueueStride ints apart (separate
// memory lines: the atomics of different queues do not serialise on one).
//
// Kind of an item (item_kind): dtype * 3 + gradient operator for shaded
// items (0..8), 9 + dtype for unshaded ones (9..11), 12 + dtype * 3 +
// operator for adaptive sampling (12..20).  The kernel is a template over
// the set of kinds it can render: every kind compiled into one function
// shares that function's register allocation, and with all 21 inlined the
// march spills; a launch therefore uses the smallest compiled set that
// holds its items' kinds (persist_kernel).
#pragma once

#include "adaptive.h"

namespace rc {

constexpr int kNumKinds = 21;

// Unit index of the i-th entry of queue q (i taken as unsigned: a counter that
// was not reset gives an index beyond every launch's units).
__device__ __forceinline__ long long queue_unit(int q, unsigned i) {
    return ((long long)(i / kQueueGroup) * kQueues + q) * kQueueGroup + (i % kQueueGroup);
}

template <int D> struct VoxOf;
template <> struct VoxOf<0> { using type = uint8_t; };
template <> struct VoxOf<1> { using type = uint16_t; };
template <> struct VoxOf<2> { using type = float; };

template <int K>
__device__ __forceinline__ void run_unit(const RenderParams& P, int tile, int lane, void* lds,
                                         int lds_bytes) {
    static_assert(K >= 0 && K < kNumKinds, "item kind");
    if constexpr (K < 9) {
        render_tile<typename VoxOf<K / 3>::type, K % 3, true>(P, P.view, tile, lane, lds,
                                                              lds_bytes);
    } else if constexpr (K < 12) {
        render_tile<typename VoxOf<K - 9>::type, RC_GRAD_CENTRAL, false>(P, P.view, tile, lane,
                                                                        lds, lds_bytes);
    } else {
        adaptive_tile<typename VoxOf<(K - 12) / 3>::type, (K - 12) % 3>(P, P.view, tile, lane, lds,
                                                                     lds_bytes);
    }
}

// The last kind of the set is the fall-through: the host only launches a
// set that holds every kind of the launch's items.
template <int K, int... Ks>
__device__ __forceinline__ void dispatch_unit(int kind, const RenderParams& P, int tile, int lane,
                                              void* lds, int lds_bytes) {
    if constexpr (sizeof...(Ks) == 0) {
        run_unit<K>(P, tile, lane, lds, lds_bytes);
    } else {
        if (kind == K) run_unit<K>(P, tile, lane, lds, lds_bytes);
        else dispatch_unit<Ks...>(kind, P, tile, lane, lds, lds_bytes);
    }
}

// WAVES: waves per SIMD the register allocation targets (3 for shaded
// marches, 6 when the set holds only unshaded kinds).  Each wave of a
// workgroup has its own lds_bytes of dynamic LDS.
// counters: kQueues queue counters (kQueueStride ints apart), all zero at launch.
template <int WAVES, int... Ks>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) void raycast_batch(
    const RenderParams* __restrict__ items, const int* __restrict__ kinds,
    const int* __restrict__ tile_off, const int* __restrict__ order, int n, int total,
    int* __restrict__ counters, int lds_bytes) {
    extern __shared__ __align__(16) unsigned char lds_all[];
    const int lane = threadIdx.x & 63;
    unsigned char* lds = lds_all + (threadIdx.x >> 6) * lds_bytes;
    // XCC_ID (hardware register 20), bits 0..3: this wave's XCD
    const int own = (int)(__builtin_amdgcn_s_getreg((15 << 11) | 20) & (kQueues - 1));
    for (int s = 0; s < kQueues; ++s) {
        const int q = (own + s) & (kQueues - 1);
        for (;;) {
            int i = 0;
            if (lane == 0) i = atomicAdd(counters + q * kQueueStride, 1);
            i = __builtin_amdgcn_readfirstlane(__shfl(i, 0));
            const long long u = queue_unit(q, (unsigned)i);
            // queue entries grow with i: the first beyond the launch empties q
            if (u >= (long long)total) break;
            const int w = (int)u;
            int lo = 0, hi = n;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (tile_off[mid] <= w) lo = mid; else hi = mid;
            }
            const int item = __builtin_amdgcn_readfirstlane(order[lo]);
            const int tile = w - tile_off[lo];
            const int kind = __builtin_amdgcn_readfirstlane(kinds[item]);
            dispatch_unit<Ks...>(kind, items[item], tile, lane, lds, lds_bytes);
        }
    }
}

using PersistFn = void (*)(const RenderParams*, const int*, const int*, const int*, int, int, int*,
                           int);

struct PersistKernel {
    unsigned mask;          // kinds the instantiation renders (bit k = kind k)
    int waves;              // its waves per SIMD
    PersistFn fn;
};

// The instantiation with the fewest kinds whose set holds every kind in
// `mask` (the generic one holds all).
const PersistKernel& persist_kernel(unsigned mask);

}  // namespace rc
