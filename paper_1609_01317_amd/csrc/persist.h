// The persistent batched kernel: resident waves pull (item, tile) work units
// from one device counter until the queue is empty and render each with the
// instantiation its item's kind selects (Section 3.10: rays are independent,
// so rays of different images can share one launch).
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
template <int WAVES, int... Ks>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) void raycast_batch(
    const RenderParams* __restrict__ items, const int* __restrict__ kinds,
    const int* __restrict__ tile_off, const int* __restrict__ order, int n, int total,
    int* __restrict__ counter, int lds_bytes) {
    extern __shared__ __align__(16) unsigned char lds_all[];
    const int lane = threadIdx.x & 63;
    unsigned char* lds = lds_all + (threadIdx.x >> 6) * lds_bytes;
    for (;;) {
        int w = 0;
        if (lane == 0) w = atomicAdd(counter, 1);
        w = __builtin_amdgcn_readfirstlane(__shfl(w, 0));
        // unsigned: a counter that is not reset (negative) also ends the loop
        if ((unsigned)w >= (unsigned)total) break;
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
