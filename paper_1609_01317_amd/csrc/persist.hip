// Instantiations of the persistent batched kernel (persist.h) and the choice
// of one per launch.  Compiled sets: every single kind (the views of one
// volume share one), the three shaded kinds of each voxel type (an orbit
// rendered with the three gradient operators), central differences over
// every voxel type, all shaded kinds, and all kinds.  Sets of unshaded kinds
// only target six waves per SIMD (they carry no gradient state), the rest
// three.
#include "persist.h"

namespace rc {

#define RC_SINGLE(K, W) PersistKernel{1u << (K), W, &raycast_batch<W, K>}

static const PersistKernel kPersist[] = {
    RC_SINGLE(0, 3), RC_SINGLE(1, 3), RC_SINGLE(2, 3), RC_SINGLE(3, 3), RC_SINGLE(4, 3),
    RC_SINGLE(5, 3), RC_SINGLE(6, 3), RC_SINGLE(7, 3), RC_SINGLE(8, 3),
    RC_SINGLE(9, 6), RC_SINGLE(10, 6), RC_SINGLE(11, 6),
    RC_SINGLE(12, 3), RC_SINGLE(13, 3), RC_SINGLE(14, 3), RC_SINGLE(15, 3), RC_SINGLE(16, 3),
    RC_SINGLE(17, 3), RC_SINGLE(18, 3), RC_SINGLE(19, 3), RC_SINGLE(20, 3),
    PersistKernel{0x7u, 3, &raycast_batch<3, 0, 1, 2>},
    PersistKernel{0x38u, 3, &raycast_batch<3, 3, 4, 5>},
    PersistKernel{0x1C0u, 3, &raycast_batch<3, 6, 7, 8>},
    PersistKernel{0x49u, 3, &raycast_batch<3, 0, 3, 6>},
    PersistKernel{0x1FFu, 3, &raycast_batch<3, 0, 1, 2, 3, 4, 5, 6, 7, 8>},
    PersistKernel{(1u << kNumKinds) - 1u, 3,
                  &raycast_batch<3, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16,
                                 17, 18, 19, 20>},
};

#undef RC_SINGLE

const PersistKernel& persist_kernel(unsigned mask) {
    const PersistKernel* best = &kPersist[sizeof(kPersist) / sizeof(kPersist[0]) - 1];
    for (const PersistKernel& k : kPersist)
        if ((k.mask & mask) == mask && __builtin_popcount(k.mask) < __builtin_popcount(best->mask))
            best = &k;
    return *best;
}

}  // namespace rc
