// The stencil variants the host may run and their launcher.  All give
// bitwise-identical fields; they differ in tile shape, steps per launch and
// speed (tiled depth-only kernels: stencil.hip; nodal: nodal.hip; tile in LDS
// over several steps, both media: blocked.hip; whole solves in LDS: resident.hip).
#include "internal.h"

namespace eig {

const StencilVariant kVariants[kNumVariants] = {
    {64, 32, EIG_MEDIUM_LAYERED, 1},   // 0: one node per lane
    {128, 32, EIG_MEDIUM_LAYERED, 1, 1},  // 1: two nodes per lane, prefetch 1
    {128, 32, EIG_MEDIUM_LAYERED, 1, 1},  // 2: two nodes per lane, prefetch 2
    {128, 64, EIG_MEDIUM_LAYERED, 1, 1},  // 3: prefetch 2
    {128, 16, EIG_MEDIUM_LAYERED, 1, 1},  // 4: prefetch 2
    {128, 64, EIG_MEDIUM_LAYERED, 1, 1},  // 5: prefetch 1
    {64, 32, EIG_MEDIUM_NODAL, 1},     // 6: nodal media
    {128, 8, EIG_MEDIUM_LAYERED, 1, 1},   // 7: prefetch 2
    {128, 16, EIG_MEDIUM_LAYERED, 1, 1},  // 8: prefetch 1
    {128, 16, EIG_MEDIUM_LAYERED, 2},  // 9: two steps per launch
    {128, 32, EIG_MEDIUM_LAYERED, 2},  // 10: two steps per launch
    {128, 64, EIG_MEDIUM_LAYERED, 2},  // 11: two steps per launch
    {128, 128, EIG_MEDIUM_LAYERED, 2}, // 12: two steps per launch
    {128, 64, EIG_MEDIUM_LAYERED, 2},  // 13: two steps, halo columns up front
    {128, 32, EIG_MEDIUM_LAYERED, 2},  // 14: two steps, halo columns up front
    {128, 64, EIG_MEDIUM_LAYERED, 3},  // 15: three steps per launch
    {128, 32, EIG_MEDIUM_LAYERED, 3},  // 16: three steps per launch
    {128, 16, EIG_MEDIUM_NODAL, 1, 1},    // 17: nodal media, two nodes per lane
    {128, 32, EIG_MEDIUM_NODAL, 1, 1},    // 18: nodal media, two nodes per lane
    {128, 16, EIG_MEDIUM_NODAL, 2},    // 19: nodal media, two steps per launch
    {128, 32, EIG_MEDIUM_NODAL, 2},    // 20: nodal media, two steps per launch
    {0, 0, EIG_MEDIUM_LAYERED, 1, 1, 1},  // 21: resident in LDS, every step in one launch
    {0, 0, EIG_MEDIUM_NODAL, 1, 1, 1},    // 22: resident in LDS, every step in one launch
    {58, 58, EIG_MEDIUM_LAYERED, 4},   // 23: four steps per launch, tile in LDS
    {58, 34, EIG_MEDIUM_NODAL, 4},     // 24: nodal, four steps, tile and medium in LDS
    {64, 24, EIG_MEDIUM_NODAL, 4, 0, 0, 1},  // 25: the same, operands read per node (forced only)
};

void launch_stencil(const SolveDesc* descs, const int2* tiles, int ntiles, int step,
                    int variant, hipStream_t s) {
    if (ntiles <= 0) return;
    if (kVariants[variant].steps == 4)
        launch_blocked_stencil(descs, tiles, ntiles, step, variant, s);
    else if (kVariants[variant].medium_kind == EIG_MEDIUM_NODAL)
        launch_nodal_stencil(descs, tiles, ntiles, step, variant, s);
    else
        launch_layered_stencil(descs, tiles, ntiles, step, variant, s);
}

}  // namespace eig
