// The j-split of the all-pairs launches (Newton, table, adjoints).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace pgh {

// All-pairs launches split the j-range over S workgroup rows when the i-range
// alone gives too few waves; the shares write partial sums [S][4][ni] that
// k_combine_split adds in order.  The split aims for 8 waves per SIMD of a
// 256-CU part (the most that are resident at 64 VGPRs): gfx950 issues two
// FP32 VALU instructions per cycle pair only from different waves, and with
// 4 waves per SIMD the pair rate of the Newton kernel is about 6% lower
// (N = 262144: 22.4 ms unsplit, 21.1 ms split in 2 or more).
constexpr int kSplitTargetWaves = 8192;

// Issue priority of an all-pairs workgroup from its remaining tiles.  Every
// workgroup has the same work, and a SIMD issues from its oldest ready wave
// first, so without this the workgroups finish in the order they started
// and the last ones run with few waves per SIMD, at a low dual-issue rate.
// Lowering the priority (s_setprio, 3 the highest) as the remaining tiles
// fall below 1/2, 1/4 and 1/8 of all lets the workgroups that are behind
// catch up, so they finish together (N = 262144 Newton, four i-particles per
// lane: 20.4 ms without, 19.0 ms with).
__device__ __forceinline__ void set_tile_prio(int rem, int ntiles)
{
    const int lvl = (2 * rem > ntiles) + (4 * rem > ntiles) + (8 * rem > ntiles);
    if (lvl >= 3)
        __builtin_amdgcn_s_setprio(3);
    else if (lvl == 2)
        __builtin_amdgcn_s_setprio(2);
    else if (lvl == 1)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

int split_count(int ni, int nj, int ki, int jt, int target_waves, size_t part_cap);
hipError_t launch_combine_split(int n, int S, const float *part, float *ax, float *ay, float *az,
                                float *phi, hipStream_t s);

}  // namespace pgh
