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
int split_count(int ni, int nj, int ki, int jt, int target_waves, size_t part_cap);
hipError_t launch_combine_split(int n, int S, const float *part, float *ax, float *ay, float *az,
                                float *phi, hipStream_t s);

}  // namespace pgh
