// Device expansion of the compact form of a batched plan (plan_descs): one
// thread per task finds its entry by a binary search over the entries'
// first task indices and forms its length; a stable radix sort orders the
// tasks longest first; one thread per rank writes the task record to its
// dealt position (and, for part 0 of a cut work, its split chunks).  The
// result is the task list plan_tasks writes on the host.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#define PGH_HD __host__ __device__
#include "plan_expand.h"
#include "pgh_internal.h"

namespace pgh {
namespace {

// the last entry whose first task is <= t (entry 0 starts at task 0)
__device__ __forceinline__ int find_desc(const PlanDesc *desc, int n_desc, int t)
{
    int lo = 0, hi = n_desc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].task0 <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_plan_keys(PlanExpandArgs a)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= a.n_tasks) return;
    const PlanDesc d = a.desc[find_desc(a.desc, a.n_desc, t)];
    int cost = 0, ns = 0, at = 0;
    SplitChunk sc[2];
    (void)desc_task(d, t - d.task0, a.part_iters, &cost, sc, &ns, &at);
    a.keys[t] = a.kmax - (unsigned)cost;
    a.vals[t] = t;
}

__global__ void __launch_bounds__(256) k_plan_write(PlanExpandArgs a)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= a.n_tasks) return;
    const int t = a.order[r];
    if (t < 0 || t >= a.n_tasks) return;
    const PlanDesc d = a.desc[find_desc(a.desc, a.n_desc, t)];
    int cost = 0, ns = 0, at = 0;
    SplitChunk sc[2];
    const Task tk = desc_task(d, t - d.task0, a.part_iters, &cost, sc, &ns, &at);
    const long long pos = dealt_position(r, a.nq, a.q_begin);
    if (pos < a.n_tasks) a.tasks[pos] = tk;
    for (int k = 0; k < ns; ++k)
        if (at + k < a.n_split) a.split[at + k] = sc[k];
}

int bits_for(unsigned v)
{
    int b = 1;
    while (b < 32 && (v >> b)) ++b;
    return b;
}

}  // namespace

hipError_t plan_expand_temp_bytes(int n_tasks, unsigned kmax, size_t *bytes)
{
    *bytes = 0;
    if (n_tasks <= 0) return hipSuccess;
    return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const unsigned *)nullptr,
                                              (unsigned *)nullptr, (const int *)nullptr,
                                              (int *)nullptr, n_tasks, 0, bits_for(kmax));
}

hipError_t launch_plan_expand(PlanExpandArgs a, void *temp, size_t temp_bytes, hipStream_t s)
{
    if (a.n_tasks <= 0) return hipSuccess;
    const int blocks = (a.n_tasks + 255) / 256;
    hipLaunchKernelGGL(k_plan_keys, dim3(blocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, a.keys, a.keys_out, a.vals, a.order,
                                           a.n_tasks, 0, bits_for(a.kmax), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_write, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace pgh
