// Task queues of the persistent batched kernels (interaction lists of
// Sec. 5.1): which sublist a wave serves and the order it takes tasks in.
//
// The host deals a plan's longest-first task list into up to kQueues
// sublists; workgroup b serves sublist b mod nq together with the other
// workgroups of that residue.  The first round of a sublist is static (its
// w-th wave takes its w-th task), so a sublist with no more tasks than waves
// issues no atomic at all; later tasks come from the sublist's counter, one
// atomic per task, taken at the start of the previous task so that its
// latency overlaps that task.  Every executed task pops exactly once, so the
// pops of a sublist return 0 .. n-1; the wave that draws n-1 knows no pop
// follows and puts the counter back to zero, so the next launch (or a replay
// of a captured graph) starts from zero with no reset kernel or memset.
#pragma once

#include <hip/hip_runtime.h>

#include "pgh_internal.h"
#ifndef PGH_HD
#define PGH_HD __host__ __device__
#endif
#include "plan_expand.h"

namespace pgh {

struct TaskStream {
    const Task *tasks;  // the sublist's tasks, longest first
    unsigned n_tasks;
    unsigned *counter;  // the sublist's counter, zero between launches
    unsigned nw_q;      // waves serving the sublist
    bool dynamic;       // more tasks than waves: later tasks come from the counter
};

__device__ __forceinline__ TaskStream task_stream(const BatchArgs &a, int waves_per_block)
{
    TaskStream ts;
    const unsigned nq = (unsigned)a.nq;
    const unsigned q = blockIdx.x % nq;
    ts.nw_q = ((gridDim.x - q + nq - 1) / nq) * (unsigned)waves_per_block;
    ts.tasks = a.tasks + a.q_begin[q];
    ts.n_tasks = (unsigned)(a.q_begin[q + 1] - a.q_begin[q]);
    ts.counter = a.queue + q * kQueueStride;
    ts.dynamic = ts.n_tasks > ts.nw_q;
    return ts;
}

// The index (in its sublist) of the wave's first task; wave-uniform.
__device__ __forceinline__ unsigned first_task(const BatchArgs &a, int waves_per_block, int wave)
{
    return __builtin_amdgcn_readfirstlane((blockIdx.x / (unsigned)a.nq) * waves_per_block + wave);
}

// Takes the ticket of the wave's next task (lane 0 issues the atomic): the
// index of that task in lane 0, n_tasks (none) when the sublist is static.
// Call with every lane active; the caller reads lane 0's value with
// readfirstlane once the atomic has returned.
__device__ __forceinline__ unsigned pop_task(const TaskStream &ts, int lane)
{
    unsigned tn = ts.n_tasks;
    if (ts.dynamic && lane == 0) {
        const unsigned k =
            __hip_atomic_fetch_add(ts.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == ts.n_tasks - 1u)  // the sublist's last pop in this launch
            __hip_atomic_store(ts.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tn = ts.nw_q + k;
    }
    return tn;
}

// The 12 fields of task t fetched with one vector load (field k in lane k),
// so the next task's fields are in flight while the current task runs
// (scalar loads after the task would make the next task wait for them, and
// scalar loads inside the pair loop would hold up its LDS waits, which share
// their counter).
__device__ __forceinline__ int task_fields(const TaskStream &ts, unsigned t, int lane)
{
    int fld = 0;
    if (t < ts.n_tasks && lane < 12) fld = ((const int *)(ts.tasks + t))[lane];
    return fld;
}

__device__ __forceinline__ Task task_of_fields(int fld)
{
    Task tk;
    tk.i_off = __builtin_amdgcn_readlane(fld, 0);
    tk.n_i = __builtin_amdgcn_readlane(fld, 1);
    tk.j_off = __builtin_amdgcn_readlane(fld, 2);
    tk.n_j = __builtin_amdgcn_readlane(fld, 3);
    tk.part = __builtin_amdgcn_readlane(fld, 4);
    tk.n_parts = __builtin_amdgcn_readlane(fld, 5);
    tk.slot = __builtin_amdgcn_readlane(fld, 6);
    tk.i_off2 = __builtin_amdgcn_readlane(fld, 7);
    tk.n_i2 = __builtin_amdgcn_readlane(fld, 8);
    tk.j_off2 = __builtin_amdgcn_readlane(fld, 9);
    tk.n_j2 = __builtin_amdgcn_readlane(fld, 10);
    tk.pad = 0;
    return tk;
}

// The static order (BatchArgs::static_order): round k of wave g of G runs
// the task of longest-first rank k G + g (k even) or k G + G - 1 - g (k odd),
// so each wave's rounds pair long tasks with short ones; the index of that
// rank in the dealt task array, or n_tasks when the wave has no round k.
__device__ __forceinline__ unsigned static_task(const BatchArgs &a, unsigned k, unsigned g,
                                                unsigned G)
{
    const unsigned long long r = (unsigned long long)k * G + ((k & 1u) ? G - 1u - g : g);
    if (r >= (unsigned long long)a.n_tasks) return (unsigned)a.n_tasks;
    return (unsigned)dealt_position((long long)r, a.nq, a.q_begin);
}

// The number of rounds of wave g of G in the static order over n tasks.
__device__ __forceinline__ unsigned static_rounds(unsigned n, unsigned g, unsigned G)
{
    const unsigned k = n / G, rest = n % G;
    return k + ((((k & 1u) ? G - 1u - g : g) < rest) ? 1u : 0u);
}

// Issue priority by remaining work.  A SIMD issues from its oldest ready
// wave first, so in a launch of about one task per wave the waves that
// arrived first finish well ahead of the last ones, which then end the
// launch running alone at a low issue rate.  Instead each wave sets its
// priority (s_setprio, 3 the highest) at every tile from the pair-slots it
// still has to process (rem: the rest of its task, and in the static order
// its later tasks at the plan's mean task size) against quarters of the
// launch's mean per wave: the waves with the most work left issue first, and
// the waves of a SIMD finish close together.  quarter = 0: no change.
__device__ __forceinline__ void set_wave_prio(unsigned long long rem, unsigned long long quarter)
{
    if (quarter == 0) return;
    const int lvl = (rem > quarter) + (rem > 2 * quarter) + (rem > 3 * quarter);
    if (lvl >= 3)
        __builtin_amdgcn_s_setprio(3);
    else if (lvl == 2)
        __builtin_amdgcn_s_setprio(2);
    else if (lvl == 1)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

// LDS operations of one wave complete in order; this keeps the compiler
// from moving reads of a wave's tile above the writes of its other lanes.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Coordinate of padding j-records: far enough that every pair term with them
// is finite and multiplied by a zero mass, small enough that its square
// stays finite in FP32.
constexpr float kFar = 1.0e10f;

}  // namespace pgh
