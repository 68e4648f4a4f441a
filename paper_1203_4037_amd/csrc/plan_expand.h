// How a wave's work is cut into tasks, and the compact form of a plan whose
// tasks are expanded on the device: the formulas the host planner applies
// and the device expansion repeats, so both give the same task list.
// Plain C++; a HIP source defines PGH_HD as __host__ __device__ before
// including it.
#pragma once

#include "plan_types.h"

#ifndef PGH_HD
#define PGH_HD
#endif

namespace pgh {

// lanes per i-particle of a chunk of n i-particles
PGH_HD inline int chunk_js(int n) { return n <= 16 ? 4 : (n <= 32 ? 2 : 1); }

// ceil(n / js) for js = 1, 2 or 4
PGH_HD inline long long lane_steps(long long n, int js) { return (n + js - 1) >> (js >> 1); }

// A work (one chunk, or two sharing the wave) whose longer j-list has njm
// entries and js lanes per i-particle runs iters = ceil(njm / js) steps.
// When that exceeds part_iters the lists are cut into `parts` parts of
// `per` entries (a multiple of 64; the last part shorter).
struct WorkCut {
    int parts, per;
    long long iters;
};

PGH_HD inline WorkCut cut_work(int njm, int js, long long part_iters)
{
    const long long iters = lane_steps(njm, js);
    if (iters <= part_iters) return {1, njm, iters};
    long long parts = (iters + part_iters - 1) / part_iters;
    long long per = (njm + parts - 1) / parts;
    per = (per + 63) / 64 * 64;
    parts = (njm + per - 1) / per;
    return {(int)parts, (int)per, iters};
}

// entries of part q of a list of n_j entries cut into parts of per entries,
// and where the part starts (the list's end for the empty parts of the
// shorter list of a pair)
PGH_HD inline int part_len(int n_j, long long per, int q)
{
    const long long r = n_j - (long long)q * per;
    return (int)(r < 0 ? 0 : (r < per ? r : per));
}

PGH_HD inline int part_start(int n_j, long long per, int q)
{
    const long long s = (long long)q * per;
    return (int)(s < n_j ? s : n_j);
}

// Length in lane steps of task q of a work (chunk a of a_n i-particles, and
// a second chunk when paired) cut as c: the key of the longest-first order.
PGH_HD inline int work_task_cost(int a_n, int a_nj, bool pair, int b_nj, const WorkCut &c, int q)
{
    if (c.parts <= 1) return (int)(c.iters > 1 ? c.iters : 1);
    const int la = part_len(a_nj, c.per, q), lb = pair ? part_len(b_nj, c.per, q) : 0;
    return (int)lane_steps(la > lb ? la : lb, pair ? 1 : chunk_js(a_n));
}

// Task q of that work, whose partial sums (when cut) start at slot `slot`.
PGH_HD inline Task work_task(int a_i, int a_n, int a_j, int a_nj, bool pair, int b_i, int b_n,
                             int b_j, int b_nj, const WorkCut &c, int q, int slot)
{
    if (c.parts <= 1) return {a_i, a_n, a_j, a_nj, 0, 1, 0, b_i, b_n, b_j, b_nj, 0};
    const int la = part_len(a_nj, c.per, q), lb = pair ? part_len(b_nj, c.per, q) : 0;
    return {a_i, a_n, a_j + part_start(a_nj, c.per, q), la, q, c.parts, slot,
            b_i, b_n, b_j + (pair ? part_start(b_nj, c.per, q) : 0), lb, 0};
}

// A compact plan entry, in the order the planner creates works: a paired
// work (n_i2 > 0: chunks (i_off, n_i) and (i_off2, n_i2), each under 64
// i-particles, one lane each) or a run of chunks (i_off .. i_off + n_i cut
// into chunks of 64, the last one shorter) against one j-list; with the
// index of its first task, partial-sum slot and split chunk in that order.
struct PlanDesc {
    int i_off, n_i, j_off, n_j;
    int i_off2, n_i2, j_off2, n_j2;
    int task0, slot0, split0, pad;
};
static_assert(sizeof(PlanDesc) == 12 * sizeof(int), "PlanDesc is 48 bytes");

// Task `local` of entry d (0 <= local < its task count): the task record,
// its cost, and for part 0 of a cut work the split chunks it owns
// (*n_split = 0, 1 or 2 written to split[0 ..], *split_at = their index).
PGH_HD inline Task desc_task(const PlanDesc &d, int local, long long part_iters, int *cost,
                             SplitChunk *split, int *n_split, int *split_at)
{
    *n_split = 0;
    *split_at = 0;
    if (d.n_i2 > 0) {
        const WorkCut c = cut_work(d.n_j > d.n_j2 ? d.n_j : d.n_j2, 1, part_iters);
        if (c.parts > 1 && local == 0) {
            split[0] = {d.i_off, d.n_i, d.slot0, c.parts, 0};
            split[1] = {d.i_off2, d.n_i2, d.slot0, c.parts, d.n_i};
            *n_split = 2;
            *split_at = d.split0;
        }
        *cost = work_task_cost(d.n_i, d.n_j, true, d.n_j2, c, local);
        return work_task(d.i_off, d.n_i, d.j_off, d.n_j, true, d.i_off2, d.n_i2, d.j_off2, d.n_j2,
                         c, local, d.slot0);
    }
    const int n_full = d.n_i >> 6, n_last = d.n_i & 63;
    const WorkCut cf = cut_work(d.n_j, 1, part_iters);
    const int full_tasks = n_full * cf.parts;
    int w, q, n;
    WorkCut c;
    if (local < full_tasks) {
        w = local / cf.parts;
        q = local - w * cf.parts;
        n = 64;
        c = cf;
    } else {
        w = n_full;
        q = local - full_tasks;
        n = n_last;
        c = cut_work(d.n_j, chunk_js(n_last), part_iters);
    }
    const int slot = d.slot0 + (cf.parts > 1 ? w * cf.parts : 0);
    if (c.parts > 1 && q == 0) {
        split[0] = {d.i_off + 64 * w, n, slot, c.parts, 0};
        *n_split = 1;
        *split_at = d.split0 + (cf.parts > 1 ? w : 0);
    }
    *cost = work_task_cost(n, d.n_j, false, 0, c, q);
    return work_task(d.i_off + 64 * w, n, d.j_off, d.n_j, false, 0, 0, 0, 0, c, q, slot);
}

// Tasks, partial-sum slots and split chunks of entry d.
PGH_HD inline void desc_counts(const PlanDesc &d, long long part_iters, int *tasks, int *slots,
                               int *splits)
{
    if (d.n_i2 > 0) {
        const WorkCut c = cut_work(d.n_j > d.n_j2 ? d.n_j : d.n_j2, 1, part_iters);
        *tasks = c.parts;
        *slots = c.parts > 1 ? c.parts : 0;
        *splits = c.parts > 1 ? 2 : 0;
        return;
    }
    const int n_full = d.n_i >> 6, n_last = d.n_i & 63;
    const WorkCut cf = cut_work(d.n_j, 1, part_iters);
    *tasks = n_full * cf.parts;
    *slots = cf.parts > 1 ? n_full * cf.parts : 0;
    *splits = cf.parts > 1 ? n_full : 0;
    if (n_last) {
        const WorkCut cl = cut_work(d.n_j, chunk_js(n_last), part_iters);
        *tasks += cl.parts;
        *slots += cl.parts > 1 ? cl.parts : 0;
        *splits += cl.parts > 1 ? 1 : 0;
    }
}

// Final position of the task of rank r of the longest-first order when the
// list is dealt into nq sublists a group of kBatchWaves tasks at a time,
// round-robin (sublist q starts at q_begin[q]).
PGH_HD inline long long dealt_position(long long r, int nq, const int *q_begin)
{
    const long long g = r / kBatchWaves;
    const long long q = nq == kQueues ? g % kQueues : g % nq;
    const long long row = nq == kQueues ? g / kQueues : g / nq;
    return q_begin[q] + row * kBatchWaves + r % kBatchWaves;
}

}  // namespace pgh
