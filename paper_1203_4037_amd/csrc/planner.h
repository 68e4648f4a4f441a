// Host planning of batched launches (planner.cpp): plain C++, no HIP types.
#pragma once

#include <string>
#include <vector>

#include "pgh.h"
#include "plan_expand.h"
#include "plan_types.h"

namespace pgh {

// A chunk of at most 64 i-particles of one item (js lanes per i-particle).
struct PlanChunk {
    int i_off, n_i, j_off, n_j, js;
};

// A wave's work: one chunk, or two that share the wave (b < 0: one), and
// how its j-list is cut: `parts` parts of `per` entries (the last shorter),
// whose partial sums take slots [slot, slot + parts) when parts > 1.
struct PlanWork {
    int a, b;
    int parts, per, slot;
};

// One task before it is written out: part `part` of work `work`.
struct PlanRef {
    int work, part;
};

// A plan of batched launches.  plan_tasks fills it; write_tasks writes its
// n_tasks task records (so the caller can put them straight into memory of
// its choice, such as a pinned upload buffer).
struct HostPlan {
    int n_tasks = 0;
    int nq = 0;                     // sublists in use
    int q_begin[kQueues + 1] = {0}; // sublist q is tasks [q_begin[q], q_begin[q + 1])
    std::vector<SplitChunk> split;  // chunks whose j-list is cut into parts
    int n_slots = 0;                // partial-sum slots (64 float4 each) of the parts
    long long interactions = 0;     // sum of n_i n_j
    std::vector<pgh_item> ordered;  // the items with n_i > 0, by i_off
    // what write_tasks reads
    std::vector<PlanChunk> chunks;
    std::vector<PlanWork> work;
    std::vector<PlanRef> dealt;     // the tasks in their final order
};

// Validates the items (non-negative fields, inside the arrays, disjoint
// i-ranges) and cuts them into wave tasks for a device that holds `waves`
// resident waves of the batched kernel.  Returns PGH_OK, or a status with a
// message in err.
int plan_tasks(const pgh_item *items, int n_items, int ni_total, int nj_total, int waves,
               HostPlan &out, std::string &err, bool pack = false);

// Writes the plan's hp.n_tasks tasks to dst, sublist after sublist, each
// sublist longest first.
void write_tasks(const HostPlan &hp, Task *dst);

// The compact form of a plan (plan_descs): the works of plan_tasks grouped
// into entries whose tasks the device expands, sorts longest first and
// deals into the same sublists, giving the same task list as plan_tasks.
struct DescPlan {
    std::vector<PlanDesc> desc;
    int n_tasks = 0, n_slots = 0, n_split = 0;
    int nq = 0;
    int q_begin[kQueues + 1] = {0};
    long long part_iters = 0;       // the part length of cut_work
    unsigned kmax = 0;              // every task cost is at most kmax
    long long interactions = 0;
    std::vector<pgh_item> ordered;  // the items with n_i > 0, by i_off
};

// plan_descs' status when the plan should be made by plan_tasks instead
// (chunks of 64 would fill less than the device's resident waves)
constexpr int kPlanOnHost = 1;

// Validates the items as plan_tasks does and makes the compact form of the
// same plan.  Returns PGH_OK, kPlanOnHost, or an error status with a
// message in err.
int plan_descs(const pgh_item *items, int n_items, int ni_total, int nj_total, int waves,
               DescPlan &out, std::string &err);

// Task lists of the table adjoint: j-major (a chunk of j-entries against the
// item's i-range) and i-major (an i-chunk against a j-range).
void plan_adjoint_tasks(const std::vector<pgh_item> &ordered, int waves, std::vector<Task> &out_j,
                        std::vector<Task> &out_i);

}  // namespace pgh
