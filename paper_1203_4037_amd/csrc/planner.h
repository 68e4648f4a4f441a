// Host planning of batched launches (planner.cpp): plain C++, no HIP types.
#pragma once

#include <string>
#include <vector>

#include "pgh.h"
#include "plan_types.h"

namespace pgh {

// Tasks of a plan as the batched kernels read them.
struct HostPlan {
    std::vector<Task> tasks;        // sublist-major; each sublist longest first
    int nq = 0;                     // sublists in use
    int q_begin[kQueues + 1] = {0}; // sublist q is tasks[q_begin[q] .. q_begin[q + 1])
    std::vector<SplitChunk> split;  // chunks whose j-list is cut into parts
    int n_slots = 0;                // partial-sum slots (64 float4 each) of the parts
    long long interactions = 0;     // sum of n_i n_j
    std::vector<pgh_item> ordered;  // the items with n_i > 0, by i_off
};

// Validates the items (non-negative fields, inside the arrays, disjoint
// i-ranges) and cuts them into wave tasks for a device that holds `waves`
// resident waves of the batched kernel.  Returns PGH_OK, or a status with a
// message in err.
int plan_tasks(const pgh_item *items, int n_items, int ni_total, int nj_total, int waves,
               HostPlan &out, std::string &err);

// Task lists of the table adjoint: j-major (a chunk of j-entries against the
// item's i-range) and i-major (an i-chunk against a j-range).
void plan_adjoint_tasks(const std::vector<pgh_item> &ordered, int waves, std::vector<Task> &out_j,
                        std::vector<Task> &out_i);

}  // namespace pgh
