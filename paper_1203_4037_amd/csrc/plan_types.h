// Task records of batched plans and the queue constants they are dealt by:
// shared by the host planner (plain C++) and the kernels.
#pragma once

namespace pgh {

// One wavefront task of a batch plan: up to 64 i-particles against one part
// of one j-list.  A chunk whose j-list is cut into n_parts > 1 parts owns
// n_parts consecutive slots of 64 partial sums starting at `slot`.
// A paired task (n_i2 > 0) also carries a second, unsplit chunk: lanes
// [0, n_i) take the first list and lanes [n_i, n_i + n_i2) the second
// (i_off2, j_off2, n_j2), one lane per i-particle, so two partly filled
// chunks share one wavefront.
struct Task {
    int i_off, n_i, j_off, n_j;
    int part, n_parts, slot;
    int i_off2, n_i2, j_off2, n_j2;
    int pad;
};
static_assert(sizeof(Task) == 12 * sizeof(int), "the batched kernel loads a task as 12 ints");

// A chunk of i-particles whose j-list is split into parts; its partial sums
// sit in lanes [lane0, lane0 + n_i) of its slots (lane0 > 0 for the second
// chunk of a paired task).
struct SplitChunk {
    int i_off, n_i, slot, n_parts, lane0;
};

// Task queues of a plan: the longest-first task list is dealt round-robin
// into kQueues sublists, each with its own counter on its own 128-byte line
// (one device-scope counter saturates at some tens of pops per microsecond).
constexpr int kQueues = 16;
constexpr int kQueueStride = 32;  // unsigned words between counters
constexpr int kBatchWaves = 4;    // wave64s per workgroup of the persistent kernels

}  // namespace pgh
