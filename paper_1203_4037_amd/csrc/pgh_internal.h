// Internal declarations shared by the host side of the library and the
// kernel translation units.  Not part of the public ABI (include/pgh.h).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pgh.h"
#include "plan_types.h"
#include "split.h"

namespace pgh {

// Largest table the kernels hold in LDS: 2^14 (G0, G1) pairs = 128 KiB of
// the 160 KiB of a gfx950 CU (one workgroup per CU at that size).  With the
// potential table (16 bytes per node) and for the table adjoint (whose LDS
// also holds the table-gradient sums) the limit is 2^13 nodes.
constexpr int kMaxTableBits = 14;
constexpr int kMaxPotTableBits = 13;
constexpr int kMaxAdjTableBits = 13;

// Arguments of the all-pairs Newton kernels.  jmem holds (x, y, z, m)
// records; eps2i may be null (then eps2_all applies to every i).
struct NewtonArgs {
    int ni;
    const float *xi, *yi, *zi, *eps2i;
    float eps2_all;
    int nj;
    const float4 *jmem;
    float *ax, *ay, *az, *phi;
    int jchunk;   // j-particles per workgroup share (set by the launcher)
    float *part;  // partial sums [S][4][ni] when the j-range is split
};

// Arguments of the all-pairs table-force kernels.
struct TableArgs {
    int ni;
    const float *xi, *yi, *zi;
    int nj;
    const float4 *jmem;
    const float2 *table;  // (G0, G1) per node, 2^(E+F) nodes
    int E, F;
    float c;     // (s_max - 2) / rcut^2
    float smax;  // 2^{2^E} (2 - 2^-F)
    float *ax, *ay, *az;
    int jchunk;
    float *part;
    const float2 *ptable;  // (P0, P1) per node of the potential table, or NULL
    float *phi;            // potential output (with ptable), or NULL
};

// Arguments of the persistent batched kernels.
struct BatchArgs {
    int n_tasks;
    const Task *tasks;  // sublist-major: sublist q is tasks[q_begin[q] .. q_begin[q+1])
    int nq;             // sublists in use (<= kQueues, <= n_tasks)
    int q_begin[kQueues + 1];
    unsigned *queue;    // counter of sublist q at queue[q * kQueueStride]; zero between launches
    int n_waves;        // waves in the grid (set by the launcher)
    // 1: every task is assigned statically (set by the launcher when the
    // plan holds few tasks per wave): wave g of G runs the tasks of
    // longest-first ranks g, 2G-1-g, 2G+g, 4G-1-g, ... and the counters are
    // not used; 0: the sublists and their counters
    int static_order;
    int n_chunks;     // split chunks
    const SplitChunk *chunks;
    float4 *partial;  // 64 partial sums per slot of a split chunk
    const float *xi, *yi, *zi, *eps2i;
    float eps2_all;
    const float *xj, *yj, *zj, *mj;
    float *ax, *ay, *az, *phi;
    // table force only
    const float2 *table;
    int E, F;
    float c, smax;
    const float2 *ptable;  // potential table (with phi), or NULL
    // Newton only: NULL, or the j-records packed (x, y, z, m) in place of
    // xj .. mj
    const float4 *jxm;
    // NULL, or packed outputs (ax, ay, az, phi) per i-particle in place of
    // the four arrays (Newton only; the potential is then always computed)
    float4 *out4;
    // table force only: NULL, or the i-side moments of the adjoint,
    // mom[k * ni_total + i] for k = 0 .. 6 (S, Mxx, Mxy, Mxz, Myy, Myz, Mzz),
    // and the partial moments of split chunks (two float4 per partial sum)
    float *mom;
    float4 *mpartial;
    int ni_total;
    // the plan's interactions, and the figures of set_wave_prio that a
    // launcher derives from them: the pair-slots of a quarter of the mean
    // work per wave of the launch and of the plan's mean task (0: wave
    // priorities are left alone)
    long long interactions;
    unsigned long long prio_quarter, prio_task;
};

struct CombineArgs {
    int n_chunks;
    const SplitChunk *chunks;
    const float4 *partial;
    float *ax, *ay, *az, *phi;
    float4 *out4;  // as in BatchArgs
    const float4 *mpartial;  // as in BatchArgs
    float *mom;
    int ni_total;
};

// Copies of the table gradient that the workgroups of the adjoint add into
// (workgroup b into copy b mod kGradCopies), summed in a fixed order at the
// end: one copy would take every workgroup's atomics on the same few bins.
constexpr int kGradCopies = 16;

struct TableBwdArgs {
    BatchArgs b;
    const float *wx, *wy, *wz;
    float *gtable;   // 2K floats
    float *gmj;
    float *gcopies;  // kGradCopies x 2K floats (context scratch)
    float *gxi, *gyi, *gzi;  // i-side position gradient (or NULL)
    // NULL, or the forward's i-side moments (BatchArgs::mom): the i-side
    // position gradient is then formed from them per row, with no i-major
    // pass; the rows of the plan's items are the ranges irange (i_off, n_i)
    // sorted by i_off
    const float *mom;
    const int2 *irange;
    int n_irange;
    // the items' j-ranges (j_off, n_j) sorted by j_off; jdisjoint: no two
    // overlap, so every j-entry is written by one j-major task (stores, no
    // zeroing) and entries outside every range are set to zero at the end
    int jdisjoint;
    const int2 *jrange;
    int n_jrange;
    int icover, jcover;  // the i- (j-) ranges cover every row (entry)
    // every i-row is in exactly one i-major task: the i-side gradient is
    // stored, not added, and needs no zeroing
    int istore;
    float *gxj, *gyj, *gzj;  // j-side position gradient (or NULL)
    int ni_total, nj_total;
};

// Kernel launchers (defined in the .hip files).
hipError_t launch_pack_j(int n, const float *x, const float *y, const float *z, const float *m,
                         float4 *dst, hipStream_t s);
hipError_t launch_fill_zero(int n, float *a, float *b, float *c, float *d, hipStream_t s);
hipError_t launch_self_potential(int n, const float *m, const float *eps2i, float eps2_all,
                                 float *phi, hipStream_t s);
hipError_t launch_table_grad_chain(int E, int F, const float *g, float *out, hipStream_t s);
// Lets a kernel launch with `bytes` of dynamic LDS when that exceeds 64 KiB
// (tables of 2^13 nodes and more); a no-op below.
hipError_t allow_dynamic_lds(const void *kernel, size_t bytes);


int newton_allpairs_variants();
const char *newton_allpairs_variant_name(int v);
int newton_allpairs_default(int ni, int nj, int num_cu);
int newton_allpairs_split(int ni, int nj, int variant, size_t part_cap);
hipError_t launch_newton_allpairs(const NewtonArgs &a, int variant, bool refine, bool guard,
                                  int S, hipStream_t s);

int table_allpairs_variants();
const char *table_allpairs_variant_name(int v);
int table_allpairs_default(int ni, int nj, int num_cu);
int table_allpairs_split(const TableArgs &a, int variant, size_t part_cap);
hipError_t launch_table_allpairs(const TableArgs &a, int variant, int S, hipStream_t s);

int batch_resident_waves(int num_cu);  // waves of the persistent grid
int newton_batch_variants();
const char *newton_batch_variant_name(int v);
int table_batch_variants();
const char *table_batch_variant_name(int v);
int table_batch_default();  // the variant used when none is chosen
// k_combine over the split chunks of a batched launch (after it, same stream)
hipError_t launch_combine(const BatchArgs &a, bool phi, hipStream_t s);
// Device expansion of a compact plan (plan_expand.hip): the tasks of the
// n_desc entries sorted longest first (keys/vals and their sorted copies
// keys_out/order, n_tasks each; a hipCUB radix sort with temp storage of
// plan_expand_temp_bytes) and written to their dealt positions in tasks,
// with the split chunks in split.
struct PlanDesc;
struct PlanExpandArgs {
    int n_tasks, n_desc, n_split, nq;
    const PlanDesc *desc;
    long long part_iters;
    unsigned kmax;
    unsigned *keys, *keys_out;
    int *vals, *order;
    Task *tasks;
    SplitChunk *split;
    int q_begin[kQueues + 1];
};
hipError_t plan_expand_temp_bytes(int n_tasks, unsigned kmax, size_t *bytes);
hipError_t launch_plan_expand(PlanExpandArgs a, void *temp, size_t temp_bytes, hipStream_t s);

hipError_t launch_newton_batch(const BatchArgs &a, int variant, bool refine, bool guard,
                               int num_cu, hipStream_t s);
hipError_t launch_table_batch(const BatchArgs &a, int variant, int num_cu, hipStream_t s);
// The table force with the i-side moments of its adjoint (a.mom, a.mpartial
// set; one i-particle per lane, the paper's (G0, G1) form).
hipError_t launch_table_batch_moments(const BatchArgs &a, int num_cu, hipStream_t s);

// Records of two float4: (x, y, z, s or s_all) and (wx, wy, wz, 0).
hipError_t launch_pack_xw(int n, const float *x, const float *y, const float *z, const float *s,
                          float s_all, const float *wx, const float *wy, const float *wz,
                          float4 *dst, hipStream_t st);
// Adjoint launches: S shares of the summed-over index (see split_count).
int adjoint_split(int n, int m, size_t part_cap);
hipError_t launch_newton_allpairs_bwd(int n, const float4 *rec, float eps2, bool refine, float *gx,
                                      float *gy, float *gz, float *gm, int S, float *part,
                                      hipStream_t s);
hipError_t launch_newton_bwd_i(int ni, const float4 *irec, int nj, const float4 *jmem,
                               bool refine, float *gx, float *gy, float *gz, int S, float *part,
                               hipStream_t s);
hipError_t launch_newton_bwd_j(int nj, const float4 *jmem, int ni, const float4 *irec,
                               bool refine, float *gx, float *gy, float *gz, float *gm, int S,
                               float *part, hipStream_t s);
// Zeroes the accumulated per-entry gradients, then runs both adjoint passes
// in one persistent launch.
hipError_t launch_table_batch_bwd(const TableBwdArgs &a, const Task *jtasks, int n_jtasks,
                                  const Task *itasks, int n_itasks, int num_cu, hipStream_t s);

// ---------------------------------------------------------------------------
// Barnes-Hut tree (tree.hip): device state and the host steps that drive it.
// ---------------------------------------------------------------------------

constexpr int kTreeMaxLevel = 21;   // 21 key bits per axis, 63-bit Morton keys
constexpr int kWalkFrontier = 4096; // nodes per frontier buffer of a walking wave

// FP64 moments of a node about its centre of mass: mass, com, and the second
// moment S = sum m (x - com)(x - com)^T as (xx, yy, zz, xy, xz, yz).
struct NodeMoments {
    double m, cx, cy, cz, sxx, syy, szz, sxy, sxz, syz;
};

struct TreeState {
    // particle arrays, capacity n_cap
    int n_cap = 0;
    unsigned long long *key = nullptr, *key_in = nullptr;
    int *perm = nullptr, *iota = nullptr;
    float *xs = nullptr, *ys = nullptr, *zs = nullptr, *ms = nullptr;
    float4 *xm = nullptr;  // the same particles packed (x, y, z, m)
    float4 *xin = nullptr;  // the input particles packed, in input order
    int *inv = nullptr;     // the key-order rank of each input particle
    float4 *res = nullptr;  // the force in key order (ax, ay, az, phi)
    int *mark = nullptr;  // group id at the first particle of each group, else -1
    // nodes, capacity node_cap (breadth first, each level in key order); the
    // moment, centre-of-mass and walk-record arrays have node_cap entries too,
    // the pseudo-particles 3 node_cap
    int node_cap = 0;
    int *begin = nullptr, *count = nullptr, *level = nullptr, *first_child = nullptr,
        *n_child = nullptr, *parent = nullptr;
    int *nc = nullptr;        // per level: children per node, chunk sums, child bounds
    long long nc_cap = 0;
    NodeMoments *mom = nullptr;
    float4 *com = nullptr;    // FP32 centre of mass per node (w unused)
    int4 *nrec = nullptr;     // walk record per node: begin, count, first child, n_child | level << 16
    float4 *pp = nullptr;     // pseudo-particles (x, y, z, m), npp per node
    // groups, capacity group_cap
    int group_cap = 0;
    int *groups = nullptr;
    float4 *glo = nullptr, *ghi = nullptr;  // bounding boxes of the groups
    long long *glen = nullptr, *goff = nullptr;  // list lengths and offsets (n_groups + 1)
    pgh_item *items = nullptr;  // device copy of the items
    // interaction lists, capacity entry_cap
    long long entry_cap = 0;
    float4 *xmj = nullptr;  // the lists, (x, y, z, m) per entry
    int *src = nullptr;  // entry source (with record_src), capacity src_cap
    long long src_cap = 0;
    // scratch of the library scans and sorts
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    unsigned *word = nullptr;  // 16 words: min/max frame, leaf count, walk overflow, frontier
    int *count_out = nullptr;
    float *rc2 = nullptr;      // (l_L / theta)^2 per level for the walk
    int *lvl = nullptr;        // first node of each level (device), kTreeMaxLevel + 3 entries
    // results of the last build / walk
    int n = 0, n_nodes = 0, n_leaves = 0, depth = 0, n_groups = 0, max_level_nodes = 0;
    int max_frontier = 0;  // largest walk frontier of the last walk
    int level_off[kTreeMaxLevel + 2] = {0};
    float frame[5] = {0, 0, 0, 0, 0};
    int n_leaf = 8, n_crit = 64, quad = 0;
    int built = 0, walked = 0;
    float theta = 0.f;
    int record_src = 0;
    long long n_entries = 0, interactions = 0;
    std::vector<pgh_item> host_items;
};

// Each returns PGH_OK or a status with a message in `err`.  Every step runs on
// stream s and waits for it where a count has to come back to the host.
int tree_build(TreeState &t, int n, const float *x, const float *y, const float *z,
               const float *m, int n_leaf, int n_crit, int quad, int num_cu, hipStream_t s,
               std::string &err);
int tree_walk(TreeState &t, float theta, int record_src, int num_cu, hipStream_t s,
              std::string &err);
void tree_release(TreeState &t);
// Copies component comp (0..3: x, y, z, m) of the list entries to out
// (device float[n_entries]).
hipError_t launch_list_component(const TreeState &t, int comp, float *out, hipStream_t s);
// Writes the force held in t.res (key order) to the caller's arrays in the
// input order (phi may be NULL).
hipError_t launch_tree_outputs(const TreeState &t, float *ax, float *ay, float *az, float *phi,
                               hipStream_t s);

}  // namespace pgh
