// Host side of the C ABI declared in include/pgh.h: contexts, argument
// checks, the j-memory, the look-up table builder, plans and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pgh_internal.h"
#include "planner.h"

using namespace pgh;

struct pgh_plan {
    pgh_ctx *owner;
    // the plan of a tree's lists, owned by the tree (pgh_tree_plan hands it
    // out read-only; pgh_plan_free rejects it, pgh_tree_free frees it)
    bool tree_owned;
    int n_items, n_tasks;
    int ni_total, nj_total;
    int waves;              // the planner's wave target when the plan was made
    long long interactions;
    int n_chunks, n_slots;  // chunks whose j-list is split, and their parts
    Task *tasks;            // device, sublist-major, each sublist longest first
    // allocated sizes (records) of tasks, partial and chunks: a plan that is
    // filled again (a tree's, at every walk) reuses them when large enough
    size_t tasks_cap, partial_cap, chunks_cap;
    int nq;                 // task sublists
    int q_begin[kQueues + 1];
    unsigned *queue;        // device, one counter per sublist, zero between launches
    float4 *partial;        // device, 64 partial sums per slot
    SplitChunk *chunks;     // device, the split chunks
    // Task lists of the table adjoint, built by its first call on the plan
    // (a forward-only plan never pays for them).
    bool adj_built;
    std::vector<pgh_item> ordered;  // the items with n_i > 0, by i_off
    int n_jtasks;           // j-major tasks of the table adjoint
    Task *jtasks;           // device
    int n_itasks;           // i-major tasks of the table adjoint (i-side positions)
    Task *itasks;           // device
    int2 *irange;           // device, the items' i-ranges (i_off, n_i) by i_off
    int n_irange;
    // the items' j-ranges (j_off, n_j) by j_off, and whether they are
    // disjoint (every j-entry in at most one list: the adjoint then stores
    // the per-entry gradients instead of adding them)
    int2 *jrange;
    int n_jrange;
    bool j_disjoint;
    // the ranges cover every row / entry (no gap to test against them)
    bool i_cover, j_cover;
    // every i-row is in exactly one i-major task of the table adjoint
    bool i_once;
    // partial moments of split chunks (pgh_batch_table_moments), grown on
    // its first call on the plan: two float4 per partial sum
    float4 *mpartial;
    size_t mpartial_cap;
    // device expansion of the compact form (tree plans): the entries, the
    // sort keys and task indices (and their sorted copies), sort temp storage
    PlanDesc *desc;
    unsigned *keys, *keys_out;
    int *vals, *order;
    void *sort_temp;
    size_t desc_cap, keys_cap, keys_out_cap, vals_cap, order_cap, sort_temp_cap;
};

struct pgh_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    float eps2_all = 0.f;
    int nj = 0;
    int jcap = 0;   // allocated j records
    int jfill = 0;  // records written so far (the upper bound of pgh_set_n)
    float4 *jmem = nullptr;
    int refine = 0;  // Newton-Raphson step after v_rsq_f32 (pgh_set_rsqrt_refine)
    int plan_device = 1;  // plans expanded on the device (pgh_set_plan_expansion)
    int plan_waves = 0;   // the planner's wave target (pgh_set_plan_waves; 0: the device's)
    int plan_pack = 0;    // chunks packed across items (pgh_set_plan_packing)
    // look-up table
    int tab_set = 0;
    int tab_E = 0, tab_F = 0;
    float tab_rcut = 0.f;
    float2 *tab = nullptr;  // device, 2^kMaxTableBits entries
    float *gcopy = nullptr;  // device, kGradCopies x 2^(kMaxAdjTableBits+1): table-adjoint scratch
    float2 *ptab = nullptr;  // device, potential table on the force table's bins
    int pot_set = 0;         // ptab matches the current force table
    int variant[4] = {-1, -1, -1, -1};
    // partial sums of j-split all-pairs launches (grown on demand)
    float *part = nullptr;
    size_t part_cap = 0;
    // scratch records of the adjoints (grown on demand)
    float4 *scr_a = nullptr, *scr_b = nullptr;
    size_t scr_a_cap = 0, scr_b_cap = 0;
    std::vector<pgh_plan *> plans;
    std::vector<pgh_tree *> trees;
    // planner output and the pinned host buffer plans are uploaded from
    HostPlan hp;
    DescPlan dp;
    void *pin = nullptr;
    size_t pin_bytes = 0;
    std::string err;
};

struct pgh_tree {
    pgh_ctx *owner;
    TreeState st;
    pgh_plan *plan;  // batched plan of the last walk (in owner->plans)
};

namespace {

// Message of the last failure of a call made without a context.
thread_local std::string g_open_error;

int fail(pgh_ctx *c, int code, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_open_error = msg;
    return code;
}

int hip_fail(pgh_ctx *c, const char *what, hipError_t e)
{
    return fail(c, PGH_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define PGH_HIP(ctx, call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, #call, e_); \
    } while (0)

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1, want;
    explicit DeviceGuard(int dev) : want(dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0 && prev != want) (void)hipSetDevice(prev);
    }
};

double smax_of(int E, int F) { return std::ldexp(1.0, 1 << E) * (2.0 - std::ldexp(1.0, -F)); }

// The FP32 scale c of s = fma(|d|^2, c, 2) (Sec. 3.4.2 with the scale applied
// to |d|^2): (s_max - 2) / rcut^2 rounded to FP32, then raised to the
// smallest FP32 value at which a pair at distance rcut (|d|^2 = fl(rcut^2))
// reaches s_max.  Rounded to nearest, about one cutoff in five would put
// such a pair one FP32 step below s_max, in the next-to-last bin, with a
// force of the size of a rounding instead of zero; since the FMA is monotone
// in |d|^2, every pair at or beyond rcut now clamps to the last node, whose
// entries are zero.
float table_scale(double smax, float rcut)
{
    const float r2 = rcut * rcut;
    float c = (float)((smax - 2.0) / ((double)rcut * (double)rcut));
    while (std::fmaf(r2, c, 2.0f) < (float)smax) c = std::nextafterf(c, INFINITY);
    return c;
}

int check_table_shape(pgh_ctx *c, int E, int F, float rcut)
{
    if (E < 0 || E > 6) return fail(c, PGH_ERANGE, "E must be in [0, 6]");
    if (F < 0 || F > 10) return fail(c, PGH_ERANGE, "F must be in [0, 10]");
    if (E + F > kMaxTableBits) return fail(c, PGH_ERANGE, "E + F must be <= 14");
    if (!(rcut > 0.f) || !std::isfinite(rcut)) return fail(c, PGH_ERANGE, "rcut must be > 0");
    return PGH_OK;
}

void free_plan_memory(pgh_plan *p)
{
    (void)hipFree(p->tasks);
    (void)hipFree(p->queue);
    (void)hipFree(p->partial);
    (void)hipFree(p->chunks);
    (void)hipFree(p->jtasks);
    (void)hipFree(p->itasks);
    (void)hipFree(p->irange);
    (void)hipFree(p->jrange);
    (void)hipFree(p->mpartial);
    (void)hipFree(p->desc);
    (void)hipFree(p->keys);
    (void)hipFree(p->keys_out);
    (void)hipFree(p->vals);
    (void)hipFree(p->order);
    (void)hipFree(p->sort_temp);
}

// Grows a scratch buffer of float4 records (synchronises before freeing).
int ensure_scratch(pgh_ctx *c, float4 **buf, size_t *cap, size_t n)
{
    if (n <= *cap) return PGH_OK;
    const size_t want = std::max(n, *cap * 2);
    float4 *nb = nullptr;
    if (hipMalloc((void **)&nb, want * sizeof(float4)) != hipSuccess)
        return fail(c, PGH_ENOMEM, "hipMalloc(scratch) failed");
    if (*buf) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(*buf);
    }
    *buf = nb;
    *cap = want;
    return PGH_OK;
}

// Upper bound of the partial-sum buffer of j-split launches (floats).
constexpr size_t kMaxSplitFloats = (size_t)64 << 20;

// Scratch of the allocation-free entry point (pgh_calc_newton_noalloc): the
// partial sums of its j-split, in a device array of fixed size that each GPU
// holds for the life of the process.  Host code never passes the array's name
// to a kernel (on the host it is a stand-in, not a device address): the
// device address is looked up once per device, with that device current, and
// kept in g_scratch_ptr.
constexpr size_t kNoAllocFloats = (size_t)1 << 20;  // 4 MiB
static __device__ __align__(256) float scratch[kNoAllocFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {nullptr};

// Looks up this device's copy of the scratch array (device current).
int resolve_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return PGH_ERANGE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return PGH_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PGH_EHIP;
    g_scratch_ptr[device] = (float *)ptr;
    return PGH_OK;
}

int ensure_part(pgh_ctx *c, size_t n)
{
    if (n <= c->part_cap) return PGH_OK;
    float *nb = nullptr;
    if (hipMalloc((void **)&nb, n * sizeof(float)) != hipSuccess)
        return fail(c, PGH_ENOMEM, "hipMalloc(partial sums) failed");
    if (c->part) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->part);
    }
    c->part = nb;
    c->part_cap = n;
    return PGH_OK;
}

int zero_outputs(pgh_ctx *c, int n, float *a, float *b, float *d, float *e)
{
    PGH_HIP(c, launch_fill_zero(n, a, b, d, e, c->stream));
    return PGH_OK;
}

}  // namespace

namespace {

// Grows a device array to at least n records (n + n/4 when it grows; the old
// contents are dropped).
template <class T>
bool grow_records(T **buf, size_t *cap, size_t n)
{
    if (n <= *cap) return true;
    (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    const size_t want = n + n / 4;
    if (hipMalloc((void **)buf, want * sizeof(T)) != hipSuccess) {
        *buf = nullptr;
        return false;
    }
    *cap = want;
    return true;
}

// Drops what a plan holds for its previous items before it is filled
// again: the table adjoint's task lists and the task counts.
void reset_plan(pgh_plan *p)
{
    (void)hipFree(p->jtasks);
    (void)hipFree(p->itasks);
    (void)hipFree(p->irange);
    (void)hipFree(p->jrange);
    p->jtasks = p->itasks = nullptr;
    p->irange = p->jrange = nullptr;
    p->n_irange = p->n_jrange = 0;
    p->j_disjoint = p->i_cover = p->j_cover = p->i_once = false;
    p->adj_built = false;
    p->n_jtasks = p->n_itasks = 0;
    p->n_tasks = 0;
    p->n_chunks = 0;
}

// The context's pinned upload buffer, at least `bytes` long.  Every upload
// from it waits for the stream, so nothing reads the old buffer.
int ensure_pinned(pgh_ctx *c, size_t bytes)
{
    if (bytes <= c->pin_bytes) return PGH_OK;
    (void)hipHostFree(c->pin);
    c->pin = nullptr;
    c->pin_bytes = 0;
    const size_t want = bytes + bytes / 4;
    if (hipHostMalloc(&c->pin, want, hipHostMallocDefault) != hipSuccess) {
        c->pin = nullptr;
        return fail(c, PGH_ENOMEM, "hipHostMalloc(plan upload buffer) failed");
    }
    c->pin_bytes = want;
    return PGH_OK;
}

// The device arrays every plan has: the sublist counters, tasks, partial
// sums and split chunks.
int ensure_plan_arrays(pgh_ctx *c, pgh_plan *p, size_t n_tasks, size_t n_slots, size_t n_split)
{
    const size_t queue_bytes = (size_t)kQueues * kQueueStride * sizeof(unsigned);
    if (!p->queue && hipMalloc((void **)&p->queue, queue_bytes) != hipSuccess) {
        p->queue = nullptr;
        return fail(c, PGH_ENOMEM, "hipMalloc(queue) failed");
    }
    if (!grow_records(&p->tasks, &p->tasks_cap, n_tasks))
        return fail(c, PGH_ENOMEM, "hipMalloc(tasks) failed");
    if (!grow_records(&p->partial, &p->partial_cap, n_slots * 64))
        return fail(c, PGH_ENOMEM, "hipMalloc(partial sums) failed");
    if (!grow_records(&p->chunks, &p->chunks_cap, n_split))
        return fail(c, PGH_ENOMEM, "hipMalloc(split chunks) failed");
    return PGH_OK;
}

void set_plan_counts(pgh_plan *p, int n_items, int ni_total, int nj_total, int n_tasks, int nq,
                     const int *q_begin, long long interactions, int n_split, int n_slots,
                     const std::vector<pgh_item> &ordered)
{
    p->n_items = n_items;
    p->n_tasks = n_tasks;
    p->nq = nq;
    std::copy(q_begin, q_begin + kQueues + 1, p->q_begin);
    p->ni_total = ni_total;
    p->nj_total = nj_total;
    p->interactions = interactions;
    p->n_chunks = n_split;
    p->n_slots = n_slots;
    p->ordered = ordered;
}

// The wave count the planner cuts work for: the context's setting, else the
// resident waves of the batched kernels on this device.
int planner_waves(const pgh_ctx *c)
{
    return c->plan_waves > 0 ? c->plan_waves : batch_resident_waves(c->num_cu);
}

// Plans the items into p on the host, reusing its device arrays when they
// are large enough.  The tasks are written straight into the context's
// pinned buffer and copied from there; waits for the stream.  On failure p
// keeps no tasks.
int plan_fill(pgh_ctx *c, pgh_plan *p, int n_items, const pgh_item *items, int ni_total,
              int nj_total)
{
    HostPlan &hp = c->hp;
    p->waves = planner_waves(c);
    {
        std::string err;
        const int st =
            plan_tasks(items, n_items, ni_total, nj_total, p->waves, hp, err, c->plan_pack != 0);
        if (st) return fail(c, st, err);
    }
    DeviceGuard g(c->device);
    reset_plan(p);
    const size_t n_t = (size_t)hp.n_tasks, n_c = hp.split.size();
    int st = ensure_plan_arrays(c, p, n_t, (size_t)hp.n_slots, n_c);
    if (st) return st;
    st = ensure_pinned(c, n_t * sizeof(Task) + n_c * sizeof(SplitChunk));
    if (st) return st;
    char *pin = (char *)c->pin;
    if (n_t) write_tasks(hp, (Task *)pin);
    if (n_c) std::memcpy(pin + n_t * sizeof(Task), hp.split.data(), n_c * sizeof(SplitChunk));
    if (hipMemsetAsync(p->queue, 0, (size_t)kQueues * kQueueStride * sizeof(unsigned),
                       c->stream) != hipSuccess ||
        (n_t && hipMemcpyAsync(p->tasks, pin, n_t * sizeof(Task), hipMemcpyHostToDevice,
                               c->stream) != hipSuccess) ||
        (n_c && hipMemcpyAsync(p->chunks, pin + n_t * sizeof(Task), n_c * sizeof(SplitChunk),
                               hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipStreamSynchronize(c->stream);  // no copy may still read the pinned buffer
        return fail(c, PGH_EHIP, "uploading the plan failed");
    }
    set_plan_counts(p, n_items, ni_total, nj_total, (int)n_t, hp.nq, hp.q_begin, hp.interactions,
                    (int)n_c, hp.n_slots, hp.ordered);
    return PGH_OK;
}

// The same plan with its tasks expanded on the device from the compact form
// (plan_descs): the host decides the pairing and the cut of each item's
// chunks, the device writes the tasks.  Plans too small for chunks of 64 go
// to plan_fill.  Waits for the stream.
int plan_fill_device(pgh_ctx *c, pgh_plan *p, int n_items, const pgh_item *items, int ni_total,
                     int nj_total)
{
    DescPlan &dp = c->dp;
    p->waves = planner_waves(c);
    // the compact form holds the unpacked cut only
    if (c->plan_pack) return plan_fill(c, p, n_items, items, ni_total, nj_total);
    {
        std::string err;
        const int st = plan_descs(items, n_items, ni_total, nj_total, p->waves, dp, err);
        if (st == kPlanOnHost) return plan_fill(c, p, n_items, items, ni_total, nj_total);
        if (st) return fail(c, st, err);
    }
    DeviceGuard g(c->device);
    reset_plan(p);
    const size_t n_t = (size_t)dp.n_tasks, n_c = (size_t)dp.n_split, n_d = dp.desc.size();
    int st = ensure_plan_arrays(c, p, n_t, (size_t)dp.n_slots, n_c);
    if (st) return st;
    size_t tb = 0;
    PGH_HIP(c, plan_expand_temp_bytes((int)n_t, dp.kmax, &tb));
    char *temp = (char *)p->sort_temp;
    const bool ok = grow_records(&p->desc, &p->desc_cap, n_d) &&
                    grow_records(&p->keys, &p->keys_cap, n_t) &&
                    grow_records(&p->keys_out, &p->keys_out_cap, n_t) &&
                    grow_records(&p->vals, &p->vals_cap, n_t) &&
                    grow_records(&p->order, &p->order_cap, n_t) &&
                    grow_records(&temp, &p->sort_temp_cap, tb);
    p->sort_temp = temp;
    if (!ok) return fail(c, PGH_ENOMEM, "hipMalloc(plan expansion arrays) failed");
    st = ensure_pinned(c, n_d * sizeof(PlanDesc));
    if (st) return st;
    if (n_d) std::memcpy(c->pin, dp.desc.data(), n_d * sizeof(PlanDesc));
    PlanExpandArgs a{};
    a.n_tasks = (int)n_t;
    a.n_desc = (int)n_d;
    a.n_split = (int)n_c;
    a.nq = dp.nq;
    a.desc = p->desc;
    a.part_iters = dp.part_iters;
    a.kmax = dp.kmax;
    a.keys = p->keys;
    a.keys_out = p->keys_out;
    a.vals = p->vals;
    a.order = p->order;
    a.tasks = p->tasks;
    a.split = p->chunks;
    std::copy(dp.q_begin, dp.q_begin + kQueues + 1, a.q_begin);
    if (hipMemsetAsync(p->queue, 0, (size_t)kQueues * kQueueStride * sizeof(unsigned),
                       c->stream) != hipSuccess ||
        (n_d && hipMemcpyAsync(p->desc, c->pin, n_d * sizeof(PlanDesc), hipMemcpyHostToDevice,
                               c->stream) != hipSuccess) ||
        launch_plan_expand(a, p->sort_temp, tb, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipStreamSynchronize(c->stream);  // no copy may still read the pinned buffer
        return fail(c, PGH_EHIP, "expanding the plan failed");
    }
    set_plan_counts(p, n_items, ni_total, nj_total, (int)n_t, dp.nq, dp.q_begin, dp.interactions,
                    (int)n_c, dp.n_slots, dp.ordered);
    return PGH_OK;
}

}  // namespace

extern "C" {

int pgh_version(void) { return 100; }

const char *pgh_last_error(const pgh_ctx *c)
{
    return c ? c->err.c_str() : g_open_error.c_str();
}

int pgh_open(pgh_ctx **out, int device, void *hip_stream)
{
    if (!out) {
        g_open_error = "out is NULL";
        return PGH_EINVAL;
    }
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) {
        g_open_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(e);
        return PGH_EHIP;
    }
    if (device < 0 || device >= ndev) {
        g_open_error = "device index out of range";
        return PGH_ERANGE;
    }
    pgh_ctx *c = new (std::nothrow) pgh_ctx;
    if (!c) {
        g_open_error = "out of host memory";
        return PGH_ENOMEM;
    }
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    DeviceGuard g(device);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        ncu > 0)
        c->num_cu = ncu;
    // the allocation-free entry point's scratch on this device (a failure
    // is reported by that entry point, which then refuses to run)
    (void)resolve_scratch(device);
    e = hipMalloc((void **)&c->tab, sizeof(float2) << kMaxTableBits);
    const size_t gcopy_bytes = (sizeof(float2) << kMaxAdjTableBits) * kGradCopies;
    if (e == hipSuccess) e = hipMalloc((void **)&c->gcopy, gcopy_bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&c->ptab, sizeof(float2) << kMaxPotTableBits);
    if (e != hipSuccess) {
        g_open_error = std::string("hipMalloc(table): ") + hipGetErrorString(e);
        (void)hipFree(c->tab);
        (void)hipFree(c->gcopy);
        (void)hipFree(c->ptab);
        delete c;
        return PGH_ENOMEM;
    }
    // the table adjoint's gradient copies start at zero and are put back to
    // zero by the kernel that sums them (k_table_bwd_tail)
    if (hipMemsetAsync(c->gcopy, 0, gcopy_bytes, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        g_open_error = "clearing the table-gradient scratch failed";
        (void)hipFree(c->tab);
        (void)hipFree(c->gcopy);
        (void)hipFree(c->ptab);
        delete c;
        return PGH_EHIP;
    }
    *out = c;
    return PGH_OK;
}

int pgh_close(pgh_ctx *c)
{
    if (!c) return PGH_OK;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (pgh_tree *t : c->trees) {
        tree_release(t->st);
        delete t;
    }
    for (pgh_plan *p : c->plans) {
        free_plan_memory(p);
        delete p;
    }
    (void)hipFree(c->scr_a);
    (void)hipFree(c->scr_b);
    (void)hipFree(c->part);
    (void)hipFree(c->jmem);
    (void)hipFree(c->tab);
    (void)hipFree(c->gcopy);
    (void)hipFree(c->ptab);
    (void)hipHostFree(c->pin);
    delete c;
    return PGH_OK;
}

int pgh_set_stream(pgh_ctx *c, void *hip_stream)
{
    if (!c) return PGH_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return PGH_OK;
}

int pgh_set_eps_to_all(pgh_ctx *c, float eps)
{
    if (!c) return PGH_EINVAL;
    if (!(eps >= 0.f) || !std::isfinite(eps)) return fail(c, PGH_ERANGE, "eps must be >= 0");
    c->eps2_all = eps * eps;
    return PGH_OK;
}

int pgh_set_n(pgh_ctx *c, int nj)
{
    if (!c) return PGH_EINVAL;
    if (nj < 0 || nj > c->jfill) return fail(c, PGH_ERANGE, "nj exceeds the j-memory filled so far");
    c->nj = nj;
    return PGH_OK;
}

int pgh_set_rsqrt_refine(pgh_ctx *c, int on)
{
    if (!c) return PGH_EINVAL;
    c->refine = on ? 1 : 0;
    return PGH_OK;
}

int pgh_set_plan_expansion(pgh_ctx *c, int on_device)
{
    if (!c) return PGH_EINVAL;
    c->plan_device = on_device ? 1 : 0;
    return PGH_OK;
}

int pgh_set_plan_waves(pgh_ctx *c, int waves)
{
    if (!c) return PGH_EINVAL;
    if (waves < 0) return fail(c, PGH_EINVAL, "the wave target must be >= 0");
    c->plan_waves = waves;
    return PGH_OK;
}

int pgh_get_plan_waves(pgh_ctx *c)
{
    if (!c) return PGH_EINVAL;
    return planner_waves(c);
}

int pgh_set_plan_packing(pgh_ctx *c, int on)
{
    if (!c) return PGH_EINVAL;
    c->plan_pack = on ? 1 : 0;
    return PGH_OK;
}

int pgh_get_plan_packing(pgh_ctx *c)
{
    if (!c) return PGH_EINVAL;
    return c->plan_pack;
}

int pgh_set_xmj(pgh_ctx *c, int adr, int nj, const float *x, const float *y, const float *z,
                const float *m)
{
    if (!c) return PGH_EINVAL;
    if (adr < 0 || nj < 0) return fail(c, PGH_EINVAL, "adr and nj must be >= 0");
    if (nj == 0) return PGH_OK;
    if (!x || !y || !z || !m) return fail(c, PGH_EINVAL, "NULL j-particle array");
    if ((long long)adr + nj > (1LL << 30)) return fail(c, PGH_ERANGE, "j-memory limit is 2^30");
    DeviceGuard g(c->device);
    const int need = adr + nj;
    if (need > c->jcap) {
        const int cap = std::max(need, std::min(2 * c->jcap, 1 << 30));
        float4 *nm = nullptr;
        hipError_t e = hipMalloc((void **)&nm, sizeof(float4) * (size_t)cap);
        if (e != hipSuccess) return fail(c, PGH_ENOMEM, "hipMalloc(j-memory) failed");
        if (c->jmem) {
            PGH_HIP(c, hipMemcpyAsync(nm, c->jmem, sizeof(float4) * (size_t)c->jcap,
                                      hipMemcpyDeviceToDevice, c->stream));
            PGH_HIP(c, hipStreamSynchronize(c->stream));
            (void)hipFree(c->jmem);
        }
        c->jmem = nm;
        c->jcap = cap;
    }
    PGH_HIP(c, launch_pack_j(nj, x, y, z, m, c->jmem + adr, c->stream));
    c->jfill = std::max(c->jfill, need);
    return PGH_OK;
}

int pgh_calc_newton(pgh_ctx *c, int ni, const float *xi, const float *yi, const float *zi,
                    const float *eps2_i, float *ax, float *ay, float *az, float *phi)
{
    if (!c) return PGH_EINVAL;
    if (ni < 0) return fail(c, PGH_EINVAL, "ni must be >= 0");
    if (ni == 0) return PGH_OK;
    if (!xi || !yi || !zi || !ax || !ay || !az)
        return fail(c, PGH_EINVAL, "NULL i-particle or output array");
    DeviceGuard g(c->device);
    if (c->nj == 0) return zero_outputs(c, ni, ax, ay, az, phi);
    NewtonArgs a{ni, xi, yi, zi, eps2_i, c->eps2_all, c->nj, c->jmem, ax, ay, az, phi, 0, nullptr};
    const bool guard = (eps2_i == nullptr) && !(c->eps2_all > 0.f);
    int v = c->variant[PGH_FAMILY_NEWTON_ALLPAIRS];
    if (v < 0) v = newton_allpairs_default(ni, c->nj, c->num_cu);
    const int S = newton_allpairs_split(ni, c->nj, v, kMaxSplitFloats);
    if (S > 1) {
        int st = ensure_part(c, (size_t)S * 4 * ni);
        if (st) return st;
        a.part = c->part;
    }
    PGH_HIP(c, launch_newton_allpairs(a, v, c->refine != 0, guard, S, c->stream));
    return PGH_OK;
}

int pgh_calc_newton_noalloc(pgh_ctx *c, int ni, const float *xi, const float *yi,
                            const float *zi, const float *eps2_i, float *ax, float *ay, float *az,
                            float *phi)
{
    if (!c) return PGH_EINVAL;
    if (ni < 0) return fail(c, PGH_EINVAL, "ni must be >= 0");
    if (ni == 0) return PGH_OK;
    if (!xi || !yi || !zi || !ax || !ay || !az)
        return fail(c, PGH_EINVAL, "NULL i-particle or output array");
    if (c->device < 0 || c->device >= kMaxDevices || !g_scratch_ptr[c->device])
        return fail(c, PGH_ESTATE, "the device's scratch array could not be located at pgh_open");
    DeviceGuard g(c->device);
    if (c->nj == 0) return zero_outputs(c, ni, ax, ay, az, phi);
    NewtonArgs a{ni, xi, yi, zi, eps2_i, c->eps2_all, c->nj, c->jmem, ax, ay, az, phi, 0, nullptr};
    const bool guard = (eps2_i == nullptr) && !(c->eps2_all > 0.f);
    int v = c->variant[PGH_FAMILY_NEWTON_ALLPAIRS];
    if (v < 0) {
        v = newton_allpairs_default(ni, c->nj, c->num_cu);
        // four i-particles per lane take their waves from the j-split, which
        // the array caps: the default here keeps one per lane
        if (v == 3) v = 0;
    }
    // the split is limited to the shares whose partial sums fit the array
    // (S * 4 * ni floats); a launch that cannot be split needs no scratch
    const int S = newton_allpairs_split(ni, c->nj, v, kNoAllocFloats);
    if (S > 1) {
        if ((size_t)S * 4 * (size_t)ni > kNoAllocFloats)
            return fail(c, PGH_ERANGE, "the j-split exceeds the scratch array");
        a.part = g_scratch_ptr[c->device];
    }
    PGH_HIP(c, launch_newton_allpairs(a, v, c->refine != 0, guard, S, c->stream));
    return PGH_OK;
}

// ---------------------------------------------------------------------------
// Look-up table (Sec. 3.4.1)
// ---------------------------------------------------------------------------

double pgh_s2pp_f_over_r(double r, void *user)
{
    const double *p = (const double *)user;
    const double eps = p[0], rcut = p[1];
    if (r >= rcut) return 0.0;
    // S2 force profile R(r, a), Eq. (s2), with x = 2r/a; both polynomial
    // branches over 35 a^2 (continuity at x = 1 and x = 2 fixes this).
    auto R_over_r = [](double rr, double a) {
        const double x = 2.0 * rr / a;
        if (x < 1.0) {
            // (224 x - 224 x^3 + 70 x^4 + 48 x^5 - 21 x^6) / (35 a^2) / r, with x/r = 2/a
            const double poly = 224.0 + x * x * (-224.0 + x * (70.0 + x * (48.0 - 21.0 * x)));
            return poly * (2.0 / a) / (35.0 * a * a);
        }
        if (x < 2.0) {
            const double poly =
                12.0 / (x * x) +
                (-224.0 + x * (896.0 + x * (-840.0 + x * (224.0 + x * (70.0 + x * (-48.0 + 7.0 * x))))));
            return poly / (35.0 * a * a) / rr;
        }
        return 1.0 / (rr * rr * rr);
    };
    return R_over_r(r, eps) - R_over_r(r, rcut);
}

int pgh_table_compute(int E, int F, float rcut, pgh_f_over_r f_over_r, void *user,
                      float *table_out)
{
    if (!f_over_r || !table_out) return fail(nullptr, PGH_EINVAL, "NULL callback or table");
    int st = check_table_shape(nullptr, E, F, rcut);
    if (st) return st;
    const int K = 1 << (E + F);
    const double smax = smax_of(E, F);
    float *t = table_out;
    // Nodes by stepping the FP32 bit pattern of s from 2.0 by one unit of the
    // F-th fraction bit: exactly s_k = 2^{bE+1}(1 + bF/2^F).
    std::vector<double> sk(K);
    unsigned bits;
    const float two = 2.0f;
    std::memcpy(&bits, &two, 4);
    for (int k = 0; k < K; ++k) {
        float s;
        const unsigned b = bits + ((unsigned)k << (23 - F));
        std::memcpy(&s, &b, 4);
        sk[k] = s;
    }
    for (int k = 0; k < K; ++k) {
        const double r = (double)rcut * std::sqrt((sk[k] - 2.0) / (smax - 2.0));
        t[2 * k] = (k == K - 1) ? 0.0f : (float)f_over_r(r, user);
    }
    for (int k = 0; k + 1 < K; ++k)
        t[2 * k + 1] = (float)(((double)t[2 * k + 2] - (double)t[2 * k]) / (sk[k + 1] - sk[k]));
    t[2 * K - 1] = 0.0f;
    return PGH_OK;
}

int pgh_build_table(pgh_ctx *c, int E, int F, float rcut, pgh_f_over_r f_over_r, void *user,
                    float *table_out)
{
    if (!c) return PGH_EINVAL;
    if (!f_over_r) return fail(c, PGH_EINVAL, "NULL callback");
    int st = check_table_shape(c, E, F, rcut);
    if (st) return st;
    std::vector<float> t(2u << (E + F));
    st = pgh_table_compute(E, F, rcut, f_over_r, user, t.data());
    if (st) return fail(c, st, "table computation failed");
    DeviceGuard g(c->device);
    PGH_HIP(c, hipMemcpyAsync(c->tab, t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice,
                              c->stream));
    PGH_HIP(c, hipStreamSynchronize(c->stream));
    c->tab_set = 1;
    c->pot_set = 0;
    c->tab_E = E;
    c->tab_F = F;
    c->tab_rcut = rcut;
    if (table_out) std::memcpy(table_out, t.data(), sizeof(float) * t.size());
    return PGH_OK;
}

int pgh_set_table(pgh_ctx *c, int E, int F, float rcut, const float *table)
{
    if (!c) return PGH_EINVAL;
    if (!table) return fail(c, PGH_EINVAL, "NULL table");
    int st = check_table_shape(c, E, F, rcut);
    if (st) return st;
    DeviceGuard g(c->device);
    PGH_HIP(c, hipMemcpyAsync(c->tab, table, sizeof(float2) << (E + F), hipMemcpyDeviceToDevice,
                              c->stream));
    c->tab_set = 1;
    c->pot_set = 0;
    c->tab_E = E;
    c->tab_F = F;
    c->tab_rcut = rcut;
    return PGH_OK;
}

int pgh_build_pot_table(pgh_ctx *c, pgh_f_over_r pot, void *user, float *table_out)
{
    if (!c) return PGH_EINVAL;
    if (!pot) return fail(c, PGH_EINVAL, "NULL callback");
    if (!c->tab_set) return fail(c, PGH_ESTATE, "set the force table first");
    if (c->tab_E + c->tab_F > kMaxPotTableBits)
        return fail(c, PGH_ERANGE, "a potential table needs E + F <= 13");
    std::vector<float> t(2u << (c->tab_E + c->tab_F));
    // the same nodes and chords as the force table, from p(r) instead of f/r
    int st = pgh_table_compute(c->tab_E, c->tab_F, c->tab_rcut, pot, user, t.data());
    if (st) return fail(c, st, "potential table computation failed");
    DeviceGuard g(c->device);
    PGH_HIP(c, hipMemcpyAsync(c->ptab, t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice,
                              c->stream));
    PGH_HIP(c, hipStreamSynchronize(c->stream));
    c->pot_set = 1;
    if (table_out) std::memcpy(table_out, t.data(), sizeof(float) * t.size());
    return PGH_OK;
}

int pgh_set_pot_table(pgh_ctx *c, const float *table)
{
    if (!c) return PGH_EINVAL;
    if (!table) return fail(c, PGH_EINVAL, "NULL table");
    if (!c->tab_set) return fail(c, PGH_ESTATE, "set the force table first");
    if (c->tab_E + c->tab_F > kMaxPotTableBits)
        return fail(c, PGH_ERANGE, "a potential table needs E + F <= 13");
    DeviceGuard g(c->device);
    PGH_HIP(c, hipMemcpyAsync(c->ptab, table, sizeof(float2) << (c->tab_E + c->tab_F),
                              hipMemcpyDeviceToDevice, c->stream));
    c->pot_set = 1;
    return PGH_OK;
}

int pgh_calc_table(pgh_ctx *c, int ni, const float *xi, const float *yi, const float *zi,
                   float *ax, float *ay, float *az, float *phi)
{
    if (!c) return PGH_EINVAL;
    if (!c->tab_set) return fail(c, PGH_ESTATE, "no force table set");
    if (phi && !c->pot_set) return fail(c, PGH_ESTATE, "no potential table set");
    if (ni < 0) return fail(c, PGH_EINVAL, "ni must be >= 0");
    if (ni == 0) return PGH_OK;
    if (!xi || !yi || !zi || !ax || !ay || !az)
        return fail(c, PGH_EINVAL, "NULL i-particle or output array");
    DeviceGuard g(c->device);
    if (c->nj == 0) return zero_outputs(c, ni, ax, ay, az, phi);
    const double smax = smax_of(c->tab_E, c->tab_F);
    TableArgs a{ni, xi, yi, zi, c->nj, c->jmem, c->tab, c->tab_E, c->tab_F,
                table_scale(smax, c->tab_rcut), (float)smax, ax, ay, az, 0, nullptr,
                phi ? c->ptab : nullptr, phi};
    int v = c->variant[PGH_FAMILY_TABLE_ALLPAIRS];
    if (v < 0) v = table_allpairs_default(ni, c->nj, c->num_cu);
    const int S = table_allpairs_split(a, v, kMaxSplitFloats);
    if (S > 1) {
        int st = ensure_part(c, (size_t)S * 4 * ni);
        if (st) return st;
        a.part = c->part;
    }
    PGH_HIP(c, launch_table_allpairs(a, v, S, c->stream));
    return PGH_OK;
}

int pgh_correct_self_potential(pgh_ctx *c, int n, const float *m, const float *eps2_i,
                               float *phi)
{
    if (!c) return PGH_EINVAL;
    if (n < 0) return fail(c, PGH_EINVAL, "n must be >= 0");
    if (n == 0) return PGH_OK;
    if (!m || !phi) return fail(c, PGH_EINVAL, "NULL mass or potential array");
    DeviceGuard g(c->device);
    PGH_HIP(c, launch_self_potential(n, m, eps2_i, c->eps2_all, phi, c->stream));
    return PGH_OK;
}

int pgh_table_grad_chain(pgh_ctx *c, int E, int F, const float *gtable, float *g0)
{
    if (!c) return PGH_EINVAL;
    int st = check_table_shape(c, E, F, 1.0f);
    if (st) return st;
    if (!gtable || !g0) return fail(c, PGH_EINVAL, "NULL gradient array");
    DeviceGuard g(c->device);
    PGH_HIP(c, launch_table_grad_chain(E, F, gtable, g0, c->stream));
    return PGH_OK;
}

// ---------------------------------------------------------------------------
// Plans and batched launches
// ---------------------------------------------------------------------------

int pgh_plan_create(pgh_ctx *c, int n_items, const pgh_item *items, int ni_total, int nj_total,
                    pgh_plan **out)
{
    if (!c) return PGH_EINVAL;
    if (!out) return fail(c, PGH_EINVAL, "out is NULL");
    *out = nullptr;
    pgh_plan *p = new (std::nothrow) pgh_plan{};
    if (!p) return fail(c, PGH_ENOMEM, "out of host memory");
    p->owner = c;
    const int st = c->plan_device ? plan_fill_device(c, p, n_items, items, ni_total, nj_total)
                                  : plan_fill(c, p, n_items, items, ni_total, nj_total);
    if (st) {
        DeviceGuard g(c->device);
        free_plan_memory(p);
        delete p;
        return st;
    }
    c->plans.push_back(p);
    *out = p;
    return PGH_OK;
}

namespace {

// Frees a plan of the context (a caller's or a tree's) once the stream has
// finished with it.
void destroy_plan(pgh_ctx *c, pgh_plan *p)
{
    auto it = std::find(c->plans.begin(), c->plans.end(), p);
    if (it == c->plans.end()) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_plan_memory(p);
    c->plans.erase(it);
    delete p;
}

}  // namespace

int pgh_plan_free(pgh_ctx *c, pgh_plan *p)
{
    if (!c) return PGH_EINVAL;
    if (!p) return PGH_OK;
    auto it = std::find(c->plans.begin(), c->plans.end(), p);
    if (it == c->plans.end()) return fail(c, PGH_EINVAL, "plan does not belong to this context");
    if (p->tree_owned)
        return fail(c, PGH_EINVAL, "the plan belongs to a tree and is freed with it");
    destroy_plan(c, p);
    return PGH_OK;
}

long long pgh_plan_interactions(const pgh_plan *p) { return p ? p->interactions : 0; }

namespace {

// A plan handle is used only once it is found among the context's live
// plans: a freed or foreign handle is never dereferenced.
int check_plan(pgh_ctx *c, const pgh_plan *p)
{
    if (!p) return fail(c, PGH_EINVAL, "NULL plan");
    if (std::find(c->plans.begin(), c->plans.end(), p) == c->plans.end())
        return fail(c, PGH_EINVAL, "plan does not belong to this context");
    return PGH_OK;
}

// Builds the table adjoint's task lists of a plan (once; allocates and
// waits for the stream).
int build_adjoint_tasks(pgh_ctx *c, pgh_plan *p)
{
    if (p->adj_built) return PGH_OK;
    std::vector<Task> jt, it_tasks;
    plan_adjoint_tasks(p->ordered, p->waves > 0 ? p->waves : planner_waves(c), jt, it_tasks);
    // the items' i-ranges (p->ordered is sorted by i_off), for the i-side
    // gradient formed from the forward's moments
    std::vector<int2> ir, jr;
    ir.reserve(p->ordered.size());
    for (const pgh_item &it : p->ordered) {
        ir.push_back(make_int2(it.i_off, it.n_i));
        if (it.n_j > 0) jr.push_back(make_int2(it.j_off, it.n_j));
    }
    std::sort(jr.begin(), jr.end(), [](const int2 &a, const int2 &b) { return a.x < b.x; });
    bool disjoint = true;
    for (size_t k = 1; k < jr.size(); ++k)
        if ((long long)jr[k - 1].x + jr[k - 1].y > jr[k].x) disjoint = false;
    long long ni_sum = 0, nj_sum = 0;
    for (const int2 &r : ir) ni_sum += r.y;
    for (const int2 &r : jr) nj_sum += r.y;
    if ((!jt.empty() && hipMalloc((void **)&p->jtasks, jt.size() * sizeof(Task)) != hipSuccess) ||
        (!it_tasks.empty() &&
         hipMalloc((void **)&p->itasks, it_tasks.size() * sizeof(Task)) != hipSuccess) ||
        (!ir.empty() && hipMalloc((void **)&p->irange, ir.size() * sizeof(int2)) != hipSuccess) ||
        (!jr.empty() && hipMalloc((void **)&p->jrange, jr.size() * sizeof(int2)) != hipSuccess)) {
        (void)hipFree(p->jtasks);
        (void)hipFree(p->itasks);
        (void)hipFree(p->irange);
        (void)hipFree(p->jrange);
        p->jtasks = p->itasks = nullptr;
        p->irange = p->jrange = nullptr;
        return fail(c, PGH_ENOMEM, "hipMalloc(adjoint tasks) failed");
    }
    if ((!jt.empty() && hipMemcpyAsync(p->jtasks, jt.data(), jt.size() * sizeof(Task),
                                       hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
        (!it_tasks.empty() &&
         hipMemcpyAsync(p->itasks, it_tasks.data(), it_tasks.size() * sizeof(Task),
                        hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
        (!ir.empty() && hipMemcpyAsync(p->irange, ir.data(), ir.size() * sizeof(int2),
                                       hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
        (!jr.empty() && hipMemcpyAsync(p->jrange, jr.data(), jr.size() * sizeof(int2),
                                       hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, PGH_EHIP, "uploading the adjoint tasks failed");
    p->n_jtasks = (int)jt.size();
    p->n_itasks = (int)it_tasks.size();
    p->n_irange = (int)ir.size();
    p->n_jrange = (int)jr.size();
    p->j_disjoint = disjoint;
    // disjoint ranges inside [0, total) whose lengths add up to it cover it
    p->i_cover = ni_sum == p->ni_total;
    p->j_cover = disjoint && nj_sum == p->nj_total;
    // each row in exactly one i-major task (no list cut into parts, no empty
    // list): the i-side gradient is then stored, with no zeroing pass
    p->i_once = p->i_cover;
    if (p->i_once) {
        std::vector<unsigned char> seen((size_t)p->ni_total, 0);
        for (const Task &t : it_tasks)
            for (int r = t.i_off; r < t.i_off + t.n_i; ++r) {
                if (seen[(size_t)r]) p->i_once = false;
                seen[(size_t)r] = 1;
            }
        for (size_t r = 0; r < seen.size() && p->i_once; ++r)
            if (!seen[r]) p->i_once = false;
    }
    p->adj_built = true;
    return PGH_OK;
}

BatchArgs batch_args(pgh_ctx *c, const pgh_plan *p)
{
    BatchArgs a{};
    a.n_tasks = p->n_tasks;
    a.tasks = p->tasks;
    a.nq = p->nq;
    std::copy(p->q_begin, p->q_begin + kQueues + 1, a.q_begin);
    a.queue = p->queue;
    a.partial = p->partial;
    a.n_chunks = p->n_chunks;
    a.chunks = p->chunks;
    a.eps2_all = c->eps2_all;
    a.interactions = p->interactions;
    return a;
}

}  // namespace

int pgh_batch_newton(pgh_ctx *c, const pgh_plan *p, const float *xi, const float *yi,
                     const float *zi, const float *eps2_i, const float *xj, const float *yj,
                     const float *zj, const float *mj, float *ax, float *ay, float *az, float *phi)
{
    if (!c) return PGH_EINVAL;
    int st = check_plan(c, p);
    if (st) return st;
    if (p->n_tasks == 0) return PGH_OK;
    if (!xi || !yi || !zi || !ax || !ay || !az)
        return fail(c, PGH_EINVAL, "NULL i-particle or output array");
    if (p->nj_total > 0 && (!xj || !yj || !zj || !mj))
        return fail(c, PGH_EINVAL, "NULL j-particle array");
    DeviceGuard g(c->device);
    BatchArgs a = batch_args(c, p);
    a.xi = xi, a.yi = yi, a.zi = zi, a.eps2i = eps2_i;
    a.xj = xj, a.yj = yj, a.zj = zj, a.mj = mj;
    a.ax = ax, a.ay = ay, a.az = az, a.phi = phi;
    const bool guard = (eps2_i == nullptr) && !(c->eps2_all > 0.f);
    const int v = std::max(0, c->variant[PGH_FAMILY_NEWTON_BATCH]);
    PGH_HIP(c, launch_newton_batch(a, v, c->refine != 0, guard, c->num_cu, c->stream));
    return PGH_OK;
}

int pgh_batch_table(pgh_ctx *c, const pgh_plan *p, const float *xi, const float *yi,
                    const float *zi, const float *xj, const float *yj, const float *zj,
                    const float *mj, float *ax, float *ay, float *az, float *phi)
{
    if (!c) return PGH_EINVAL;
    int st = check_plan(c, p);
    if (st) return st;
    if (!c->tab_set) return fail(c, PGH_ESTATE, "no force table set");
    if (phi && !c->pot_set) return fail(c, PGH_ESTATE, "no potential table set");
    if (p->n_tasks == 0) return PGH_OK;
    if (!xi || !yi || !zi || !ax || !ay || !az)
        return fail(c, PGH_EINVAL, "NULL i-particle or output array");
    if (p->nj_total > 0 && (!xj || !yj || !zj || !mj))
        return fail(c, PGH_EINVAL, "NULL j-particle array");
    DeviceGuard g(c->device);
    BatchArgs a = batch_args(c, p);
    a.xi = xi, a.yi = yi, a.zi = zi;
    a.xj = xj, a.yj = yj, a.zj = zj, a.mj = mj;
    a.ax = ax, a.ay = ay, a.az = az;
    a.phi = phi;
    a.ptable = phi ? c->ptab : nullptr;
    const double smax = smax_of(c->tab_E, c->tab_F);
    a.table = c->tab;
    a.E = c->tab_E;
    a.F = c->tab_F;
    a.c = table_scale(smax, c->tab_rcut);
    a.smax = (float)smax;
    const int v = c->variant[PGH_FAMILY_TABLE_BATCH];
    PGH_HIP(c, launch_table_batch(a, v < 0 ? table_batch_default() : v, c->num_cu, c->stream));
    return PGH_OK;
}

int pgh_batch_table_moments(pgh_ctx *c, pgh_plan *p, const float *xi, const float *yi,
                            const float *zi, const float *xj, const float *yj, const float *zj,
                            const float *mj, float *ax, float *ay, float *az, float *mom)
{
    if (!c) return PGH_EINVAL;
    int st = check_plan(c, p);
    if (st) return st;
    if (!c->tab_set) return fail(c, PGH_ESTATE, "no force table set");
    if (c->tab_E + c->tab_F > kMaxAdjTableBits)
        return fail(c, PGH_ERANGE, "the table adjoint needs E + F <= 13");
    if (p->n_tasks == 0) return PGH_OK;
    if (!xi || !yi || !zi || !ax || !ay || !az || !mom)
        return fail(c, PGH_EINVAL, "NULL i-particle, output or moment array");
    if (p->nj_total > 0 && (!xj || !yj || !zj || !mj))
        return fail(c, PGH_EINVAL, "NULL j-particle array");
    DeviceGuard g(c->device);
    const size_t n_mp = (size_t)p->n_slots * 64 * 2;
    if (n_mp > p->mpartial_cap) {
        // a smaller array may still be read by launches in flight
        PGH_HIP(c, hipStreamSynchronize(c->stream));
        if (!grow_records(&p->mpartial, &p->mpartial_cap, n_mp))
            return fail(c, PGH_ENOMEM, "hipMalloc(partial moments) failed");
    }
    BatchArgs a = batch_args(c, p);
    a.xi = xi, a.yi = yi, a.zi = zi;
    a.xj = xj, a.yj = yj, a.zj = zj, a.mj = mj;
    a.ax = ax, a.ay = ay, a.az = az;
    const double smax = smax_of(c->tab_E, c->tab_F);
    a.table = c->tab;
    a.E = c->tab_E;
    a.F = c->tab_F;
    a.c = table_scale(smax, c->tab_rcut);
    a.smax = (float)smax;
    a.mom = mom;
    a.mpartial = p->mpartial;
    a.ni_total = p->ni_total;
    PGH_HIP(c, launch_table_batch_moments(a, c->num_cu, c->stream));
    return PGH_OK;
}

int pgh_newton_allpairs_bwd(pgh_ctx *c, int n, const float *x, const float *y, const float *z,
                            const float *m, float eps2, const float *wx, const float *wy,
                            const float *wz, float *gx, float *gy, float *gz, float *gm)
{
    if (!c) return PGH_EINVAL;
    if (n < 0) return fail(c, PGH_EINVAL, "n must be >= 0");
    if (n == 0) return PGH_OK;
    if (!x || !y || !z || !m || !wx || !wy || !wz || !gx || !gy || !gz)
        return fail(c, PGH_EINVAL, "NULL array");
    if (!(eps2 > 0.f) || !std::isfinite(eps2)) return fail(c, PGH_ERANGE, "eps2 must be > 0");
    DeviceGuard g(c->device);
    int st = ensure_scratch(c, &c->scr_a, &c->scr_a_cap, 2 * (size_t)n);
    if (st) return st;
    PGH_HIP(c, launch_pack_xw(n, x, y, z, m, 0.f, wx, wy, wz, c->scr_a, c->stream));
    const int S = adjoint_split(n, n, kMaxSplitFloats);
    if (S > 1 && (st = ensure_part(c, (size_t)S * 4 * n))) return st;
    PGH_HIP(c, launch_newton_allpairs_bwd(n, c->scr_a, eps2, c->refine != 0, gx, gy, gz, gm, S,
                                          c->part, c->stream));
    return PGH_OK;
}

int pgh_newton_ij_bwd(pgh_ctx *c, int ni, const float *xi, const float *yi, const float *zi,
                      const float *eps2_i, int nj, const float *xj, const float *yj,
                      const float *zj, const float *mj, const float *wx, const float *wy,
                      const float *wz, float *gxi, float *gyi, float *gzi, float *gxj,
                      float *gyj, float *gzj, float *gmj)
{
    if (!c) return PGH_EINVAL;
    if (ni < 0 || nj < 0) return fail(c, PGH_EINVAL, "counts must be >= 0");
    const bool want_i = gxi || gyi || gzi;
    const bool want_j = gxj || gyj || gzj;
    if (want_i && !(gxi && gyi && gzi)) return fail(c, PGH_EINVAL, "gxi, gyi, gzi: all or none");
    if (want_j && !(gxj && gyj && gzj)) return fail(c, PGH_EINVAL, "gxj, gyj, gzj: all or none");
    if (ni > 0 && (!xi || !yi || !zi || !wx || !wy || !wz))
        return fail(c, PGH_EINVAL, "NULL i-particle or weight array");
    if (nj > 0 && (!xj || !yj || !zj || !mj)) return fail(c, PGH_EINVAL, "NULL j-particle array");
    if (!eps2_i && !(c->eps2_all > 0.f))
        return fail(c, PGH_ERANGE, "the softening must be > 0 for the adjoint");
    DeviceGuard g(c->device);
    if (ni == 0 || nj == 0) {
        if (want_i) {
            int st = zero_outputs(c, ni, gxi, gyi, gzi, nullptr);
            if (st) return st;
        }
        return zero_outputs(c, nj, gxj, gyj, gzj, gmj);
    }
    int st = ensure_scratch(c, &c->scr_a, &c->scr_a_cap, 2 * (size_t)ni);
    if (st) return st;
    st = ensure_scratch(c, &c->scr_b, &c->scr_b_cap, (size_t)nj);
    if (st) return st;
    PGH_HIP(c, launch_pack_xw(ni, xi, yi, zi, eps2_i, c->eps2_all, wx, wy, wz, c->scr_a, c->stream));
    PGH_HIP(c, launch_pack_j(nj, xj, yj, zj, mj, c->scr_b, c->stream));
    const bool rf = c->refine != 0;
    // the two passes run one after the other on the stream and share the
    // partial-sum buffer
    const int Si = adjoint_split(ni, nj, kMaxSplitFloats);
    const int Sj = adjoint_split(nj, ni, kMaxSplitFloats);
    const size_t need = std::max(Si > 1 ? (size_t)Si * 4 * ni : 0, Sj > 1 ? (size_t)Sj * 4 * nj : 0);
    if (need && (st = ensure_part(c, need))) return st;
    if (want_i)
        PGH_HIP(c, launch_newton_bwd_i(ni, c->scr_a, nj, c->scr_b, rf, gxi, gyi, gzi, Si, c->part,
                                       c->stream));
    if (want_j || gmj)
        PGH_HIP(c, launch_newton_bwd_j(nj, c->scr_b, ni, c->scr_a, rf, gxj, gyj, gzj, gmj, Sj,
                                       c->part, c->stream));
    return PGH_OK;
}

namespace {

int table_bwd(pgh_ctx *c, const pgh_plan *p, const float *xi, const float *yi, const float *zi,
              const float *xj, const float *yj, const float *zj, const float *mj,
              const float *wx, const float *wy, const float *wz, const float *mom,
              float *gtable, float *gmj, float *gxi, float *gyi, float *gzi, float *gxj,
              float *gyj, float *gzj)
{
    if (!c) return PGH_EINVAL;
    int st = check_plan(c, p);
    if (st) return st;
    if (!c->tab_set) return fail(c, PGH_ESTATE, "no force table set");
    if (c->tab_E + c->tab_F > kMaxAdjTableBits)
        return fail(c, PGH_ERANGE, "the table adjoint needs E + F <= 13");
    if ((!gxi) != (!gyi) || (!gxi) != (!gzi) || (!gxj) != (!gyj) || (!gxj) != (!gzj))
        return fail(c, PGH_EINVAL, "position gradients come in x, y, z triples");
    if (!gtable && !gmj && !gxi && !gxj) return PGH_OK;
    if (p->ni_total > 0 && (!xi || !yi || !zi || !wx || !wy || !wz))
        return fail(c, PGH_EINVAL, "NULL i-particle or weight array");
    if (p->nj_total > 0 && (!xj || !yj || !zj || !mj))
        return fail(c, PGH_EINVAL, "NULL j-particle array");
    DeviceGuard g(c->device);
    st = build_adjoint_tasks(c, const_cast<pgh_plan *>(p));
    if (st) return st;
    TableBwdArgs A{};
    A.b = batch_args(c, p);
    A.b.xi = xi, A.b.yi = yi, A.b.zi = zi;
    A.b.xj = xj, A.b.yj = yj, A.b.zj = zj, A.b.mj = mj;
    const double smax = smax_of(c->tab_E, c->tab_F);
    A.b.table = c->tab;
    A.b.E = c->tab_E;
    A.b.F = c->tab_F;
    A.b.c = table_scale(smax, c->tab_rcut);
    A.b.smax = (float)smax;
    A.wx = wx, A.wy = wy, A.wz = wz;
    A.gtable = gtable;
    A.gmj = gmj;
    A.gcopies = c->gcopy;
    A.gxi = gxi, A.gyi = gyi, A.gzi = gzi;
    A.gxj = gxj, A.gyj = gyj, A.gzj = gzj;
    A.ni_total = p->ni_total;
    A.nj_total = p->nj_total;
    A.mom = mom;
    A.irange = p->irange;
    A.n_irange = p->n_irange;
    A.jdisjoint = p->j_disjoint ? 1 : 0;
    A.icover = p->i_cover ? 1 : 0;
    A.jcover = p->j_cover ? 1 : 0;
    A.istore = p->i_once ? 1 : 0;
    A.jrange = p->jrange;
    A.n_jrange = p->n_jrange;
    PGH_HIP(c, launch_table_batch_bwd(A, p->jtasks, p->n_jtasks, p->itasks, p->n_itasks,
                                      c->num_cu, c->stream));
    return PGH_OK;
}

}  // namespace

int pgh_batch_table_bwd(pgh_ctx *c, const pgh_plan *p, const float *xi, const float *yi,
                        const float *zi, const float *xj, const float *yj, const float *zj,
                        const float *mj, const float *wx, const float *wy, const float *wz,
                        float *gtable, float *gmj, float *gxi, float *gyi, float *gzi,
                        float *gxj, float *gyj, float *gzj)
{
    return table_bwd(c, p, xi, yi, zi, xj, yj, zj, mj, wx, wy, wz, nullptr, gtable, gmj, gxi, gyi,
                     gzi, gxj, gyj, gzj);
}

int pgh_batch_table_bwd_moments(pgh_ctx *c, const pgh_plan *p, const float *xi, const float *yi,
                                const float *zi, const float *xj, const float *yj,
                                const float *zj, const float *mj, const float *wx,
                                const float *wy, const float *wz, const float *mom,
                                float *gtable, float *gmj, float *gxi, float *gyi, float *gzi,
                                float *gxj, float *gyj, float *gzj)
{
    if (c && !mom) return fail(c, PGH_EINVAL, "NULL moment array");
    return table_bwd(c, p, xi, yi, zi, xj, yj, zj, mj, wx, wy, wz, mom, gtable, gmj, gxi, gyi,
                     gzi, gxj, gyj, gzj);
}

// ---------------------------------------------------------------------------
// Variants
// ---------------------------------------------------------------------------

int pgh_variant_count(int family)
{
    switch (family) {
        case PGH_FAMILY_NEWTON_ALLPAIRS: return newton_allpairs_variants();
        case PGH_FAMILY_TABLE_ALLPAIRS: return table_allpairs_variants();
        case PGH_FAMILY_NEWTON_BATCH: return newton_batch_variants();
        case PGH_FAMILY_TABLE_BATCH: return table_batch_variants();
        default: return 0;
    }
}

const char *pgh_variant_name(int family, int v)
{
    switch (family) {
        case PGH_FAMILY_NEWTON_ALLPAIRS: return newton_allpairs_variant_name(v);
        case PGH_FAMILY_TABLE_ALLPAIRS: return table_allpairs_variant_name(v);
        case PGH_FAMILY_NEWTON_BATCH: return newton_batch_variant_name(v);
        case PGH_FAMILY_TABLE_BATCH: return table_batch_variant_name(v);
        default: return nullptr;
    }
}

int pgh_set_variant(pgh_ctx *c, int family, int v)
{
    if (!c) return PGH_EINVAL;
    if (family < 0 || family > 3) return fail(c, PGH_ERANGE, "unknown kernel family");
    if (v < -1 || v >= pgh_variant_count(family)) return fail(c, PGH_ERANGE, "unknown variant");
    c->variant[family] = v;
    return PGH_OK;
}

int pgh_get_variant(const pgh_ctx *c, int family)
{
    if (!c || family < 0 || family > 3) return -1;
    return c->variant[family];
}

}  // extern "C"

namespace {

// Times every variant of `family` (one warm-up, then `reps` calls between
// hipEvents on the context stream), keeps the fastest in c->variant and
// returns its index, or restores the previous choice and returns a status.
template <class Call>
int tune_family(pgh_ctx *c, int family, int reps, float *best_ms, Call call)
{
    reps = std::max(1, reps);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = -1;
    float best_t = 0.f;
    const int saved = c->variant[family];
    int status = PGH_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        status = fail(c, PGH_EHIP, "hipEventCreate failed");
    } else {
        const int nv = pgh_variant_count(family);
        // The device raises its clocks over the first milliseconds of work
        // after an idle spell (the first calls of a table sweep ran up to a
        // quarter slower): run the first variant for about 2 ms, in batches
        // of 1, 2, 4 and then 8 calls, before timing any, so that the order
        // of the variants does not favour the later ones.
        c->variant[family] = 0;
        float warm = 0.f;
        if (hipEventRecord(e0, c->stream) != hipSuccess) status = PGH_EHIP;
        for (int w = 0; w < 64 && warm < 2.0f && status == PGH_OK; ++w) {
            for (int k = 0; k < (w < 3 ? 1 << w : 8) && status == PGH_OK; ++k) status = call();
            if (status == PGH_OK && (hipEventRecord(e1, c->stream) != hipSuccess ||
                                     hipEventSynchronize(e1) != hipSuccess ||
                                     hipEventElapsedTime(&warm, e0, e1) != hipSuccess))
                status = fail(c, PGH_EHIP, "warming up for the timing failed");
        }
        for (int v = 0; v < nv && status == PGH_OK; ++v) {
            c->variant[family] = v;
            if ((status = call()) != PGH_OK) break;  // warm-up
            if (hipEventRecord(e0, c->stream) != hipSuccess) status = PGH_EHIP;
            for (int r = 0; r < reps && status == PGH_OK; ++r) status = call();
            if (status == PGH_OK && (hipEventRecord(e1, c->stream) != hipSuccess ||
                                     hipEventSynchronize(e1) != hipSuccess))
                status = fail(c, PGH_EHIP, "timing the variants failed");
            float ms = 0.f;
            if (status == PGH_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
                ms /= reps;
                if (best < 0 || ms < best_t) {
                    best = v;
                    best_t = ms;
                }
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(c->stream);
    if (status != PGH_OK || best < 0) {
        c->variant[family] = saved;
        return status != PGH_OK ? status : fail(c, PGH_EHIP, "no variant could be timed");
    }
    c->variant[family] = best;
    if (best_ms) *best_ms = best_t;
    return best;
}

}  // namespace

extern "C" {

int pgh_autotune(pgh_ctx *c, int family, int ni, const float *xi, const float *yi,
                 const float *zi, int reps, float *best_ms)
{
    if (!c) return PGH_EINVAL;
    if (family != PGH_FAMILY_NEWTON_ALLPAIRS && family != PGH_FAMILY_TABLE_ALLPAIRS)
        return fail(c, PGH_ERANGE, "pgh_autotune tunes the all-pairs families");
    if (ni <= 0 || !xi || !yi || !zi) return fail(c, PGH_EINVAL, "need ni > 0 i-particles");
    if (c->nj <= 0) return fail(c, PGH_ESTATE, "set j-particles (pgh_set_xmj, pgh_set_n) first");
    if (family == PGH_FAMILY_TABLE_ALLPAIRS && !c->tab_set)
        return fail(c, PGH_ESTATE, "no force table set");
    DeviceGuard g(c->device);
    float *out = nullptr;
    if (hipMalloc((void **)&out, 4 * sizeof(float) * (size_t)ni) != hipSuccess)
        return fail(c, PGH_ENOMEM, "hipMalloc(tuning outputs) failed");
    const int r = tune_family(c, family, reps, best_ms, [&]() {
        if (family == PGH_FAMILY_NEWTON_ALLPAIRS)
            return pgh_calc_newton(c, ni, xi, yi, zi, nullptr, out, out + ni, out + 2 * ni,
                                   out + 3 * (size_t)ni);
        return pgh_calc_table(c, ni, xi, yi, zi, out, out + ni, out + 2 * ni, nullptr);
    });
    (void)hipFree(out);
    return r;
}

int pgh_autotune_plan(pgh_ctx *c, int family, const pgh_plan *p, const float *xi,
                      const float *yi, const float *zi, const float *xj, const float *yj,
                      const float *zj, const float *mj, int reps, float *best_ms)
{
    if (!c) return PGH_EINVAL;
    if (family != PGH_FAMILY_NEWTON_BATCH && family != PGH_FAMILY_TABLE_BATCH)
        return fail(c, PGH_ERANGE, "pgh_autotune_plan tunes the batched families");
    if (int st = check_plan(c, p)) return st;
    if (p->ni_total > 0 && (!xi || !yi || !zi)) return fail(c, PGH_EINVAL, "null i-arrays");
    if (p->nj_total > 0 && (!xj || !yj || !zj || !mj)) return fail(c, PGH_EINVAL, "null j-arrays");
    if (family == PGH_FAMILY_TABLE_BATCH && !c->tab_set)
        return fail(c, PGH_ESTATE, "no force table set");
    if (p->n_tasks == 0) return fail(c, PGH_EINVAL, "the plan holds no work to time");
    DeviceGuard g(c->device);
    const size_t ni = (size_t)p->ni_total;
    float *out = nullptr;
    if (hipMalloc((void **)&out, 4 * sizeof(float) * ni) != hipSuccess)
        return fail(c, PGH_ENOMEM, "hipMalloc(tuning outputs) failed");
    const int r = tune_family(c, family, reps, best_ms, [&]() {
        if (family == PGH_FAMILY_NEWTON_BATCH)
            return pgh_batch_newton(c, p, xi, yi, zi, nullptr, xj, yj, zj, mj, out, out + ni,
                                    out + 2 * ni, out + 3 * ni);
        return pgh_batch_table(c, p, xi, yi, zi, xj, yj, zj, mj, out, out + ni, out + 2 * ni,
                               nullptr);
    });
    (void)hipFree(out);
    return r;
}

// ---------------------------------------------------------------------------
// Barnes-Hut tree
// ---------------------------------------------------------------------------

namespace {

// As check_plan: a tree handle is used only once found among the context's
// live trees.
int check_tree(pgh_ctx *c, const pgh_tree *t)
{
    if (!t) return fail(c, PGH_EINVAL, "NULL tree");
    if (std::find(c->trees.begin(), c->trees.end(), t) == c->trees.end())
        return fail(c, PGH_EINVAL, "tree does not belong to this context");
    return PGH_OK;
}

}  // namespace

int pgh_tree_create(pgh_ctx *c, pgh_tree **out)
{
    if (!c) return PGH_EINVAL;
    if (!out) return fail(c, PGH_EINVAL, "out is NULL");
    pgh_tree *t = new (std::nothrow) pgh_tree;
    if (!t) return fail(c, PGH_ENOMEM, "out of host memory");
    t->owner = c;
    t->plan = nullptr;
    c->trees.push_back(t);
    *out = t;
    return PGH_OK;
}

int pgh_tree_free(pgh_ctx *c, pgh_tree *t)
{
    if (!c) return PGH_EINVAL;
    if (!t) return PGH_OK;
    auto it = std::find(c->trees.begin(), c->trees.end(), t);
    if (it == c->trees.end()) return fail(c, PGH_EINVAL, "tree does not belong to this context");
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (t->plan) destroy_plan(c, t->plan);
    tree_release(t->st);
    c->trees.erase(it);
    delete t;
    return PGH_OK;
}

int pgh_tree_build(pgh_ctx *c, pgh_tree *t, int n, const float *x, const float *y,
                   const float *z, const float *m, int n_leaf, int n_crit, int quad)
{
    if (!c) return PGH_EINVAL;
    int st = check_tree(c, t);
    if (st) return st;
    if (n < 0) return fail(c, PGH_EINVAL, "n must be >= 0");
    if (n > 0 && (!x || !y || !z || !m)) return fail(c, PGH_EINVAL, "NULL particle array");
    if (n_leaf < 1 || n_leaf > 64) return fail(c, PGH_ERANGE, "n_leaf must be in [1, 64]");
    if (n_crit < n_leaf) return fail(c, PGH_ERANGE, "n_crit must be >= n_leaf");
    DeviceGuard g(c->device);
    std::string err;
    st = tree_build(t->st, n, x, y, z, m, n_leaf, n_crit, quad, c->num_cu, c->stream, err);
    if (st) return fail(c, st, err);
    return PGH_OK;
}

int pgh_tree_walk(pgh_ctx *c, pgh_tree *t, float theta, int record_src)
{
    if (!c) return PGH_EINVAL;
    int st = check_tree(c, t);
    if (st) return st;
    if (!t->st.built) return fail(c, PGH_ESTATE, "build the tree first");
    if (!(theta >= 0.f) || !std::isfinite(theta)) return fail(c, PGH_ERANGE, "theta must be >= 0");
    DeviceGuard g(c->device);
    // The tree keeps its plan from walk to walk: the plan of the new lists
    // is written into it, reusing its device memory.
    auto drop_plan = [&] {
        if (t->plan) destroy_plan(c, t->plan);
        t->plan = nullptr;
    };
    std::string err;
    st = tree_walk(t->st, theta, record_src, c->num_cu, c->stream, err);
    if (st) {
        drop_plan();
        return fail(c, st, err);
    }
    const TreeState &s = t->st;
    if (s.n_groups > 0) {
        if (!t->plan) {
            t->plan = new (std::nothrow) pgh_plan{};
            if (!t->plan) return fail(c, PGH_ENOMEM, "out of host memory");
            t->plan->owner = c;
            t->plan->tree_owned = true;
            c->plans.push_back(t->plan);
        }
        st = c->plan_device ? plan_fill_device(c, t->plan, s.n_groups, s.host_items.data(), s.n,
                                               (int)s.n_entries)
                            : plan_fill(c, t->plan, s.n_groups, s.host_items.data(), s.n,
                                        (int)s.n_entries);
        if (st) {
            drop_plan();
            t->st.walked = 0;
            return st;
        }
    } else {
        drop_plan();
    }
    return PGH_OK;
}

int pgh_tree_newton(pgh_ctx *c, pgh_tree *t, float *ax, float *ay, float *az, float *phi)
{
    if (!c) return PGH_EINVAL;
    int st = check_tree(c, t);
    if (st) return st;
    if (!t->st.walked) return fail(c, PGH_ESTATE, "walk the tree first");
    const TreeState &s = t->st;
    if (s.n == 0) return PGH_OK;
    if (!ax || !ay || !az) return fail(c, PGH_EINVAL, "NULL output array");
    DeviceGuard g(c->device);
    // the batched kernel writes packed results in key order (coalesced), and
    // one gather per particle puts them in the input order
    BatchArgs a = batch_args(c, t->plan);
    a.xi = s.xs, a.yi = s.ys, a.zi = s.zs, a.eps2i = nullptr;
    a.jxm = s.xmj;
    a.out4 = s.res;
    const bool guard = !(c->eps2_all > 0.f);
    const int v = std::max(0, c->variant[PGH_FAMILY_NEWTON_BATCH]);
    PGH_HIP(c, launch_newton_batch(a, v, c->refine != 0, guard, c->num_cu, c->stream));
    PGH_HIP(c, launch_tree_outputs(s, ax, ay, az, phi, c->stream));
    return PGH_OK;
}

int pgh_tree_stats_get(const pgh_tree *t, pgh_tree_stats *out)
{
    if (!t || !out) return PGH_EINVAL;
    const TreeState &s = t->st;
    out->n = s.n;
    out->n_nodes = s.n_nodes;
    out->n_leaves = s.n_leaves;
    out->depth = s.depth;
    out->n_groups = s.n_groups;
    out->max_level_nodes = s.max_level_nodes;
    out->max_frontier = s.walked ? s.max_frontier : 0;
    out->n_leaf = s.n_leaf;
    out->n_crit = s.n_crit;
    out->quad = s.quad;
    out->walked = s.walked;
    out->theta = s.theta;
    std::copy(s.frame, s.frame + 5, out->frame);
    out->n_entries = s.walked ? s.n_entries : -1;
    out->interactions = s.walked ? s.interactions : 0;
    return PGH_OK;
}

const pgh_plan *pgh_tree_plan(const pgh_tree *t) { return t && t->st.walked ? t->plan : nullptr; }

int pgh_tree_get(pgh_ctx *c, const pgh_tree *t, int field, void *dst, long long capacity,
                 long long *count)
{
    if (!c) return PGH_EINVAL;
    int st = check_tree(c, t);
    if (st) return st;
    const TreeState &s = t->st;
    if (!s.built) return fail(c, PGH_ESTATE, "build the tree first");
    const void *src = nullptr;
    long long n = 0;
    size_t elem = 4;
    const long long npp = s.quad ? 3 : 1;
    const bool list = field >= PGH_TREE_LIST_X && field <= PGH_TREE_LIST_SRC;
    if (list && !s.walked) return fail(c, PGH_ESTATE, "walk the tree first");
    switch (field) {
    case PGH_TREE_PERM: src = s.perm, n = s.n; break;
    case PGH_TREE_KEYS: src = s.key, n = s.n, elem = 8; break;
    case PGH_TREE_X: src = s.xs, n = s.n; break;
    case PGH_TREE_Y: src = s.ys, n = s.n; break;
    case PGH_TREE_Z: src = s.zs, n = s.n; break;
    case PGH_TREE_M: src = s.ms, n = s.n; break;
    case PGH_TREE_NODE_BEGIN: src = s.begin, n = s.n_nodes; break;
    case PGH_TREE_NODE_COUNT: src = s.count, n = s.n_nodes; break;
    case PGH_TREE_NODE_LEVEL: src = s.level, n = s.n_nodes; break;
    case PGH_TREE_NODE_FIRST_CHILD: src = s.first_child, n = s.n_nodes; break;
    case PGH_TREE_NODE_N_CHILD: src = s.n_child, n = s.n_nodes; break;
    case PGH_TREE_NODE_PARENT: src = s.parent, n = s.n_nodes; break;
    case PGH_TREE_MOMENTS: src = s.mom, n = s.n_nodes, elem = sizeof(NodeMoments); break;
    case PGH_TREE_PSEUDO: src = s.pp, n = s.n_nodes * npp, elem = sizeof(float4); break;
    case PGH_TREE_GROUPS: src = s.groups, n = s.n_groups; break;
    case PGH_TREE_ITEMS:
        if (!s.walked) return fail(c, PGH_ESTATE, "walk the tree first");
        src = s.items, n = s.n_groups, elem = sizeof(pgh_item);
        break;
    case PGH_TREE_LIST_X:
    case PGH_TREE_LIST_Y:
    case PGH_TREE_LIST_Z:
    case PGH_TREE_LIST_M: n = s.n_entries; break;  // one component of the packed entries
    case PGH_TREE_LIST_SRC:
        if (!s.record_src) return fail(c, PGH_ESTATE, "walk with record_src to keep sources");
        src = s.src, n = s.n_entries;
        break;
    default: return fail(c, PGH_ERANGE, "unknown tree field");
    }
    if (count) *count = n;
    if (n == 0 || (!dst && capacity == 0)) return PGH_OK;  // a size query
    if (capacity < n) return fail(c, PGH_ERANGE, "destination too small for the tree field");
    if (!dst) return fail(c, PGH_EINVAL, "NULL destination");
    DeviceGuard g(c->device);
    if (field >= PGH_TREE_LIST_X && field <= PGH_TREE_LIST_M) {
        float *tmp = nullptr;
        if (hipMalloc((void **)&tmp, sizeof(float) * (size_t)n) != hipSuccess)
            return fail(c, PGH_ENOMEM, "hipMalloc(list component) failed");
        hipError_t e = launch_list_component(s, field - PGH_TREE_LIST_X, tmp, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst, tmp, sizeof(float) * (size_t)n, hipMemcpyDefault, c->stream);
        const hipError_t e2 = hipStreamSynchronize(c->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return hip_fail(c, "copying a list component", e);
        if (e2 != hipSuccess) return hip_fail(c, "copying a list component", e2);
        return PGH_OK;
    }
    PGH_HIP(c, hipMemcpyAsync(dst, src, elem * (size_t)n, hipMemcpyDefault, c->stream));
    PGH_HIP(c, hipStreamSynchronize(c->stream));
    return PGH_OK;
}

}  // extern "C"
