// Interaction lists in one persistent launch (tree / TreePM groups of
// Sec. 5.1: many i-groups, each with its own j-list).
//
// Work decomposition (built on the host by pgh_plan_create):
//   * an item (i-group, j-list) is cut into wave tasks of at most 64
//     i-particles; a chunk of <= 32 (<= 16) i-particles is computed by 2 (4)
//     lanes per i-particle that take alternate j-particles, so small groups
//     still fill the wavefront;
//   * a long j-list is cut into parts so no task is much longer than the
//     average work of a wave; the parts of one chunk write partial sums to
//     the plan's scratch, and a small second kernel adds them in part order
//     (deterministic) and writes the outputs;
//   * tasks are sorted by decreasing length (longest-processing-time first).
// Execution: a grid sized to fill every CU (or smaller, when there are fewer
// tasks than resident waves); the task list is dealt into up to 16
// sublists, each served by the workgroups b = q mod nq through its own
// counter.  Each wave64 runs independently, taking its first task of the
// sublist by its index and later ones from the sublist's counter with one
// atomic each.  Every task executed pops exactly once, so the pops of a
// sublist return 0 .. n-1; the wave that draws n-1 knows no pop follows and
// puts the counter back to zero, so the next launch (or a replay of a
// captured graph) starts from zero with no reset kernel or memset.  The
// second kernel runs only when some list is split.
//
// Each wave stages its j-list through its own LDS slice, 64 records per
// tile (one coalesced load per coordinate array), double-buffered in
// registers; the pair arithmetic is the one of the all-pairs kernels.  The
// table force over the same plans is k_batch_table (batch_table.hip).
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "batch_queue.h"
#include "newton_pair.h"

namespace pgh {
namespace {

constexpr int kWaves = kBatchWaves;

// REFINE: the Newton-Raphson step after v_rsq_f32; GUARD: zero softening
// (a coincident pair adds nothing); PHI: the potential; RCP: rho^2 from
// v_rcp_f32; U: pairs per lane unrolled in a full tile.
template <bool RCP, bool REFINE, bool GUARD, bool PHI, int U>
__global__ void __launch_bounds__(256, 8) k_batch(BatchArgs a)
{
    // [wave][buffer][list][record], double-buffered
    __shared__ float4 jt[kWaves][2][2][64];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const float mscale = REFINE ? -0.5f : 1.0f;

    const TaskStream ts = task_stream(a, kWaves);
    unsigned t = first_task(a, kWaves, wave);
    Task tk_next{};
    if (t < ts.n_tasks) tk_next = ts.tasks[t];

    while (t < ts.n_tasks) {
        const Task tk = tk_next;
        const unsigned tn = pop_task(ts, lane);

        // lane -> (list, i slot, j phase).  A plain task runs js lanes per
        // i-particle (js = 4, 2 for chunks of <= 16, <= 32) taking alternate
        // j-particles; a paired task runs its two chunks side by side, one
        // lane per i-particle, each lane over its own list.
        const bool paired = tk.n_i2 > 0;
        int jlog = 0, il = lane, ph = 0;  // js = 1 << jlog
        const bool second = paired && lane >= tk.n_i;
        if (paired) {
            il = second ? lane - tk.n_i : lane;
        } else {
            jlog = tk.n_i <= 16 ? 2 : (tk.n_i <= 32 ? 1 : 0);
            il = lane & (63 >> jlog);
            ph = lane >> (6 - jlog);
        }
        const int js = 1 << jlog;
        const bool active = il < (second ? tk.n_i2 : tk.n_i);
        const int i = (second ? tk.i_off2 : tk.i_off) + (active ? il : 0);

        const float px = a.xi[i], py = a.yi[i], pz = a.zi[i];
        const float pe = a.eps2i ? a.eps2i[i] : a.eps2_all;

        float tx = 0.f, ty = 0.f, tz = 0.f, tp = 0.f;
        const int nj = paired ? max(tk.n_j, tk.n_j2) : tk.n_j;
        const int ntiles = (nj + 63) >> 6;

        // j records of a tile, one per lane (and one of the second list);
        // entries past a list's end are zero-mass records far away, whose
        // terms are exactly zero even for zero softening
        float4 pre, pre2;
        auto load = [&](int tile) {
            const int jj = tile * 64 + lane;
            auto record = [&](int j) {
                if (a.jxm) {  // packed j-records
                    float4 v = a.jxm[j];
                    v.w *= mscale;
                    return v;
                }
                return make_float4(a.xj[j], a.yj[j], a.zj[j], a.mj[j] * mscale);
            };
            pre = make_float4(kFar, kFar, kFar, 0.f);
            if (jj < tk.n_j) pre = record(tk.j_off + jj);
            if (paired) {
                pre2 = make_float4(kFar, kFar, kFar, 0.f);
                if (jj < tk.n_j2) pre2 = record(tk.j_off2 + jj);
            }
        };
        auto store = [&](int b) {
            jt[wave][b][0][lane] = pre;
            if (paired) jt[wave][b][1][lane] = pre2;
        };
        const int list = second ? 1 : 0;  // this lane's list
        load(0);
        // vmcnt(0): the i-particle and first-tile loads (and the ticket's
        // atomic).  Waiting here keeps the compiler from placing a full wait
        // inside the pair loop, where it would also wait for the prefetch of
        // the next tile.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        const unsigned t_next = __builtin_amdgcn_readfirstlane(tn);
        const int fld = task_fields(ts, t_next, lane);
        store(0);
        wave_sync();
        for (int tile = 0; tile < ntiles; ++tile) {
            const int cur = tile & 1;
            if (tile + 1 < ntiles) load(tile + 1);
            const float4 *src = jt[wave][cur][list];
            const int cnt = min(64, nj - tile * 64);
            // every lane runs the same trip count; records past cnt are padding
            const int trips = (cnt + js - 1) >> jlog;
            float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f;
            if (cnt == 64) {
                // a full tile: 64 / js records per lane from this lane's
                // phase, with the stride a compile-time constant so the LDS
                // reads take immediate offsets
                auto full_tile = [&](auto stride) {
                    constexpr int S = decltype(stride)::value;
                    const float4 *b = src + ph;
#pragma unroll U
                    for (int it = 0; it < 64 / S; ++it)
                        newton_pair<REFINE, GUARD, PHI, RCP>(b[it * S], px, py, pz, pe, sx, sy,
                                                             sz, sp);
                };
                if (jlog == 0)
                    full_tile(std::integral_constant<int, 1>{});
                else if (jlog == 1)
                    full_tile(std::integral_constant<int, 2>{});
                else
                    full_tile(std::integral_constant<int, 4>{});
            } else {
#pragma unroll 2
                for (int it = 0; it < trips; ++it)
                    newton_pair<REFINE, GUARD, PHI, RCP>(src[it * js + ph], px, py, pz, pe, sx, sy,
                                                         sz, sp);
            }
            tx += sx;
            ty += sy;
            tz += sz;
            tp += sp;
            if (tile + 1 < ntiles) store(cur ^ 1);
            wave_sync();
        }

        // combine the j phases of each i-particle
        if (js >= 4) {
            tx += __shfl_xor(tx, 16);
            ty += __shfl_xor(ty, 16);
            tz += __shfl_xor(tz, 16);
            tp += __shfl_xor(tp, 16);
        }
        if (js >= 2) {
            tx += __shfl_xor(tx, 32);
            ty += __shfl_xor(ty, 32);
            tz += __shfl_xor(tz, 32);
            tp += __shfl_xor(tp, 32);
        }
        const float ascale = (REFINE && !RCP) ? 0.25f : 1.0f;
        tx *= ascale;
        ty *= ascale;
        tz *= ascale;

        if (tk.n_parts <= 1) {
            if (active && ph == 0) {
                if (a.out4) {  // packed outputs
                    a.out4[i] = make_float4(tx, ty, tz, tp);
                } else {
                    a.ax[i] = tx;
                    a.ay[i] = ty;
                    a.az[i] = tz;
                    if (PHI) a.phi[i] = tp;
                }
            }
        } else if (ph == 0) {
            // partial sums of one part of a split j-list; k_combine adds the
            // parts of the chunk in order after this launch
            a.partial[(size_t)(tk.slot + tk.part) * 64 + lane] = make_float4(tx, ty, tz, tp);
        }
        t = t_next;
        if (t < ts.n_tasks) tk_next = task_of_fields(fld);
    }
}

// Runs after k_batch on the same stream: adds the partial sums of every split
// chunk in part order (deterministic) and writes its outputs.  One wave per
// split chunk.
__global__ void __launch_bounds__(64) k_combine(CombineArgs a)
{
    const int lane = threadIdx.x;
    if ((int)blockIdx.x >= a.n_chunks) return;
    const SplitChunk ch = a.chunks[blockIdx.x];
    if (lane >= ch.n_i) return;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 *p = a.partial + (size_t)ch.slot * 64 + ch.lane0 + lane;
    for (int q = 0; q < ch.n_parts; ++q) {
        const float4 v = p[(size_t)q * 64];
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
        s.w += v.w;
    }
    const int i = ch.i_off + lane;
    if (a.out4) {
        a.out4[i] = s;
        return;
    }
    a.ax[i] = s.x;
    a.ay[i] = s.y;
    a.az[i] = s.z;
    if (a.phi) a.phi[i] = s.w;
    if (a.mom) {
        // the i-side moments of the table adjoint, two float4 per partial sum
        float m[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        const size_t at = (size_t)ch.slot * 64 + ch.lane0 + lane;
        for (int q = 0; q < ch.n_parts; ++q) {
            const float4 u = a.mpartial[2 * (at + (size_t)q * 64)];
            const float4 v = a.mpartial[2 * (at + (size_t)q * 64) + 1];
            m[0] += u.x, m[1] += u.y, m[2] += u.z, m[3] += u.w;
            m[4] += v.x, m[5] += v.y, m[6] += v.z;
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) a.mom[(size_t)c * a.ni_total + i] = m[c];
    }
}

using BatchKernel = void (*)(BatchArgs);

template <bool RCP, int U>
BatchKernel newton_kernel_t(bool refine, bool guard, bool phi)
{
    const int sel = (refine ? 4 : 0) | (guard ? 2 : 0) | (phi ? 1 : 0);
    switch (sel) {
        case 0: return k_batch<RCP, false, false, false, U>;
        case 1: return k_batch<RCP, false, false, true, U>;
        case 2: return k_batch<RCP, false, true, false, U>;
        case 3: return k_batch<RCP, false, true, true, U>;
        case 4: return k_batch<RCP, true, false, false, U>;
        case 5: return k_batch<RCP, true, false, true, U>;
        case 6: return k_batch<RCP, true, true, false, U>;
        default: return k_batch<RCP, true, true, true, U>;
    }
}

// The tile shapes the autotuner chooses among: the unroll of the pair loop
// over a 64-record j-tile (pairs per lane in flight) and the rho^2 form
// (v_rsq_f32 squared, or v_rcp_f32 of r^2).
struct NewtonBatchVariant {
    const char *name;
    BatchKernel (*pick)(bool refine, bool guard, bool phi);
};
const NewtonBatchVariant kNewtonBatchVariants[] = {
    {"ki=1 jt=64 u=8", newton_kernel_t<false, 8>},  // the default
    {"ki=1 jt=64 u=8 rcp", newton_kernel_t<true, 8>},
    {"ki=1 jt=64 u=4", newton_kernel_t<false, 4>},
    {"ki=1 jt=64 u=2", newton_kernel_t<false, 2>},
    {"ki=1 jt=64 u=16", newton_kernel_t<false, 16>},
};
constexpr int kNumNewtonBatchVariants =
    sizeof(kNewtonBatchVariants) / sizeof(kNewtonBatchVariants[0]);

BatchKernel newton_kernel(bool refine, bool guard, bool phi, int variant = 0)
{
    if (variant < 0 || variant >= kNumNewtonBatchVariants) variant = 0;
    return kNewtonBatchVariants[variant].pick(refine, guard, phi);
}

// Workgroups that fit on one CU at once (registers, LDS), so the persistent
// grid is exactly one resident wave of workgroups.
int resident_blocks(BatchKernel k, size_t lds)
{
    static std::mutex mu;
    static std::map<std::pair<const void *, size_t>, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair((const void *)k, lds);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 256, lds) != hipSuccess || n < 1) n = 1;
    cache[key] = n;
    return n;
}

hipError_t launch(BatchKernel k, const BatchArgs &a0, int num_cu, hipStream_t s, bool phi)
{
    if (a0.n_tasks <= 0) return hipSuccess;
    BatchArgs a = a0;
    // one resident wave of workgroups, or fewer when there are fewer tasks
    // than waves (then every wave runs at most one task and the counter is
    // never touched)
    const int cap = num_cu * resident_blocks(k, 0);
    // at least one workgroup per task sublist
    const int blocks = std::max(a.nq, std::min(cap, (a.n_tasks + kWaves - 1) / kWaves));
    a.n_waves = blocks * kWaves;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.n_chunks == 0) return e;
    return launch_combine(a, phi, s);
}

}  // namespace

hipError_t launch_combine(const BatchArgs &a, bool phi, hipStream_t s)
{
    if (a.n_chunks == 0) return hipSuccess;
    CombineArgs c{a.n_chunks, a.chunks, a.partial, a.ax, a.ay, a.az, phi ? a.phi : nullptr,
                  a.out4, a.mpartial, a.mom, a.ni_total};
    hipLaunchKernelGGL(k_combine, dim3(a.n_chunks), dim3(64), 0, s, c);
    return hipGetLastError();
}

int batch_resident_waves(int num_cu)
{
    return num_cu * kWaves * resident_blocks(newton_kernel(true, false, true), 0);
}

int newton_batch_variants() { return kNumNewtonBatchVariants; }

const char *newton_batch_variant_name(int v)
{
    return (v >= 0 && v < kNumNewtonBatchVariants) ? kNewtonBatchVariants[v].name : nullptr;
}

hipError_t launch_newton_batch(const BatchArgs &a, int variant, bool refine, bool guard,
                               int num_cu, hipStream_t s)
{
    // packed outputs always carry the potential
    const bool phi = a.phi != nullptr || a.out4 != nullptr;
    return launch(newton_kernel(refine, guard, phi, variant), a, num_cu, s, phi);
}

}  // namespace pgh
