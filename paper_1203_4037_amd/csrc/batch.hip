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
// registers; the pair arithmetic is the one of the all-pairs kernels.
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "pairs.h"
#include "pgh_internal.h"

namespace pgh {
namespace {

constexpr int kWaves = kBatchWaves;
// coordinate of padding records: far enough that every pair term with them
// is finite and multiplied by a zero mass, small enough that its square
// stays finite in FP32
constexpr float kFar = 1.0e10f;

__device__ __forceinline__ void wave_sync()
{
    // LDS operations of one wave complete in order; this keeps the compiler
    // from moving reads of the tile above the writes of other lanes.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// KIND 0: Newton (REFINE, GUARD, PHI apply; ALT = the rcp form);
// KIND 1: table force (ALT = the (H, G1) table form; PHI = also the
// potential from the second table, a.ptable).
template <int KIND, bool ALT, bool REFINE, bool GUARD, bool PHI>
__global__ void __launch_bounds__(256, 8) k_batch(BatchArgs a)
{
    extern __shared__ float4 dyn4[];  // table force only: 2^(E+F) entries
    float2 *stab = (float2 *)dyn4;    // (G0, G1)
    float4 *stab4 = dyn4;             // (G0, G1, P0, P1), with PHI
    // [wave][buffer][list][record]: the Newton kernel double-buffers its
    // tiles; the table kernel, whose table also sits in LDS, uses one buffer
    constexpr int NB = KIND == 0 ? 2 : 1;
    __shared__ float4 jt[kWaves][NB][2][64];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const float mscale = (KIND == 0 && REFINE) ? -0.5f : 1.0f;

    // this workgroup serves task sublist q with the other workgroups b = q mod nq
    const unsigned nq = (unsigned)a.nq;
    const unsigned q = blockIdx.x % nq;
    const unsigned nw_q = ((gridDim.x - q + nq - 1) / nq) * kWaves;  // waves serving q
    const Task *tasks = a.tasks + a.q_begin[q];
    const unsigned n_tasks = (unsigned)(a.q_begin[q + 1] - a.q_begin[q]);
    unsigned *counter = a.queue + q * kQueueStride;
    const bool dynamic = n_tasks > nw_q;
    // (readfirstlane: the index is wave-uniform, so task fields load as scalars)
    unsigned t = __builtin_amdgcn_readfirstlane((blockIdx.x / nq) * kWaves + wave);
    // the first task's fields are fetched before the table copy, whose
    // latency they share
    Task tk_next{};
    if (t < n_tasks) tk_next = tasks[t];

    unsigned shift = 0, nbits = 0, hmask = 0;
    if (KIND == 1) {
        const int K = 1 << (a.E + a.F);
        shift = 23u - (unsigned)a.F;
        if (PHI)
            tables_to_lds<ALT>(stab4, a.table, a.ptable, K, shift);
        else
            table_to_lds<ALT>(stab, a.table, K, shift);
        nbits = (unsigned)(a.E + a.F);
        hmask = ~((1u << shift) - 1u);
        __syncthreads();  // the only workgroup barrier: waves are independent after it
    }

    // The first round of a sublist is assigned statically (its w-th wave
    // takes its w-th task), so a sublist with no more tasks than waves issues
    // no atomic at all; later tasks come from the sublist's counter, one
    // atomic per task, taken at the start of the previous task so that its
    // latency overlaps that task.
    while (t < n_tasks) {
        const Task tk = tk_next;
        unsigned tn = n_tasks;
        if (dynamic && lane == 0) {
            const unsigned k =
                __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (k == n_tasks - 1u)  // the sublist's last pop in this launch
                __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tn = nw_q + k;
        }

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
        const float pe = (KIND == 0) ? (a.eps2i ? a.eps2i[i] : a.eps2_all) : 0.f;

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
                if (KIND == 0 && a.jxm) {  // packed j-records: Newton only
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
        // vmcnt(0): the i-particle and first-tile loads (and the counter's
        // atomic).  Waiting here keeps the compiler from placing a full wait
        // inside the pair loop, where it would also wait for the prefetch of
        // the next tile.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        // The next task's index is known now: its 12 fields are fetched with
        // one vector load (field k in lane k) while this task runs, instead
        // of by scalar loads after it, whose latency the next task would
        // wait for (scalar loads inside the loop would also hold up its LDS
        // waits, which share their counter).
        const unsigned t_next = __builtin_amdgcn_readfirstlane(tn);
        int fld = 0;
        if (t_next < n_tasks && lane < 12) fld = ((const int *)(tasks + t_next))[lane];
        if (NB == 2) {
            store(0);
            wave_sync();
        }
        for (int tile = 0; tile < ntiles; ++tile) {
            const int cur = NB == 2 ? (tile & 1) : 0;
            if (NB == 1) {
                wave_sync();  // the previous tile's reads are done
                store(0);
                wave_sync();
            }
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
#pragma unroll 4
                    for (int it = 0; it < 64 / S; ++it) {
                        const float4 p = b[it * S];
                        if (KIND == 0)
                            newton_pair<REFINE, GUARD, PHI, ALT>(p, px, py, pz, pe, sx, sy, sz,
                                                                 sp);
                        else if (PHI)
                            table_pair_pot<ALT>(p, px, py, pz, stab4, a.c, a.smax, shift, nbits,
                                                hmask, sx, sy, sz, sp);
                        else
                            table_pair<ALT>(p, px, py, pz, stab, a.c, a.smax, shift, nbits, hmask,
                                            sx, sy, sz);
                    }
                };
                if (jlog == 0)
                    full_tile(std::integral_constant<int, 1>{});
                else if (jlog == 1)
                    full_tile(std::integral_constant<int, 2>{});
                else
                    full_tile(std::integral_constant<int, 4>{});
            } else {
#pragma unroll 2
                for (int it = 0; it < trips; ++it) {
                    const float4 p = src[it * js + ph];
                    if (KIND == 0)
                        newton_pair<REFINE, GUARD, PHI, ALT>(p, px, py, pz, pe, sx, sy, sz, sp);
                    else if (PHI)
                        table_pair_pot<ALT>(p, px, py, pz, stab4, a.c, a.smax, shift, nbits, hmask,
                                            sx, sy, sz, sp);
                    else
                        table_pair<ALT>(p, px, py, pz, stab, a.c, a.smax, shift, nbits, hmask, sx,
                                        sy, sz);
                }
            }
            tx += sx;
            ty += sy;
            tz += sz;
            tp += sp;
            if (NB == 2) {
                if (tile + 1 < ntiles) store(cur ^ 1);
                wave_sync();
            }
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
        const float ascale = (KIND == 0 && REFINE && !ALT) ? 0.25f : 1.0f;
        tx *= ascale;
        ty *= ascale;
        tz *= ascale;

        if (tk.n_parts <= 1) {
            if (active && ph == 0) {
                if (KIND == 0 && a.out4) {  // packed outputs: Newton only
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
        if (t < n_tasks) {
            tk_next.i_off = __builtin_amdgcn_readlane(fld, 0);
            tk_next.n_i = __builtin_amdgcn_readlane(fld, 1);
            tk_next.j_off = __builtin_amdgcn_readlane(fld, 2);
            tk_next.n_j = __builtin_amdgcn_readlane(fld, 3);
            tk_next.part = __builtin_amdgcn_readlane(fld, 4);
            tk_next.n_parts = __builtin_amdgcn_readlane(fld, 5);
            tk_next.slot = __builtin_amdgcn_readlane(fld, 6);
            tk_next.i_off2 = __builtin_amdgcn_readlane(fld, 7);
            tk_next.n_i2 = __builtin_amdgcn_readlane(fld, 8);
            tk_next.j_off2 = __builtin_amdgcn_readlane(fld, 9);
            tk_next.n_j2 = __builtin_amdgcn_readlane(fld, 10);
        }
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
}

using BatchKernel = void (*)(BatchArgs);

template <bool ALT>
BatchKernel newton_kernel_t(bool refine, bool guard, bool phi)
{
    const int sel = (refine ? 4 : 0) | (guard ? 2 : 0) | (phi ? 1 : 0);
    switch (sel) {
        case 0: return k_batch<0, ALT, false, false, false>;
        case 1: return k_batch<0, ALT, false, false, true>;
        case 2: return k_batch<0, ALT, false, true, false>;
        case 3: return k_batch<0, ALT, false, true, true>;
        case 4: return k_batch<0, ALT, true, false, false>;
        case 5: return k_batch<0, ALT, true, false, true>;
        case 6: return k_batch<0, ALT, true, true, false>;
        default: return k_batch<0, ALT, true, true, true>;
    }
}

BatchKernel newton_kernel(bool refine, bool guard, bool phi, bool rcp = false)
{
    return rcp ? newton_kernel_t<true>(refine, guard, phi) : newton_kernel_t<false>(refine, guard, phi);
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

hipError_t launch(BatchKernel k, const BatchArgs &a0, size_t lds, int num_cu, hipStream_t s,
                  bool phi)
{
    if (a0.n_tasks <= 0) return hipSuccess;
    BatchArgs a = a0;
    // one resident wave of workgroups, or fewer when there are fewer tasks
    // than waves (then every wave runs at most one task and the counter is
    // never touched)
    const int cap = num_cu * resident_blocks(k, lds);
    // at least one workgroup per task sublist
    const int blocks = std::max(a.nq, std::min(cap, (a.n_tasks + kWaves - 1) / kWaves));
    a.n_waves = blocks * kWaves;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.n_chunks == 0) return hipSuccess;
    CombineArgs c{a.n_chunks, a.chunks, a.partial, a.ax, a.ay, a.az, phi ? a.phi : nullptr,
                  a.out4};
    hipLaunchKernelGGL(k_combine, dim3(a.n_chunks), dim3(64), 0, s, c);
    return hipGetLastError();
}

}  // namespace

int batch_resident_waves(int num_cu)
{
    return num_cu * kWaves * resident_blocks(newton_kernel(true, false, true), 0);
}

const char *const kNewtonBatchNames[] = {"lds j-tiles", "lds j-tiles rcp"};
const char *const kTableBatchNames[] = {"lds j-tiles", "lds j-tiles htab"};

int batch_variants(int family) { return 2; }

const char *batch_variant_name(int family, int v)
{
    if (v < 0 || v > 1) return nullptr;
    return family == 2 ? kNewtonBatchNames[v] : kTableBatchNames[v];
}

hipError_t launch_newton_batch(const BatchArgs &a, int variant, bool refine, bool guard,
                               int num_cu, hipStream_t s)
{
    // packed outputs always carry the potential
    const bool phi = a.phi != nullptr || a.out4 != nullptr;
    return launch(newton_kernel(refine, guard, phi, variant == 1), a, 0, num_cu, s, phi);
}

hipError_t launch_table_batch(const BatchArgs &a, int variant, int num_cu, hipStream_t s)
{
    const bool phi = a.phi && a.ptable;
    const size_t lds = (phi ? sizeof(float4) : sizeof(float2)) << (a.E + a.F);
    BatchKernel k;
    if (variant == 1)
        k = phi ? k_batch<1, true, false, false, true> : k_batch<1, true, false, false, false>;
    else
        k = phi ? k_batch<1, false, false, false, true> : k_batch<1, false, false, false, false>;
    return launch(k, a, lds, num_cu, s, phi);
}

}  // namespace pgh
