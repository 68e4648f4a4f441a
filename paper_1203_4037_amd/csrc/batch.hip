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
// Execution: a grid sized to fill every CU; each wave64 runs independently,
// taking its first task by its index and later ones from a device counter
// with one atomic each.  The second kernel also resets the counter, so the
// next launch (or a replay of a captured graph) starts from zero without a
// memset.
//
// Each wave stages its j-list through its own LDS slice, 64 records per
// tile (one coalesced load per coordinate array), double-buffered in
// registers; the pair arithmetic is the one of the all-pairs kernels.
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "pairs.h"
#include "pgh_internal.h"

namespace pgh {
namespace {

constexpr int kWaves = 4;  // wave64s per workgroup

__device__ __forceinline__ void wave_sync()
{
    // LDS operations of one wave complete in order; this keeps the compiler
    // from moving reads of the tile above the writes of other lanes.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// KIND 0: Newton (REFINE, GUARD, PHI apply; ALT = the rcp form);
// KIND 1: table force (ALT = the (H, G1) table form).
template <int KIND, bool ALT, bool REFINE, bool GUARD, bool PHI>
__global__ void __launch_bounds__(256) k_batch(BatchArgs a)
{
    extern __shared__ float2 stab[];  // table force only: 2^(E+F) entries
    __shared__ float4 jt[kWaves][2][64];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const float mscale = (KIND == 0 && REFINE) ? -0.5f : 1.0f;

    unsigned shift = 0, nbits = 0, hmask = 0;
    if (KIND == 1) {
        const int K = 1 << (a.E + a.F);
        shift = 23u - (unsigned)a.F;
        table_to_lds<ALT>(stab, a.table, K, shift);
        nbits = (unsigned)(a.E + a.F);
        hmask = ~((1u << shift) - 1u);
        __syncthreads();  // the only workgroup barrier: waves are independent after it
    }

    // The first round of tasks is assigned statically (wave w takes task w),
    // so a launch with no more tasks than waves issues no atomic at all; the
    // later tasks come from the counter, one atomic per task, taken at the
    // start of the previous task so its latency overlaps that task.  (All
    // waves hitting one counter at once serialises at the memory side.)
    const unsigned n_tasks = (unsigned)a.n_tasks;
    const bool dynamic = n_tasks > (unsigned)a.n_waves;
    unsigned t = blockIdx.x * kWaves + wave;
    while (t < n_tasks) {
        const Task tk = a.tasks[t];
        unsigned tn = n_tasks;
        if (dynamic && lane == 0)
            tn = (unsigned)a.n_waves +
                 __hip_atomic_fetch_add(&a.queue[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        // lanes per i-particle (js) and the lane's i slot and j phase
        const int js = tk.n_i <= 16 ? 4 : (tk.n_i <= 32 ? 2 : 1);
        const int wlog = js == 4 ? 4 : (js == 2 ? 5 : 6);
        const int il = lane & ((1 << wlog) - 1);
        const int ph = lane >> wlog;
        const bool active = il < tk.n_i;
        const int i = tk.i_off + (active ? il : 0);

        const float px = a.xi[i], py = a.yi[i], pz = a.zi[i];
        const float pe = (KIND == 0) ? (a.eps2i ? a.eps2i[i] : a.eps2_all) : 0.f;

        float tx = 0.f, ty = 0.f, tz = 0.f, tp = 0.f;
        const int nj = tk.n_j;
        const int ntiles = (nj + 63) >> 6;

        float4 pre;
        auto load = [&](int tile) {
            const int j = tk.j_off + tile * 64 + lane;
            pre = make_float4(0.f, 0.f, 0.f, 0.f);
            if (tile * 64 + lane < nj) pre = make_float4(a.xj[j], a.yj[j], a.zj[j], a.mj[j]);
        };
        load(0);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): i-particle and first tile loads
        {
            float4 v = pre;
            v.w *= mscale;
            jt[wave][0][lane] = v;
        }
        wave_sync();

        for (int tile = 0; tile < ntiles; ++tile) {
            const int cur = tile & 1;
            if (tile + 1 < ntiles) load(tile + 1);
            const int cnt = min(64, nj - tile * 64);
            // every lane runs the same trip count; records past cnt are the
            // zero-mass padding written above
            const int trips = (cnt + js - 1) / js;
            float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f;
            if (trips == 64) {
#pragma unroll 4
                for (int it = 0; it < 64; ++it) {
                    const float4 p = jt[wave][cur][it];
                    if (KIND == 0)
                        newton_pair<REFINE, GUARD, PHI, ALT>(p, px, py, pz, pe, sx, sy, sz, sp);
                    else
                        table_pair<ALT>(p, px, py, pz, stab, a.c, a.smax, shift, nbits, hmask, sx, sy,
                                   sz);
                }
            } else {
#pragma unroll 2
                for (int it = 0; it < trips; ++it) {
                    const float4 p = jt[wave][cur][it * js + ph];
                    if (KIND == 0)
                        newton_pair<REFINE, GUARD, PHI, ALT>(p, px, py, pz, pe, sx, sy, sz, sp);
                    else
                        table_pair<ALT>(p, px, py, pz, stab, a.c, a.smax, shift, nbits, hmask, sx, sy,
                                   sz);
                }
            }
            tx += sx;
            ty += sy;
            tz += sz;
            tp += sp;
            if (tile + 1 < ntiles) {
                float4 v = pre;
                v.w *= mscale;
                jt[wave][cur ^ 1][lane] = v;
            }
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
        const float ascale = (KIND == 0 && REFINE && !ALT) ? 0.25f : 1.0f;
        tx *= ascale;
        ty *= ascale;
        tz *= ascale;

        if (tk.n_parts <= 1) {
            if (active && ph == 0) {
                a.ax[i] = tx;
                a.ay[i] = ty;
                a.az[i] = tz;
                if (KIND == 0 && PHI) a.phi[i] = tp;
            }
        } else if (ph == 0) {
            // partial sums of one part of a split j-list; k_combine adds the
            // parts of the chunk in order after this launch
            a.partial[(size_t)(tk.slot + tk.part) * 64 + lane] = make_float4(tx, ty, tz, tp);
        }
        t = __builtin_amdgcn_readfirstlane(tn);
    }
}

// Runs after k_batch on the same stream: adds the partial sums of every split
// chunk in part order (deterministic) and writes its outputs, and resets the
// task counter for the next launch.  One wave per split chunk.
__global__ void __launch_bounds__(64) k_combine(CombineArgs a)
{
    const int lane = threadIdx.x;
    if (blockIdx.x == 0 && lane == 0) a.queue[0] = 0u;
    if ((int)blockIdx.x >= a.n_chunks) return;
    const SplitChunk ch = a.chunks[blockIdx.x];
    if (lane >= ch.n_i) return;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 *p = a.partial + (size_t)ch.slot * 64 + lane;
    for (int q = 0; q < ch.n_parts; ++q) {
        const float4 v = p[(size_t)q * 64];
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
        s.w += v.w;
    }
    const int i = ch.i_off + lane;
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
    const int blocks = num_cu * resident_blocks(k, lds);
    a.n_waves = blocks * kWaves;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    CombineArgs c{a.n_chunks, a.chunks, a.partial, a.queue, a.ax, a.ay, a.az,
                  phi ? a.phi : nullptr};
    hipLaunchKernelGGL(k_combine, dim3(std::max(1, a.n_chunks)), dim3(64), 0, s, c);
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
    return launch(newton_kernel(refine, guard, a.phi != nullptr, variant == 1), a, 0, num_cu, s,
                  a.phi != nullptr);
}

hipError_t launch_table_batch(const BatchArgs &a, int variant, int num_cu, hipStream_t s)
{
    const size_t lds = sizeof(float2) << (a.E + a.F);
    if (variant == 1) return launch(k_batch<1, true, false, false, false>, a, lds, num_cu, s, false);
    return launch(k_batch<1, false, false, false, false>, a, lds, num_cu, s, false);
}

}  // namespace pgh
