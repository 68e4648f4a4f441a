// Table force over interaction lists in one persistent launch: the force
// procedure of Sec. 3.4.2 on the (i-group, j-list) items of a tree or TreePM
// code (Sec. 5.1), over the same plans as the batched Newton kernel
// (batch.hip: wave tasks of at most 64 i-particles, pairs of partly filled
// chunks sharing a wave, long lists cut into parts, longest-first sublists).
//
// What differs from the Newton kernel:
//   * KI i-particles per lane (1 or 2).  Each lane reads one j-record from
//     LDS per step and uses it for KI pairs: the j-record broadcast and the
//     table gather share the CU's LDS bandwidth, and with one i-particle per
//     lane the LDS, not the VALU, would bound the pair rate.  A chunk of n
//     i-particles with js lanes per i-particle (chunk_js) runs P = KI js
//     phases of R = 64 / P lanes; lane (phase p, row r) holds the chunk's
//     slots r + k R (k < KI) and takes the list's entries p, p + P, ...  A
//     paired task runs P = KI phases; its first chunk holds rows
//     [0, ceil(n_1 / KI)), the second the rows after them (the planner pairs
//     two chunks only when both fit in that many rows).
//   * The j-tile of a task without a second list is 64 TW records (TW
//     records per lane per tile), so short steps (P = 8) still get long
//     tiles.
//   * Each wave sets its issue priority from the work it has left
//     (set_wave_prio), so the waves of a SIMD finish together instead of in
//     the order they arrived.
//   * The pair arithmetic (table_pair_v) keeps every uniform operand in a
//     VGPR and finds the bin's byte offset with a shift and a mask; the
//     table sits in static LDS (2^TB entries at most), so its base folds
//     into the LDS read's offset field.
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "batch_queue.h"
#include "table_pairs.h"

namespace pgh {
namespace {

// plans of at most this many tasks per wave run in the static order
constexpr int kStaticRounds = 4;

// The lanes of one task: lane (phase, row) holds slots q + k stride
// (k < KI) of its chunk (i-particles i0 + slot, the chunk's partial-sum
// lanes from lane0), and takes the list's entries phase, phase + P, ...
template <int KI>
struct TaskLanes {
    bool paired, second;
    int plog, P, R, phase, q, stride, nl, i0, lane0;
    int T, nj, ntiles;  // records per tile and list, entries, tiles
    bool act[KI];
    float px[KI], py[KI], pz[KI];
};

// KI i-particles per lane, TW j-records per lane per tile (unpaired tasks),
// 2^TB table entries at most, HT the (H, G1) form, PHI the potential table,
// WPB waves per workgroup (one table copy per workgroup).
template <int KI, int TW, int TB, bool HT, bool PHI, int WPB, bool PF, bool MOM = false>
// eight waves per SIMD whatever the workgroup size (64 VGPRs at most)
__global__ void __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_batch_table(BatchArgs a)
{
    // MOM: also the i-side moments of the adjoint (table_pairs_mom), in the
    // paper's form, without a potential
    static_assert(!MOM || (!HT && !PHI), "moments take the paper's form, no potential");
    using Entry = std::conditional_t<PHI, float4, float2>;
    constexpr int kEntryLog = PHI ? 4 : 3;
    __shared__ Entry stab[1 << TB];
    // a wave's j-tile: 128 records and 8 of padding, read (and unused) by
    // the prefetch after a tile's last step
    __shared__ float4 jt[WPB][136];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // Task order: static (few tasks per wave: no atomics, and the next
    // task's fields load while the current task runs) or the sublists.
    const bool stat = a.static_order != 0;
    const TaskStream ts = task_stream(a, WPB);
    const unsigned G = gridDim.x * WPB;
    const unsigned gw = __builtin_amdgcn_readfirstlane(blockIdx.x * WPB + wave);
    const Task *const tbase = stat ? a.tasks : ts.tasks;
    const unsigned n_t = stat ? (unsigned)a.n_tasks : ts.n_tasks;
    unsigned round = 0;
    unsigned t = stat ? static_task(a, 0, gw, G) : first_task(a, WPB, wave);
    const unsigned rounds_g = stat ? static_rounds(n_t, gw, G) : 0u;  // the wave's static tasks
    float4 *tile = jt[wave];

    // j-records of tile tl of a task, TW per lane (a paired task: one of each
    // list); entries past a list's end are zero-mass records far away
    float4 pre[2];
    auto record = [&](int j_off, int n, int j) {
        float4 v = make_float4(kFar, kFar, kFar, 0.f);
        if (j < n) {
            const int jj = j_off + j;
            v = make_float4(a.xj[jj], a.yj[jj], a.zj[jj], a.mj[jj]);
        }
        return v;
    };
    auto load = [&](const Task &tk, const TaskLanes<KI> &L, int tl) {
        if (L.paired) {
            pre[0] = record(tk.j_off, tk.n_j, tl * 64 + lane);
            pre[1] = record(tk.j_off2, tk.n_j2, tl * 64 + lane);
        } else {
#pragma unroll
            for (int w = 0; w < TW; ++w) pre[w] = record(tk.j_off, tk.n_j, tl * L.T + w * 64 + lane);
        }
    };
    auto store = [&](const TaskLanes<KI> &L) {
        tile[lane] = pre[0];
        if (L.paired || TW == 2) tile[64 + lane] = pre[1];
    };
    // lane -> (phase, row) -> (list, slots); issues the task's i-particle
    // loads and the loads of its first tile
    auto begin = [&](const Task &tk) {
        TaskLanes<KI> L;
        L.paired = tk.n_i2 > 0;
        L.plog = (KI == 2 ? 1 : 0) + (L.paired ? 0 : (tk.n_i <= 16 ? 2 : (tk.n_i <= 32 ? 1 : 0)));
        L.P = 1 << L.plog;
        L.R = 64 >> L.plog;
        L.phase = lane >> (6 - L.plog);
        const int row = lane & (L.R - 1);
        L.stride = L.R, L.q = row, L.nl = tk.n_i, L.i0 = tk.i_off, L.lane0 = 0;
        L.second = false;
        if (L.paired) {
            const int ra = (tk.n_i + KI - 1) / KI, rb = (tk.n_i2 + KI - 1) / KI;
            L.second = row >= ra;
            L.stride = L.second ? rb : ra;
            L.q = L.second ? row - ra : row;
            L.nl = L.second ? tk.n_i2 : tk.n_i;
            L.i0 = L.second ? tk.i_off2 : tk.i_off;
            L.lane0 = L.second ? tk.n_i : 0;
        }
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int slot = L.q + k * L.stride;
            L.act[k] = L.q < L.stride && slot < L.nl;
            const int i = L.i0 + (L.act[k] ? slot : 0);
            L.px[k] = a.xi[i];
            L.py[k] = a.yi[i];
            L.pz[k] = a.zi[i];
        }
        L.T = L.paired ? 64 : 64 * TW;
        L.nj = L.paired ? max(tk.n_j, tk.n_j2) : tk.n_j;
        L.ntiles = (L.nj + L.T - 1) / L.T;
        load(tk, L, 0);
        return L;
    };

    // The first task's fields, i-particles and first tile are loaded before
    // the table copy, whose latency they share.
    Task tk{};
    TaskLanes<KI> L{};
    if (t < n_t) {
        tk = tbase[t];
        L = begin(tk);
    }
    {
        const int K = 1 << (a.E + a.F);
        const unsigned shift = 23u - (unsigned)a.F;
        if (PHI)
            tables_to_lds<HT>((float4 *)stab, a.table, a.ptable, K, shift);
        else
            table_to_lds<HT>((float2 *)stab, a.table, K, shift);
    }
    const TableConsts kc = table_consts(a.c, a.smax, a.E, a.F, kEntryLog);
    const char *tab = (const char *)stab;
    __syncthreads();  // the only workgroup barrier: waves are independent after it
    if (a.prio_quarter) __builtin_amdgcn_s_setprio(3);

    while (t < n_t) {
        const unsigned tn = stat ? 0u : pop_task(ts, lane);
        // vmcnt(0): the i-particle and first-tile loads (and the ticket's
        // atomic).  Waiting here keeps the compiler from placing a full wait
        // inside the pair loop, where it would also wait for the prefetch of
        // the next tile.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        const unsigned t_next =
            stat ? static_task(a, ++round, gw, G) : __builtin_amdgcn_readfirstlane(tn);
        int fld = 0;
        if (t_next < n_t && lane < 12) fld = ((const int *)(tbase + t_next))[lane];

        float tx[KI], ty[KI], tz[KI], tp[KI];
        float tm[MOM ? 7 : 1][KI];
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            tx[k] = ty[k] = tz[k] = tp[k] = 0.f;
#pragma unroll
            for (int c = 0; c < (MOM ? 7 : 1); ++c) tm[c][k] = 0.f;
        }
        const float4 *src = tile + (L.second ? 64 : 0) + L.phase;
        // the wave's static tasks after this one (round is this task's + 1)
        const unsigned more = stat ? rounds_g - round : 0u;
        for (int tl = 0; tl < L.ntiles; ++tl) {
            // pair-slots left: the task's remaining records times the i-slots
            // each serves (64 over the lanes per i-particle), and the later
            // tasks at the mean size
            set_wave_prio(((unsigned long long)(L.nj - tl * L.T) << (6 - (L.plog - (KI == 2 ? 1 : 0)))) +
                              (unsigned long long)more * a.prio_task,
                          a.prio_quarter);
            wave_sync();  // the previous tile's reads are done
            store(L);
            wave_sync();
            if (tl + 1 < L.ntiles) load(tk, L, tl + 1);
            const int cnt = min(L.T, L.nj - tl * L.T);
            auto step = [&](const float4 p) {
                if constexpr (MOM)
                    table_pairs_mom<KI>(p, L.px, L.py, L.pz, tab, kc, tx, ty, tz, tm);
                else
                    table_pairs_v<KI, HT, PHI>(p, L.px, L.py, L.pz, tab, kc, tx, ty, tz, tp);
            };
            if (cnt == L.T) {
                // a full tile: T / P records per lane with a compile-time
                // stride, so the LDS reads take immediate offsets
                auto full = [&](auto stride_c, auto trips_c) {
                    constexpr int S = decltype(stride_c)::value;
                    constexpr int N = decltype(trips_c)::value;
                    if constexpr (PF) {
                        // the next record is read before this step's
                        // table gathers are waited for, so one LDS round
                        // trip per step remains on the wave's path
                        float4 p = src[0];
#pragma unroll 2
                        for (int it = 0; it < N; ++it) {
                            TableGather<KI, PHI> q;
                            table_head<KI, HT, PHI>(p, L.px, L.py, L.pz, tab, kc, q);
                            const float4 pn = src[(it + 1) * S];
                            // nothing of the sums moves above the next
                            // record's read
                            __builtin_amdgcn_sched_barrier(0);
                            if constexpr (MOM)
                                table_tail_mom<KI>(p.w, q, tx, ty, tz, tm);
                            else
                                table_tail<KI, PHI>(p.w, q, tx, ty, tz, tp);
                            p = pn;
                        }
                    } else {
#pragma unroll 2
                        for (int it = 0; it < N; ++it) step(src[it * S]);
                    }
                };
                using std::integral_constant;
                if (L.paired) {
                    full(integral_constant<int, KI>{}, integral_constant<int, 64 / KI>{});
                } else if (L.plog == (KI == 2 ? 1 : 0)) {
                    full(integral_constant<int, KI>{}, integral_constant<int, 64 * TW / KI>{});
                } else if (L.plog == (KI == 2 ? 2 : 1)) {
                    full(integral_constant<int, 2 * KI>{}, integral_constant<int, 32 * TW / KI>{});
                } else {
                    full(integral_constant<int, 4 * KI>{}, integral_constant<int, 16 * TW / KI>{});
                }
            } else {
                const int trips = (cnt + L.P - 1) >> L.plog;
#pragma unroll 2
                for (int it = 0; it < trips; ++it) step(src[it * L.P]);
            }
        }

        // add the phases of each row (lanes row, row + R, ...)
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            for (int d = L.R; d < 64; d <<= 1) {
                tx[k] += __shfl_xor(tx[k], d);
                ty[k] += __shfl_xor(ty[k], d);
                tz[k] += __shfl_xor(tz[k], d);
                if (PHI) tp[k] += __shfl_xor(tp[k], d);
                if constexpr (MOM) {
#pragma unroll
                    for (int c = 0; c < 7; ++c) tm[c][k] += __shfl_xor(tm[c][k], d);
                }
            }
        }
        if (L.phase == 0) {
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                if (!L.act[k]) continue;
                const int slot = L.q + k * L.stride;
                if (tk.n_parts <= 1) {
                    const int i = L.i0 + slot;
                    a.ax[i] = tx[k];
                    a.ay[i] = ty[k];
                    a.az[i] = tz[k];
                    if (PHI) a.phi[i] = tp[k];
                    if constexpr (MOM) {
#pragma unroll
                        for (int c = 0; c < 7; ++c) a.mom[(size_t)c * a.ni_total + i] = tm[c][k];
                    }
                } else {
                    // partial sums of one part of a split j-list; k_combine
                    // adds the parts of the chunk in order after this launch
                    const size_t at = (size_t)(tk.slot + tk.part) * 64 + L.lane0 + slot;
                    a.partial[at] = make_float4(tx[k], ty[k], tz[k], tp[k]);
                    if constexpr (MOM) {
                        a.mpartial[2 * at] = make_float4(tm[0][k], tm[1][k], tm[2][k], tm[3][k]);
                        a.mpartial[2 * at + 1] = make_float4(tm[4][k], tm[5][k], tm[6][k], 0.f);
                    }
                }
            }
        }
        t = t_next;
        if (t < n_t) {
            tk = task_of_fields(fld);
            L = begin(tk);
        }
    }
}

using TableKernel = void (*)(BatchArgs);

// A kernel of a variant for a table of 2^tb nodes, and its waves per
// workgroup.  The table's LDS bounds the workgroups per CU, so larger tables
// take wider workgroups whatever the variant's own width: up to 2^10 nodes
// the variant's; up to 2^12 (32 KiB, 64 KiB with the potential) 16 waves,
// two workgroups per CU (one with the potential); beyond (128 KiB at 2^14,
// or at 2^13 with the potential) 12 waves, the most whose j-tiles (2176
// bytes each) fit beside the table in the 160 KiB of a CU.  With its own two
// waves per workgroup a variant would leave SIMDs idle there.
constexpr int kMidWaves = 16;
constexpr int kWideWaves = 12;

struct TableKernelPick {
    TableKernel k;
    int wpb;
};

template <int KI, int TW, bool HT, int WPB, bool PF = false>
TableKernelPick pick(int tb, bool phi)
{
    if (tb <= 10)
        return {phi ? k_batch_table<KI, TW, 10, HT, true, WPB, PF>
                    : k_batch_table<KI, TW, 10, HT, false, WPB, PF>, WPB};
    if (tb <= 12)
        return {phi ? k_batch_table<KI, TW, 12, HT, true, kMidWaves, PF>
                    : k_batch_table<KI, TW, 12, HT, false, kMidWaves, PF>, kMidWaves};
    return {phi ? k_batch_table<KI, TW, 13, HT, true, kWideWaves, PF>
                : k_batch_table<KI, TW, 14, HT, false, kWideWaves, PF>, kWideWaves};
}

struct TableBatchVariant {
    const char *name;
    int wpb;  // waves per workgroup (tables of at most 2^10 nodes)
    TableKernelPick (*pick)(int tb, bool phi);
};

// The tile shapes the autotuner chooses among: i-particles per lane (KI),
// j-records per lane per tile (TW), waves per workgroup, the one-record
// prefetch (pf) and the table form.  The "htab" variants keep the (H, G1)
// form in LDS (two instructions fewer per pair): the same interpolant with
// one more FP32 rounding per node, of H_k = G0_k - G1_k s_k, which is
// relative to G1_k s_k rather than to g; near rcut, where g goes to zero,
// that rounding can be a large part of the little force there, so these
// variants are parity-checked against the oracle's (H, G1) table and, for the
// method's accuracy, against the analytic force.
const TableBatchVariant kTableBatchVariants[] = {
    {"ki=1 tw=1 wg=4", 4, pick<1, 1, false, 4>},
    {"ki=2 tw=1 wg=4", 4, pick<2, 1, false, 4>},
    {"ki=2 tw=2 wg=4", 4, pick<2, 2, false, 4>},
    {"ki=1 tw=1 wg=16", 16, pick<1, 1, false, 16>},
    {"ki=2 tw=2 wg=16", 16, pick<2, 2, false, 16>},
    {"ki=1 tw=1 wg=4 pf", 4, pick<1, 1, false, 4, true>},
    {"ki=2 tw=1 wg=4 htab", 4, pick<2, 1, true, 4>},
    {"ki=2 tw=2 wg=4 htab", 4, pick<2, 2, true, 4>},
    {"ki=2 tw=2 wg=2 htab", 2, pick<2, 2, true, 2>},
};
constexpr int kNumTableBatchVariants = sizeof(kTableBatchVariants) / sizeof(kTableBatchVariants[0]);

int resident_blocks(TableKernel k, int wpb)
{
    static std::mutex mu;
    static std::map<const void *, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find((const void *)k);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * wpb, 0) != hipSuccess || n < 1)
        n = 1;
    cache[(const void *)k] = n;
    return n;
}

}  // namespace

int table_batch_variants() { return kNumTableBatchVariants; }

const char *table_batch_variant_name(int v)
{
    return (v >= 0 && v < kNumTableBatchVariants) ? kTableBatchVariants[v].name : nullptr;
}

int table_batch_default() { return 2; }

// The pair-slot figures of set_wave_prio: a quarter of the plan's
// interactions per wave of the launch, and its mean task.
static void set_prio_args(BatchArgs &a)
{
    const unsigned long long inter = a.interactions > 0 ? (unsigned long long)a.interactions : 0ull;
    a.prio_quarter = inter / (4ull * (unsigned long long)std::max(1, a.n_waves));
    a.prio_task = inter / (unsigned long long)std::max(1, a.n_tasks);
}

hipError_t launch_table_batch_moments(const BatchArgs &a0, int num_cu, hipStream_t s)
{
    if (a0.n_tasks <= 0) return hipSuccess;
    // two-wave workgroups: their LDS holds a CU to six waves per SIMD, so
    // the seven moment sums per i-particle fit in registers without spills
    // (16.3 us against 18.1 us with four-wave workgroups on 8^3 cell lists
    // of 65536 particles), and the next record read from LDS before the
    // current pair's table gathers are waited for (16.0 against 16.3 us); a
    // table of 2^12 nodes or more leaves room for two workgroups per CU or
    // one, which then run 16 waves each
    const int tb = a0.E + a0.F;
    const int wpb = tb <= 10 ? 2 : 16;
    const TableKernel k = tb <= 10   ? k_batch_table<1, 2, 10, false, false, 2, true, true>
                          : tb <= 12 ? k_batch_table<1, 2, 12, false, false, 16, false, true>
                                     : k_batch_table<1, 2, 13, false, false, 16, false, true>;
    BatchArgs a = a0;
    a.phi = nullptr;
    a.ptable = nullptr;
    const int cap = num_cu * resident_blocks(k, wpb);
    const int blocks = std::max(a.nq, std::min(cap, (a.n_tasks + wpb - 1) / wpb));
    a.n_waves = blocks * wpb;
    a.static_order = (long long)a.n_tasks <= kStaticRounds * (long long)a.n_waves ? 1 : 0;
    set_prio_args(a);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * wpb), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.n_chunks == 0) return e;
    return launch_combine(a, false, s);
}

hipError_t launch_table_batch(const BatchArgs &a0, int variant, int num_cu, hipStream_t s)
{
    if (a0.n_tasks <= 0) return hipSuccess;
    if (variant < 0 || variant >= kNumTableBatchVariants) variant = table_batch_default();
    const bool phi = a0.phi && a0.ptable;
    const TableKernelPick pk = kTableBatchVariants[variant].pick(a0.E + a0.F, phi);
    const TableKernel k = pk.k;
    const int wpb = pk.wpb;
    BatchArgs a = a0;
    // one resident wave of workgroups, or fewer when there are fewer tasks
    // than waves; at least one workgroup per task sublist
    const int cap = num_cu * resident_blocks(k, wpb);
    const int blocks = std::max(a.nq, std::min(cap, (a.n_tasks + wpb - 1) / wpb));
    a.n_waves = blocks * wpb;
    a.static_order = (long long)a.n_tasks <= kStaticRounds * (long long)a.n_waves ? 1 : 0;
    set_prio_args(a);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * wpb), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.n_chunks == 0) return e;
    return launch_combine(a, phi, s);
}

}  // namespace pgh
