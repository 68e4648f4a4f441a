// Adjoints of L = sum_i w_i . a_i for both forces (derived from
// Eq. newton_force and from the interpolation of Sec. 3.4.2).  Pair terms are
// recomputed, never stored.
//
// Newton, with d = r_j - r_i, rho = (|d|^2 + eps_i^2)^{-1/2} and the pair
// term T = m_j rho^3 (w_i . d):
//   dT/dd = m_j [rho^3 w_i - 3 rho^5 (w_i . d) d],  dd/dr_j = I, dd/dr_i = -I,
//   dT/dm_j = rho^3 (w_i . d).
//
// All-pairs over one shared set (i-set = j-set, one eps): both roles of a
// particle k fold into one gather over l (d = r_l - r_k):
//   g_k  = m_k sum_l rho^3 w_l - w_k sum_l m_l rho^3
//          + 3 sum_l rho^5 [m_l (w_k . d) - m_k (w_l . d)] d
//   gm_k = -sum_l rho^3 (w_l . d)
// which is 26 VALU ops and one rsqrt per pair (29 with the Newton-Raphson
// step), against 13 (16) for the forward pass.  The j-records carry
// (x, y, z, m) and (wx, wy, wz) in two 16-byte LDS entries.
//
// Separate sets: an i-major pass gives gxi, a j-major pass (j in registers,
// i streamed through LDS) gives gxj and gmj.
//
// Table force, with g = G0_k + G1_k (s - s_k), T = m_j g (w_i . d):
//   dL/dG0_k = sum over pairs in bin k of m_j (w_i . d)
//   dL/dG1_k = sum over pairs in bin k of m_j (s - s_k) (w_i . d)
//   dL/dm_j  = sum_i g (w_i . d)
// One j-major pass over the lists gives both: the table gradient is
// accumulated in LDS with float atomics per workgroup and flushed once
// (pairs clamped to the last node, beyond rcut where s - s_k = 0, add to a
// per-lane register instead, so the common out-of-range pair costs no
// atomic), and dL/dm_j is each lane's own sum.
#include <algorithm>

#include "table_pairs.h"
#include "pgh_internal.h"

namespace pgh {

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_pack_xw(int n, const float *__restrict__ x,
                                                 const float *__restrict__ y,
                                                 const float *__restrict__ z,
                                                 const float *__restrict__ s, float s_all,
                                                 const float *__restrict__ wx,
                                                 const float *__restrict__ wy,
                                                 const float *__restrict__ wz,
                                                 float4 *__restrict__ dst)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        dst[2 * i] = make_float4(x[i], y[i], z[i], s ? s[i] : s_all);
        dst[2 * i + 1] = make_float4(wx[i], wy[i], wz[i], 0.f);
    }
}

hipError_t launch_pack_xw(int n, const float *x, const float *y, const float *z, const float *s,
                          float s_all, const float *wx, const float *wy, const float *wz,
                          float4 *dst, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_xw, dim3((n + 255) / 256), dim3(256), 0, st, n, x, y, z, s, s_all,
                       wx, wy, wz, dst);
    return hipGetLastError();
}

namespace {

template <bool REFINE>
__device__ __forceinline__ float rsqrt_of(float q)
{
    const float y = __builtin_amdgcn_rsqf(q);
    if (!REFINE) return y;
    return y * __builtin_fmaf(-0.5f * q, y * y, 1.5f);
}

// ---------------------------------------------------------------------------
// all-pairs Newton adjoint over one shared set
// ---------------------------------------------------------------------------

// Output of a (possibly j-split) adjoint launch: with one share the four
// results go to their arrays, with several to partial sums [S][4][n].
struct Out4 {
    float *a, *b, *c, *d;
    float *part;
    int jchunk;
};

__device__ __forceinline__ void store4(const Out4 &o, int n, int i, float va, float vb, float vc,
                                       float vd)
{
    if (gridDim.y > 1) {
        float *p = o.part + (size_t)blockIdx.y * 4 * n;
        p[i] = va;
        p[n + i] = vb;
        p[2 * n + i] = vc;
        p[3 * n + i] = vd;
    } else {
        if (o.a) {
            o.a[i] = va;
            o.b[i] = vb;
            o.c[i] = vc;
        }
        if (o.d) o.d[i] = vd;
    }
}

template <int JT, bool REFINE>
__global__ void __launch_bounds__(256) k_newton_allpairs_bwd(int n, const float4 *__restrict__ rec,
                                                             float eps2, Out4 o)
{
    static_assert(JT % 256 == 0, "tile must be a multiple of the workgroup");
    constexpr int PER = JT / 256;
    __shared__ float4 tile[2][JT][2];
    const int tid = threadIdx.x;
    const int k = blockIdx.x * 256 + tid;
    const int kc = k < n ? k : n - 1;
    const float4 pk = rec[2 * kc], wk = rec[2 * kc + 1];

    float Ax = 0.f, Ay = 0.f, Az = 0.f, B = 0.f, Cx = 0.f, Cy = 0.f, Cz = 0.f, G = 0.f;
    const int jbase = blockIdx.y * o.jchunk;
    const int nj = max(0, min(o.jchunk, n - jbase));
    const float4 *__restrict__ jrec = rec + 2 * (size_t)jbase;
    const int ntiles = (nj + JT - 1) / JT;
    float4 pre[PER][2];
    auto load = [&](int t) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int j = t * JT + r * 256 + tid;
            float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
            if (j < nj) {
                a = jrec[2 * j];
                b = jrec[2 * j + 1];
            }
            pre[r][0] = a;
            pre[r][1] = b;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            tile[buf][r * 256 + tid][0] = pre[r][0];
            tile[buf][r * 256 + tid][1] = pre[r][1];
        }
    };
    load(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store(0);
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
        const int cur = t & 1;
        set_tile_prio(ntiles - t, ntiles);
        if (t + 1 < ntiles) load(t + 1);
        const int cnt = min(JT, nj - t * JT);
        float ax = 0.f, ay = 0.f, az = 0.f, b = 0.f, cx = 0.f, cy = 0.f, cz = 0.f, gg = 0.f;
        // The tile holding this workgroup's own particles (global tile index
        // == blockIdx.x, as JT equals the workgroup size and shares start on
        // tile boundaries) skips each lane's self pair, whose term is
        // identically zero but would enter A and B as +-m_k w_k/eps^3 and
        // cancel only to rounding.
        const int self = (jbase / JT + t == (int)blockIdx.x) ? tid : -1;
        auto pair = [&](const float4 p, const float4 w) {
            const float dx = p.x - pk.x, dy = p.y - pk.y, dz = p.z - pk.z;
            float q = __builtin_fmaf(dx, dx, eps2);
            q = __builtin_fmaf(dy, dy, q);
            q = __builtin_fmaf(dz, dz, q);
            const float r1 = rsqrt_of<REFINE>(q);
            const float r2 = r1 * r1;
            const float r3 = r2 * r1;
            const float r5 = r3 * r2;
            ax = __builtin_fmaf(r3, w.x, ax);
            ay = __builtin_fmaf(r3, w.y, ay);
            az = __builtin_fmaf(r3, w.z, az);
            b = __builtin_fmaf(p.w, r3, b);
            float wld = w.x * dx;
            wld = __builtin_fmaf(w.y, dy, wld);
            wld = __builtin_fmaf(w.z, dz, wld);
            float wkd = wk.x * dx;
            wkd = __builtin_fmaf(wk.y, dy, wkd);
            wkd = __builtin_fmaf(wk.z, dz, wkd);
            const float e = __builtin_fmaf(p.w, wkd, -pk.w * wld);
            const float f = r5 * e;
            cx = __builtin_fmaf(f, dx, cx);
            cy = __builtin_fmaf(f, dy, cy);
            cz = __builtin_fmaf(f, dz, cz);
            gg = __builtin_fmaf(r3, wld, gg);
        };
        if (self < 0) {
#pragma unroll 4
            for (int jj = 0; jj < cnt; ++jj) pair(tile[cur][jj][0], tile[cur][jj][1]);
        } else {
            for (int jj = 0; jj < cnt; ++jj) {
                // a zero-weight, zero-mass stand-in for the self pair adds 0
                float4 p = tile[cur][jj][0], w = tile[cur][jj][1];
                if (jj == self) {
                    p = make_float4(pk.x + 1.f, pk.y, pk.z, 0.f);
                    w = make_float4(0.f, 0.f, 0.f, 0.f);
                }
                pair(p, w);
            }
        }
        Ax += ax, Ay += ay, Az += az, B += b, Cx += cx, Cy += cy, Cz += cz, G += gg;
        if (t + 1 < ntiles) store(cur ^ 1);
        __syncthreads();
    }
    if (k < n)
        store4(o, n, k, pk.w * Ax - wk.x * B + 3.f * Cx, pk.w * Ay - wk.y * B + 3.f * Cy,
               pk.w * Az - wk.z * B + 3.f * Cz, -G);
}

// ---------------------------------------------------------------------------
// separate sets: i-major pass (gxi) and j-major pass (gxj, gmj)
// ---------------------------------------------------------------------------

// i-records: (x, y, z, eps2), (wx, wy, wz, -); j-records: (x, y, z, m).
template <int JT, bool REFINE>
__global__ void __launch_bounds__(256) k_newton_bwd_i(int ni, const float4 *__restrict__ irec,
                                                      int nj_all, const float4 *__restrict__ jall,
                                                      Out4 o)
{
    constexpr int PER = JT / 256;
    __shared__ float4 tile[2][JT];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * 256 + tid;
    const int ic = i < ni ? i : ni - 1;
    const float4 pi = irec[2 * ic], wi = irec[2 * ic + 1];
    float B = 0.f, Cx = 0.f, Cy = 0.f, Cz = 0.f;
    const int jbase = blockIdx.y * o.jchunk;
    const int nj = max(0, min(o.jchunk, nj_all - jbase));
    const float4 *__restrict__ jmem = jall + jbase;
    const int ntiles = (nj + JT - 1) / JT;
    float4 pre[PER];
    auto load = [&](int t) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int j = t * JT + r * 256 + tid;
            pre[r] = j < nj ? jmem[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < PER; ++r) tile[buf][r * 256 + tid] = pre[r];
    };
    load(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store(0);
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
        const int cur = t & 1;
        set_tile_prio(ntiles - t, ntiles);
        if (t + 1 < ntiles) load(t + 1);
        const int cnt = min(JT, nj - t * JT);
        float b = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
#pragma unroll 4
        for (int jj = 0; jj < cnt; ++jj) {
            const float4 p = tile[cur][jj];
            const float dx = p.x - pi.x, dy = p.y - pi.y, dz = p.z - pi.z;
            float q = __builtin_fmaf(dx, dx, pi.w);
            q = __builtin_fmaf(dy, dy, q);
            q = __builtin_fmaf(dz, dz, q);
            const float r1 = rsqrt_of<REFINE>(q);
            const float r2 = r1 * r1;
            const float mr3 = p.w * (r2 * r1);
            b += mr3;
            float wid = wi.x * dx;
            wid = __builtin_fmaf(wi.y, dy, wid);
            wid = __builtin_fmaf(wi.z, dz, wid);
            const float f = mr3 * r2 * wid;
            cx = __builtin_fmaf(f, dx, cx);
            cy = __builtin_fmaf(f, dy, cy);
            cz = __builtin_fmaf(f, dz, cz);
        }
        B += b, Cx += cx, Cy += cy, Cz += cz;
        if (t + 1 < ntiles) store(cur ^ 1);
        __syncthreads();
    }
    if (i < ni) store4(o, ni, i, 3.f * Cx - wi.x * B, 3.f * Cy - wi.y * B, 3.f * Cz - wi.z * B, 0.f);
}

template <int IT, bool REFINE>
__global__ void __launch_bounds__(256) k_newton_bwd_j(int nj, const float4 *__restrict__ jmem,
                                                      int ni_all, const float4 *__restrict__ iall,
                                                      Out4 o)
{
    constexpr int PER = IT / 256;
    __shared__ float4 tile[2][IT][2];
    const int tid = threadIdx.x;
    const int j = blockIdx.x * 256 + tid;
    const int jc = j < nj ? j : nj - 1;
    const float4 pj = jmem[jc];
    float Ax = 0.f, Ay = 0.f, Az = 0.f, Cx = 0.f, Cy = 0.f, Cz = 0.f, G = 0.f;
    const int ibase = blockIdx.y * o.jchunk;
    const int ni = max(0, min(o.jchunk, ni_all - ibase));
    const float4 *__restrict__ irec = iall + 2 * (size_t)ibase;
    const int ntiles = (ni + IT - 1) / IT;
    float4 pre[PER][2];
    auto load = [&](int t) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = t * IT + r * 256 + tid;
            // padding i-records: unit softening, zero weight -> no contribution
            float4 a = make_float4(0.f, 0.f, 0.f, 1.f), b = make_float4(0.f, 0.f, 0.f, 0.f);
            if (i < ni) {
                a = irec[2 * i];
                b = irec[2 * i + 1];
            }
            pre[r][0] = a;
            pre[r][1] = b;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            tile[buf][r * 256 + tid][0] = pre[r][0];
            tile[buf][r * 256 + tid][1] = pre[r][1];
        }
    };
    load(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store(0);
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
        const int cur = t & 1;
        set_tile_prio(ntiles - t, ntiles);
        if (t + 1 < ntiles) load(t + 1);
        const int cnt = min(IT, ni - t * IT);
        float ax = 0.f, ay = 0.f, az = 0.f, cx = 0.f, cy = 0.f, cz = 0.f, gg = 0.f;
#pragma unroll 4
        for (int ii = 0; ii < cnt; ++ii) {
            const float4 p = tile[cur][ii][0];
            const float4 w = tile[cur][ii][1];
            const float dx = pj.x - p.x, dy = pj.y - p.y, dz = pj.z - p.z;
            float q = __builtin_fmaf(dx, dx, p.w);
            q = __builtin_fmaf(dy, dy, q);
            q = __builtin_fmaf(dz, dz, q);
            const float r1 = rsqrt_of<REFINE>(q);
            const float r2 = r1 * r1;
            const float r3 = r2 * r1;
            ax = __builtin_fmaf(r3, w.x, ax);
            ay = __builtin_fmaf(r3, w.y, ay);
            az = __builtin_fmaf(r3, w.z, az);
            float wid = w.x * dx;
            wid = __builtin_fmaf(w.y, dy, wid);
            wid = __builtin_fmaf(w.z, dz, wid);
            gg = __builtin_fmaf(r3, wid, gg);
            const float f = r3 * r2 * wid;
            cx = __builtin_fmaf(f, dx, cx);
            cy = __builtin_fmaf(f, dy, cy);
            cz = __builtin_fmaf(f, dz, cz);
        }
        Ax += ax, Ay += ay, Az += az, Cx += cx, Cy += cy, Cz += cz, G += gg;
        if (t + 1 < ntiles) store(cur ^ 1);
        __syncthreads();
    }
    if (j < nj)
        store4(o, nj, j, pj.w * (Ax - 3.f * Cx), pj.w * (Ay - 3.f * Cy), pj.w * (Az - 3.f * Cz), G);
}

// ---------------------------------------------------------------------------
// table-force adjoint over a plan
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wave_sync()
{
    // LDS operations of one wave complete in order; the fences keep the
    // compiler from moving tile reads across the writes of other lanes.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The table-force adjoint over the lists of a plan.  Task kinds (one index
// space):
//
// [0, n_m): j-major tasks, a chunk of <= 64 j-entries of a list (one per
// lane; chunks of <= 32 or <= 16 run 2 or 4 lanes per entry on alternate
// i-records) against its item's i-range, streamed through a per-wave LDS
// tile of 64 i-records (position and weight), the next tile prefetched into
// registers.  With g = G0_k + G1_k ds, ds = s - s_k, each pair adds
//   dL/dm_j   += g (w_i . d)
//   dL/dG0_k  += m_j (w_i . d),  dL/dG1_k += m_j (w_i . d) ds
//   dL/dr_j   += m_j [ g w_i + 2c G1_k (w_i . d) d ]
// the table terms into LDS bins with float atomics (pairs clamped to s_max,
// the common case, into one register instead), flushed with one global
// atomic per non-zero bin and workgroup into one of kGradCopies copies,
// which a last small kernel adds; the per-entry sums go to gmj and gxj with
// one atomic per entry and task (an entry can belong to several lists).
//
// [n_m, n_m + n_i): i-major tasks (only for the i-side position gradient),
// an i-chunk of <= 64 against a part of its j-list, j-records streamed:
//   dL/dr_i   -= m_j [ g w_i + 2c G1_k (w_i . d) d ]
// summed per lane and added to gxi with one atomic per i and task, or
// stored when every row is in exactly one such task (A.istore: no list cut
// into parts and no row left out, so no zeroing pass either).
//
// Tasks of each kind are sorted longest first.  With at most four per wave
// every wave follows a static order; with more, the waves of a workgroup
// share its own static sequence of tasks through an LDS counter, so they
// balance among themselves without a chip-wide atomic per task.  (One global
// counter for all tasks serialised the pops: on 4^3-cell lists of 262144
// particles with E = 4, F = 7 the whole adjoint took 290 us, its passes run
// alone 160 us; 103 us with the workgroup counters.)
// IMAJ: the i-major tasks are compiled in (the j-major-only instantiation
// holds fewer registers, so more waves fit).  W waves per workgroup.
template <bool IMAJ, int W>
__global__ void __launch_bounds__(64 * W) k_table_bwd(TableBwdArgs A, const Task *jtasks,
                                                      int n_m, const Task *itasks, int n_i)
{
    // declared as float4 so that the dynamic region, placed after the
    // static arrays, starts 16-byte aligned for the 8-byte table reads
    extern __shared__ float4 dyn4[];
    float *dyn = (float *)dyn4;
    const BatchArgs &a = A.b;
    const int K = 1 << (a.E + a.F);
    float2 *stab = (float2 *)dyn;  // K (G0, G1)
    float *gt = dyn + 2 * K;       // 2K gradient accumulators
    // per wave: 64 i-records (x, y, z, wx) or j-records, and the (wy, wz)
    // of the i-records
    // (4 records of padding: the j-major loop reads one record ahead, up to
    // record 64 + 3, and leaves it unused)
    __shared__ float4 buf[W][68];
    __shared__ float2 wbuf[W][68];
    __shared__ unsigned wg_next;  // the next position in the workgroup's sequence
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) wg_next = W;
    const bool want_tab = A.gtable != nullptr, want_m = A.gmj != nullptr;
    const bool want_xj = A.gxj != nullptr;
    const bool need_g = want_m || want_xj || n_i > 0;
    if (need_g) table_to_lds<false>(stab, a.table, K, 0u);
    if (want_tab)
        for (int k = threadIdx.x; k < K; k += 64 * W) {
            gt[2 * k] = 0.f;
            gt[2 * k + 1] = 0.f;
        }
    __syncthreads();
    // bins as byte offsets into the (G0, G1) table, uniform operands in
    // VGPRs (the forward's table_pairs_v); offset `last` is the clamped node
    const TableConsts kc = table_consts(a.c, a.smax, a.E, a.F, 3);
    const unsigned last = kc.am;
    const char *tab = (const char *)stab;
    char *gtb = (char *)gt;
    const float c2 = 2.0f * a.c;
    float4 *tile = buf[wave];
    float2 *wtile = wbuf[wave];
    float last0 = 0.f;  // clamped pairs: dL/dG0 of the last node

    const unsigned n_all = (unsigned)(n_m + n_i);
    const unsigned n_waves = gridDim.x * W;
    // The static orders zig-zag (round k of member g of G takes task
    // k G + g, or k G + G - 1 - g for odd k), pairing long tasks with short
    // ones.  At most four tasks per wave: the waves are the members, with no
    // atomics; else the workgroups are, and the waves of one take the rounds
    // of its sequence in turn from wg_next (rounds 0 .. W-1 by wave index).
    // Either sequence rises with the round, so a wave stops at its first
    // task beyond n_all.
    const bool stat = n_all <= 4u * n_waves;
    const unsigned gw = __builtin_amdgcn_readfirstlane(blockIdx.x * W + wave);
    const unsigned nb = gridDim.x, b = blockIdx.x;
    auto wg_task = [&](unsigned k) {
        const unsigned long long r =
            (unsigned long long)k * nb + ((k & 1u) ? nb - 1u - b : b);
        return r < n_all ? (unsigned)r : n_all;
    };
    unsigned round = 0;
    // (read as uniform: the compiler cannot tell that the wave index is, and
    // would otherwise keep the task index and its decoding in vector registers)
    for (unsigned t = __builtin_amdgcn_readfirstlane(stat ? gw : wg_task((unsigned)wave));
         t < n_all;) {
        unsigned tn = n_all;
        if (stat) {
            ++round;
            const unsigned long long r =
                (unsigned long long)round * n_waves + ((round & 1u) ? n_waves - 1u - gw : gw);
            tn = r < n_all ? (unsigned)r : n_all;
        } else if (lane == 0) {
            tn = wg_task(atomicAdd(&wg_next, 1u));
        }
        const bool jmajor = !IMAJ || t < (unsigned)n_m;
        // jmajor: i_off/n_i = the j-chunk, j_off/n_j = the i-range; else an
        // i-chunk and a part of its j-list
        const Task tk = jmajor ? jtasks[t] : itasks[t - (unsigned)n_m];
        // a chunk of <= 32 (<= 16) entries runs 2 (4) lanes per entry on
        // alternate records, added inside the wave at the end
        const int jlog = tk.n_i <= 16 ? 2 : (tk.n_i <= 32 ? 1 : 0);
        const int js = 1 << jlog;
        const int el = lane & (63 >> jlog), ph = lane >> (6 - jlog);
        const bool active = el < tk.n_i;
        const int e = tk.i_off + (active ? el : 0);  // this lane's entry
        if (jmajor) {
            const int j = e;
            const float qx = a.xj[j], qy = a.yj[j], qz = a.zj[j];
            const float mj = active ? a.mj[j] : 0.f;
            float G = 0.f, Ux = 0.f, Uy = 0.f, Uz = 0.f, Vx = 0.f, Vy = 0.f, Vz = 0.f;
            float4 pp;
            float2 pw;
            // i-records past the range: far away with zero weight
            auto load = [&](int base) {
                pp = make_float4(1.0e10f, 1.0e10f, 1.0e10f, 0.f);
                pw = make_float2(0.f, 0.f);
                const int i = tk.j_off + base + lane;
                if (base + lane < tk.n_j) {
                    pp = make_float4(a.xi[i], a.yi[i], a.zi[i], A.wx[i]);
                    pw = make_float2(A.wy[i], A.wz[i]);
                }
            };
            // a pair in two halves: the head forms s and issues the table
            // gather, the tail uses it, so that the next record can be read
            // from LDS in between
            struct Head {
                float dx, dy, dz, ds, wd;
                unsigned off;
                float2 g01;
            };
            auto head = [&](const float4 p, const float2 w) {
                Head h;
                h.dx = qx - p.x, h.dy = qy - p.y, h.dz = qz - p.z;
                float r2 = h.dx * h.dx;
                r2 = __builtin_fmaf(h.dy, h.dy, r2);
                r2 = __builtin_fmaf(h.dz, h.dz, r2);
                const unsigned u = min(__float_as_uint(__builtin_fmaf(r2, kc.c, 2.0f)), kc.smax_bits);
                h.off = (u >> kc.sh) & kc.am;  // 8 k for bin k
                h.ds = __uint_as_float(u) - __uint_as_float(u & kc.hm);
                float wd = p.w * h.dx;
                wd = __builtin_fmaf(w.x, h.dy, wd);
                h.wd = __builtin_fmaf(w.y, h.dz, wd);
                if (want_m || want_xj) h.g01 = *(const float2 *)(tab + h.off);
                return h;
            };
            auto tail = [&](const Head &h, const float4 p, const float2 w) {
                const float dx = h.dx, dy = h.dy, dz = h.dz, ds = h.ds, wd = h.wd;
                const unsigned off = h.off;
                if (want_m || want_xj) {
                    const float2 g01 = h.g01;
                    const float g = __builtin_fmaf(g01.y, ds, g01.x);
                    if (want_m) G = __builtin_fmaf(g, wd, G);
                    if (want_xj) {
                        Ux = __builtin_fmaf(g, p.w, Ux);
                        Uy = __builtin_fmaf(g, w.x, Uy);
                        Uz = __builtin_fmaf(g, w.y, Uz);
                        const float q = g01.y * wd;
                        Vx = __builtin_fmaf(q, dx, Vx);
                        Vy = __builtin_fmaf(q, dy, Vy);
                        Vz = __builtin_fmaf(q, dz, Vz);
                    }
                }
                if (want_tab) {
                    const float v0 = mj * wd;
                    if (off == last) {
                        last0 += v0;
                    } else if (active) {
                        atomicAdd((float *)(gtb + off), v0);
                        atomicAdd((float *)(gtb + off + 4), v0 * ds);
                    }
                }
            };
            auto pair = [&](const float4 p, const float2 w) { tail(head(p, w), p, w); };
            load(0);
            for (int base = 0; base < tk.n_j; base += 64) {
                wave_sync();
                tile[lane] = pp;
                wtile[lane] = pw;
                wave_sync();
                if (base + 64 < tk.n_j) load(base + 64);
                const int cnt = min(64, tk.n_j - base);
                if (cnt == 64) {
                    // the next record is read before this pair's table gather
                    // is waited for (the last read, past the tile's 64
                    // records, lands in its padding and goes unused)
                    const int full = 64 >> jlog;
                    float4 p = tile[ph];
                    float2 w = wtile[ph];
#pragma unroll 2
                    for (int ii = 0; ii < full; ++ii) {
                        const Head h = head(p, w);
                        const int rn = ((ii + 1) << jlog) + ph;
                        const float4 pn = tile[rn];
                        const float2 wn = wtile[rn];
                        __builtin_amdgcn_sched_barrier(0);
                        tail(h, p, w);
                        p = pn;
                        w = wn;
                    }
                } else {
                    // records past cnt are zero-weight padding
                    const int trips = (cnt + js - 1) >> jlog;
                    for (int ii = 0; ii < trips; ++ii) {
                        const int r = (ii << jlog) + ph;
                        pair(tile[r], wtile[r]);
                    }
                }
            }
            auto lanes_sum = [&](float &v) {
                if (jlog >= 2) v += __shfl_xor(v, 16);
                if (jlog >= 1) v += __shfl_xor(v, 32);
            };
            // one task per entry when the lists' j-ranges are disjoint:
            // stores; otherwise the entry's lists add up
            if (want_m) {
                lanes_sum(G);
                if (active && ph == 0) {
                    if (A.jdisjoint) A.gmj[j] = G;
                    else atomicAdd(&A.gmj[j], G);
                }
            }
            if (want_xj) {
                lanes_sum(Ux), lanes_sum(Uy), lanes_sum(Uz);
                lanes_sum(Vx), lanes_sum(Vy), lanes_sum(Vz);
                if (active && ph == 0) {
                    const float gx = mj * __builtin_fmaf(c2, Vx, Ux);
                    const float gy = mj * __builtin_fmaf(c2, Vy, Uy);
                    const float gz = mj * __builtin_fmaf(c2, Vz, Uz);
                    if (A.jdisjoint) {
                        A.gxj[j] = gx, A.gyj[j] = gy, A.gzj[j] = gz;
                    } else {
                        atomicAdd(&A.gxj[j], gx);
                        atomicAdd(&A.gyj[j], gy);
                        atomicAdd(&A.gzj[j], gz);
                    }
                }
            }
        } else {
            // i-side position gradient: lane = i-particle, j-records streamed
            const int i = e;
            const float px = a.xi[i], py = a.yi[i], pz = a.zi[i];
            const float wx = A.wx[i], wy = A.wy[i], wz = A.wz[i];
            float S = 0.f, Vx = 0.f, Vy = 0.f, Vz = 0.f;
            float4 pre;
            auto load = [&](int base) {
                pre = make_float4(1.0e10f, 1.0e10f, 1.0e10f, 0.f);
                const int j = tk.j_off + base + lane;
                if (base + lane < tk.n_j) pre = make_float4(a.xj[j], a.yj[j], a.zj[j], a.mj[j]);
            };
            auto pair = [&](const float4 p) {
                const float dx = p.x - px, dy = p.y - py, dz = p.z - pz;
                float r2 = dx * dx;
                r2 = __builtin_fmaf(dy, dy, r2);
                r2 = __builtin_fmaf(dz, dz, r2);
                const unsigned u = min(__float_as_uint(__builtin_fmaf(r2, kc.c, 2.0f)), kc.smax_bits);
                const float ds = __uint_as_float(u) - __uint_as_float(u & kc.hm);
                const float2 g01 = *(const float2 *)(tab + ((u >> kc.sh) & kc.am));
                const float g = __builtin_fmaf(g01.y, ds, g01.x);
                float wd = wx * dx;
                wd = __builtin_fmaf(wy, dy, wd);
                wd = __builtin_fmaf(wz, dz, wd);
                S = __builtin_fmaf(p.w, g, S);
                const float q = p.w * g01.y * wd;
                Vx = __builtin_fmaf(q, dx, Vx);
                Vy = __builtin_fmaf(q, dy, Vy);
                Vz = __builtin_fmaf(q, dz, Vz);
            };
            load(0);
            for (int base = 0; base < tk.n_j; base += 64) {
                wave_sync();
                tile[lane] = pre;
                wave_sync();
                if (base + 64 < tk.n_j) load(base + 64);
                const int cnt = min(64, tk.n_j - base);
                if (cnt == 64) {
                    const int full = 64 >> jlog;
#pragma unroll 4
                    for (int jj = 0; jj < full; ++jj) pair(tile[(jj << jlog) + ph]);
                } else {
                    const int trips = (cnt + js - 1) >> jlog;
                    for (int jj = 0; jj < trips; ++jj) pair(tile[(jj << jlog) + ph]);
                }
            }
            auto lanes_sum = [&](float &v) {
                if (jlog >= 2) v += __shfl_xor(v, 16);
                if (jlog >= 1) v += __shfl_xor(v, 32);
            };
            lanes_sum(S), lanes_sum(Vx), lanes_sum(Vy), lanes_sum(Vz);
            if (active && ph == 0) {
                const float gx = -__builtin_fmaf(c2, Vx, S * wx);
                const float gy = -__builtin_fmaf(c2, Vy, S * wy);
                const float gz = -__builtin_fmaf(c2, Vz, S * wz);
                if (A.istore) {
                    A.gxi[i] = gx;
                    A.gyi[i] = gy;
                    A.gzi[i] = gz;
                } else {
                    atomicAdd(&A.gxi[i], gx);
                    atomicAdd(&A.gyi[i], gy);
                    atomicAdd(&A.gzi[i], gz);
                }
            }
        }
        t = __builtin_amdgcn_readfirstlane(tn);
    }
    if (want_tab) {
        // wave sum of the clamped-bin register, then flush this workgroup's bins
        for (int off = 32; off > 0; off >>= 1) last0 += __shfl_xor(last0, off);
        if (lane == 0 && last0 != 0.f) atomicAdd(&gt[2 * (K - 1)], last0);
        __syncthreads();
        float *dst = A.gcopies + (size_t)(blockIdx.x % kGradCopies) * 2 * K;
        for (int k = threadIdx.x; k < 2 * K; k += 64 * W)
            if (gt[k] != 0.f) atomicAdd(&dst[k], gt[k]);
    }
}

// Zeroes the per-entry gradients that are added up (lists sharing
// j-entries; the i-major pass) ahead of k_table_bwd (a kernel rather than
// memsets, so the sequence can be captured in a graph).
// Up to 8 arrays of the given lengths (NULL: skipped).
struct ZeroList {
    float *p[8];
    int n[8];
};

__global__ void __launch_bounds__(256) k_table_bwd_prologue(ZeroList z)
{
    const int stride = gridDim.x * 256;
    const int t0 = blockIdx.x * 256 + threadIdx.x;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (z.p[q])
            for (int k = t0; k < z.n[q]; k += stride) z.p[q][k] = 0.f;
}

// The work after k_table_bwd, in one launch:
//   * gtable[k] = the sum of the kGradCopies partial copies, in copy order;
//     the copies are put back to zero for the next call;
//   * with disjoint j-ranges, the per-entry gradients of j-entries in no
//     list (which no task stored) are set to zero;
//   * with the forward's moments (TableBwdArgs::mom), the i-side position
//     gradient: row i of an item gets dL/dr_i = -(S_i w_i + 2c M_i w_i), rows
//     in no item 0.
struct BwdTail {
    int n_tab;  // 2K, or 0 without a table gradient
    float *copies, *gtable;
    int nj;  // j-entries to check against the ranges, or 0
    const int2 *jrange;
    int n_jrange;
    float *gmj, *gxj, *gyj, *gzj;
    int ni;  // i-rows of the moment gradient, or 0
    const float *mom;  // [7][ni]
    const float *wx, *wy, *wz;
    float *gxi, *gyi, *gzi;
    const int2 *irange;
    int n_irange;
    int icover;  // every i-row is in an item
    float c2;    // 2c
};

// Whether index r lies in one of the n ranges (off, len) sorted by off.
__device__ __forceinline__ bool in_ranges(const int2 *rg, int n, int r)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rg[mid].x <= r) lo = mid + 1;
        else hi = mid;
    }
    return lo > 0 && r < rg[lo - 1].x + rg[lo - 1].y;
}

__global__ void __launch_bounds__(256) k_table_bwd_tail(BwdTail t)
{
    const int stride = gridDim.x * 256;
    const int t0 = blockIdx.x * 256 + threadIdx.x;
    for (int k = t0; k < t.n_tab; k += stride) {
        float v = 0.f;
#pragma unroll
        for (int q = 0; q < kGradCopies; ++q) {
            v += t.copies[(size_t)q * t.n_tab + k];
            t.copies[(size_t)q * t.n_tab + k] = 0.f;
        }
        t.gtable[k] = v;
    }
    for (int j = t0; j < t.nj; j += stride) {
        if (in_ranges(t.jrange, t.n_jrange, j)) continue;
        if (t.gmj) t.gmj[j] = 0.f;
        if (t.gxj) t.gxj[j] = t.gyj[j] = t.gzj[j] = 0.f;
    }
    for (int i = t0; i < t.ni; i += stride) {
        float gx = 0.f, gy = 0.f, gz = 0.f;
        if (t.icover || in_ranges(t.irange, t.n_irange, i)) {
            const float *m = t.mom + i;
            const size_t n = (size_t)t.ni;
            const float S = m[0], mxx = m[n], mxy = m[2 * n], mxz = m[3 * n], myy = m[4 * n],
                        myz = m[5 * n], mzz = m[6 * n];
            const float wx = t.wx[i], wy = t.wy[i], wz = t.wz[i];
            gx = -__builtin_fmaf(t.c2, mxx * wx + mxy * wy + mxz * wz, S * wx);
            gy = -__builtin_fmaf(t.c2, mxy * wx + myy * wy + myz * wz, S * wy);
            gz = -__builtin_fmaf(t.c2, mxz * wx + myz * wy + mzz * wz, S * wz);
        }
        t.gxi[i] = gx;
        t.gyi[i] = gy;
        t.gzi[i] = gz;
    }
}

int resident(const void *k, size_t lds, int threads = 256)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, threads, lds) != hipSuccess || n < 1)
        n = 1;
    return n;
}

}  // namespace

namespace {

// Launches an adjoint kernel over n outputs with its other index range m split
// into S shares, then adds the shares.
template <typename Kern, typename... Args>
hipError_t launch_split(Kern k, int n, int m, int S, float *part, float *a, float *b, float *c,
                        float *d, hipStream_t s, Args... args)
{
    S = std::max(1, S);
    const int chunk = (int)(((long)m + (long)S * 256 - 1) / ((long)S * 256) * 256);
    S = std::max(1, (m + chunk - 1) / chunk);
    Out4 o{a, b, c, d, part, std::max(chunk, 1)};
    hipLaunchKernelGGL(k, dim3((n + 255) / 256, S), dim3(256), 0, s, args..., o);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || S == 1) return e;
    if (a) e = launch_combine_split(n, S, part, a, b, c, d, s);
    else if (d) {
        // only the fourth result: combine into it through its own slot
        e = launch_combine_split(n, S, part, nullptr, nullptr, nullptr, d, s);
    }
    return e;
}

}  // namespace

int adjoint_split(int n, int m, size_t part_cap)
{
    return split_count(n, m, 1, 256, kSplitTargetWaves, part_cap);
}

hipError_t launch_newton_allpairs_bwd(int n, const float4 *rec, float eps2, bool refine, float *gx,
                                      float *gy, float *gz, float *gm, int S, float *part,
                                      hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    auto k = refine ? k_newton_allpairs_bwd<256, true> : k_newton_allpairs_bwd<256, false>;
    return launch_split(k, n, n, S, part, gx, gy, gz, gm, s, n, rec, eps2);
}

hipError_t launch_newton_bwd_i(int ni, const float4 *irec, int nj, const float4 *jmem,
                               bool refine, float *gx, float *gy, float *gz, int S, float *part,
                               hipStream_t s)
{
    if (ni <= 0) return hipSuccess;
    auto k = refine ? k_newton_bwd_i<256, true> : k_newton_bwd_i<256, false>;
    return launch_split(k, ni, nj, S, part, gx, gy, gz, (float *)nullptr, s, ni, irec, nj, jmem);
}

hipError_t launch_newton_bwd_j(int nj, const float4 *jmem, int ni, const float4 *irec,
                               bool refine, float *gx, float *gy, float *gz, float *gm, int S,
                               float *part, hipStream_t s)
{
    if (nj <= 0) return hipSuccess;
    auto k = refine ? k_newton_bwd_j<256, true> : k_newton_bwd_j<256, false>;
    return launch_split(k, nj, ni, S, part, gx, gy, gz, gm, s, nj, jmem, ni, irec);
}

hipError_t launch_table_batch_bwd(const TableBwdArgs &A, const Task *jtasks, int n_jtasks,
                                  const Task *itasks, int n_itasks, int num_cu, hipStream_t s)
{
    const int K = 1 << (A.b.E + A.b.F);
    // the i-side gradient: from the forward's moments in the tail kernel
    // (each row written once), or accumulated by the i-major tasks
    const bool from_mom = A.gxi && A.mom;
    const bool store_j = A.jdisjoint != 0;
    ZeroList z{};
    int nz = 0, longest = 0;
    auto add = [&](float *p, int n) {
        if (!p || n <= 0) return;
        z.p[nz] = p;
        z.n[nz++] = n;
        longest = std::max(longest, n);
    };
    if (!store_j) {
        add(A.gmj, A.nj_total);
        add(A.gxj, A.nj_total), add(A.gyj, A.nj_total), add(A.gzj, A.nj_total);
    }
    if (!from_mom && !A.istore)
        add(A.gxi, A.ni_total), add(A.gyi, A.ni_total), add(A.gzi, A.ni_total);
    hipError_t e = hipSuccess;
    if (nz > 0) {
        const int zb = std::max(1, std::min(1024, (longest + 255) / 256));
        hipLaunchKernelGGL(k_table_bwd_prologue, dim3(zb), dim3(256), 0, s, z);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const bool jside = A.gtable || A.gmj || A.gxj;
    const int n_m = jside ? n_jtasks : 0;
    const int n_i = (A.gxi && !from_mom) ? n_itasks : 0;
    if (n_m + n_i > 0) {
        // the table and its gradient sums: 16 bytes per node.  From 2^12
        // nodes (64 KiB) on they leave room for at most two workgroups per
        // CU, which then run 16 waves each (24 KiB of record buffers beside
        // 128 KiB of table at 2^13 nodes) rather than 4.
        const size_t lds = (size_t)K * 4 * sizeof(float);
        const bool wide = lds >= 65536;
        const int W = wide ? 16 : 4;
        const auto kern = n_i > 0 ? (wide ? k_table_bwd<true, 16> : k_table_bwd<true, 4>)
                                  : (wide ? k_table_bwd<false, 16> : k_table_bwd<false, 4>);
        if ((e = allow_dynamic_lds((const void *)kern, lds)) != hipSuccess) return e;
        const int cap = num_cu * resident((const void *)kern, lds, 64 * W);
        const int blocks = std::max(1, std::min(cap, (n_m + n_i + W - 1) / W));
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * W), lds, s, A, jtasks, n_m, itasks,
                           n_i);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    BwdTail t{};
    if (A.gtable) t.n_tab = 2 * K, t.copies = A.gcopies, t.gtable = A.gtable;
    if (store_j && !A.jcover && (A.gmj || A.gxj)) {
        t.nj = A.nj_total, t.jrange = A.jrange, t.n_jrange = A.n_jrange;
        t.gmj = A.gmj, t.gxj = A.gxj, t.gyj = A.gyj, t.gzj = A.gzj;
    }
    if (from_mom) {
        t.ni = A.ni_total, t.mom = A.mom, t.wx = A.wx, t.wy = A.wy, t.wz = A.wz;
        t.gxi = A.gxi, t.gyi = A.gyi, t.gzi = A.gzi;
        t.irange = A.irange, t.n_irange = A.n_irange, t.icover = A.icover;
        t.c2 = 2.0f * A.b.c;
    }
    const int work = std::max(t.n_tab, std::max(t.nj, t.ni));
    if (work > 0) {
        const int tb = std::max(1, std::min(1024, (work + 255) / 256));
        hipLaunchKernelGGL(k_table_bwd_tail, dim3(tb), dim3(256), 0, s, t);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace pgh
