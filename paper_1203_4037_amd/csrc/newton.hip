// All-pairs Newton force and potential on gfx950: Eq. (newton_force) of
// Sec. 3 with the loop of Sec. 3.3 (difference, softened square distance,
// inverse square root, m/r into the potential, m/r^3 times the difference
// into the acceleration).
//
// Mapping.  A workgroup of 256 lanes (four wave64) owns 256*KI i-particles,
// KI per lane, held in VGPRs for the whole launch.  The j-particles stream
// through LDS in tiles of JT (x, y, z, m) records: every lane loads JT/256
// records with one coalesced 16-byte load each, the tile is written to LDS,
// and the inner loop reads record jj with one ds_read_b128 at a lane-uniform
// address, which the LDS broadcasts to all 64 lanes without bank conflicts.
// Tiles are double-buffered: the global loads for tile t+1 are in flight
// while tile t is consumed, and one barrier per tile separates the phases.
//
// Arithmetic per pair (KI independent chains per lane):
//   3 sub, 3 fma (|d|^2 + eps^2), v_rsq_f32, then either
//   refine=0: m*y, y*y, (m y)*(y y)                       3 mul
//   refine=1: one Newton-Raphson step folded into the products:
//             y2 = y*y, t = q*y2 - 3, u = y*t (= -2 rho), mr = (-m/2)*u
//             (= m rho), u2 = u*u, mr3 = mr*u2 (= 4 m rho^3); the 4 is
//             removed by an exact scale of the sums at the end   6 ops
//   phi -= m rho (1 op), a += mr3 * d (3 fma).
// The mass in LDS is pre-scaled by -1/2 when refining, so the step costs
// three VALU ops per pair, not four.  The "rcp" variants take rho^2 = 1/q
// from v_rcp_f32 instead of squaring (mr3 = m rho * rcp(q)): the
// transcendental unit issues beside the VALU, so this trades one VALU op
// per pair for a second transcendental.
//
// Accuracy.  Sums over a tile are formed in fresh registers and added to
// the running totals once per tile, so FP32 rounding grows with
// JT + nj/JT rather than nj.
#include <algorithm>

#include "newton_pair.h"
#include "pgh_internal.h"

namespace pgh {

__global__ void __launch_bounds__(256) k_pack_j(int n, const float *__restrict__ x,
                                                const float *__restrict__ y,
                                                const float *__restrict__ z,
                                                const float *__restrict__ m,
                                                float4 *__restrict__ dst)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = make_float4(x[i], y[i], z[i], m[i]);
}

hipError_t launch_pack_j(int n, const float *x, const float *y, const float *z, const float *m,
                         float4 *dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_j, dim3((n + 255) / 256), dim3(256), 0, s, n, x, y, z, m, dst);
    return hipGetLastError();
}

// Adds the S partial sums [S][4][n] of a j-split launch in split order
// (ax..az and phi each optional).
__global__ void __launch_bounds__(256) k_combine_split(int n, int S, const float *__restrict__ part,
                                                       float *ax, float *ay, float *az, float *phi)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f;
    for (int s = 0; s < S; ++s) {
        const float *p = part + (size_t)s * 4 * n;
        if (ax) {
            sx += p[i];
            sy += p[n + i];
            sz += p[2 * n + i];
        }
        if (phi) sp += p[3 * n + i];
    }
    if (ax) {
        ax[i] = sx;
        ay[i] = sy;
        az[i] = sz;
    }
    if (phi) phi[i] = sp;
}

hipError_t launch_combine_split(int n, int S, const float *part, float *ax, float *ay, float *az,
                                float *phi, hipStream_t s)
{
    if (n <= 0 || S <= 1) return hipSuccess;
    hipLaunchKernelGGL(k_combine_split, dim3((n + 255) / 256), dim3(256), 0, s, n, S, part, ax, ay,
                       az, phi);
    return hipGetLastError();
}

int split_count(int ni, int nj, int ki, int jt, int target_waves, size_t part_cap)
{
    const long waves = ((long)ni + 64L * ki - 1) / (64L * ki);
    long S = (target_waves + waves - 1) / waves;
    // at least two tiles per share, or one of 64 records (small i-sets,
    // whose waves come from the split alone)
    S = std::min(S, std::max(1L, (long)nj / (jt > 64 ? 2L * jt : (long)jt)));
    if (ni > 0) S = std::min(S, (long)(part_cap / (4 * (size_t)ni)));
    return (int)std::max(1L, S);
}

__global__ void __launch_bounds__(256) k_fill_zero(int n, float *a, float *b, float *c, float *d)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        if (a) a[i] = 0.f;
        if (b) b[i] = 0.f;
        if (c) c[i] = 0.f;
        if (d) d[i] = 0.f;
    }
}

hipError_t launch_fill_zero(int n, float *a, float *b, float *c, float *d, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3((n + 255) / 256), dim3(256), 0, s, n, a, b, c, d);
    return hipGetLastError();
}

namespace {

template <int KI, int JT, int U, bool RCP, bool REFINE, bool GUARD, bool PHI>
__global__ void __launch_bounds__(256) k_newton_allpairs(NewtonArgs a)
{
    static_assert(JT % 256 == 0 || JT == 64, "a tile is 64 records or whole workgroup rounds");
    constexpr int PER = JT >= 256 ? JT / 256 : 1;  // records each thread loads per tile
    __shared__ float4 tile[2][JT];

    const int tid = threadIdx.x;
    const int ibase = blockIdx.x * (256 * KI) + tid;
    const float mscale = REFINE ? -0.5f : 1.0f;

    float px[KI], py[KI], pz[KI], pe[KI];
    float tx[KI], ty[KI], tz[KI], tp[KI];
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        int i = ibase + k * 256;
        i = i < a.ni ? i : a.ni - 1;
        px[k] = a.xi[i];
        py[k] = a.yi[i];
        pz[k] = a.zi[i];
        pe[k] = a.eps2i ? a.eps2i[i] : a.eps2_all;
        tx[k] = ty[k] = tz[k] = tp[k] = 0.f;
    }

    // this workgroup's share of the j-particles (blockIdx.y splits them)
    const int jbase = blockIdx.y * a.jchunk;
    const int nj = max(0, min(a.jchunk, a.nj - jbase));
    const float4 *__restrict__ jm = a.jmem + jbase;
    const int ntiles = (nj + JT - 1) / JT;
    float4 pre[PER];

    // (a 64-record tile is loaded by the first wave of the workgroup)
    auto load_tile = [&](int t) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int j = t * JT + r * 256 + tid;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if ((JT >= 256 || tid < JT) && j < nj) v = jm[j];
            pre[r] = v;  // not touched until stored, so the load stays in flight
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            float4 v = pre[r];
            v.w *= mscale;
            if (JT >= 256 || tid < JT) tile[buf][r * 256 + tid] = v;
        }
    };

    load_tile(0);
    // Every global load so far (i-particles, first tile) must land before the
    // tile loop; waiting here, on a path every thread takes, keeps the
    // compiler from waiting on them (and on the next tile's prefetch queued
    // behind them) inside the inner loop.
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    store_tile(0);
    __syncthreads();

    for (int t = 0; t < ntiles; ++t) {
        const int cur = t & 1;
        set_tile_prio(ntiles - t, ntiles);
        if (t + 1 < ntiles) load_tile(t + 1);
        const int cnt = min(JT, nj - t * JT);

        float sx[KI], sy[KI], sz[KI], sp[KI];
#pragma unroll
        for (int k = 0; k < KI; ++k) sx[k] = sy[k] = sz[k] = sp[k] = 0.f;

        if (cnt == JT) {
#pragma unroll U
            for (int jj = 0; jj < JT; ++jj) {
                const float4 p = tile[cur][jj];
#pragma unroll
                for (int k = 0; k < KI; ++k)
                    newton_pair<REFINE, GUARD, PHI, RCP>(p, px[k], py[k], pz[k], pe[k], sx[k], sy[k],
                                                    sz[k], sp[k]);
            }
        } else {
#pragma unroll 2
            for (int jj = 0; jj < cnt; ++jj) {
                const float4 p = tile[cur][jj];
#pragma unroll
                for (int k = 0; k < KI; ++k)
                    newton_pair<REFINE, GUARD, PHI, RCP>(p, px[k], py[k], pz[k], pe[k], sx[k], sy[k],
                                                    sz[k], sp[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            tx[k] += sx[k];
            ty[k] += sy[k];
            tz[k] += sz[k];
            tp[k] += sp[k];
        }
        if (t + 1 < ntiles) store_tile(cur ^ 1);
        __syncthreads();
    }

    const float ascale = (REFINE && !RCP) ? 0.25f : 1.0f;
    // one j-share: write the outputs; several: partial sums for k_combine_split
    float *ox = a.ax, *oy = a.ay, *oz = a.az, *op = a.phi;
    if (gridDim.y > 1) {
        ox = a.part + (size_t)blockIdx.y * 4 * a.ni;
        oy = ox + a.ni;
        oz = oy + a.ni;
        op = oz + a.ni;
    }
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int i = ibase + k * 256;
        if (i < a.ni) {
            ox[i] = tx[k] * ascale;
            oy[i] = ty[k] * ascale;
            oz[i] = tz[k] * ascale;
            if (PHI) op[i] = tp[k];
        }
    }
}

using NewtonKernel = void (*)(NewtonArgs);

template <int KI, int JT, int U, bool RCP>
struct NewtonSet {
    static NewtonKernel get(bool refine, bool guard, bool phi)
    {
        const int sel = (refine ? 4 : 0) | (guard ? 2 : 0) | (phi ? 1 : 0);
        switch (sel) {
            case 0: return k_newton_allpairs<KI, JT, U, RCP, false, false, false>;
            case 1: return k_newton_allpairs<KI, JT, U, RCP, false, false, true>;
            case 2: return k_newton_allpairs<KI, JT, U, RCP, false, true, false>;
            case 3: return k_newton_allpairs<KI, JT, U, RCP, false, true, true>;
            case 4: return k_newton_allpairs<KI, JT, U, RCP, true, false, false>;
            case 5: return k_newton_allpairs<KI, JT, U, RCP, true, false, true>;
            case 6: return k_newton_allpairs<KI, JT, U, RCP, true, true, false>;
            default: return k_newton_allpairs<KI, JT, U, RCP, true, true, true>;
        }
    }
};

struct NewtonVariant {
    const char *name;
    int ki, jt;
    NewtonKernel (*get)(bool, bool, bool);
};

const NewtonVariant kNewtonVariants[] = {
    {"ki=1 jt=256 u=8", 1, 256, &NewtonSet<1, 256, 8, false>::get},
    {"ki=1 jt=64 u=8", 1, 64, &NewtonSet<1, 64, 8, false>::get},
    {"ki=2 jt=256 u=4", 2, 256, &NewtonSet<2, 256, 4, false>::get},
    {"ki=4 jt=256 u=2", 4, 256, &NewtonSet<4, 256, 2, false>::get},
    {"ki=2 jt=512 u=8", 2, 512, &NewtonSet<2, 512, 8, false>::get},
    {"ki=1 jt=256 u=8 rcp", 1, 256, &NewtonSet<1, 256, 8, true>::get},
    {"ki=2 jt=256 u=4 rcp", 2, 256, &NewtonSet<2, 256, 4, true>::get},
    {"ki=4 jt=256 u=2 rcp", 4, 256, &NewtonSet<4, 256, 2, true>::get},
};
constexpr int kNumNewtonVariants = sizeof(kNewtonVariants) / sizeof(kNewtonVariants[0]);

}  // namespace

int newton_allpairs_variants() { return kNumNewtonVariants; }

const char *newton_allpairs_variant_name(int v)
{
    return (v >= 0 && v < kNumNewtonVariants) ? kNewtonVariants[v].name : nullptr;
}

int newton_allpairs_default(int ni, int nj, int num_cu)
{
    (void)nj;
    // Measured with the j-split that holds 8 waves per SIMD: from 2^17
    // i-particles up, four per lane (fewer j-tile reads per pair) are the
    // fastest (N = 262144: 20.3 ms against 21.5 for one per lane); below, one
    // per lane keeps the shares long enough; an i-set of at most 16 waves per
    // 256 CUs takes the 64-record tiles, so that the j-split (one tile per
    // share at least) gives it a wave per CU or more.  pgh_autotune confirms
    // or replaces the choice for a given workload.
    if (ni <= 4 * num_cu) return 1;
    return ni >= (1 << 17) ? 3 : 0;
}

int newton_allpairs_split(int ni, int nj, int variant, size_t part_cap)
{
    const NewtonVariant &v = kNewtonVariants[variant];
    return split_count(ni, nj, v.ki, v.jt, kSplitTargetWaves, part_cap);
}

hipError_t launch_newton_allpairs(const NewtonArgs &a0, int variant, bool refine, bool guard,
                                  int S, hipStream_t s)
{
    if (a0.ni <= 0) return hipSuccess;
    const NewtonVariant &v = kNewtonVariants[variant];
    NewtonArgs a = a0;
    S = std::max(1, S);
    a.jchunk = (int)(((long)a.nj + (long)S * v.jt - 1) / ((long)S * v.jt) * v.jt);
    S = std::max(1, (a.nj + a.jchunk - 1) / a.jchunk);
    const int per_block = 256 * v.ki;
    const dim3 grid((a.ni + per_block - 1) / per_block, S);
    hipLaunchKernelGGL(v.get(refine, guard, a.phi != nullptr), grid, dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || S == 1) return e;
    return launch_combine_split(a.ni, S, a.part, a0.ax, a0.ay, a0.az, a0.phi, s);
}

}  // namespace pgh
