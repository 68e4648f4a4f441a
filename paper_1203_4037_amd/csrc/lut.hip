// All-pairs central force of arbitrary shape from the bit-binned look-up
// table on gfx950: Eq. (arbitrary_force) of Sec. 3 with the force procedure
// of Sec. 3.4.2.
//
// Per pair (unscaled FP32 positions; the paper pre-scales positions by
// sqrt(s_max-2)/rcut instead, which rounds every absolute coordinate once
// more and loses digits for close pairs, so the scale is applied to |d|^2):
//   d = r_j - r_i                                       3 sub
//   s = min(c |d|^2 + 2, s_max), c = (s_max-2)/rcut^2    mul, 2 fma, fma, min
//   k = bits(s)[23-F .. 23+E)  (low E exponent bits and high F fraction bits,
//       one v_bfe_u32), byte address 8k                  2 int
//   s_k = bits(s) with the low 23-F bits cleared         1 int
//   (G0, G1) = T[k], one ds_read_b64 from the LDS copy of the table
//   g = G0 + G1 (s - s_k)                                sub, fma
//   a += (m g) d                                         mul, 3 fma
// The table (2^(E+F) (G0, G1) pairs, at most 128 KiB) is copied into LDS once
// per workgroup; j-particles stream through LDS tiles exactly as in the
// Newton kernel.  Pairs beyond the cutoff clamp to s_max, whose node is the
// last one, where G0 = G1 = 0, so they add exactly zero.
#include <algorithm>

#include "table_pairs.h"
#include "pgh_internal.h"

namespace pgh {
namespace {

// PHI: also the potential from the second table (a.ptable, a.phi); the LDS
// table then holds (G0, G1, P0, P1) per node.  NT threads per workgroup.
template <int KI, int JT, int U, bool HT, bool PHI, int NT = 256>
__global__ void __launch_bounds__(NT) k_table_allpairs(TableArgs a)
{
    static_assert(JT % NT == 0, "tile must be a multiple of the workgroup");
    constexpr int PER = JT / NT;
    extern __shared__ float4 dyn4[];
    float2 *stab = (float2 *)dyn4;  // (G0, G1) per node
    float4 *stab4 = dyn4;           // (G0, G1, P0, P1) per node, with PHI
    __shared__ float4 tile[2][JT];

    const int tid = threadIdx.x;
    const int ibase = blockIdx.x * (NT * KI) + tid;
    const int K = 1 << (a.E + a.F);
    const unsigned shift = 23u - (unsigned)a.F;
    const unsigned nbits = (unsigned)(a.E + a.F);
    const unsigned hmask = ~((1u << shift) - 1u);
    const float c = a.c, smax = a.smax;

    if (PHI)
        tables_to_lds<HT>(stab4, a.table, a.ptable, K, shift);
    else
        table_to_lds<HT>(stab, a.table, K, shift);

    float px[KI], py[KI], pz[KI];
    float tx[KI], ty[KI], tz[KI], tp[KI];
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        int i = ibase + k * NT;
        i = i < a.ni ? i : a.ni - 1;
        px[k] = a.xi[i];
        py[k] = a.yi[i];
        pz[k] = a.zi[i];
        tx[k] = ty[k] = tz[k] = tp[k] = 0.f;
    }

    // this workgroup's share of the j-particles (blockIdx.y splits them)
    const int jbase = blockIdx.y * a.jchunk;
    const int nj = max(0, min(a.jchunk, a.nj - jbase));
    const float4 *__restrict__ jm = a.jmem + jbase;
    const int ntiles = (nj + JT - 1) / JT;
    float4 pre[PER];
    auto load_tile = [&](int t) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int j = t * JT + r * NT + tid;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < nj) v = jm[j];
            pre[r] = v;
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int r = 0; r < PER; ++r) tile[buf][r * NT + tid] = pre[r];
    };

    load_tile(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): see the Newton kernel
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
        auto pair = [&](const float4 p) {
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                if (PHI)
                    table_pair_pot<HT>(p, px[k], py[k], pz[k], stab4, c, smax, shift, nbits, hmask,
                                       sx[k], sy[k], sz[k], sp[k]);
                else
                    table_pair<HT>(p, px[k], py[k], pz[k], stab, c, smax, shift, nbits, hmask,
                                   sx[k], sy[k], sz[k]);
            }
        };
        if (cnt == JT) {
#pragma unroll U
            for (int jj = 0; jj < JT; ++jj) pair(tile[cur][jj]);
        } else {
#pragma unroll 2
            for (int jj = 0; jj < cnt; ++jj) pair(tile[cur][jj]);
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

    float *ox = a.ax, *oy = a.ay, *oz = a.az, *op = a.phi;
    if (gridDim.y > 1) {
        ox = a.part + (size_t)blockIdx.y * 4 * a.ni;
        oy = ox + a.ni;
        oz = oy + a.ni;
        op = oz + a.ni;
    }
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int i = ibase + k * NT;
        if (i < a.ni) {
            ox[i] = tx[k];
            oy[i] = ty[k];
            oz[i] = tz[k];
            if (PHI) op[i] = tp[k];
        }
    }
}

using TableKernel = void (*)(TableArgs);

// Tables of more than 32 KiB in LDS (2^13 nodes and more, or 2^12 with the
// potential) leave room for one or two workgroups per CU, so they run
// workgroups of 12 waves (three per SIMD) over 768-record j-tiles: 128 KiB
// of table and 24 KiB of tiles fit the 160 KiB of a CU.  With four-wave
// workgroups such a table left one or two waves per SIMD, too few to hide
// the LDS latency of the table reads or to pair FP32 issue.
constexpr int kWideNT = 768;
constexpr size_t kWideTableBytes = 32768;
// the j-split target of wide launches: three rounds of one workgroup on each
// of 256 CUs
constexpr int kWideTargetWaves = 3 * (kWideNT / 64) * 256;

struct TableVariant {
    const char *name;
    int ki, jt;
    TableKernel fn, fn_phi;      // force only; force and potential
    TableKernel wide, wide_phi;  // the same with kWideNT threads and tiles
};

#define PGH_TABLE_VARIANT(name, KI, JT, U, HT)                                                   \
    {name,                                                                                     \
     KI,                                                                                       \
     JT,                                                                                       \
     k_table_allpairs<KI, JT, U, HT, false>,                                                   \
     k_table_allpairs<KI, JT, U, HT, true>,                                                    \
     k_table_allpairs<KI, kWideNT, U, HT, false, kWideNT>,                                     \
     k_table_allpairs<KI, kWideNT, U, HT, true, kWideNT>}
const TableVariant kTableVariants[] = {
    PGH_TABLE_VARIANT("ki=1 jt=256 u=4", 1, 256, 4, false),
    PGH_TABLE_VARIANT("ki=2 jt=256 u=4", 2, 256, 4, false),
    PGH_TABLE_VARIANT("ki=4 jt=256 u=2", 4, 256, 2, false),
    PGH_TABLE_VARIANT("ki=1 jt=256 u=4 htab", 1, 256, 4, true),
    PGH_TABLE_VARIANT("ki=2 jt=256 u=4 htab", 2, 256, 4, true),
};
#undef PGH_TABLE_VARIANT
constexpr int kNumTableVariants = sizeof(kTableVariants) / sizeof(kTableVariants[0]);

bool is_phi(const TableArgs &a) { return a.phi && a.ptable; }

size_t table_lds_bytes(const TableArgs &a)
{
    return (is_phi(a) ? sizeof(float4) : sizeof(float2)) << (a.E + a.F);
}

}  // namespace

int table_allpairs_variants() { return kNumTableVariants; }

const char *table_allpairs_variant_name(int v)
{
    return (v >= 0 && v < kNumTableVariants) ? kTableVariants[v].name : nullptr;
}

int table_allpairs_default(int ni, int nj, int num_cu)
{
    (void)nj;
    const long waves_ki2 = (long)(ni + 127) / 128;
    return waves_ki2 >= 4L * num_cu ? 1 : 0;
}

int table_allpairs_split(const TableArgs &a, int variant, size_t part_cap)
{
    const TableVariant &v = kTableVariants[variant];
    if (table_lds_bytes(a) > kWideTableBytes)
        return split_count(a.ni, a.nj, v.ki, kWideNT, kWideTargetWaves, part_cap);
    return split_count(a.ni, a.nj, v.ki, v.jt, kSplitTargetWaves, part_cap);
}

hipError_t launch_table_allpairs(const TableArgs &a0, int variant, int S, hipStream_t s)
{
    if (a0.ni <= 0) return hipSuccess;
    const TableVariant &v = kTableVariants[variant];
    TableArgs a = a0;
    const bool phi = is_phi(a);
    const size_t lds = table_lds_bytes(a);
    const bool wide = lds > kWideTableBytes;
    const int nt = wide ? kWideNT : 256, jt = wide ? kWideNT : v.jt;
    S = std::max(1, S);
    a.jchunk = (int)(((long)a.nj + (long)S * jt - 1) / ((long)S * jt) * jt);
    S = std::max(1, (a.nj + a.jchunk - 1) / a.jchunk);
    const int per_block = nt * v.ki;
    const dim3 grid((a.ni + per_block - 1) / per_block, S);
    const auto kern = wide ? (phi ? v.wide_phi : v.wide) : (phi ? v.fn_phi : v.fn);
    hipError_t e = allow_dynamic_lds((const void *)kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(nt), lds, s, a);
    e = hipGetLastError();
    if (e != hipSuccess || S == 1) return e;
    return launch_combine_split(a.ni, S, a.part, a0.ax, a0.ay, a0.az, phi ? a0.phi : nullptr, s);
}

namespace {

// Gradient with respect to the node values when the slopes are derived from
// them, G1_k = (G0_{k+1} - G0_k) / (s_{k+1} - s_k) for k < K-1 (the table
// definition of Sec. 3.4.1), given the gradients with respect to G0 and G1
// as independent entries (interleaved like the table):
//   dL/dG0_k (total) = dL/dG0_k + dL/dG1_{k-1} / ds_{k-1} - dL/dG1_k / ds_k,
// each term present where its index exists (G1_{K-1} is the constant 0).
__global__ void __launch_bounds__(256) k_table_grad_chain(int K, unsigned shift,
                                                          const float *__restrict__ g,
                                                          float *__restrict__ out)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    // node s_k: the FP32 bits of 2.0 stepped by k units of the F-th fraction bit
    auto node = [&](int q) { return __uint_as_float(0x40000000u + ((unsigned)q << shift)); };
    float v = g[2 * k];
    if (k >= 1) v += g[2 * (k - 1) + 1] / (node(k) - node(k - 1));
    if (k + 1 < K) v -= g[2 * k + 1] / (node(k + 1) - node(k));
    out[k] = v;
}

}  // namespace

hipError_t launch_table_grad_chain(int E, int F, const float *g, float *out, hipStream_t s)
{
    const int K = 1 << (E + F);
    hipLaunchKernelGGL(k_table_grad_chain, dim3((K + 255) / 256), dim3(256), 0, s, K,
                       23u - (unsigned)F, g, out);
    return hipGetLastError();
}

}  // namespace pgh
