// Per-pair arithmetic of the table force: one interaction of
// Eq. arbitrary_force through the bit-binned table (Sec. 3.4.2), in the forms
// of the all-pairs, batched and adjoint kernels, and the table's copy into
// LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace pgh {

// HT (the "htab" variants): the LDS copy holds (H_k, G1_k) with
// H_k = G0_k - G1_k s_k (one FMA rounding per node, formed when the table is
// copied into LDS), so the interpolation is g = H_k + G1_k s: the same number
// in exact arithmetic without the s - s_k subtraction and the mask that finds
// s_k.  The price is that rounding, up to 2^-24 |G1_k| s_k: against the
// force at the bin it is small except near rcut, where g goes to zero while
// G1_k s_k does not, so these are variants and not the default.
template <bool HT>
__device__ __forceinline__ void table_pair(const float4 p, float px, float py, float pz,
                                           const float2 *__restrict__ stab, float c, float smax,
                                           unsigned shift, unsigned nbits, unsigned hmask,
                                           float &sx, float &sy, float &sz)
{
    const float dx = p.x - px;
    const float dy = p.y - py;
    const float dz = p.z - pz;
    float r2 = dx * dx;
    r2 = __builtin_fmaf(dy, dy, r2);
    r2 = __builtin_fmaf(dz, dz, r2);
    const float s = __builtin_fminf(__builtin_fmaf(r2, c, 2.0f), smax);
    const unsigned u = __float_as_uint(s);
    const unsigned k = __builtin_amdgcn_ubfe(u, shift, nbits);
    const float2 g01 = stab[k];
    float g;
    if (HT) {
        g = __builtin_fmaf(g01.y, s, g01.x);
    } else {
        const float sk = __uint_as_float(u & hmask);
        g = __builtin_fmaf(g01.y, s - sk, g01.x);
    }
    const float mg = p.w * g;
    sx = __builtin_fmaf(mg, dx, sx);
    sy = __builtin_fmaf(mg, dy, sy);
    sz = __builtin_fmaf(mg, dz, sz);
}

// Copies the 2^(E+F) (G0, G1) table into LDS (all threads of the
// workgroup), converting to (H, G1) for the HT form.  shift = 23 - F.
// Four loads per thread are in flight at once (a table of 1024 entries is
// one round for 256 threads), so the copy costs one memory latency.
template <bool HT>
__device__ __forceinline__ void table_to_lds(float2 *stab, const float2 *__restrict__ table, int K,
                                             unsigned shift)
{
    const int nt = blockDim.x;
    for (int k0 = threadIdx.x; k0 < K; k0 += 4 * nt) {
        float2 e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * nt;
            e[u] = k < K ? table[k] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * nt;
            if (k < K) {
                if (HT) {
                    // node s_k: the FP32 bits of 2.0 stepped by k units of the F-th fraction bit
                    const float sk = __uint_as_float(0x40000000u + ((unsigned)k << shift));
                    e[u].x = __builtin_fmaf(-e[u].y, sk, e[u].x);
                }
                stab[k] = e[u];
            }
        }
    }
}

// The table force with the potential from a second table on the same bins
// (P0_k = p(r_k) and chords P1_k): the LDS copy holds (G0, G1, P0, P1) per
// node (in the HT form (H, G1, PH, P1) with PH_k = P0_k - P1_k s_k), read
// with one ds_read_b128; phi_i += m_j (P0 + P1 (s - s_k)).
template <bool HT>
__device__ __forceinline__ void table_pair_pot(const float4 p, float px, float py, float pz,
                                               const float4 *__restrict__ stab, float c,
                                               float smax, unsigned shift, unsigned nbits,
                                               unsigned hmask, float &sx, float &sy, float &sz,
                                               float &sp)
{
    const float dx = p.x - px;
    const float dy = p.y - py;
    const float dz = p.z - pz;
    float r2 = dx * dx;
    r2 = __builtin_fmaf(dy, dy, r2);
    r2 = __builtin_fmaf(dz, dz, r2);
    const float s = __builtin_fminf(__builtin_fmaf(r2, c, 2.0f), smax);
    const unsigned u = __float_as_uint(s);
    const unsigned k = __builtin_amdgcn_ubfe(u, shift, nbits);
    const float4 t = stab[k];
    float g, q;
    if (HT) {
        g = __builtin_fmaf(t.y, s, t.x);
        q = __builtin_fmaf(t.w, s, t.z);
    } else {
        const float ds = s - __uint_as_float(u & hmask);
        g = __builtin_fmaf(t.y, ds, t.x);
        q = __builtin_fmaf(t.w, ds, t.z);
    }
    const float mg = p.w * g;
    sx = __builtin_fmaf(mg, dx, sx);
    sy = __builtin_fmaf(mg, dy, sy);
    sz = __builtin_fmaf(mg, dz, sz);
    sp = __builtin_fmaf(p.w, q, sp);
}

// Copies the force and potential tables into one LDS array of (G0, G1, P0,
// P1) per node (HT: the constant terms in the (H, G1) form).  shift = 23 - F.
template <bool HT>
__device__ __forceinline__ void tables_to_lds(float4 *stab, const float2 *__restrict__ table,
                                              const float2 *__restrict__ ptable, int K,
                                              unsigned shift)
{
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float2 g = table[k], q = ptable[k];
        float4 e = make_float4(g.x, g.y, q.x, q.y);
        if (HT) {
            const float sk = __uint_as_float(0x40000000u + ((unsigned)k << shift));
            e.x = __builtin_fmaf(-e.y, sk, e.x);
            e.z = __builtin_fmaf(-e.w, sk, e.z);
        }
        stab[k] = e;
    }
}

// ---------------------------------------------------------------------------
// The table pair of the batched kernels, written for gfx950's issue rates
// (measured on the device): FP32 add, sub, mul and FMA, and the integer
// shift, and, or, xor and add, issue at twice the rate of v_min/v_max,
// v_bfe_u32 and v_lshl_add_u32, and any VALU instruction that reads an SGPR
// operand issues at the lower rate.  So every uniform operand is held in a
// VGPR, and the bin's byte offset in the LDS table is a shift and a mask of
// bits(s) (two fast instructions) rather than v_bfe_u32 and v_lshl_add_u32
// (two slow ones); the clamp at s_max is the one slow instruction per pair.
// ---------------------------------------------------------------------------

// A uniform value moved into a VGPR, so that the compiler does not read it
// from an SGPR in every pair.
__device__ __forceinline__ float in_vgpr(float x)
{
    float r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

__device__ __forceinline__ unsigned in_vgpr(unsigned x)
{
    unsigned r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// Operands of table_pair_v (each in a VGPR).  For an LDS table of entries
// of 2^eb bytes (eb = 3: (G0, G1); eb = 4: (G0, G1, P0, P1)):
//   sh = 23 - F - eb: (bits(s) >> sh) & am is the byte offset of s's node,
//   am = (2^(E+F) - 1) << eb,
//   hm = ~(2^(23-F) - 1): bits(s) & hm are the bits of the node s_k.
struct TableConsts {
    float c;
    unsigned smax_bits;  // bits(s_max)
    unsigned sh, am, hm;
};

__device__ __forceinline__ TableConsts table_consts(float c, float smax, int E, int F, int eb)
{
    TableConsts k;
    k.c = in_vgpr(c);
    k.smax_bits = in_vgpr(__float_as_uint(smax));
    k.sh = in_vgpr((unsigned)(23 - F - eb));
    k.am = in_vgpr((((1u << (E + F)) - 1u) << eb));
    k.hm = in_vgpr(~((1u << (23 - F)) - 1u));
    return k;
}

// KI pairs of Eq. arbitrary_force through the table (the steps of
// Sec. 3.4.2): one j-record p against the lane's KI i-particles, with the
// table at byte address `tab` in LDS; with PHI the entries are
// (G0, G1, P0, P1) and sp accumulates m_j p(s).  HT: the constant terms are
// in the (H, G1) form, g = H_k + G1_k s.  The KI pairs are written step by
// step side by side so that their LDS gathers are in flight together.  The
// clamp at s_max compares the bit patterns (v_min_u32): for s >= 2 their
// order is the order of the numbers, and unlike v_min_f32 it needs no
// quieting of its operands.
// The pairs' state between issuing their table gathers and using them.
template <int KI, bool PHI>
struct TableGather {
    using Entry = std::conditional_t<PHI, float4, float2>;
    float dx[KI], dy[KI], dz[KI], ds[KI];
    Entry t[KI];
};

// First half of table_pairs_v: differences, s, the bin's offset and its LDS
// gather (issued, not waited for) and s - s_k.
template <int KI, bool HT, bool PHI>
__device__ __forceinline__ void table_head(const float4 p, const float *px, const float *py,
                                           const float *pz, const char *__restrict__ tab,
                                           const TableConsts &k, TableGather<KI, PHI> &q)
{
    using Entry = typename TableGather<KI, PHI>::Entry;
    unsigned u[KI];
#pragma unroll
    for (int i = 0; i < KI; ++i) {
        q.dx[i] = p.x - px[i];
        q.dy[i] = p.y - py[i];
        q.dz[i] = p.z - pz[i];
    }
#pragma unroll
    for (int i = 0; i < KI; ++i) {
        float r2 = q.dx[i] * q.dx[i];
        r2 = __builtin_fmaf(q.dy[i], q.dy[i], r2);
        r2 = __builtin_fmaf(q.dz[i], q.dz[i], r2);
        u[i] = min(__float_as_uint(__builtin_fmaf(r2, k.c, 2.0f)), k.smax_bits);
    }
#pragma unroll
    for (int i = 0; i < KI; ++i) q.t[i] = *(const Entry *)(tab + ((u[i] >> k.sh) & k.am));
#pragma unroll
    for (int i = 0; i < KI; ++i)
        q.ds[i] = HT ? __uint_as_float(u[i]) : __uint_as_float(u[i]) - __uint_as_float(u[i] & k.hm);
}

// Second half: the interpolated g (and p) and the sums; mj the j-mass.
template <int KI, bool PHI>
__device__ __forceinline__ void table_tail(const float mj, const TableGather<KI, PHI> &q,
                                           float *sx, float *sy, float *sz, float *sp)
{
#pragma unroll
    for (int i = 0; i < KI; ++i) {
        const float g = __builtin_fmaf(q.t[i].y, q.ds[i], q.t[i].x);
        const float mg = mj * g;
        sx[i] = __builtin_fmaf(mg, q.dx[i], sx[i]);
        sy[i] = __builtin_fmaf(mg, q.dy[i], sy[i]);
        sz[i] = __builtin_fmaf(mg, q.dz[i], sz[i]);
        if constexpr (PHI) sp[i] = __builtin_fmaf(mj, __builtin_fmaf(q.t[i].w, q.ds[i], q.t[i].z), sp[i]);
    }
}

// table_tail in the paper's form with the i-side moments of the adjoint of
// L = sum_i w_i . a_i: the derivative of m_j g d with respect to r_i is
// -m_j (g I + 2c G1_k d d^T) inside a bin, so dL/dr_i = -(S_i w_i +
// 2c M_i w_i) with S_i = sum_j m_j g and M_i = sum_j m_j G1_k d d^T
// (sm[0][.] = S, sm[1..6][.] = Mxx, Mxy, Mxz, Myy, Myz, Mzz).
template <int KI>
__device__ __forceinline__ void table_tail_mom(const float mj, const TableGather<KI, false> &q,
                                               float *sx, float *sy, float *sz, float (*sm)[KI])
{
#pragma unroll
    for (int i = 0; i < KI; ++i) {
        const float g = __builtin_fmaf(q.t[i].y, q.ds[i], q.t[i].x);
        const float mg = mj * g;
        sx[i] = __builtin_fmaf(mg, q.dx[i], sx[i]);
        sy[i] = __builtin_fmaf(mg, q.dy[i], sy[i]);
        sz[i] = __builtin_fmaf(mg, q.dz[i], sz[i]);
        sm[0][i] += mg;
        const float mg1 = mj * q.t[i].y;
        const float ux = mg1 * q.dx[i], uy = mg1 * q.dy[i];
        sm[1][i] = __builtin_fmaf(ux, q.dx[i], sm[1][i]);
        sm[2][i] = __builtin_fmaf(ux, q.dy[i], sm[2][i]);
        sm[3][i] = __builtin_fmaf(ux, q.dz[i], sm[3][i]);
        sm[4][i] = __builtin_fmaf(uy, q.dy[i], sm[4][i]);
        sm[5][i] = __builtin_fmaf(uy, q.dz[i], sm[5][i]);
        sm[6][i] = __builtin_fmaf(mg1 * q.dz[i], q.dz[i], sm[6][i]);
    }
}

template <int KI>
__device__ __forceinline__ void table_pairs_mom(const float4 p, const float *px, const float *py,
                                                const float *pz, const char *__restrict__ tab,
                                                const TableConsts &k, float *sx, float *sy,
                                                float *sz, float (*sm)[KI])
{
    TableGather<KI, false> q;
    table_head<KI, false, false>(p, px, py, pz, tab, k, q);
    table_tail_mom<KI>(p.w, q, sx, sy, sz, sm);
}

template <int KI, bool HT, bool PHI>
__device__ __forceinline__ void table_pairs_v(const float4 p, const float *px, const float *py,
                                              const float *pz, const char *__restrict__ tab,
                                              const TableConsts &k, float *sx, float *sy,
                                              float *sz, float *sp)
{
    TableGather<KI, PHI> q;
    table_head<KI, HT, PHI>(p, px, py, pz, tab, k, q);
    table_tail<KI, PHI>(p.w, q, sx, sy, sz, sp);
}

}  // namespace pgh
