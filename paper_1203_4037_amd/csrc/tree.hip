// Barnes-Hut tree on gfx950 that produces the (i-group, j-list) interaction
// lists of the tree code of Sec. 5 (Barnes' shared lists for groups of
// i-particles; opening parameter theta; monopole moments, or quadrupole
// moments carried by pseudo-particles after Kawai & Makino) for the batched
// force kernels.
//
// Definitions (the FP64 oracle the tests compare against implements the same
// definitions in code of its own):
//   frame   lo = componentwise minimum of the positions, extent = the largest
//           axis range, scale = 2^21 / extent, all FP32;
//   keys    per axis min(floor((x - lo) * scale), 2^21 - 1) (FP32 subtract and
//           multiply, no contraction), 3-bit digits x|y|z from the top;
//   order   sort by (key, original index) -- a stable radix sort of the keys;
//   octree  a node of level L holds the particles sharing its first 3L key
//           bits; it splits into its non-empty octants when it holds more than
//           n_leaf particles and L < 21; nodes numbered breadth first, each
//           level in key order; node size extent / 2^L;
//   moments FP64 mass, centre of mass (plain mean when the mass is zero) and
//           second moment about it;
//   pseudo  monopole: (com, M); quadrupole: three particles of mass M/3 at
//           com + a cos(2 pi k/3) e1 + b sin(2 pi k/3) e2 from the principal
//           axes of S (a^2 = 2 (l1 - l3)/M, b^2 = 2 (l2 - l3)/M): the node's
//           mass, zero dipole and the traceless part of S;
//   groups  nodes holding at most n_crit particles (or leaves) whose parent
//           holds more, in key order;
//   walk    breadth first from the root per group; g and its ancestors are
//           opened; another node is accepted when (l/theta)^2 < d^2, d the
//           distance from its com to the group's bounding box, and adds its
//           pseudo-particles; an opened leaf adds its particles.
//
// The build launches every level with its size in a device table and waits
// for the stream once, at its end (the walk waits after its counting pass);
// neither is meant for graph capture.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "pgh_internal.h"

namespace pgh {
namespace {

constexpr unsigned long long kMask21 = (1ull << 21) - 1;

__device__ inline unsigned ord_of(float f)
{
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

float float_of_ord(unsigned o)
{
    const unsigned u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
}

__global__ void k_init_words(unsigned *w)
{
    const int i = threadIdx.x;
    if (i < 16) w[i] = (i < 3) ? 0xffffffffu : 0u;  // min ords, max ords, counters
}

// Componentwise min / max of the positions into w[0..2] / w[3..5] as ordered
// integers (atomics on the order-preserving image of the float).
__global__ void __launch_bounds__(256) k_frame(int n, const float *__restrict__ x,
                                               const float *__restrict__ y,
                                               const float *__restrict__ z, unsigned *w)
{
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float v[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], v[a]);
            hi[a] = fmaxf(hi[a], v[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
        for (int o = 32; o > 0; o >>= 1) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
        }
    // the workgroup's four waves, then one atomic per workgroup and value
    // (one per wave would queue thousands on the same six words)
    __shared__ float part[4][6];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) part[wv][a] = lo[a], part[wv][3 + a] = hi[a];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        float v = part[0][a];
        for (int k = 1; k < 4; ++k) v = a < 3 ? fminf(v, part[k][a]) : fmaxf(v, part[k][a]);
        if (a < 3)
            atomicMin(&w[a], ord_of(v));
        else
            atomicMax(&w[a], ord_of(v));
    }
}

// 21-bit integer -> bits at positions 0, 3, 6, ... (shift-and-mask spreading)
__device__ inline unsigned long long spread3(unsigned long long v)
{
    v &= kMask21;
    v = (v | (v << 32)) & 0x001F00000000FFFFull;
    v = (v | (v << 16)) & 0x001F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline unsigned long long cell_of(float v, float lo, float scale)
{
    const float t = __fmul_rn(__fsub_rn(v, lo), scale);
    const float f = fminf(fmaxf(floorf(t), 0.f), 2097151.f);
    return (unsigned long long)f;
}

// Keys in input order, with the particles packed (x, y, z, m) in input order
// for the gather (one 16-byte load per particle instead of four 4-byte ones).
__global__ void __launch_bounds__(256) k_keys(int n, const float *__restrict__ x,
                                              const float *__restrict__ y,
                                              const float *__restrict__ z,
                                              const float *__restrict__ m, float lox, float loy,
                                              float loz, float scale,
                                              unsigned long long *__restrict__ key,
                                              int *__restrict__ iota, float4 *__restrict__ xin)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float px = x[i], py = y[i], pz = z[i];
    const unsigned long long kx = cell_of(px, lox, scale), ky = cell_of(py, loy, scale),
                             kz = cell_of(pz, loz, scale);
    key[i] = (spread3(kx) << 2) | (spread3(ky) << 1) | spread3(kz);
    iota[i] = i;
    xin[i] = make_float4(px, py, pz, m[i]);
}

// The particles in key order, and each particle's rank (inv[perm[r]] = r).
__global__ void __launch_bounds__(256) k_gather(int n, const int *__restrict__ perm,
                                                const float4 *__restrict__ xin, float *xs,
                                                float *ys, float *zs, float *ms, float4 *xm,
                                                int *__restrict__ inv)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const int i = perm[r];
    inv[i] = r;
    const float4 v = xin[i];
    xs[r] = v.x;
    ys[r] = v.y;
    zs[r] = v.z;
    ms[r] = v.w;
    xm[r] = v;
}

// Level table of the octree build: level L holds nodes [lvl[L], lvl[L + 1]);
// the write kernel of level L sets lvl[L + 2].  All sizes stay on the device:
// the host launches every level without waiting for the one before.
constexpr int kLvl = kTreeMaxLevel + 3;
// word indices in TreeState::word
constexpr int kWordLeaves = 6, kWordOverflow = 9, kWordMaxLevel = 10;

__global__ void k_root(int n, int *begin, int *count, int *level, int *parent, int *lvl)
{
    begin[0] = 0;
    count[0] = n;
    level[0] = 0;
    parent[0] = -1;
    lvl[0] = 0;
    lvl[1] = 1;
    for (int L = 2; L < kLvl; ++L) lvl[L] = 1;
}

__device__ inline int digit_of(unsigned long long k, int L)
{
    return (int)((k >> (3 * (kTreeMaxLevel - L))) & 7ull);
}

// First r in [lo, hi) whose digit at level L is >= d (keys sorted and sharing
// the digits above L, so the digit is non-decreasing in r).
__device__ inline int lower_digit(const unsigned long long *key, int lo, int hi, int d, int L)
{
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (digit_of(key[mid], L) < d)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// The split of level L in three kernels, with the level's size read on the
// device: k_split_count (block b takes the b-th of kSplitBlocks contiguous
// chunks of the level's nodes), k_split_scan (one workgroup: the chunks'
// offsets and the next level's size), k_split_write (the same chunks again:
// each node's children go to the next level at its offset).
constexpr int kSplitBlocks = 2048;

// Inclusive prefix sum over the 64 lanes of a wave (all lanes active) by DPP
// lane moves: the sums of up to four lanes inside each row of 16 (row shifts
// by 1, 2 and 3 of the value), then of eight and of the whole row (row shifts
// by 4 and 8 of the partial sums into the upper banks), then across rows (lane
// 15 of row 0 and 2 broadcast into rows 1 and 3, lane 31 into rows 2 and 3).
__device__ inline int wave_incl_scan(int x)
{
    int v = x + __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true);          // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, x, 0x113, 0xF, 0xF, true);          // row_shr:3
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xE, false);         // row_shr:4, banks 1-3
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xC, false);         // row_shr:8, banks 2-3
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);         // row_bcast:15, rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);         // row_bcast:31, rows 2, 3
    return v;
}

// Inclusive scan over a workgroup of 256 (wave scans, then the wave totals);
// *total receives the workgroup's sum.  Every thread of the workgroup calls it.
__device__ inline int block_incl_scan(int v, int *sh, int *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wave_incl_scan(v);
    if (lane == 63) sh[wv] = v;
    __syncthreads();
    int add = 0;
    for (int k = 0; k < wv; ++k) add += sh[k];
    *total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return v + add;
}

__device__ inline void split_chunk(int n, int *lo, int *hi)
{
    const int chunk = (n + kSplitBlocks - 1) / kSplitBlocks;
    *lo = min(n, (int)blockIdx.x * chunk);
    *hi = min(n, *lo + chunk);
}

// nc[i] = non-empty children of the i-th node of level L (0 for a leaf),
// bnd[7 i + d - 1] = the first particle of its child digits >= d (d = 1..7;
// for split nodes only), bsum[b] = the children of chunk b;
// w[kWordLeaves] counts the leaves (one atomic per workgroup).  Eight lanes
// take a node, lane d - 1 searching boundary d over the whole node (the
// searches are independent, so a node costs one binary search of latency).
__global__ void __launch_bounds__(256) k_split_count(int L, int n_leaf,
                                                     const int *__restrict__ lvl,
                                                     const int *__restrict__ begin,
                                                     const int *__restrict__ count,
                                                     const unsigned long long *__restrict__ key,
                                                     int *__restrict__ nc, int *__restrict__ bnd,
                                                     int *__restrict__ bsum, unsigned *w)
{
    __shared__ int sh[4];
    if (w[kWordOverflow]) return;
    const int off = lvl[L], n_level = lvl[L + 1] - off;
    int lo, hi;
    split_chunk(n_level, &lo, &hi);
    const int g = (int)threadIdx.x >> 3, j = (int)threadIdx.x & 7;
    int kids = 0, leaves = 0;
    for (int i0 = lo; i0 < hi; i0 += 32) {  // uniform trip count for the workgroup
        const int i = i0 + g;
        int b = 0, c = 0;
        if (i < hi) {
            b = begin[off + i];
            c = count[off + i];
        }
        const bool split = i < hi && c > n_leaf && L < kTreeMaxLevel;
        int p = b + c;  // lane 7: the node's end
        if (split && j < 7) p = lower_digit(key, b, b + c, j + 1, L + 1);
        // child j of the node is [boundary j, boundary j + 1), boundary 0 = b
        // (DPP lane moves: the lane before, then the sum over the group by
        // the pairs inside each quad and the half-row mirror)
        const int q = __builtin_amdgcn_update_dpp(0, p, 0x111, 0xF, 0xF, true);  // row_shr:1
        const int start = j == 0 ? b : q;
        int k = (split && p > start) ? 1 : 0;
        k += __builtin_amdgcn_update_dpp(0, k, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        k += __builtin_amdgcn_update_dpp(0, k, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
        k += __builtin_amdgcn_update_dpp(0, k, 0x141, 0xF, 0xF, false);  // row_half_mirror
        if (split && j < 7) bnd[7 * (size_t)i + j] = p;
        if (i < hi && j == 0) {
            nc[i] = k;
            kids += k;
            leaves += k == 0;
        }
    }
    int tot = 0;
    block_incl_scan(kids, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
    block_incl_scan(leaves, sh, &tot);
    if (threadIdx.x == 0 && tot) atomicAdd(&w[kWordLeaves], (unsigned)tot);
}

// The chunks' exclusive offsets in bsum, and the next level's size in
// lvl[L + 2].  Children that would pass the node capacity set the overflow
// word instead: every later kernel of the build returns at once, and the
// host builds again with more room.
__global__ void __launch_bounds__(256) k_split_scan(int L, int cap, int *lvl, int *bsum,
                                                    unsigned *w)
{
    __shared__ int sh[4];
    if (w[kWordOverflow]) return;
    constexpr int per = kSplitBlocks / 256;
    int v[per], sum = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = bsum[per * threadIdx.x + k];
        sum += v[k];
    }
    int tot = 0;
    int run = block_incl_scan(sum, sh, &tot) - sum;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        bsum[per * threadIdx.x + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) {
        const int next_off = lvl[L + 1];
        if ((long long)next_off + tot > cap) {
            atomicOr(&w[kWordOverflow], 1u);
            lvl[L + 2] = next_off;
        } else {
            lvl[L + 2] = next_off + tot;
            atomicMax(&w[kWordMaxLevel], (unsigned)tot);
        }
    }
}

// Writes the children of level L (from the bounds k_split_count kept) at
// lvl[L + 1] + the node's offset.
__global__ void __launch_bounds__(256) k_split_write(int L, const int *__restrict__ lvl,
                                                     const int *__restrict__ nc,
                                                     const int *__restrict__ bnd,
                                                     const int *__restrict__ bsum, int *begin,
                                                     int *count, int *level, int *first_child,
                                                     int *n_child, int *parent,
                                                     const unsigned *w)
{
    __shared__ int sh[4];
    if (w[kWordOverflow]) return;
    const int off = lvl[L], n_level = lvl[L + 1] - off, next_off = lvl[L + 1];
    int lo, hi;
    split_chunk(n_level, &lo, &hi);
    int run = bsum[blockIdx.x];
    for (int t0 = lo; t0 < hi; t0 += 256) {  // uniform trip count for the workgroup
        const int i = t0 + (int)threadIdx.x;
        const int k = i < hi ? nc[i] : 0;
        int tot = 0;
        const int incl = block_incl_scan(k, sh, &tot);
        if (i < hi) {
            const int node = off + i;
            const int fc = next_off + run + incl - k;
            if (k) {
                const int b = begin[node], c = count[node];
                int prev = b, j = fc;
                for (int d = 1; d <= 8; ++d) {
                    const int p = d == 8 ? b + c : bnd[7 * (size_t)i + d - 1];
                    if (p > prev) {
                        begin[j] = prev;
                        count[j] = p - prev;
                        level[j] = L + 1;
                        parent[j] = node;
                        ++j;
                    }
                    prev = p;
                }
            }
            first_child[node] = k ? fc : -1;
            n_child[node] = k;
        }
        run += tot;
    }
}

// v from another lane of the same 8-lane group by a DPP lane pattern (a
// VALU move, no LDS round trip): both 32-bit halves.
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 8 lanes of a node's lane group, the same in every lane: the
// lane pairs i ^ 1 and i ^ 2 inside each quad (quad_perm [1,0,3,2] and
// [2,3,0,1]), then the two quads (the half-row mirror, i <-> 7 - i).
__device__ inline double group_sum(double v)
{
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    return v;
}

// Moments of the nodes of one level, in FP64: a leaf from its particles, an
// internal node from its children (parallel-axis theorem).  Eight lanes take
// a node, each a share of its particles or children; the centre is the
// mass-weighted mean (the particle-count-weighted mean when the mass is zero).
__global__ void __launch_bounds__(256) k_moments(int L, const int *__restrict__ lvl,
                                                 const unsigned *__restrict__ w,
                                                 const int *__restrict__ begin,
                                                 const int *__restrict__ count,
                                                 const int *__restrict__ first_child,
                                                 const int *__restrict__ n_child,
                                                 const float4 *__restrict__ xm, NodeMoments *mom)
{
    if (w[kWordOverflow]) return;
    const int off = lvl[L], n_level = lvl[L + 1] - off;
    const int g = (int)threadIdx.x >> 3, j = (int)threadIdx.x & 7;
    for (int i0 = (int)blockIdx.x * 32; i0 < n_level; i0 += (int)gridDim.x * 32) {
        const int i = i0 + g;
        const bool valid = i < n_level;
        const int node = off + (valid ? i : 0);
        const int nch = valid ? n_child[node] : 0;
        // this lane's items: particles [k0, k1) of a leaf, or children
        const int k0 = nch ? first_child[node] : begin[node];
        const int k1 = valid ? k0 + (nch ? nch : count[node]) : k0;
        auto item = [&](int k, double *m, double *x, double *y, double *z, double *cnt) {
            if (nch) {
                const NodeMoments &q = mom[k];
                *m = q.m, *x = q.cx, *y = q.cy, *z = q.cz, *cnt = count[k];
            } else {
                const float4 p = xm[k];
                *m = p.w, *x = p.x, *y = p.y, *z = p.z, *cnt = 1.0;
            }
        };
        double M = 0, sx = 0, sy = 0, sz = 0, np = 0, px = 0, py = 0, pz = 0;
        for (int k = k0 + j; k < k1; k += 8) {
            double m, x, y, z, cnt;
            item(k, &m, &x, &y, &z, &cnt);
            M += m;
            sx += m * x, sy += m * y, sz += m * z;
            np += cnt;
            px += cnt * x, py += cnt * y, pz += cnt * z;
        }
        M = group_sum(M);
        sx = group_sum(sx), sy = group_sum(sy), sz = group_sum(sz);
        np = group_sum(np);
        px = group_sum(px), py = group_sum(py), pz = group_sum(pz);
        if (M != 0.0)
            sx /= M, sy /= M, sz /= M;
        else if (np != 0.0)
            sx = px / np, sy = py / np, sz = pz / np;
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
        for (int k = k0 + j; k < k1; k += 8) {
            double m, x, y, z, cnt;
            item(k, &m, &x, &y, &z, &cnt);
            if (nch) {
                const NodeMoments &q = mom[k];
                a0 += q.sxx, a1 += q.syy, a2 += q.szz, a3 += q.sxy, a4 += q.sxz, a5 += q.syz;
            }
            const double dx = x - sx, dy = y - sy, dz = z - sz;
            a0 += m * dx * dx, a1 += m * dy * dy, a2 += m * dz * dz;
            a3 += m * dx * dy, a4 += m * dx * dz, a5 += m * dy * dz;
        }
        a0 = group_sum(a0), a1 = group_sum(a1), a2 = group_sum(a2);
        a3 = group_sum(a3), a4 = group_sum(a4), a5 = group_sum(a5);
        // the group stores the 10 doubles side by side: lane j field j, lanes 0
        // and 1 also fields 8 and 9
        if (valid) {
            static_assert(sizeof(NodeMoments) == 10 * sizeof(double), "NodeMoments layout");
            double *dst = reinterpret_cast<double *>(mom + node);
            const double v = j == 0 ? M : j == 1 ? sx : j == 2 ? sy : j == 3 ? sz
                           : j == 4 ? a0 : j == 5 ? a1 : j == 6 ? a2 : a3;
            dst[j] = v;
            if (j < 2) dst[8 + j] = j == 0 ? a4 : a5;
        }
    }
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations (the symmetric
// Schur rotation of Golub & Van Loan, Sec. 8.5): eigenvalues in descending
// order in w, eigenvectors as the columns of V.
__device__ void jacobi3(const NodeMoments &q, double w[3], double V[3][3])
{
    double A[3][3] = {{q.sxx, q.sxy, q.sxz}, {q.sxy, q.syy, q.syz}, {q.sxz, q.syz, q.szz}};
    double Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 32; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        // converged when the off-diagonal elements are at FP64 rounding of the
        // diagonal (rotations leave residues of that size, so a tighter
        // bound only runs sweeps that change nothing)
        if (off == 0.0 || off <= 1e-30 * dia) break;
        for (int p = 0; p < 2; ++p)
            for (int r = p + 1; r < 3; ++r) {
                const double apr = A[p][r];
                if (apr == 0.0) continue;
                const double tau = (A[r][r] - A[p][p]) / (2.0 * apr);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < 3; ++k) {
                    const double u = A[k][p], v = A[k][r];
                    A[k][p] = c * u - s * v;
                    A[k][r] = s * u + c * v;
                }
                for (int k = 0; k < 3; ++k) {
                    const double u = A[p][k], v = A[r][k];
                    A[p][k] = c * u - s * v;
                    A[r][k] = s * u + c * v;
                }
                for (int k = 0; k < 3; ++k) {
                    const double u = Q[k][p], v = Q[k][r];
                    Q[k][p] = c * u - s * v;
                    Q[k][r] = s * u + c * v;
                }
            }
    }
    int o[3] = {0, 1, 2};
    if (A[o[1]][o[1]] > A[o[0]][o[0]]) { const int t = o[0]; o[0] = o[1]; o[1] = t; }
    if (A[o[2]][o[2]] > A[o[1]][o[1]]) { const int t = o[1]; o[1] = o[2]; o[2] = t; }
    if (A[o[1]][o[1]] > A[o[0]][o[0]]) { const int t = o[0]; o[0] = o[1]; o[1] = t; }
    for (int c = 0; c < 3; ++c) {
        w[c] = A[o[c]][o[c]];
        for (int r = 0; r < 3; ++r) V[r][c] = Q[r][o[c]];
    }
}

__global__ void __launch_bounds__(256) k_pseudo(const int *__restrict__ lvl,
                                                const unsigned *__restrict__ w,
                                                const NodeMoments *__restrict__ mom, int quad,
                                                float4 *__restrict__ pp, float4 *__restrict__ com)
{
    if (w[kWordOverflow]) return;
    const int n_nodes = lvl[kTreeMaxLevel + 1];
    for (int t = blockIdx.x * 256 + threadIdx.x; t < n_nodes; t += gridDim.x * 256) {
    const NodeMoments q = mom[t];
    com[t] = make_float4((float)q.cx, (float)q.cy, (float)q.cz, 0.f);
    if (!quad) {
        pp[t] = make_float4((float)q.cx, (float)q.cy, (float)q.cz, (float)q.m);
        continue;
    }
    double w[3], V[3][3];
    jacobi3(q, w, V);
    double a2 = 0.0, b2 = 0.0;
    if (q.m > 0.0) {
        a2 = 2.0 * (w[0] - w[2]) / q.m;
        b2 = 2.0 * (w[1] - w[2]) / q.m;
    }
    const double a = sqrt(fmax(a2, 0.0)), b = sqrt(fmax(b2, 0.0));
    const double h = 0.86602540378443864676;  // sin(2 pi / 3)
    const double cs[3] = {1.0, -0.5, -0.5}, sn[3] = {0.0, h, -h};
    for (int k = 0; k < 3; ++k) {
        const double u = a * cs[k], v = b * sn[k];
        pp[3 * t + k] = make_float4((float)(q.cx + u * V[0][0] + v * V[0][1]),
                                    (float)(q.cy + u * V[1][0] + v * V[1][1]),
                                    (float)(q.cz + u * V[2][0] + v * V[2][1]), (float)(q.m / 3.0));
    }
    }
}

// Walk record of a node: (begin, count, first child, n_child | level << 16).
__global__ void __launch_bounds__(256) k_pack_nodes(const int *__restrict__ lvl,
                                                    const unsigned *__restrict__ w,
                                                    const int *__restrict__ begin,
                                                    const int *__restrict__ count,
                                                    const int *__restrict__ first_child,
                                                    const int *__restrict__ n_child,
                                                    const int *__restrict__ level,
                                                    int4 *__restrict__ rec)
{
    if (w[kWordOverflow]) return;
    const int n_nodes = lvl[kTreeMaxLevel + 1];
    for (int t = blockIdx.x * 256 + threadIdx.x; t < n_nodes; t += gridDim.x * 256)
        rec[t] = make_int4(begin[t], count[t], first_child[t], n_child[t] | (level[t] << 16));
}

__global__ void __launch_bounds__(256) k_fill_int(int n, int *a, int v)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void __launch_bounds__(256) k_group_mark(const int *__restrict__ lvl,
                                                    const unsigned *__restrict__ w,
                                                    const int *__restrict__ begin,
                                                    const int *__restrict__ count,
                                                    const int *__restrict__ n_child,
                                                    const int *__restrict__ parent, int n_crit,
                                                    int *__restrict__ mark)
{
    if (w[kWordOverflow]) return;
    const int n_nodes = lvl[kTreeMaxLevel + 1];
    for (int t = blockIdx.x * 256 + threadIdx.x; t < n_nodes; t += gridDim.x * 256) {
        const bool small = count[t] <= n_crit || n_child[t] == 0;
        const int p = parent[t];
        const bool top = p < 0 || count[p] > n_crit;
        if (small && top) mark[begin[t]] = t;
    }
}

struct NonNegative {
    __host__ __device__ bool operator()(const int &v) const { return v >= 0; }
};

// One wave per group: bounding box of its particles and the i-side of its item.
__global__ void __launch_bounds__(256) k_group_info(const int *__restrict__ n_groups_dev,
                                                    const int *__restrict__ groups,
                                                    const int *__restrict__ begin,
                                                    const int *__restrict__ count,
                                                    const float *__restrict__ xs,
                                                    const float *__restrict__ ys,
                                                    const float *__restrict__ zs, float4 *glo,
                                                    float4 *ghi, pgh_item *items)
{
    const int n_groups = *n_groups_dev;
    const int lane = threadIdx.x & 63;
    for (int g = blockIdx.x * 4 + (threadIdx.x >> 6); g < n_groups; g += gridDim.x * 4) {
    const int t = groups[g];
    const int b = begin[t], c = count[t];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = b + lane; k < b + c; k += 64) {
        const float v[3] = {xs[k], ys[k], zs[k]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], v[a]);
            hi[a] = fmaxf(hi[a], v[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
        for (int o = 32; o > 0; o >>= 1) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
        }
    if (lane == 0) {
        glo[g] = make_float4(lo[0], lo[1], lo[2], 0.f);
        ghi[g] = make_float4(hi[0], hi[1], hi[2], 0.f);
        items[g].i_off = b;
        items[g].n_i = c;
    }
    }
}

struct WalkArgs {
    int n_groups;
    const int *groups;
    const float4 *glo, *ghi;
    const int4 *node;  // walk records (k_pack_nodes)
    const float4 *com, *pp;
    int npp;
    const float *rc2;  // (l_L / theta)^2 per level, device
    const float4 *xm;  // particles (x, y, z, m) in key order
    long long *glen;        // pass 1 output: list length per group
    const long long *goff;  // pass 2 input: list offset per group
    float4 *xmj;  // the lists: (x, y, z, m) per entry
    int *src;               // pass 2, optional
    unsigned *overflow;
    unsigned *max_frontier; // pass 1: the largest frontier met
};


// LDS written by some lanes of a wave and then read by others.
__device__ inline void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

constexpr int kWalkWaves = 2;  // waves per workgroup, each walking its own groups
constexpr int kMapSeg = 256;  // entries per segment of the write pass's map

// Breadth-first walk of one group per wave.  The 64 lanes test 64 frontier
// nodes at a time; wave prefix sums place each lane's contributions in the
// list and its opened children in the next frontier (double-buffered in LDS).
// Pass 1 (WRITE = false) only counts; pass 2 writes the entries at the
// offsets of the scanned counts, in the same order: the contributions of 64
// nodes form one contiguous block of the list, which the lanes write entry
// by entry (coalesced), each finding its entry's node by a binary search over
// the wave's inclusive counts.
template <bool WRITE, int FCAP>
__global__ void __launch_bounds__(64 * kWalkWaves) k_walk(WalkArgs a)
{
    __shared__ int fr[kWalkWaves][2][FCAP];
    // write pass: each lane's first entry and source code, and the lane that
    // owns each entry of a segment of kMapSeg entries
    __shared__ int s_start[kWalkWaves][64], s_src[kWalkWaves][64];
    __shared__ unsigned char s_map[kWalkWaves][kMapSeg];
    __shared__ float rc2[kTreeMaxLevel + 1];
    if (threadIdx.x <= kTreeMaxLevel) rc2[threadIdx.x] = a.rc2[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n_waves = gridDim.x * kWalkWaves;
    int maxf = 0;  // largest frontier this wave met (one atomic at the end)
    for (int g = blockIdx.x * kWalkWaves + w; g < a.n_groups; g += n_waves) {
        const int gn = a.groups[g];
        const float4 lo = a.glo[g], hi = a.ghi[g];
        const int4 grec = a.node[gn];
        const int gb = grec.x, glev = grec.w >> 16;
        const long long out = WRITE ? a.goff[g] : 0;
        long long len = 0;
        int cur = 0, ncur = 1;
        bool over = false;
        if (lane == 0) fr[w][0][0] = 0;
        wave_sync_lds();
        while (ncur > 0) {
            int nnext = 0;
            for (int c0 = 0; c0 < ncur; c0 += 64) {
                const int idx = c0 + lane;
                int emit = 0, push = 0, code = 0, fc = 0;
                if (idx < ncur) {
                    const int t = fr[w][cur][idx];
                    const int4 r = a.node[t];
                    const int b = r.x, c = r.y, nch = r.w & 0xffff, L = r.w >> 16;
                    fc = r.z;
                    const bool anc = L <= glev && b <= gb && gb < b + c;
                    bool acc = false;
                    if (!anc) {
                        const float4 cm = a.com[t];
                        const float ex = fmaxf(fmaxf(lo.x - cm.x, cm.x - hi.x), 0.f);
                        const float ey = fmaxf(fmaxf(lo.y - cm.y, cm.y - hi.y), 0.f);
                        const float ez = fmaxf(fmaxf(lo.z - cm.z, cm.z - hi.z), 0.f);
                        acc = rc2[L] < ex * ex + ey * ey + ez * ez;
                    }
                    if (acc) {
                        emit = a.npp;
                        code = t * a.npp;  // first pseudo-particle
                    } else if (nch == 0) {
                        emit = c;
                        code = -1 - b;     // first particle
                    } else {
                        push = nch;
                    }
                }
                const int e_inc = wave_incl_scan(emit);
                const int p_inc = wave_incl_scan(push);
                const int e_tot = __builtin_amdgcn_readlane(e_inc, 63);
                const int p_tot = __builtin_amdgcn_readlane(p_inc, 63);
                if (nnext + p_tot > FCAP) {
                    over = true;
                    break;
                }
                for (int k = 0; k < push; ++k) fr[w][cur ^ 1][nnext + p_inc - push + k] = fc + k;
                if (WRITE && e_tot > 0) {
                    const int r0 = e_inc - emit;  // this lane's first entry
                    s_start[w][lane] = r0;
                    s_src[w][lane] = code;
                    const long long base = out + len;
                    // segment by segment: every lane marks its entries in the
                    // map, then the entries are written 64 at a time, each lane
                    // finding its entry's source through the map
                    for (int seg = 0; seg < e_tot; seg += kMapSeg) {
                        const int m0 = max(r0, seg), m1 = min(e_inc, seg + kMapSeg);
                        for (int e = m0; e < m1; ++e) s_map[w][e - seg] = (unsigned char)lane;
                        wave_sync_lds();
                        const int seg_end = min(e_tot, seg + kMapSeg);
                        for (int e = seg + lane; e < seg_end; e += 64) {
                            const int l = s_map[w][e - seg];
                            const int k = e - s_start[w][l];
                            const int cd = s_src[w][l];
                            a.xmj[base + e] = cd >= 0 ? a.pp[cd + k] : a.xm[-1 - cd + k];
                            if (a.src) a.src[base + e] = cd >= 0 ? -(1 + cd + k) : -1 - cd + k;
                        }
                        wave_sync_lds();
                    }
                }
                len += e_tot;
                nnext += p_tot;
            }
            if (over) break;
            maxf = max(maxf, nnext);
            wave_sync_lds();
            cur ^= 1;
            ncur = nnext;
        }
        if (over) {
            if (lane == 0) atomicOr(a.overflow, 1u);
            len = 0;
        }
        if (!WRITE && lane == 0) a.glen[g] = len;
        wave_sync_lds();
    }
    if (!WRITE && lane == 0 && maxf > 0) atomicMax(a.max_frontier, (unsigned)maxf);
}

__global__ void k_tail_zero(long long *p) { *p = 0; }

__global__ void __launch_bounds__(256) k_items_j(int n_groups, const long long *__restrict__ goff,
                                                 const long long *__restrict__ glen,
                                                 pgh_item *items)
{
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= n_groups) return;
    items[g].j_off = (int)goff[g];
    items[g].n_j = (int)glen[g];
}

int blocks_of(long long n, int per) { return (int)std::max(1LL, (n + per - 1) / per); }

template <class T>
bool grow(T **p, long long *cap_now, long long cap_new)
{
    T *q = nullptr;
    if (hipMalloc((void **)&q, sizeof(T) * (size_t)std::max(1LL, cap_new)) != hipSuccess)
        return false;
    (void)hipFree(*p);
    *p = q;
    *cap_now = cap_new;
    return true;
}

#define TREE_HIP(call)                                                    \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) {                                           \
            err = std::string(#call) + ": " + hipGetErrorString(e_);      \
            return PGH_EHIP;                                              \
        }                                                                 \
    } while (0)

#define TREE_ALLOC(ok)                                                    \
    do {                                                                  \
        if (!(ok)) {                                                      \
            err = "tree: device allocation failed";                       \
            return PGH_ENOMEM;                                            \
        }                                                                 \
    } while (0)

size_t temp_bytes_for(int n, int ngroups)
{
    size_t a = 0, b = 0, c = 0, d = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, (unsigned long long *)nullptr,
                                             (unsigned long long *)nullptr, (int *)nullptr,
                                             (int *)nullptr, n, 0, 63);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, b, (int *)nullptr, (int *)nullptr, n + 1);
    (void)hipcub::DeviceSelect::If(nullptr, c, (int *)nullptr, (int *)nullptr, (int *)nullptr, n,
                                   NonNegative());
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, d, (long long *)nullptr,
                                           (long long *)nullptr, ngroups + 1);
    return std::max(std::max(a, b), std::max(c, d));
}

int ensure_tmp(TreeState &t, int n, std::string &err)
{
    const size_t want = temp_bytes_for(n, n);
    if (want <= t.tmp_bytes) return PGH_OK;
    (void)hipFree(t.tmp);
    t.tmp = nullptr;
    t.tmp_bytes = 0;
    TREE_ALLOC(hipMalloc(&t.tmp, want) == hipSuccess);
    t.tmp_bytes = want;
    return PGH_OK;
}

}  // namespace

void tree_release(TreeState &t)
{
    void *ps[] = {t.key, t.key_in, t.perm, t.iota, t.xs, t.ys, t.zs, t.ms, t.mark, t.xin, t.inv, t.res,
                  t.begin, t.count, t.level, t.first_child, t.n_child, t.parent, t.nc, t.mom, t.com, t.pp, t.groups, t.glo, t.ghi, t.glen, t.goff,
                  t.items, t.xmj, t.src, t.tmp, t.word, t.count_out, t.rc2, t.lvl,
                  t.xm, t.nrec};
    for (void *p : ps) (void)hipFree(p);
    t = TreeState();
}

int tree_build(TreeState &t, int n, const float *x, const float *y, const float *z,
               const float *m, int n_leaf, int n_crit, int quad, int num_cu, hipStream_t s,
               std::string &err)
{
    t.built = t.walked = 0;
    t.n = n;
    t.n_leaf = n_leaf;
    t.n_crit = n_crit;
    t.quad = quad ? 1 : 0;
    t.n_nodes = t.n_leaves = t.depth = t.n_groups = t.max_level_nodes = 0;
    t.n_entries = t.interactions = 0;
    std::fill(t.level_off, t.level_off + kTreeMaxLevel + 2, 0);
    std::fill(t.frame, t.frame + 5, 0.f);
    t.host_items.clear();
    if (!t.word) {
        TREE_ALLOC(hipMalloc((void **)&t.word, 16 * sizeof(unsigned)) == hipSuccess);
        TREE_ALLOC(hipMalloc((void **)&t.count_out, sizeof(int)) == hipSuccess);
        TREE_ALLOC(hipMalloc((void **)&t.rc2, (kTreeMaxLevel + 1) * sizeof(float)) == hipSuccess);
        TREE_ALLOC(hipMalloc((void **)&t.lvl, kLvl * sizeof(int)) == hipSuccess);
    }
    if (n == 0) {
        t.built = 1;
        return PGH_OK;
    }
    if (n > t.n_cap) {
        const long long cap = std::max(n, 1024);
        long long dummy = 0;
        bool ok = grow(&t.key, &dummy, cap) && grow(&t.key_in, &dummy, cap) &&
                  grow(&t.perm, &dummy, cap) && grow(&t.iota, &dummy, cap) &&
                  grow(&t.xs, &dummy, cap) && grow(&t.ys, &dummy, cap) &&
                  grow(&t.zs, &dummy, cap) && grow(&t.ms, &dummy, cap) &&
                  grow(&t.mark, &dummy, cap) && grow(&t.xm, &dummy, cap) &&
                  grow(&t.xin, &dummy, cap) && grow(&t.inv, &dummy, cap) &&
                  grow(&t.res, &dummy, cap);
        if (!ok) {
            t.n_cap = 0;
            err = "tree: device allocation failed";
            return PGH_ENOMEM;
        }
        t.n_cap = (int)cap;
        int st = ensure_tmp(t, (int)cap, err);
        if (st) return st;
    }
    // 1. frame
    hipLaunchKernelGGL(k_init_words, dim3(1), dim3(64), 0, s, t.word);
    hipLaunchKernelGGL(k_frame, dim3(std::min(blocks_of(n, 256), num_cu)), dim3(256), 0, s, n,
                       x, y, z, t.word);
    TREE_HIP(hipGetLastError());
    unsigned wv[6];
    TREE_HIP(hipMemcpyAsync(wv, t.word, sizeof wv, hipMemcpyDeviceToHost, s));
    TREE_HIP(hipStreamSynchronize(s));
    float lo[3], hi[3], ext = 0.f;
    for (int a = 0; a < 3; ++a) {
        lo[a] = float_of_ord(wv[a]);
        hi[a] = float_of_ord(wv[3 + a]);
        const float e = hi[a] - lo[a];
        if (e > ext) ext = e;
    }
    if (!std::isfinite(ext)) {
        err = "tree: positions must be finite";
        return PGH_ERANGE;
    }
    const float scale = ext > 0.f ? 2097152.0f / ext : 0.f;
    t.frame[0] = lo[0], t.frame[1] = lo[1], t.frame[2] = lo[2], t.frame[3] = ext;
    t.frame[4] = scale;
    // 2. keys, sort, gather
    hipLaunchKernelGGL(k_keys, dim3(blocks_of(n, 256)), dim3(256), 0, s, n, x, y, z, m, lo[0],
                       lo[1], lo[2], scale, t.key_in, t.iota, t.xin);
    TREE_HIP(hipGetLastError());
    size_t tb = t.tmp_bytes;
    TREE_HIP(hipcub::DeviceRadixSort::SortPairs(t.tmp, tb, t.key_in, t.key, t.iota, t.perm, n, 0,
                                                63, s));
    hipLaunchKernelGGL(k_gather, dim3(blocks_of(n, 256)), dim3(256), 0, s, n, t.perm, t.xin,
                       t.xs, t.ys, t.zs, t.ms, t.xm, t.inv);
    TREE_HIP(hipGetLastError());
    // 3-5. octree, moments, pseudo-particles and groups, launched with no
    // wait: the level sizes stay in a device table (lvl).  The node arrays
    // start at 2n (a tree needs about n / 2 with leaves of 8); a build that
    // outgrows them sets the overflow word, returns from every later kernel,
    // and runs again with twice the room.
    if (t.group_cap < n) {
        const long long cap = std::max(n, 1024);
        long long dummy = 0;
        TREE_ALLOC(grow(&t.groups, &dummy, cap) && grow(&t.glo, &dummy, cap) &&
                   grow(&t.ghi, &dummy, cap) && grow(&t.glen, &dummy, cap + 1) &&
                   grow(&t.goff, &dummy, cap + 1) && grow(&t.items, &dummy, cap));
        t.group_cap = (int)cap;
    }
    // per level: children per node, chunk sums, child bounds (7 per node)
    const long long nc_need = 8LL * (n + 1) + kSplitBlocks + 1;
    if (t.nc_cap < nc_need) {
        long long dummy = 0;
        const long long cap = 8LL * (std::max(n, 1024) + 1) + kSplitBlocks + 1;
        TREE_ALLOC(grow(&t.nc, &dummy, cap));
        t.nc_cap = cap;
    }
    long long want = std::max<long long>(2LL * n + 64, 4096);
    for (;;) {
        if (want > INT_MAX) {
            err = "tree: too many nodes";
            return PGH_ERANGE;
        }
        if (t.node_cap < want) {
            const long long cap = want;
            long long dummy = 0;
            TREE_ALLOC(grow(&t.begin, &dummy, cap) && grow(&t.count, &dummy, cap) &&
                       grow(&t.level, &dummy, cap) && grow(&t.first_child, &dummy, cap) &&
                       grow(&t.n_child, &dummy, cap) && grow(&t.parent, &dummy, cap) &&
                       grow(&t.mom, &dummy, cap) && grow(&t.com, &dummy, cap) &&
                       grow(&t.pp, &dummy, 3 * cap) && grow(&t.nrec, &dummy, cap));
            t.node_cap = (int)cap;
        }
        const int cap = t.node_cap;
        hipLaunchKernelGGL(k_init_words, dim3(1), dim3(64), 0, s, t.word);
        hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, s, n, t.begin, t.count, t.level, t.parent,
                           t.lvl);
        TREE_HIP(hipGetLastError());
        // level L has at most min(n, 8^L) nodes
        auto level_bound = [&](int L) {
            long long b = 1;
            for (int k = 0; k < L && b < n; ++k) b *= 8;
            return (int)std::min<long long>(b, n);
        };
        int *cnt = t.nc, *bsum = t.nc + (n + 1), *bnd = bsum + kSplitBlocks + 1;
        for (int L = 0; L <= kTreeMaxLevel; ++L) {
            hipLaunchKernelGGL(k_split_count, dim3(kSplitBlocks), dim3(256), 0, s, L, n_leaf,
                               t.lvl, t.begin, t.count, t.key, cnt, bnd, bsum, t.word);
            hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(256), 0, s, L, cap, t.lvl, bsum,
                               t.word);
            hipLaunchKernelGGL(k_split_write, dim3(kSplitBlocks), dim3(256), 0, s, L, t.lvl, cnt,
                               bnd, bsum, t.begin, t.count, t.level, t.first_child, t.n_child,
                               t.parent, t.word);
            TREE_HIP(hipGetLastError());
        }
        for (int L = kTreeMaxLevel; L >= 0; --L) {
            const int grid = std::min(blocks_of(level_bound(L), 32), 16 * num_cu);
            hipLaunchKernelGGL(k_moments, dim3(grid), dim3(256), 0, s, L, t.lvl, t.word, t.begin,
                               t.count, t.first_child, t.n_child, t.xm, t.mom);
        }
        const int gnodes = std::min(blocks_of(cap, 256), 16 * num_cu);
        hipLaunchKernelGGL(k_pseudo, dim3(gnodes), dim3(256), 0, s, t.lvl, t.word, t.mom, t.quad,
                           t.pp, t.com);
        hipLaunchKernelGGL(k_pack_nodes, dim3(gnodes), dim3(256), 0, s, t.lvl, t.word, t.begin,
                           t.count, t.first_child, t.n_child, t.level, t.nrec);
        hipLaunchKernelGGL(k_fill_int, dim3(blocks_of(n, 256)), dim3(256), 0, s, n, t.mark, -1);
        hipLaunchKernelGGL(k_group_mark, dim3(gnodes), dim3(256), 0, s, t.lvl, t.word, t.begin,
                           t.count, t.n_child, t.parent, n_crit, t.mark);
        TREE_HIP(hipGetLastError());
        tb = t.tmp_bytes;
        TREE_HIP(hipcub::DeviceSelect::If(t.tmp, tb, t.mark, t.groups, t.count_out, n,
                                          NonNegative(), s));
        hipLaunchKernelGGL(k_group_info, dim3(std::min(blocks_of(n, 4), 16 * num_cu)), dim3(256), 0,
                           s, t.count_out, t.groups, t.begin, t.count, t.xs, t.ys, t.zs, t.glo,
                           t.ghi, t.items);
        TREE_HIP(hipGetLastError());
        // the one wait of the build: sizes and flags
        int lv[kLvl];
        unsigned wv2[16];
        TREE_HIP(hipMemcpyAsync(lv, t.lvl, sizeof lv, hipMemcpyDeviceToHost, s));
        TREE_HIP(hipMemcpyAsync(wv2, t.word, sizeof wv2, hipMemcpyDeviceToHost, s));
        TREE_HIP(hipMemcpyAsync(&t.n_groups, t.count_out, sizeof(int), hipMemcpyDeviceToHost, s));
        TREE_HIP(hipStreamSynchronize(s));
        if (wv2[kWordOverflow]) {
            want = 2LL * cap;
            continue;
        }
        t.n_nodes = lv[kTreeMaxLevel + 1];
        t.depth = 0;
        for (int L = 0; L <= kTreeMaxLevel; ++L) {
            t.level_off[L] = lv[L];
            if (lv[L + 1] > lv[L]) t.depth = L;
        }
        t.level_off[kTreeMaxLevel + 1] = lv[kTreeMaxLevel + 1];
        t.n_leaves = (int)wv2[kWordLeaves];
        t.max_level_nodes = std::max(1, (int)wv2[kWordMaxLevel]);
        break;
    }
    t.built = 1;
    return PGH_OK;
}

int tree_walk(TreeState &t, float theta, int record_src, int num_cu, hipStream_t s,
              std::string &err)
{
    t.walked = 0;
    t.max_frontier = 0;
    t.theta = theta;
    t.record_src = record_src ? 1 : 0;
    t.n_entries = t.interactions = 0;
    t.host_items.clear();
    if (t.n_groups == 0) {
        t.walked = 1;
        return PGH_OK;
    }
    // (l_L / theta)^2 per level, rounded once from double
    float rc2[kTreeMaxLevel + 1];
    for (int L = 0; L <= kTreeMaxLevel; ++L) {
        const double l = std::ldexp((double)t.frame[3], -L);
        rc2[L] = theta > 0.f ? (float)((l / theta) * (l / theta)) : INFINITY;
    }
    TREE_HIP(hipMemcpyAsync(t.rc2, rc2, sizeof rc2, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_init_words, dim3(1), dim3(64), 0, s, t.word);
    WalkArgs a{};
    a.n_groups = t.n_groups;
    a.groups = t.groups;
    a.glo = t.glo;
    a.ghi = t.ghi;
    a.node = t.nrec;
    a.com = t.com;
    a.pp = t.pp;
    a.npp = t.quad ? 3 : 1;
    a.rc2 = t.rc2;
    a.xm = t.xm;
    a.glen = t.glen;
    a.goff = t.goff;
    a.overflow = t.word + 7;
    a.max_frontier = t.word + 8;
    // Pass 1 counts the lists; their scan, the items and the status words
    // come back to the host in one wait.  It runs with the small frontier
    // (LDS for 2 walking waves per SIMD); if a group's frontier outgrew it,
    // it runs again with the large one (1 per SIMD).
    const int grid_small = std::min(blocks_of(t.n_groups, kWalkWaves), 4 * num_cu);
    const int grid_large = std::min(blocks_of(t.n_groups, kWalkWaves), 2 * num_cu);
    bool large = false;
    unsigned over = 0, maxf = 0;
    long long total = 0;
    t.host_items.resize(t.n_groups);
    for (;;) {
        if (large)
            hipLaunchKernelGGL((k_walk<false, kWalkFrontier>), dim3(grid_large),
                               dim3(64 * kWalkWaves), 0, s, a);
        else
            hipLaunchKernelGGL((k_walk<false, kWalkFrontier / 2>), dim3(grid_small),
                               dim3(64 * kWalkWaves), 0, s, a);
        TREE_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_tail_zero, dim3(1), dim3(1), 0, s, t.glen + t.n_groups);
        TREE_HIP(hipGetLastError());
        size_t tb = t.tmp_bytes;
        TREE_HIP(hipcub::DeviceScan::ExclusiveSum(t.tmp, tb, t.glen, t.goff, t.n_groups + 1, s));
        hipLaunchKernelGGL(k_items_j, dim3(blocks_of(t.n_groups, 256)), dim3(256), 0, s,
                           t.n_groups, t.goff, t.glen, t.items);
        TREE_HIP(hipGetLastError());
        TREE_HIP(hipMemcpyAsync(&over, t.word + 7, sizeof over, hipMemcpyDeviceToHost, s));
        TREE_HIP(hipMemcpyAsync(&maxf, t.word + 8, sizeof maxf, hipMemcpyDeviceToHost, s));
        TREE_HIP(hipMemcpyAsync(&total, t.goff + t.n_groups, sizeof total, hipMemcpyDeviceToHost, s));
        TREE_HIP(hipMemcpyAsync(t.host_items.data(), t.items, sizeof(pgh_item) * t.n_groups,
                                hipMemcpyDeviceToHost, s));
        TREE_HIP(hipStreamSynchronize(s));
        if (!over || large) break;
        large = true;
        hipLaunchKernelGGL(k_init_words, dim3(1), dim3(64), 0, s, t.word);
    }
    if (over) {
        err = "tree walk: a frontier exceeded " + std::to_string(kWalkFrontier) +
              " nodes (theta too small for this tree)";
        return PGH_ERANGE;
    }
    t.max_frontier = (int)maxf;
    if (total > INT_MAX) {
        err = "tree walk: the lists exceed 2^31 - 1 entries";
        return PGH_ERANGE;
    }
    if (total > t.entry_cap) {
        const long long cap = total + total / 4 + 1024;
        long long c1 = 0;
        TREE_ALLOC(grow(&t.xmj, &c1, cap));
        t.entry_cap = cap;
    }
    if (record_src && total > t.src_cap) {
        const long long cap = total + total / 4 + 1024;
        TREE_ALLOC(grow(&t.src, &t.src_cap, cap));
    }
    // The writing pass runs while the caller plans the batched launch from
    // the items (the plan's upload is ordered after it on the stream).
    a.xmj = t.xmj;
    a.src = record_src ? t.src : nullptr;
    if (large)
        hipLaunchKernelGGL((k_walk<true, kWalkFrontier>), dim3(grid_large),
                           dim3(64 * kWalkWaves), 0, s, a);
    else
        hipLaunchKernelGGL((k_walk<true, kWalkFrontier / 2>), dim3(grid_small),
                           dim3(64 * kWalkWaves), 0, s, a);
    TREE_HIP(hipGetLastError());
    long long inter = 0;
    for (const pgh_item &it : t.host_items) inter += (long long)it.n_i * it.n_j;
    t.n_entries = total;
    t.interactions = inter;
    t.walked = 1;
    return PGH_OK;
}

// The tree force in the input order: particle i's packed result (ax, ay, az,
// phi) sits at its rank inv[i]; a coalesced write of each output array from
// one 16-byte gather.
__global__ void __launch_bounds__(256) k_tree_out(int n, const int *__restrict__ inv,
                                                  const float4 *__restrict__ res, float *ax,
                                                  float *ay, float *az, float *phi)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 v = res[inv[i]];
    ax[i] = v.x;
    ay[i] = v.y;
    az[i] = v.z;
    if (phi) phi[i] = v.w;
}

hipError_t launch_tree_outputs(const TreeState &t, float *ax, float *ay, float *az, float *phi,
                               hipStream_t s)
{
    if (t.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tree_out, dim3(blocks_of(t.n, 256)), dim3(256), 0, s, t.n, t.inv, t.res,
                       ax, ay, az, phi);
    return hipGetLastError();
}

// One component (0..3: x, y, z, m) of the packed list entries.
__global__ void __launch_bounds__(256) k_list_component(long long n, const float4 *__restrict__ xmj,
                                                        int comp, float *__restrict__ out)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float4 v = xmj[e];
    out[e] = comp == 0 ? v.x : comp == 1 ? v.y : comp == 2 ? v.z : v.w;
}

hipError_t launch_list_component(const TreeState &t, int comp, float *out, hipStream_t s)
{
    if (t.n_entries <= 0) return hipSuccess;
    const long long blocks = (t.n_entries + 255) / 256;
    hipLaunchKernelGGL(k_list_component, dim3((unsigned)blocks), dim3(256), 0, s, t.n_entries,
                       t.xmj, comp, out);
    return hipGetLastError();
}

}  // namespace pgh
