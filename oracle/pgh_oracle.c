/*
 * pgh_oracle.c -- FP64 reference implementation of the direct-summation
 * force path of Phantom-GRAPE (Tanikawa, Yoshikawa, Nitadori & Okamoto,
 * arXiv:1203.4037).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library package may include,
 * link, load or call this file; only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark do.  It shares no code, header, table or
 * constant with the GPU path: every formula here is written out again from the
 * paper, in double precision, with plain loops.
 *
 * Conventions (the readings of the paper this file follows):
 *   - G = 1: the paper's API carries no gravitational constant (Sec. 3.6), so
 *     masses carry the units.
 *   - The potential is phi_i = -sum_j m_j / sqrt(r_ij^2 + eps_i^2): the Newton
 *     kernel of Sec. 3.3 subtracts m_j/r from the potential register at every
 *     step (step 7 with the listing's subtract semantics).
 *   - Softening is per i-particle (the i-particle structure of Sec. 3.1 holds
 *     eps^2 for each i).
 *   - A pair at zero softened distance (eps = 0 and coincident particles)
 *     contributes nothing: the paper does not discuss it and 1/0 is undefined.
 *   - Every array argument is double.  Callers pass the same FP32 values the
 *     GPU receives, widened exactly, so the quantisation of the inputs is
 *     shared and is not counted as error; finite-difference checks perturb
 *     them in double.
 *   - The table bin of a pair is the one integer decision of the table
 *     force: it is taken from the pair's single-precision s, whose bits the
 *     method reads (pgo_pair_bin); everything else is in double.
 *
 * Parallelism: OpenMP over i-particles (or over independent items), which is
 * how the paper spreads groups of i-particles over cores (Sec. 3.5).
 * Compile with -O2 -fopenmp and without -ffast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PGO_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Newton's force and potential: Eq. (newton_force), Sec. 3.                 */
/* ------------------------------------------------------------------------ */

/*
 * a_i   =  sum_j m_j (r_j - r_i) / (|r_j - r_i|^2 + eps_i^2)^{3/2}
 * phi_i = -sum_j m_j            / (|r_j - r_i|^2 + eps_i^2)^{1/2}
 *
 * self_j: NULL, or for every i the index of the j-particle that is i itself
 * (-1 for none).  That pair is skipped ("physical" potential, the way the
 * paper's double-precision reference avoids the self-interaction, Sec. 4.1).
 * With self_j == NULL every pair is summed, including a coincident j = i,
 * which leaves the self term -m_i/eps_i in phi_i ("raw" potential, the way the
 * SIMD kernel accumulates it, Sec. 4.1).
 */
PGO_EXPORT void pgo_newton(long ni, const double *xi, const double *yi, const double *zi,
                           const double *eps2i, long nj, const double *xj, const double *yj,
                           const double *zj, const double *mj, const long *self_j,
                           double *ax, double *ay, double *az, double *phi)
{
    long i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < ni; i++) {
        double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
        const double px = xi[i], py = yi[i], pz = zi[i], e2 = eps2i[i];
        const long skip = self_j ? self_j[i] : -1;
        for (long j = 0; j < nj; j++) {
            if (j == skip) continue;
            const double dx = (double)xj[j] - px;
            const double dy = (double)yj[j] - py;
            const double dz = (double)zj[j] - pz;
            const double q = dx * dx + dy * dy + dz * dz + e2;
            if (q == 0.0) continue;
            const double rinv = 1.0 / sqrt(q);
            const double rinv3 = rinv * rinv * rinv;
            const double m = mj[j];
            sx += m * dx * rinv3;
            sy += m * dy * rinv3;
            sz += m * dz * rinv3;
            sp -= m * rinv;
        }
        ax[i] = sx;
        ay[i] = sy;
        az[i] = sz;
        if (phi) phi[i] = sp;
    }
}

/*
 * Interaction lists: item t couples the i-particles [i_off, i_off+n_i) with the
 * j-particles [j_off, j_off+n_j) of the given arrays (a tree or cell-list
 * group sharing one list, Sec. 5.1).  items is int32 [n_items][4] =
 * {i_off, n_i, j_off, n_j}.  i-ranges are disjoint; rows not covered by an
 * item are left untouched.
 */
PGO_EXPORT void pgo_newton_items(long n_items, const int32_t *items, const double *xi,
                                 const double *yi, const double *zi, const double *eps2i,
                                 const double *xj, const double *yj, const double *zj,
                                 const double *mj, double *ax, double *ay, double *az,
                                 double *phi)
{
    long t;
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < n_items; t++) {
        const long i0 = items[4 * t + 0], n_i = items[4 * t + 1];
        const long j0 = items[4 * t + 2], n_j = items[4 * t + 3];
        pgo_newton(n_i, xi + i0, yi + i0, zi + i0, eps2i + i0, n_j, xj + j0, yj + j0, zj + j0,
                   mj + j0, NULL, ax + i0, ay + i0, az + i0, phi ? phi + i0 : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Force shapes f(r) with a finite cutoff: Eq. (arbitrary_force), Sec. 4.2.  */
/* ------------------------------------------------------------------------ */

/*
 * S2 force profile R(r, a) of Hockney & Eastwood, Eq. (s2), with xi = 2r/a.
 * Both polynomial branches are divided by 35 a^2: continuity at xi = 1
 * (both give 97) and at xi = 2 (the second gives 35, i.e. 1/a^2 = 1/r^2)
 * fixes the denominator that the printed second branch garbles.
 */
PGO_EXPORT double pgo_s2_R(double r, double a)
{
    const double xi = 2.0 * r / a;
    if (xi < 1.0) {
        const double x2 = xi * xi, x3 = x2 * xi, x4 = x3 * xi, x5 = x4 * xi, x6 = x5 * xi;
        return (224.0 * xi - 224.0 * x3 + 70.0 * x4 + 48.0 * x5 - 21.0 * x6) / (35.0 * a * a);
    }
    if (xi < 2.0) {
        const double x2 = xi * xi, x3 = x2 * xi, x4 = x3 * xi, x5 = x4 * xi, x6 = x5 * xi;
        return (12.0 / x2 - 224.0 + 896.0 * xi - 840.0 * x2 + 224.0 * x3 + 70.0 * x4
                - 48.0 * x5 + 7.0 * x6) / (35.0 * a * a);
    }
    return 1.0 / (r * r);
}

/* Particle-particle part of the S2 split, Eq. (s2pp): f = R(r,eps) - R(r,rcut). */
PGO_EXPORT double pgo_s2pp_f(double r, double eps, double rcut)
{
    if (r >= rcut) return 0.0;
    return pgo_s2_R(r, eps) - pgo_s2_R(r, rcut);
}

/*
 * Shapes of h(r) = f(r)/r, the quantity the table holds (G0_k = f(r_k)/r_k,
 * Sec. 3.4.1).  params = {eps, rcut}.
 *   PGO_SHAPE_S2PP    f = R(r,eps) - R(r,rcut); h(0) is its analytic limit,
 *                     R(r,a)/r -> 448/(35 a^3) as r -> 0 (first branch).
 *   PGO_SHAPE_PLUMMER_TAPER  h = (r^2+eps^2)^{-3/2} T(r/rcut), T = 1 on
 *                     [0, 1/2], a quintic smoothstep down to 0 at 1: inside
 *                     rcut/2 this is exactly the softened Newtonian f/r.
 *   PGO_SHAPE_SOFT_CUT  the pair potential p(r) = -u^3 / sqrt(q), u = 1 -
 *                     r^2/rcut^2, q = r^2 + eps^2 (zero with its derivative
 *                     at rcut), and h = p'(r)/r = 6 u^2/(rcut^2 sqrt q) +
 *                     u^3 q^{-3/2}, the f/r of the force a_i = sum_j m_j h d
 *                     that goes with phi_i = sum_j m_j p (for p = -1/r,
 *                     h = 1/r^3: Newton).
 */
enum { PGO_SHAPE_S2PP = 0, PGO_SHAPE_PLUMMER_TAPER = 1, PGO_SHAPE_SOFT_CUT = 2 };

static double taper(double x)
{
    if (x <= 0.5) return 1.0;
    if (x >= 1.0) return 0.0;
    const double t = (x - 0.5) / 0.5;
    return 1.0 - t * t * t * (10.0 - 15.0 * t + 6.0 * t * t);
}

PGO_EXPORT double pgo_shape_h(int shape, double r, const double *params)
{
    const double eps = params[0], rcut = params[1];
    if (r >= rcut) return 0.0;
    if (shape == PGO_SHAPE_S2PP) {
        if (r == 0.0) return 448.0 / (35.0 * eps * eps * eps) - 448.0 / (35.0 * rcut * rcut * rcut);
        return pgo_s2pp_f(r, eps, rcut) / r;
    }
    if (shape == PGO_SHAPE_SOFT_CUT) {
        const double u = 1.0 - r * r / (rcut * rcut), q = r * r + eps * eps;
        return 6.0 * u * u / (rcut * rcut * sqrt(q)) + u * u * u / (q * sqrt(q));
    }
    /* PGO_SHAPE_PLUMMER_TAPER */
    const double q = r * r + eps * eps;
    return taper(r / rcut) / (q * sqrt(q));
}

/* Pair potential p(r) of the shapes that define one (PGO_SHAPE_SOFT_CUT);
 * 0 at and beyond rcut. */
PGO_EXPORT double pgo_shape_p(int shape, double r, const double *params)
{
    const double eps = params[0], rcut = params[1];
    if (r >= rcut || shape != PGO_SHAPE_SOFT_CUT) return 0.0;
    const double u = 1.0 - r * r / (rcut * rcut);
    return -u * u * u / sqrt(r * r + eps * eps);
}

/* ------------------------------------------------------------------------ */
/* Bit-binned look-up table: Sec. 3.4.1 (Eqs. for s, s_{bE,bF}, G0, G1).    */
/* ------------------------------------------------------------------------ */

/* s_max = 2^{2^E} (2 - 2^{-F}); s_min = 2. */
PGO_EXPORT double pgo_smax(int E, int F)
{
    return ldexp(1.0, 1 << E) * (2.0 - ldexp(1.0, -F));
}

/* Node k = 2^F bE + bF sits at s_k = 2^{bE+1} (1 + bF / 2^F). */
PGO_EXPORT double pgo_node_s(int E, int F, long k)
{
    (void)E;
    const long bE = k / (1L << F), bF = k % (1L << F);
    return ldexp(1.0, (int)bE + 1) * (1.0 + (double)bF / (double)(1L << F));
}

/* Radius of node k: s = r^2 (s_max - 2)/rcut^2 + 2 solved for r. */
PGO_EXPORT double pgo_node_r(int E, int F, double rcut, long k)
{
    const double s = pgo_node_s(E, F, k);
    return rcut * sqrt((s - 2.0) / (pgo_smax(E, F) - 2.0));
}

/*
 * Table index of s in [2, s_max], written from the arithmetic meaning of the
 * extracted bits rather than from the bits: bE = floor(log2 s) - 1 and
 * bF = floor((s / 2^{bE+1} - 1) 2^F), k = 2^F bE + bF.  frexp gives
 * s = mant 2^e with mant in [1/2, 1), so floor(log2 s) = e - 1 exactly.
 * Writes s_k (the node at or below s) to *s_node when non-NULL.
 */
PGO_EXPORT long pgo_lut_index(double s, int E, int F, double *s_node)
{
    int e;
    (void)frexp(s, &e);
    const long bE = (long)(e - 1) - 1;
    const double scaled = ldexp(s, -(int)(bE + 1)); /* in [1, 2) */
    const long bF = (long)floor((scaled - 1.0) * ldexp(1.0, F));
    const long k = bE * (1L << F) + bF;
    if (s_node) *s_node = pgo_node_s(E, F, k);
    return k;
}

/*
 * The single-precision scale of the pair's s: the smallest FP32 number c_f
 * with fl(fl(rcut^2) c_f + 2) >= s_max, so that a pair at exactly rcut lands
 * on the last node, where the node equation of Sec. 3.4.1 puts rcut.  Found
 * from the rounded quotient by stepping one float at a time either way.
 */
PGO_EXPORT float pgo_scale_f32(int E, int F, double rcut)
{
    const double smax = pgo_smax(E, F);
    const float smaxf = (float)smax;
    const float rf = (float)rcut;
    const float r2 = rf * rf;
    float c = (float)((smax - 2.0) / ((double)rf * (double)rf));
    while (fmaf(r2, c, 2.0f) < smaxf) c = nextafterf(c, INFINITY);
    while (fmaf(r2, nextafterf(c, 0.0f), 2.0f) >= smaxf) c = nextafterf(c, 0.0f);
    return c;
}

/*
 * The bin of a pair as the method takes it.  The force procedure of
 * Sec. 3.4.2 reads the table index off the bits of the single-precision s,
 * so for a pair whose s lies within a rounding of a node the bin is a
 * single-precision decision.  It is made here from s formed in FP32 the way
 * the pair step forms it (d = fl(x_j - x_i) per component, |d|^2 by fused
 * multiply-adds, s = fl(|d|^2 c_f + 2) with c_f from pgo_scale_f32, clamped
 * to s_max), while the callers interpolate with s in double.  The force does
 * not depend on the choice (the interpolant is continuous at the nodes); its
 * derivatives, which take the bin's slope G1, and the table gradient, which
 * lands in the bin, do.  Returns k; its node s_k goes to *sk, and whether the
 * FP32 s sits on the clamp to *clamped.
 */
PGO_EXPORT long pgo_pair_bin(double xi, double yi, double zi, double xj, double yj, double zj,
                             float c_f, int E, int F, double *sk, int *clamped)
{
    const float smaxf = (float)pgo_smax(E, F);
    const float dx = (float)xj - (float)xi;
    const float dy = (float)yj - (float)yi;
    const float dz = (float)zj - (float)zi;
    float r2 = dx * dx;
    r2 = fmaf(dy, dy, r2);
    r2 = fmaf(dz, dz, r2);
    float s = fmaf(r2, c_f, 2.0f);
    *clamped = s >= smaxf;
    if (*clamped) s = smaxf;
    return pgo_lut_index((double)s, E, F, sk);
}

/*
 * Table of (G0_k, G1_k), interleaved as float[2K] (the paper's
 * Force_table[K][2]).  G0_k = fl32(h(r_k)); G0 at the last node, r = rcut, is
 * set to 0 because f(rcut) = 0.  G1_k = fl32((G0_{k+1} - G0_k)/(s_{k+1} - s_k))
 * from the rounded G0, and G1 of the last node is 0.
 */
PGO_EXPORT void pgo_table_build(int E, int F, double rcut, int shape, const double *params,
                                float *table)
{
    const long K = 1L << (E + F);
    for (long k = 0; k < K; k++) {
        const double r = pgo_node_r(E, F, rcut, k);
        table[2 * k] = (k == K - 1) ? 0.0f : (float)pgo_shape_h(shape, r, params);
    }
    for (long k = 0; k < K - 1; k++) {
        const double ds = pgo_node_s(E, F, k + 1) - pgo_node_s(E, F, k);
        table[2 * k + 1] = (float)(((double)table[2 * k + 2] - (double)table[2 * k]) / ds);
    }
    table[2 * K - 1] = 0.0f;
}

/* Linear interpolation of h at affine-transformed distance s (steps 1-5 of
 * the force procedure, Sec. 3.4.2): g = G0_k + G1_k (s - s_k). */
PGO_EXPORT double pgo_lut_eval(double s, int E, int F, const double *table)
{
    const double smax = pgo_smax(E, F);
    if (s > smax) s = smax;
    double sk;
    const long k = pgo_lut_index(s, E, F, &sk);
    return (double)table[2 * k] + (double)table[2 * k + 1] * (s - sk);
}

/*
 * Central force from the table, Eq. (arbitrary_force) with the force
 * procedure of Sec. 3.4.2.  absum_i = sum_j m_j |g| |d| (NULL to skip) is the
 * scale that errors of this sum with cancellation are measured against.  The paper pre-scales positions by
 * sqrt(s_max-2)/rcut so that s = |dr~|^2 + 2 and rescales the sum at the end;
 * here s = (s_max-2)/rcut^2 |d|^2 + 2 with unscaled d, which is the same
 * number in exact arithmetic and needs no rescale.
 */
PGO_EXPORT void pgo_lut_items(long n_items, const int32_t *items, const double *xi,
                              const double *yi, const double *zi, const double *xj,
                              const double *yj, const double *zj, const double *mj, int E, int F,
                              double rcut, const double *table, double *ax, double *ay,
                              double *az, double *absum)
{
    const double smax = pgo_smax(E, F);
    const double c = (smax - 2.0) / (rcut * rcut);
    const float c_f = pgo_scale_f32(E, F, rcut);
    long t;
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < n_items; t++) {
        const long i0 = items[4 * t + 0], n_i = items[4 * t + 1];
        const long j0 = items[4 * t + 2], n_j = items[4 * t + 3];
        for (long i = i0; i < i0 + n_i; i++) {
            double sx = 0.0, sy = 0.0, sz = 0.0, sa = 0.0;
            for (long j = j0; j < j0 + n_j; j++) {
                const double dx = (double)xj[j] - (double)xi[i];
                const double dy = (double)yj[j] - (double)yi[i];
                const double dz = (double)zj[j] - (double)zi[i];
                const double r2 = dx * dx + dy * dy + dz * dz;
                double s = c * r2 + 2.0;
                double sk;
                int clamped;
                const long k = pgo_pair_bin(xi[i], yi[i], zi[i], xj[j], yj[j], zj[j], c_f, E, F,
                                            &sk, &clamped);
                if (clamped) s = smax;
                const double g = (double)table[2 * k] + (double)table[2 * k + 1] * (s - sk);
                const double m = mj[j];
                sx += m * g * dx;
                sy += m * g * dy;
                sz += m * g * dz;
                sa += fabs(m * g) * sqrt(r2);
            }
            ax[i] = sx;
            ay[i] = sy;
            az[i] = sz;
            if (absum) absum[i] = sa;
        }
    }
}

/*
 * Analytic companion of the table force: a_i = sum_j m_j h(r_ij) d_ij with the
 * exact h = f/r, for measuring the table error.  Two scales per i (NULL to
 * skip): absum_i = sum_j m_j |h| |d| (the scale of the PP sum itself), and
 * fullsum_i = sum over pairs with 0 < r < rcut of m_j F(r), F the whole
 * force the PP part belongs to: R(r, eps) for the S2 split (PP plus PM,
 * the quantity the paper's accuracy test of Sec. 4.2 measures errors
 * against) and r (r^2+eps^2)^{-3/2} for the softened Newtonian shape.
 */
PGO_EXPORT void pgo_central_items(long n_items, const int32_t *items, const double *xi,
                                  const double *yi, const double *zi, const double *xj,
                                  const double *yj, const double *zj, const double *mj, int shape,
                                  const double *params, double *ax, double *ay, double *az,
                                  double *absum, double *fullsum)
{
    const double eps = params[0], rcut = params[1];
    long t;
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < n_items; t++) {
        const long i0 = items[4 * t + 0], n_i = items[4 * t + 1];
        const long j0 = items[4 * t + 2], n_j = items[4 * t + 3];
        for (long i = i0; i < i0 + n_i; i++) {
            double sx = 0.0, sy = 0.0, sz = 0.0, sa = 0.0, sf = 0.0;
            for (long j = j0; j < j0 + n_j; j++) {
                const double dx = (double)xj[j] - (double)xi[i];
                const double dy = (double)yj[j] - (double)yi[i];
                const double dz = (double)zj[j] - (double)zi[i];
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                const double h = pgo_shape_h(shape, r, params);
                const double m = mj[j];
                sx += m * h * dx;
                sy += m * h * dy;
                sz += m * h * dz;
                sa += fabs(m * h) * r;
                if (r > 0.0 && r < rcut) {
                    if (shape == PGO_SHAPE_S2PP)
                        sf += m * pgo_s2_R(r, eps);
                    else
                        sf += m * r / pow(r * r + eps * eps, 1.5);
                }
            }
            ax[i] = sx;
            ay[i] = sy;
            az[i] = sz;
            if (absum) absum[i] = sa;
            if (fullsum) fullsum[i] = sf;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Adjoints of L = sum_i w_i . a_i (chain rule applied to the two forces).   */
/* ------------------------------------------------------------------------ */

/*
 * Newton, general i/j sets.  With d = r_j - r_i, rho = (|d|^2+eps_i^2)^{-1/2}
 * and the pair term T = m_j rho^3 (w_i . d):
 *   dT/dd = m_j [rho^3 w_i - 3 rho^5 (w_i . d) d],  dd/dr_j = I,  dd/dr_i = -I,
 *   dT/dm_j = rho^3 (w_i . d).
 * gxi_i = -sum_j dT/dd;  gxj_j = sum_i dT/dd;  gmj_j = sum_i rho^3 (w_i . d).
 * absi_i, absj_j and absm_j are the scales of these sums for error measures:
 * the sums of the magnitudes of every product the pair terms expand into,
 * with the dot product w_i . d counted as |w_x d_x| + |w_y d_y| + |w_z d_z|
 * (an FP32 evaluation of w_i . d errs by a rounding of those, not of
 * |w_i . d|, which can cancel to nothing):
 *   absi_i = sum_j m_j (rho^3 |w_i| + 3 rho^5 a_ij |d|),  absj_j likewise
 *   over i,  absm_j = sum_i rho^3 a_ij,  a_ij = sum_c |w_i,c d_c|.
 * Any output pointer may be NULL (gxi..gzi together, gxj..gzj together).
 * Pairs with zero softened distance are skipped like in the forward sum.
 */
PGO_EXPORT void pgo_newton_bwd(long ni, const double *xi, const double *yi, const double *zi,
                               const double *eps2i, long nj, const double *xj, const double *yj,
                               const double *zj, const double *mj, const double *wx,
                               const double *wy, const double *wz, double *gxi, double *gyi,
                               double *gzi, double *gxj, double *gyj, double *gzj, double *gmj,
                               double *absi, double *absj, double *absm)
{
    long i, j;
    if (gxi) {
#pragma omp parallel for schedule(dynamic, 16)
        for (i = 0; i < ni; i++) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, sa = 0.0;
            for (long jj = 0; jj < nj; jj++) {
                const double dx = (double)xj[jj] - xi[i];
                const double dy = (double)yj[jj] - yi[i];
                const double dz = (double)zj[jj] - zi[i];
                const double q = dx * dx + dy * dy + dz * dz + (double)eps2i[i];
                if (q == 0.0) continue;
                const double rho = 1.0 / sqrt(q);
                const double rho3 = rho * rho * rho, rho5 = rho3 * rho * rho;
                const double wd = (double)wx[i] * dx + (double)wy[i] * dy + (double)wz[i] * dz;
                const double m = mj[jj];
                const double t0 = m * (rho3 * wx[i] - 3.0 * rho5 * wd * dx);
                const double t1 = m * (rho3 * wy[i] - 3.0 * rho5 * wd * dy);
                const double t2 = m * (rho3 * wz[i] - 3.0 * rho5 * wd * dz);
                const double awd = fabs((double)wx[i] * dx) + fabs((double)wy[i] * dy) +
                                   fabs((double)wz[i] * dz);
                const double wn = sqrt((double)wx[i] * wx[i] + (double)wy[i] * wy[i] +
                                       (double)wz[i] * wz[i]);
                s0 -= t0;
                s1 -= t1;
                s2 -= t2;
                sa += fabs(m) * (rho3 * wn + 3.0 * rho5 * awd * sqrt(dx * dx + dy * dy + dz * dz));
            }
            gxi[i] = s0;
            gyi[i] = s1;
            gzi[i] = s2;
            if (absi) absi[i] = sa;
        }
    }
    if (gxj || gmj || absj || absm) {
#pragma omp parallel for schedule(dynamic, 16)
        for (j = 0; j < nj; j++) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, sm = 0.0, sa = 0.0, sb = 0.0;
            for (long ii = 0; ii < ni; ii++) {
                const double dx = (double)xj[j] - xi[ii];
                const double dy = (double)yj[j] - yi[ii];
                const double dz = (double)zj[j] - zi[ii];
                const double q = dx * dx + dy * dy + dz * dz + (double)eps2i[ii];
                if (q == 0.0) continue;
                const double rho = 1.0 / sqrt(q);
                const double rho3 = rho * rho * rho, rho5 = rho3 * rho * rho;
                const double wd = (double)wx[ii] * dx + (double)wy[ii] * dy + (double)wz[ii] * dz;
                const double m = mj[j];
                const double t0 = m * (rho3 * wx[ii] - 3.0 * rho5 * wd * dx);
                const double t1 = m * (rho3 * wy[ii] - 3.0 * rho5 * wd * dy);
                const double t2 = m * (rho3 * wz[ii] - 3.0 * rho5 * wd * dz);
                const double awd = fabs((double)wx[ii] * dx) + fabs((double)wy[ii] * dy) +
                                   fabs((double)wz[ii] * dz);
                const double wn = sqrt((double)wx[ii] * wx[ii] + (double)wy[ii] * wy[ii] +
                                       (double)wz[ii] * wz[ii]);
                s0 += t0;
                s1 += t1;
                s2 += t2;
                sm += rho3 * wd;
                sa += fabs(m) * (rho3 * wn + 3.0 * rho5 * awd * sqrt(dx * dx + dy * dy + dz * dz));
                sb += rho3 * awd;
            }
            if (gxj) {
                gxj[j] = s0;
                gyj[j] = s1;
                gzj[j] = s2;
            }
            if (gmj) gmj[j] = sm;
            if (absj) absj[j] = sa;
            if (absm) absm[j] = sb;
        }
    }
}

/*
 * Table force adjoint over interaction lists.  With g = G0_k + G1_k (s - s_k)
 * and the pair term T = m_j g (w_i . d):
 *   dL/dG0_k = sum over pairs in bin k of m_j (w_i . d)
 *   dL/dG1_k = sum over pairs in bin k of m_j (s - s_k) (w_i . d)
 *   dL/dm_j  = sum_i g (w_i . d)
 * G0 and G1 are treated as independent leaves.  gtab_abs (2K), when not
 * NULL, receives the sums of the absolute terms; gmj_abs (nj_total) receives
 * sum_i a_ij (|G0_k| + |G1_k| (s_{k+1} - s_k)), the size g can take in its
 * bin (its G1 part scaled by the bin width rather than by s - s_k, which an
 * FP32 evaluation of s knows only to one rounding of s).  Here, and in
 * gtab_abs, the dot product counts as a_ij = sum_c |w_i,c d_c|: an FP32
 * evaluation of w_i . d errs by a rounding of those products, not of
 * |w_i . d|, which can cancel to nothing.
 * gtab is double[2K]
 * interleaved like the table; gmj is per j entry of the arrays (an entry used
 * by several items accumulates over them).  Items run one after another so
 * that no two threads add into the same j entry or bin.
 */
PGO_EXPORT void pgo_lut_bwd_items(long n_items, const int32_t *items, const double *xi,
                                  const double *yi, const double *zi, const double *xj,
                                  const double *yj, const double *zj, const double *mj,
                                  const double *wx, const double *wy, const double *wz, int E,
                                  int F, double rcut, const double *table, double *gtab,
                                  double *gmj, long nj_total, double *gtab_abs, double *gmj_abs)
{
    const long K = 1L << (E + F);
    const double smax = pgo_smax(E, F);
    const double c = (smax - 2.0) / (rcut * rcut);
    const float c_f = pgo_scale_f32(E, F, rcut);
    memset(gtab, 0, sizeof(double) * 2 * K);
    if (gmj) memset(gmj, 0, sizeof(double) * nj_total);
    if (gtab_abs) memset(gtab_abs, 0, sizeof(double) * 2 * K);
    if (gmj_abs) memset(gmj_abs, 0, sizeof(double) * nj_total);
    for (long t = 0; t < n_items; t++) {
        const long i0 = items[4 * t + 0], n_i = items[4 * t + 1];
        const long j0 = items[4 * t + 2], n_j = items[4 * t + 3];
        for (long i = i0; i < i0 + n_i; i++) {
            for (long j = j0; j < j0 + n_j; j++) {
                const double dx = (double)xj[j] - (double)xi[i];
                const double dy = (double)yj[j] - (double)yi[i];
                const double dz = (double)zj[j] - (double)zi[i];
                double s = c * (dx * dx + dy * dy + dz * dz) + 2.0;
                double sk;
                int clamped;
                const long k = pgo_pair_bin(xi[i], yi[i], zi[i], xj[j], yj[j], zj[j], c_f, E, F,
                                            &sk, &clamped);
                if (clamped) s = smax;
                const double g = (double)table[2 * k] + (double)table[2 * k + 1] * (s - sk);
                const double wd = (double)wx[i] * dx + (double)wy[i] * dy + (double)wz[i] * dz;
                const double m = mj[j];
                gtab[2 * k] += m * wd;
                gtab[2 * k + 1] += m * (s - sk) * wd;
                if (gmj) gmj[j] += g * wd;
                const double awd = fabs((double)wx[i] * dx) + fabs((double)wy[i] * dy) +
                                   fabs((double)wz[i] * dz);
                if (gtab_abs) {
                    gtab_abs[2 * k] += fabs(m) * awd;
                    gtab_abs[2 * k + 1] += fabs(m * (s - sk)) * awd;
                }
                if (gmj_abs) {
                    const double width = (k + 1 < K) ? pgo_node_s(E, F, k + 1) - sk : 0.0;
                    gmj_abs[j] += awd * (fabs(table[2 * k]) + fabs(table[2 * k + 1]) * width);
                }
            }
        }
    }
}

/*
 * Gradient with respect to the node values of a table whose slopes follow
 * them: with G1_k = (G0_{k+1} - G0_k) / (s_{k+1} - s_k) for k < K-1 and
 * G1_{K-1} = 0 (the table of Sec. 3.4.1), the chain rule on
 * L(G0, G1(G0)) gives
 *   dL/dG0_k (total) = dL/dG0_k + dL/dG1_{k-1} / (s_k - s_{k-1})
 *                                - dL/dG1_k / (s_{k+1} - s_k),
 * each term present where its index exists.  gtab: double[2K] (interleaved
 * G0, G1 gradients); g0: double[K].
 */
PGO_EXPORT void pgo_table_grad_chain(int E, int F, const double *gtab, double *g0)
{
    const long K = 1L << (E + F);
    for (long k = 0; k < K; k++) {
        double v = gtab[2 * k];
        if (k >= 1) v += gtab[2 * (k - 1) + 1] / (pgo_node_s(E, F, k) - pgo_node_s(E, F, k - 1));
        if (k + 1 < K) v -= gtab[2 * k + 1] / (pgo_node_s(E, F, k + 1) - pgo_node_s(E, F, k));
        g0[k] = v;
    }
}

/*
 * Position gradients of L = sum_i w_i . a_i for the table force over
 * interaction lists.  The interpolant g(s) = G0_k + G1_k (s - s_k) is linear
 * in s inside bin k, so dg/ds = G1_k there (and 0 on the clamp s = s_max),
 * with s = c |d|^2 + 2, ds/dd = 2 c d.  For the pair term
 * T = m_j g (w_i . d), d = r_j - r_i:
 *   dT/dd = m_j [ g w_i + 2 c G1_k (w_i . d) d ]
 * gxi_i = -sum_j dT/dd, gxj_j = sum_i dT/dd (an entry used by several lists
 * accumulates).  absi / absj (may be NULL) receive the sums of the
 * magnitudes of the products: m_j (|g| |w_i| + 2 c |G1_k| a_ij |d|),
 * a_ij = sum_c |w_i,c d_c|, with |g| <= |G0_k| + |G1_k| (s_{k+1} - s_k).
 */
PGO_EXPORT void pgo_lut_bwd_pos_items(long n_items, const int32_t *items, const double *xi,
                                      const double *yi, const double *zi, const double *xj,
                                      const double *yj, const double *zj, const double *mj,
                                      const double *wx, const double *wy, const double *wz,
                                      int E, int F, double rcut, const double *table,
                                      long ni_total, long nj_total, double *gxi, double *gyi,
                                      double *gzi, double *gxj, double *gyj, double *gzj,
                                      double *absi, double *absj)
{
    const long K = 1L << (E + F);
    const double smax = pgo_smax(E, F);
    const double c = (smax - 2.0) / (rcut * rcut);
    const float c_f = pgo_scale_f32(E, F, rcut);
    memset(gxi, 0, sizeof(double) * ni_total);
    memset(gyi, 0, sizeof(double) * ni_total);
    memset(gzi, 0, sizeof(double) * ni_total);
    memset(gxj, 0, sizeof(double) * nj_total);
    memset(gyj, 0, sizeof(double) * nj_total);
    memset(gzj, 0, sizeof(double) * nj_total);
    if (absi) memset(absi, 0, sizeof(double) * ni_total);
    if (absj) memset(absj, 0, sizeof(double) * nj_total);
    for (long t = 0; t < n_items; t++) {
        const long i0 = items[4 * t + 0], n_i = items[4 * t + 1];
        const long j0 = items[4 * t + 2], n_j = items[4 * t + 3];
        for (long i = i0; i < i0 + n_i; i++) {
            for (long j = j0; j < j0 + n_j; j++) {
                const double dx = (double)xj[j] - (double)xi[i];
                const double dy = (double)yj[j] - (double)yi[i];
                const double dz = (double)zj[j] - (double)zi[i];
                double s = c * (dx * dx + dy * dy + dz * dz) + 2.0;
                double sk;
                int clamped;
                const long k = pgo_pair_bin(xi[i], yi[i], zi[i], xj[j], yj[j], zj[j], c_f, E, F,
                                            &sk, &clamped);
                if (clamped) s = smax;
                const double G0 = table[2 * k], G1 = table[2 * k + 1];
                const double g = G0 + G1 * (s - sk);
                const double dgds = clamped ? 0.0 : G1;
                const double wd = (double)wx[i] * dx + (double)wy[i] * dy + (double)wz[i] * dz;
                const double m = mj[j];
                const double t0 = m * (g * wx[i] + 2.0 * c * dgds * wd * dx);
                const double t1 = m * (g * wy[i] + 2.0 * c * dgds * wd * dy);
                const double t2 = m * (g * wz[i] + 2.0 * c * dgds * wd * dz);
                gxi[i] -= t0;
                gyi[i] -= t1;
                gzi[i] -= t2;
                gxj[j] += t0;
                gyj[j] += t1;
                gzj[j] += t2;
                if (absi || absj) {
                    const double width = (k + 1 < K) ? pgo_node_s(E, F, k + 1) - sk : 0.0;
                    const double awd = fabs((double)wx[i] * dx) + fabs((double)wy[i] * dy) +
                                       fabs((double)wz[i] * dz);
                    const double wn = sqrt((double)wx[i] * wx[i] + (double)wy[i] * wy[i] +
                                           (double)wz[i] * wz[i]);
                    const double a = fabs(m) * ((fabs(G0) + fabs(G1) * width) * wn +
                                                2.0 * c * fabs(dgds) * awd *
                                                    sqrt(dx * dx + dy * dy + dz * dz));
                    if (absi) absi[i] += a;
                    if (absj) absj[j] += a;
                }
            }
        }
    }
}

/*
 * Potential table on the bins of the force table (the node equation of
 * Sec. 3.4.1 applied to a pair potential p instead of f/r): P0_k = p(r_k),
 * 0 at the last node (p vanishes at rcut), P1_k the chord to the next node
 * from the rounded P0 values; interleaved (P0_0, P1_0, P0_1, ...).
 */
PGO_EXPORT void pgo_pot_table_build(int E, int F, double rcut, int shape, const double *params,
                                    float *table)
{
    const long K = 1L << (E + F);
    for (long k = 0; k < K; k++) {
        const double r = pgo_node_r(E, F, rcut, k);
        table[2 * k] = (k == K - 1) ? 0.0f : (float)pgo_shape_p(shape, r, params);
    }
    for (long k = 0; k < K - 1; k++) {
        const double ds = pgo_node_s(E, F, k + 1) - pgo_node_s(E, F, k);
        table[2 * k + 1] = (float)(((double)table[2 * k + 2] - (double)table[2 * k]) / ds);
    }
    table[2 * K - 1] = 0.0f;
}

/*
 * Potential from a potential table over interaction lists:
 * phi_i = sum_j m_j (P0_k + P1_k (s - s_k)), with s and k as for the force
 * (steps 1-5 of Sec. 3.4.2 on the second table).  absum_i (may be NULL) =
 * sum_j |m_j| (|P0_k| + |P1_k| (s_{k+1} - s_k)), the scale of the sum.
 * phi and absum: double[ni_total], zeroed first.
 */
PGO_EXPORT void pgo_lut_pot_items(long n_items, const int32_t *items, const double *xi,
                                  const double *yi, const double *zi, const double *xj,
                                  const double *yj, const double *zj, const double *mj, int E,
                                  int F, double rcut, const double *ptable, long ni_total,
                                  double *phi, double *absum)
{
    const long K = 1L << (E + F);
    const double smax = pgo_smax(E, F);
    const double c = (smax - 2.0) / (rcut * rcut);
    const float c_f = pgo_scale_f32(E, F, rcut);
    memset(phi, 0, sizeof(double) * ni_total);
    if (absum) memset(absum, 0, sizeof(double) * ni_total);
    for (long t = 0; t < n_items; t++) {
        const long i0 = items[4 * t + 0], n_i = items[4 * t + 1];
        const long j0 = items[4 * t + 2], n_j = items[4 * t + 3];
#pragma omp parallel for schedule(static)
        for (long i = i0; i < i0 + n_i; i++) {
            double sp = 0.0, sa = 0.0;
            for (long j = j0; j < j0 + n_j; j++) {
                const double dx = (double)xj[j] - (double)xi[i];
                const double dy = (double)yj[j] - (double)yi[i];
                const double dz = (double)zj[j] - (double)zi[i];
                double s = c * (dx * dx + dy * dy + dz * dz) + 2.0;
                double sk;
                int clamped;
                const long k = pgo_pair_bin(xi[i], yi[i], zi[i], xj[j], yj[j], zj[j], c_f, E, F,
                                            &sk, &clamped);
                if (clamped) s = smax;
                const double P0 = ptable[2 * k], P1 = ptable[2 * k + 1];
                sp += mj[j] * (P0 + P1 * (s - sk));
                const double width = (k + 1 < K) ? pgo_node_s(E, F, k + 1) - sk : 0.0;
                sa += fabs(mj[j]) * (fabs(P0) + fabs(P1) * width);
            }
            phi[i] += sp;
            if (absum) absum[i] += sa;
        }
    }
}
