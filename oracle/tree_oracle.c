/*
 * tree_oracle.c -- FP64 reference of the Barnes-Hut tree that produces the
 * (i-group, j-list) interaction lists of the paper's tree-code experiment
 * (Sec. 5, the Plummer and King models with opening parameter 0.75, monopole
 * moments, or monopole and quadrupole moments carried by pseudo-particles).
 *
 * TEST INFRASTRUCTURE ONLY, like pgh_oracle.c: the library package never
 * includes, links or calls it, and it shares nothing with the GPU path.
 *
 * The paper fixes the method only in outline (a Barnes-Hut tree with Barnes'
 * shared lists for groups of i-particles, opening parameter theta = 0.75,
 * quadrupole moments represented as pseudo-particles after Kawai & Makino);
 * the precise definitions below are this implementation's readings, and the
 * GPU tree follows the same ones:
 *
 *   Frame.  lo = componentwise minimum of the positions; extent = the largest
 *     of (max - min) over the three axes; scale = 2^21 / extent (0 when the
 *     extent is 0).  All in FP32, the precision of the positions, so that the
 *     integer keys are the same on every implementation.
 *   Keys.  k_a = min(floor((x_a - lo_a) * scale), 2^21 - 1) per axis (FP32
 *     subtraction and product), interleaved into a 63-bit Morton key with x
 *     in the most significant bit of each 3-bit digit, then y, then z.
 *   Order.  Particles sorted by (key, original index).
 *   Octree.  The root (level 0) holds every particle.  A node at level L
 *     holds the particles whose keys share its first 3L bits; it is a leaf
 *     when it holds at most n_leaf particles or L = 21, else its children are
 *     its non-empty octants in digit order.  Nodes are numbered breadth
 *     first, each level in key order.  Node size l = extent / 2^L.
 *   Moments.  M = sum m, com = sum m x / M (the plain mean of the positions
 *     when M = 0), S = sum m (x - com)(x - com)^T, all from the node's own
 *     particles in double precision.
 *   Pseudo-particles.  Monopole: one particle of mass M at com.  Quadrupole:
 *     three particles of mass M/3 at com + alpha cos(2 pi k/3) e1 +
 *     beta sin(2 pi k/3) e2 (k = 0, 1, 2), with S = sum lambda_i e_i e_i^T,
 *     lambda1 >= lambda2 >= lambda3, alpha^2 = 2 (lambda1 - lambda3)/M,
 *     beta^2 = 2 (lambda2 - lambda3)/M.  The set has the node's mass, zero
 *     dipole about com and second moment S - lambda3 I, whose traceless part
 *     (the quadrupole that enters the potential) is that of S.
 *   Groups.  The i-groups are the nodes that hold at most n_crit particles
 *     (or are leaves) and whose parent holds more (or that are the root),
 *     in key order; they partition the particles.
 *   Walk.  For group g with the bounding box [b_lo, b_hi] of its particles,
 *     the nodes are visited breadth first from the root, each level in the
 *     order its nodes were reached.  A node that is g or an ancestor of g is
 *     opened.  Any other node is accepted when l < theta d, d the distance
 *     from its com to the box (0 inside), and then contributes its
 *     pseudo-particles; otherwise a leaf contributes its particles and an
 *     internal node has its children visited on the next level.  The list is
 *     the contributions in the order of the visit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PGO_EXPORT __attribute__((visibility("default")))

#define TREE_BITS 21
#define TREE_MAX_LEVEL 21

/* lo[3], extent, scale: FP32 values in out[0..4]. */
PGO_EXPORT void pgo_tree_frame(long n, const float *x, const float *y, const float *z,
                               float *out)
{
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
    const float *p[3] = {x, y, z};
    for (int a = 0; a < 3; a++) {
        if (n > 0) lo[a] = hi[a] = p[a][0];
        for (long i = 1; i < n; i++) {
            if (p[a][i] < lo[a]) lo[a] = p[a][i];
            if (p[a][i] > hi[a]) hi[a] = p[a][i];
        }
    }
    float ext = 0.f;
    for (int a = 0; a < 3; a++) {
        const float e = hi[a] - lo[a];
        if (e > ext) ext = e;
    }
    out[0] = lo[0];
    out[1] = lo[1];
    out[2] = lo[2];
    out[3] = ext;
    out[4] = ext > 0.f ? (float)(2097152.0f / ext) : 0.f;
}

static uint64_t axis_cell(float v, float lo, float scale)
{
    const float d = v - lo;  /* FP32 */
    const float t = d * scale;
    const double f = floor((double)t);
    long k = (long)f;
    if (k < 0) k = 0;
    if (k > (1L << TREE_BITS) - 1) k = (1L << TREE_BITS) - 1;
    return (uint64_t)k;
}

PGO_EXPORT void pgo_tree_keys(long n, const float *x, const float *y, const float *z,
                              const float *frame, uint64_t *key)
{
    for (long i = 0; i < n; i++) {
        const uint64_t kx = axis_cell(x[i], frame[0], frame[4]);
        const uint64_t ky = axis_cell(y[i], frame[1], frame[4]);
        const uint64_t kz = axis_cell(z[i], frame[2], frame[4]);
        uint64_t k = 0;
        for (int b = TREE_BITS - 1; b >= 0; b--) {
            k = (k << 3) | (((kx >> b) & 1u) << 2) | (((ky >> b) & 1u) << 1) | ((kz >> b) & 1u);
        }
        key[i] = k;
    }
}

typedef struct {
    uint64_t key;
    long idx;
} KeyIdx;

static int cmp_key_idx(const void *a, const void *b)
{
    const KeyIdx *p = (const KeyIdx *)a, *q = (const KeyIdx *)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

/* perm[r] = original index of the particle of rank r. */
PGO_EXPORT void pgo_tree_sort(long n, const uint64_t *key, long *perm)
{
    KeyIdx *v = (KeyIdx *)malloc(sizeof(KeyIdx) * (n > 0 ? n : 1));
    for (long i = 0; i < n; i++) {
        v[i].key = key[i];
        v[i].idx = i;
    }
    qsort(v, (size_t)n, sizeof(KeyIdx), cmp_key_idx);
    for (long i = 0; i < n; i++) perm[i] = v[i].idx;
    free(v);
}

static int digit_at(uint64_t key, int level)
{
    /* the 3-bit digit that selects the child at `level` (1..21) */
    return (int)((key >> (3 * (TREE_MAX_LEVEL - level))) & 7u);
}

/*
 * Octree over sorted keys.  Returns the node count, or -1 when max_nodes is
 * too small (nothing beyond max_nodes is written; at most 22 n nodes exist).
 */
PGO_EXPORT long pgo_tree_build(long n, const uint64_t *ks, int n_leaf, long max_nodes,
                               long *begin, long *count, int *level, long *first_child,
                               int *n_child, long *parent)
{
    if (n <= 0) return 0;
    if (max_nodes < 1) return -1;
    long nn = 1;
    long head = 0;
    begin[0] = 0;
    count[0] = n;
    level[0] = 0;
    parent[0] = -1;
    /* breadth-first: nodes are appended in the order their parents are processed */
    while (head < nn) {
        const long b = begin[head], c = count[head];
        const int L = level[head];
        first_child[head] = -1;
        n_child[head] = 0;
        if (c > n_leaf && L < TREE_MAX_LEVEL) {
            long r = b;
            first_child[head] = nn;
            while (r < b + c) {
                const int dg = digit_at(ks[r], L + 1);
                long e = r;
                while (e < b + c && digit_at(ks[e], L + 1) == dg) e++;
                if (nn >= max_nodes) return -1;
                begin[nn] = r;
                count[nn] = e - r;
                level[nn] = L + 1;
                parent[nn] = head;
                nn++;
                n_child[head]++;
                r = e;
            }
        }
        head++;
    }
    return nn;
}

PGO_EXPORT void pgo_tree_moments(long n_nodes, const long *begin, const long *count,
                                 const double *xs, const double *ys, const double *zs,
                                 const double *ms, double *mass, double *com, double *S)
{
    long t;
#pragma omp parallel for schedule(dynamic, 64)
    for (t = 0; t < n_nodes; t++) {
        const long b = begin[t], c = count[t];
        double M = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
        for (long i = b; i < b + c; i++) {
            M += ms[i];
            cx += ms[i] * xs[i];
            cy += ms[i] * ys[i];
            cz += ms[i] * zs[i];
        }
        if (M != 0.0) {
            cx /= M;
            cy /= M;
            cz /= M;
        } else {
            cx = cy = cz = 0.0;
            for (long i = b; i < b + c; i++) {
                cx += xs[i];
                cy += ys[i];
                cz += zs[i];
            }
            cx /= (double)c;
            cy /= (double)c;
            cz /= (double)c;
        }
        double sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
        for (long i = b; i < b + c; i++) {
            const double dx = xs[i] - cx, dy = ys[i] - cy, dz = zs[i] - cz;
            sxx += ms[i] * dx * dx;
            syy += ms[i] * dy * dy;
            szz += ms[i] * dz * dz;
            sxy += ms[i] * dx * dy;
            sxz += ms[i] * dx * dz;
            syz += ms[i] * dy * dz;
        }
        mass[t] = M;
        com[3 * t + 0] = cx;
        com[3 * t + 1] = cy;
        com[3 * t + 2] = cz;
        S[6 * t + 0] = sxx;
        S[6 * t + 1] = syy;
        S[6 * t + 2] = szz;
        S[6 * t + 3] = sxy;
        S[6 * t + 4] = sxz;
        S[6 * t + 5] = syz;
    }
}

/*
 * Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations
 * (Golub & Van Loan, Sec. 8.5): w[3] eigenvalues in descending order, V the
 * eigenvectors as columns (V[3*r + c], column c for w[c]).
 */
PGO_EXPORT void pgo_sym3_eigen(const double *S6, double *w, double *V)
{
    double A[3][3] = {{S6[0], S6[3], S6[4]}, {S6[3], S6[1], S6[5]}, {S6[4], S6[5], S6[2]}};
    double Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 64; sweep++) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-40 * dia || off == 0.0) break;
        for (int p = 0; p < 2; p++) {
            for (int q = p + 1; q < 3; q++) {
                if (A[p][q] == 0.0) continue;
                /* rotation that zeroes A[p][q] */
                const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double tn = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(tn * tn + 1.0), sn = tn * cs;
                for (int k = 0; k < 3; k++) {  /* A <- A J */
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq;
                    A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; k++) {  /* A <- J^T A */
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk;
                    A[q][k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 3; k++) {  /* Q <- Q J */
                    const double qkp = Q[k][p], qkq = Q[k][q];
                    Q[k][p] = cs * qkp - sn * qkq;
                    Q[k][q] = sn * qkp + cs * qkq;
                }
            }
        }
    }
    int ord[3] = {0, 1, 2};
    for (int a = 0; a < 3; a++)
        for (int b = a + 1; b < 3; b++)
            if (A[ord[b]][ord[b]] > A[ord[a]][ord[a]]) {
                const int t = ord[a];
                ord[a] = ord[b];
                ord[b] = t;
            }
    for (int c = 0; c < 3; c++) {
        w[c] = A[ord[c]][ord[c]];
        for (int r = 0; r < 3; r++) V[3 * r + c] = Q[r][ord[c]];
    }
}

/* Pseudo-particles of every node: n_pp = (quad ? 3 : 1) per node, node-major. */
PGO_EXPORT void pgo_tree_pseudo(long n_nodes, const double *mass, const double *com,
                                const double *S, int quad, double *px, double *py, double *pz,
                                double *pm)
{
    long t;
#pragma omp parallel for schedule(static)
    for (t = 0; t < n_nodes; t++) {
        const double M = mass[t];
        const double *c = com + 3 * t;
        if (!quad) {
            px[t] = c[0];
            py[t] = c[1];
            pz[t] = c[2];
            pm[t] = M;
            continue;
        }
        double w[3], V[9];
        pgo_sym3_eigen(S + 6 * t, w, V);
        double a2 = 0.0, b2 = 0.0;
        if (M > 0.0) {
            a2 = 2.0 * (w[0] - w[2]) / M;
            b2 = 2.0 * (w[1] - w[2]) / M;
        }
        const double al = sqrt(a2 > 0 ? a2 : 0.0), be = sqrt(b2 > 0 ? b2 : 0.0);
        const double h = sqrt(3.0) / 2.0;
        const double cosk[3] = {1.0, -0.5, -0.5}, sink[3] = {0.0, h, -h};
        for (int k = 0; k < 3; k++) {
            const double u = al * cosk[k], v = be * sink[k];
            px[3 * t + k] = c[0] + u * V[0] + v * V[1];
            py[3 * t + k] = c[1] + u * V[3] + v * V[4];
            pz[3 * t + k] = c[2] + u * V[6] + v * V[7];
            pm[3 * t + k] = M / 3.0;
        }
    }
}

/* The i-groups in key order; returns their count. */
PGO_EXPORT long pgo_tree_groups(long n_nodes, const long *begin, const long *count,
                                const int *n_child, const long *parent, int n_crit, long *groups)
{
    /* a group is found from the node side; key order = order of begin */
    long ng = 0;
    for (long t = 0; t < n_nodes; t++) {
        const int small = count[t] <= n_crit || n_child[t] == 0;
        const int top = parent[t] < 0 || count[parent[t]] > n_crit;
        if (small && top) groups[ng++] = t;
    }
    /* sort by begin: insertion into position (groups are disjoint ranges) */
    for (long a = 1; a < ng; a++) {
        const long g = groups[a];
        long b = a - 1;
        while (b >= 0 && begin[groups[b]] > begin[g]) {
            groups[b + 1] = groups[b];
            b--;
        }
        groups[b + 1] = g;
    }
    return ng;
}

/*
 * Interaction list of group node g.  src (may be NULL, capacity cap): entry
 * e >= 0 is the sorted particle of rank e, entry -(1 + q) is pseudo-particle q
 * (node t's are q = n_pp t .. n_pp t + n_pp - 1).  Returns the list length
 * (entries beyond cap are counted, not written).  margin (may be NULL): the
 * smallest |d - l/theta| / s over the nodes tested against the criterion, s
 * the largest magnitude among the com and box coordinates, 1 + |.| guarded:
 * how far the nearest decision was from flipping, in units of the
 * coordinates' size.
 */
PGO_EXPORT long pgo_tree_walk(long n_nodes, const long *begin, const long *count,
                              const int *level, const long *first_child, const int *n_child,
                              const double *com, double extent, const double *xs,
                              const double *ys, const double *zs, long g, double theta, int quad,
                              long cap, long *src, double *margin)
{
    (void)n_nodes;
    const int npp = quad ? 3 : 1;
    double lo[3], hi[3];
    const long gb = begin[g], gc = count[g];
    lo[0] = hi[0] = xs[gb];
    lo[1] = hi[1] = ys[gb];
    lo[2] = hi[2] = zs[gb];
    for (long i = gb + 1; i < gb + gc; i++) {
        const double v[3] = {xs[i], ys[i], zs[i]};
        for (int a = 0; a < 3; a++) {
            if (v[a] < lo[a]) lo[a] = v[a];
            if (v[a] > hi[a]) hi[a] = v[a];
        }
    }
    long *cur = (long *)malloc(sizeof(long) * 16), *nxt = NULL;
    long ncur = 1, cap_cur = 16;
    cur[0] = 0;
    long len = 0;
    double mg = INFINITY;
    while (ncur > 0) {
        long nnxt = 0, cap_nxt = 16;
        nxt = (long *)malloc(sizeof(long) * cap_nxt);
        for (long f = 0; f < ncur; f++) {
            const long t = cur[f];
            const int anc = level[t] <= level[g] && begin[t] <= gb && gb < begin[t] + count[t];
            int accept = 0;
            if (!anc) {
                double d2 = 0.0, s = 1.0;
                for (int a = 0; a < 3; a++) {
                    const double c = com[3 * t + a];
                    const double e = c < lo[a] ? lo[a] - c : (c > hi[a] ? c - hi[a] : 0.0);
                    d2 += e * e;
                    if (fabs(c) > s) s = fabs(c);
                    if (fabs(lo[a]) > s) s = fabs(lo[a]);
                    if (fabs(hi[a]) > s) s = fabs(hi[a]);
                }
                const double l = extent / (double)(1L << level[t]);
                const double d = sqrt(d2);
                accept = l < theta * d;
                const double m = fabs(d - l / theta) / s;
                if (m < mg) mg = m;
            }
            if (accept) {
                for (int k = 0; k < npp; k++) {
                    if (src && len < cap) src[len] = -(1 + (long)npp * t + k);
                    len++;
                }
            } else if (n_child[t] == 0) {
                for (long i = begin[t]; i < begin[t] + count[t]; i++) {
                    if (src && len < cap) src[len] = i;
                    len++;
                }
            } else {
                for (int k = 0; k < n_child[t]; k++) {
                    if (nnxt == cap_nxt) {
                        cap_nxt *= 2;
                        nxt = (long *)realloc(nxt, sizeof(long) * cap_nxt);
                    }
                    nxt[nnxt++] = first_child[t] + k;
                }
            }
        }
        free(cur);
        cur = nxt;
        ncur = nnxt;
        cap_cur = cap_nxt;
    }
    (void)cap_cur;
    free(cur);
    if (margin) *margin = mg;
    return len;
}
