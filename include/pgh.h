/*
 * pgh.h -- C ABI of an MI355X (gfx950) direct-summation force library in the
 * shape of Phantom-GRAPE (Tanikawa, Yoshikawa, Nitadori & Okamoto,
 * arXiv:1203.4037).
 *
 * The library computes, for a set of i-particles and a set of j-particles,
 *   (1) the Plummer-softened Newtonian acceleration and potential,
 *       Eq. (newton_force) of Sec. 3, with G = 1;
 *   (2) a central force of arbitrary shape f(r) with a finite cutoff,
 *       Eq. (arbitrary_force) of Sec. 3, read from a look-up table of f(r)/r
 *       whose bins are the low E exponent bits and high F fraction bits of the
 *       affine-transformed squared distance s (Sec. 3.4.1, Table 4);
 * for one i-set against one j-set (the GRAPE calls of Sec. 3.6), or for many
 * (i-group, j-list) interaction lists in one launch (the tree and TreePM use
 * of Sec. 5.1), plus the adjoints of both forces for a loss L = sum_i w_i.a_i.
 *
 * Conventions for every call:
 *   - Arrays are FP32 structure-of-arrays in DEVICE memory (hipMalloc'd or a
 *     torch CUDA/HIP tensor), unless a comment says "host".  The caller owns
 *     every array it passes; the library never frees or keeps them.
 *   - Calls are asynchronous on the context's stream (pgh_set_stream); none
 *     synchronises unless it says so.  Inputs must stay valid until the work
 *     on the stream has finished.
 *   - Every call returns PGH_OK (0) or a negative status and never aborts;
 *     pgh_last_error() describes the last failure on that context.
 *   - ni = 0 or nj = 0 is legal: outputs of the ni rows are written as 0.
 *   - A NaN in an input propagates to the outputs it touches; inputs are not
 *     checked for NaN.
 *   - Units: G = 1 (the paper's API has no G argument, Sec. 3.6).
 *   - A context is not thread-safe; use one per host thread or stream.
 */
#ifndef PGH_H
#define PGH_H

#ifdef __cplusplus
extern "C" {
#endif

#define PGH_API __attribute__((visibility("default")))

typedef struct pgh_ctx pgh_ctx;
typedef struct pgh_plan pgh_plan;

enum pgh_status {
    PGH_OK = 0,
    PGH_EINVAL = -1, /* a NULL required pointer or a negative count              */
    PGH_ESTATE = -2, /* a call out of order, e.g. a table force with no table    */
    PGH_ENOMEM = -3, /* a device or host allocation failed                       */
    PGH_EHIP = -4,   /* a HIP runtime call or kernel launch failed               */
    PGH_ERANGE = -5  /* an argument outside its documented range                 */
};

/* Force kinds, used by plans and by the tuner. */
enum pgh_kind {
    PGH_KIND_NEWTON = 0, /* Eq. (newton_force)                                     */
    PGH_KIND_TABLE = 1   /* Eq. (arbitrary_force) through the look-up table        */
};

/* ---------------------------------------------------------------------- */
/* Context: the GRAPE-5 style set-up calls of Sec. 3.6 (g5_open, g5_close,  */
/* g5_set_eps_to_all, g5_set_n, g5_set_xmj).                                */
/* ---------------------------------------------------------------------- */

/* Opens a context on HIP device `device` (g5_open).  `hip_stream` is a
 * hipStream_t the calls run on (NULL: the default stream).  Nothing of the
 * approximate-rsqrt bias calibration of g5_open is needed: the kernels use
 * the hardware rsqrt, accurate to about 1 ulp (pgh_set_rsqrt_refine adds a
 * Newton-Raphson step).
 * On failure *out is NULL and the message is available from
 * pgh_last_error(NULL). */
PGH_API int pgh_open(pgh_ctx **out, int device, void *hip_stream);

/* Frees the context and its device memory (g5_close).  Waits for the
 * context's stream first.  pgh_close(NULL) is a no-op. */
PGH_API int pgh_close(pgh_ctx *c);

/* Message of the last failed call on c (c == NULL: the last failure on this
 * thread of a call made without a context, such as pgh_open).  The string
 * lives until the next call on c. */
PGH_API const char *pgh_last_error(const pgh_ctx *c);

/* Library version as 10000*major + 100*minor + patch. */
PGH_API int pgh_version(void);

/* Sets the stream later calls run on. */
PGH_API int pgh_set_stream(pgh_ctx *c, void *hip_stream);

/* Softening length for every i-particle (g5_set_eps_to_all): eps^2 is stored
 * in FP32 and used when a call passes eps2_i == NULL.  eps >= 0; with eps = 0
 * a pair at zero distance contributes nothing (the guarded kernel runs). */
PGH_API int pgh_set_eps_to_all(pgh_ctx *c, float eps);

/* Number of j-particles the all-pairs calls sum over (g5_set_n), 0 <= nj <=
 * the j-memory size reached by pgh_set_xmj. */
PGH_API int pgh_set_n(pgh_ctx *c, int nj);

/* Copies nj j-particles (positions x,y,z and masses m, device SoA) into the
 * context's j-memory at [adr, adr+nj) (g5_set_xmj, Sec. 3.6: the data are
 * copied into the library's own j-particle records).  The j-memory grows as
 * needed; growing synchronises the stream.  Records are packed as 16-byte
 * (x, y, z, m) so one j-particle is one aligned load (the j-particle record
 * of Sec. 3.1).  Does not change the count set by pgh_set_n. */
PGH_API int pgh_set_xmj(pgh_ctx *c, int adr, int nj, const float *x, const float *y,
                const float *z, const float *m);

/* Newton-Raphson refinement of the hardware rsqrt: off (0, default) or on (1).
 * Sec. 2 of the paper refines its 12-bit approximate inverse square root
 * to reach single precision; gfx950's v_rsq_f32 is accurate to about one
 * ulp already, and the step (3 more FP32 operations per pair) adds its own
 * roundings instead of removing error: measured per-pair force errors are
 * max 4.7e-7 without and 5.7e-7 with it.  Kept selectable.  Applies to the
 * Newton forward and adjoint kernels. */
PGH_API int pgh_set_rsqrt_refine(pgh_ctx *c, int on);

/* ---------------------------------------------------------------------- */
/* Newton's force: Eq. (newton_force), the loop of Sec. 3.3.                */
/* ---------------------------------------------------------------------- */

/* Accelerations and potentials of ni i-particles from the nj = pgh_set_n
 * j-particles of the j-memory (g5_calculate_force_on_x):
 *   a_i   =  sum_j m_j (r_j - r_i) / (|r_j - r_i|^2 + eps_i^2)^{3/2}
 *   phi_i = -sum_j m_j / (|r_j - r_i|^2 + eps_i^2)^{1/2}
 * xi, yi, zi: ni positions.  eps2_i: ni squared softenings (each > 0), or
 * NULL to use pgh_set_eps_to_all.  ax, ay, az: ni outputs.  phi: ni outputs,
 * or NULL to skip the potential.  The sum runs over every j, so when an
 * i-particle is also a j-particle phi_i includes its self term -m_i/eps_i
 * (the paper's convention, Sec. 4.1); its force term is zero.  Outputs must
 * not alias inputs. */
PGH_API int pgh_calc_newton(pgh_ctx *c, int ni, const float *xi, const float *yi, const float *zi,
                    const float *eps2_i, float *ax, float *ay, float *az, float *phi);

/* pgh_calc_newton for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and errors as pgh_calc_newton, the same
 * results up to FP32 summation order (its j-split, and with no variant
 * selected its tile shape, can differ), and it calls no hipMalloc, hipFree
 * or allocating library routine.  Where
 * pgh_calc_newton grows a context buffer for the partial sums of its
 * j-split, this entry point uses a fixed device array of 2^20 floats
 * (4 MiB) that the library holds on each GPU it runs on until the process
 * ends (located at pgh_open; PGH_ESTATE if that failed): the split is
 * limited to the shares whose partial sums (S x 4 x ni floats) fit it, and a
 * launch that cannot be split uses none of it, so no input size is
 * rejected.  Every call on one GPU shares that array: calls that overlap on
 * one GPU (two contexts or streams at once) race and must be ordered by the
 * caller.  Nothing in the array has to start at zero; each call overwrites
 * the part it reads.  The j-memory must already hold the j-particles
 * (pgh_set_xmj, which may allocate, is called before). */
PGH_API int pgh_calc_newton_noalloc(pgh_ctx *c, int ni, const float *xi, const float *yi,
                                    const float *zi, const float *eps2_i, float *ax, float *ay,
                                    float *az, float *phi);

/* ---------------------------------------------------------------------- */
/* Central force of arbitrary shape through the bit-binned table (Sec. 3.4) */
/* ---------------------------------------------------------------------- */

/* Host callback returning h(r) = f(r)/r (the table stores G0_k = f(r_k)/r_k,
 * Sec. 3.4.1).  It is called at r = 0 for the first node, where it must
 * return the limit of f(r)/r. */
typedef double (*pgh_f_over_r)(double r, void *user);

/* Builds the table for exponent bits E (0..6), fraction bits F (0..10),
 * E + F <= 14, and cutoff rcut > 0 from a host callback (the table setter of
 * Sec. 3.6) and makes it the context's table.  Node k = 2^F bE + bF sits at
 * s_k = 2^{bE+1}(1 + bF/2^F) (the node equation of Sec. 3.4.1), i.e. at
 * r_k = rcut ((s_k - 2)/(s_max - 2))^{1/2} with s_max = 2^{2^E}(2 - 2^-F);
 * G0_k = fl32(h(r_k)) with G0 of the last node (r = rcut) set to 0;
 * G1_k = fl32((G0_{k+1} - G0_k)/(s_{k+1} - s_k)) and G1 of the last node 0.
 * The nodes and quotients are evaluated in double on the host.
 * table_out: NULL, or host float[2 * 2^(E+F)] receiving (G0_0, G1_0, G0_1, ...).
 * Synchronous (uploads the table). */
PGH_API int pgh_build_table(pgh_ctx *c, int E, int F, float rcut, pgh_f_over_r f_over_r, void *user,
                    float *table_out);

/* The same table computed into host memory only (no context, no device):
 * table_out is host float[2 * 2^(E+F)].  Returns PGH_EINVAL for a NULL
 * pointer and PGH_ERANGE for an E, F or rcut out of range. */
PGH_API int pgh_table_compute(int E, int F, float rcut, pgh_f_over_r f_over_r, void *user,
                              float *table_out);

/* Sets the context's table from a device array of 2 * 2^(E+F) floats,
 * interleaved (G0_0, G1_0, G0_1, G1_1, ...) like the paper's
 * Force_table[K][2]; same E, F, rcut ranges as pgh_build_table.  The values
 * are copied on the stream. */
PGH_API int pgh_set_table(pgh_ctx *c, int E, int F, float rcut, const float *table);

/* Built-in f(r)/r of the particle-particle part of the S2 force split,
 * f = R(r, eps) - R(r, rcut) with R the S2 profile of Hockney & Eastwood
 * (Eqs. s2pp and s2 of Sec. 4.2), and its analytic limit at r = 0.
 * user points to double[2] = {eps, rcut}.  Usable as a pgh_f_over_r. */
PGH_API double pgh_s2pp_f_over_r(double r, void *user);

/* Potential table on the bins of the current force table (same E, F and
 * rcut; the force procedure of Sec. 3.4.2 applied to a second table): from
 * a host callback returning the pair potential p(r) (called at r = 0 for
 * the first node; p must vanish at rcut: the last node is set to 0), nodes
 * P0_k = fl32(p(r_k)) and chords P1_k as for the force table.  table_out:
 * NULL or host float[2 * 2^(E+F)].  PGH_ESTATE before a force table is set;
 * PGH_ERANGE when the force table has E + F > 13 (the two tables share the
 * kernels' LDS); setting a new force table discards the potential table.
 * Synchronous. */
PGH_API int pgh_build_pot_table(pgh_ctx *c, pgh_f_over_r pot, void *user, float *table_out);

/* The potential table from a device array of 2 * 2^(E+F) floats (P0_0,
 * P1_0, P0_1, ...), on the current force table's bins; the same states and
 * the same E + F <= 13 as pgh_build_pot_table. */
PGH_API int pgh_set_pot_table(pgh_ctx *c, const float *table);

/* Table-force accelerations of ni i-particles from the nj = pgh_set_n
 * j-particles of the j-memory: a_i = sum_j m_j g(s_ij) (r_j - r_i) with
 * s = min((s_max - 2)|r_j - r_i|^2 / rcut^2 + 2, s_max) and
 * g = G0_k + G1_k (s - s_k), k the bin of s (the force procedure of
 * Sec. 3.4.2).  Differences are taken on unscaled positions, which gives the
 * paper's scaled-position result without its final rescale.  phi (or NULL):
 * the potential phi_i = sum_j m_j (P0_k + P1_k (s - s_k)) from the potential
 * table (PGH_ESTATE if none is set).  PGH_ESTATE if no force table is set. */
PGH_API int pgh_calc_table(pgh_ctx *c, int ni, const float *xi, const float *yi, const float *zi,
                           float *ax, float *ay, float *az, float *phi);

/* ---------------------------------------------------------------------- */
/* Interaction lists in one persistent launch (tree / TreePM groups,        */
/* Sec. 5.1).                                                              */
/* ---------------------------------------------------------------------- */

/* One interaction list: i-particles [i_off, i_off + n_i) of the i-arrays
 * against j-particles [j_off, j_off + n_j) of the j-arrays. */
typedef struct pgh_item {
    int i_off, n_i, j_off, n_j;
} pgh_item;

/* Builds an execution plan for n_items lists given in HOST memory: checks
 * every range against ni_total / nj_total, requires the i-ranges to be
 * disjoint (PGH_EINVAL otherwise), cuts groups into wavefront tasks, orders
 * the tasks by decreasing cost and uploads the queue.  A plan is bound to the
 * context and can be launched any number of times; it is freed by
 * pgh_plan_free or pgh_close.  Synchronous. */
PGH_API int pgh_plan_create(pgh_ctx *c, int n_items, const pgh_item *items, int ni_total, int nj_total,
                    pgh_plan **out);
PGH_API int pgh_plan_free(pgh_ctx *c, pgh_plan *p);

/* Where plans (pgh_plan_create, and the plan of each tree walk) get their
 * task list: 1 (default) = the host decides the pairing and the cut of each
 * list's chunks and the device writes the tasks from one compact entry per
 * list or pair; 0 = the host writes every task.  Both give the same tasks;
 * plans whose chunks of 64 would fill less than the device's resident waves
 * are always made on the host. */
PGH_API int pgh_set_plan_expansion(pgh_ctx *c, int on_device);

/* The number of waves the planner cuts the work of later plans (and tree
 * walks) for: groups are cut into chunks of 64, or of 32 or 16 i-particles
 * while fewer tasks than this would result, and long j-lists into parts of
 * an eighth of this count's average share of the work (the schedule of
 * Sec. 5.1's lists; it changes no result beyond FP32 summation order).  0
 * (default) = the resident waves of the batched kernels on the context's
 * device; PGH_EINVAL if negative.  A tuning dimension for callers that
 * time plans (the binding's Context.plan_tuned). */
PGH_API int pgh_set_plan_waves(pgh_ctx *c, int waves);

/* The wave target later plans will be cut for (the setting, or the device's
 * resident waves when it is 0); a negative status on error. */
PGH_API int pgh_get_plan_waves(pgh_ctx *c);

/* Packing of later plans (and tree walks): with on != 0, the rows that an
 * item (in i_off order) leaves empty in its last chunk of 64 are filled with
 * the first i-particles of the next item, as a task of two chunks, each
 * lane over its own item's list, when one wave running the longer list
 * costs fewer lane-iterations than the two apart (the schedule of Sec. 5.1's
 * lists; no result changes beyond FP32 summation order).  Fewer, fuller
 * tasks for streams of groups of about 64 i-particles, such as cell lists.
 * Applies when the plan is cut into chunks of 64; packed plans are made on
 * the host.  Default 0.  A tuning dimension for callers that time plans
 * (the binding's Context.plan_tuned). */
PGH_API int pgh_set_plan_packing(pgh_ctx *c, int on);

/* The packing setting (0 or 1); a negative status on error. */
PGH_API int pgh_get_plan_packing(pgh_ctx *c);

/* Number of interactions sum n_i n_j of a plan (host value, no sync). */
PGH_API long long pgh_plan_interactions(const pgh_plan *p);

/* Newton force of every list of the plan in one launch.  Each item writes
 * ax, ay, az (and phi unless NULL) of its own i-rows; rows in no item are
 * left untouched.  eps2_i: per-i squared softening (> 0) or NULL for
 * pgh_set_eps_to_all.  The persistent workgroups take tasks from a device
 * queue that the launch resets itself, so a captured graph can be replayed. */
PGH_API int pgh_batch_newton(pgh_ctx *c, const pgh_plan *p, const float *xi, const float *yi,
                     const float *zi, const float *eps2_i, const float *xj, const float *yj,
                     const float *zj, const float *mj, float *ax, float *ay, float *az,
                     float *phi);

/* Table force of every list of the plan (the context's table), and the
 * potential from the potential table when phi is not NULL. */
PGH_API int pgh_batch_table(pgh_ctx *c, const pgh_plan *p, const float *xi, const float *yi,
                            const float *zi, const float *xj, const float *yj, const float *zj,
                            const float *mj, float *ax, float *ay, float *az, float *phi);

/* ---------------------------------------------------------------------- */
/* Adjoints of L = sum_i w_i . a_i (derived from Eq. newton_force and the   */
/* interpolation of Sec. 3.4.2; pair terms are recomputed, never stored).   */
/* ---------------------------------------------------------------------- */

/* All-pairs Newton with one shared particle set (i-set = j-set = x, y, z, m,
 * uniform eps2 > 0, else PGH_ERANGE): gradients of L for w = (wx, wy, wz)
 * per particle, both roles of each particle folded into one gather:
 *   gx_k = sum_{l != k} [rho^3 u - 3 rho^5 (u . d) d],  u = m_k w_l - m_l w_k,
 *   gm_k = -sum_{l != k} rho^3 (w_l . d),  d = r_l - r_k,
 *   rho = (|d|^2 + eps2)^{-1/2}.
 * The self pair, whose term is identically zero, is skipped.  The particle
 * records are packed into context scratch (grown on demand, which
 * synchronises).  gx, gy, gz, gm: n outputs (gm may be NULL). */
PGH_API int pgh_newton_allpairs_bwd(pgh_ctx *c, int n, const float *x, const float *y, const float *z,
                            const float *m, float eps2, const float *wx, const float *wy,
                            const float *wz, float *gx, float *gy, float *gz, float *gm);

/* Newton adjoint for separate i- and j-sets (eps2_i per i, > 0; NULL for
 * pgh_set_eps_to_all, which must then be > 0) with T = m_j rho^3 (w_i . d),
 * d = r_j - r_i:
 *   gxi_i = -sum_j m_j [rho^3 w_i - 3 rho^5 (w_i . d) d]
 *   gxj_j =  sum_i m_j [rho^3 w_i - 3 rho^5 (w_i . d) d]
 *   gmj_j =  sum_i rho^3 (w_i . d)
 * Any output triple may be NULL (gxi..: NULL skips the i pass; gxj.. and gmj
 * NULL skip the j pass).  When the two sets are the same particles, each
 * self pair adds opposite terms m rho^3 w to gxi and gxj that cancel only
 * when the caller adds them; pgh_newton_allpairs_bwd avoids that. */
PGH_API int pgh_newton_ij_bwd(pgh_ctx *c, int ni, const float *xi, const float *yi, const float *zi,
                      const float *eps2_i, int nj, const float *xj, const float *yj,
                      const float *zj, const float *mj, const float *wx, const float *wy,
                      const float *wz, float *gxi, float *gyi, float *gzi, float *gxj,
                      float *gyj, float *gzj, float *gmj);

/* Table-force adjoint over a plan (derived from the interpolation of
 * Sec. 3.4.2), with G0 and G1 independent leaves; with g = G0_k + G1_k (s - s_k)
 * and s = c |d|^2 + 2 (g is linear in s inside a bin, dg/ds = G1_k, and 0 on
 * the clamp):
 *   gtable[2k]   = sum over pairs in bin k of m_j (w_i . d)
 *   gtable[2k+1] = sum over pairs in bin k of m_j (s - s_k)(w_i . d)
 *   gmj_j        = sum over pairs with j of g (w_i . d)
 *   g{x,y,z}j_j  = sum over pairs with j of m_j [ g w_i + 2c G1_k (w_i . d) d ]
 *   g{x,y,z}i_i  = - the same sum over the pairs of i
 * gtable: device float[2 * 2^(E+F)] (or NULL), overwritten.  gmj and
 * g{x,y,z}j: device float[nj_total] (or NULL), overwritten; an entry used by
 * several lists accumulates.  g{x,y,z}i: device float[ni_total] (or NULL),
 * overwritten; rows in no list get 0.  Position gradients come in triples
 * (PGH_EINVAL otherwise).  The sums use float atomics, so their order (and
 * last bits) may vary from call to call.  The first call on a plan builds
 * the plan's adjoint task lists (allocates, uploads and waits for the
 * stream); later calls allocate nothing and may be captured in a graph.
 * PGH_ERANGE when the force table has E + F > 13 (the LDS holds the table
 * and its gradient sums). */
PGH_API int pgh_batch_table_bwd(pgh_ctx *c, const pgh_plan *p, const float *xi, const float *yi,
                                const float *zi, const float *xj, const float *yj,
                                const float *zj, const float *mj, const float *wx,
                                const float *wy, const float *wz, float *gtable, float *gmj,
                                float *gxi, float *gyi, float *gzi, float *gxj, float *gyj,
                                float *gzj);

/* pgh_batch_table (no potential) that also writes the i-side moments of the
 * adjoint of L = sum_i w_i . a_i (derived from Sec. 3.4.2: inside a bin the
 * interpolant is linear in s = c |d|^2 + 2, so the derivative of m_j g d
 * with respect to r_i is -m_j (g I + 2c G1_k d d^T)).  For each i-row of an
 * item, mom[k * ni_total + i] holds, for k = 0 .. 6, S_i = sum_j m_j g_ij
 * and the symmetric M_i = sum_j m_j G1_k(ij) d d^T as Mxx, Mxy, Mxz, Myy,
 * Myz, Mzz; rows in no item are left untouched.  mom: device float
 * [7 * ni_total], caller-owned.  With them pgh_batch_table_bwd_moments forms
 * dL/dr_i = -(S_i w_i + 2c M_i w_i) per row instead of evaluating every pair
 * a second time.  One i-particle per lane and the paper's (G0, G1) form
 * whatever the selected variant.  The first call on a plan with split lists
 * allocates the plan's partial moments (and waits); later calls allocate
 * nothing.  PGH_ESTATE without a force table; PGH_ERANGE for one with
 * E + F > 13, as for the adjoint. */
PGH_API int pgh_batch_table_moments(pgh_ctx *c, pgh_plan *p, const float *xi, const float *yi,
                                    const float *zi, const float *xj, const float *yj,
                                    const float *zj, const float *mj, float *ax, float *ay,
                                    float *az, float *mom);

/* pgh_batch_table_bwd with the i-side position gradient formed from the
 * moments that pgh_batch_table_moments wrote for the same plan, positions,
 * masses and table (mom, device float[7 * ni_total]): each i-row of an item
 * gets -(S_i w_i + 2c M_i w_i), rows in no item 0, and the pairs are
 * evaluated once (the j-major pass) instead of twice.  The other gradients
 * and every argument as in pgh_batch_table_bwd; PGH_EINVAL for a NULL mom. */
PGH_API int pgh_batch_table_bwd_moments(pgh_ctx *c, const pgh_plan *p, const float *xi,
                                        const float *yi, const float *zi, const float *xj,
                                        const float *yj, const float *zj, const float *mj,
                                        const float *wx, const float *wy, const float *wz,
                                        const float *mom, float *gtable, float *gmj, float *gxi,
                                        float *gyi, float *gzi, float *gxj, float *gyj,
                                        float *gzj);

/* Removes the self term from raw potentials (Sec. 4.1): phi[i] += m[i] /
 * eps_i for i in [0, n), with eps_i^2 from eps2_i (device, may be NULL: the
 * context's pgh_set_eps_to_all value).  For i-particles that are also
 * j-particles, whose raw potential from pgh_calc_newton contains -m_i/eps_i.
 * Entries with eps_i = 0 are left as they are (the guarded kernel gives the
 * zero-distance pair nothing).  m, phi: device float[n]; phi is updated in
 * place.  Asynchronous on the context stream. */
PGH_API int pgh_correct_self_potential(pgh_ctx *c, int n, const float *m, const float *eps2_i,
                                       float *phi);

/* Chains a table gradient to the node values (derived from the table
 * definition of Sec. 3.4.1, where G1_k = (G0_{k+1} - G0_k) / (s_{k+1} - s_k)
 * for k < K-1 and G1_{K-1} = 0).  gtable: device float[2K], the gradient with
 * respect to the table entries as independent leaves, interleaved like the
 * table (as pgh_batch_table_bwd writes it).  g0: device float[K], receives
 *   g0_k = dL/dG0_k + dL/dG1_{k-1} / (s_k - s_{k-1}) - dL/dG1_k / (s_{k+1} - s_k),
 * each term present where its index exists: the gradient with respect to
 * the node values G0_k = f(r_k)/r_k when the slopes follow them.  (The
 * builder fixes G0_{K-1} = 0; its entry is still written.)  K = 2^(E+F);
 * PGH_ERANGE for E, F outside the table limits.  Asynchronous. */
PGH_API int pgh_table_grad_chain(pgh_ctx *c, int E, int F, const float *gtable, float *g0);

/* ---------------------------------------------------------------------- */
/* Tuning                                                                   */
/* ---------------------------------------------------------------------- */

/* Kernel families with tunable tile shapes. */
enum pgh_family {
    PGH_FAMILY_NEWTON_ALLPAIRS = 0,
    PGH_FAMILY_TABLE_ALLPAIRS = 1,
    PGH_FAMILY_NEWTON_BATCH = 2,
    PGH_FAMILY_TABLE_BATCH = 3
};

/* Number of compiled variants of a family, and a host string describing
 * variant v (e.g. "ki=2 jt=256 u=4"); NULL for an unknown pair. */
PGH_API int pgh_variant_count(int family);
PGH_API const char *pgh_variant_name(int family, int v);

/* Selects variant v of a family for later calls on c (-1: the built-in
 * default). */
PGH_API int pgh_set_variant(pgh_ctx *c, int family, int v);
PGH_API int pgh_get_variant(const pgh_ctx *c, int family);

/* Tunes an all-pairs family (PGH_FAMILY_NEWTON_ALLPAIRS or
 * PGH_FAMILY_TABLE_ALLPAIRS) on the caller's workload: times every variant
 * (one warm-up, then `reps` calls, hipEvents on the context stream) for the
 * ni i-particles xi, yi, zi (device) against the current j-memory (and
 * table), selects the fastest for later calls on c and returns its index
 * (>= 0), or a negative status.  *best_ms (may be NULL) receives its time per
 * call.  Synchronous; allocates and frees temporary outputs.  Persisting
 * the choice across runs is left to the caller (the Python binding keeps a
 * JSON cache keyed by device, family and problem shape). */
PGH_API int pgh_autotune(pgh_ctx *c, int family, int ni, const float *xi, const float *yi,
                         const float *zi, int reps, float *best_ms);

/* Tunes a batched family (PGH_FAMILY_NEWTON_BATCH or PGH_FAMILY_TABLE_BATCH)
 * on plan p of c with the caller's particle arrays (device, as for
 * pgh_batch_newton / pgh_batch_table; the Newton family runs with the
 * context's eps_to_all), the same way as pgh_autotune: returns the fastest
 * variant's index (>= 0) and selects it, or a negative status (PGH_EINVAL
 * for a plan of another context or with no work, PGH_ESTATE without a table
 * for the table family).  Synchronous; allocates temporary outputs. */
PGH_API int pgh_autotune_plan(pgh_ctx *c, int family, const pgh_plan *p, const float *xi,
                              const float *yi, const float *zi, const float *xj,
                              const float *yj, const float *zj, const float *mj, int reps,
                              float *best_ms);

/* ---------------------------------------------------------------------- */
/* Barnes-Hut tree producing the interaction lists of the tree code of      */
/* Sec. 5: groups of i-particles that share one list (Barnes' modification),*/
/* opening parameter theta (the paper uses 0.75), monopole moments or       */
/* quadrupole moments carried by pseudo-particles (Kawai & Makino), all     */
/* built on the device and fed to the batched Newton kernel.                */
/*                                                                          */
/* The paper fixes the method only in outline; this library's definitions: */
/*   - a Morton-ordered octree over the bounding cube of the particles (the */
/*     componentwise minimum and the largest axis range, 21 key bits per    */
/*     axis computed in FP32), particles sorted by (key, input index);      */
/*   - a node splits into its non-empty octants while it holds more than    */
/*     n_leaf particles (at most 21 levels); node size = extent / 2^level;  */
/*   - FP64 moments per node; pseudo-particles: monopole, one of mass M at  */
/*     the centre of mass; quadrupole, three of mass M/3 in the plane of    */
/*     the two largest principal axes of the second moment, which carry    */
/*     the node's mass, zero dipole and its traceless quadrupole;           */
/*   - the i-groups are the nodes that hold at most n_crit particles (or    */
/*     are leaves) and whose parent holds more, in key order;               */
/*   - a group's list: walking breadth first from the root, a node that is  */
/*     the group or one of its ancestors is opened; any other node is       */
/*     accepted when its size l < theta d, d the distance from its centre   */
/*     of mass to the bounding box of the group's particles, and adds its   */
/*     pseudo-particles; an opened leaf adds its particles.  The group's    */
/*     own particles are in its list (so the raw potential includes the     */
/*     self term, as for every other call here).                            */
/* ---------------------------------------------------------------------- */

typedef struct pgh_tree pgh_tree;

/* Creates an empty tree owned by context c (freed with it at pgh_close). */
PGH_API int pgh_tree_create(pgh_ctx *c, pgh_tree **out);
/* Frees the tree's device memory; waits for the context's stream first. */
PGH_API int pgh_tree_free(pgh_ctx *c, pgh_tree *t);

/* Builds the octree of n particles (device arrays, read during the call),
 * their moments, pseudo-particles (quad != 0: three per node) and the
 * i-groups.  Synchronous: waits for the stream at its end.
 * n_leaf in [1, 64], n_crit >= n_leaf (PGH_ERANGE otherwise); positions must
 * be finite (PGH_ERANGE).  Invalidates the lists of an earlier walk. */
PGH_API int pgh_tree_build(pgh_ctx *c, pgh_tree *t, int n, const float *x, const float *y,
                           const float *z, const float *m, int n_leaf, int n_crit, int quad);

/* Walks the tree for every group with opening parameter theta >= 0 and
 * writes the lists (device memory owned by the tree) and a batched plan for
 * them.  record_src != 0 also keeps each entry's source (PGH_TREE_LIST_SRC).
 * The plan is made in compact form on the host (one entry per group or pair
 * of partly filled chunks) and expanded into its tasks on the device; it
 * holds the same tasks as pgh_plan_create would make from the lists.
 * Synchronous.  PGH_ESTATE before a build; PGH_ERANGE when theta is too
 * small for the walk's frontier (more than 4096 nodes to test on one level
 * for one group) or the lists exceed 2^31 - 1 entries. */
PGH_API int pgh_tree_walk(pgh_ctx *c, pgh_tree *t, float theta, int record_src);

/* Newton's force and raw potential on every particle from the lists of the
 * last walk, with the context's eps (pgh_set_eps_to_all): the batched kernel
 * runs over the particles in key order and writes each result to the
 * particle's input position in ax, ay, az, phi (device float[n]; phi may be
 * NULL).  Asynchronous.  PGH_ESTATE before a walk. */
PGH_API int pgh_tree_newton(pgh_ctx *c, pgh_tree *t, float *ax, float *ay, float *az,
                            float *phi);

typedef struct pgh_tree_stats {
    int n, n_nodes, n_leaves, depth, n_groups, max_level_nodes;
    int max_frontier;        /* most nodes one group tested on one level */
    int n_leaf, n_crit, quad, walked;
    float theta;
    float frame[5];          /* lo x, y, z, extent, key scale (2^21 / extent) */
    long long n_entries;     /* list entries of the last walk */
    long long interactions;  /* sum over groups of n_i n_j */
} pgh_tree_stats;

/* Counts of the last build and walk (host struct). */
PGH_API int pgh_tree_stats_get(const pgh_tree *t, pgh_tree_stats *out);

/* The plan of the last walk (owned by the tree; NULL before a walk and after
 * a build), for pgh_batch_newton / pgh_batch_table with the arrays of
 * pgh_tree_get.  Every walk writes its plan into the same object, reusing
 * its device memory, so launches captured in a graph before a walk must be
 * captured again after it. */
PGH_API const pgh_plan *pgh_tree_plan(const pgh_tree *t);

/* Arrays of a tree, for pgh_tree_get: element type and count. */
enum pgh_tree_field {
    PGH_TREE_PERM = 0,        /* int32[n]: input index of the particle of rank r */
    PGH_TREE_KEYS = 1,        /* uint64[n]: sorted keys */
    PGH_TREE_X = 2,           /* float[n]: positions and masses in key order */
    PGH_TREE_Y = 3,
    PGH_TREE_Z = 4,
    PGH_TREE_M = 5,
    PGH_TREE_NODE_BEGIN = 6,  /* int32[n_nodes]: first particle rank */
    PGH_TREE_NODE_COUNT = 7,  /* int32[n_nodes] */
    PGH_TREE_NODE_LEVEL = 8,  /* int32[n_nodes] */
    PGH_TREE_NODE_FIRST_CHILD = 9, /* int32[n_nodes], -1 for a leaf */
    PGH_TREE_NODE_N_CHILD = 10,    /* int32[n_nodes] */
    PGH_TREE_NODE_PARENT = 11,     /* int32[n_nodes], -1 for the root */
    PGH_TREE_MOMENTS = 12,    /* double[n_nodes][10]: M, com x y z, S xx yy zz xy xz yz */
    PGH_TREE_PSEUDO = 13,     /* float[n_nodes * (quad ? 3 : 1)][4]: x, y, z, m */
    PGH_TREE_GROUPS = 14,     /* int32[n_groups]: node of each group, key order */
    PGH_TREE_ITEMS = 15,      /* pgh_item[n_groups]: i-range in key order, j-range */
    PGH_TREE_LIST_X = 16,     /* float[n_entries]: the lists, group after group */
    PGH_TREE_LIST_Y = 17,
    PGH_TREE_LIST_Z = 18,
    PGH_TREE_LIST_M = 19,
    PGH_TREE_LIST_SRC = 20    /* int32[n_entries] (walk with record_src): the
                                 particle rank, or -(1 + q) for pseudo-particle q */
};

/* Copies field `field` into dst (device or host memory) of `capacity`
 * elements; *count (may be NULL) receives the element count.  dst NULL with
 * capacity 0 only reports the count.  Synchronous.
 * PGH_ERANGE if capacity is too small or the field is unknown; PGH_ESTATE
 * for list fields before a walk (or LIST_SRC without record_src). */
PGH_API int pgh_tree_get(pgh_ctx *c, const pgh_tree *t, int field, void *dst,
                         long long capacity, long long *count);

#ifdef __cplusplus
}
#endif
#endif /* PGH_H */
