/*
 * grape5.h -- GRAPE-5-compatible host interface over the pgh library: the
 * calls of Sec. 3.6 of arXiv:1203.4037 (g5_open, g5_close, g5_set_eps_to_all,
 * g5_set_n, g5_set_xmj, g5_calculate_force_on_x), for codes written against
 * that library, plus the table setter by function pointer that the paper
 * adds for the arbitrary force shape.
 *
 * Conventions (those of the GRAPE-5 library, not of pgh.h):
 *   - Arrays are HOST memory in double precision; positions and forces are
 *     arrays of 3-vectors (double (*)[3]).  Values are rounded to FP32 for
 *     the device and the results widened back to double.
 *   - One process-wide state on HIP device 0 (select the GPU with
 *     HIP_VISIBLE_DEVICES); not thread-safe.
 *   - Calls are synchronous: g5_calculate_force_on_x returns with the
 *     results in ai and pi.  Each call copies its arrays over PCIe, so the
 *     rate of this interface includes those transfers (pgh.h takes device
 *     arrays and avoids them).
 *   - The GRAPE-5 calls return nothing.  A failure (no GPU, no memory, a
 *     negative count, a call before g5_open) leaves the outputs untouched
 *     and is reported by g5_last_error() (NULL when the last call
 *     succeeded).
 *   - G = 1; the potential is the raw sum, including -m_i/eps of an
 *     i-particle that is also a j-particle (as the paper's library returns
 *     it; Sec. 4.1 corrects it on the caller's side).
 */
#ifndef PGH_GRAPE5_H
#define PGH_GRAPE5_H

#include "pgh.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Opens the state (a pgh context on device 0).  A second call is a no-op. */
PGH_API void g5_open(void);

/* Frees the state and its device memory. */
PGH_API void g5_close(void);

/* Softening length of every i-particle. */
PGH_API void g5_set_eps_to_all(double eps);

/* Number of j-particles the next force calls use (the first nj entries of
 * the j-memory); may be called before those entries are set by g5_set_xmj
 * (it is applied by g5_calculate_force_on_x, which fails if fewer entries
 * have been set). */
PGH_API void g5_set_n(int nj);

/* Stores nj j-particles (positions xj[k][0..2], masses mj[k]) at j-memory
 * entries [adr, adr + nj); the memory grows as needed. */
PGH_API void g5_set_xmj(int adr, int nj, double (*xj)[3], double *mj);

/* Accelerations ai[k][0..2] and potentials pi[k] (pi may be NULL) of the ni
 * i-particles at xi against the first n j-particles set by g5_set_n: the
 * Newtonian force (Eq. newton_force), or, after g5_set_force_table, the
 * table force (Eq. arbitrary_force; pi is then set to 0, the table gives no
 * potential). */
PGH_API void g5_calculate_force_on_x(double (*xi)[3], double (*ai)[3], double *pi, int ni);

/* Not in GRAPE-5 (the paper's addition for the arbitrary force shape):
 * builds the look-up table from h(r) = f(r)/r (called at r = 0 for the
 * first node, where it must return the limit), with E exponent bits, F
 * fraction bits and cutoff rcut (see pgh_build_table), and switches
 * g5_calculate_force_on_x to the table force.  Returns a pgh status. */
PGH_API int g5_set_force_table(int E, int F, double rcut, double (*f_over_r)(double r));

/* Switches g5_calculate_force_on_x back to the Newtonian force. */
PGH_API void g5_use_newton(void);

/* Description of the last failure of a g5_ call, or NULL. */
PGH_API const char *g5_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PGH_GRAPE5_H */
