/*
 * orth_measure.h -- measurement and test helpers of liborth.so (gfx950).
 *
 * Not part of the method's interface (include/orth.h): these entry points
 * time the library's own launches, give Arnoldi drivers a test operator and
 * calibrate the hardware byte counters.  They live in the same shared
 * library and follow the conventions stated at the top of orth.h (device
 * pointers, FP64 column-major matrices, streams passed as void*, ORTH_*
 * return codes).
 */
#ifndef ORTH_MEASURE_H_
#define ORTH_MEASURE_H_

#include <stddef.h>
#include <stdint.h>

#include "orth.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Profiler, test operator and counter probe: measurement helpers, no passage
 * of the paper defines them (the paper measures its own machine's peak and
 * bandwidth with a stream benchmark, Sec. 6.2; these play that role here).
 */

/* Kernel classes timed by the profiler (one class per launch site). */
enum orth_kernel_class {
    ORTH_K_LEAF_GRAM = 0,      /* leaves, sweep-1 Gram [Q_i W_i]^T W_i          */
    ORTH_K_LEAF_CHOL = 1,      /* leaves, per-leaf Cholesky (both sweeps)       */
    ORTH_K_LEAF_CORRECT = 2,   /* leaves, u1 = (w - q P1) N1^-1                 */
    ORTH_K_ROOT_GRAM = 3,      /* reduction level, sweep-1 Gram                 */
    ORTH_K_ROOT_CHOL = 4,      /* reduction level Cholesky and pre-sums         */
    ORTH_K_ROOT_CORRECT = 5,   /* reduction level correction                    */
    ORTH_K_ROOT_FINALIZE = 6,  /* reduction level new columns [P~_i; N~_i]      */
    ORTH_K_LEAF_FINALIZE = 7,  /* leaves: U_i appended, explicit U assembled    */
    ORTH_K_APPLY = 8,          /* orth_apply_Q launches                         */
    ORTH_K_LEAF_GRAM2 = 9,     /* leaves, sweep-2 Gram [Q_i U1_i]^T U1_i        */
    ORTH_K_ROOT_GRAM2 = 10,    /* reduction level, sweep-2 Gram                 */
    ORTH_K_LEAF_FALLBACK = 11, /* mixed form: FP64 redo of the first sweep      */
    ORTH_K_LEAF_HH_PANEL = 12, /* Householder leaves: panel factorisation       */
    ORTH_K_LEAF_HH_SMALL = 13, /* Householder leaves: per-leaf T, Z, E C work   */
    ORTH_K_COUNT = 14
};

/*
 * orth_profile_enable -- on != 0: every later launch of the handle is
 * bracketed by a pair of HIP events recorded on the handle's stream; on = 0
 * stops recording.  Events are host-side objects (no device allocation).
 * Errors: ARG, HIP.
 */
int orth_profile_enable(orth_t *h, int32_t on);

/*
 * orth_profile_select -- restrict the bracketing to the classes whose bit
 * (1u << class) is set in class_mask; the default is every class.  Each
 * event pair adds a short gap on the stream, so a timing run that needs one
 * class's launch durations brackets only that class.
 * Measurement helper, no passage.  Errors: ARG.
 */
int orth_profile_select(orth_t *h, uint32_t class_mask);

/*
 * orth_profile_read -- synchronise the stream, then add the elapsed time of
 * every recorded event pair to per-class totals and clear the record.
 *   total_ms   array of ORTH_K_COUNT doubles: milliseconds per class
 *   launches   array of ORTH_K_COUNT int64: launches per class
 * Totals accumulate across reads until orth_profile_reset.
 * Measurement helper, no passage.  Errors: ARG, HIP.
 */
int orth_profile_read(orth_t *h, double *total_ms, int64_t *launches);

/* orth_profile_reset -- drop pending events and zero the totals
 * (measurement helper, no passage). */
int orth_profile_reset(orth_t *h);

/*
 * orth_laplacian_apply -- test operator for Arnoldi drivers (not part of the
 * method): Y = A X for the Dirichlet finite-difference Laplacian on an
 * nx x ny (nz = 1: 5-point, diagonal 4) or nx x ny x nz (7-point, diagonal
 * 6) grid plus `shift` on the diagonal, unknowns ordered i + nx*j + nx*ny*l.
 * X and Y are n x s (n = nx*ny*nz) column-major, ldx, ldy >= n, must not
 * overlap.  The paper names no operator (no passage); the Laplacians stand
 * in for it.  Errors: ARG, HIP.
 */
int orth_laplacian_apply(const double *d_X, int64_t ldx, double *d_Y,
                         int64_t ldy, int32_t s, int32_t nx, int32_t ny,
                         int32_t nz, double shift, void *stream);

/*
 * orth_probe_copy -- measurement probe: dst[i] = src[i] for i < count
 * doubles.  A plain streaming copy of known size, used to calibrate the
 * hardware byte counters and the achievable HBM bandwidth (the role the
 * stream benchmark plays in Sec. 6.2; no passage defines it).
 * Errors: ARG, HIP.
 */
int orth_probe_copy(const double *d_src, double *d_dst, int64_t count,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ORTH_MEASURE_H_ */
