/*
 * sp-DBA for multimode digital backpropagation (DBP), Supplementary Section
 * S5: C ABI of libspdba.so, beside include/spdba.h (whose status codes and
 * dtype values it uses).
 *
 * Model (S5.1): dE/dz = (D + N) E for M coupled modes on a periodic time
 * window T of n samples; D = -alpha/2 I - i beta2/2 d^2/dt^2 I + i K with the
 * constant Hermitian coupling K (caller-supplied); N = i gamma 8/9
 * (sum_m |E_m|^2) I, the Manakov-averaged Kerr rotation.  Back-propagation
 * runs the same model with reversed parameters (-alpha, -beta2, -gamma, -K).
 *
 * Step (S5.2): symmetric split step -- a linear half-step on the spectra, the
 * inverse transforms, the Kerr rotation E_m <- E_m exp(i gamma 8/9 P dz) with
 * P = sum_m |E_m|^2 at the start of the step, the forward transforms, a linear
 * half-step.  The linear half-step of the paper, U_c(dz/4) h(omega) U_c(dz/4)
 * with the scalar h(omega) = exp[(-alpha/2 + i beta2/2 omega^2) dz/2] and
 * U_c(delta) = exp(i delta K), is applied per frequency bin as
 * h(omega) W E(omega) with W = exp(i dz/2 K) (the scalar commutes); W is
 * computed once at plan creation in FP64 (scaling and squaring of the Taylor
 * series) and rounded once to the kernel's precision.
 * omega = 2 pi m / T for the signed bin index m (numpy's FFT order).
 *
 * Activation (S5.3, the total modal spectral power): a(omega) = sum_m
 * (re^2 + im^2) of the spectra entering the half-step, FP64, modes in order,
 * omega = 0 left out; a_b = block maximum; G = max_b a_b; block b active iff
 * a_b > fl(tau^2 G) or it holds omega = 0 and SPDBA_MDBP_PIN_K0 is set.  A
 * relative threshold is scale-free, so the attenuation rescaling of S5.3 is
 * implied.  Active blocks update all M modes; frozen blocks keep theirs.  The
 * Kerr step changes every bin, so every half-step measures in full.
 *
 * Layout: M arrays of n interleaved complex values (FP32 or FP64 pairs), mode
 * after mode; spectra in FFT order; time fields with t = (j - n/2) T/n.
 * Errors as in spdba_rcd.h; M beyond 64 (FP32) or 32 (FP64) returns
 * SPDBA_EUNSUPPORTED.
 */
#ifndef SPDBA_MDBP_H
#define SPDBA_MDBP_H

#include <stddef.h>
#include <stdint.h>

#include "spdba.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SPDBA_MDBP_DENSE = 1u << 0,  /* Regular: every block updates, no measure   */
    SPDBA_MDBP_PIN_K0 = 1u << 1, /* the block holding omega = 0 is always active */
    SPDBA_MDBP_TIMING = 1u << 2, /* HIP events around the stages (stats)       */
    SPDBA_MDBP_GRAPH = 1u << 3   /* spdba_mdbp_step replays one captured step as
                                    a HIP graph (captured on the first call; the
                                    plan's stream must not be the legacy default
                                    stream); not with SPDBA_MDBP_TIMING
                                    (EUNSUPPORTED)                             */
};

typedef struct {
    int32_t M;        /* modes, >= 1                                              */
    int32_t block;    /* frequency bins per block, power of two dividing n        */
    int64_t n;        /* samples, power of two, >= 16                             */
    int32_t dtype;    /* SPDBA_F32 or SPDBA_F64                                   */
    uint32_t flags;   /* SPDBA_MDBP_*                                             */
    double tau;       /* relative threshold, >= 0                                 */
    double T;         /* time window > 0                                          */
    double dz;        /* step > 0                                                 */
    double alpha, beta2, gamma;
} spdba_mdbp_desc;

typedef struct {
    int64_t n_blocks;
    int64_t active_blocks; /* of the last half-step                                */
    double G;              /* of the last half-step (0 for Regular)                */
    float stage_ms[4];     /* SPDBA_MDBP_TIMING, last step: linear half-steps      */
                           /* (measure, compaction and update, both halves),       */
                           /* transforms, Kerr, 0                                  */
} spdba_mdbp_stats_t;

typedef struct spdba_mdbp_s *spdba_mdbp_plan;

/* Validate, compute W = exp(i dz/2 K) from the host K (M x M complex,
 * row-major interleaved FP64; Hermitian within 1e-12 relative, else EINVAL),
 * create the rocFFT plans. stream: a hipStream_t (NULL = default). */
spdba_status spdba_mdbp_create(const spdba_mdbp_desc *desc, const double *K, void *stream,
                               spdba_mdbp_plan *out);
spdba_status spdba_mdbp_buffer_sizes(spdba_mdbp_plan plan, size_t *state_bytes, size_t *work_bytes);
spdba_status spdba_mdbp_bind(spdba_mdbp_plan plan, void *d_state, void *d_work);

/* Spectra (device, the layout above) in or out. */
spdba_status spdba_mdbp_set_spectrum(spdba_mdbp_plan plan, const void *d_src);
spdba_status spdba_mdbp_get_spectrum(spdba_mdbp_plan plan, void *d_dst);
/* Time-domain fields in (forward transforms) or out (inverse, divided by n). */
spdba_status spdba_mdbp_set_field(spdba_mdbp_plan plan, const void *d_time);
spdba_status spdba_mdbp_get_field(spdba_mdbp_plan plan, void *d_time);

/* One linear half-step (measure, threshold and compaction, update). */
spdba_status spdba_mdbp_apply(spdba_mdbp_plan plan);
/* n_steps symmetric split steps. */
spdba_status spdba_mdbp_step(spdba_mdbp_plan plan, int32_t n_steps);

/* Synchronising read-backs of the last half-step. */
spdba_status spdba_mdbp_indicator(spdba_mdbp_plan plan, double *host_ab, size_t n, double *host_G);
spdba_status spdba_mdbp_active_mask(spdba_mdbp_plan plan, uint8_t *host_mask, size_t n, int64_t *count);
spdba_status spdba_mdbp_stats(spdba_mdbp_plan plan, spdba_mdbp_stats_t *out);
spdba_status spdba_mdbp_destroy(spdba_mdbp_plan plan);

/* Host only, no device: W = exp(i delta K) for the host K (M x M complex,
 * row-major interleaved FP64) into the host array out (same layout). */
spdba_status spdba_mdbp_coupling(int32_t M, const double *K, double delta, double *out);

#ifdef __cplusplus
}
#endif
#endif /* SPDBA_MDBP_H */
