/*
 * sp-DBA for multicomponent reaction--cross-diffusion (RCD), Supplementary
 * Section S4: C ABI of libspdba.so, beside include/spdba.h (whose status codes
 * and dtype values it uses).
 *
 * Model (S4.1): du/dt = D lap(u) + R(u) for M real components u_1..u_M on a
 * periodic grid; D is the symmetric circulant cross-diffusion matrix with
 * diagonal d_diag + 2 d_cross and -d_cross for the two periodic neighbours of
 * each component (one off-diagonal entry for M = 2); R is the generalised
 * Lotka--Volterra reaction R_i = u_i (r - a u_i - sum_{j != i} alpha_ij u_j)
 * with alpha_ij = beta + alpha for the periodic neighbours and beta otherwise.
 *
 * Step (S4.2): per component the inverse transform, R(u) in real space, its
 * forward transform, then the semi-implicit update of every stored mode
 *   u'(k) = (I + dt k^2 D)^{-1} [u(k) + dt R(k)],
 * applied in the eigen form of S4.3, D = V diag(lambda) V^T computed once at
 * plan creation (FP64 cyclic Jacobi; V orthogonal since D is symmetric):
 *   u'(k) = V diag(1 / (1 + dt k^2 lambda)) V^T [u(k) + dt R(k)].
 *
 * Activation (S4.2, the component RMS amplitude with "any mode above"): per
 * mode a(k) = sum_m (re^2 + im^2) of the state entering the update in FP64,
 * components in order, k = 0 left out; a_b = block maximum; G = max_b a_b;
 * block b active iff a_b > fl(tau^2 G), or it holds k = 0 and
 * SPDBA_RCD_PIN_K0 is set.  The RMS 1/M and square root cancel in this
 * relative rule.  Active blocks update all M components; frozen blocks keep
 * their coefficients bit for bit.  The update kernel keeps the measure of the
 * blocks it stores (the same FP64 sums of the stored values), so a step after
 * an update reduces G without a pass over the frozen blocks; after a load
 * (set_field, set_spectrum) the next update measures in full.
 *
 * Layout: a spectrum is M arrays of N = dims[0]*dims[1]*dims[2] interleaved
 * complex values (FP32 pairs or FP64 pairs per dtype), component after
 * component, each in natural FFT order, C order over dims (slowest first).
 * Real fields: M arrays of N reals.  Blocks: C order over the block grid.
 *
 * Ownership and errors: the caller owns every device buffer (sized by
 * spdba_rcd_buffer_sizes) and the stream; the plan owns host metadata and its
 * rocFFT plans.  Descriptor errors return SPDBA_EINVAL before any device call;
 * M beyond the kernels' tiles (64 in FP32, 48 in FP64, for both forms of the
 * update) returns SPDBA_EUNSUPPORTED; calls before bind return SPDBA_ESTATE; HIP and rocFFT
 * failures return SPDBA_EDEVICE / SPDBA_EFFT.  Calls are asynchronous on the
 * plan's stream unless stated.  A plan is not thread-safe.
 */
#ifndef SPDBA_RCD_H
#define SPDBA_RCD_H

#include <stddef.h>
#include <stdint.h>

#include "spdba.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SPDBA_RCD_DENSE = 1u << 0,  /* Regular: every block updates, no measure   */
    SPDBA_RCD_PIN_K0 = 1u << 1, /* the block holding k = 0 is always active  */
    SPDBA_RCD_TIMING = 1u << 2, /* HIP events around the stages (stats)       */
    SPDBA_RCD_DIRECT = 1u << 3  /* the coupled update as written in S4.2: per
                                   mode a solve of I + dt k^2 D (SPD) -- a
                                   Cholesky factor in registers to M = 8, one
                                   wave's elimination per mode beyond --
                                   instead of the eigen form of S4.3          */
};

typedef struct {
    int32_t ndim;      /* 1, 2 or 3                                              */
    int32_t M;         /* components, >= 2                                       */
    int64_t dims[3];   /* slowest .. fastest, unused = 1; powers of two          */
    int32_t block[3];  /* block edge per axis (unused = 1), power of two dividing dims */
    int32_t dtype;     /* SPDBA_F32 or SPDBA_F64                                 */
    uint32_t flags;    /* SPDBA_RCD_*                                            */
    double tau;        /* relative threshold, >= 0                               */
    double dt, dx;     /* time step > 0, grid spacing > 0 (k = 2 pi m / (n dx))  */
    double d_diag, d_cross;      /* D (S4.1); d_diag > 0, d_cross >= 0           */
    double alpha, beta, r, a;    /* reaction (S4.1)                              */
} spdba_rcd_desc;

typedef struct {
    int64_t n_blocks;      /* blocks per component                                */
    int64_t active_blocks; /* of the last update                                  */
    double G;              /* of the last update (0 for Regular)                  */
    float stage_ms[4];     /* SPDBA_RCD_TIMING, last step: transforms + reaction, */
                           /* measure pass, G + threshold + compaction, update    */
                           /* (else zeros)                                        */
} spdba_rcd_stats_t;

typedef struct spdba_rcd_s *spdba_rcd_plan;

/* Validate the descriptor, compute the eigen form of D, create the rocFFT
 * plans.  stream: a hipStream_t (NULL = default stream). */
spdba_status spdba_rcd_create(const spdba_rcd_desc *desc, void *stream, spdba_rcd_plan *out);

/* Device bytes the caller provides: state (the M spectra) and work (the
 * right-hand side spectra, transform workspace, block tables). */
spdba_status spdba_rcd_buffer_sizes(spdba_rcd_plan plan, size_t *state_bytes, size_t *work_bytes);

/* Bind caller-owned device buffers (256-byte aligned). */
spdba_status spdba_rcd_bind(spdba_rcd_plan plan, void *d_state, void *d_work);

/* Copy M spectra in or out (device pointers, the layout above). */
spdba_status spdba_rcd_set_spectrum(spdba_rcd_plan plan, const void *d_src);
spdba_status spdba_rcd_get_spectrum(spdba_rcd_plan plan, void *d_dst);

/* Load M real fields (forward transforms) or write them out (inverse
 * transforms of a copy, divided by N). */
spdba_status spdba_rcd_set_field(spdba_rcd_plan plan, const void *d_real);
spdba_status spdba_rcd_get_field(spdba_rcd_plan plan, void *d_real);

/* Update stage only (measure, threshold and compaction, update) with the
 * caller's right-hand side spectra R(k) (device, the layout above). */
spdba_status spdba_rcd_apply(spdba_rcd_plan plan, const void *d_rhs_hat);

/* n_steps full steps (S4.2). */
spdba_status spdba_rcd_step(spdba_rcd_plan plan, int32_t n_steps);

/* Synchronising read-backs of the last update: a_b (n = n_blocks values) and
 * G; the mask (n_blocks bytes, 1 = active) and the active count. */
spdba_status spdba_rcd_indicator(spdba_rcd_plan plan, double *host_ab, size_t n, double *host_G);
spdba_status spdba_rcd_active_mask(spdba_rcd_plan plan, uint8_t *host_mask, size_t n, int64_t *count);

/* Synchronising statistics. */
spdba_status spdba_rcd_stats(spdba_rcd_plan plan, spdba_rcd_stats_t *out);

/* Release the plan.  NULL-safe. */
spdba_status spdba_rcd_destroy(spdba_rcd_plan plan);

/* Host only, no device: the eigen form the plan uses (S4.3) for M components
 * (2 .. 1024): V (M x M, row-major, V[i*M + j] = component i of eigenvector
 * j, orthonormal columns) and lambda (M values) with D = V diag(lambda) V^T,
 * by FP64 cyclic Jacobi rotations on the circulant D of S4.1.  Caller-owned
 * host arrays of M*M and M doubles. */
spdba_status spdba_rcd_eigen(int32_t M, double d_diag, double d_cross, double *V, double *lambda);

#ifdef __cplusplus
}
#endif
#endif /* SPDBA_RCD_H */
