/*
 * spdba_oracle.h -- CPU reference for the sp-DBA transform-domain update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the test suite, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the HIP library.
 *
 * Conventions (all arrays are C order, slowest axis first, x fastest):
 *   - a grid is always described as three extents dims[3] = {nz, ny, nx};
 *     unused leading axes have extent 1 (2-D: {1, n, n}; 1-D: {1, 1, n}).
 *     All used axes must have the same extent n.
 *   - complex data are interleaved (re, im) pairs.
 *   - forward transform  F[q]_k = sum_j q_j exp(-2 pi i j.k / n)  (unnormalised);
 *     inverse transform includes the 1/N factor (N = number of grid points).
 *   - signed wavenumber index m(i) = i for i < n/2, else i - n; k = 2 pi m / (n dx).
 */
#ifndef SPDBA_ORACLE_H
#define SPDBA_ORACLE_H
#include <stdint.h>

#define OR_OP_CH 1   /* conserved (Cahn-Hilliard form) semi-implicit update    */
#define OR_OP_GS 2   /* two-species semi-implicit reaction-diffusion update     */
#define OR_OP_NLSE 3 /* split-step linear half-step (dispersion, attenuation)  */

#define OR_FLAG_DENSE 1u  /* Regular mode: every block updated, no indicator */
#define OR_FLAG_PIN_K0 2u /* the block holding k = 0 is always active        */

/* Errors returned by the oracle (0 = success). */
#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENONFINITE 6

typedef struct {
    int32_t op;       /* OR_OP_* */
    int32_t flags;    /* OR_FLAG_* */
    int64_t dims[3];  /* {nz, ny, nx}, unused = 1, used axes equal */
    int32_t block[3]; /* block edge per axis, divides dims */
    int32_t pad;
    double tau;       /* relative threshold on |dq| (compared squared) */
    double dx;        /* grid spacing (NLSE: sample spacing)             */
    double dt;        /* time step (NLSE: propagation step h)            */
    double p[8];      /* CH {M, kappa}; GS {Du, Dv, F, k}; NLSE {beta2, gamma, alpha} */
} or_inst;

/* n-D complex FFT in place. sign = -1 forward (unnormalised), +1 inverse (1/N). */
int or_fft(double *a, const int64_t dims[3], int sign);

/* sin and cos of x by Cody-Waite reduction and Taylor polynomials. */
void or_sincos(double x, double *s, double *c);

/* Kernel-level adaptive (or dense) update of one instance, FP64 arithmetic.
 *   q     : state, nspec x N complex128, updated in place on active blocks
 *   rhs   : CH: N-hat; GS: R_u-hat then R_v-hat; NLSE: unused (may be NULL)
 *   skip  : optional per-block skip set (proposer); NULL = none
 *   a_b   : out, per-block indicator (0 for skipped / dense)
 *   G     : out, instance global max of a_b
 *   mask  : out, per-block 0/1
 *   wl    : out, ascending active block ids; count: out, their number       */
int or_apply_f64(const or_inst *d, double *q, const double *rhs, const uint8_t *skip,
                 double *a_b, double *G, uint8_t *mask, uint32_t *wl, int64_t *count);

/* Same in FP32 working precision.  For CH and GS the k = 0 coefficient of each
 * species is held in FP64 in k0[] (in/out) with its right-hand side in
 * rhs_k0[]; slot 0 of the float arrays is ignored on input and written 0. */
int or_apply_f32(const or_inst *d, float *q, const float *rhs, double *k0,
                 const double *rhs_k0, const uint8_t *skip, double *a_b, double *G,
                 uint8_t *mask, uint32_t *wl, int64_t *count);

/* Full FP64 time steps of one instance.
 *   state: CH: c-hat (N complex); GS: u-hat, v-hat; NLSE: E(t) (time domain)
 *   masks: optional out [nsteps][mask_per_step][nb]   (NLSE: 2 per step)
 *   diag : optional out [nsteps][4], diagnostics of the state entering the step:
 *          CH {mass, free energy, 0, 0}; GS {mean u, mean v, 0, 0};
 *          NLSE {sum |E|^2, 0, 0, 0}
 *   ab   : optional out [nsteps][mask_per_step][nb] indicator values
 *   active_steps: optional out [nb], number of steps each block was active  */
int or_step_f64(const or_inst *d, int64_t nsteps, double *state, uint8_t *masks,
                double *diag, double *ab, int64_t *active_steps);

/* Free energy and mass of a CH spectrum (FP64). */
int or_ch_energy(const or_inst *d, const double *chat, double *energy, double *mass);

#endif
