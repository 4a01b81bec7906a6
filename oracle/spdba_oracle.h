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
#define OR_OP_XPFC 4 /* conserved XPFC density, ETD4 multistep update (S3.1-S3.2) */

#define OR_FLAG_DENSE 1u  /* Regular mode: every block updated, no indicator */
#define OR_FLAG_PIN_K0 2u /* the block holding k = 0 is always active        */
/* consistency control (Supplementary S1.1, S1.3) */
#define OR_FLAG_TRANSITION 4u /* frozen face neighbours of active blocks take a tapered increment */
#define OR_FLAG_REFRESH 8u    /* every refresh_period-th step activates every block            */
#define OR_FLAG_DYN_TAU 16u   /* the threshold follows a target ratio of non-frozen blocks      */
/* state-amplitude measure (the paper's state-based indicators: block energy
 * in the main text's XPFC section, the component RMS amplitude of S4.2 with
 * "any mode above", the modal spectral power of S5.3): a(k) = sum over
 * species of |q(k)|^2 of the state entering the update, a_b its block
 * maximum; the k = 0 mode is left out (it carries the mean; its block is
 * pinned) */
#define OR_FLAG_STATE 32u
/* half-spectrum layout of a real field (CH, GS; Supplementary S1.2): each
 * row keeps the columns x = 0 .. nx/2 of the forward transform (nx/2 + 1
 * values; the others are q(-k) = conj q(k)).  Blocks: those of the columns
 * below nx/2, C order over (z, y, x) block coordinates, then one block per
 * (z, y) block row holding the column nx/2, C order over (z, y).  The inverse
 * is or_c2r.  Requires nx >= 2 with the x block edge dividing nx/2; not
 * combined with OR_FLAG_TRANSITION. */
#define OR_FLAG_HALF 64u
/* block energy (the main text's XPFC indicator; the modal spectral power of
 * S5.3 for NLSE): with OR_FLAG_STATE, a_b = sum over the block's modes of
 * a(k) = sum over species of |q(k)|^2 (k = 0 left out) instead of the block
 * maximum, accumulated in FP64 in ascending mode order */
#define OR_FLAG_ENERGY 128u

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
    /* consistency control */
    int32_t refresh_period; /* REFRESH: steps n with (n + 1) % refresh_period == 0 are full */
    int32_t full_steps;     /* steps n < full_steps are full (every block active)             */
    int32_t interval;       /* DYN_TAU: controlled steps per control interval (>= 1)          */
    int32_t full_now;       /* apply only: 1 = this update activates every block              */
    double target_ratio;    /* DYN_TAU: target mean ratio of non-frozen blocks, (0, 1]        */
    double deadband;        /* DYN_TAU: relative deadband eta, [0, 1)                          */
    int32_t hist_valid;     /* XPFC steps: 1 = the state carries the three older nonlinear
                               transforms; 0 = they are set to the first step's own      */
    int32_t pad2;
} or_inst;

/* XPFC (Supplementary S3.1-S3.2).  p = {q0, sigma, alpha, omega, u, rho, beta}.
 * Dynamics d psi/dt = lap[psi - C2 * psi - (omega/2) psi^2 + (u/3) psi^3] on a
 * periodic grid; in Fourier space d psi/dt = L psi + (-k^2) H with
 *   L(k)  = -k^2 (1 - C2(k)),
 *   C2(k) = exp(-(k - q0)^2 / (2 alpha^2)) exp(-sigma^2 q0^2 / (2 rho beta)),
 *   H     = F[-(omega/2) psi^2 + (u/3) psi^3].
 * ETD4 (Cox-Matthews multistep, backward differences of H):
 *   psi' = e^z psi + B1 H_n + B2 (H_n - H_{n-1}) + B3 (H_n - 2 H_{n-1} + H_{n-2})
 *          + B4 (H_n - 3 H_{n-1} + 3 H_{n-2} - H_{n-3}),
 *   z = L dt,  B_l = -k^2 Phi_l,  Phi_1 = dt phi_1, Phi_2 = dt phi_2,
 *   Phi_3 = dt (phi_2 / 2 + phi_3),  Phi_4 = dt (phi_2 / 3 + phi_3 + phi_4),
 *   phi_l(z) = sum_{j >= 0} z^j / (l + j)!.
 * Apply: rhs holds the four transforms H_n, H_{n-1}, H_{n-2}, H_{n-3} (4 N
 * complex, newest first).  Steps: the state holds psi-hat followed by the
 * three older transforms H_{n-1}, H_{n-2}, H_{n-3} (4 N complex); with
 * hist_valid = 0 the first step fills them with its own H_0. */

/* e^z and phi_1 .. phi_4 at z (FP64): out = {e^z, phi_1, phi_2, phi_3, phi_4}.
 * |z| <= 1: phi_4 from its series to the term z^14 / 18! (Horner, explicit
 * fma), then phi_l = 1/l! + z phi_{l+1} for l = 3, 2, 1 and e^z = 1 + z phi_1;
 * |z| > 1: e^z from e^w, w = z / 2^s (|w| <= 1, the same series), squared s
 * times, then phi_1 = (e^z - 1)/z, phi_{l+1} = (phi_l - 1/l!)/z. */
void or_etd4_phi(double z, double out[5]);

/* ETD4 coefficients of one mode: out = {e^z, B1, B2, B3, B4} with
 * B_l = mk2 Phi_l (mk2 = -k^2 for XPFC; 1 for a plain ODE dy/dt = L y + N). */
void or_etd4_coef(double z, double dt, double mk2, double out[5]);

/* L(k) of the XPFC operator at k^2 (FP64; the order of operations of the
 * definition above: k = sqrt(k^2), d = k - q0, peak = exp(-(d d) / (2 (alpha
 * alpha))), dw = exp(-((sigma sigma) (q0 q0)) / (2 (rho beta))), C2 = peak dw,
 * L = -k^2 (1 - C2)). */
double or_xpfc_linear(const or_inst *d, double k2);

/* XPFC free energy and mean density of a spectrum psi-hat (FP64):
 * F = dx^d [sum_x (psi^2/2 - omega psi^3/6 + u psi^4/12)
 *           - (1/(2N)) sum_k C2(k) |psi-hat_k|^2]. */
int or_xpfc_energy(const or_inst *d, const double *psihat, double *energy, double *mean);

/* n-D complex FFT in place. sign = -1 forward (unnormalised), +1 inverse (1/N). */
int or_fft(double *a, const int64_t dims[3], int sign);

/* Half spectrum of a real field (nz*ny*nx doubles in, nz*ny*(nx/2+1)
 * complex out): the forward transform's columns 0 .. nx/2.  nx a power of
 * two, at least 2. */
int or_r2c(const int64_t dims[3], const double *real, double *half);

/* Real field of a half spectrum: the omitted columns are filled with
 * q(-k) = conj q(k) of the stored ones, the stored columns 0 and nx/2 are
 * used as given, and the real part of the inverse (1/N) is returned. */
int or_c2r(const int64_t dims[3], const double *half, double *real);

/* sin and cos of x by Cody-Waite reduction and Taylor polynomials. */
void or_sincos(double x, double *s, double *c);

/* Block states (values of mask[]): 0 frozen, 1 active, 2 transition.  With
 * OR_FLAG_TRANSITION a block that is not active but has an active face
 * neighbour (periodic block grid, axes with more than one block) is a
 * transition block; it takes q + sigma (q' - q), sigma being the product over
 * its faces that border frozen blocks of the taper w(i) = (1 - cos(pi i /
 * (B - 1))) / 2 (w = 1 for B = 1), i the mode's index within the block
 * counted from that face (Supplementary S1.1).  wl lists the non-frozen
 * blocks, ascending.  d->full_now = 1 makes every block active. */

/* Kernel-level adaptive (or dense) update of one instance, FP64 arithmetic.
 *   q     : state, nspec x N complex128, updated in place on active blocks
 *           (N stored modes: nz*ny*nx, or nz*ny*(nx/2+1) with OR_FLAG_HALF)
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
 *   state: CH: c-hat (N complex); GS: u-hat, v-hat; NLSE: E(t) (time domain);
 *          with OR_FLAG_HALF the half spectra, real space by or_c2r / or_r2c
 *   masks: optional out [nsteps][mask_per_step][nb]   (NLSE: 2 per step)
 *   diag : optional out [nsteps][4], diagnostics of the state entering the step:
 *          CH {mass, free energy, 0, 0}; GS {mean u, mean v, 0, 0};
 *          NLSE {sum |E|^2, 0, 0, 0}
 *   ab   : optional out [nsteps][mask_per_step][nb] indicator values
 *   active_steps: optional out [nb], number of steps each block was active  */
int or_step_f64(const or_inst *d, int64_t nsteps, double *state, uint8_t *masks,
                double *diag, double *ab, int64_t *active_steps);

/* The same with the step schedule of consistency control (Supplementary
 * S1.3).  Step n (from 0) is full when n < full_steps or, with REFRESH,
 * (n + 1) % refresh_period == 0.  With DYN_TAU, every step that is not full
 * contributes r_n = (non-frozen blocks over the step's updates) / (blocks x
 * updates per step); after `interval` such steps the mean r of the interval,
 * rho = r / target_ratio, sets tau <- 2 tau (rho > 2), tau (1 + eta) (rho >
 * 1 + eta), tau / 2 (rho < 1/2), tau (1 - eta) (rho < 1 - eta), else tau.
 * tau_trace: optional out [nsteps], the tau each step used. */
int or_step_ctl_f64(const or_inst *d, int64_t nsteps, double *state, uint8_t *masks,
                    double *diag, double *ab, int64_t *active_steps, double *tau_trace);

/* The taper w(i), i = 0 .. B-1, of block edge B (FP64; Supplementary S1.1). */
void or_taper(int64_t B, double *w);

/* Free energy and mass of a CH spectrum (FP64).  Half layout: the gradient
 * sum counts the stored columns 1 .. nx/2 - 1 twice (their partners). */
/* The descriptor's check and extents: stored modes per species and blocks
 * (OR_EINVAL for a descriptor the other routines refuse).  The array sizes
 * the routines above assume follow from these. */
int or_sizes(const or_inst *d, int64_t *n_modes, int64_t *n_blocks);

int or_ch_energy(const or_inst *d, const double *chat, double *energy, double *mass);

#endif
