/*
 * spdba.h -- C ABI of the MI355X (gfx950) sp-DBA transform-domain update.
 *
 * The method (spectral dynamic block activation): the transformed field is
 * split into k-space blocks; each step, every block gets one decision from an
 * activity measure compared with a threshold; active blocks run the model's
 * update core and frozen blocks keep their stored coefficients (Methods,
 * "Spectral dynamic block activation"; Supplementary S2.1).  The transforms are
 * rocFFT calls, untouched.  This library implements the per-step indicator, the
 * compaction of the active-block list, the active-only update, the dense update
 * (Regular mode) and the fused real-space nonlinear term, as HIP kernels.
 *
 * Entry points map onto the paper's integration interface (Supplementary S2.1,
 * "Pseudocode for integration of sp-DBA into a solver"):
 *     spdba_init     -> spdba_plan_create + spdba_plan_bind
 *     spdba_apply    -> spdba_apply (update stage only) / spdba_step (full step)
 *     spdba_destroy  -> spdba_destroy
 *
 * Conventions
 *   - Grids: dims[3] = {nz, ny, nx} slowest..fastest, unused leading axes = 1;
 *     used extents are equal powers of two.  Complex data are interleaved
 *     (re, im), natural FFT order (index i <-> signed wavenumber index
 *     m = i for i < n/2, else i - n), C order, x fastest, full c2c spectrum.
 *   - Blocks: block[3] edges per axis, dividing dims; block ids are C order over
 *     the block grid; block 0 holds k = 0.
 *   - Threshold: with the candidate increment dq(k) = q'(k) - q(k) of the
 *     current step, a(k) = |dq(k)|^2 (FP64; Gray-Scott sums both species),
 *     a_b = max over the block, G = max over the instance; block b is active iff
 *     a_b > fl(fl(tau*tau) * G), or b = 0 with SPDBA_FLAG_PIN_K0 (Supplementary
 *     S6.1 keeps the zero-frequency block active).
 *   - Precision: SPDBA_F64 computes in FP64 throughout.  SPDBA_F32 keeps fields,
 *     transforms and the update in FP32 complex; the k = 0 coefficient of the
 *     real-field operators (CH, GS) is held as an FP64 scalar per species (its
 *     FP32 array slot stays 0), and a(k), a_b, G and all sums are FP64.
 *   - Memory: the caller allocates and owns the state and work buffers (sizes
 *     from spdba_plan_buffer_sizes) and the stream; the library never allocates
 *     device memory.  All device pointers are HIP device pointers.  Host output
 *     arrays are caller-owned.
 *   - Errors: every call returns an spdba_status.  Validation errors return
 *     immediately and leave the plan unchanged.  Device and rocFFT errors return
 *     SPDBA_EDEVICE / SPDBA_EFFT.  A non-finite indicator value raises a device
 *     flag that surfaces as SPDBA_ENONFINITE at the next synchronising call
 *     (spdba_active_mask, spdba_indicator, spdba_worklist, spdba_stats,
 *     spdba_get_spectrum).  Calls are asynchronous on the plan's stream unless
 *     stated.  A plan is not thread-safe; separate plans are independent.
 */
#ifndef SPDBA_H
#define SPDBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t spdba_status;
enum {
    SPDBA_OK = 0,
    SPDBA_EINVAL = 1,       /* invalid argument or descriptor            */
    SPDBA_EUNSUPPORTED = 2, /* valid but unsupported combination         */
    SPDBA_ESTATE = 3,       /* call out of order (e.g. before bind)      */
    SPDBA_EDEVICE = 4,      /* HIP runtime error                         */
    SPDBA_EFFT = 5,         /* rocFFT error                              */
    SPDBA_ENONFINITE = 6    /* a non-finite indicator value was produced */
};

/* Operators (update cores).  op_params per operator (M, kappa, Du, Dv must be
 * non-negative: the implicit denominators are then at least 1):
 *   CAHN_HILLIARD {M, kappa}: c' = (c - dt M k^2 N)/(1 + dt M kappa k^4),
 *       N = F[c^3 - c]; conserved dynamics of Supplementary S3.1 with a
 *       double-well f(c) = (c^2 - 1)^2 / 4, semi-implicit as in S4.2.
 *   GRAY_SCOTT {Du, Dv, F, k}: u' = (u + dt R_u)/(1 + dt Du k^2), likewise v,
 *       R_u = -u v^2 + F (1 - u), R_v = u v^2 - (F + k) v (S4.2 semi-implicit
 *       update with a diagonal diffusion matrix).
 *   NLSE {beta2, gamma, alpha}: symmetric split step (S5.2); each linear half
 *       step E' = exp[(-alpha/2 + i beta2 w^2/2) h/2] E is one sp-DBA update,
 *       the Kerr step E <- E exp(i gamma |E|^2 h) runs in the time domain.
 *       dx is the sample spacing, dt the step h; w = 2 pi m / (n dx).
 *   XPFC {q0, sigma, alpha, omega, u, rho, beta} (alpha > 0, rho beta > 0):
 *       conserved phase-field-crystal density of Supplementary S3.1,
 *       d psi/dt = lap[psi - C2 * psi - (omega/2) psi^2 + (u/3) psi^3], with
 *       C2(k) = exp(-(k - q0)^2/(2 alpha^2)) exp(-sigma^2 q0^2/(2 rho beta)),
 *       advanced by the ETD4 multistep update of S3.2 in backward differences
 *       of the nonlinear transforms H_n .. H_{n-3}, H = F[-(omega/2) psi^2 +
 *       (u/3) psi^3]: psi' = e^z psi + B1 H_n + B2 dH + B3 d2H + B4 d3H, z = L dt,
 *       L = -k^2 (1 - C2), B_l = -k^2 Phi_l (Phi_1 = dt phi_1, Phi_2 = dt phi_2,
 *       Phi_3 = dt (phi_2/2 + phi_3), Phi_4 = dt (phi_2/3 + phi_3 + phi_4)).
 *       The coefficients are formed per mode in FP64 from L (a per-instance
 *       table over (|m_z|, |m_y|, |m_x|) of (n/2 + 1)^ndim FP64 values, filled
 *       on the host; more than 2^28: EUNSUPPORTED) -- phi_4 by its series for
 *       |z| <= 1 and phi_l = 1/l! + z phi_{l+1}, else e^z by scaling and
 *       squaring and the closed forms -- and rounded once.  The four
 *       transforms rotate through slots of the state buffer; the first step
 *       after a field load sets the three older ones to its own.  Requires
 *       SPDBA_FLAG_STATE_INDICATOR (the paper's block energy with
 *       SPDBA_FLAG_BLOCK_ENERGY, or its maximum form) or SPDBA_FLAG_DENSE
 *       (else EUNSUPPORTED); not with SPDBA_FLAG_HALF_SPECTRUM; spdba_apply
 *       takes H_n as its right-hand side and keeps the older ones itself;
 *       spdba_stats reports no energy (NaN).                                 */
enum { SPDBA_OP_CAHN_HILLIARD = 1, SPDBA_OP_GRAY_SCOTT = 2, SPDBA_OP_NLSE = 3, SPDBA_OP_XPFC = 4 };
enum { SPDBA_F32 = 0, SPDBA_F64 = 1 };

enum {
    SPDBA_FLAG_DENSE = 1u << 0,        /* Regular mode (paper mode 0): update every block */
    SPDBA_FLAG_PIN_K0 = 1u << 1,       /* block 0 (k = 0) always active                    */
    SPDBA_FLAG_GRAPH = 1u << 2,        /* spdba_step replays a captured HIP graph          */
    SPDBA_FLAG_TIMING = 1u << 3,       /* record per-stage HIP events (stats.stage_ms)     */
    /* consistency control (Supplementary S1.1, S1.3); the update then walks
     * the block list (launch variant 3 is ignored) */
    SPDBA_FLAG_TRANSITION = 1u << 4,   /* (EUNSUPPORTED for a block edge above 4096 or
                                          2^25 or more blocks over the plan)
                                          non-active face neighbours of active blocks
                                          (periodic block grid) are transition blocks:
                                          q + sigma (q' - q), sigma the product of the
                                          roll-off w(i) = (1 - cos(pi i/(B-1)))/2 over
                                          the faces that border frozen blocks (w = 1
                                          for B = 1), i counted from that face; FP32:
                                          fmaf(fl32(sigma), q' - q, q)                 */
    SPDBA_FLAG_REFRESH = 1u << 5,      /* steps n with (n + 1) % refresh_period == 0
                                          update every block                          */
    SPDBA_FLAG_STATE_INDICATOR = 1u << 7, /* activity measure a(k) = sum over species of
                                          |q(k)|^2 of the state entering the update
                                          (the paper's state-based indicators: block
                                          energy, main text; component RMS amplitude
                                          with any mode above, S4.2; modal spectral
                                          power, S5.3) instead of the increment; k = 0
                                          is left out of a_b and G; no right-hand side
                                          is read                                      */
    SPDBA_FLAG_HALF_SPECTRUM = 1u << 8, /* real fields (CH, GS; ndim 2 or 3) store the
                                          half spectrum of Supplementary S1.2: each row
                                          keeps the columns x = 0 .. nx/2 (n = nz*ny*
                                          (nx/2 + 1) stored modes per species; the
                                          others are conj q(-k)); transforms are rocFFT
                                          real-to-complex / complex-to-real.  Blocks:
                                          those of the columns below nx/2, C order over
                                          (z, y, x) block coordinates, then one block
                                          per (z, y) block row for the column nx/2, C
                                          order over (z, y).  The x block edge must
                                          divide nx/2 and nx/(2 block[2]) + 1 <= 2048;
                                          grids of at most 2^18 points (larger ones:
                                          EUNSUPPORTED, until a device fault seen
                                          on 256^3 runs is explained).  With
                                          SPDBA_FLAG_TRANSITION (x block edge >= 2,
                                          else EUNSUPPORTED) a neighbour in the
                                          omitted half is its conjugate counterpart:
                                          the x-low neighbour of the first x block is
                                          that block at the mirrored rows (-ky, -kz);
                                          the x-high neighbour of the column nx/2 is
                                          the last block below it at the mirrored
                                          rows, which in turn has both the column
                                          nx/2 of its own rows and of the mirrored
                                          rows as x-high neighbours (a face borders
                                          frozen blocks when every block it touches
                                          is frozen; the column nx/2 rolls off with
                                          w = 1).  The update walks the block list
                                          whatever update variant is set             */
    SPDBA_FLAG_BLOCK_ENERGY = 1u << 9, /* with SPDBA_FLAG_STATE_INDICATOR (else EINVAL):
                                          a_b = the block's FP64 sum of a(k), the
                                          block energy of the main text (XPFC) and the
                                          modal spectral power of S5.3, instead of the
                                          block maximum; summed per lane over rows in
                                          order, then over lanes and waves in a fixed
                                          order (bit-reproducible run to run, equal to
                                          other summation orders within rounding).  For
                                          CH and GS the update kernel keeps it, as it
                                          keeps the maximum: the blocks it stores get
                                          their sum (per lane over its slots, then over
                                          lanes and waves in a fixed order), the others
                                          keep theirs, and a step needs no full pass.
                                          Not with SPDBA_FLAG_HALF_SPECTRUM
                                          (EUNSUPPORTED)                               */
    SPDBA_FLAG_DYN_THRESHOLD = 1u << 6 /* tau follows target_ratio: after every
                                          control_interval steps that are not full, the
                                          mean ratio r of non-frozen blocks (over the
                                          step's updates) gives rho = r / target_ratio
                                          and tau <- 2 tau (rho > 2), tau (1 + eta)
                                          (rho > 1 + eta), tau / 2 (rho < 1/2),
                                          tau (1 - eta) (rho < 1 - eta), eta = deadband */
};

typedef struct {
    int32_t ndim;          /* 1, 2 or 3                                           */
    int32_t op;            /* SPDBA_OP_*, equal for every instance of a plan      */
    int64_t dims[3];       /* {nz, ny, nx}, unused leading axes 1                 */
    int32_t block[3];      /* block edges per axis, unused 1                      */
    int32_t dtype;         /* SPDBA_F32 / SPDBA_F64, equal for every instance     */
    uint32_t flags;        /* SPDBA_FLAG_*, equal for every instance              */
    int32_t reserved;      /* must be 0                                           */
    double threshold;      /* tau >= 0                                            */
    double dx;             /* grid spacing (NLSE: sample spacing)                 */
    double dt;             /* time step (NLSE: propagation step h)                */
    double op_params[8];   /* see the operator list above; unused entries 0       */
    /* consistency control.  Step n counts the steps of this instance since
     * its last spdba_set_field / spdba_set_spectrum (which also restore tau):
     * one spdba_step step, or one spdba_apply call (CH, GS) / two calls (NLSE,
     * one per linear half step).  Steps n < full_steps update every block
     * (with or without the flags).  Not with SPDBA_FLAG_DENSE (EUNSUPPORTED). */
    int32_t refresh_period;   /* SPDBA_FLAG_REFRESH: >= 1                          */
    int32_t full_steps;       /* >= 0                                              */
    int32_t control_interval; /* SPDBA_FLAG_DYN_THRESHOLD: >= 1                    */
    int32_t reserved2;        /* must be 0                                         */
    double target_ratio;      /* SPDBA_FLAG_DYN_THRESHOLD: in (0, 1]                */
    double deadband;          /* SPDBA_FLAG_DYN_THRESHOLD: in [0, 1)                */
} spdba_instance_desc;

typedef struct {
    int64_t steps;            /* completed spdba_step steps                         */
    int64_t active_blocks;    /* active blocks of this instance in the last update  */
    int64_t total_blocks;     /* blocks of this instance                            */
    double G;                 /* instance max of a_b in the last update             */
    double mean[2];           /* per-species mean of the current field              */
    double energy;            /* CH: free energy of the state entering the last step
                                 (dx^d sum f(c) + kappa/2 dx^d/N sum k^2 |c_k|^2);
                                 NaN when not available                             */
    double stage_ms[6];       /* SPDBA_FLAG_TIMING: mean over the last (up to 64)
                                 spdba_step steps of the per-stage GPU time in ms:
                                 fft, nonlinear, indicator, compaction, update,
                                 whole step (plan-wide); HIP events on the plan
                                 stream, eager steps only                          */
    int32_t input_preserving_fft; /* 1 if out-of-place inverse transforms keep their
                                     input (probed at bind), 0 if a copy is used    */
    int32_t graph_replay;     /* 1 if spdba_step replays a captured HIP graph       */
    double indicator_kernel_ms; /* SPDBA_FLAG_TIMING: mean indicator kernel time per
                                   step (sum of both half steps for NLSE), from
                                   events recorded at the dispatch's own start and
                                   end (no queue gap); 0 when not available         */
    int64_t transition_blocks;  /* transition blocks of this instance in the last
                                   update (active_blocks counts active ones)        */
    double tau;                 /* threshold in use for the next step              */
    int64_t control_step;       /* consistency-control step counter                */
    double nonfrozen_ratio_mean; /* plans with consistency control: non-frozen
                                    (active + transition) blocks over all updates
                                    since the reset / (blocks x updates); NaN
                                    otherwise                                        */
} spdba_stats_t;

typedef struct spdba_plan_s *spdba_plan;

/* Create a plan for n_inst >= 1 instances advancing independently (a batch).
 * stream: hipStream_t on which all work is enqueued (NULL = default stream).
 * Validates every descriptor: EINVAL for ndim not in {1,2,3}, unequal or
 * non-power-of-two used extents, block edges not dividing dims, tau < 0 or NaN,
 * dt <= 0, dx <= 0, NULL pointers, n_inst < 1; EUNSUPPORTED for mixed op/dtype/
 * flags across instances or unknown op/dtype.  Creates the rocFFT plans (one
 * per distinct grid size).  On success *out receives the plan.  Requires a GPU. */
spdba_status spdba_plan_create(const spdba_instance_desc *inst, int32_t n_inst, void *stream,
                               spdba_plan *out);

/* Host-only audit of the memory layout a plan for these descriptors would
 * use; needs no device and allocates no device memory.  It builds the
 * instance table, the grid groups and the region offsets of the state and
 * work buffers exactly as spdba_plan_create does, then checks every transform
 * the plan executes (its input and output span, from the lengths, strides,
 * distances and batch it is created with) and every device-to-device copy
 * against the buffer region it is run on: the stored spectra, the work
 * spectra W and R, the XPFC history slots, the half layout's real slots.  The
 * half layout's grid-size limit does not apply here.  Not covered: the
 * transforms' own work area (sized by rocFFT at plan creation) and the
 * kernels' indexing.  Returns SPDBA_OK when every span fits, SPDBA_EINVAL
 * with the first violation described in msg (msg_len bytes, NUL-terminated;
 * msg may be NULL), or the status plan creation would return for invalid or
 * unsupported descriptors. */
spdba_status spdba_plan_audit(const spdba_instance_desc *inst, int32_t n_inst, char *msg, size_t msg_len);

/* Device bytes the caller must provide: state (persistent: spectra, FP64 k = 0
 * scalars) and work (scratch: transform buffer, rocFFT work area, indicator,
 * mask, worklist, partial sums).  Both 256-byte aligned sizes. */
spdba_status spdba_plan_buffer_sizes(spdba_plan plan, size_t *state_bytes, size_t *work_bytes);

/* Bind caller-owned device buffers (at least the sizes above, 256-byte aligned).
 * Uploads the instance table and probes the transforms.  The state contents
 * are undefined until spdba_set_field / spdba_set_spectrum. */
spdba_status spdba_plan_bind(spdba_plan plan, void *d_state, void *d_work);

/* Load instance `inst`'s initial field (real space / time domain), device
 * array in the working precision: CH n reals (c); GS 2n reals (u then v);
 * NLSE n complex (E).  Transforms it into the stored state. */
spdba_status spdba_set_field(spdba_plan plan, int32_t inst, const void *d_real);

/* Write instance `inst`'s current field to d_out (same layout as set_field). */
spdba_status spdba_get_field(spdba_plan plan, int32_t inst, void *d_out);

/* Raw access to the stored transform-domain state of `inst` (nspec x n
 * complex, n the stored modes per species; working precision; for NLSE the spectrum that the next update
 * acts on).  For F32 CH/GS the k = 0 coefficients are exchanged in FP64 via
 * h_k0 (host, nspec doubles; NULL in set_spectrum = take slot 0 of d_hat;
 * get_spectrum then writes slot 0 of d_hat as 0).  get_spectrum synchronises. */
spdba_status spdba_set_spectrum(spdba_plan plan, int32_t inst, const void *d_hat, const double *h_k0);
spdba_status spdba_get_spectrum(spdba_plan plan, int32_t inst, void *d_hat, double *h_k0);

/* n_steps full steps of every instance (asynchronous).  Per step for CH/GS:
 * inverse FFT, fused nonlinear term, forward FFT, indicator, compaction, active
 * update (or dense update); NLSE: two linear half steps around the Kerr step,
 * each half step with its own indicator and mask. */
spdba_status spdba_step(spdba_plan plan, int32_t n_steps);

/* Update stage only (the paper's spdba_apply): with right-hand side d_rhs_hat
 * (device, all instances concatenated in instance order, nspec x n complex
 * each; ignored for NLSE, may be NULL) and, for F32 CH/GS, its FP64 k = 0 values
 * h_rhs_k0 (host, n_inst x nspec doubles, NULL = slot 0 of d_rhs_hat). */
spdba_status spdba_apply(spdba_plan plan, const void *d_rhs_hat, const double *h_rhs_k0);

/* Skip set for the learned proposer: d_skip (device, one byte per block over
 * all instances, 1 = frozen without evaluation; caller-owned, must stay valid)
 * is read by every later update; NULL clears it.  Block 0 of an instance with
 * PIN_K0 is never skipped.  Skipped blocks report a_b = 0 and are excluded
 * from G. */
spdba_status spdba_set_skip(spdba_plan plan, const uint8_t *d_skip);

/* Synchronising read-backs of the last update of instance `inst` (host arrays):
 * the mask (n >= blocks; 0 frozen, 1 active, 2 transition), a_b values and G (n >= blocks), and the ordered
 * active-block worklist as instance-local block ids (n >= blocks).  The update
 * itself needs no order (it walks an unordered append list, or the strips);
 * the first spdba_worklist call after an update builds the ascending list
 * from the mask, once. */
spdba_status spdba_active_mask(spdba_plan plan, int32_t inst, uint8_t *host_out, size_t n);
spdba_status spdba_indicator(spdba_plan plan, int32_t inst, double *host_ab, size_t n, double *host_G);
spdba_status spdba_worklist(spdba_plan plan, int32_t inst, uint32_t *host_out, size_t n, int64_t *count);

/* Device views for on-device consumers (the proposer): pointers into the work
 * buffer -- per-block a_b (FP64), per-block mask (u8), per-instance G of the
 * last completed update (FP64) -- valid for the plan's lifetime and rewritten
 * by every update; NULL arguments are skipped. */
spdba_status spdba_device_views(spdba_plan plan, const double **d_ab, const uint8_t **d_mask,
                                const double **d_G, int64_t *total_blocks);

/* Synchronising statistics of instance `inst`. */
spdba_status spdba_stats(spdba_plan plan, int32_t inst, spdba_stats_t *out);

/* Launch geometry (autotuner hook); kernels 0..4 never change results: kernel 0 =
 * indicator (value = waves per workgroup, power of two 1..16), 1 = persistent
 * active update (workgroups per compute unit, 1..64; both the block-list walk
 * and the strip walk), 2 = dense update (threads per workgroup, power of two
 * 64..1024), 3 = active-update variant (0 = persistent walk of the block list
 * appended by a one-pass threshold kernel, 1 = persistent strip walk that
 * applies the threshold itself and
 * skips strips whose largest block value is at or below it, 2 = block-list
 * walk with four entries in flight per workgroup, 3 = block-list walk with
 * one wave per entry, each lane issuing up to four 16-byte slots' loads before
 * its stores, for blocks of at least 64 slots on the full layout; 4 = run walk:
 * x-adjacent active blocks of a block row are cut into aligned pieces of up to
 * 16 blocks and each piece into bands of rows as wide as the piece, one wave
 * per band, for CH and GS on the full layout with equal blocks of 256 or 512
 * slots, no transition blocks and no block-energy sum; default 1).
 * Where a variant does not apply (1 and 2 with the kept state measure, 2 on
 * blocks of more than 256 slots, 3 on blocks of fewer than 64, 4 where its
 * conditions fail) the update runs as variant 0; on the half layout every variant runs that layout's own
 * block-list walk.  4 = strip-walk update (waves per workgroup, power of two
 * 1..16).  5 = placement of the step's forward transform of the nonlinear
 * term (CH and GS on the full layout, else EUNSUPPORTED for 1): 0 out of
 * place into the right-hand-side buffer (default), 1 in place in the
 * transform buffer, which the update then reads as its right-hand side (and
 * spdba_apply fills).  rocFFT runs different kernels for the two, so this
 * knob, unlike the others, changes the transform's FP32/FP64 rounding.
 * Resets the stage-time ring. */
spdba_status spdba_set_launch(spdba_plan plan, int32_t kernel, int32_t value);

/* The update stage of one instance without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): what spdba_apply does for a plan
 * of this one instance -- indicator pass, threshold, compaction, active
 * update, or the dense update -- with the same kernels and results, but with
 * no plan: the scratch memory (instance table, a_b, list, counters, G,
 * partial sums) is a file-scope device array of about 8.9 MB that each GPU
 * the library runs on holds until the process ends.  Its address is taken
 * once per device at the first call.  Every call on a GPU shares that array,
 * so calls that overlap on one GPU race; each call resets what it reads.
 *   desc     : one descriptor; CH or GS on the full layout, no consistency
 *              control, no SPDBA_FLAG_GRAPH (else EUNSUPPORTED); at most 2^18
 *              blocks and 2^17 x 1024 (FP32) / 2^17 x 512 (FP64) complex
 *              values per species (else EUNSUPPORTED); other checks as
 *              spdba_plan_create (EINVAL / EUNSUPPORTED)
 *   d_state  : device, nspec x N complex, the stored spectrum, updated in
 *              place on the active blocks (FP32 CH/GS: slot 0 of each species
 *              is written 0, its value lives in d_k0)
 *   d_rhs_hat: device, nspec x N complex, the right-hand side (slot 0 of an
 *              FP32 CH/GS species is not read)
 *   d_k0, d_rhs_k0: device, FP32 CH/GS only (may be NULL otherwise): the
 *              FP64 k = 0 values per species, d_k0 updated in place
 *   d_mask   : device, one byte per block (C order over the block grid),
 *              written with the mask of this update
 *   stream   : hipStream_t (NULL = default stream); the call is asynchronous
 * A non-finite indicator value is not reported by this entry point (it has
 * no synchronising read-back).  Requires a GPU. */
spdba_status spdba_apply_noalloc(const spdba_instance_desc *desc, void *d_state, const void *d_rhs_hat, double *d_k0,
                                 const double *d_rhs_k0, uint8_t *d_mask, void *stream);

/* Release the plan (host metadata, rocFFT plans, graphs).  NULL-safe. */
spdba_status spdba_destroy(spdba_plan plan);

/* Static description of a status code. */
const char *spdba_status_string(spdba_status s);

#ifdef __cplusplus
}
#endif
#endif /* SPDBA_H */
