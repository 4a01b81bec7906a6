/*
 * spdba_oracle.c -- plain, slow CPU reference for the sp-DBA hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  Never linked into or called by the library.
 *
 * What it computes, and where the paper defines it:
 *   - Blockwise activation (Methods, "Spectral dynamic block activation"): the
 *     transformed field is split into blocks; each block gets one decision from
 *     an activity measure compared with a threshold; active blocks run the model
 *     update, frozen blocks keep their stored coefficients.
 *   - The activity measure used here is the squared size of the candidate
 *     increment, a(k) = |q'(k) - q(k)|^2, its block maximum a_b and the instance
 *     maximum G; a block is active when a_b > tau^2 G.  The paper leaves the
 *     measure application-specific (block energy, RMS amplitude, spectral power);
 *     this increment form and the relative threshold are the workload's choice.
 *   - The zero-frequency block is kept active (S6.1) when PIN_K0 is set.
 *   - Update cores:
 *       CH   : conserved dynamics d c/dt = M lap(f'(c) - kappa lap c) (S3.1 form),
 *              semi-implicit: c' = (c - dt M k^2 N) / (1 + dt M kappa k^4),
 *              N = F[c^3 - c].
 *       GS   : semi-implicit reaction-diffusion update (S4.2) with a diagonal
 *              diffusion matrix: u' = (u + dt R_u)/(1 + dt Du k^2), same for v.
 *       NLSE : linear half-step of the symmetric split-step method (S5.2),
 *              E' = exp[(-alpha/2 + i beta2 w^2 / 2) h/2] E.
 *   - Rounding order is pinned so that an implementation in the same working
 *     precision reproduces every bit: coefficients are formed in FP64 from the
 *     exact integer m^2, rounded once to the working precision, and the
 *     candidate is fma(-s, N, q) * a (CH), fma(dt, R, q) * a (GS),
 *     (Hr E_r - Hi E_i, Hr E_i + Hi E_r) with one fma each (NLSE).  The
 *     increment is squared in FP64 without contraction.
 *
 * Build with -ffp-contract=off: every fused multiply-add below is explicit.
 */
#include "spdba_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------------ */
/* geometry                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n[3];   /* extents nz, ny, nx */
    int64_t b[3];   /* block edges        */
    int64_t nb3[3]; /* blocks per axis    */
    int64_t nb;     /* number of blocks   */
    int64_t N;      /* number of stored modes per species */
    int64_t ext;    /* common extent of the used axes */
    int nspec;      /* species per mode   */
    /* half-spectrum layout (real fields, Supplementary S1.2): x keeps the
     * columns 0 .. nx/2 of each row; the blocks of the columns below nx/2 come
     * first in C order over (z, y, x) block coordinates, then one block per
     * (z, y) block row for the column nx/2.  Full layout: xs = nx, no such
     * blocks. */
    int half;
    int64_t xs;     /* stored x extent (row length) */
    int64_t nbxm;   /* blocks along x below the column nx/2 */
    int64_t nbm;    /* blocks of those columns */
    int64_t Nreal;  /* grid points per species */
} geom_t;

static int make_geom(const or_inst *d, geom_t *g) {
    int64_t ext = 0;
    if (d->op != OR_OP_CH && d->op != OR_OP_GS && d->op != OR_OP_NLSE && d->op != OR_OP_XPFC) return OR_EINVAL;
    g->N = 1;
    g->nb = 1;
    for (int a = 0; a < 3; ++a) {
        int64_t n = d->dims[a];
        int64_t b = d->block[a];
        if (n < 1 || b < 1 || n % b != 0) return OR_EINVAL;
        if (n > 1) {
            if (ext == 0) ext = n;
            else if (ext != n) return OR_EINVAL;
        }
        g->n[a] = n;
        g->b[a] = b;
        g->nb3[a] = n / b;
        g->N *= n;
        g->nb *= n / b;
    }
    g->ext = ext ? ext : 1;
    g->nspec = (d->op == OR_OP_GS) ? 2 : 1;
    if (!(d->tau >= 0.0) || !(d->dt > 0.0) || !(d->dx > 0.0)) return OR_EINVAL;
    /* the block energy sums the state measure */
    if ((d->flags & OR_FLAG_ENERGY) && !(d->flags & OR_FLAG_STATE)) return OR_EINVAL;
    g->half = (d->flags & OR_FLAG_HALF) != 0;
    g->Nreal = g->N;
    g->xs = g->n[2];
    g->nbxm = g->nb3[2];
    g->nbm = g->nb;
    if (g->half) {
        /* real fields only */
        if (d->op == OR_OP_NLSE || d->op == OR_OP_XPFC) return OR_EINVAL;
        if (g->n[2] < 2 || (g->n[2] / 2) % g->b[2] != 0) return OR_EINVAL;
        /* transition states: X_0 must hold the columns 0 and 1 (see half_face) */
        if ((d->flags & OR_FLAG_TRANSITION) && g->b[2] < 2) return OR_EINVAL;
        g->xs = g->n[2] / 2 + 1;
        g->nbxm = g->n[2] / (2 * g->b[2]);
        g->nbm = g->nb3[0] * g->nb3[1] * g->nbxm;
        g->nb = g->nbm + g->nb3[0] * g->nb3[1];
        g->N = g->n[0] * g->n[1] * g->xs;
    }
    return OR_OK;
}

/* grid indices of stored mode i (rows of xs columns) */
static inline void mode_idx(const geom_t *g, int64_t i, int64_t *iz, int64_t *iy, int64_t *ix) {
    *ix = i % g->xs;
    *iy = (i / g->xs) % g->n[1];
    *iz = i / (g->xs * g->n[1]);
}

/* m = i for i < n/2, else i - n (the Nyquist index maps to -n/2; n = 1 gives 0) */
static inline int64_t signed_index(int64_t i, int64_t n) { return (2 * i < n) ? i : i - n; }

/* block id of mode (iz, iy, ix): C order over the block grid; in the half
 * layout the column nx/2 forms one block per (z, y) block row, numbered after
 * all others */
static inline int64_t block_of(const geom_t *g, int64_t iz, int64_t iy, int64_t ix) {
    const int64_t row = (iz / g->b[0]) * g->nb3[1] + iy / g->b[1];
    if (g->half && 2 * ix == g->n[2]) return g->nbm + row;
    return row * g->nbxm + ix / g->b[2];
}

/* k^2 = (2 pi / (n dx))^2 * (mz^2 + my^2 + mx^2), the integer sum exact */
static inline double kk_base(const geom_t *g, double dx) {
    double K = TWO_PI / ((double)g->ext * dx);
    return K * K;
}

static inline int64_t m2_of(const geom_t *g, int64_t iz, int64_t iy, int64_t ix) {
    int64_t mz = signed_index(iz, g->n[0]);
    int64_t my = signed_index(iy, g->n[1]);
    int64_t mx = signed_index(ix, g->n[2]);
    return mz * mz + my * my + mx * mx;
}

/* ------------------------------------------------------------------------ */
/* FFT: iterative radix-2 (Cooley-Tukey) on each line, twiddles per index   */
/* ------------------------------------------------------------------------ */

static void fft_line(double *a, int64_t n, int sign, const double *tw) {
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < n; ++i) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double tr = a[2 * i], ti = a[2 * i + 1];
            a[2 * i] = a[2 * j];
            a[2 * i + 1] = a[2 * j + 1];
            a[2 * j] = tr;
            a[2 * j + 1] = ti;
        }
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len >> 1, stride = n / len;
        for (int64_t s = 0; s < n; s += len) {
            for (int64_t k = 0; k < half; ++k) {
                double wr = tw[2 * k * stride];
                double wi = (double)sign * tw[2 * k * stride + 1];
                double *u = a + 2 * (s + k), *v = a + 2 * (s + k + half);
                double vr = v[0] * wr - v[1] * wi;
                double vi = v[0] * wi + v[1] * wr;
                v[0] = u[0] - vr;
                v[1] = u[1] - vi;
                u[0] = u[0] + vr;
                u[1] = u[1] + vi;
            }
        }
    }
}

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

int or_fft(double *a, const int64_t dims[3], int sign) {
    int64_t N = dims[0] * dims[1] * dims[2];
    for (int ax = 0; ax < 3; ++ax)
        if (!is_pow2(dims[ax])) return OR_EINVAL;
    for (int ax = 0; ax < 3; ++ax) {
        int64_t n = dims[ax];
        if (n == 1) continue;
        /* element stride along this axis, and the number of lines */
        int64_t stride = 1;
        for (int b = ax + 1; b < 3; ++b) stride *= dims[b];
        int64_t lines = N / n;
        double *tw = (double *)malloc(sizeof(double) * (size_t)n);
        for (int64_t j = 0; j < n / 2; ++j) {
            double ang = TWO_PI * (double)j / (double)n;
            tw[2 * j] = cos(ang);
            tw[2 * j + 1] = sin(ang);
        }
#pragma omp parallel
        {
            double *buf = (double *)malloc(sizeof(double) * 2 * (size_t)n);
#pragma omp for schedule(static)
            for (int64_t l = 0; l < lines; ++l) {
                /* line l: inner index (below this axis) and outer index (above) */
                int64_t inner = l % stride, outer = l / stride;
                double *base = a + 2 * (outer * n * stride + inner);
                for (int64_t i = 0; i < n; ++i) {
                    buf[2 * i] = base[2 * i * stride];
                    buf[2 * i + 1] = base[2 * i * stride + 1];
                }
                fft_line(buf, n, sign, tw);
                for (int64_t i = 0; i < n; ++i) {
                    base[2 * i * stride] = buf[2 * i];
                    base[2 * i * stride + 1] = buf[2 * i + 1];
                }
            }
            free(buf);
        }
        free(tw);
    }
    if (sign > 0) {
        double inv = 1.0 / (double)N;
        for (int64_t i = 0; i < 2 * N; ++i) a[i] *= inv;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* sin/cos: Cody-Waite reduction by pi/2 in three parts, then Taylor series */
/* of sin and cos on |r| <= pi/4 evaluated by Horner's rule with fma.       */
/* ------------------------------------------------------------------------ */

#define PIO2_1 1.57079632673412561417e+00  /* first 33 bits of pi/2  */
#define PIO2_2 6.07710050630396597660e-11  /* next 33 bits           */
#define PIO2_3 2.02226624879595063154e-21  /* pi/2 - PIO2_1 - PIO2_2 */
#define TWO_OVER_PI 6.36619772367581382433e-01

void or_sincos(double x, double *s, double *c) {
    double q = nearbyint(x * TWO_OVER_PI);
    double r = fma(-q, PIO2_1, x);
    r = fma(-q, PIO2_2, r);
    r = fma(-q, PIO2_3, r);
    double r2 = r * r;
    /* sin r = r + r^3 (-1/3! + r^2/5! - ... + r^14/17!) */
    double ps = 1.0 / 355687428096000.0;         /*  1/17! */
    ps = fma(ps, r2, -1.0 / 1307674368000.0);    /* -1/15! */
    ps = fma(ps, r2, 1.0 / 6227020800.0);        /*  1/13! */
    ps = fma(ps, r2, -1.0 / 39916800.0);         /* -1/11! */
    ps = fma(ps, r2, 1.0 / 362880.0);            /*  1/9!  */
    ps = fma(ps, r2, -1.0 / 5040.0);             /* -1/7!  */
    ps = fma(ps, r2, 1.0 / 120.0);               /*  1/5!  */
    ps = fma(ps, r2, -1.0 / 6.0);                /* -1/3!  */
    double sn = fma(r * r2, ps, r);
    /* cos r = 1 + r^2 (-1/2! + r^2/4! - ... - r^16/18!) */
    double pc = -1.0 / 6402373705728000.0;       /* -1/18! */
    pc = fma(pc, r2, 1.0 / 20922789888000.0);    /*  1/16! */
    pc = fma(pc, r2, -1.0 / 87178291200.0);      /* -1/14! */
    pc = fma(pc, r2, 1.0 / 479001600.0);         /*  1/12! */
    pc = fma(pc, r2, -1.0 / 3628800.0);          /* -1/10! */
    pc = fma(pc, r2, 1.0 / 40320.0);             /*  1/8!  */
    pc = fma(pc, r2, -1.0 / 720.0);              /* -1/6!  */
    pc = fma(pc, r2, 1.0 / 24.0);                /*  1/4!  */
    pc = fma(pc, r2, -0.5);                      /* -1/2!  */
    double cs = fma(r2, pc, 1.0);
    long qi = (long)q & 3;
    switch (qi) {
        case 0: *s = sn; *c = cs; break;
        case 1: *s = cs; *c = -sn; break;
        case 2: *s = -sn; *c = -cs; break;
        default: *s = -cs; *c = sn; break;
    }
}

/* ------------------------------------------------------------------------ */
/* Per-operator constants, formed once per instance in FP64                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    double K2;        /* (2 pi / (n dx))^2 */
    /* CH */
    double dtM, dtMk; /* dt*M, dt*M*kappa */
    /* GS */
    double dt, dtDu, dtDv;
    /* NLSE: theta = cth * m^2, amplitude A */
    double cth, A;
} consts_t;

static void make_consts(const or_inst *d, const geom_t *g, consts_t *c) {
    memset(c, 0, sizeof(*c));
    c->K2 = kk_base(g, d->dx);
    c->dt = d->dt;
    if (d->op == OR_OP_CH) {
        c->dtM = d->dt * d->p[0];
        c->dtMk = c->dtM * d->p[1];
    } else if (d->op == OR_OP_GS) {
        c->dtDu = d->dt * d->p[0];
        c->dtDv = d->dt * d->p[1];
    } else {
        /* H = exp[(-alpha/2 + i beta2 w^2/2) h/2]: phase beta2 w^2 h / 4 */
        c->cth = ((d->p[0] * d->dt) * 0.25) * c->K2;
        c->A = exp(-(d->p[2] * d->dt) * 0.25);
    }
}

/* CH coefficients at m^2: s = dt M k^2, a = 1/(1 + dt M kappa k^4) */
static inline void ch_coef(const consts_t *c, int64_t m2, double *s, double *a) {
    double k2 = c->K2 * (double)m2;
    *s = c->dtM * k2;
    *a = 1.0 / (1.0 + c->dtMk * (k2 * k2));
}

/* GS coefficients at m^2: a_u = 1/(1 + dt Du k^2), a_v likewise */
static inline void gs_coef(const consts_t *c, int64_t m2, double *au, double *av) {
    double k2 = c->K2 * (double)m2;
    *au = 1.0 / (1.0 + c->dtDu * k2);
    *av = 1.0 / (1.0 + c->dtDv * k2);
}

/* NLSE half-step factor H at m^2 */
static inline void nlse_coef(const consts_t *c, int64_t m2, double *hr, double *hi) {
    double th = c->cth * (double)m2;
    double sn, cs;
    or_sincos(th, &sn, &cs);
    *hr = c->A * cs;
    *hi = c->A * sn;
}


/* ------------------------------------------------------------------------ */
/* XPFC: linear operator and ETD4 coefficients (Supplementary S3.1-S3.2)   */
/* ------------------------------------------------------------------------ */

/* 1/n! rounded once (n! is exact in double for n <= 18) */
static double inv_fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return 1.0 / f;
}

/* phi_4(w) by its series to the term w^14/18!, then phi_3, phi_2, phi_1 and
 * e^w by phi_l = 1/l! + w phi_{l+1}, e^w = 1 + w phi_1 (|w| <= 1) */
static void phi_series(double w, double out[5]) {
    double p4 = inv_fact(18);
    for (int j = 13; j >= 0; --j) p4 = fma(p4, w, inv_fact(4 + j));
    const double p3 = fma(w, p4, inv_fact(3));
    const double p2 = fma(w, p3, inv_fact(2));
    const double p1 = fma(w, p2, 1.0);
    out[0] = fma(w, p1, 1.0);
    out[1] = p1;
    out[2] = p2;
    out[3] = p3;
    out[4] = p4;
}

void or_etd4_phi(double z, double out[5]) {
    if (fabs(z) <= 1.0) {
        phi_series(z, out);
        return;
    }
    int s = 0;
    double w = z;
    while (fabs(w) > 1.0) {
        w *= 0.5;
        ++s;
    }
    double t[5];
    phi_series(w, t);
    double e = t[0];
    for (int i = 0; i < s; ++i) e = e * e;
    out[0] = e;
    out[1] = (e - 1.0) / z;
    out[2] = (out[1] - 1.0) / z;
    out[3] = (out[2] - inv_fact(2)) / z;
    out[4] = (out[3] - inv_fact(3)) / z;
}

void or_etd4_coef(double z, double dt, double mk2, double out[5]) {
    double ph[5];
    or_etd4_phi(z, ph);
    const double P1 = dt * ph[1];
    const double P2 = dt * ph[2];
    const double P3 = dt * (0.5 * ph[2] + ph[3]);
    const double P4 = dt * ((ph[2] / 3.0 + ph[3]) + ph[4]);
    out[0] = ph[0];
    out[1] = mk2 * P1;
    out[2] = mk2 * P2;
    out[3] = mk2 * P3;
    out[4] = mk2 * P4;
}

double or_xpfc_linear(const or_inst *d, double k2) {
    const double q0 = d->p[0], sg = d->p[1], al = d->p[2], rho = d->p[5], be = d->p[6];
    const double k = sqrt(k2);
    const double dk = k - q0;
    const double peak = exp(-(dk * dk) / (2.0 * (al * al)));
    const double dw = exp(-((sg * sg) * (q0 * q0)) / (2.0 * (rho * be)));
    const double c2 = peak * dw;
    return -k2 * (1.0 - c2);
}

/* XPFC candidate of one mode in FP64: psi' from psi and the four transforms
 * h[0..3] (newest first), in the order of the ETD4 formula */
static inline void xpfc_cand64(const double co[5], double q, const double h[4], double *out) {
    const double d1 = h[0] - h[1];
    const double d2 = fma(-2.0, h[1], h[0]) + h[2];
    const double d3 = fma(3.0, h[2], fma(-3.0, h[1], h[0])) - h[3];
    double acc = co[0] * q;
    acc = fma(co[1], h[0], acc);
    acc = fma(co[2], d1, acc);
    acc = fma(co[3], d2, acc);
    acc = fma(co[4], d3, acc);
    *out = acc;
}

static inline void xpfc_cand32(const float co[5], float q, const float h[4], float *out) {
    const float d1 = h[0] - h[1];
    const float d2 = fmaf(-2.0f, h[1], h[0]) + h[2];
    const float d3 = fmaf(3.0f, h[2], fmaf(-3.0f, h[1], h[0])) - h[3];
    float acc = co[0] * q;
    acc = fmaf(co[1], h[0], acc);
    acc = fmaf(co[2], d1, acc);
    acc = fmaf(co[3], d2, acc);
    acc = fmaf(co[4], d3, acc);
    *out = acc;
}

/* coefficients {e^z, B1..B4} of the mode with integer |m|^2 */
static inline void xpfc_coef(const or_inst *d, const consts_t *c, int64_t m2, double co[5]) {
    const double k2 = c->K2 * (double)m2;
    const double z = or_xpfc_linear(d, k2) * d->dt;
    or_etd4_coef(z, d->dt, -k2, co);
}

/* ------------------------------------------------------------------------ */
/* Kernel-level apply: candidate for all modes, indicator, mask, update     */
/* ------------------------------------------------------------------------ */

/* squared increment, FP64, no contraction */
static inline double sq2(double dr, double di) { return dr * dr + di * di; }

/* ------------------------------------------------------------------------ */
/* consistency control: block states and transition weights (S1.1)          */
/* ------------------------------------------------------------------------ */

#define OR_PI 3.141592653589793238462643383279

void or_taper(int64_t B, double *w) {
    if (B <= 1) {
        w[0] = 1.0;
        return;
    }
    for (int64_t i = 0; i < B; ++i) {
        double sn, cs;
        or_sincos((OR_PI * (double)i) / (double)(B - 1), &sn, &cs);
        w[i] = 0.5 * (1.0 - cs);
    }
}

typedef struct {
    double *w[3]; /* taper per axis, length b[a] */
} tapers_t;

static void make_tapers(const geom_t *g, tapers_t *t) {
    for (int a = 0; a < 3; ++a) {
        t->w[a] = (double *)malloc(sizeof(double) * (size_t)g->b[a]);
        or_taper(g->b[a], t->w[a]);
    }
}
static void free_tapers(tapers_t *t) {
    for (int a = 0; a < 3; ++a) free(t->w[a]);
}

static inline int64_t block_id3(const geom_t *g, const int64_t bc[3]) {
    return (bc[0] * g->nb3[1] + bc[1]) * g->nb3[2] + bc[2];
}

/* Neighbours on the half-spectrum layout (Supplementary S1.2).  A stored
 * block is (bz, by, bx) with bx = 0 .. nbxm - 1 for the columns below nx/2
 * (X_0 .. X_{nbxm-1}) and bx = nbxm for the column nx/2 (X_N).  Along z and
 * y the block grid is periodic as in the full layout; along x the stored
 * columns are a chain X_0 - ... - X_{nbxm-1} - X_N.  A neighbour in the
 * omitted half is replaced by its conjugate counterpart, q(-k) = q*(k),
 * taken mode by mode: the column -1 left of kx = 0 is the conjugate of
 * column 1 (in X_0, the x block edge being at least 2), the column right of
 * nx/2 the conjugate of column nx/2 - 1 (in X_{nbxm-1}), each at the
 * mirrored rows -y, -z.  Since the self-conjugate column nx/2 holds each of
 * its modes twice (at rows y and -y), the column left of it, X_{nbxm-1},
 * meets both X_N at its own rows and X_N at the mirrored rows.  So:
 *   x low of X_0:          X_0 at the mirrored rows (kx = 0 is a symmetry
 *                          boundary: a block there neighbours its partners)
 *   x high of X_N:         X_{nbxm-1} at the mirrored rows
 *   x high of X_{nbxm-1}:  X_N at its rows and at the mirrored rows
 * and the chain otherwise.  Rows [i b, i b + b) mirror to row (n - i b) mod n,
 * the first row of block (nb - i) mod nb, and rows below it, in block
 * (nb - i - 1) mod nb: up to two blocks per axis.  The relation is symmetric
 * (an active block's neighbours are the blocks that count it as theirs). */
static inline void half_coords(const geom_t *g, int64_t b, int64_t *bz, int64_t *by, int64_t *bx) {
    int64_t row;
    if (b >= g->nbm) {
        row = b - g->nbm;
        *bx = g->nbxm;
    } else {
        row = b / g->nbxm;
        *bx = b % g->nbxm;
    }
    *bz = row / g->nb3[1];
    *by = row % g->nb3[1];
}
static inline int64_t half_id(const geom_t *g, int64_t bz, int64_t by, int64_t bx) {
    const int64_t row = bz * g->nb3[1] + by;
    return bx == g->nbxm ? g->nbm + row : row * g->nbxm + bx;
}
/* the blocks that hold the mirrored rows of block i of an axis: 1 or 2 */
static int mirror_blocks(int64_t i, int64_t nb, int64_t b, int64_t out[2]) {
    out[0] = (nb - i) % nb;
    if (b < 2) return 1;
    out[1] = (nb - i - 1 + nb) % nb;
    return out[1] == out[0] ? 1 : 2;
}
/* append the blocks of column bx at the mirrored rows of (bz, by) */
static int add_mirrored(const geom_t *g, int64_t bz, int64_t by, int64_t bx, int64_t *out, int n) {
    int64_t mz[2], my[2];
    const int nz = mirror_blocks(bz, g->nb3[0], g->b[0], mz);
    const int ny = mirror_blocks(by, g->nb3[1], g->b[1], my);
    for (int i = 0; i < nz; ++i)
        for (int k = 0; k < ny; ++k) {
            const int64_t id = half_id(g, mz[i], my[k], bx);
            int dup = 0;
            for (int j = 0; j < n; ++j) dup |= out[j] == id;
            if (!dup) out[n++] = id;
        }
    return n;
}
/* stored blocks standing for the neighbour across face f (0 z low, 1 z high,
 * 2 y low, 3 y high, 4 x low, 5 x high) of stored block b; returns how many
 * (0: an axis with one block), at most 5 */
static int half_face(const geom_t *g, int64_t b, int f, int64_t out[8]) {
    int64_t bz, by, bx;
    half_coords(g, b, &bz, &by, &bx);
    const int a = f / 2, side = f % 2 ? 1 : -1;
    if (a < 2) {
        const int64_t nb = g->nb3[a];
        if (nb < 2) return 0;
        const int64_t j = ((a == 0 ? bz : by) + side + nb) % nb;
        out[0] = a == 0 ? half_id(g, j, by, bx) : half_id(g, bz, j, bx);
        return 1;
    }
    if (side < 0) {
        if (bx > 0) {
            out[0] = half_id(g, bz, by, bx - 1);
            return 1;
        }
        return add_mirrored(g, bz, by, 0, out, 0); /* kx = 0 */
    }
    if (bx == g->nbxm) return add_mirrored(g, bz, by, g->nbxm - 1, out, 0); /* beyond nx/2 */
    out[0] = half_id(g, bz, by, bx + 1);
    if (bx + 1 < g->nbxm) return 1;
    return add_mirrored(g, bz, by, g->nbxm, out, 1); /* X_{nbxm-1}: X_N at both row sets */
}

/* states from the active decisions: a block that is not active and has an
 * active face neighbour becomes 2 (transition).  Axes with one block have
 * no neighbours; the block grid is periodic.  Half layout: the neighbours
 * of half_face. */
static void add_transition(const geom_t *g, uint8_t *mask) {
    if (g->half) {
        uint8_t *act = (uint8_t *)malloc((size_t)g->nb);
        for (int64_t b = 0; b < g->nb; ++b) act[b] = mask[b] == 1;
        for (int64_t b = 0; b < g->nb; ++b) {
            if (act[b]) continue;
            int near = 0;
            for (int f = 0; f < 6 && !near; ++f) {
                int64_t nbr[8];
                const int n = half_face(g, b, f, nbr);
                for (int i = 0; i < n; ++i) near |= act[nbr[i]];
            }
            if (near) mask[b] = 2;
        }
        free(act);
        return;
    }
    for (int64_t b = 0; b < g->nb; ++b) {
        if (mask[b] != 0) continue;
        const int64_t bc[3] = {b / (g->nb3[1] * g->nb3[2]), (b / g->nb3[2]) % g->nb3[1], b % g->nb3[2]};
        int near = 0;
        for (int a = 0; a < 3 && !near; ++a) {
            if (g->nb3[a] < 2) continue;
            for (int side = -1; side <= 1; side += 2) {
                int64_t nc[3] = {bc[0], bc[1], bc[2]};
                nc[a] = (bc[a] + side + g->nb3[a]) % g->nb3[a];
                if (mask[block_id3(g, nc)] == 1) near = 1;
            }
        }
        if (near) mask[b] = 2;
    }
}

/* transition weight of mode (iz, iy, ix) of block b: product over the faces
 * that border frozen blocks, in the order z low, z high, y low, y high,
 * x low, x high */
static double sigma_of(const geom_t *g, const tapers_t *t, const uint8_t *mask, int64_t b, int64_t iz,
                       int64_t iy, int64_t ix) {
    if (g->half) { /* a face borders frozen blocks when every block standing for its neighbour is frozen */
        const int64_t li[3] = {iz % g->b[0], iy % g->b[1], 2 * ix == g->n[2] ? 0 : ix % g->b[2]};
        const int64_t bw[3] = {g->b[0], g->b[1], 2 * ix == g->n[2] ? 1 : g->b[2]};
        double s = 1.0;
        for (int f = 0; f < 6; ++f) {
            int64_t nbr[8];
            const int n = half_face(g, b, f, nbr);
            int frozen = n > 0;
            for (int i = 0; i < n; ++i) frozen &= mask[nbr[i]] == 0;
            if (!frozen) continue;
            const int a = f / 2;
            const double *w = bw[a] == 1 ? NULL : t->w[a];
            const double v = w ? w[f % 2 ? bw[a] - 1 - li[a] : li[a]] : 1.0;
            s = s * v;
        }
        return s;
    }
    const int64_t bc[3] = {b / (g->nb3[1] * g->nb3[2]), (b / g->nb3[2]) % g->nb3[1], b % g->nb3[2]};
    const int64_t li[3] = {iz % g->b[0], iy % g->b[1], ix % g->b[2]};
    double s = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (g->nb3[a] < 2) continue;
        int64_t lo[3] = {bc[0], bc[1], bc[2]}, hi[3] = {bc[0], bc[1], bc[2]};
        lo[a] = (bc[a] - 1 + g->nb3[a]) % g->nb3[a];
        hi[a] = (bc[a] + 1) % g->nb3[a];
        if (mask[block_id3(g, lo)] == 0) s = s * t->w[a][li[a]];
        if (mask[block_id3(g, hi)] == 0) s = s * t->w[a][g->b[a] - 1 - li[a]];
    }
    return s;
}

/* the per-block decision shared by both precisions; returns the number of
 * non-frozen blocks and lists them ascending in wl */
static int64_t block_states(const or_inst *d, const geom_t *g, const double *a_b, double thr,
                            const uint8_t *skip, uint8_t *mask, uint32_t *wl) {
    const int dense = (d->flags & OR_FLAG_DENSE) != 0;
    const int pin = (d->flags & OR_FLAG_PIN_K0) != 0;
    const int full = d->full_now != 0;
    for (int64_t b = 0; b < g->nb; ++b) {
        int on;
        if (dense || full) on = 1;
        else if (pin && b == 0) on = 1;
        else if (skip && skip[b]) on = 0;
        else on = a_b[b] > thr;
        mask[b] = (uint8_t)on;
    }
    if ((d->flags & OR_FLAG_TRANSITION) && !dense && !full) add_transition(g, mask);
    int64_t cnt = 0;
    for (int64_t b = 0; b < g->nb; ++b)
        if (mask[b]) wl[cnt++] = (uint32_t)b;
    return cnt;
}

int or_apply_f64(const or_inst *d, double *q, const double *rhs, const uint8_t *skip,
                 double *a_b, double *G, uint8_t *mask, uint32_t *wl, int64_t *count) {
    geom_t g;
    int rc = make_geom(d, &g);
    if (rc) return rc;
    if (d->op != OR_OP_NLSE && rhs == NULL) return OR_EINVAL;
    consts_t c;
    make_consts(d, &g, &c);
    const int64_t N = g.N;
    const int dense = (d->flags & OR_FLAG_DENSE) != 0;
    const int pin = (d->flags & OR_FLAG_PIN_K0) != 0;

    /* step 1: candidate q' for every mode, and a(k) */
    double *cand = (double *)malloc(sizeof(double) * 2 * (size_t)(N * g.nspec));
    double *ak = (double *)malloc(sizeof(double) * (size_t)N);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < N; ++i) {
        int64_t iz, iy, ix;
        mode_idx(&g, i, &iz, &iy, &ix);
        int64_t m2 = m2_of(&g, iz, iy, ix);
        double a;
        if (d->op == OR_OP_CH) {
            double s, f;
            ch_coef(&c, m2, &s, &f);
            double qr = q[2 * i], qi = q[2 * i + 1];
            double nr = rhs[2 * i], ni = rhs[2 * i + 1];
            double cr = fma(-s, nr, qr) * f, ci = fma(-s, ni, qi) * f;
            cand[2 * i] = cr;
            cand[2 * i + 1] = ci;
            a = sq2(cr - qr, ci - qi);
        } else if (d->op == OR_OP_GS) {
            double au, av;
            gs_coef(&c, m2, &au, &av);
            const double *u = q, *v = q + 2 * N, *ru = rhs, *rv = rhs + 2 * N;
            double ur = fma(c.dt, ru[2 * i], u[2 * i]) * au;
            double ui = fma(c.dt, ru[2 * i + 1], u[2 * i + 1]) * au;
            double vr = fma(c.dt, rv[2 * i], v[2 * i]) * av;
            double vi = fma(c.dt, rv[2 * i + 1], v[2 * i + 1]) * av;
            cand[2 * i] = ur;
            cand[2 * i + 1] = ui;
            cand[2 * N + 2 * i] = vr;
            cand[2 * N + 2 * i + 1] = vi;
            a = sq2(ur - u[2 * i], ui - u[2 * i + 1]) + sq2(vr - v[2 * i], vi - v[2 * i + 1]);
        } else if (d->op == OR_OP_XPFC) {
            double co[5];
            xpfc_coef(d, &c, m2, co);
            const double hr[4] = {rhs[2 * i], rhs[2 * (N + i)], rhs[2 * (2 * N + i)], rhs[2 * (3 * N + i)]};
            const double hi[4] = {rhs[2 * i + 1], rhs[2 * (N + i) + 1], rhs[2 * (2 * N + i) + 1],
                                  rhs[2 * (3 * N + i) + 1]};
            double cr, ci;
            xpfc_cand64(co, q[2 * i], hr, &cr);
            xpfc_cand64(co, q[2 * i + 1], hi, &ci);
            cand[2 * i] = cr;
            cand[2 * i + 1] = ci;
            a = sq2(cr - q[2 * i], ci - q[2 * i + 1]);
        } else {
            double hr, hi;
            nlse_coef(&c, m2, &hr, &hi);
            double er = q[2 * i], ei = q[2 * i + 1];
            double cr = fma(hr, er, -(hi * ei));
            double ci = fma(hr, ei, hi * er);
            cand[2 * i] = cr;
            cand[2 * i + 1] = ci;
            a = sq2(cr - er, ci - ei);
        }
        if (d->flags & OR_FLAG_STATE) { /* the state amplitude instead of the increment */
            a = 0.0;
            if (i != 0)
                for (int s = 0; s < g.nspec; ++s) a = a + sq2(q[2 * (s * N + i)], q[2 * (s * N + i) + 1]);
        }
        if (!(a <= DBL_MAX)) bad |= 1;
        ak[i] = a;
    }

    /* steps 2-4: a_b = max over the block, G = max over evaluated blocks,
     * active iff a_b > fl(tau^2 G), or the block holds k = 0 and PIN_K0 */
    for (int64_t b = 0; b < g.nb; ++b) a_b[b] = 0.0;
    if (!dense) {
        for (int64_t i = 0; i < N; ++i) {
            int64_t iz, iy, ix;
            mode_idx(&g, i, &iz, &iy, &ix);
            int64_t b = block_of(&g, iz, iy, ix);
            if (skip && skip[b] && !(pin && b == 0)) continue;
            if (d->flags & OR_FLAG_ENERGY) a_b[b] += ak[i]; /* block energy */
            else if (ak[i] > a_b[b]) a_b[b] = ak[i];
        }
    }
    double gmax = 0.0;
    if (!dense)
        for (int64_t b = 0; b < g.nb; ++b)
            if (a_b[b] > gmax) gmax = a_b[b];
    double thr = (d->tau * d->tau) * gmax;
    *count = block_states(d, &g, a_b, thr, skip, mask, wl);
    *G = gmax;

    /* step 5: active blocks take the candidate, transition blocks the
     * weighted increment q + sigma (q' - q), frozen blocks keep q */
    tapers_t tp;
    make_tapers(&g, &tp);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int64_t iz, iy, ix;
        mode_idx(&g, i, &iz, &iy, &ix);
        const int64_t b = block_of(&g, iz, iy, ix);
        if (!mask[b]) continue;
        const double sig = mask[b] == 2 ? sigma_of(&g, &tp, mask, b, iz, iy, ix) : 1.0;
        for (int s = 0; s < g.nspec; ++s) {
            const int64_t j = 2 * (s * N + i);
            if (mask[b] == 1) {
                q[j] = cand[j];
                q[j + 1] = cand[j + 1];
            } else {
                q[j] = fma(sig, cand[j] - q[j], q[j]);
                q[j + 1] = fma(sig, cand[j + 1] - q[j + 1], q[j + 1]);
            }
        }
    }
    free_tapers(&tp);
    free(cand);
    free(ak);
    return (bad && !dense) ? OR_ENONFINITE : OR_OK;
}

int or_apply_f32(const or_inst *d, float *q, const float *rhs, double *k0,
                 const double *rhs_k0, const uint8_t *skip, double *a_b, double *G,
                 uint8_t *mask, uint32_t *wl, int64_t *count) {
    geom_t g;
    int rc = make_geom(d, &g);
    if (rc) return rc;
    if (d->op != OR_OP_NLSE && (rhs == NULL || k0 == NULL || rhs_k0 == NULL)) return OR_EINVAL;
    consts_t c;
    make_consts(d, &g, &c);
    const int64_t N = g.N;
    const int dense = (d->flags & OR_FLAG_DENSE) != 0;
    const int pin = (d->flags & OR_FLAG_PIN_K0) != 0;
    const int k0path = (d->op != OR_OP_NLSE); /* real fields: k = 0 kept in FP64 */
    const float dtf = (float)c.dt;

    float *cand = (float *)malloc(sizeof(float) * 2 * (size_t)(N * g.nspec));
    double *ak = (double *)malloc(sizeof(double) * (size_t)N);
    double k0c[2] = {0.0, 0.0};
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < N; ++i) {
        int64_t iz, iy, ix;
        mode_idx(&g, i, &iz, &iy, &ix);
        int64_t m2 = m2_of(&g, iz, iy, ix);
        double a;
        if (k0path && i == 0) {
            /* the k = 0 mode in FP64 (coefficients at k = 0) */
            if (d->op == OR_OP_CH) {
                double s, f;
                ch_coef(&c, 0, &s, &f);
                k0c[0] = fma(-s, rhs_k0[0], k0[0]) * f;
                double dr = k0c[0] - k0[0];
                a = sq2(dr, 0.0);
            } else if (d->op == OR_OP_XPFC) {
                /* L(0) = 0 and the factor -k^2 of the nonlinear terms is 0:
                 * the mean density is kept */
                k0c[0] = k0[0];
                a = 0.0;
            } else {
                double au, av;
                gs_coef(&c, 0, &au, &av);
                k0c[0] = fma(c.dt, rhs_k0[0], k0[0]) * au;
                k0c[1] = fma(c.dt, rhs_k0[1], k0[1]) * av;
                a = sq2(k0c[0] - k0[0], 0.0) + sq2(k0c[1] - k0[1], 0.0);
            }
            for (int s = 0; s < g.nspec; ++s) {
                cand[2 * (s * N)] = 0.0f;
                cand[2 * (s * N) + 1] = 0.0f;
            }
        } else if (d->op == OR_OP_CH) {
            double s, f;
            ch_coef(&c, m2, &s, &f);
            float sf = (float)s, ff = (float)f;
            float qr = q[2 * i], qi = q[2 * i + 1];
            float cr = fmaf(-sf, rhs[2 * i], qr) * ff;
            float ci = fmaf(-sf, rhs[2 * i + 1], qi) * ff;
            cand[2 * i] = cr;
            cand[2 * i + 1] = ci;
            a = sq2((double)cr - (double)qr, (double)ci - (double)qi);
        } else if (d->op == OR_OP_GS) {
            double au, av;
            gs_coef(&c, m2, &au, &av);
            float auf = (float)au, avf = (float)av;
            const float *u = q, *v = q + 2 * N, *ru = rhs, *rv = rhs + 2 * N;
            float ur = fmaf(dtf, ru[2 * i], u[2 * i]) * auf;
            float ui = fmaf(dtf, ru[2 * i + 1], u[2 * i + 1]) * auf;
            float vr = fmaf(dtf, rv[2 * i], v[2 * i]) * avf;
            float vi = fmaf(dtf, rv[2 * i + 1], v[2 * i + 1]) * avf;
            cand[2 * i] = ur;
            cand[2 * i + 1] = ui;
            cand[2 * N + 2 * i] = vr;
            cand[2 * N + 2 * i + 1] = vi;
            a = sq2((double)ur - (double)u[2 * i], (double)ui - (double)u[2 * i + 1]) +
                sq2((double)vr - (double)v[2 * i], (double)vi - (double)v[2 * i + 1]);
        } else if (d->op == OR_OP_XPFC) {
            double co[5];
            xpfc_coef(d, &c, m2, co);
            const float cf[5] = {(float)co[0], (float)co[1], (float)co[2], (float)co[3], (float)co[4]};
            const float hr[4] = {rhs[2 * i], rhs[2 * (N + i)], rhs[2 * (2 * N + i)], rhs[2 * (3 * N + i)]};
            const float hi[4] = {rhs[2 * i + 1], rhs[2 * (N + i) + 1], rhs[2 * (2 * N + i) + 1],
                                 rhs[2 * (3 * N + i) + 1]};
            float cr, ci;
            xpfc_cand32(cf, q[2 * i], hr, &cr);
            xpfc_cand32(cf, q[2 * i + 1], hi, &ci);
            cand[2 * i] = cr;
            cand[2 * i + 1] = ci;
            a = sq2((double)cr - (double)q[2 * i], (double)ci - (double)q[2 * i + 1]);
        } else {
            double hr, hi;
            nlse_coef(&c, m2, &hr, &hi);
            float hrf = (float)hr, hif = (float)hi;
            float er = q[2 * i], ei = q[2 * i + 1];
            float cr = fmaf(hrf, er, -(hif * ei));
            float ci = fmaf(hrf, ei, hif * er);
            cand[2 * i] = cr;
            cand[2 * i + 1] = ci;
            a = sq2((double)cr - (double)er, (double)ci - (double)ei);
        }
        if (d->flags & OR_FLAG_STATE) { /* the state amplitude instead of the increment */
            a = 0.0;
            if (i != 0)
                for (int s = 0; s < g.nspec; ++s)
                    a = a + sq2((double)q[2 * (s * N + i)], (double)q[2 * (s * N + i) + 1]);
        }
        if (!(a <= DBL_MAX)) bad |= 1;
        ak[i] = a;
    }

    for (int64_t b = 0; b < g.nb; ++b) a_b[b] = 0.0;
    if (!dense) {
        for (int64_t i = 0; i < N; ++i) {
            int64_t iz, iy, ix;
            mode_idx(&g, i, &iz, &iy, &ix);
            int64_t b = block_of(&g, iz, iy, ix);
            if (skip && skip[b] && !(pin && b == 0)) continue;
            if (d->flags & OR_FLAG_ENERGY) a_b[b] += ak[i]; /* block energy */
            else if (ak[i] > a_b[b]) a_b[b] = ak[i];
        }
    }
    double gmax = 0.0;
    if (!dense)
        for (int64_t b = 0; b < g.nb; ++b)
            if (a_b[b] > gmax) gmax = a_b[b];
    double thr = (d->tau * d->tau) * gmax;
    *count = block_states(d, &g, a_b, thr, skip, mask, wl);
    *G = gmax;

    /* transition increments in FP32: delta = q' - q, then fma(fl32(sigma), delta, q) */
    tapers_t tp;
    make_tapers(&g, &tp);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int64_t iz, iy, ix;
        mode_idx(&g, i, &iz, &iy, &ix);
        const int64_t b = block_of(&g, iz, iy, ix);
        if (!mask[b]) continue;
        const float sig = mask[b] == 2 ? (float)sigma_of(&g, &tp, mask, b, iz, iy, ix) : 1.0f;
        for (int s = 0; s < g.nspec; ++s) {
            const int64_t j = 2 * (s * N + i);
            if (mask[b] == 1) {
                q[j] = cand[j];
                q[j + 1] = cand[j + 1];
            } else {
                const float dr = cand[j] - q[j], di = cand[j + 1] - q[j + 1];
                q[j] = fmaf(sig, dr, q[j]);
                q[j + 1] = fmaf(sig, di, q[j + 1]);
            }
        }
    }
    if (k0path) {
        if (mask[0] == 1)
            for (int s = 0; s < g.nspec; ++s) k0[s] = k0c[s];
        else if (mask[0] == 2) {
            /* block 0 in transition: the FP64 k = 0 value takes its weighted increment */
            const double sig0 = sigma_of(&g, &tp, mask, 0, 0, 0, 0);
            for (int s = 0; s < g.nspec; ++s) k0[s] = fma(sig0, k0c[s] - k0[s], k0[s]);
        }
        for (int s = 0; s < g.nspec; ++s) {
            q[2 * (s * N)] = 0.0f;
            q[2 * (s * N) + 1] = 0.0f;
        }
    }
    free_tapers(&tp);
    free(cand);
    free(ak);
    return (bad && !dense) ? OR_ENONFINITE : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Full FP64 steps                                                           */
/* ------------------------------------------------------------------------ */

/* Real field of a half spectrum (Supplementary S1.2): the omitted columns
 * nx/2 + 1 .. nx - 1 are filled by q(-k) = conj q(k) from the stored ones,
 * the stored columns 0 and nx/2 are taken as they are, and the real part of
 * the complex inverse is returned (1/N included). */
int or_c2r(const int64_t dims[3], const double *half, double *real) {
    const int64_t nz = dims[0], ny = dims[1], nx = dims[2];
    if (nx < 2 || !is_pow2(nx)) return OR_EINVAL;
    const int64_t xs = nx / 2 + 1, N = nz * ny * nx;
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    for (int64_t iz = 0; iz < nz; ++iz)
        for (int64_t iy = 0; iy < ny; ++iy)
            for (int64_t ix = 0; ix < nx; ++ix) {
                double *o = w + 2 * ((iz * ny + iy) * nx + ix);
                if (ix < xs) {
                    const double *src = half + 2 * ((iz * ny + iy) * xs + ix);
                    o[0] = src[0];
                    o[1] = src[1];
                } else {
                    const int64_t jz = (nz - iz) % nz, jy = (ny - iy) % ny, jx = nx - ix;
                    const double *src = half + 2 * ((jz * ny + jy) * xs + jx);
                    o[0] = src[0];
                    o[1] = -src[1];
                }
            }
    int rc = or_fft(w, dims, +1);
    for (int64_t i = 0; i < N; ++i) real[i] = w[2 * i];
    free(w);
    return rc;
}

/* Half spectrum of a real field: the forward transform, columns 0 .. nx/2. */
int or_r2c(const int64_t dims[3], const double *real, double *half) {
    const int64_t nz = dims[0], ny = dims[1], nx = dims[2];
    if (nx < 2 || !is_pow2(nx)) return OR_EINVAL;
    const int64_t xs = nx / 2 + 1, N = nz * ny * nx;
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        w[2 * i] = real[i];
        w[2 * i + 1] = 0.0;
    }
    int rc = or_fft(w, dims, -1);
    for (int64_t r = 0; r < nz * ny; ++r)
        for (int64_t ix = 0; ix < xs; ++ix) {
            half[2 * (r * xs + ix)] = w[2 * (r * nx + ix)];
            half[2 * (r * xs + ix) + 1] = w[2 * (r * nx + ix) + 1];
        }
    free(w);
    return rc;
}

int or_sizes(const or_inst *d, int64_t *n_modes, int64_t *n_blocks) {
    geom_t g;
    const int rc = make_geom(d, &g);
    if (rc != OR_OK) return rc;
    if (n_modes) *n_modes = g.N;
    if (n_blocks) *n_blocks = g.nb;
    return OR_OK;
}

int or_ch_energy(const or_inst *d, const double *chat, double *energy, double *mass) {
    /* F = dx^d sum_x f(c) + (kappa/2) (dx^d / N) sum_k k^2 |c_k|^2,
     * f(c) = (c^2 - 1)^2 / 4 (so f'(c) = c^3 - c); mass = mean of c.
     * Half layout: c from or_c2r; the stored columns 1 .. nx/2 - 1 stand for
     * themselves and their conjugate partners, so they count twice. */
    geom_t g;
    int rc = make_geom(d, &g);
    if (rc) return rc;
    const int64_t N = g.N, NR = g.Nreal;
    int ndim = (g.n[0] > 1) + (g.n[1] > 1) + (g.n[2] > 1);
    if (ndim == 0) ndim = 1;
    double dvol = 1.0;
    for (int k = 0; k < ndim; ++k) dvol *= d->dx;
    double *c = (double *)malloc(sizeof(double) * (size_t)NR);
    if (g.half) {
        or_c2r(g.n, chat, c);
    } else {
        double *w = (double *)malloc(sizeof(double) * 2 * (size_t)N);
        memcpy(w, chat, sizeof(double) * 2 * (size_t)N);
        or_fft(w, g.n, +1);
        for (int64_t i = 0; i < N; ++i) c[i] = w[2 * i];
        free(w);
    }
    double K2 = kk_base(&g, d->dx);
    double bulk = 0.0, grad = 0.0;
    for (int64_t i = 0; i < NR; ++i) {
        double t = c[i] * c[i] - 1.0;
        bulk += 0.25 * t * t;
    }
    for (int64_t i = 0; i < N; ++i) {
        int64_t iz, iy, ix;
        mode_idx(&g, i, &iz, &iy, &ix);
        double k2 = K2 * (double)m2_of(&g, iz, iy, ix);
        double wgt = (g.half && ix != 0 && 2 * ix != g.n[2]) ? 2.0 : 1.0;
        grad += wgt * (k2 * (chat[2 * i] * chat[2 * i] + chat[2 * i + 1] * chat[2 * i + 1]));
    }
    free(c);
    *energy = dvol * bulk + 0.5 * d->p[1] * (dvol / (double)NR) * grad;
    *mass = chat[0] / (double)NR;
    return OR_OK;
}

int or_step_f64(const or_inst *d, int64_t nsteps, double *state, uint8_t *masks,
                double *diag, double *ab, int64_t *active_steps) {
    return or_step_ctl_f64(d, nsteps, state, masks, diag, ab, active_steps, NULL);
}

int or_step_ctl_f64(const or_inst *d0, int64_t nsteps, double *state, uint8_t *masks,
                    double *diag, double *ab, int64_t *active_steps, double *tau_trace) {
    geom_t g;
    int rc = make_geom(d0, &g);
    if (rc) return rc;
    const int refresh = (d0->flags & OR_FLAG_REFRESH) != 0;
    const int dyn = (d0->flags & OR_FLAG_DYN_TAU) != 0;
    if (refresh && d0->refresh_period < 1) return OR_EINVAL;
    if (d0->full_steps < 0) return OR_EINVAL;
    if (dyn && (d0->interval < 1 || !(d0->target_ratio > 0.0 && d0->target_ratio <= 1.0) ||
                !(d0->deadband >= 0.0 && d0->deadband < 1.0)))
        return OR_EINVAL;
    or_inst dd = *d0; /* per step: the current tau and the full flag */
    const or_inst *d = &dd;
    double ctl_sum = 0.0;
    int64_t ctl_n = 0;
    const int64_t N = g.N, nb = g.nb;
    const int per = (d->op == OR_OP_NLSE) ? 2 : 1;
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)(N * g.nspec));
    double *re = (double *)malloc(sizeof(double) * (size_t)(g.Nreal * g.nspec)); /* half layout */
    double *a_b = (double *)malloc(sizeof(double) * (size_t)nb);
    uint8_t *mk = (uint8_t *)malloc((size_t)nb);
    uint32_t *wl = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nb);
    /* XPFC: the four nonlinear transforms of a step, newest first */
    double *h4 = d->op == OR_OP_XPFC ? (double *)malloc(sizeof(double) * 8 * (size_t)N) : NULL;
    if (active_steps)
        for (int64_t b = 0; b < nb; ++b) active_steps[b] = 0;
    rc = OR_OK;
    int64_t nonfrozen = 0; /* non-frozen blocks over the current step's updates */
    for (int64_t st = 0; st < nsteps && rc == OR_OK; ++st) {
        double G;
        int64_t cnt;
        /* the step schedule (Supplementary S1.3) */
        const int full = st < d0->full_steps || (refresh && (st + 1) % d0->refresh_period == 0);
        dd.full_now = full;
        if (tau_trace) tau_trace[st] = dd.tau;
        nonfrozen = 0;
        if (d->op == OR_OP_CH) {
            if (diag) {
                double F, m;
                or_ch_energy(d, state, &F, &m);
                diag[4 * st] = m;
                diag[4 * st + 1] = F;
                diag[4 * st + 2] = 0.0;
                diag[4 * st + 3] = 0.0;
            }
            /* real space: c = Re F^-1[c-hat]; nonlinear term c^3 - c; N-hat */
            if (g.half) {
                or_c2r(g.n, state, re);
                for (int64_t i = 0; i < g.Nreal; ++i) re[i] = re[i] * re[i] * re[i] - re[i];
                or_r2c(g.n, re, w);
            } else {
                memcpy(w, state, sizeof(double) * 2 * (size_t)N);
                or_fft(w, g.n, +1);
                for (int64_t i = 0; i < N; ++i) {
                    double cc = w[2 * i];
                    w[2 * i] = cc * cc * cc - cc;
                    w[2 * i + 1] = 0.0;
                }
                or_fft(w, g.n, -1);
            }
            rc = or_apply_f64(d, state, w, NULL, a_b, &G, mk, wl, &cnt);
        } else if (d->op == OR_OP_GS) {
            /* R_u = -u v^2 + F (1 - u), R_v = u v^2 - (F + k) v */
            const double Fp = d->p[2], kp = d->p[3];
            const int64_t NR = g.Nreal;
            double *ru = re, *rv = re + NR;
            if (g.half) {
                or_c2r(g.n, state, ru);
                or_c2r(g.n, state + 2 * N, rv);
            } else {
                memcpy(w, state, sizeof(double) * 4 * (size_t)N);
                or_fft(w, g.n, +1);
                or_fft(w + 2 * N, g.n, +1);
                for (int64_t i = 0; i < N; ++i) {
                    ru[i] = w[2 * i];
                    rv[i] = w[2 * N + 2 * i];
                }
            }
            if (diag) {
                double su = 0.0, sv = 0.0;
                for (int64_t i = 0; i < NR; ++i) {
                    su += ru[i];
                    sv += rv[i];
                }
                diag[4 * st] = su / (double)NR;
                diag[4 * st + 1] = sv / (double)NR;
                diag[4 * st + 2] = 0.0;
                diag[4 * st + 3] = 0.0;
            }
            for (int64_t i = 0; i < NR; ++i) {
                double u = ru[i], v = rv[i];
                double uvv = u * v * v;
                ru[i] = -uvv + Fp * (1.0 - u);
                rv[i] = uvv - (Fp + kp) * v;
            }
            if (g.half) {
                or_r2c(g.n, ru, w);
                or_r2c(g.n, rv, w + 2 * N);
            } else {
                for (int64_t i = 0; i < N; ++i) {
                    w[2 * i] = ru[i];
                    w[2 * i + 1] = 0.0;
                    w[2 * N + 2 * i] = rv[i];
                    w[2 * N + 2 * i + 1] = 0.0;
                }
                or_fft(w, g.n, -1);
                or_fft(w + 2 * N, g.n, -1);
            }
            rc = or_apply_f64(d, state, w, NULL, a_b, &G, mk, wl, &cnt);
        } else if (d->op == OR_OP_XPFC) {
            if (diag) {
                double F, m;
                or_xpfc_energy(d, state, &F, &m);
                diag[4 * st] = m;
                diag[4 * st + 1] = F;
                diag[4 * st + 2] = 0.0;
                diag[4 * st + 3] = 0.0;
            }
            /* psi = Re F^-1[psi-hat]; H_n = F[-(omega/2) psi^2 + (u/3) psi^3] */
            const double om = d->p[3], uu = d->p[4];
            memcpy(h4, state, sizeof(double) * 2 * (size_t)N);
            or_fft(h4, g.n, +1);
            for (int64_t i = 0; i < N; ++i) {
                const double ps = h4[2 * i];
                const double t = ps * ps;
                h4[2 * i] = -(om / 2.0) * t + (uu / 3.0) * (t * ps);
                h4[2 * i + 1] = 0.0;
            }
            or_fft(h4, g.n, -1);
            /* the older transforms: carried by the state, or (first step of an
             * unset history) the initial nonlinear term itself */
            for (int k = 1; k < 4; ++k) {
                const double *src = (st == 0 && !d0->hist_valid) ? h4 : state + 2 * (size_t)k * N;
                memcpy(h4 + 2 * (size_t)k * N, src, sizeof(double) * 2 * (size_t)N);
            }
            rc = or_apply_f64(d, state, h4, NULL, a_b, &G, mk, wl, &cnt);
            /* shift: the state keeps H_n, H_{n-1}, H_{n-2} */
            memcpy(state + 2 * (size_t)N, h4, sizeof(double) * 6 * (size_t)N);
        } else {
            /* symmetric split step: linear half, Kerr rotation, linear half */
            if (diag) {
                double p = 0.0;
                for (int64_t i = 0; i < N; ++i)
                    p += state[2 * i] * state[2 * i] + state[2 * i + 1] * state[2 * i + 1];
                diag[4 * st] = p;
                diag[4 * st + 1] = diag[4 * st + 2] = diag[4 * st + 3] = 0.0;
            }
            const double gam = d->p[1], h = d->dt;
            for (int half = 0; half < 2 && rc == OR_OK; ++half) {
                or_fft(state, g.n, -1);
                rc = or_apply_f64(d, state, NULL, NULL, a_b, &G, mk, wl, &cnt);
                or_fft(state, g.n, +1);
                nonfrozen += cnt;
                if (masks) memcpy(masks + (st * per + half) * nb, mk, (size_t)nb);
                if (ab) memcpy(ab + (st * per + half) * nb, a_b, sizeof(double) * (size_t)nb);
                if (active_steps)
                    for (int64_t b = 0; b < nb; ++b) active_steps[b] += mk[b] != 0;
                if (half == 0) {
                    for (int64_t i = 0; i < N; ++i) {
                        double er = state[2 * i], ei = state[2 * i + 1];
                        double ph = gam * (er * er + ei * ei) * h;
                        double cs = cos(ph), sn = sin(ph);
                        state[2 * i] = er * cs - ei * sn;
                        state[2 * i + 1] = er * sn + ei * cs;
                    }
                }
            }
        }
        if (d->op != OR_OP_NLSE) nonfrozen = cnt;
        /* threshold control on the steps that are not full */
        if (dyn && !full && rc == OR_OK) {
            ctl_sum += (double)nonfrozen / (double)(nb * per);
            if (++ctl_n == d0->interval) {
                const double rho = (ctl_sum / (double)d0->interval) / d0->target_ratio;
                const double eta = d0->deadband;
                if (rho > 2.0) dd.tau = dd.tau * 2.0;
                else if (rho > 1.0 + eta) dd.tau = dd.tau * (1.0 + eta);
                else if (rho < 0.5) dd.tau = dd.tau * 0.5;
                else if (rho < 1.0 - eta) dd.tau = dd.tau * (1.0 - eta);
                ctl_sum = 0.0;
                ctl_n = 0;
            }
        }
        if (d->op == OR_OP_NLSE) continue;
        if (masks) memcpy(masks + st * nb, mk, (size_t)nb);
        if (ab) memcpy(ab + st * nb, a_b, sizeof(double) * (size_t)nb);
        if (active_steps)
            for (int64_t b = 0; b < nb; ++b) active_steps[b] += mk[b] != 0;
    }
    free(w);
    free(re);
    free(a_b);
    free(mk);
    free(wl);
    free(h4);
    return rc;
}

int or_xpfc_energy(const or_inst *d, const double *psihat, double *energy, double *mean) {
    geom_t g;
    int rc = make_geom(d, &g);
    if (rc) return rc;
    if (d->op != OR_OP_XPFC) return OR_EINVAL;
    const int64_t N = g.N;
    int ndim = (g.n[0] > 1) + (g.n[1] > 1) + (g.n[2] > 1);
    if (ndim == 0) ndim = 1;
    double dvol = 1.0;
    for (int k = 0; k < ndim; ++k) dvol *= d->dx;
    const double om = d->p[3], uu = d->p[4];
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    memcpy(w, psihat, sizeof(double) * 2 * (size_t)N);
    or_fft(w, g.n, +1);
    double bulk = 0.0, sum = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        const double ps = w[2 * i];
        const double p2 = ps * ps;
        bulk += 0.5 * p2 - (om / 6.0) * (p2 * ps) + (uu / 12.0) * (p2 * p2);
        sum += ps;
    }
    free(w);
    const double K2 = kk_base(&g, d->dx);
    const double q0 = d->p[0], sg = d->p[1], al = d->p[2], rho = d->p[5], be = d->p[6];
    const double dw = exp(-((sg * sg) * (q0 * q0)) / (2.0 * (rho * be)));
    double corr = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t iz, iy, ix;
        mode_idx(&g, i, &iz, &iy, &ix);
        const double k = sqrt(K2 * (double)m2_of(&g, iz, iy, ix));
        const double dk = k - q0;
        const double c2 = exp(-(dk * dk) / (2.0 * (al * al))) * dw;
        corr += c2 * sq2(psihat[2 * i], psihat[2 * i + 1]);
    }
    *energy = dvol * (bulk - corr / (2.0 * (double)N));
    *mean = sum / (double)N;
    return OR_OK;
}
