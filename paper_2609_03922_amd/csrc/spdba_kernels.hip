// spdba_kernels.hip -- gfx950 kernels of the sp-DBA transform-domain update.
//
// Stages of one step (Methods, "Spectral dynamic block activation"; the
// transformed-field update of Supplementary S2.1):
//   k_nonlinear  fused real-space term on the inverse-transformed field
//   k_indicator  candidate increment of every mode, FP64 a(k), block max a_b,
//                instance max G (order-free atomic max on the bit pattern)
//   k_compact_*  threshold, per-block mask and the ascending active-block list
//   k_update     persistent walk of the active list: model update of every mode
//                of each active block; frozen blocks are never touched
//   k_dense      Regular mode: the same update core over every mode
//
// Memory-bound throughout: vector loads of 16 B per lane, each wave row covers
// at least 1 KiB of contiguous coefficients, partial sums in FP64 in a fixed
// order (no floating-point atomics), integer-exact compaction.  The rounding
// of the update core is fixed (explicit fma, coefficients formed in FP64 from
// the exact integer m^2 and rounded once) so that masks are reproducible bit
// for bit by any implementation of the same arithmetic.
//
// Built with -ffp-contract=off: every fused multiply-add is written out.

#include "spdba_internal.h"

#include <hip/hip_ext.h>

#include <float.h>

namespace spdba {

// -------------------------------------------------------------------------
// small helpers
// -------------------------------------------------------------------------

__device__ __forceinline__ int sidx(int i, int n) { return (2 * i < n) ? i : i - n; }

__device__ __forceinline__ int find_by_offset(const InstDev *ins, int n, int64_t id, int which) {
    // binary search for the last instance whose offset (strip/tile) <= id
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int64_t o = which == 0 ? ins[mid].strip_off : ins[mid].tile_off;
        if (o <= id) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T> struct CV;
template <> struct CV<float> {
    static constexpr int V = 2;  // complex values per 16-byte lane access
    __device__ static void ld(const float *p, float (&re)[2], float (&im)[2]) {
        float4 v = *reinterpret_cast<const float4 *>(p);
        re[0] = v.x; im[0] = v.y; re[1] = v.z; im[1] = v.w;
    }
    __device__ static void st(float *p, const float (&re)[2], const float (&im)[2]) {
        *reinterpret_cast<float4 *>(p) = make_float4(re[0], im[0], re[1], im[1]);
    }
};
template <> struct CV<double> {
    static constexpr int V = 1;
    __device__ static void ld(const double *p, double (&re)[1], double (&im)[1]) {
        double2 v = *reinterpret_cast<const double2 *>(p);
        re[0] = v.x; im[0] = v.y;
    }
    __device__ static void st(double *p, const double (&re)[1], const double (&im)[1]) {
        *reinterpret_cast<double2 *>(p) = make_double2(re[0], im[0]);
    }
};

__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ void sc_t(float x, float &s, float &c) { sincosf(x, &s, &c); }
__device__ __forceinline__ void sc_t(double x, double &s, double &c) { sincos(x, &s, &c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// sin and cos: Cody-Waite reduction by pi/2 (three-part constant, fdlibm
// split) and Taylor series of sin / cos on |r| <= pi/4, Horner with fma.
__device__ __forceinline__ void sincos_cw(double x, double &sn, double &cs) {
    const double q = rint(x * 6.36619772367581382433e-01);
    double r = __builtin_fma(-q, 1.57079632673412561417e+00, x);
    r = __builtin_fma(-q, 6.07710050630396597660e-11, r);
    r = __builtin_fma(-q, 2.02226624879595063154e-21, r);
    const double r2 = r * r;
    double ps = 1.0 / 355687428096000.0;
    ps = __builtin_fma(ps, r2, -1.0 / 1307674368000.0);
    ps = __builtin_fma(ps, r2, 1.0 / 6227020800.0);
    ps = __builtin_fma(ps, r2, -1.0 / 39916800.0);
    ps = __builtin_fma(ps, r2, 1.0 / 362880.0);
    ps = __builtin_fma(ps, r2, -1.0 / 5040.0);
    ps = __builtin_fma(ps, r2, 1.0 / 120.0);
    ps = __builtin_fma(ps, r2, -1.0 / 6.0);
    const double s = __builtin_fma(r * r2, ps, r);
    double pc = -1.0 / 6402373705728000.0;
    pc = __builtin_fma(pc, r2, 1.0 / 20922789888000.0);
    pc = __builtin_fma(pc, r2, -1.0 / 87178291200.0);
    pc = __builtin_fma(pc, r2, 1.0 / 479001600.0);
    pc = __builtin_fma(pc, r2, -1.0 / 3628800.0);
    pc = __builtin_fma(pc, r2, 1.0 / 40320.0);
    pc = __builtin_fma(pc, r2, -1.0 / 720.0);
    pc = __builtin_fma(pc, r2, 1.0 / 24.0);
    pc = __builtin_fma(pc, r2, -0.5);
    const double c = __builtin_fma(r2, pc, 1.0);
    const int qi = (int)((long long)q & 3);
    if (qi == 0) { sn = s; cs = c; }
    else if (qi == 1) { sn = c; cs = -s; }
    else if (qi == 2) { sn = -s; cs = -c; }
    else { sn = -c; cs = s; }
}

// -------------------------------------------------------------------------
// update cores (identical arithmetic in indicator, active update and dense)
// -------------------------------------------------------------------------

// CH: s = dt M k^2, a = 1/(1 + dt M kappa k^4) in FP64, then working precision.
// Operator constants in registers.  Hot loops take them by value: read
// through the instance table they would be re-fetched after every store to
// the state (the compiler cannot rule out aliasing).
struct Coef {
    double K2, c0, c1, c2;
    __device__ static Coef of(const InstDev &I) {
        Coef k;
        k.K2 = I.K2;
        k.c0 = I.c0;
        k.c1 = I.c1;
        k.c2 = I.c2;
        return k;
    }
};

// 1/t for finite t >= 1: the hardware reciprocal estimate, two Newton-Raphson
// refinements and one residual correction (Markstein).  Without exponent
// scaling, which no such t needs, these are the steps of the IEEE-correct
// division 1/t, so the result is the correctly rounded reciprocal.
__device__ __forceinline__ double recip_ge1(double t) {
    double r = __builtin_amdgcn_rcp(t);
    double e = __builtin_fma(-t, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-t, r, 1.0);
    r = __builtin_fma(r, e, r);
    const double rem = __builtin_fma(-t, r, 1.0);
    return __builtin_fma(rem, r, r);
}

// Coefficients of one mode from its integer |m|^2, passed as an exact double.
template <typename T>
__device__ __forceinline__ void ch_coef(const Coef &K, double m2, T &s, T &a) {
    const double k2 = K.K2 * m2;
    const double sd = K.c0 * k2;
    const double ad = recip_ge1(1.0 + K.c1 * (k2 * k2));
    s = (T)sd;
    a = (T)ad;
}
template <typename T>
__device__ __forceinline__ void gs_coef(const Coef &K, double m2, T &au, T &av) {
    const double k2 = K.K2 * m2;
    au = (T)recip_ge1(1.0 + K.c1 * k2);
    av = (T)recip_ge1(1.0 + K.c2 * k2);
}
template <typename T>
__device__ __forceinline__ void nlse_coef(const Coef &K, double m2, T &hr, T &hi) {
    double sn, cs;
    sincos_cw(K.c0 * m2, sn, cs);
    hr = (T)(K.c1 * cs);
    hi = (T)(K.c1 * sn);
}

// NLSE, one dimension: the propagator H depends on |m| only, so it is read
// from a per-instance table built by k_htable with nlse_coef itself (same
// bits as evaluating it here).  x: grid index, n: length; |m| = x for
// x <= n/2, n - x above.
template <typename T>
__device__ __forceinline__ void nlse_tab_ld(const T *tab, int x, int n, T (&hr)[CV<T>::V], T (&hi)[CV<T>::V]) {
#pragma unroll
    for (int v = 0; v < CV<T>::V; ++v) {
        const int j = (2 * (x + v) <= n) ? x + v : n - x - v;
        hr[v] = tab[2 * j];
        hi[v] = tab[2 * j + 1];
    }
}

// |m|^2 parts as exact doubles (integers far below 2^53)
__device__ __forceinline__ double sq_d(int m) {
    const double d = (double)m;
    return d * d;
}

__device__ __forceinline__ double sq2(double dr, double di) { return dr * dr + di * di; }

// Candidate of one CH mode and its squared increment.
template <typename T>
__device__ __forceinline__ double ch_cand(T s, T a, T qr, T qi, T nr, T ni, T &cr, T &ci) {
    cr = fmat(-s, nr, qr) * a;
    ci = fmat(-s, ni, qi) * a;
    return sq2((double)cr - (double)qr, (double)ci - (double)qi);
}
template <typename T>
__device__ __forceinline__ double gs_cand(T dt, T a, T qr, T qi, T rr, T ri, T &cr, T &ci) {
    cr = fmat(dt, rr, qr) * a;
    ci = fmat(dt, ri, qi) * a;
    return sq2((double)cr - (double)qr, (double)ci - (double)qi);
}
template <typename T>
__device__ __forceinline__ double nlse_cand(T hr, T hi, T er, T ei, T &cr, T &ci) {
    cr = fmat(hr, er, -(hi * ei));
    ci = fmat(hr, ei, hi * er);
    return sq2((double)cr - (double)er, (double)ci - (double)ei);
}

// FP64 k = 0 candidate of the real-field operators (coefficients at k = 0).
__device__ __forceinline__ double k0_cand(const InstDev &I, int op, const double *k0,
                                          const double *rk0, double *out) {
    if (op == OP_XPFC) {  // L(0) = 0 and the nonlinear terms carry -k^2 = 0: the mean is kept
        out[0] = k0[0];
        return 0.0;
    }
    if (op == OP_CH) {
        const double s = I.c0 * 0.0;
        const double a = 1.0 / (1.0 + I.c1 * (0.0 * 0.0));
        out[0] = __builtin_fma(-s, rk0[0], k0[0]) * a;
        return sq2(out[0] - k0[0], 0.0);
    }
    const double au = 1.0 / (1.0 + I.c1 * 0.0);
    const double av = 1.0 / (1.0 + I.c2 * 0.0);
    out[0] = __builtin_fma(I.c0, rk0[0], k0[0]) * au;
    out[1] = __builtin_fma(I.c0, rk0[1], k0[1]) * av;
    return sq2(out[0] - k0[0], 0.0) + sq2(out[1] - k0[1], 0.0);
}

// -------------------------------------------------------------------------
// XPFC update core (Supplementary S3.2): the ETD4 multistep update in
// backward differences of the nonlinear transforms H_n .. H_{n-3},
//   psi' = e^z psi + B1 H_n + B2 dH + B3 d2H + B4 d3H,  B_l = -k^2 Phi_l,
// z = L dt with L(k) = -k^2 (1 - C2(k)) read from a per-instance FP64 table
// by (|m_z|, |m_y|, |m_x|) (filled on the host at plan creation).  The coefficients
// are formed in FP64 -- phi_4 from its series for |z| <= 1 and the
// recurrence phi_l = 1/l! + z phi_{l+1} (e^z = 1 + z phi_1), else e^z by
// scaling and squaring and phi_1 .. phi_4 in closed form -- and rounded
// once to the working precision; every operation explicit (fma where
// fused), so any implementation of the same steps gives the same bits.
// -------------------------------------------------------------------------

struct InvFact {
    double v[19];
};
// 1/n!, n = 0 .. 18, each rounded once (n! is exact in double up to 18!)
constexpr InvFact make_inv_fact() {
    InvFact t{};
    double f = 1.0;
    for (int n = 0; n < 19; ++n) {
        if (n >= 2) f *= (double)n;
        t.v[n] = 1.0 / f;
    }
    return t;
}

__device__ __forceinline__ void phi_series(double w, double (&o)[5]) {
    constexpr InvFact F = make_inv_fact();
    double p4 = F.v[18];
#pragma unroll
    for (int j = 13; j >= 0; --j) p4 = __builtin_fma(p4, w, F.v[4 + j]);
    const double p3 = __builtin_fma(w, p4, F.v[3]);
    const double p2 = __builtin_fma(w, p3, F.v[2]);
    const double p1 = __builtin_fma(w, p2, 1.0);
    o[0] = __builtin_fma(w, p1, 1.0);
    o[1] = p1;
    o[2] = p2;
    o[3] = p3;
    o[4] = p4;
}

// {e^z, phi_1 .. phi_4}
__device__ __forceinline__ void etd4_phi(double z, double (&o)[5]) {
    if (__builtin_fabs(z) <= 1.0) {
        phi_series(z, o);
        return;
    }
    constexpr InvFact F = make_inv_fact();
    int s = 0;
    double w = z;
    while (__builtin_fabs(w) > 1.0) {
        w *= 0.5;
        ++s;
    }
    double t[5];
    phi_series(w, t);
    double e = t[0];
    for (int i = 0; i < s; ++i) e = e * e;
    o[0] = e;
    o[1] = (e - 1.0) / z;
    o[2] = (o[1] - 1.0) / z;
    o[3] = (o[2] - F.v[2]) / z;
    o[4] = (o[3] - F.v[3]) / z;
}

// The L table of an instance is indexed by (|m_z|, |m_y|, |m_x|), C order
// over extents n/2 + 1 (1 on unused axes): a row of it serves a grid row.
__device__ __forceinline__ const double *xpfc_row(const Ctx &c, const InstDev &I, int z, int y) {
    const int h1 = (I.n[1] >> 1) + 1, h2 = (I.n[2] >> 1) + 1;
    const int az = abs(sidx(z, I.n[0])), ay = abs(sidx(y, I.n[1]));
    return c.ltab + I.ltab_off + ((int64_t)az * h1 + ay) * h2;
}

// {e^z, B1 .. B4} of the mode with integer |m|^2 = m2 and |m_x| = ax on the
// table row lrow (dt = K.c0)
template <typename T>
__device__ __forceinline__ void xpfc_coef(const Coef &K, const double *lrow, int ax, double m2, T (&co)[5]) {
    const double k2 = K.K2 * m2;
    const double dt = K.c0;
    const double z = lrow[ax] * dt;
    double ph[5];
    etd4_phi(z, ph);
    const double P1 = dt * ph[1];
    const double P2 = dt * ph[2];
    const double P3 = dt * (0.5 * ph[2] + ph[3]);
    const double P4 = dt * ((ph[2] / 3.0 + ph[3]) + ph[4]);
    const double mk2 = -k2;
    co[0] = (T)ph[0];
    co[1] = (T)(mk2 * P1);
    co[2] = (T)(mk2 * P2);
    co[3] = (T)(mk2 * P3);
    co[4] = (T)(mk2 * P4);
}

// one real component: psi' from psi and H_n .. H_{n-3}, terms in the order of
// the update formula
template <typename T>
__device__ __forceinline__ T xpfc_cand1(const T (&co)[5], T q, T h0, T h1, T h2, T h3) {
    const T d1 = h0 - h1;
    const T d2 = fmat((T)-2, h1, h0) + h2;
    const T d3 = fmat((T)3, h2, fmat((T)-3, h1, h0)) - h3;
    T acc = co[0] * q;
    acc = fmat(co[1], h0, acc);
    acc = fmat(co[2], d1, acc);
    acc = fmat(co[3], d2, acc);
    acc = fmat(co[4], d3, acc);
    return acc;
}

// -------------------------------------------------------------------------
// deterministic reductions
// -------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum over the workgroup in a fixed order: butterfly within each wave, then
// wave totals added in wave order by thread 0.  Result valid in thread 0.
template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ], double *lds /* [NQ][16] */) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NQ; ++q) lds[q * 16 + w] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double t = 0.0;
            for (int i = 0; i < nw; ++i) t += lds[q * 16 + i];
            v[q] = t;
        }
    }
}

// -------------------------------------------------------------------------
// fused real-space nonlinear term (one pass, in place on the transform buffer)
// -------------------------------------------------------------------------

template <typename T, int OP>
__global__ void __launch_bounds__(1024) k_nonlinear(Ctx c) {
    constexpr int V = CV<T>::V;
    constexpr int TE = tile_elems<T>();
    __shared__ double lds[2 * 16];
    const int64_t tile = blockIdx.x;
    const int ii = find_by_offset(c.inst, c.n_inst, tile, 1);
    const InstDev &I = c.inst[ii];
    const int64_t t0 = (tile - I.tile_off) * TE;
    T *base = reinterpret_cast<T *>(OP == OP_NLSE ? c.state : c.work) + 2 * I.off;
    double acc[2] = {0.0, 0.0};
    if (OP == OP_CH) {
        const T invN = (T)I.invN;
        if (I.k0path) {
            // W holds N (c - cbar) (the k = 0 slot is 0).  The nonlinear term is
            // expanded about the FP64 mean, f'(cbar + d) - f'(cbar) =
            // d (3 cbar^2 - 1 + d (3 cbar + d)), so c = cbar + d is never rounded
            // to FP32; the dropped constant only reaches k = 0, which the FP64
            // side path carries.  The FP64 sums use the full c.
            const double cbar = c.k0[2 * ii] * I.invN;
            const T A1 = (T)(3.0 * cbar * cbar - 1.0), A2 = (T)(3.0 * cbar);
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= I.N) break;
                T re[V], im[V];
                CV<T>::ld(base + 2 * e, re, im);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T d = re[v] * invN;
                    re[v] = d * (A1 + d * (A2 + d));
                    im[v] = (T)0;
                    const double cd = cbar + (double)d;
                    const double t = cd * cd - 1.0;
                    acc[0] += 0.25 * (t * t);
                    acc[1] += cd * cd * cd - cd;
                }
                CV<T>::st(base + 2 * e, re, im);
            }
        } else {
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= I.N) break;
                T re[V], im[V];
                CV<T>::ld(base + 2 * e, re, im);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T cc = re[v] * invN;
                    re[v] = cc * cc * cc - cc;
                    im[v] = (T)0;
                    const double cd = (double)cc;
                    const double t = cd * cd - 1.0;
                    acc[0] += 0.25 * (t * t);
                    acc[1] += (double)re[v];
                }
                CV<T>::st(base + 2 * e, re, im);
            }
        }
    } else if (OP == OP_GS) {
        const T invN = (T)I.invN;
        const T F = (T)I.q0, Fk = (T)(I.q0 + I.q1);
        T *bu = base, *bv = base + 2 * I.N;
        if (I.k0path) {
            // deviations from the FP64 means: with P = uv^2 - ubar vbar^2 =
            // ubar dv (2 vbar + dv) + du v^2, R_u - R_u(means) = -P - F du and
            // R_v - R_v(means) = P - (F + k) dv; the constants only reach k = 0.
            // The FP64 sums (the k = 0 right-hand side) use the full u, v.
            const double ub = c.k0[2 * ii] * I.invN, vb = c.k0[2 * ii + 1] * I.invN;
            const T Uf = (T)ub, Vf = (T)vb, V2 = (T)(2.0 * vb);
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= I.N) break;
                T ur[V], ui[V], vr[V], vi[V];
                CV<T>::ld(bu + 2 * e, ur, ui);
                CV<T>::ld(bv + 2 * e, vr, vi);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T du = ur[v] * invN, dv = vr[v] * invN;
                    const T vv = Vf + dv;
                    const T P = Uf * (dv * (V2 + dv)) + du * (vv * vv);
                    ur[v] = -P - F * du;
                    vr[v] = P - Fk * dv;
                    ui[v] = (T)0;
                    vi[v] = (T)0;
                    const double u64 = ub + (double)du, v64 = vb + (double)dv;
                    const double uvv = u64 * v64 * v64;
                    acc[0] += -uvv + I.q0 * (1.0 - u64);
                    acc[1] += uvv - (I.q0 + I.q1) * v64;
                }
                CV<T>::st(bu + 2 * e, ur, ui);
                CV<T>::st(bv + 2 * e, vr, vi);
            }
        } else {
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= I.N) break;
                T ur[V], ui[V], vr[V], vi[V];
                CV<T>::ld(bu + 2 * e, ur, ui);
                CV<T>::ld(bv + 2 * e, vr, vi);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T u = ur[v] * invN;
                    const T w = vr[v] * invN;
                    const T uvv = u * w * w;
                    ur[v] = -uvv + F * ((T)1 - u);
                    vr[v] = uvv - Fk * w;
                    ui[v] = (T)0;
                    vi[v] = (T)0;
                    acc[0] += (double)ur[v];
                    acc[1] += (double)vr[v];
                }
                CV<T>::st(bu + 2 * e, ur, ui);
                CV<T>::st(bv + 2 * e, vr, vi);
            }
        }
    } else if (OP == OP_XPFC) {
        // H = F[-(omega/2) psi^2 + (u/3) psi^3] (Supplementary S3.1); q0 = omega, q1 = u
        const T invN = (T)I.invN;
        if (I.k0path) {
            // W holds N (psi - psibar); expanded about the FP64 mean, the
            // term is d (a1 + d (a2 + d a3)) plus a constant that only
            // reaches k = 0, where the update's nonlinear coefficients are 0
            const double pb = c.k0[2 * ii] * I.invN;
            const T a1 = (T)(I.q1 * (pb * pb) - I.q0 * pb), a2 = (T)(I.q1 * pb - 0.5 * I.q0), a3 = (T)(I.q1 / 3.0);
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= I.N) break;
                T re[V], im[V];
                CV<T>::ld(base + 2 * e, re, im);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T d = re[v] * invN;
                    re[v] = d * fmat(d, fmat(d, a3, a2), a1);
                    im[v] = (T)0;
                }
                CV<T>::st(base + 2 * e, re, im);
            }
        } else {
            const T hw = (T)(-(I.q0 / 2.0)), u3 = (T)(I.q1 / 3.0);
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= I.N) break;
                T re[V], im[V];
                CV<T>::ld(base + 2 * e, re, im);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T ps = re[v] * invN;
                    const T t = ps * ps;
                    re[v] = hw * t + u3 * (t * ps);
                    im[v] = (T)0;
                }
                CV<T>::st(base + 2 * e, re, im);
            }
        }
    } else {
        const T sc = (T)(I.invN * I.invN);  // stored field carries a factor N^2 here
        const T gh = (T)I.q0;
        for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
            const int64_t e = t0 + j;
            if (e >= I.N) break;
            T re[V], im[V];
            CV<T>::ld(base + 2 * e, re, im);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const T er = re[v] * sc, ei = im[v] * sc;
                const T ph = gh * (er * er + ei * ei);
                T sn, cs;
                sc_t(ph, sn, cs);
                re[v] = er * cs - ei * sn;
                im[v] = er * sn + ei * cs;
            }
            CV<T>::st(base + 2 * e, re, im);
        }
        return;
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        c.nl_part[2 * tile] = acc[0];
        c.nl_part[2 * tile + 1] = acc[1];
    }
}

// FP64 totals of the per-tile partials of each instance, fixed order.
// mode 0: nonlinear right-hand side at k = 0 (GS) -> rhs_k0; mode 1: field
// sums -> k0 (set_field).
__global__ void __launch_bounds__(256) k_k0_total(Ctx c, int mode, int only_inst) {
    __shared__ double lds[2 * 16];
    const int ii = only_inst >= 0 ? only_inst : (int)blockIdx.x;
    const InstDev &I = c.inst[ii];
    double acc[2] = {0.0, 0.0};
    for (int64_t t = threadIdx.x; t < I.ntiles; t += blockDim.x) {
        acc[0] += c.nl_part[2 * (I.tile_off + t)];
        acc[1] += c.nl_part[2 * (I.tile_off + t) + 1];
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        double *dst = mode == 0 ? c.rhs_k0 : c.k0;
        dst[2 * ii] = acc[0];
        dst[2 * ii + 1] = I.nspec > 1 ? acc[1] : 0.0;
    }
}

// Strip geometry in registers: the instance fields a row walk needs.
struct Geo {
    int lch, lb1, b1m, ln1, ln2, n0, n1, n2, z0, y0;
    __device__ static Geo of(const InstDev &I, int sbz, int sby) {
        Geo g;
        g.lch = I.lchunks;
        g.lb1 = I.lb[1];
        g.b1m = I.b[1] - 1;
        g.ln1 = I.ln[1];
        g.ln2 = I.ln[2];
        g.n0 = I.n[0];
        g.n1 = I.n[1];
        g.n2 = I.n[2];
        g.z0 = sbz << I.lb[0];
        g.y0 = sby << I.lb[1];
        return g;
    }
};

// -------------------------------------------------------------------------
// indicator: one workgroup per strip of S x-adjacent blocks; its waves split
// the rows of the strip; lanes cover 16 contiguous bytes each.
// -------------------------------------------------------------------------

// Row walk of one strip for the indicator.  MC: a block row spans several
// 64-lane chunks (one block per strip); otherwise every lane keeps its x for
// the whole strip and its |m_x|^2 is computed once.  Lanes that are off
// (beyond a narrow strip, or in the skip set) never load: their registers stay
// zero, which every operator maps to a zero increment and zero energy.
// HT: every instance has an H table (one-dimensional NLSE plans), so the
// evaluation path is not compiled in.  SI: the state-amplitude measure
// a(k) = sum over species of |q(k)|^2 (no right-hand side read, no
// candidate); z_lane marks the lane holding k = 0, which it leaves out.
template <typename T, int OP, bool MC, bool HT = false, bool SI = false>
__device__ __forceinline__ void indicator_rows(const Ctx &c, const InstDev &I, int ii, int sbz, int sby,
                                               int x_lane, bool lane_on, bool k0_lane, int w, int nw,
                                               bool want_eb, double &amax, double &esum, double &ebs,
                                               bool &bad, bool z_lane = false) {
    constexpr int V = CV<T>::V;
    // rows in flight per wave (GS: two species, half; the state measure reads no
    // right-hand side, so it keeps twice the rows in flight)
    constexpr int U = (SI ? 2 : 1) * (OP == OP_GS ? 2 : 4);
    // every instance field the row loop needs, read once (fields first read
    // inside the predicated load block would be re-fetched row by row)
    const Geo g = Geo::of(I, sbz, sby);
    const Coef K = Coef::of(I);
    const int chunks = I.chunks;
    const int total_it = (I.b[0] * I.b[1]) << g.lch;
    const T *q0p = reinterpret_cast<const T *>(c.state) + 2 * I.off;
    const T *r0p = reinterpret_cast<const T *>(c.rhs) + 2 * I.off;
    const T *q1p = q0p + 2 * I.N;
    const T *r1p = r0p + 2 * I.N;
    const T c0s = (OP == OP_GS) ? (T)K.c0 : (T)0;
    // NLSE in one dimension: H from the table, into the (otherwise unused)
    // right-hand-side registers
    const T *htab = (OP == OP_NLSE && (HT || I.ht_off >= 0)) ? reinterpret_cast<const T *>(c.htab) + 2 * I.ht_off
                                                             : nullptr;
    double mx2[V];
#pragma unroll
    for (int v = 0; v < V; ++v) mx2[v] = sq_d(sidx(x_lane + v, g.n2));
    T qr[U][V], qi[U][V], nr[U][V], ni[U][V], q2r[U][V], q2i[U][V], n2r[U][V], n2i[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            qr[u][v] = qi[u][v] = nr[u][v] = ni[u][v] = (T)0;
            q2r[u][v] = q2i[u][v] = n2r[u][v] = n2i[u][v] = (T)0;
        }
    for (int it0 = w; it0 < total_it; it0 += nw * U) {
        double myz[U];
        int xs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int it = it0 + u * nw;  // wave-uniform
            const int r = MC ? it >> g.lch : it, ch = MC ? it & (chunks - 1) : 0;
            const int z = g.z0 + (r >> g.lb1);
            const int y = g.y0 + (r & g.b1m);
            const int x = x_lane + ch * 64 * V;
            xs[u] = x;
            myz[u] = sq_d(sidx(z, g.n0)) + sq_d(sidx(y, g.n1));
            if (it < total_it && lane_on) {
                const int64_t e = ((((int64_t)z << g.ln1) + y) << g.ln2) + x;
                CV<T>::ld(q0p + 2 * e, qr[u], qi[u]);
                if (SI) {
                } else if (OP != OP_NLSE) CV<T>::ld(r0p + 2 * e, nr[u], ni[u]);
                else if (htab) nlse_tab_ld<T>(htab, x, g.n2, nr[u], ni[u]);
                if (OP == OP_GS) {
                    CV<T>::ld(q1p + 2 * e, q2r[u], q2i[u]);
                    if (!SI) CV<T>::ld(r1p + 2 * e, n2r[u], n2i[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (it0 + u * nw >= total_it) continue;  // wave-uniform
#pragma unroll
            for (int v = 0; v < V; ++v) {
                double m2;
                if (MC) {
                    const double mx = (double)sidx(xs[u] + v, g.n2);
                    m2 = __builtin_fma(mx, mx, myz[u]);
                } else {
                    m2 = myz[u] + mx2[v];
                }
                double a;
                if (SI) {
                    a = sq2((double)qr[u][v], (double)qi[u][v]);
                    if (OP == OP_GS) a = a + sq2((double)q2r[u][v], (double)q2i[u][v]);
                    if (v == 0 && u == 0 && z_lane && it0 == 0) a = 0.0;  // k = 0 is left out
                    if (OP == OP_CH) esum += (K.K2 * m2) * sq2((double)qr[u][v], (double)qi[u][v]);
                } else if (OP == OP_CH) {
                    T s, f, cr, ci;
                    ch_coef<T>(K, m2, s, f);
                    a = ch_cand<T>(s, f, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
                    esum += (K.K2 * m2) * sq2((double)qr[u][v], (double)qi[u][v]);
                } else if (OP == OP_GS) {
                    T au, av, cr, ci;
                    gs_coef<T>(K, m2, au, av);
                    a = gs_cand<T>(c0s, au, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
                    a = a + gs_cand<T>(c0s, av, q2r[u][v], q2i[u][v], n2r[u][v], n2i[u][v], cr, ci);
                } else {
                    T hr = nr[u][v], hi = ni[u][v], cr, ci;
                    if (!HT && !htab) nlse_coef<T>(K, m2, hr, hi);
                    a = nlse_cand<T>(hr, hi, qr[u][v], qi[u][v], cr, ci);
                }
                // the FP32 slot of k = 0 (real-field operators) is held at
                // zero; its increment comes from the FP64 side path
                const bool k0s = v == 0 && u == 0 && k0_lane && it0 == 0;
                a = k0s ? 0.0 : a;
                bad |= !(a <= DBL_MAX);
                if (SI && c.ab_sum) amax = amax + a;  // block energy: the lane's sum, rows in order
                else amax = fmax(amax, a);
                if (want_eb) {
                    double e2 = sq2((double)qr[u][v], (double)qi[u][v]);
                    if (OP == OP_GS) e2 += sq2((double)q2r[u][v], (double)q2i[u][v]);
                    ebs += k0s ? 0.0 : e2;
                }
            }
        }
    }
}

// EB: per-block energies requested (c.e_b set; proposer audits).  Without
// them the kernel carries neither the accumulation nor its LDS array.
template <typename T, int OP, bool EB, bool SI>
__global__ void __launch_bounds__(1024) k_indicator(Ctx c) {
    constexpr int V = CV<T>::V;
    __shared__ double lds_max[16][64];
    __shared__ double lds_eb[EB ? 16 : 1][64];
    __shared__ double lds_sum[16];
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    // wave index made scalar: the row loop is then uniform per wave and
    // compiles to scalar branches, so no exec-mask joins split the loads
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t strip = blockIdx.x;
    const int ii = find_by_offset(c.inst, c.n_inst, strip, 0);
    const InstDev &I = c.inst[ii];
    const int64_t ls = strip - I.strip_off;
    const int lnsx = I.lnbk[2] - I.lS;  // log2 strips per block row
    const int sx = (int)(ls & ((1 << lnsx) - 1));
    const int64_t t = ls >> lnsx;
    const int sby = (int)(t & ((1 << I.lnbk[1]) - 1));
    const int sbz = (int)(t >> I.lnbk[1]);
    const int chunks = I.chunks;
    const int x_lane = ((sx << I.lS) << I.lb[2]) + lane * V;  // x of this lane in chunk 0
    // lanes beyond the strip width stay idle (narrow grids); lanes whose block
    // is in the skip set issue no loads at all
    const int LB = chunks > 1 ? 64 : (I.b[2] / V);
    const int lane_bx = (sx << I.lS) + (chunks > 1 ? 0 : lane / LB);
    const int64_t lane_lb = ((((int64_t)sbz << I.lnbk[1]) + sby) << I.lnbk[2]) + lane_bx;
    bool lane_on = chunks > 1 || lane * V < (I.S << I.lb[2]);
    if (lane_on && c.skip && c.skip[I.blk_off + lane_lb] && !(I.pin && lane_lb == 0)) lane_on = false;
    const bool k0_lane = I.k0path && ls == 0 && lane == 0;
    const bool z_lane = ls == 0 && lane == 0;

    double amax = 0.0, esum = 0.0, ebs = 0.0;
    constexpr bool want_eb = EB;
    bool bad = false;
    if (chunks > 1)
        indicator_rows<T, OP, true, false, SI>(c, I, ii, sbz, sby, x_lane, lane_on, k0_lane, w, nw, want_eb, amax,
                                               esum, ebs, bad, z_lane);
    else
        indicator_rows<T, OP, false, false, SI>(c, I, ii, sbz, sby, x_lane, lane_on, k0_lane, w, nw, want_eb, amax,
                                                esum, ebs, bad, z_lane);
    if (k0_lane && w == 0) {
        double tmp[2];
        // the state measure leaves k = 0 out; the increment rule takes its
        // FP64 candidate
        const double a = SI ? 0.0 : k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
        bad |= !(a <= DBL_MAX);
        amax = fmax(amax, a);
        if (want_eb)
            for (int s = 0; s < I.nspec; ++s) ebs += c.k0[2 * ii + s] * c.k0[2 * ii + s];
    }
    // per-block maximum (block energy: sum) over the lanes of the block, then
    // over the waves in wave order
    const bool esum_b = SI && c.ab_sum;
    for (int off = 1; off < LB; off <<= 1) {
        const double o = __shfl_xor(amax, off, 64);
        amax = esum_b ? amax + o : fmax(amax, o);
    }
    lds_max[w][lane] = amax;
    if (want_eb) {
        for (int off = 1; off < LB; off <<= 1) ebs += __shfl_xor(ebs, off, 64);
        lds_eb[w][lane] = ebs;
    }
    if (OP == OP_CH) {
        esum = wave_sum(esum);
        if (lane == 0) lds_sum[w] = esum;
    }
    if (bad) atomicOr(c.nonfinite, 1u);
    __syncthreads();
    if (w == 0) {
        double m = lds_max[0][lane];
        for (int i = 1; i < nw; ++i) m = esum_b ? m + lds_max[i][lane] : fmax(m, lds_max[i][lane]);
        const int nblk = chunks > 1 ? 1 : I.S;
        if (lane % LB == 0 && lane / LB < nblk) {
            const int bx = (sx << I.lS) + lane / LB;
            const int64_t lb = ((((int64_t)sbz << I.lnbk[1]) + sby) << I.lnbk[2]) + bx;
            const int64_t gb = I.blk_off + lb;
            const bool skipped = c.skip && c.skip[gb] && !(I.pin && lb == 0);
            c.a_b[gb] = skipped ? 0.0 : m;
            if (skipped) m = 0.0;
            if (want_eb) {
                double es = 0.0;
                for (int i = 0; i < nw; ++i) es += lds_eb[i][lane];
                c.e_b[gb] = skipped ? 0.0 : es;
            }
        } else {
            m = 0.0;
        }
        const double sm = wave_max(m);
        if (lane == 0) {
            if (strip == 0) *c.count = 0u;  // the one-pass compaction appends to it
            c.strip_max[strip] = sm;  // lets the update drop whole frozen strips
            if (sm > 0.0) atomicMax(c.G + ii, (unsigned long long)__double_as_longlong(sm));
        }
        if (OP == OP_CH && lane == 0) {
            double tsum = 0.0;
            for (int i = 0; i < nw; ++i) tsum += lds_sum[i];
            c.ind_part[strip] = tsum;
        }
    }
}

// Indicator for plans whose block rows span several wave rows (1-D blocks of
// 1024 bins, say): each such strip is one block, and one wave takes a whole
// strip -- every row and chunk, four in flight -- so the data path has no LDS
// and no barrier.  The instance maxima of the workgroup's waves are combined
// in LDS and sent with one atomic per instance: device-scope atomics on G
// serialise (all instances' G share a cache line), so one per strip would cap
// the rate at short strips.
template <typename T, int OP, bool EB, bool HT, bool SI>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) k_indicator_wave(Ctx c) {
    __shared__ double s_m[16];
    __shared__ int s_i[16];
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t strip = (int64_t)blockIdx.x * nw + w;
    double m = 0.0;
    int ii = -1;
    if (strip < c.n_strips) {  // wave-uniform
        // one block per strip: strip ids are block ids, so the owning
        // instance is one table read (no search over the instances)
        ii = __builtin_amdgcn_readfirstlane(c.blk_inst[strip]);
        const InstDev &I = c.inst[ii];
        const int64_t ls = strip - I.strip_off;
        const int sx = (int)(ls & ((1 << I.lnbk[2]) - 1));
        const int64_t t = ls >> I.lnbk[2];
        const int sby = (int)(t & ((1 << I.lnbk[1]) - 1));
        const int sbz = (int)(t >> I.lnbk[1]);
        const int x_lane = (sx << I.lb[2]) + lane * CV<T>::V;
        const int64_t gb = I.blk_off + ls;
        const bool skipped = c.skip && c.skip[gb] && !(I.pin && ls == 0);
        const bool k0_lane = I.k0path && ls == 0 && lane == 0;
        double amax = 0.0, esum = 0.0, ebs = 0.0;
        bool bad = false;
        indicator_rows<T, OP, true, HT, SI>(c, I, ii, sbz, sby, x_lane, !skipped, k0_lane, 0, 1, EB, amax, esum,
                                            ebs, bad, ls == 0 && lane == 0);
        if (k0_lane) {
            double tmp[2];
            const double a = SI ? 0.0 : k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
            bad |= !(a <= DBL_MAX);
            amax = fmax(amax, a);
            if (EB)
                for (int sp = 0; sp < I.nspec; ++sp) ebs += c.k0[2 * ii + sp] * c.k0[2 * ii + sp];
        }
        amax = (SI && c.ab_sum) ? wave_sum(amax) : wave_max(amax);  // block energy: the sum
        if (OP == OP_CH) esum = wave_sum(esum);
        if (EB) ebs = wave_sum(ebs);
        if (__any(bad) && lane == 0) atomicOr(c.nonfinite, 1u);
        m = skipped ? 0.0 : amax;
        if (lane == 0) {
            c.a_b[gb] = m;
            if (EB) c.e_b[gb] = skipped ? 0.0 : ebs;
            if (strip == 0) *c.count = 0u;  // the one-pass compaction appends to it
            c.strip_max[strip] = m;
            if (OP == OP_CH) c.ind_part[strip] = esum;
        }
    }
    if (lane == 0) {
        s_m[w] = m;
        s_i[w] = ii;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // runs of one instance (its strips are contiguous)
        int cur = -1;
        double cm = 0.0;
        for (int k = 0; k <= nw; ++k) {
            const int ik = k < nw ? s_i[k] : -1;
            if (ik != cur) {
                if (cur >= 0 && cm > 0.0) atomicMax(c.G + cur, (unsigned long long)__double_as_longlong(cm));
                cur = ik;
                cm = 0.0;
            }
            if (k < nw) cm = fmax(cm, s_m[k]);
        }
    }
}

// Incremental state measure: the blocks the previous update stored (mask
// nonzero) take the measure the update kernel wrote for them, the others keep
// theirs; G of every instance is the maximum.  Each thread takes GMAX_PER = 8
// consecutive blocks and issues their loads at once (one 8-byte mask word,
// 64 bytes of a_b and of a_next); a wave whose blocks lie in one instance
// reduces them, and the workgroup sends one atomic per instance of its waves
// (device-scope atomics on one address serialise, so one per wave would
// dominate the kernel); threads whose blocks span instances send their own.
// Clears the append counter, as the indicator does.
constexpr int GMAX_PER = 8;
__global__ void __launch_bounds__(256) k_gmax(Ctx c) {
    __shared__ double wmax[4];
    __shared__ int winst[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t b0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * GMAX_PER;
    if (b0 == 0) *c.count = 0u;
    double v = 0.0;
    int ii = -1;  // instance of every block of this thread, -2 if they differ
    if (b0 + GMAX_PER <= c.nb_total) {  // whole group: vector loads (nb_total is not always a multiple of 8)
        const uint64_t mw = *reinterpret_cast<const uint64_t *>(c.mask + b0);
        double a[GMAX_PER], an[GMAX_PER];
#pragma unroll
        for (int k = 0; k < GMAX_PER; k += 2) {
            const double2 x = *reinterpret_cast<const double2 *>(c.a_b + b0 + k);
            const double2 y = *reinterpret_cast<const double2 *>(c.a_next + b0 + k);
            a[k] = x.x;
            a[k + 1] = x.y;
            an[k] = y.x;
            an[k + 1] = y.y;
        }
#pragma unroll
        for (int k = 0; k < GMAX_PER; ++k) {
            if ((mw >> (8 * k)) & 0xFFull) {
                a[k] = an[k];
                c.a_b[b0 + k] = a[k];
            }
            v = fmax(v, a[k]);
        }
        ii = c.blk_inst[b0];
        if (c.blk_inst[b0 + GMAX_PER - 1] != ii) ii = -2;
    } else {
        for (int64_t gb = b0; gb < c.nb_total; ++gb) {
            double a = c.a_b[gb];
            if (c.mask[gb]) {
                a = c.a_next[gb];
                c.a_b[gb] = a;
            }
            const int ib = c.blk_inst[gb];
            ii = (ii == -1 || ii == ib) ? ib : -2;
            v = fmax(v, a);
        }
    }
    if (ii == -2) {  // this thread's blocks span instances: one atomic per block
        for (int64_t gb = b0; gb < b0 + GMAX_PER && gb < c.nb_total; ++gb) {
            const double a = c.a_b[gb];
            if (a > 0.0) atomicMax(c.G + c.blk_inst[gb], (unsigned long long)__double_as_longlong(a));
        }
    }
    // lanes with no block (ii == -1) or spanning ones (-2) join with value 0
    int i0 = __shfl(ii, 0, 64);
    if (i0 < 0) {  // the first lane with a single-instance group names the wave's instance
        const uint64_t ok = __ballot(ii >= 0);
        i0 = ok ? __shfl(ii, __builtin_ctzll(ok), 64) : -1;
    }
    const bool uni = i0 >= 0 && __all(ii == i0 || ii < 0);
    double m = 0.0;
    if (uni) {
        m = wave_max(ii >= 0 ? v : 0.0);
    } else if (ii >= 0 && v > 0.0) {
        atomicMax(c.G + ii, (unsigned long long)__double_as_longlong(v));
    }
    if (lane == 0) {
        wmax[w] = m;
        winst[w] = uni ? i0 : -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 4; ++k) {
            if (winst[k] < 0) continue;
            double mm = wmax[k];
            for (int q = k + 1; q < 4; ++q)
                if (winst[q] == winst[k]) {
                    mm = fmax(mm, wmax[q]);
                    winst[q] = -1;
                }
            if (mm > 0.0) atomicMax(c.G + winst[k], (unsigned long long)__double_as_longlong(mm));
        }
    }
}

// -------------------------------------------------------------------------
// compaction: chunk counts, then ordered write of the active-block list
// -------------------------------------------------------------------------

__device__ __forceinline__ bool block_active(const Ctx &c, int64_t gb) {
    const int ii = c.blk_inst[gb];
    const InstDev &I = c.inst[ii];
    const int64_t lb = gb - I.blk_off;
    if (c.dense) return true;
    if (I.pin && lb == 0) return true;
    if (c.skip && c.skip[gb]) return false;
    const double G = __longlong_as_double((long long)c.G[ii]);
    const double thr = I.tau2 * G;
    return c.a_b[gb] > thr;
}

__global__ void __launch_bounds__(256) k_compact_count(Ctx c, int from_mask) {
    __shared__ uint32_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * CHUNK_BLOCKS;
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < CHUNK_BLOCKS / 256; ++k) {
        const int64_t gb = base + k * 256 + threadIdx.x;
        if (gb < c.nb_total) {
            bool on;
            if (from_mask) {
                on = c.mask[gb] != 0;
            } else {
                on = block_active(c, gb);
                c.mask[gb] = on ? 1 : 0;
            }
            n += on ? 1u : 0u;
        }
    }
    // integer sum: order-free
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) n += __shfl_xor(n, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) c.chunk_cnt[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

__global__ void __launch_bounds__(256) k_compact_write(Ctx c) {
    __shared__ uint32_t scan[256];
    __shared__ uint32_t red[4];
    const int64_t chunk = blockIdx.x;
    // offset = sum of the counts of the preceding chunks
    uint32_t pre = 0;
    for (int64_t k = threadIdx.x; k < chunk; k += 256) pre += c.chunk_cnt[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) pre += __shfl_xor(pre, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pre;
    // each thread owns 4 consecutive blocks of the chunk
    const int64_t b0 = chunk * CHUNK_BLOCKS + 4 * threadIdx.x;
    uint32_t bits = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (b0 + k < c.nb_total && c.mask[b0 + k]) bits |= 1u << k;
    const uint32_t mine = __popc(bits);
    scan[threadIdx.x] = mine;
    __syncthreads();
    const uint32_t offset = red[0] + red[1] + red[2] + red[3];
    // inclusive Hillis-Steele scan over 256 entries
    for (int d = 1; d < 256; d <<= 1) {
        const uint32_t v = threadIdx.x >= d ? scan[threadIdx.x - d] : 0u;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t pos = offset + scan[threadIdx.x] - mine;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (bits & (1u << k)) c.worklist[pos++] = (uint32_t)(b0 + k);
    if (chunk == c.n_chunks - 1 && threadIdx.x == 255) *c.count = offset + scan[255];
}

// Append the blocks flagged in `bits` (thread t owns blocks b0..b0+3) to the
// unordered list: exclusive prefix within the wave (shift-up scan), then
// across the four waves, then one atomic per workgroup.
__device__ __forceinline__ void append_bits(const Ctx &c, uint32_t bits, int64_t b0, uint32_t *wsum,
                                            uint32_t &base) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t mine = __popc(bits);
    uint32_t incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d, 64);
        if (lane >= d) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        base = tot ? atomicAdd(c.count, tot) : 0u;
    }
    __syncthreads();
    uint32_t pos = base + incl - mine;
    for (int i = 0; i < w; ++i) pos += wsum[i];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (bits & (1u << k)) c.worklist[pos++] = (uint32_t)(b0 + k);
}

// One-pass compaction for the update: threshold and mask of a chunk of 1024
// blocks, then one atomic append of the chunk's active blocks (ascending
// within the chunk).  The update needs no global order; the ordered list the
// API returns is rebuilt from the mask when it is read.  The last workgroup to
// arrive hands G over, as the strip walk does (not when G_last is null: the
// block-activity stage of the other plan types keeps G).  The indicator clears
// the counter.
__global__ void __launch_bounds__(256) k_compact_append(Ctx c) {
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t base;
    const int64_t b0 = (int64_t)blockIdx.x * CHUNK_BLOCKS + 4 * threadIdx.x;
    uint32_t bits = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t gb = b0 + k;
        if (gb < c.nb_total) {
            const bool on = block_active(c, gb);
            c.mask[gb] = on ? 1 : 0;
            bits |= (on ? 1u : 0u) << k;
        }
    }
    append_bits(c, bits, b0, wsum, base);
    // every G read of this workgroup happened before the barriers above
    if (c.G_last && threadIdx.x == 0) {
        const unsigned int done = atomicAdd(c.done, 1u);
        if (done == gridDim.x - 1) {
            for (int i = 0; i < c.n_inst; ++i) {
                c.G_last[i] = c.G[i];
                c.G[i] = 0ull;
            }
            *c.done = 0u;
        }
    }
}

// -------------------------------------------------------------------------
// consistency control (Supplementary S1.1, S1.3): transition blocks, the
// roll-off weights, the step schedule and the threshold controller
// -------------------------------------------------------------------------

// instance-local block id from block coordinates (power-of-two block grid)
__device__ __forceinline__ int64_t blk_id(const InstDev &I, int bz, int by, int bx) {
    return ((((int64_t)bz << I.lnbk[1]) + by) << I.lnbk[2]) + bx;
}

// Threshold rule of a control plan for instance-local block lb: every block
// in a full step, the pinned k = 0 block, else a_b > fl(tau^2 G) with the
// controlled threshold (skipped blocks never).
__device__ __forceinline__ bool active_ctl(const Ctx &c, const InstDev &I, int64_t lb, double thr, bool full) {
    if (full) return true;
    if (I.pin && lb == 0) return true;
    const int64_t gb = I.blk_off + lb;
    if (c.skip && c.skip[gb]) return false;
    return c.a_b[gb] > thr;
}

// threshold rule of a neighbour (never in a full step: there no block is
// left inactive); a_b is loaded unconditionally so that the six neighbour
// loads issue together
__device__ __forceinline__ bool nb_on(const Ctx &c, const InstDev &I, int64_t lb, double thr) {
    const int64_t gb = I.blk_off + lb;
    bool on = c.a_b[gb] > thr;
    if (c.skip) on = on && !c.skip[gb];
    return on || (I.pin && lb == 0);
}

// a block with an active face neighbour (periodic block grid)
__device__ __forceinline__ bool near_active(const Ctx &c, const InstDev &I, int64_t lb, double thr) {
    const int bx = (int)(lb & (I.nbk[2] - 1));
    const int64_t t = lb >> I.lnbk[2];
    const int by = (int)(t & (I.nbk[1] - 1));
    const int bz = (int)(t >> I.lnbk[1]);
    bool nr = false;
    if (I.nbk[0] > 1) {
        const int k = I.nbk[0] - 1;
        nr = nr | nb_on(c, I, blk_id(I, (bz - 1) & k, by, bx), thr);
        nr = nr | nb_on(c, I, blk_id(I, (bz + 1) & k, by, bx), thr);
    }
    if (I.nbk[1] > 1) {
        const int k = I.nbk[1] - 1;
        nr = nr | nb_on(c, I, blk_id(I, bz, (by - 1) & k, bx), thr);
        nr = nr | nb_on(c, I, blk_id(I, bz, (by + 1) & k, bx), thr);
    }
    if (I.nbk[2] > 1) {
        const int k = I.nbk[2] - 1;
        nr = nr | nb_on(c, I, blk_id(I, bz, by, (bx - 1) & k), thr);
        nr = nr | nb_on(c, I, blk_id(I, bz, by, (bx + 1) & k), thr);
    }
    return nr;
}

// Half-spectrum layout: the stored blocks standing for the neighbour across
// face f (0 z low, 1 z high, 2 y low, 3 y high, 4 x low, 5 x high) of the
// stored block (bz, by, bx), bx = nbxm for the column nx/2.  z and y are
// periodic; along x the stored columns are a chain X_0 .. X_{nbxm-1}, X_N,
// and a neighbour in the omitted half is its conjugate counterpart, mode by
// mode: across kx = 0 the blocks of X_0 at the mirrored rows -y, -z, beyond
// nx/2 the blocks of X_{nbxm-1} at the mirrored rows, and X_{nbxm-1} meets
// X_N at its own and at the mirrored rows (the column nx/2 holds each of its
// modes at y and -y).  Rows of block i mirror into blocks (nb - i) mod nb and
// (nb - i - 1) mod nb.  Returns the count (at most 5; 0 for an axis with one
// block).
__device__ __forceinline__ int64_t half_blk(const InstDev &I, int bz, int by, int bx) {
    const int64_t row = ((int64_t)bz << I.lnbk[1]) + by;
    return bx == I.nbxm ? I.nbm + row : (row << I.lnbxm) + bx;
}
__device__ __forceinline__ int half_mirrored(const InstDev &I, int bz, int by, int bx, int64_t *out, int n) {
    const int nz0 = (I.nbk[0] - bz) & (I.nbk[0] - 1), ny0 = (I.nbk[1] - by) & (I.nbk[1] - 1);
    const int mz[2] = {nz0, (nz0 - 1) & (I.nbk[0] - 1)}, my[2] = {ny0, (ny0 - 1) & (I.nbk[1] - 1)};
    const int cz = (I.b[0] > 1 && mz[1] != mz[0]) ? 2 : 1, cy = (I.b[1] > 1 && my[1] != my[0]) ? 2 : 1;
    for (int i = 0; i < cz; ++i)
        for (int k = 0; k < cy; ++k) {
            const int64_t id = half_blk(I, mz[i], my[k], bx);
            bool dup = false;
            for (int j = 0; j < n; ++j) dup |= out[j] == id;
            if (!dup) out[n++] = id;
        }
    return n;
}
__device__ __forceinline__ int half_face(const InstDev &I, int bz, int by, int bx, int f, int64_t *out) {
    const int a = f >> 1;
    const int d = (f & 1) ? 1 : -1;
    if (a < 2) {
        const int nb = I.nbk[a];
        if (nb < 2) return 0;
        if (a == 0) out[0] = half_blk(I, (bz + d) & (nb - 1), by, bx);
        else out[0] = half_blk(I, bz, (by + d) & (nb - 1), bx);
        return 1;
    }
    if (d < 0) {
        if (bx > 0) {
            out[0] = half_blk(I, bz, by, bx - 1);
            return 1;
        }
        return half_mirrored(I, bz, by, 0, out, 0);  // across kx = 0
    }
    if (bx == I.nbxm) return half_mirrored(I, bz, by, I.nbxm - 1, out, 0);  // beyond nx/2
    out[0] = half_blk(I, bz, by, bx + 1);
    if (bx + 1 < I.nbxm) return 1;
    return half_mirrored(I, bz, by, I.nbxm, out, 1);
}
__device__ __forceinline__ void half_coords(const InstDev &I, int64_t lb, int &bz, int &by, int &bx) {
    int64_t row;
    if (lb >= I.nbm) {
        row = lb - I.nbm;
        bx = I.nbxm;
    } else {
        row = lb >> I.lnbxm;
        bx = (int)(lb & (I.nbxm - 1));
    }
    by = (int)(row & (I.nbk[1] - 1));
    bz = (int)(row >> I.lnbk[1]);
}
// a block of the half layout with an active neighbour
__device__ __forceinline__ bool half_near_active(const Ctx &c, const InstDev &I, int64_t lb, double thr) {
    int bz, by, bx;
    half_coords(I, lb, bz, by, bx);
    bool nr = false;
    for (int f = 0; f < 6; ++f) {
        int64_t nb[8];
        const int n = half_face(I, bz, by, bx, f, nb);
        for (int i = 0; i < n; ++i) nr = nr | nb_on(c, I, nb[i], thr);
    }
    return nr;
}

// Transition weight of the mode at block-local (lz, ly, lx): the product of
// the roll-off values over the faces that border frozen blocks, in the fixed
// order z low, z high, y low, y high, x low, x high; a face without a frozen
// neighbour contributes an exact factor 1.  w: the roll-off tables (table of
// edge B at [B, 2B)), b: the block edges.
__device__ __forceinline__ double sigma_at(const double *w, uint32_t f, int b0, int b1, int b2, int lz, int ly,
                                           int lx) {
    const double zl = (f & 1u) ? w[b0 + lz] : 1.0;
    const double zh = (f & 2u) ? w[2 * b0 - 1 - lz] : 1.0;
    const double yl = (f & 4u) ? w[b1 + ly] : 1.0;
    const double yh = (f & 8u) ? w[2 * b1 - 1 - ly] : 1.0;
    const double xl = (f & 16u) ? w[b2 + lx] : 1.0;
    const double xh = (f & 32u) ? w[2 * b2 - 1 - lx] : 1.0;
    return ((((zl * zh) * yl) * yh) * xl) * xh;
}

// Update-list entry of a control plan with transition blocks: the global
// block id in the low 25 bits (kEntryId), the frozen-face bits in bits
// 25..30 (bit 25 + 2a: the low face of axis a = z, y, x borders a frozen
// block; bit 26 + 2a: the high face) and the transition flag in bit 31.

// Compaction of a control plan, one block per thread: the state of the block
// (1 active, 2 transition: not active with an active face neighbour, 0
// frozen) from the threshold rule of the block and of its neighbours (no
// grid-wide wait for a finished mask); a transition block also gets the
// frozen-face bits of its update, from the neighbours' own states.  The
// non-frozen blocks are appended to the update list and counted per instance
// for the controller (one atomic per workgroup when the chunk lies in one
// instance).  G is handed over by the update kernel, which reads none of it.
__global__ void __launch_bounds__(256) k_compact_states(Ctx c) {
    __shared__ uint32_t wsum[4], wown[4];
    __shared__ uint32_t base;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t gb = (int64_t)blockIdx.x * 256 + threadIdx.x;
    // the instance of the chunk's first block collects the chunk's count
    const int64_t g0 = (int64_t)blockIdx.x * 256;
    const int iw = c.blk_inst[g0];
    const bool one = c.blk_inst[min(g0 + 255, c.nb_total - 1)] == iw;  // blocks of an instance are contiguous
    bool on = false;
    int ii = iw;
    uint32_t entry = 0;
    if (gb < c.nb_total) {
        ii = c.blk_inst[gb];
        const InstDev &I = c.inst[ii];
        const CtlDev &C = c.ctl[ii];
        const double thr = C.tau2 * __longlong_as_double((long long)c.G[ii]);
        const int64_t lb = gb - I.blk_off;
        uint8_t st = active_ctl(c, I, lb, thr, C.full != 0) ? 1 : 0;
        entry = (uint32_t)gb;
        if (c.half) {  // the neighbours of the stored half (conjugate counterparts at its ends)
            if (!st && c.trans && half_near_active(c, I, lb, thr)) {
                st = 2;
                int bz, by, bx;
                half_coords(I, lb, bz, by, bx);
                uint32_t f = 0;
                for (int fc = 0; fc < 6; ++fc) {
                    int64_t nb[8];
                    const int n = half_face(I, bz, by, bx, fc, nb);
                    bool fr = n > 0;  // every block standing for the neighbour is frozen
                    for (int i = 0; i < n; ++i) fr = fr && !(nb_on(c, I, nb[i], thr) | half_near_active(c, I, nb[i], thr));
                    f |= fr ? 1u << fc : 0u;
                }
                entry |= (f << 25) | (1u << 31);
            }
        } else if (!st && c.trans && near_active(c, I, lb, thr)) {
            st = 2;
            // a neighbour is frozen when neither it nor any of its own
            // neighbours passes the threshold rule
            const int bx = (int)(lb & (I.nbk[2] - 1));
            const int64_t t = lb >> I.lnbk[2];
            const int by = (int)(t & (I.nbk[1] - 1));
            const int bz = (int)(t >> I.lnbk[1]);
            uint32_t f = 0;
            for (int a = 0; a < 3; ++a) {
                if (I.nbk[a] < 2) continue;
                const int k = I.nbk[a] - 1;
                for (int side = 0; side < 2; ++side) {
                    const int d = side ? 1 : -1;
                    const int64_t nb = a == 0 ? blk_id(I, (bz + d) & k, by, bx)
                                     : a == 1 ? blk_id(I, bz, (by + d) & k, bx)
                                              : blk_id(I, bz, by, (bx + d) & k);
                    const bool fr = !(nb_on(c, I, nb, thr) | near_active(c, I, nb, thr));
                    f |= fr ? 1u << (2 * a + side) : 0u;
                }
            }
            entry |= (f << 25) | (1u << 31);
        }
        c.mask[gb] = st;
        on = st != 0;
    }
    const uint64_t bal = __ballot(on);
    const uint32_t pre = __popcll(bal & ((1ull << lane) - 1));
    if (lane == 0) wsum[w] = __popcll(bal);
    if (!one && on && ii != iw) atomicAdd(&c.ctl[ii].nf_upd, 1u);
    const uint64_t mine = __ballot(on && ii == iw);  // every lane votes
    if (lane == 0) wown[w] = (uint32_t)__popcll(mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        base = tot ? atomicAdd(c.count, tot) : 0u;
        const uint32_t own = wown[0] + wown[1] + wown[2] + wown[3];
        if (own) atomicAdd(&c.ctl[iw].nf_upd, own);
    }
    __syncthreads();
    uint32_t pos = base + pre;
    for (int i = 0; i < w; ++i) pos += wsum[i];
    if (on) c.worklist[pos] = entry;
}

// End of an update of instance i: fold the update's count into the step; at
// the end of a step, the threshold controller (steps that are not full) and
// the schedule of the next step.
__device__ __forceinline__ void control_inst(const Ctx &c, int i) {
    const InstDev &I = c.inst[i];
    CtlDev &C = c.ctl[i];
    C.nf_step += C.nf_upd;
    C.nf_total += C.nf_upd;
    C.nf_upd = 0u;
    if (++C.upd < I.per) return;
    C.upd = 0;
    if (I.interval > 0 && !C.full) {
        C.sum += (double)C.nf_step / (double)(I.nb * I.per);
        if (++C.n == I.interval) {
            const double rho = (C.sum / (double)I.interval) / I.target;
            const double eta = I.deadband;
            if (rho > 2.0) C.tau = C.tau * 2.0;
            else if (rho > 1.0 + eta) C.tau = C.tau * (1.0 + eta);
            else if (rho < 0.5) C.tau = C.tau * 0.5;
            else if (rho < 1.0 - eta) C.tau = C.tau * (1.0 - eta);
            C.sum = 0.0;
            C.n = 0;
        }
    }
    C.nf_step = 0u;
    C.step += 1;
    C.full = (C.step < I.full_steps || (I.refresh > 0 && (C.step + 1) % I.refresh == 0)) ? 1 : 0;
    C.tau2 = C.tau * C.tau;
}

// NLSE in one dimension: H(|m|) for |m| = 0..n/2 of every instance with a
// table, by nlse_coef (so a table read equals the evaluation).
template <typename T>
__global__ void __launch_bounds__(256) k_htable(Ctx c) {
    const InstDev &I = c.inst[blockIdx.y];
    if (I.ht_off < 0) return;
    const Coef K = Coef::of(I);
    T *tab = reinterpret_cast<T *>(const_cast<void *>(c.htab)) + 2 * I.ht_off;
    const int half = I.n[2] >> 1;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j <= half; j += gridDim.x * blockDim.x) {
        T hr, hi;
        nlse_coef<T>(K, sq_d(j), hr, hi);
        tab[2 * j] = hr;
        tab[2 * j + 1] = hi;
    }
}

// control state of one instance (only >= 0) or of all after a field load
__global__ void __launch_bounds__(64) k_ctl_reset(Ctx c, int only) {
    for (int i = threadIdx.x; i < c.n_inst; i += blockDim.x) {
        if (only >= 0 && i != only) continue;
        const InstDev &I = c.inst[i];
        CtlDev &C = c.ctl[i];
        C.tau = I.tau0;
        C.tau2 = I.tau0 * I.tau0;
        C.sum = 0.0;
        C.step = 0;
        C.full = (I.full_steps > 0 || I.refresh == 1) ? 1 : 0;
        C.upd = 0;
        C.n = 0;
        C.pad0 = 0;
        C.nf_step = 0u;
        C.nf_upd = 0u;
        C.nf_total = 0ull;
    }
}

// Roll-off tables w(i) = (1 - cos(pi i / (B - 1))) / 2 (w = 1 for B = 1) of
// every block edge B = 2^blockIdx.x in use, stored at [B, 2B).
__global__ void __launch_bounds__(256) k_tapers(Ctx c, double *w) {
    if (!((c.taper_bs >> blockIdx.x) & 1u)) return;
    const int B = 1 << blockIdx.x;
    for (int i = threadIdx.x; i < B; i += blockDim.x) {
        double v = 1.0;
        if (B > 1) {
            double sn, cs;
            sincos_cw((3.141592653589793 * (double)i) / (double)(B - 1), sn, cs);
            v = 0.5 * (1.0 - cs);
        }
        w[B + i] = v;
    }
}

// -------------------------------------------------------------------------
// active-block update: persistent workgroups walk the ordered list.  The list
// is cut into 8 contiguous segments, one per XCD (workgroup id mod 8), so
// x-adjacent active blocks that share cache lines meet in the same L2.
// -------------------------------------------------------------------------

// TR: the list may hold transition blocks (mask 2), which take
// q + sigma (q' - q) with sigma from the roll-off tables; FP32 forms the
// increment in FP32 and applies fl32(sigma) with one fma.
// With c.ab_inc (state measure, CH and GS) the workgroup also writes the
// block's next measure (a_next) from the state it stores, so the next step
// needs no pass over the frozen blocks (their state, and so their a_b, is
// unchanged); a_b itself keeps the values that decided this update.
// The block is served by `nthr` threads of the workgroup (tid = 0 .. nthr - 1,
// whole waves): a workgroup takes several small blocks at once.  `valid` is
// false for a group without an entry in this iteration; it still takes part
// in the workgroup's barriers.
template <typename T, int OP, bool TR>
__device__ __forceinline__ void update_block(const Ctx &c, uint32_t entry, bool valid, double *sig, double *red,
                                             int tid, int nthr) {
    // TR: entries carry the transition flag and the frozen-face bits
    if (!valid) entry = 0u;  // geometry of block 0, no slot is touched
    const int64_t gb = TR ? (int64_t)(entry & kEntryId) : (int64_t)entry;
    constexpr int V = CV<T>::V;
    const int ii = c.blk_inst[gb];
    const InstDev &I = c.inst[ii];
    const int64_t lb = gb - I.blk_off;
    const int bx = (int)(lb & (I.nbk[2] - 1));
    const int64_t t = lb >> I.lnbk[2];
    const int by = (int)(t & (I.nbk[1] - 1));
    const int bz = (int)(t >> I.lnbk[1]);
    const int llpr = I.lb[2] - (V == 2 ? 1 : 0);  // log2 lanes per block row
    const int slots = (I.b[0] * I.b[1]) << llpr;
    const Geo g = Geo::of(I, bz, by);
    const Coef K = Coef::of(I);
    const int x_blk = bx << I.lb[2];
    const bool k0_blk = I.k0path && lb == 0;
    T *q0p = reinterpret_cast<T *>(c.state) + 2 * I.off;
    const T *r0p = reinterpret_cast<const T *>(c.rhs) + 2 * I.off;
    T *q1p = q0p + 2 * I.N;
    const T *r1p = r0p + 2 * I.N;
    const T dt = (OP == OP_GS) ? (T)K.c0 : (T)0;
    const T *htab = (OP == OP_NLSE && I.ht_off >= 0) ? reinterpret_cast<const T *>(c.htab) + 2 * I.ht_off : nullptr;
    const T *h1p = reinterpret_cast<const T *>(c.hist1) + 2 * I.off;  // XPFC history
    const T *h2p = reinterpret_cast<const T *>(c.hist2) + 2 * I.off;
    const T *h3p = reinterpret_cast<const T *>(c.hist3) + 2 * I.off;
    const bool trn = TR && (entry >> 31);  // workgroup-uniform
    const uint32_t faces = (entry >> 25) & 63u;
    const int b0 = I.b[0], b1 = I.b[1], b2 = I.b[2];
    const bool ab = OP != OP_NLSE && c.ab_inc;  // workgroup-uniform
    const bool esum = c.ab_sum;                  // block energy: the sum, else the maximum
    double amax = 0.0;
    for (int s = tid; valid && s < slots; s += nthr) {
        const int r = s >> llpr, l = s & ((1 << llpr) - 1);
        const int z = g.z0 + (r >> g.lb1);
        const int y = g.y0 + (r & g.b1m);
        const int x0 = x_blk + l * V;
        const int64_t e = ((((int64_t)z << g.ln1) + y) << g.ln2) + x0;
        const double myz = sq_d(sidx(z, g.n0)) + sq_d(sidx(y, g.n1));
        T qr[V], qi[V], nr[V], ni[V], q2r[V], q2i[V], n2r[V], n2i[V];
        T h1r[V], h1i[V], h2r[V], h2i[V], h3r[V], h3i[V];
        CV<T>::ld(q0p + 2 * e, qr, qi);
        if (OP != OP_NLSE) CV<T>::ld(r0p + 2 * e, nr, ni);
        else if (htab) nlse_tab_ld<T>(htab, x0, g.n2, nr, ni);
        if (OP == OP_GS) {
            CV<T>::ld(q1p + 2 * e, q2r, q2i);
            CV<T>::ld(r1p + 2 * e, n2r, n2i);
        }
        const double *lrow = nullptr;
        if (OP == OP_XPFC) {
            CV<T>::ld(h1p + 2 * e, h1r, h1i);
            CV<T>::ld(h2p + 2 * e, h2r, h2i);
            CV<T>::ld(h3p + 2 * e, h3r, h3i);
            lrow = xpfc_row(c, I, z, y);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const double mx = (double)sidx(x0 + v, g.n2);
            const double m2 = __builtin_fma(mx, mx, myz);
            T cr, ci, dr = (T)0, di = (T)0;
            if (OP == OP_CH) {
                T sc, f;
                ch_coef<T>(K, m2, sc, f);
                ch_cand<T>(sc, f, qr[v], qi[v], nr[v], ni[v], cr, ci);
            } else if (OP == OP_GS) {
                T au, av;
                gs_coef<T>(K, m2, au, av);
                gs_cand<T>(dt, au, qr[v], qi[v], nr[v], ni[v], cr, ci);
                gs_cand<T>(dt, av, q2r[v], q2i[v], n2r[v], n2i[v], dr, di);
            } else if (OP == OP_XPFC) {
                T co[5];
                xpfc_coef<T>(K, lrow, abs(sidx(x0 + v, g.n2)), m2, co);
                cr = xpfc_cand1<T>(co, qr[v], nr[v], h1r[v], h2r[v], h3r[v]);
                ci = xpfc_cand1<T>(co, qi[v], ni[v], h1i[v], h2i[v], h3i[v]);
            } else {
                T hr = nr[v], hi = ni[v];
                if (!htab) nlse_coef<T>(K, m2, hr, hi);
                nlse_cand<T>(hr, hi, qr[v], qi[v], cr, ci);
            }
            if (TR && trn) {
                const T sg = (T)sigma_at(sig, faces, b0, b1, b2, r >> g.lb1, r & g.b1m, l * V + v);
                cr = fmat(sg, cr - qr[v], qr[v]);
                ci = fmat(sg, ci - qi[v], qi[v]);
                if (OP == OP_GS) {
                    dr = fmat(sg, dr - q2r[v], q2r[v]);
                    di = fmat(sg, di - q2i[v], q2i[v]);
                }
            }
            qr[v] = cr;
            qi[v] = ci;
            if (OP == OP_GS) {
                q2r[v] = dr;
                q2i[v] = di;
            }
        }
        // the FP32 slot of k = 0 stays zero (its value lives in FP64)
        if (k0_blk && s == 0) {
            qr[0] = qi[0] = (T)0;
            q2r[0] = q2i[0] = (T)0;
        }
        if (ab) {  // the state measure of what is stored; k = 0 left out
#pragma unroll
            for (int v = 0; v < V; ++v) {
                double a = sq2((double)qr[v], (double)qi[v]);
                if (OP == OP_GS) a = a + sq2((double)q2r[v], (double)q2i[v]);
                if (lb == 0 && s == 0 && v == 0) a = 0.0;
                amax = esum ? amax + a : fmax(amax, a);
            }
        }
        CV<T>::st(q0p + 2 * e, qr, qi);
        if (OP == OP_GS) CV<T>::st(q1p + 2 * e, q2r, q2i);
    }
    if (ab) {  // block energy: lanes, then the group's waves in order
        amax = esum ? wave_sum(amax) : wave_max(amax);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
        __syncthreads();
        if (valid && tid == 0) {
            const int w0 = threadIdx.x >> 6, nw = nthr >> 6;
            double m = red[w0];
            for (int k = 1; k < nw; ++k) m = esum ? m + red[w0 + k] : fmax(m, red[w0 + k]);
            c.a_next[gb] = m;
        }
        __syncthreads();  // red is free for the next block
    }
    if (valid && k0_blk && tid == 0) {
        double tmp[2];
        k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
        if (TR && trn) {  // block 0 in transition: the weighted increment in FP64
            const double s0 = sigma_at(sig, faces, b0, b1, b2, 0, 0, 0);
            tmp[0] = __builtin_fma(s0, tmp[0] - c.k0[2 * ii], c.k0[2 * ii]);
            if (OP == OP_GS) tmp[1] = __builtin_fma(s0, tmp[1] - c.k0[2 * ii + 1], c.k0[2 * ii + 1]);
        }
        c.k0[2 * ii] = tmp[0];
        if (OP == OP_GS) c.k0[2 * ii + 1] = tmp[1];
    }
}


// CTL: workgroup 0 first closes the update's control step for every
// instance (one wave) and hands G over (G_last, then zero for the next
// indicator).  Nothing in this kernel reads the control state or G, and the
// counts it folds were completed by the compaction kernel, so no other
// workgroup waits for it.  TR: the roll-off tables of the plan's block
// edges are copied into dynamic LDS once per workgroup.
template <typename T, int OP, bool TR, bool CTL>
__global__ void __launch_bounds__(256) k_update(Ctx c) {
    extern __shared__ double sig[];
    __shared__ double red[4];
    if (CTL && blockIdx.x == 0 && threadIdx.x < 64)
        for (int i = threadIdx.x; i < c.n_inst; i += 64) {
            control_inst(c, i);
            c.G_last[i] = c.G[i];
            c.G[i] = 0ull;
        }
    if (TR) {
        for (uint32_t bs = c.taper_bs; bs; bs &= bs - 1) {
            const int B = 1 << __builtin_ctz(bs);
            for (int i = threadIdx.x; i < B; i += blockDim.x) sig[B + i] = c.taper[B + i];
        }
        __syncthreads();
    }
    const uint32_t total = *c.count;
    const int P = gridDim.x;  // multiple of 8
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, per = P >> 3;
    const uint32_t seg = (total + 7) / 8;
    const uint32_t lo = min(total, seg * xcd), hi = min(total, seg * (xcd + 1));
    // G consecutive entries per iteration (x-adjacent blocks of one block
    // row), one group of blockDim / G threads each; entry lo + G m + sub goes
    // to workgroup m mod per, so every entry of the segment is taken once
    const int G = c.upd_group > 1 ? c.upd_group : 1;
    const int nthr = (int)blockDim.x / G, sub = (int)threadIdx.x / nthr, tid = (int)threadIdx.x - sub * nthr;
    for (uint32_t e = lo + (uint32_t)(local * G); e < hi; e += (uint32_t)(per * G)) {  // workgroup-uniform
        const uint32_t my = e + (uint32_t)sub;
        const bool valid = my < hi;
        update_block<T, OP, TR>(c, valid ? c.worklist[my] : 0u, valid, sig, red, tid, nthr);
    }
}

// several list entries per workgroup iteration: all their loads are issued
// before any store, so more bytes are in flight per thread
template <typename T, int OP, int UB>
__global__ void __launch_bounds__(256) k_update_multi(Ctx c) {
    constexpr int V = CV<T>::V;
    const uint32_t total = *c.count;
    const int P = gridDim.x;  // multiple of 8
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, per = P >> 3;
    const uint32_t seg = (total + 7) / 8;
    const uint32_t lo = min(total, seg * xcd), hi = min(total, seg * (xcd + 1));
    for (uint32_t e0 = lo + local; e0 < hi; e0 += per * UB) {
        T qr[UB][V], qi[UB][V], nr[UB][V], ni[UB][V], q2r[UB][V], q2i[UB][V], n2r[UB][V], n2i[UB][V];
        int64_t eidx[UB], base[UB];
        double myz[UB];
        int xs[UB], iis[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const uint32_t e = e0 + u * per;
            eidx[u] = -1;
            if (e >= hi) continue;
            const int64_t gb = c.worklist[e];
            const int ii = c.blk_inst[gb];
            const InstDev &I = c.inst[ii];
            const int llpr = I.lb[2] - (V == 2 ? 1 : 0);
            const int slots = (I.b[0] * I.b[1]) << llpr;
            if ((int)threadIdx.x >= slots) continue;  // blocks of at most 256 slots here
            const int64_t lb = gb - I.blk_off;
            const int bx = (int)(lb & (I.nbk[2] - 1));
            const int64_t t = lb >> I.lnbk[2];
            const int by = (int)(t & (I.nbk[1] - 1));
            const int bz = (int)(t >> I.lnbk[1]);
            const int s = threadIdx.x;
            const int r = s >> llpr, l = s & ((1 << llpr) - 1);
            const int z = (bz << I.lb[0]) + (r >> I.lb[1]);
            const int y = (by << I.lb[1]) + (r & (I.b[1] - 1));
            const int x0 = (bx << I.lb[2]) + l * V;
            const int64_t el = ((((int64_t)z << I.ln[1]) + y) << I.ln[2]) + x0;
            myz[u] = sq_d(sidx(z, I.n[0])) + sq_d(sidx(y, I.n[1]));
            xs[u] = x0;
            iis[u] = ii;
            eidx[u] = el;
            base[u] = 2 * I.off;
            const T *q0p = reinterpret_cast<const T *>(c.state) + base[u];
            const T *r0p = reinterpret_cast<const T *>(c.rhs) + base[u];
            CV<T>::ld(q0p + 2 * el, qr[u], qi[u]);
            if (OP != OP_NLSE) CV<T>::ld(r0p + 2 * el, nr[u], ni[u]);
            else if (I.ht_off >= 0)
                nlse_tab_ld<T>(reinterpret_cast<const T *>(c.htab) + 2 * I.ht_off, x0, I.n[2], nr[u], ni[u]);
            if (OP == OP_GS) {
                CV<T>::ld(q0p + 2 * I.N + 2 * el, q2r[u], q2i[u]);
                CV<T>::ld(r0p + 2 * I.N + 2 * el, n2r[u], n2i[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            if (eidx[u] < 0) continue;
            const int ii = iis[u];
            const InstDev &I = c.inst[ii];
            const Coef K = Coef::of(I);
            const int n2 = I.n[2];
            const int64_t N = I.N;
            const bool k0s = I.k0path && eidx[u] == 0;
            const int64_t el = eidx[u];
            const T dt = (OP == OP_GS) ? (T)K.c0 : (T)0;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double mx = (double)sidx(xs[u] + v, n2);
                const double m2 = __builtin_fma(mx, mx, myz[u]);
                T cr, ci;
                if (OP == OP_CH) {
                    T s, f;
                    ch_coef<T>(K, m2, s, f);
                    ch_cand<T>(s, f, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
                } else if (OP == OP_GS) {
                    T au, av, dr, di;
                    gs_coef<T>(K, m2, au, av);
                    gs_cand<T>(dt, au, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
                    gs_cand<T>(dt, av, q2r[u][v], q2i[u][v], n2r[u][v], n2i[u][v], dr, di);
                    q2r[u][v] = dr;
                    q2i[u][v] = di;
                } else {
                    T hr = nr[u][v], hi2 = ni[u][v];
                    if (I.ht_off < 0) nlse_coef<T>(K, m2, hr, hi2);
                    nlse_cand<T>(hr, hi2, qr[u][v], qi[u][v], cr, ci);
                }
                qr[u][v] = cr;
                qi[u][v] = ci;
            }
            if (k0s) {  // the FP32 slot of k = 0 stays zero
                qr[u][0] = qi[u][0] = (T)0;
                q2r[u][0] = q2i[u][0] = (T)0;
            }
            T *q0p = reinterpret_cast<T *>(c.state) + base[u];
            CV<T>::st(q0p + 2 * el, qr[u], qi[u]);
            if (OP == OP_GS) CV<T>::st(q0p + 2 * N + 2 * el, q2r[u], q2i[u]);
            if (k0s) {
                const InstDev &J = c.inst[ii];
                double tmp[2];
                k0_cand(J, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
                c.k0[2 * ii] = tmp[0];
                if (OP == OP_GS) c.k0[2 * ii + 1] = tmp[1];
            }
        }
    }
}

// Update of one listed block by one wave (the block-list walk, wave form):
// the lanes take the block's 16-byte slots in chunks of UB x 64 and issue all
// loads of a chunk before any store.  With the kept state measure the block
// maximum is a wave reduction, so no workgroup barrier separates one list
// entry from the next (the block energy: the lanes' sums over their slots in
// order, then a fixed butterfly over the lanes).  Blocks of at least 64 slots
// keep every lane busy.
template <typename T, int OP>
__device__ __forceinline__ void update_block_wave(const Ctx &c, uint32_t gb, int lane) {
    constexpr int V = CV<T>::V, UB = 4;
    const int ii = c.blk_inst[gb];
    const InstDev &I = c.inst[ii];
    const int64_t lb = (int64_t)gb - I.blk_off;
    const int bx = (int)(lb & (I.nbk[2] - 1));
    const int64_t t = lb >> I.lnbk[2];
    const int by = (int)(t & (I.nbk[1] - 1));
    const int bz = (int)(t >> I.lnbk[1]);
    const int llpr = I.lb[2] - (V == 2 ? 1 : 0);  // log2 lanes per block row
    const int slots = (I.b[0] * I.b[1]) << llpr;
    const Geo g = Geo::of(I, bz, by);
    const Coef K = Coef::of(I);
    const int x_blk = bx << I.lb[2];
    const bool k0_blk = I.k0path && lb == 0;
    T *q0p = reinterpret_cast<T *>(c.state) + 2 * I.off;
    const T *r0p = reinterpret_cast<const T *>(c.rhs) + 2 * I.off;
    T *q1p = q0p + 2 * I.N;
    const T *r1p = r0p + 2 * I.N;
    const T dt = (OP == OP_GS) ? (T)K.c0 : (T)0;
    const T *htab = (OP == OP_NLSE && I.ht_off >= 0) ? reinterpret_cast<const T *>(c.htab) + 2 * I.ht_off : nullptr;
    const T *h1p = reinterpret_cast<const T *>(c.hist1) + 2 * I.off;  // XPFC history
    const T *h2p = reinterpret_cast<const T *>(c.hist2) + 2 * I.off;
    const T *h3p = reinterpret_cast<const T *>(c.hist3) + 2 * I.off;
    const bool ab = OP != OP_NLSE && c.ab_inc;  // wave-uniform
    const bool esum = c.ab_sum;                  // block energy: the sum, else the maximum
    double amax = 0.0;
    for (int s0 = 0; s0 < slots; s0 += 64 * UB) {
        T qr[UB][V], qi[UB][V], nr[UB][V], ni[UB][V], q2r[UB][V], q2i[UB][V], n2r[UB][V], n2i[UB][V];
        T h1r[UB][V], h1i[UB][V], h2r[UB][V], h2i[UB][V], h3r[UB][V], h3i[UB][V];
        int64_t ex[UB];
        int x0s[UB];
        double myz[UB];
        const double *lrows[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int s = s0 + u * 64 + lane;
            ex[u] = -1;
            if (s >= slots) continue;
            const int r = s >> llpr, l = s & ((1 << llpr) - 1);
            const int z = g.z0 + (r >> g.lb1);
            const int y = g.y0 + (r & g.b1m);
            const int x0 = x_blk + l * V;
            const int64_t e = ((((int64_t)z << g.ln1) + y) << g.ln2) + x0;
            ex[u] = e;
            x0s[u] = x0;
            myz[u] = sq_d(sidx(z, g.n0)) + sq_d(sidx(y, g.n1));
            CV<T>::ld(q0p + 2 * e, qr[u], qi[u]);
            if (OP != OP_NLSE) CV<T>::ld(r0p + 2 * e, nr[u], ni[u]);
            else if (htab) nlse_tab_ld<T>(htab, x0, g.n2, nr[u], ni[u]);
            if (OP == OP_GS) {
                CV<T>::ld(q1p + 2 * e, q2r[u], q2i[u]);
                CV<T>::ld(r1p + 2 * e, n2r[u], n2i[u]);
            }
            if (OP == OP_XPFC) {
                CV<T>::ld(h1p + 2 * e, h1r[u], h1i[u]);
                CV<T>::ld(h2p + 2 * e, h2r[u], h2i[u]);
                CV<T>::ld(h3p + 2 * e, h3r[u], h3i[u]);
                lrows[u] = xpfc_row(c, I, z, y);
            }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            if (ex[u] < 0) continue;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double mx = (double)sidx(x0s[u] + v, g.n2);
                const double m2 = __builtin_fma(mx, mx, myz[u]);
                T cr, ci, dr = (T)0, di = (T)0;
                if (OP == OP_CH) {
                    T sc, f;
                    ch_coef<T>(K, m2, sc, f);
                    ch_cand<T>(sc, f, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
                } else if (OP == OP_GS) {
                    T au, av;
                    gs_coef<T>(K, m2, au, av);
                    gs_cand<T>(dt, au, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
                    gs_cand<T>(dt, av, q2r[u][v], q2i[u][v], n2r[u][v], n2i[u][v], dr, di);
                } else if (OP == OP_XPFC) {
                    T co[5];
                    xpfc_coef<T>(K, lrows[u], abs(sidx(x0s[u] + v, g.n2)), m2, co);
                    cr = xpfc_cand1<T>(co, qr[u][v], nr[u][v], h1r[u][v], h2r[u][v], h3r[u][v]);
                    ci = xpfc_cand1<T>(co, qi[u][v], ni[u][v], h1i[u][v], h2i[u][v], h3i[u][v]);
                } else {
                    T hr = nr[u][v], hi = ni[u][v];
                    if (!htab) nlse_coef<T>(K, m2, hr, hi);
                    nlse_cand<T>(hr, hi, qr[u][v], qi[u][v], cr, ci);
                }
                qr[u][v] = cr;
                qi[u][v] = ci;
                if (OP == OP_GS) {
                    q2r[u][v] = dr;
                    q2i[u][v] = di;
                }
            }
            const bool first = s0 == 0 && u == 0 && lane == 0;  // slot 0 holds k = 0 in block 0
            if (k0_blk && first) {  // the FP32 slot of k = 0 stays zero (its value lives in FP64)
                qr[u][0] = qi[u][0] = (T)0;
                q2r[u][0] = q2i[u][0] = (T)0;
            }
            if (ab) {  // the state measure of what is stored; k = 0 left out
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    double a = sq2((double)qr[u][v], (double)qi[u][v]);
                    if (OP == OP_GS) a = a + sq2((double)q2r[u][v], (double)q2i[u][v]);
                    if (lb == 0 && first && v == 0) a = 0.0;
                    amax = esum ? amax + a : fmax(amax, a);
                }
            }
            CV<T>::st(q0p + 2 * ex[u], qr[u], qi[u]);
            if (OP == OP_GS) CV<T>::st(q1p + 2 * ex[u], q2r[u], q2i[u]);
        }
    }
    if (ab) {
        amax = esum ? wave_sum(amax) : wave_max(amax);
        if (lane == 0) c.a_next[gb] = amax;
    }
    if (k0_blk && lane == 0) {
        double tmp[2];
        k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
        c.k0[2 * ii] = tmp[0];
        if (OP == OP_GS) c.k0[2 * ii + 1] = tmp[1];
    }
}

// persistent walk of the list, one wave per entry: the list is split into one
// segment per XCD as in k_update, and the waves of a workgroup take
// consecutive entries of their segment
template <typename T, int OP>
__global__ void __launch_bounds__(256) k_update_wave(Ctx c) {
    const uint32_t total = *c.count;
    const int P = gridDim.x;  // multiple of 8
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, per = P >> 3;
    const uint32_t wpg = blockDim.x >> 6, w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint32_t seg = (total + 7) / 8;
    const uint32_t lo = min(total, seg * xcd), hi = min(total, seg * (xcd + 1));
    for (uint32_t e = lo + (uint32_t)local * wpg + w; e < hi; e += (uint32_t)per * wpg)
        update_block_wave<T, OP>(c, c.worklist[e], lane);
}

// -------------------------------------------------------------------------
// active update, run walk (launch variant 4): the active blocks of one block
// row that are x-neighbours form runs; each run is cut into aligned pieces of
// L = 2^k blocks (L <= the plan's run_lmax) and each piece into L bands of
// rows, one list entry per band.  A band is one block's worth of slots (the
// list keeps one entry per active block), but its rows are L blocks wide, so
// a wave row reads L x 64 contiguous bytes (FP32 8^3 blocks) instead of one
// 64-byte block row.  List entry: first block of the piece (bits 0..23),
// log2 L (bits 24..26), band (bits 27..30).  The kept measure of a block is
// the maximum over its L bands: the compaction zeroes a_next of every active
// block, and each band sends one atomic maximum per block (non-negative
// doubles order as their bit patterns).
// -------------------------------------------------------------------------

constexpr uint32_t kRunId = (1u << 24) - 1;
constexpr int RUN_GROUP = 16;  // blocks per compaction thread (aligned group)

// blocks a and b (a <= b) lie in one block row of one instance
__device__ __forceinline__ bool same_row(const Ctx &c, int64_t a, int64_t b) {
    const int ia = c.blk_inst[a];
    if (c.blk_inst[b] != ia) return false;
    const InstDev &I = c.inst[ia];
    return ((a - I.blk_off) >> I.lnbk[2]) == ((b - I.blk_off) >> I.lnbk[2]);
}

// Positions for `mine` entries per thread: exclusive prefix within the wave,
// then across the four waves, then one atomic per workgroup.
__device__ __forceinline__ uint32_t list_slots(const Ctx &c, uint32_t mine, uint32_t *wsum, uint32_t &base) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d, 64);
        if (lane >= d) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        base = tot ? atomicAdd(c.count, tot) : 0u;
    }
    __syncthreads();
    uint32_t pos = base + incl - mine;
    for (int i = 0; i < w; ++i) pos += wsum[i];
    return pos;
}

// Threshold, mask and the band list.  Thread t owns the aligned group of
// RUN_GROUP blocks starting at 16 t of its workgroup's range; pieces never
// cross a group, a block row or an instance.  The last workgroup to arrive
// hands G over (as k_compact_append).
__global__ void __launch_bounds__(256) k_compact_runs(Ctx c) {
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t base;
    const int64_t b0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * RUN_GROUP;
    uint32_t bits = 0;
    for (int k = 0; k < RUN_GROUP; ++k) {
        const int64_t gb = b0 + k;
        if (gb < c.nb_total) {
            const bool on = block_active(c, gb);
            c.mask[gb] = on ? 1 : 0;
            if (on && c.ab_inc) c.a_next[gb] = 0.0;
            bits |= (on ? 1u : 0u) << k;
        }
    }
    uint32_t pos = list_slots(c, (uint32_t)__popc(bits), wsum, base);
    int k = 0;
    while (k < RUN_GROUP) {
        if (!((bits >> k) & 1u)) {
            ++k;
            continue;
        }
        int L = c.run_lmax;
        for (; L > 1; L >>= 1) {
            if ((k & (L - 1)) != 0 || k + L > RUN_GROUP) continue;
            const uint32_t m = ((1u << L) - 1u) << k;
            if ((bits & m) == m && same_row(c, b0 + k, b0 + k + L - 1)) break;
        }
        const uint32_t lg = (uint32_t)__builtin_ctz((unsigned)L);
        for (int q = 0; q < L; ++q) c.worklist[pos++] = (uint32_t)(b0 + k) | (lg << 24) | ((uint32_t)q << 27);
        k += L;
    }
    // every G read of this workgroup happened before the barriers above
    if (threadIdx.x == 0) {
        const unsigned int done = atomicAdd(c.done, 1u);
        if (done == gridDim.x - 1) {
            for (int i = 0; i < c.n_inst; ++i) {
                c.G_last[i] = c.G[i];
                c.G[i] = 0ull;
            }
            *c.done = 0u;
        }
    }
}

// One band of a piece by one wave.  UB = slots per block / 64: every lane
// issues UB loads of 16 bytes per array before its stores; the lanes of one
// piece row are contiguous, so lane l sits in block j = (l mod (lpr L)) / lpr
// for every load (lpr = lanes per block row).
template <typename T, int OP, int UB>
__device__ __forceinline__ void update_band(const Ctx &c, uint32_t entry, int lane) {
    constexpr int V = CV<T>::V;
    const int64_t gb0 = (int64_t)(entry & kRunId);
    const int lgL = (int)((entry >> 24) & 7u);
    const int band = (int)(entry >> 27);
    const int ii = c.blk_inst[gb0];
    const InstDev &I = c.inst[ii];
    const int64_t lb0 = gb0 - I.blk_off;
    const int bx0 = (int)(lb0 & (I.nbk[2] - 1));
    const int64_t t = lb0 >> I.lnbk[2];
    const int by = (int)(t & (I.nbk[1] - 1));
    const int bz = (int)(t >> I.lnbk[1]);
    const int llpr = I.lb[2] - (V == 2 ? 1 : 0);  // log2 lanes per block row
    const int lrow = llpr + lgL;                  // log2 lanes per piece row (<= 6)
    const int lstep = 6 - lrow;                   // log2 piece rows per wave load
    const int r0 = band << (I.lb[0] + I.lb[1] - lgL);
    const int col = lane & ((1 << lrow) - 1);
    const int j = col >> llpr;
    const int x0 = ((bx0 + j) << I.lb[2]) + (col & ((1 << llpr) - 1)) * V;
    const int64_t lb = lb0 + j;
    const Geo g = Geo::of(I, bz, by);
    const Coef K = Coef::of(I);
    T *q0p = reinterpret_cast<T *>(c.state) + 2 * I.off;
    const T *r0p = reinterpret_cast<const T *>(c.rhs) + 2 * I.off;
    T *q1p = q0p + 2 * I.N;
    const T *r1p = r0p + 2 * I.N;
    const T dt = (OP == OP_GS) ? (T)K.c0 : (T)0;
    const bool ab = c.ab_inc;  // wave-uniform
    double mx2[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const double m = (double)sidx(x0 + v, g.n2);
        mx2[v] = m * m;
    }
    T qr[UB][V], qi[UB][V], nr[UB][V], ni[UB][V], q2r[UB][V], q2i[UB][V], n2r[UB][V], n2i[UB][V];
    int64_t ex[UB];
    double myz[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const int r = r0 + (u << lstep) + (lane >> lrow);
        const int z = g.z0 + (r >> g.lb1);
        const int y = g.y0 + (r & g.b1m);
        const int64_t e = ((((int64_t)z << g.ln1) + y) << g.ln2) + x0;
        ex[u] = e;
        myz[u] = sq_d(sidx(z, g.n0)) + sq_d(sidx(y, g.n1));
        CV<T>::ld(q0p + 2 * e, qr[u], qi[u]);
        CV<T>::ld(r0p + 2 * e, nr[u], ni[u]);
        if (OP == OP_GS) {
            CV<T>::ld(q1p + 2 * e, q2r[u], q2i[u]);
            CV<T>::ld(r1p + 2 * e, n2r[u], n2i[u]);
        }
    }
    // the lane holding k = 0 (block 0 of the instance, row 0, column 0)
    const bool z_lane = lb == 0 && x0 == 0 && r0 == 0 && (lane >> lrow) == 0;
    double amax = 0.0;
#pragma unroll
    for (int u = 0; u < UB; ++u) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const double m2 = myz[u] + mx2[v];
            T cr, ci, dr = (T)0, di = (T)0;
            if (OP == OP_CH) {
                T sc, f;
                ch_coef<T>(K, m2, sc, f);
                ch_cand<T>(sc, f, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
            } else {
                T au, av;
                gs_coef<T>(K, m2, au, av);
                gs_cand<T>(dt, au, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
                gs_cand<T>(dt, av, q2r[u][v], q2i[u][v], n2r[u][v], n2i[u][v], dr, di);
            }
            qr[u][v] = cr;
            qi[u][v] = ci;
            if (OP == OP_GS) {
                q2r[u][v] = dr;
                q2i[u][v] = di;
            }
        }
        if (I.k0path && z_lane && u == 0) {  // the FP32 slot of k = 0 stays zero (its value lives in FP64)
            qr[0][0] = qi[0][0] = (T)0;
            q2r[0][0] = q2i[0][0] = (T)0;
        }
        if (ab) {  // the state measure of what is stored; k = 0 left out
#pragma unroll
            for (int v = 0; v < V; ++v) {
                double a = sq2((double)qr[u][v], (double)qi[u][v]);
                if (OP == OP_GS) a = a + sq2((double)q2r[u][v], (double)q2i[u][v]);
                if (z_lane && u == 0 && v == 0) a = 0.0;
                amax = fmax(amax, a);
            }
        }
        CV<T>::st(q0p + 2 * ex[u], qr[u], qi[u]);
        if (OP == OP_GS) CV<T>::st(q1p + 2 * ex[u], q2r[u], q2i[u]);
    }
    if (ab) {  // maximum over the lanes of block j: sub-row lanes, then rows
        for (int off = 1; off < (1 << llpr); off <<= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
        for (int off = 1 << lrow; off < 64; off <<= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
        if (lane < (1 << lrow) && (lane & ((1 << llpr) - 1)) == 0 && amax > 0.0)
            atomicMax(reinterpret_cast<unsigned long long *>(c.a_next) + (I.blk_off + lb),
                      (unsigned long long)__double_as_longlong(amax));
    }
    if (I.k0path && z_lane) {
        double tmp[2];
        k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
        c.k0[2 * ii] = tmp[0];
        if (OP == OP_GS) c.k0[2 * ii + 1] = tmp[1];
    }
}

// persistent walk of the band list, one wave per entry, one segment of the
// list per XCD as in k_update
template <typename T, int OP, int UB>
__global__ void __launch_bounds__(256) k_update_run(Ctx c) {
    const uint32_t total = *c.count;
    const int P = gridDim.x;  // multiple of 8
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, per = P >> 3;
    const uint32_t wpg = blockDim.x >> 6, w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint32_t seg = (total + 7) / 8;
    const uint32_t lo = min(total, seg * xcd), hi = min(total, seg * (xcd + 1));
    for (uint32_t e = lo + (uint32_t)local * wpg + w; e < hi; e += (uint32_t)per * wpg)
        update_band<T, OP, UB>(c, c.worklist[e], lane);
}

// -------------------------------------------------------------------------
// active update, strip variant: the indicator's traversal (one workgroup per
// strip of S x-adjacent blocks, waves split the rows, 16 B per lane, 1 KiB per
// wave row) with every lane predicated on its block's mask.  Frozen blocks
// issue no loads or stores; a strip with no active block exits at once.  Long
// contiguous rows keep DRAM pages busy when many neighbouring blocks are
// active, where the block-list walk moves 64-byte row pieces.
// -------------------------------------------------------------------------

template <typename T, int OP>
__device__ __forceinline__ void update_strip_body(const Ctx &c, const InstDev &I, int ii, bool lane_on,
                                                  int sbz, int sby, int sx, int lane, int w, int nw,
                                                  bool k0_lane) {
    constexpr int V = CV<T>::V;
    constexpr int U = OP == OP_GS ? 2 : 4;
    const int chunks = I.chunks;
    const Geo g = Geo::of(I, sbz, sby);
    const Coef K = Coef::of(I);
    const int total_it = (I.b[0] * I.b[1]) << g.lch;
    const int x_lane = ((sx << I.lS) << I.lb[2]) + lane * V;
    T *q0p = reinterpret_cast<T *>(c.state) + 2 * I.off;
    const T *r0p = reinterpret_cast<const T *>(c.rhs) + 2 * I.off;
    T *q1p = q0p + 2 * I.N;
    const T *r1p = r0p + 2 * I.N;
    const T dt = (OP == OP_GS) ? (T)K.c0 : (T)0;
    const T *htab = (OP == OP_NLSE && I.ht_off >= 0) ? reinterpret_cast<const T *>(c.htab) + 2 * I.ht_off : nullptr;
    // frozen lanes never load or store; their registers are set once so that
    // the unconditional arithmetic below reads defined values
    T qr[U][V], qi[U][V], nr[U][V], ni[U][V], q2r[U][V], q2i[U][V], n2r[U][V], n2i[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            qr[u][v] = qi[u][v] = nr[u][v] = ni[u][v] = (T)0;
            q2r[u][v] = q2i[u][v] = n2r[u][v] = n2i[u][v] = (T)0;
        }
    for (int it0 = w; it0 < total_it; it0 += nw * U) {
        int xs[U];
        double myz[U];
        int64_t eidx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int it = it0 + u * nw;  // wave-uniform
            const int r = it >> g.lch, ch = it & (chunks - 1);
            const int z = g.z0 + (r >> g.lb1);
            const int y = g.y0 + (r & g.b1m);
            const int x = x_lane + ch * 64 * V;
            xs[u] = x;
            myz[u] = sq_d(sidx(z, g.n0)) + sq_d(sidx(y, g.n1));
            eidx[u] = ((((int64_t)z << g.ln1) + y) << g.ln2) + x;
            if (it < total_it && lane_on) {
                const int64_t e = eidx[u];
                CV<T>::ld(q0p + 2 * e, qr[u], qi[u]);
                if (OP != OP_NLSE) CV<T>::ld(r0p + 2 * e, nr[u], ni[u]);
                else if (htab) nlse_tab_ld<T>(htab, x, g.n2, nr[u], ni[u]);
                if (OP == OP_GS) {
                    CV<T>::ld(q1p + 2 * e, q2r[u], q2i[u]);
                    CV<T>::ld(r1p + 2 * e, n2r[u], n2i[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (it0 + u * nw >= total_it) continue;  // wave-uniform
            T cq[V], cqi[V], cq2[V], cq2i[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double mx = (double)sidx(xs[u] + v, g.n2);
                const double m2 = __builtin_fma(mx, mx, myz[u]);
                T cr, ci;
                if (OP == OP_CH) {
                    T s, f;
                    ch_coef<T>(K, m2, s, f);
                    ch_cand<T>(s, f, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
                } else if (OP == OP_GS) {
                    T au, av, dr, di;
                    gs_coef<T>(K, m2, au, av);
                    gs_cand<T>(dt, au, qr[u][v], qi[u][v], nr[u][v], ni[u][v], cr, ci);
                    gs_cand<T>(dt, av, q2r[u][v], q2i[u][v], n2r[u][v], n2i[u][v], dr, di);
                    cq2[v] = dr;
                    cq2i[v] = di;
                } else {
                    T hr = nr[u][v], hi = ni[u][v];
                    if (!htab) nlse_coef<T>(K, m2, hr, hi);
                    nlse_cand<T>(hr, hi, qr[u][v], qi[u][v], cr, ci);
                }
                cq[v] = cr;
                cqi[v] = ci;
            }
            // the FP32 slot of k = 0 stays zero (its value lives in FP64)
            if (u == 0 && k0_lane && it0 == 0) {
                cq[0] = cqi[0] = (T)0;
                if (OP == OP_GS) cq2[0] = cq2i[0] = (T)0;
            }
            if (lane_on) {
                CV<T>::st(q0p + 2 * eidx[u], cq, cqi);
                if (OP == OP_GS) CV<T>::st(q1p + 2 * eidx[u], cq2, cq2i);
            }
        }
    }
    if (k0_lane && w == 0 && lane_on) {
        double tmp[2];
        k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
        c.k0[2 * ii] = tmp[0];
        if (OP == OP_GS) c.k0[2 * ii + 1] = tmp[1];
    }
}

// Strip walk with the threshold fused in, persistent: each workgroup takes
// strips in a grid stride.  A strip whose largest block value is at or below
// the instance threshold is frozen as a whole (one 8-byte read, its mask bytes
// cleared); otherwise each lane decides its block (the compaction's rule), the
// lane leaders write the mask and the waves walk the rows of the active lanes.
// Every wave holds the same lanes, so a wave-wide vote replaces any barrier.
template <typename T, int OP>
__global__ void __launch_bounds__(1024) k_update_strip(Ctx c) {
    constexpr int V = CV<T>::V;
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t strip = blockIdx.x; strip < c.n_strips; strip += gridDim.x) {
        const int ii = find_by_offset(c.inst, c.n_inst, strip, 0);
        const InstDev &I = c.inst[ii];
        const int64_t ls = strip - I.strip_off;
        const int lnsx = I.lnbk[2] - I.lS;
        const int sx = (int)(ls & ((1 << lnsx) - 1));
        const int64_t t = ls >> lnsx;
        const int sby = (int)(t & ((1 << I.lnbk[1]) - 1));
        const int sbz = (int)(t >> I.lnbk[1]);
        const int chunks = I.chunks;
        const int LB = chunks > 1 ? 64 : (I.b[2] / V);
        const int lane_bx = (sx << I.lS) + (chunks > 1 ? 0 : lane / LB);
        const int64_t lane_lb = ((((int64_t)sbz << I.lnbk[1]) + sby) << I.lnbk[2]) + lane_bx;
        const bool in_strip = chunks > 1 || lane * V < (I.S << I.lb[2]);
        const double thr = I.tau2 * __longlong_as_double((long long)c.G[ii]);
        const bool live = c.dense || (I.pin && ls == 0) || c.strip_max[strip] > thr;
        bool lane_on = false;
        if (in_strip) {
            const int64_t gb = I.blk_off + lane_lb;
            bool on = false;
            if (live) {
                if (c.dense) on = true;
                else if (I.pin && lane_lb == 0) on = true;
                else if (c.skip && c.skip[gb]) on = false;
                else on = c.a_b[gb] > thr;
            }
            lane_on = on;
            if (w == 0 && (chunks > 1 ? lane == 0 : (lane % LB) == 0)) c.mask[gb] = on ? 1 : 0;
        }
        const bool k0_lane = I.k0path && ls == 0 && lane == 0;
        if (__any(lane_on)) update_strip_body<T, OP>(c, I, ii, lane_on, sbz, sby, sx, lane, w, nw, k0_lane);
    }
    // every G value this workgroup used was consumed before the barrier, so
    // the last workgroup to arrive may hand G over: read-back copy, cleared for
    // the next indicator pass (the kernel boundary publishes the writes)
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int done = atomicAdd(c.done, 1u);
        if (done == gridDim.x - 1) {
            for (int i = 0; i < c.n_inst; ++i) {
                c.G_last[i] = c.G[i];
                c.G[i] = 0ull;
            }
            *c.done = 0u;
        }
    }
}

// -------------------------------------------------------------------------
// Regular (dense) update: the same core over every mode, elementwise tiles
// -------------------------------------------------------------------------

template <typename T, int OP>
__global__ void __launch_bounds__(1024) k_dense(Ctx c) {
    constexpr int V = CV<T>::V;
    constexpr int TE = tile_elems<T>();
    __shared__ double lds[16];
    const int64_t tile = blockIdx.x;
    const int ii = find_by_offset(c.inst, c.n_inst, tile, 1);
    const InstDev &I = c.inst[ii];
    const int64_t t0 = (tile - I.tile_off) * TE;
    const Coef K = Coef::of(I);
    const int64_t N = I.N;
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2], ln1 = I.ln[1], ln2 = I.ln[2];
    const bool k0_tile = I.k0path && t0 == 0;
    T *q0p = reinterpret_cast<T *>(c.state) + 2 * I.off;
    const T *r0p = reinterpret_cast<const T *>(c.rhs) + 2 * I.off;
    T *q1p = q0p + 2 * N;
    const T *r1p = r0p + 2 * N;
    const T dt = (OP == OP_GS) ? (T)K.c0 : (T)0;
    const T *htab = (OP == OP_NLSE && I.ht_off >= 0) ? reinterpret_cast<const T *>(c.htab) + 2 * I.ht_off : nullptr;
    const T *h1p = reinterpret_cast<const T *>(c.hist1) + 2 * I.off;  // XPFC history
    const T *h2p = reinterpret_cast<const T *>(c.hist2) + 2 * I.off;
    const T *h3p = reinterpret_cast<const T *>(c.hist3) + 2 * I.off;
    double acc[1] = {0.0};
    const int jstep = blockDim.x * V;
    for (int j = threadIdx.x * V; j < TE; j += jstep) {
        const int64_t e = t0 + j;
        if (e >= N) break;
        const int x0 = (int)(e & (n2 - 1));
        const int64_t zy = e >> ln2;
        const int y = (int)(zy & (n1 - 1));
        const int z = (int)(zy >> ln1);
        const double myz = sq_d(sidx(z, n0)) + sq_d(sidx(y, n1));
        T qr[V], qi[V], nr[V], ni[V], q2r[V], q2i[V], n2r[V], n2i[V];
        T h1r[V], h1i[V], h2r[V], h2i[V], h3r[V], h3i[V];
        CV<T>::ld(q0p + 2 * e, qr, qi);
        if (OP != OP_NLSE) CV<T>::ld(r0p + 2 * e, nr, ni);
        else if (htab) nlse_tab_ld<T>(htab, x0, n2, nr, ni);
        if (OP == OP_GS) {
            CV<T>::ld(q1p + 2 * e, q2r, q2i);
            CV<T>::ld(r1p + 2 * e, n2r, n2i);
        }
        const double *lrow = nullptr;
        if (OP == OP_XPFC) {
            CV<T>::ld(h1p + 2 * e, h1r, h1i);
            CV<T>::ld(h2p + 2 * e, h2r, h2i);
            CV<T>::ld(h3p + 2 * e, h3r, h3i);
            lrow = xpfc_row(c, I, z, y);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const double mx = (double)sidx(x0 + v, n2);
            const double m2 = __builtin_fma(mx, mx, myz);
            T cr, ci;
            if (OP == OP_CH) {
                T s, f;
                ch_coef<T>(K, m2, s, f);
                // zero at k = 0 (m2 = 0), where the FP32 slot holds zero
                acc[0] += (K.K2 * m2) * sq2((double)qr[v], (double)qi[v]);
                ch_cand<T>(s, f, qr[v], qi[v], nr[v], ni[v], cr, ci);
            } else if (OP == OP_GS) {
                T au, av, dr, di;
                gs_coef<T>(K, m2, au, av);
                gs_cand<T>(dt, au, qr[v], qi[v], nr[v], ni[v], cr, ci);
                gs_cand<T>(dt, av, q2r[v], q2i[v], n2r[v], n2i[v], dr, di);
                q2r[v] = dr;
                q2i[v] = di;
            } else if (OP == OP_XPFC) {
                T co[5];
                xpfc_coef<T>(K, lrow, abs(sidx(x0 + v, n2)), m2, co);
                cr = xpfc_cand1<T>(co, qr[v], nr[v], h1r[v], h2r[v], h3r[v]);
                ci = xpfc_cand1<T>(co, qi[v], ni[v], h1i[v], h2i[v], h3i[v]);
            } else {
                T hr = nr[v], hi = ni[v];
                if (!htab) nlse_coef<T>(K, m2, hr, hi);
                nlse_cand<T>(hr, hi, qr[v], qi[v], cr, ci);
            }
            qr[v] = cr;
            qi[v] = ci;
        }
        if (k0_tile && j == 0) {  // the FP32 slot of k = 0 stays zero
            qr[0] = qi[0] = (T)0;
            q2r[0] = q2i[0] = (T)0;
        }
        CV<T>::st(q0p + 2 * e, qr, qi);
        if (OP == OP_GS) CV<T>::st(q1p + 2 * e, q2r, q2i);
    }
    if (k0_tile && threadIdx.x == 0) {
        double tmp[2];
        k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
        c.k0[2 * ii] = tmp[0];
        if (OP == OP_GS) c.k0[2 * ii + 1] = tmp[1];
    }
    if (OP == OP_CH) {
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) c.dense_part[tile] = acc[0];
    }
}

__global__ void k_reset(Ctx c) {
    for (int i = threadIdx.x; i < c.n_inst; i += blockDim.x) c.G[i] = c.G_last[i] = 0ull;
    if (threadIdx.x == 0) *c.count = 0u;
}

// -------------------------------------------------------------------------
// field <-> state helpers (one instance)
// -------------------------------------------------------------------------

// W[s][i] = (real[s][i], 0)
template <typename T>
__global__ void k_real_to_complex(Ctx c, int ii, const T *real) {
    const InstDev &I = c.inst[ii];
    T *w = reinterpret_cast<T *>(c.work) + 2 * I.off;
    const int64_t n = I.N * I.nspec;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        w[2 * i] = real[i];
        w[2 * i + 1] = (T)0;
    }
}

// per-tile FP64 sums of a real field (both species) -> nl_part
template <typename T>
__global__ void __launch_bounds__(256) k_real_tile_sums(Ctx c, int ii, const T *real) {
    constexpr int TE = tile_elems<T>();
    __shared__ double lds[2 * 16];
    const InstDev &I = c.inst[ii];
    const int64_t t0 = (int64_t)blockIdx.x * TE;
    double acc[2] = {0.0, 0.0};
    for (int j = threadIdx.x; j < TE; j += blockDim.x) {
        const int64_t e = t0 + j;
        if (e >= I.Nreal) break;
        acc[0] += (double)real[e];
        if (I.nspec > 1) acc[1] += (double)real[I.Nreal + e];
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        c.nl_part[2 * (I.tile_off + blockIdx.x)] = acc[0];
        c.nl_part[2 * (I.tile_off + blockIdx.x) + 1] = acc[1];
    }
}

// copy an instance spectrum src -> dst; slot 0 of each species is stored
// (widened to FP64) in k0_dst[species] when given, and zeroed with zero_slot0
template <typename T>
__global__ void k_copy_spectrum(Ctx c, int ii, const T *src, T *dst, int zero_slot0, double *k0_dst) {
    const InstDev &I = c.inst[ii];
    const int64_t n = I.N * I.nspec;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T re = src[2 * i], im = src[2 * i + 1];
        if ((i % I.N) == 0) {
            if (k0_dst) k0_dst[i / I.N] = (double)re;
            if (zero_slot0) {
                re = (T)0;
                im = (T)0;
            }
        }
        dst[2 * i] = re;
        dst[2 * i + 1] = im;
    }
}

// out[s][i] = Re(W[s][i]) / N + mean_s
template <typename T>
__global__ void k_work_to_real(Ctx c, int ii, T *out) {
    const InstDev &I = c.inst[ii];
    const T *w = reinterpret_cast<const T *>(c.work) + 2 * I.off;
    const int64_t n = I.N * I.nspec;
    const T invN = (T)I.invN;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(i / I.N);
        const T mean = I.k0path ? (T)(c.k0[2 * ii + s] * I.invN) : (T)0;
        out[i] = w[2 * i] * invN + mean;
    }
}

template <typename T>
__global__ void k_scale_copy(int64_t n, const T *src, T *dst, T scale) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] * scale;
}

// device-to-device copy in 8-byte words (a kernel node, not a copy node, when
// a step is captured into a graph)
__global__ void k_copy8(const unsigned long long *src, unsigned long long *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

template <typename T>
__global__ void k_fill_pattern(T *buf, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n;
         i += (int64_t)gridDim.x * blockDim.x)
        buf[i] = (T)((i * 2654435761ull) % 1000003ull) * (T)1e-3;
}
template <typename T>
__global__ void k_check_pattern(const T *buf, int64_t n, uint32_t *bad) {
    uint32_t b = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n;
         i += (int64_t)gridDim.x * blockDim.x)
        b |= buf[i] != (T)((i * 2654435761ull) % 1000003ull) * (T)1e-3;
    if (b) atomicOr(bad, 1u);
}

// -------------------------------------------------------------------------
// half-spectrum layout of the real fields (CH, GS; Supplementary S1.2)
// -------------------------------------------------------------------------
// A species holds nz*ny rows of xs = nx/2 + 1 complex values, the columns
// 0 .. nx/2 of the forward transform; the omitted columns are the conjugates
// of stored ones and are never touched.  Blocks of the columns below nx/2
// come first (C order over (z, y, x) block coordinates), then one block per
// (z, y) block row for the column nx/2.  With nx/2 + 1 values per row, rows
// start on 8-byte boundaries only (FP32), so a lane moves one complex value.
// The real fields between the transforms are plain arrays of nz*ny*nx values
// per species in W, from the instance's first real (roff) on.

template <typename T> struct RV;
template <> struct RV<float> {
    static constexpr int V = 4;  // reals per 16-byte lane access
    __device__ static void ld(const float *p, float (&v)[4]) {
        const float4 x = *reinterpret_cast<const float4 *>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
    __device__ static void st(float *p, const float (&v)[4]) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
};
template <> struct RV<double> {
    static constexpr int V = 2;
    __device__ static void ld(const double *p, double (&v)[2]) {
        const double2 x = *reinterpret_cast<const double2 *>(p);
        v[0] = x.x; v[1] = x.y;
    }
    __device__ static void st(double *p, const double (&v)[2]) {
        *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    }
};

template <typename T>
__device__ __forceinline__ void ld1(const T *p, T &re, T &im) {
    if (sizeof(T) == 4) {
        const float2 v = *reinterpret_cast<const float2 *>(p);
        re = (T)v.x;
        im = (T)v.y;
    } else {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        re = (T)v.x;
        im = (T)v.y;
    }
}
template <typename T>
__device__ __forceinline__ void st1(T *p, T re, T im) {
    if (sizeof(T) == 4) *reinterpret_cast<float2 *>(p) = make_float2((float)re, (float)im);
    else *reinterpret_cast<double2 *>(p) = make_double2((double)re, (double)im);
}

// Fused nonlinear term on the real fields: the per-element arithmetic and the
// FP64 sums of k_nonlinear, on tiles of tile_elems reals.
template <typename T, int OP>
__global__ void __launch_bounds__(1024) k_nonlinear_h(Ctx c) {
    constexpr int V = RV<T>::V;
    constexpr int TE = tile_elems<T>();
    __shared__ double lds[2 * 16];
    const int64_t tile = blockIdx.x;
    const int ii = find_by_offset(c.inst, c.n_inst, tile, 1);
    const InstDev &I = c.inst[ii];
    const int64_t t0 = (tile - I.tile_off) * TE;
    const int64_t NR = I.Nreal;
    T *base = reinterpret_cast<T *>(c.work) + I.roff;
    double acc[2] = {0.0, 0.0};
    const T invN = (T)I.invN;
    if (OP == OP_CH) {
        if (I.k0path) {
            // W holds N (c - cbar): expanded about the FP64 mean (as k_nonlinear)
            const double cbar = c.k0[2 * ii] * I.invN;
            const T A1 = (T)(3.0 * cbar * cbar - 1.0), A2 = (T)(3.0 * cbar);
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= NR) break;
                T r[V];
                RV<T>::ld(base + e, r);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T d = r[v] * invN;
                    r[v] = d * (A1 + d * (A2 + d));
                    const double cd = cbar + (double)d;
                    const double t = cd * cd - 1.0;
                    acc[0] += 0.25 * (t * t);
                    acc[1] += cd * cd * cd - cd;
                }
                RV<T>::st(base + e, r);
            }
        } else {
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= NR) break;
                T r[V];
                RV<T>::ld(base + e, r);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T cc = r[v] * invN;
                    r[v] = cc * cc * cc - cc;
                    const double cd = (double)cc;
                    const double t = cd * cd - 1.0;
                    acc[0] += 0.25 * (t * t);
                    acc[1] += (double)r[v];
                }
                RV<T>::st(base + e, r);
            }
        }
    } else {
        const T F = (T)I.q0, Fk = (T)(I.q0 + I.q1);
        T *bu = base, *bv = base + NR;
        if (I.k0path) {
            const double ub = c.k0[2 * ii] * I.invN, vb = c.k0[2 * ii + 1] * I.invN;
            const T Uf = (T)ub, Vf = (T)vb, V2 = (T)(2.0 * vb);
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= NR) break;
                T ur[V], vr[V];
                RV<T>::ld(bu + e, ur);
                RV<T>::ld(bv + e, vr);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T du = ur[v] * invN, dv = vr[v] * invN;
                    const T vv = Vf + dv;
                    const T P = Uf * (dv * (V2 + dv)) + du * (vv * vv);
                    ur[v] = -P - F * du;
                    vr[v] = P - Fk * dv;
                    const double u64 = ub + (double)du, v64 = vb + (double)dv;
                    const double uvv = u64 * v64 * v64;
                    acc[0] += -uvv + I.q0 * (1.0 - u64);
                    acc[1] += uvv - (I.q0 + I.q1) * v64;
                }
                RV<T>::st(bu + e, ur);
                RV<T>::st(bv + e, vr);
            }
        } else {
            for (int j = threadIdx.x * V; j < TE; j += blockDim.x * V) {
                const int64_t e = t0 + j;
                if (e >= NR) break;
                T ur[V], vr[V];
                RV<T>::ld(bu + e, ur);
                RV<T>::ld(bv + e, vr);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const T u = ur[v] * invN;
                    const T w = vr[v] * invN;
                    const T uvv = u * w * w;
                    ur[v] = -uvv + F * ((T)1 - u);
                    vr[v] = uvv - Fk * w;
                    acc[0] += (double)ur[v];
                    acc[1] += (double)vr[v];
                }
                RV<T>::st(bu + e, ur);
                RV<T>::st(bv + e, vr);
            }
        }
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        c.nl_part[2 * tile] = acc[0];
        c.nl_part[2 * tile + 1] = acc[1];
    }
}

// Candidate and measure of one stored mode (CH or GS); returns a(k).
template <typename T, int OP, bool SI>
__device__ __forceinline__ double half_mode(const Coef &K, T c0s, double m2, T qr, T qi, T nr, T ni, T q2r,
                                            T q2i, T n2r, T n2i) {
    if (SI) {
        double a = sq2((double)qr, (double)qi);
        if (OP == OP_GS) a = a + sq2((double)q2r, (double)q2i);
        return a;
    }
    T cr, ci;
    if (OP == OP_CH) {
        T s, f;
        ch_coef<T>(K, m2, s, f);
        return ch_cand<T>(s, f, qr, qi, nr, ni, cr, ci);
    }
    T au, av;
    gs_coef<T>(K, m2, au, av);
    double a = gs_cand<T>(c0s, au, qr, qi, nr, ni, cr, ci);
    return a + gs_cand<T>(c0s, av, q2r, q2i, n2r, n2i, cr, ci);
}

// Indicator on the half layout: one workgroup per (z, y) block row of one
// instance.  Lanes take 64 consecutive columns below nx/2, the waves split
// the rows (several in flight); each lane keeps the maximum of its column, the
// lanes of one block combine by shuffles, the waves in LDS (dynamic: waves x
// half_nb doubles).  The column nx/2 is one value per row: there the lanes
// take rows.  CH also sums the FP64 gradient energy of the state, each stored
// column below nx/2 other than 0 counted twice (its omitted partner).
template <typename T, int OP, bool SI>
__global__ void __launch_bounds__(256) k_indicator_h(Ctx c) {
    extern __shared__ double hred[];  // [waves][half_nb]
    __shared__ double s_sum[4], s_max[4];
    constexpr int U = OP == OP_GS ? 4 : 8;  // rows in flight per wave (8-byte lanes)
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NB = c.half_nb;
    const int64_t strip = blockIdx.x;
    const int ii = find_by_offset(c.inst, c.n_inst, strip, 0);
    const InstDev &I = c.inst[ii];
    const int64_t rb = strip - I.strip_off;  // (z, y) block row
    const int by = (int)(rb & (I.nbk[1] - 1));
    const int bz = (int)(rb >> I.lnbk[1]);
    const Coef K = Coef::of(I);
    const int lb1 = I.lb[1], b1m = I.b[1] - 1, ln1 = I.ln[1];
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2];
    const int z0 = bz << I.lb[0], y0 = by << lb1;
    const int R = I.b[0] * I.b[1];
    const int xs = I.xs, xh = n2 >> 1;
    const int nbxm = I.nbxm;
    const T *q0p = reinterpret_cast<const T *>(c.state) + 2 * I.off;
    const T *r0p = reinterpret_cast<const T *>(c.rhs) + 2 * I.off;
    const T *q1p = q0p + 2 * I.N;
    const T *r1p = r0p + 2 * I.N;
    const T c0s = (OP == OP_GS) ? (T)K.c0 : (T)0;
    const int64_t row_lb = rb * nbxm;  // local id of the row's first block
    for (int i = threadIdx.x; i < nw * NB; i += blockDim.x) hred[i] = 0.0;
    __syncthreads();
    double esum = 0.0;
    bool bad = false;
    const int LB = I.b[2] < 64 ? I.b[2] : 64;  // lanes of one block in a chunk
    for (int x0 = 0; x0 < xh; x0 += 64) {
        const int x = x0 + lane;
        const int bx = x >> I.lb[2];
        bool on = x < xh;
        if (on && c.skip && c.skip[I.blk_off + row_lb + bx] && !(I.pin && row_lb + bx == 0)) on = false;
        const double mx2 = sq_d(x);
        const double wgt = x == 0 ? 1.0 : 2.0;
        const bool zl = rb == 0 && x == 0;  // the lane of k = 0 (row 0)
        double amax = 0.0;
        for (int r0 = w; r0 < R; r0 += nw * U) {
            T qr[U], qi[U], nr[U], ni[U], q2r[U], q2i[U], n2r[U], n2i[U];
            double myz[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                qr[u] = qi[u] = nr[u] = ni[u] = q2r[u] = q2i[u] = n2r[u] = n2i[u] = (T)0;
                const int r = r0 + u * nw;  // wave-uniform
                const int z = z0 + (r >> lb1), y = y0 + (r & b1m);
                myz[u] = sq_d(sidx(z, n0)) + sq_d(sidx(y, n1));
                if (r < R && on) {
                    const int64_t e = ((int64_t)((z << ln1) + y)) * xs + x;
                    ld1<T>(q0p + 2 * e, qr[u], qi[u]);
                    if (!SI) ld1<T>(r0p + 2 * e, nr[u], ni[u]);
                    if (OP == OP_GS) {
                        ld1<T>(q1p + 2 * e, q2r[u], q2i[u]);
                        if (!SI) ld1<T>(r1p + 2 * e, n2r[u], n2i[u]);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (r0 + u * nw >= R) continue;  // wave-uniform
                const double m2 = myz[u] + mx2;
                double a = half_mode<T, OP, SI>(K, c0s, m2, qr[u], qi[u], nr[u], ni[u], q2r[u], q2i[u], n2r[u],
                                                n2i[u]);
                // k = 0: left out of the state measure; for FP32 its slot is
                // zero and the increment comes from the FP64 side path
                if (zl && r0 == 0 && u == 0 && (SI || I.k0path)) a = 0.0;
                bad |= !(a <= DBL_MAX);
                amax = fmax(amax, a);
                if (OP == OP_CH) esum += wgt * ((K.K2 * m2) * sq2((double)qr[u], (double)qi[u]));
            }
        }
        for (int off = 1; off < LB; off <<= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
        if (x < xh && (lane & (LB - 1)) == 0) hred[w * NB + bx] = fmax(hred[w * NB + bx], amax);
    }
    if (!SI && I.k0path && rb == 0 && threadIdx.x == 0) {  // the FP64 k = 0 candidate
        double tmp[2];
        const double a = k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
        bad |= !(a <= DBL_MAX);
        hred[0] = fmax(hred[0], a);
    }
    {  // the column nx/2: lanes over rows
        const int64_t gq = I.blk_off + I.nbm + rb;
        const bool qon = !(c.skip && c.skip[gq]);
        const double mx2 = sq_d(xh);
        double amax = 0.0;
        for (int r = threadIdx.x; r < R && qon; r += blockDim.x) {
            const int z = z0 + (r >> lb1), y = y0 + (r & b1m);
            const int64_t e = ((int64_t)((z << ln1) + y)) * xs + xh;
            T qr, qi, nr = (T)0, ni = (T)0, q2r = (T)0, q2i = (T)0, n2r = (T)0, n2i = (T)0;
            ld1<T>(q0p + 2 * e, qr, qi);
            if (!SI) ld1<T>(r0p + 2 * e, nr, ni);
            if (OP == OP_GS) {
                ld1<T>(q1p + 2 * e, q2r, q2i);
                if (!SI) ld1<T>(r1p + 2 * e, n2r, n2i);
            }
            const double m2 = sq_d(sidx(z, n0)) + sq_d(sidx(y, n1)) + mx2;
            const double a = half_mode<T, OP, SI>(K, c0s, m2, qr, qi, nr, ni, q2r, q2i, n2r, n2i);
            bad |= !(a <= DBL_MAX);
            amax = fmax(amax, a);
            if (OP == OP_CH) esum += (K.K2 * m2) * sq2((double)qr, (double)qi);
        }
        amax = wave_max(amax);
        if (lane == 0) hred[w * NB + nbxm] = fmax(hred[w * NB + nbxm], amax);
    }
    if (OP == OP_CH) {
        esum = wave_sum(esum);
        if (lane == 0) s_sum[w] = esum;
    }
    if (bad) atomicOr(c.nonfinite, 1u);
    __syncthreads();
    double gm = 0.0;
    for (int t = threadIdx.x; t <= nbxm; t += blockDim.x) {
        double m = hred[t];
        for (int k = 1; k < nw; ++k) m = fmax(m, hred[k * NB + t]);
        const int64_t lb = t < nbxm ? row_lb + t : I.nbm + rb;
        const int64_t gb = I.blk_off + lb;
        if (c.skip && c.skip[gb] && !(I.pin && lb == 0)) m = 0.0;
        c.a_b[gb] = m;
        gm = fmax(gm, m);
    }
    gm = wave_max(gm);
    if (lane == 0) s_max[w] = gm;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = s_max[0];
        for (int k = 1; k < nw; ++k) m = fmax(m, s_max[k]);
        if (strip == 0) *c.count = 0u;  // the one-pass compaction appends to it
        if (m > 0.0) atomicMax(c.G + ii, (unsigned long long)__double_as_longlong(m));
        if (OP == OP_CH) {
            double ts = 0.0;
            for (int k = 0; k < nw; ++k) ts += s_sum[k];
            c.ind_part[strip] = ts;
        }
    }
}

// Update of one listed block on the half layout (as update_block, one
// complex value per lane; the column-nx/2 blocks are one column wide).  Each
// thread issues the loads of two slots before it computes either, so a block
// of 512 values is one round trip for 256 threads.  red: two sets of per-wave
// maxima used alternately (par), so one barrier per block suffices.
// TR: the entry carries the transition flag and the frozen-face bits; a
// transition block takes q + sigma (q' - q) with sigma from the roll-off
// tables in sig (the column nx/2 has edge 1 along x).
template <typename T, int OP, bool TR>
__device__ __forceinline__ void update_block_h(const Ctx &c, uint32_t entry, double (*red)[4], int par,
                                               const double *sig) {
    constexpr int UB = 2;
    const int64_t gb = TR ? (int64_t)(entry & kEntryId) : (int64_t)entry;
    const bool trn = TR && (entry >> 31);  // workgroup-uniform
    const uint32_t faces = (entry >> 25) & 63u;
    const int ii = c.blk_inst[gb];
    const InstDev &I = c.inst[ii];
    const int64_t lb = gb - I.blk_off;
    const bool nyq = lb >= I.nbm;  // workgroup-uniform
    int bz, by, x_blk, lbx;
    if (!nyq) {
        const int64_t t = lb >> I.lnbxm;
        x_blk = (int)(lb & (I.nbxm - 1)) << I.lb[2];
        by = (int)(t & (I.nbk[1] - 1));
        bz = (int)(t >> I.lnbk[1]);
        lbx = I.lb[2];
    } else {
        const int64_t j = lb - I.nbm;
        by = (int)(j & (I.nbk[1] - 1));
        bz = (int)(j >> I.lnbk[1]);
        x_blk = I.n[2] >> 1;
        lbx = 0;
    }
    const int slots = (I.b[0] * I.b[1]) << lbx;
    const Coef K = Coef::of(I);
    const int lb1 = I.lb[1], b1m = I.b[1] - 1, ln1 = I.ln[1];
    const int bxe = 1 << lbx;  // block edge along x: 1 for the column nx/2
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2], xs = I.xs;
    const int z0 = bz << I.lb[0], y0 = by << lb1;
    const bool k0_blk = I.k0path && lb == 0;
    T *q0p = reinterpret_cast<T *>(c.state) + 2 * I.off;
    const T *r0p = reinterpret_cast<const T *>(c.rhs) + 2 * I.off;
    T *q1p = q0p + 2 * I.N;
    const T *r1p = r0p + 2 * I.N;
    const T dt = (OP == OP_GS) ? (T)K.c0 : (T)0;
    const bool ab = c.ab_inc;  // workgroup-uniform
    double amax = 0.0;
    const int step = blockDim.x;
    for (int s0 = threadIdx.x; s0 < slots; s0 += UB * step) {
        T qr[UB], qi[UB], nr[UB], ni[UB], q2r[UB], q2i[UB], n2r[UB], n2i[UB];
        int64_t e[UB];
        double m2[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int s = s0 + u * step;
            qr[u] = qi[u] = nr[u] = ni[u] = q2r[u] = q2i[u] = n2r[u] = n2i[u] = (T)0;
            e[u] = -1;
            if (s >= slots) continue;
            const int r = s >> lbx, l = s & ((1 << lbx) - 1);
            const int z = z0 + (r >> lb1), y = y0 + (r & b1m), x = x_blk + l;
            e[u] = ((int64_t)((z << ln1) + y)) * xs + x;
            const double mx = (double)sidx(x, n2);
            m2[u] = __builtin_fma(mx, mx, sq_d(sidx(z, n0)) + sq_d(sidx(y, n1)));
            ld1<T>(q0p + 2 * e[u], qr[u], qi[u]);
            ld1<T>(r0p + 2 * e[u], nr[u], ni[u]);
            if (OP == OP_GS) {
                ld1<T>(q1p + 2 * e[u], q2r[u], q2i[u]);
                ld1<T>(r1p + 2 * e[u], n2r[u], n2i[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            if (e[u] < 0) continue;
            T cr, ci, dr = (T)0, di = (T)0;
            if (OP == OP_CH) {
                T sc, f;
                ch_coef<T>(K, m2[u], sc, f);
                ch_cand<T>(sc, f, qr[u], qi[u], nr[u], ni[u], cr, ci);
            } else {
                T au, av;
                gs_coef<T>(K, m2[u], au, av);
                gs_cand<T>(dt, au, qr[u], qi[u], nr[u], ni[u], cr, ci);
                gs_cand<T>(dt, av, q2r[u], q2i[u], n2r[u], n2i[u], dr, di);
            }
            if (TR && trn) {
                const int s = s0 + u * step, r = s >> lbx;
                const T sg = (T)sigma_at(sig, faces, I.b[0], I.b[1], bxe, r >> lb1, r & b1m, s & (bxe - 1));
                cr = fmat(sg, cr - qr[u], qr[u]);
                ci = fmat(sg, ci - qi[u], qi[u]);
                if (OP == OP_GS) {
                    dr = fmat(sg, dr - q2r[u], q2r[u]);
                    di = fmat(sg, di - q2i[u], q2i[u]);
                }
            }
            if (k0_blk && e[u] == 0) cr = ci = dr = di = (T)0;  // the FP32 slot of k = 0 stays zero
            if (ab) {  // the state measure of what is stored; k = 0 left out
                double a = sq2((double)cr, (double)ci);
                if (OP == OP_GS) a = a + sq2((double)dr, (double)di);
                if (lb == 0 && e[u] == 0) a = 0.0;
                amax = fmax(amax, a);
            }
            st1<T>(q0p + 2 * e[u], cr, ci);
            if (OP == OP_GS) st1<T>(q1p + 2 * e[u], dr, di);
        }
    }
    if (ab) {
        amax = wave_max(amax);
        if ((threadIdx.x & 63) == 0) red[par][threadIdx.x >> 6] = amax;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = red[par][0];
            for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = fmax(m, red[par][k]);
            c.a_next[gb] = m;
        }
    }
    if (k0_blk && threadIdx.x == 0) {
        double tmp[2];
        k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
        if (TR && trn) {  // block 0 in transition: the weighted increment in FP64
            const double s0 = sigma_at(sig, faces, I.b[0], I.b[1], bxe, 0, 0, 0);
            tmp[0] = __builtin_fma(s0, tmp[0] - c.k0[2 * ii], c.k0[2 * ii]);
            if (OP == OP_GS) tmp[1] = __builtin_fma(s0, tmp[1] - c.k0[2 * ii + 1], c.k0[2 * ii + 1]);
        }
        c.k0[2 * ii] = tmp[0];
        if (OP == OP_GS) c.k0[2 * ii + 1] = tmp[1];
    }
}

// persistent walk of the appended list, one segment per XCD (as k_update);
// CTL: workgroup 0 first closes the update's control step and hands G over;
// TR: the roll-off tables are copied into dynamic LDS once per workgroup
template <typename T, int OP, bool TR, bool CTL>
__global__ void __launch_bounds__(256) k_update_h(Ctx c) {
    extern __shared__ double sig[];
    __shared__ double red[2][4];
    if (CTL && blockIdx.x == 0 && threadIdx.x < 64)
        for (int i = threadIdx.x; i < c.n_inst; i += 64) {
            control_inst(c, i);
            c.G_last[i] = c.G[i];
            c.G[i] = 0ull;
        }
    if (TR) {
        for (uint32_t bs = c.taper_bs; bs; bs &= bs - 1) {
            const int B = 1 << __builtin_ctz(bs);
            for (int i = threadIdx.x; i < B; i += blockDim.x) sig[B + i] = c.taper[B + i];
        }
        __syncthreads();
    }
    const uint32_t total = *c.count;
    const int P = gridDim.x;  // multiple of 8
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, per = P >> 3;
    const uint32_t seg = (total + 7) / 8;
    const uint32_t lo = min(total, seg * xcd), hi = min(total, seg * (xcd + 1));
    int par = 0;
    for (uint32_t e = lo + local; e < hi; e += per, par ^= 1)
        update_block_h<T, OP, TR>(c, c.worklist[e], red, par, sig);
}

// Regular mode on the half layout: every stored mode, tiles of tile_elems
// consecutive values (rows are contiguous); FP64 gradient-energy partials
// per tile for CH (every tile writes its partial, zero past the data).
template <typename T, int OP>
__global__ void __launch_bounds__(1024) k_dense_h(Ctx c) {
    constexpr int TE = tile_elems<T>();
    __shared__ double lds[16];
    const int64_t tile = blockIdx.x;
    const int ii = find_by_offset(c.inst, c.n_inst, tile, 1);
    const InstDev &I = c.inst[ii];
    const int64_t t0 = (tile - I.tile_off) * TE;
    const Coef K = Coef::of(I);
    const int64_t N = I.N;
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2], ln1 = I.ln[1], xs = I.xs, xh = n2 >> 1;
    const bool k0_tile = I.k0path && t0 == 0;
    T *q0p = reinterpret_cast<T *>(c.state) + 2 * I.off;
    const T *r0p = reinterpret_cast<const T *>(c.rhs) + 2 * I.off;
    T *q1p = q0p + 2 * N;
    const T *r1p = r0p + 2 * N;
    const T dt = (OP == OP_GS) ? (T)K.c0 : (T)0;
    double acc[1] = {0.0};
    // (row, x) of this thread's first value, then a fixed stride
    const int64_t e0 = t0 + threadIdx.x;
    int64_t row = e0 / xs;
    int x = (int)(e0 - row * xs);
    const int drow = (int)(blockDim.x / xs), dx = (int)(blockDim.x - drow * xs);
    for (int j = threadIdx.x; j < TE; j += blockDim.x) {
        const int64_t e = t0 + j;
        if (e >= N) break;
        if (x > xh) {  // a padding column of the row pitch
            x += dx;
            row += drow;
            if (x >= xs) {
                x -= xs;
                ++row;
            }
            continue;
        }
        const int y = (int)(row & (n1 - 1));
        const int z = (int)(row >> ln1);
        const double mx = (double)sidx(x, n2);
        const double m2 = __builtin_fma(mx, mx, sq_d(sidx(z, n0)) + sq_d(sidx(y, n1)));
        T qr, qi, nr, ni, q2r = (T)0, q2i = (T)0, n2r, n2i;
        ld1<T>(q0p + 2 * e, qr, qi);
        ld1<T>(r0p + 2 * e, nr, ni);
        if (OP == OP_GS) {
            ld1<T>(q1p + 2 * e, q2r, q2i);
            ld1<T>(r1p + 2 * e, n2r, n2i);
        }
        T cr, ci, dr = (T)0, di = (T)0;
        if (OP == OP_CH) {
            T s, f;
            ch_coef<T>(K, m2, s, f);
            const double wgt = (x == 0 || x == xh) ? 1.0 : 2.0;
            acc[0] += wgt * ((K.K2 * m2) * sq2((double)qr, (double)qi));
            ch_cand<T>(s, f, qr, qi, nr, ni, cr, ci);
        } else {
            T au, av;
            gs_coef<T>(K, m2, au, av);
            gs_cand<T>(dt, au, qr, qi, nr, ni, cr, ci);
            gs_cand<T>(dt, av, q2r, q2i, n2r, n2i, dr, di);
        }
        if (k0_tile && j == 0) cr = ci = dr = di = (T)0;  // the FP32 slot of k = 0 stays zero
        st1<T>(q0p + 2 * e, cr, ci);
        if (OP == OP_GS) st1<T>(q1p + 2 * e, dr, di);
        x += dx;
        row += drow;
        if (x >= xs) {
            x -= xs;
            ++row;
        }
    }
    if (k0_tile && threadIdx.x == 0) {
        double tmp[2];
        k0_cand(I, OP, c.k0 + 2 * ii, c.rhs_k0 + 2 * ii, tmp);
        c.k0[2 * ii] = tmp[0];
        if (OP == OP_GS) c.k0[2 * ii + 1] = tmp[1];
    }
    if (OP == OP_CH) {
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) c.dense_part[tile] = acc[0];
    }
}

// compact half spectrum (nspec x nz*ny rows of nx/2 + 1) <-> pitched state layout
template <typename T>
__global__ void k_copy_half(Ctx c, int ii, const T *src, T *dst, int to_pitched, int zero_slot0, double *k0_dst) {
    const InstDev &I = c.inst[ii];
    const int64_t w = (I.n[2] >> 1) + 1;
    const int64_t nc = (int64_t)I.n[0] * I.n[1] * w;  // compact values per species
    const int64_t n = nc * I.nspec;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / nc, j = i - s * nc;
        const int64_t row = j / w;
        const int64_t pi = s * I.N + row * I.xs + (j - row * w);
        if (to_pitched) {
            T re = src[2 * i], im = src[2 * i + 1];
            if (j == 0) {
                if (k0_dst) k0_dst[s] = (double)re;
                if (zero_slot0) {
                    re = (T)0;
                    im = (T)0;
                }
            }
            dst[2 * pi] = re;
            dst[2 * pi + 1] = im;
        } else {
            dst[2 * i] = src[2 * pi];
            dst[2 * i + 1] = src[2 * pi + 1];
        }
    }
}

// real field (nspec x Nreal values, caller's array) -> the instance's reals in W
template <typename T>
__global__ void k_real_to_slots(Ctx c, int ii, const T *real) {
    const InstDev &I = c.inst[ii];
    T *w = reinterpret_cast<T *>(c.work) + I.roff;
    const int64_t n = I.Nreal * I.nspec;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        w[i] = real[i];
}

// out[s][i] = W_s[i] / N + mean_s (the inverse of the half spectrum in W)
template <typename T>
__global__ void k_slots_to_real(Ctx c, int ii, T *out) {
    const InstDev &I = c.inst[ii];
    const T *w = reinterpret_cast<const T *>(c.work) + I.roff;
    const int64_t n = I.Nreal * I.nspec;
    const T invN = (T)I.invN;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / I.Nreal;
        const T mean = I.k0path ? (T)(c.k0[2 * ii + s] * I.invN) : (T)0;
        out[i] = w[i] * invN + mean;
    }
}

// -------------------------------------------------------------------------
// launchers
// -------------------------------------------------------------------------

template <typename T>
static hipError_t nl_launch(const Ctx &c, int waves, hipStream_t s) {
    dim3 grid((unsigned)c.n_tiles), block(64 * waves);
    if (c.half) {
        if (c.op == OP_CH) hipLaunchKernelGGL((k_nonlinear_h<T, OP_CH>), grid, block, 0, s, c);
        else hipLaunchKernelGGL((k_nonlinear_h<T, OP_GS>), grid, block, 0, s, c);
        return hipGetLastError();
    }
    if (c.op == OP_CH) hipLaunchKernelGGL((k_nonlinear<T, OP_CH>), grid, block, 0, s, c);
    else if (c.op == OP_GS) hipLaunchKernelGGL((k_nonlinear<T, OP_GS>), grid, block, 0, s, c);
    else if (c.op == OP_XPFC) hipLaunchKernelGGL((k_nonlinear<T, OP_XPFC>), grid, block, 0, s, c);
    else hipLaunchKernelGGL((k_nonlinear<T, OP_NLSE>), grid, block, 0, s, c);
    return hipGetLastError();
}
hipError_t launch_nonlinear(const Ctx &c, bool dbl, int waves, hipStream_t s) {
    return dbl ? nl_launch<double>(c, waves, s) : nl_launch<float>(c, waves, s);
}

hipError_t launch_k0_rhs(const Ctx &c, hipStream_t s) {
    hipLaunchKernelGGL(k_k0_total, dim3(c.n_inst), dim3(256), 0, s, c, 0, -1);
    return hipGetLastError();
}

// one indicator dispatch: the kernel variant for (T, OP, EB, SI), with an
// event pair the dispatch itself stamps its start and end
template <typename T, int OP, bool EB, bool SI>
static void ind_launch_v(const Ctx &c, int waves, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (c.wave_ind) {  // one wave per strip, 16 strips per workgroup
        const dim3 gw((unsigned)((c.n_strips + 15) / 16)), b(1024);
        if (OP == OP_NLSE && c.htab_all)
            hipExtLaunchKernelGGL((k_indicator_wave<T, OP, EB, true, SI>), gw, b, 0, s, e0, e1, 0, c);
        else
            hipExtLaunchKernelGGL((k_indicator_wave<T, OP, EB, false, SI>), gw, b, 0, s, e0, e1, 0, c);
        return;
    }
    hipExtLaunchKernelGGL((k_indicator<T, OP, EB, SI>), dim3((unsigned)c.n_strips), dim3(64 * waves), 0, s, e0, e1,
                          0, c);
}
template <typename T, int OP>
static void ind_launch_op(const Ctx &c, int waves, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (c.e_b) {
        if (c.state_ind) ind_launch_v<T, OP, true, true>(c, waves, s, e0, e1);
        else ind_launch_v<T, OP, true, false>(c, waves, s, e0, e1);
    } else {
        if (c.state_ind) ind_launch_v<T, OP, false, true>(c, waves, s, e0, e1);
        else ind_launch_v<T, OP, false, false>(c, waves, s, e0, e1);
    }
}
template <typename T, int OP>
static void ind_launch_half(const Ctx &c, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 grid((unsigned)c.n_strips), block(256);
    const size_t lds = (size_t)4 * c.half_nb * sizeof(double);
    if (c.state_ind) hipExtLaunchKernelGGL((k_indicator_h<T, OP, true>), grid, block, lds, s, e0, e1, 0, c);
    else hipExtLaunchKernelGGL((k_indicator_h<T, OP, false>), grid, block, lds, s, e0, e1, 0, c);
}
template <typename T>
static hipError_t ind_launch(const Ctx &c, int waves, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (c.half) {  // four waves per workgroup
        if (c.op == OP_CH) ind_launch_half<T, OP_CH>(c, s, e0, e1);
        else ind_launch_half<T, OP_GS>(c, s, e0, e1);
        return hipGetLastError();
    }
    if (c.op == OP_CH) ind_launch_op<T, OP_CH>(c, waves, s, e0, e1);
    else if (c.op == OP_GS) ind_launch_op<T, OP_GS>(c, waves, s, e0, e1);
    else if (c.op == OP_XPFC) {  // the state-amplitude measures only
        if (c.e_b) ind_launch_v<T, OP_XPFC, true, true>(c, waves, s, e0, e1);
        else ind_launch_v<T, OP_XPFC, false, true>(c, waves, s, e0, e1);
    } else ind_launch_op<T, OP_NLSE>(c, waves, s, e0, e1);
    return hipGetLastError();
}
hipError_t launch_indicator(const Ctx &c, bool dbl, int waves, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return dbl ? ind_launch<double>(c, waves, s, e0, e1) : ind_launch<float>(c, waves, s, e0, e1);
}

hipError_t launch_compact_append(const Ctx &c, hipStream_t s) {
    hipLaunchKernelGGL(k_compact_append, dim3((unsigned)c.n_chunks), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_compact_runs(const Ctx &c, hipStream_t s) {
    const int64_t per = 256 * RUN_GROUP;
    hipLaunchKernelGGL(k_compact_runs, dim3((unsigned)((c.nb_total + per - 1) / per)), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_gmax(const Ctx &c, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    hipExtLaunchKernelGGL(k_gmax, dim3((unsigned)((c.nb_total + 256 * GMAX_PER - 1) / (256 * GMAX_PER))), dim3(256), 0,
                          s, e0, e1, 0, c);
    return hipGetLastError();
}

hipError_t launch_compact_states(const Ctx &c, hipStream_t s) {
    hipLaunchKernelGGL(k_compact_states, dim3((unsigned)((c.nb_total + 255) / 256)), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_ctl_reset(const Ctx &c, int only_inst, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, s, c, only_inst);
    return hipGetLastError();
}

hipError_t launch_htable(const Ctx &c, bool dbl, hipStream_t s) {
    const dim3 grid(64, (unsigned)c.n_inst);
    if (dbl) hipLaunchKernelGGL(k_htable<double>, grid, dim3(256), 0, s, c);
    else hipLaunchKernelGGL(k_htable<float>, grid, dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_tapers(const Ctx &c, hipStream_t s) {
    hipLaunchKernelGGL(k_tapers, dim3(32), dim3(256), 0, s, c, const_cast<double *>(c.taper));
    return hipGetLastError();
}

hipError_t launch_compact(const Ctx &c, hipStream_t s, int from_mask) {
    hipLaunchKernelGGL(k_compact_count, dim3((unsigned)c.n_chunks), dim3(256), 0, s, c, from_mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_compact_write, dim3((unsigned)c.n_chunks), dim3(256), 0, s, c);
    return hipGetLastError();
}

// aux of a BlockStage: the instance record and the owner table (all
// instance 0), each 256-byte aligned
static size_t stage_al(size_t o) { return (o + 255) & ~(size_t)255; }
static int64_t stage_chunks(int64_t nb) { return (nb + CHUNK_BLOCKS - 1) / CHUNK_BLOCKS; }

size_t block_stage_bytes(int64_t nb) {
    return stage_al(stage_al(sizeof(InstDev)) + sizeof(uint16_t) * (size_t)nb);
}

static Ctx stage_ctx(const BlockStage &b) {
    char *aux = static_cast<char *>(b.aux);
    Ctx c{};
    c.inst = reinterpret_cast<const InstDev *>(aux);
    c.n_inst = 1;
    c.blk_inst = reinterpret_cast<const uint16_t *>(aux + stage_al(sizeof(InstDev)));
    c.a_b = b.a_b;
    c.a_next = const_cast<double *>(b.a_next);
    c.mask = b.mask;
    c.worklist = b.list;
    c.count = b.count;
    c.G = b.G;  // G_last stays null: the append keeps G
    c.nb_total = b.nb;
    c.n_chunks = stage_chunks(b.nb);
    return c;
}

hipError_t block_stage_init(const BlockStage &b, double tau2, int pin, hipStream_t s) {
    InstDev I{};
    I.nb = b.nb;
    I.tau2 = tau2;
    I.pin = pin;
    const Ctx c = stage_ctx(b);
    hipError_t e = hipMemcpyAsync(const_cast<InstDev *>(c.inst), &I, sizeof(I), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(const_cast<uint16_t *>(c.blk_inst), 0, sizeof(uint16_t) * (size_t)b.nb, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // I lives on this stack frame
    return e;
}

hipError_t launch_block_stage(const BlockStage &b, hipStream_t s) {
    const Ctx c = stage_ctx(b);
    hipError_t e = launch_gmax(c, s);  // also clears the list counter
    if (e != hipSuccess) return e;
    return launch_compact_append(c, s);
}

template <typename T, int OP>
static void upd_launch_op(const Ctx &c, int grid, int multi, bool tr, bool ctl, hipStream_t s) {
    if (ctl && tr)
        hipLaunchKernelGGL((k_update<T, OP, true, true>), dim3(grid), dim3(256), (size_t)c.sig_bytes, s, c);
    else if (ctl) hipLaunchKernelGGL((k_update<T, OP, false, true>), dim3(grid), dim3(256), 0, s, c);
    else if (multi == 3) {  // the run walk: CH and GS
        if constexpr (OP == OP_CH || OP == OP_GS) {
            if (c.run_ub == 8) hipLaunchKernelGGL((k_update_run<T, OP, 8>), dim3(grid), dim3(256), 0, s, c);
            else hipLaunchKernelGGL((k_update_run<T, OP, 4>), dim3(grid), dim3(256), 0, s, c);
        }
    } else if (multi == 2) hipLaunchKernelGGL((k_update_wave<T, OP>), dim3(grid), dim3(256), 0, s, c);
    else if (multi && OP != OP_XPFC) {  // four entries in flight: not with a kept measure, so never XPFC
        if constexpr (OP != OP_XPFC) hipLaunchKernelGGL((k_update_multi<T, OP, 4>), dim3(grid), dim3(256), 0, s, c);
    }
    else hipLaunchKernelGGL((k_update<T, OP, false, false>), dim3(grid), dim3(256), 0, s, c);
}
template <typename T>
static hipError_t upd_launch(const Ctx &c, int grid, int multi, bool tr, bool ctl, hipStream_t s) {
    if (c.half) {  // the block-list walk only
        const size_t lds = tr ? (size_t)c.sig_bytes : 0;
        if (c.op == OP_CH) {
            if (ctl && tr) hipLaunchKernelGGL((k_update_h<T, OP_CH, true, true>), dim3(grid), dim3(256), lds, s, c);
            else if (ctl) hipLaunchKernelGGL((k_update_h<T, OP_CH, false, true>), dim3(grid), dim3(256), 0, s, c);
            else hipLaunchKernelGGL((k_update_h<T, OP_CH, false, false>), dim3(grid), dim3(256), 0, s, c);
        } else {
            if (ctl && tr) hipLaunchKernelGGL((k_update_h<T, OP_GS, true, true>), dim3(grid), dim3(256), lds, s, c);
            else if (ctl) hipLaunchKernelGGL((k_update_h<T, OP_GS, false, true>), dim3(grid), dim3(256), 0, s, c);
            else hipLaunchKernelGGL((k_update_h<T, OP_GS, false, false>), dim3(grid), dim3(256), 0, s, c);
        }
        return hipGetLastError();
    }
    if (c.op == OP_CH) upd_launch_op<T, OP_CH>(c, grid, multi, tr, ctl, s);
    else if (c.op == OP_GS) upd_launch_op<T, OP_GS>(c, grid, multi, tr, ctl, s);
    else if (c.op == OP_XPFC) upd_launch_op<T, OP_XPFC>(c, grid, multi == 1 ? 0 : multi, tr, ctl, s);
    else upd_launch_op<T, OP_NLSE>(c, grid, multi, tr, ctl, s);
    return hipGetLastError();
}
hipError_t launch_update(const Ctx &c, bool dbl, int grid, int multi, hipStream_t s, bool tr, bool ctl) {
    return dbl ? upd_launch<double>(c, grid, multi, tr, ctl, s) : upd_launch<float>(c, grid, multi, tr, ctl, s);
}

template <typename T>
static hipError_t upd_strip_launch(const Ctx &c, int waves, int grid, hipStream_t s) {
    dim3 g((unsigned)grid), block(64 * waves);
    if (c.op == OP_CH) hipLaunchKernelGGL((k_update_strip<T, OP_CH>), g, block, 0, s, c);
    else if (c.op == OP_GS) hipLaunchKernelGGL((k_update_strip<T, OP_GS>), g, block, 0, s, c);
    else if (c.op == OP_XPFC) return hipErrorInvalidValue;  // the strip walk is the increment measure's
    else hipLaunchKernelGGL((k_update_strip<T, OP_NLSE>), g, block, 0, s, c);
    return hipGetLastError();
}
hipError_t launch_update_strip(const Ctx &c, bool dbl, int waves, int grid, hipStream_t s) {
    return dbl ? upd_strip_launch<double>(c, waves, grid, s) : upd_strip_launch<float>(c, waves, grid, s);
}

template <typename T>
static hipError_t dense_launch(const Ctx &c, int threads, hipStream_t s) {
    dim3 grid((unsigned)c.n_tiles), block(threads);
    if (c.half) {
        if (c.op == OP_CH) hipLaunchKernelGGL((k_dense_h<T, OP_CH>), grid, block, 0, s, c);
        else hipLaunchKernelGGL((k_dense_h<T, OP_GS>), grid, block, 0, s, c);
        return hipGetLastError();
    }
    if (c.op == OP_CH) hipLaunchKernelGGL((k_dense<T, OP_CH>), grid, block, 0, s, c);
    else if (c.op == OP_GS) hipLaunchKernelGGL((k_dense<T, OP_GS>), grid, block, 0, s, c);
    else if (c.op == OP_XPFC) hipLaunchKernelGGL((k_dense<T, OP_XPFC>), grid, block, 0, s, c);
    else hipLaunchKernelGGL((k_dense<T, OP_NLSE>), grid, block, 0, s, c);
    return hipGetLastError();
}
hipError_t launch_dense(const Ctx &c, bool dbl, int threads, hipStream_t s) {
    return dbl ? dense_launch<double>(c, threads, s) : dense_launch<float>(c, threads, s);
}

hipError_t launch_reset(const Ctx &c, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, c);
    return hipGetLastError();
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

hipError_t launch_real_to_complex(const Ctx &c, bool dbl, int inst, const void *real, int64_t n,
                                  hipStream_t s) {
    if (c.half) {  // n = nspec x grid points
        if (dbl) hipLaunchKernelGGL(k_real_to_slots<double>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (const double *)real);
        else hipLaunchKernelGGL(k_real_to_slots<float>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (const float *)real);
        return hipGetLastError();
    }
    if (dbl) hipLaunchKernelGGL(k_real_to_complex<double>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (const double *)real);
    else hipLaunchKernelGGL(k_real_to_complex<float>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (const float *)real);
    return hipGetLastError();
}

hipError_t launch_real_sums_to_k0(const Ctx &c, bool dbl, int inst, const void *real,
                                  int64_t ntiles, hipStream_t s) {
    if (dbl) hipLaunchKernelGGL(k_real_tile_sums<double>, dim3((unsigned)ntiles), dim3(256), 0, s, c, inst, (const double *)real);
    else hipLaunchKernelGGL(k_real_tile_sums<float>, dim3((unsigned)ntiles), dim3(256), 0, s, c, inst, (const float *)real);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_k0_total, dim3(1), dim3(256), 0, s, c, 1, inst);
    return hipGetLastError();
}

hipError_t launch_work_to_real(const Ctx &c, bool dbl, int inst, void *out, int64_t n,
                               hipStream_t s) {
    if (c.half) {  // n = nspec x grid points
        if (dbl) hipLaunchKernelGGL(k_slots_to_real<double>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (double *)out);
        else hipLaunchKernelGGL(k_slots_to_real<float>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (float *)out);
        return hipGetLastError();
    }
    if (dbl) hipLaunchKernelGGL(k_work_to_real<double>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (double *)out);
    else hipLaunchKernelGGL(k_work_to_real<float>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (float *)out);
    return hipGetLastError();
}

hipError_t launch_scale_copy(bool dbl, const void *src, void *dst, int64_t n, double scale,
                             hipStream_t s) {
    if (dbl) hipLaunchKernelGGL(k_scale_copy<double>, dim3(grid_for(2 * n)), dim3(256), 0, s, n, (const double *)src, (double *)dst, scale);
    else hipLaunchKernelGGL(k_scale_copy<float>, dim3(grid_for(2 * n)), dim3(256), 0, s, n, (const float *)src, (float *)dst, (float)scale);
    return hipGetLastError();
}

hipError_t launch_copy_spectrum(const Ctx &c, bool dbl, int inst, const void *src, void *dst,
                                int64_t n, int zero_slot0, double *k0_dst, hipStream_t s) {
    if (dbl) hipLaunchKernelGGL(k_copy_spectrum<double>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (const double *)src, (double *)dst, zero_slot0, k0_dst);
    else hipLaunchKernelGGL(k_copy_spectrum<float>, dim3(grid_for(n)), dim3(256), 0, s, c, inst, (const float *)src, (float *)dst, zero_slot0, k0_dst);
    return hipGetLastError();
}

hipError_t launch_copy_half(const Ctx &c, bool dbl, int inst, const void *src, void *dst, bool to_pitched,
                            int zero_slot0, double *k0_dst, hipStream_t s) {
    const unsigned g = 4096;
    if (dbl) hipLaunchKernelGGL(k_copy_half<double>, dim3(g), dim3(256), 0, s, c, inst, (const double *)src, (double *)dst, to_pitched ? 1 : 0, zero_slot0, k0_dst);
    else hipLaunchKernelGGL(k_copy_half<float>, dim3(g), dim3(256), 0, s, c, inst, (const float *)src, (float *)dst, to_pitched ? 1 : 0, zero_slot0, k0_dst);
    return hipGetLastError();
}

hipError_t launch_copy8(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 8);
    hipLaunchKernelGGL(k_copy8, dim3(grid_for(n)), dim3(256), 0, s, (const unsigned long long *)src,
                       (unsigned long long *)dst, n);
    return hipGetLastError();
}

hipError_t launch_fill_pattern(void *buf, int64_t n, bool dbl, hipStream_t s) {
    if (dbl) hipLaunchKernelGGL(k_fill_pattern<double>, dim3(grid_for(2 * n)), dim3(256), 0, s, (double *)buf, n);
    else hipLaunchKernelGGL(k_fill_pattern<float>, dim3(grid_for(2 * n)), dim3(256), 0, s, (float *)buf, n);
    return hipGetLastError();
}
hipError_t launch_check_pattern(const void *buf, int64_t n, bool dbl, uint32_t *bad, hipStream_t s) {
    if (dbl) hipLaunchKernelGGL(k_check_pattern<double>, dim3(grid_for(2 * n)), dim3(256), 0, s, (const double *)buf, n, bad);
    else hipLaunchKernelGGL(k_check_pattern<float>, dim3(grid_for(2 * n)), dim3(256), 0, s, (const float *)buf, n, bad);
    return hipGetLastError();
}

}  // namespace spdba
