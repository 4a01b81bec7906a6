// sp-DBA for multicomponent reaction--cross-diffusion (Supplementary S4):
// kernels and the C ABI of include/spdba_rcd.h.
//
// Kernels (one plan, one instance, M components stored component after
// component, N modes each):
//   k_rcd_reaction   real space: u = Re(W)/N per component, W <- R(u) (S4.1)
//   k_rcd_measure    per block: a_b = max over modes of sum_m |q_m|^2 (FP64,
//                    components in order, k = 0 left out); one workgroup per
//                    block; clears the block's mask (no kept measure to merge)
//   G, the threshold, the mask and the list of active blocks: the
//                    block-activity stage of the main plan (spdba::launch_block_stage;
//                    after an update G merges the measure the update kept for
//                    the blocks it stored)
//   k_rcd_update     persistent walk of the list (or of every block for the
//                    Regular update): per mode b = q + dt R, then the eigen form
//                    of S4.3, x = V diag(1/(1 + dt k^2 lambda)) V^T b, with V^T
//                    and lambda in LDS (read as broadcasts) and b, x in
//                    registers (MM-wide tiles, zero-padded past M); it also
//                    keeps the measure of every block it stores (the next
//                    update's state is what it stored, frozen blocks are
//                    unchanged), so only a load is followed by a full pass;
//                    with the direct form of S4.2 a per-mode Cholesky solve
//                    of I + dt k^2 D in one thread's registers (M <= 8)
//   k_rcd_update_direct  the direct form for M > 8: one wave per mode, a row
//                    of [A | b] per lane, elimination and back substitution
//                    with the pivot row's entries broadcast from its lane
//
// The per-mode contraction moves 24 M bytes (FP32) for 4 MM^2 FMAs; up to
// MM = 16 that is well below the balance point of FP32 vector arithmetic
// against HBM, so it runs on the vector units (tiles 2, 4, 8, 16 in FP32 and
// 2, 4, 8 in FP64, the widths whose operands stay in registers without
// scratch).  Wider FP32 tiles (32, 48, 64) are dense contractions and run as two
// GEMMs per chunk of modes on the matrix cores (k_rcd_update_mfma).

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "spdba_internal.h"
#include "spdba_rcd.h"

namespace {

constexpr double kTwoPiR = 6.283185307179586476925286766559;
constexpr int kMaxMF32 = 64, kMaxMF64 = 48;  // register tiles to 16 (FP32) / 8 (FP64), then matrix-core GEMMs
constexpr int kMaxMReg = 8;  // the direct form's factor in one thread's registers: MM (MM + 1) / 2 values

struct RGeo {
    int n[3], ln[3], b[3], lb[3], nbk[3], lnbk[3];
    int64_t N, nb;
    int bvol, lbvol;
    double kf[3];  // 2 pi / (n dx) per axis
};

struct RCtx {
    RGeo g;
    int M;
    void *state;         // M x N complex
    const void *rhs;     // M x N complex
    double *ab;          // [nb]
    double *anext;       // [nb] measure of the blocks the update stored
    int keep;            // the update writes anext
    uint8_t *mask;       // [nb]
    uint32_t *list;      // [nb]
    uint32_t *count;     // active blocks
    unsigned long long *G;
    const void *vt;      // [MM][MM] V^T, zero-padded
    const void *dm;      // [MM][MM] D, zero-padded (direct form)
    int direct;
    const void *lam;     // [MM], zero-padded
    double tau2, dt, invN;
    double alpha, beta, r, a;
    int pin, dense, mm;
};

__device__ __forceinline__ double rsq2(double x, double y) { return x * x + y * y; }

// signed frequency index of position i on an axis of n points (n = 1: 0)
__device__ __forceinline__ int rsidx(int i, int n) { return i <= ((n - 1) >> 1) ? i : i - n; }

__device__ __forceinline__ double rwave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <typename T> struct C2;
template <> struct C2<float> { using t = float2; };
template <> struct C2<double> { using t = double2; };

// mode index and |k|^2 of slot s of block b
__device__ __forceinline__ void mode_of(const RGeo &g, int64_t b, int s, int64_t &e, double &k2) {
    const int bx = (int)(b & (g.nbk[2] - 1));
    const int by = (int)((b >> g.lnbk[2]) & (g.nbk[1] - 1));
    const int bz = (int)(b >> (g.lnbk[2] + g.lnbk[1]));
    const int lx = s & (g.b[2] - 1);
    const int ly = (s >> g.lb[2]) & (g.b[1] - 1);
    const int lz = s >> (g.lb[2] + g.lb[1]);
    const int z = (bz << g.lb[0]) + lz, y = (by << g.lb[1]) + ly, x = (bx << g.lb[2]) + lx;
    e = ((((int64_t)z << g.ln[1]) + y) << g.ln[2]) + x;
    const double kz = rsidx(z, g.n[0]) * g.kf[0], ky = rsidx(y, g.n[1]) * g.kf[1], kx = rsidx(x, g.n[2]) * g.kf[2];
    k2 = kz * kz + ky * ky + kx * kx;
}

__global__ void k_rcd_reset(RCtx c) {
    if (threadIdx.x == 0) {
        *c.G = 0ull;
        *c.count = 0u;
    }
}

// R(u) in place on the inverse transforms: Re(W)/N per component; the
// interaction sum as beta (S - u_i) + alpha (u_{i-1} + u_{i+1}) for M >= 3
// and (beta + alpha) u_{1-i} for M = 2 (S4.1)
template <typename T, int MM>
__global__ void __launch_bounds__(256) k_rcd_reaction(RCtx c, typename C2<T>::t *w) {
    const int M = c.M;
    const int64_t N = c.g.N;
    const T invN = (T)c.invN, r = (T)c.r, a = (T)c.a, al = (T)c.alpha, be = (T)c.beta;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        T u[MM];
        T S = (T)0;
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            u[m] = m < M ? w[m * N + p].x * invN : (T)0;
            S = S + u[m];
        }
        T ulast = (T)0;
#pragma unroll
        for (int m = 0; m < MM; ++m)
            if (m == M - 1) ulast = u[m];
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            if (m >= M) continue;
            T inter;
            if (M == 2) {
                inter = (al + be) * (m == 0 ? u[1] : u[0]);
            } else {
                const T left = m == 0 ? ulast : u[m > 0 ? m - 1 : 0];
                const T right = m == M - 1 ? u[0] : u[m + 1 < MM ? m + 1 : 0];
                inter = be * (S - u[m]) + al * (left + right);
            }
            typename C2<T>::t o;
            o.x = u[m] * (r - a * u[m] - inter);
            o.y = (T)0;
            w[m * N + p] = o;
        }
    }
}

// XCD-aware: workgroup i runs on XCD i % 8, so the blocks are dealt out in
// eight contiguous ranges, one per XCD.  x-adjacent blocks of 8 FP32 values
// per row share 128-byte lines; on one XCD the second read hits its L2.
template <typename T>
__global__ void __launch_bounds__(256) k_rcd_measure(RCtx c) {
    __shared__ double red[4];
    using V2 = typename C2<T>::t;
    const V2 *q = reinterpret_cast<const V2 *>(c.state);
    const int64_t per = (c.g.nb + 7) >> 3;
    const int64_t b = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (b >= c.g.nb) return;  // workgroup-uniform, before any barrier
    const int64_t N = c.g.N;
    double amax = 0.0;
    for (int s = threadIdx.x; s < c.g.bvol; s += blockDim.x) {
        int64_t e;
        double k2;
        mode_of(c.g, b, s, e, k2);
        double acc = 0.0;
        for (int m = 0; m < c.M; ++m) {
            const V2 v = q[m * N + e];
            acc = acc + rsq2((double)v.x, (double)v.y);
        }
        if (e == 0) acc = 0.0;
        amax = fmax(amax, acc);
    }
    amax = rwave_max(amax);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = fmax(m, red[k]);
        c.ab[b] = m;
        c.mask[b] = 0;  // a fresh measure: nothing for the stage's G pass to merge
    }
}

// DIRECT: the coupled update of S4.2 as written, a per-mode solve of
// (I + dt k^2 D) x = b by Cholesky (the matrix is symmetric positive definite:
// D's eigenvalues are at least d_diag > 0), D in LDS in place of V^T, the
// factor in registers with the reciprocals of its diagonal
template <typename T, int MM, bool DIRECT>
__global__ void __launch_bounds__(256) k_rcd_update(RCtx c) {
    using V2 = typename C2<T>::t;
    __shared__ T vt[MM * MM];  // V^T, or D (DIRECT); zero-padded past M
    __shared__ T lam[MM];
    __shared__ double red[4];
    const T *msrc = reinterpret_cast<const T *>(DIRECT ? c.dm : c.vt);
    for (int i = threadIdx.x; i < MM * MM; i += blockDim.x) vt[i] = msrc[i];
    for (int i = threadIdx.x; i < MM; i += blockDim.x) lam[i] = reinterpret_cast<const T *>(c.lam)[i];
    __syncthreads();
    V2 *q = reinterpret_cast<V2 *>(c.state);
    const V2 *rh = reinterpret_cast<const V2 *>(c.rhs);
    const int M = c.M;
    const int64_t N = c.g.N;
    const T dt = (T)c.dt;
    const int64_t total = c.dense ? c.g.nb : (int64_t)*c.count;
    // one contiguous segment of the list per XCD (grid a multiple of 8): the
    // list is in block order within each wave's append, so x-adjacent blocks,
    // which share 128-byte lines, are updated on one XCD
    const int xcd = blockIdx.x & 7, per = gridDim.x >> 3;
    const int64_t seg = (total + 7) >> 3;
    const int64_t lo = std::min<int64_t>(total, seg * xcd), hi = std::min<int64_t>(total, seg * (xcd + 1));
    for (int64_t ent = lo + (blockIdx.x >> 3); ent < hi; ent += per) {
        const int64_t b = c.dense ? ent : (int64_t)c.list[ent];
        double amax = 0.0;
        for (int s = threadIdx.x; s < c.g.bvol; s += blockDim.x) {
            int64_t e;
            double k2;
            mode_of(c.g, b, s, e, k2);
            const T dk = (T)(c.dt * k2);
            T br[MM], bi[MM];
#pragma unroll
            for (int m = 0; m < MM; ++m) {
                br[m] = bi[m] = (T)0;
                if (m < M) {
                    const V2 v = q[m * N + e], f = rh[m * N + e];
                    br[m] = fma(dt, f.x, v.x);
                    bi[m] = fma(dt, f.y, v.y);
                }
            }
            T xr[MM], xi[MM];
#pragma unroll
            for (int m = 0; m < MM; ++m) xr[m] = xi[m] = (T)0;
            if constexpr (DIRECT) {
                T L[MM][MM];  // lower factor; L[j][j] holds 1 / l_jj
#pragma unroll
                for (int j = 0; j < MM; ++j) {
                    asm volatile("" ::: "memory");  // D read from LDS where used
                    T d = (T)1 + dk * vt[j * MM + j];
#pragma unroll
                    for (int k = 0; k < j; ++k) d = fma(-L[j][k], L[j][k], d);
                    const T inv = (T)1 / sqrt(d);
                    L[j][j] = inv;
#pragma unroll
                    for (int i = j + 1; i < MM; ++i) {
                        T t = dk * vt[i * MM + j];
#pragma unroll
                        for (int k = 0; k < j; ++k) t = fma(-L[i][k], L[j][k], t);
                        L[i][j] = t * inv;
                    }
                }
#pragma unroll
                for (int i = 0; i < MM; ++i) {  // L y = b
                    T yr = br[i], yi = bi[i];
#pragma unroll
                    for (int k = 0; k < i; ++k) {
                        yr = fma(-L[i][k], xr[k], yr);
                        yi = fma(-L[i][k], xi[k], yi);
                    }
                    xr[i] = yr * L[i][i];
                    xi[i] = yi * L[i][i];
                }
#pragma unroll
                for (int i = MM - 1; i >= 0; --i) {  // L^T x = y
                    T yr = xr[i], yi = xi[i];
#pragma unroll
                    for (int k = i + 1; k < MM; ++k) {
                        yr = fma(-L[k][i], xr[k], yr);
                        yi = fma(-L[k][i], xi[k], yi);
                    }
                    xr[i] = yr * L[i][i];
                    xi[i] = yi * L[i][i];
                }
            } else
#pragma unroll
            for (int j = 0; j < MM; ++j) {
                // keeps V^T in LDS: read where used (broadcasts), not hoisted
                // out of the mode loops into registers
                asm volatile("" ::: "memory");
                T wr = (T)0, wi = (T)0;
#pragma unroll
                for (int i = 0; i < MM; ++i) {
                    const T v = vt[j * MM + i];
                    wr = fma(v, br[i], wr);
                    wi = fma(v, bi[i], wi);
                }
                const T sj = (T)1 / ((T)1 + dk * lam[j]);
                wr = wr * sj;
                wi = wi * sj;
#pragma unroll
                for (int m = 0; m < MM; ++m) {
                    const T v = vt[j * MM + m];
                    xr[m] = fma(v, wr, xr[m]);
                    xi[m] = fma(v, wi, xi[m]);
                }
            }
#pragma unroll
            for (int m = 0; m < MM; ++m)
                if (m < M) {
                    V2 o;
                    o.x = xr[m];
                    o.y = xi[m];
                    q[m * N + e] = o;
                }
            if (c.keep) {  // the measure of what is stored, as k_rcd_measure sums it
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < MM; ++m)
                    if (m < M) acc = acc + rsq2((double)xr[m], (double)xi[m]);
                if (e == 0) acc = 0.0;
                amax = fmax(amax, acc);
            }
        }
        if (c.keep) {  // workgroup-uniform
            amax = rwave_max(amax);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
            __syncthreads();
            if (threadIdx.x == 0) {
                double mx = red[0];
                for (int k = 1; k < (int)(blockDim.x >> 6); ++k) mx = fmax(mx, red[k]);
                c.anext[b] = mx;
            }
            __syncthreads();  // red is free for the next entry
        }
    }
}

// one lane's value as a wave-uniform one (v_readlane; l a constant)
__device__ __forceinline__ float rlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rlane(double v, int l) {
    const long long x = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(x & 0xffffffffll), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The direct form for wide systems (M > 8): one wave per mode, lane i holding
// row i of A = I + dt k^2 D and component i of b = q + dt R.  Gaussian
// elimination without pivoting (A is symmetric positive definite: every pivot
// is positive) on [A | b]: at column j the pivot row's entries are taken from
// lane j as wave-uniform values and each lane below subtracts its multiple;
// back substitution then runs column by column, x_j formed from lane j's
// values and removed from the rows above.  A row's entries sit in registers
// at fixed indices, so every access names a constant register and a constant
// lane.  Lanes from M on hold identity rows (D zero-padded), which no other
// row reads; lanes from MM on hold zeros.  The kept measure sums the
// components of x in order.  (Broadcasting the pivot row through LDS instead
// measured slower: each column then waits on a store and a load.)
template <typename T, int MM>
__global__ void __launch_bounds__(256) k_rcd_update_direct(RCtx c) {
    using V2 = typename C2<T>::t;
    __shared__ T dl[MM * MM];  // D, zero-padded; symmetric, so lane i reads column i (consecutive words)
    __shared__ double red[4];
    for (int i = threadIdx.x; i < MM * MM; i += blockDim.x) dl[i] = reinterpret_cast<const T *>(c.dm)[i];
    __syncthreads();
    V2 *q = reinterpret_cast<V2 *>(c.state);
    const V2 *rh = reinterpret_cast<const V2 *>(c.rhs);
    const int M = c.M, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t N = c.g.N;
    const T dt = (T)c.dt;
    const int64_t total = c.dense ? c.g.nb : (int64_t)*c.count;
    const int xcd = blockIdx.x & 7, per = gridDim.x >> 3;
    const int64_t seg = (total + 7) >> 3;
    const int64_t lo = std::min<int64_t>(total, seg * xcd), hi = std::min<int64_t>(total, seg * (xcd + 1));
    for (int64_t ent = lo + (blockIdx.x >> 3); ent < hi; ent += per) {
        const int64_t b = c.dense ? ent : (int64_t)c.list[ent];
        double amax = 0.0;
        for (int s = wave; s < c.g.bvol; s += 4) {  // wave-uniform
            const int ln = lane;
            int64_t e;
            double k2;
            mode_of(c.g, b, s, e, k2);
            const T dk = (T)(c.dt * k2);
            T a[MM];
#pragma unroll
            for (int k = 0; k < MM; ++k) {
                asm volatile("" ::: "memory");  // D read from LDS where used
                a[k] = ln < MM ? dk * dl[k * MM + ln] : (T)0;
                if (k == ln) a[k] = a[k] + (T)1;
            }
            T br = (T)0, bi = (T)0;
            if (ln < M) {
                const V2 v = q[ln * N + e], f = rh[ln * N + e];
                br = fma(dt, f.x, v.x);
                bi = fma(dt, f.y, v.y);
            }
#pragma unroll
            for (int j = 0; j < MM; ++j) {  // eliminate column j below the pivot
                const T piv = rlane(a[j], j);  // every readlane in wave-uniform flow
                const T g = a[j] / piv;
                const T f = ln > j ? g : (T)0;
#pragma unroll
                for (int k = j + 1; k < MM; ++k) a[k] = fma(-f, rlane(a[k], j), a[k]);
                br = fma(-f, rlane(br, j), br);
                bi = fma(-f, rlane(bi, j), bi);
            }
            T xr = (T)0, xi = (T)0;
#pragma unroll
            for (int j = MM - 1; j >= 0; --j) {  // x_j, then its terms out of the rows above
                const T d = rlane(a[j], j);
                const T yr = rlane(br, j) / d, yi = rlane(bi, j) / d;
                if (ln == j) {
                    xr = yr;
                    xi = yi;
                }
                const T u = ln < j ? a[j] : (T)0;
                br = fma(-u, yr, br);
                bi = fma(-u, yi, bi);
            }
            if (ln < M) {
                V2 o;
                o.x = xr;
                o.y = xi;
                q[ln * N + e] = o;
            }
            if (c.keep) {  // the measure of what is stored, as k_rcd_measure sums it
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < MM; ++m)
                    if (m < M) acc = acc + rsq2((double)rlane(xr, m), (double)rlane(xi, m));
                if (e == 0) acc = 0.0;
                amax = fmax(amax, acc);
            }
        }
        if (c.keep) {  // workgroup-uniform; amax is uniform within each wave
            if (lane == 0) red[wave] = amax;
            __syncthreads();
            if (threadIdx.x == 0) c.anext[b] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            __syncthreads();  // red is free for the next entry
        }
    }
}

// Wide components (FP32, 16 < M <= 64): the eigen form as two small GEMMs on
// the matrix cores.  Per chunk of up to 64 modes of a block, B holds the
// modes' b = q + dt R as 128 real columns (re, im of each mode) over MM
// component rows; then
//   W = V^T B        (MM x MM times MM x 128, v_mfma_f32_16x16x4f32)
//   W_jc *= 1 / (1 + dt k^2 lambda_j)
//   X = V W
// and X goes back through LDS so that the stores are the loads' coalesced
// pattern and the kept measure sums the components in order.  Four waves
// share the 16 x 16 output tiles; LDS: V^T, V, B (reused for X), W.
// the 16 x 16 x 4 matrix-core product in the kernel's precision
template <typename T> struct RMf;
// Operands: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] in both
// precisions.  Result element r of lane l is D[drow(l / 16, r)][l % 16]: rows
// 4 (l / 16) + r in FP32, l / 16 + 4 r in FP64 (the FP64 row order checked on
// the device with one-hot operands).
template <> struct RMf<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int kq, int r) { return kq * 4 + r; }
};
template <> struct RMf<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int kq, int r) { return kq + 4 * r; }
};

template <typename T, int MM>
__global__ void __launch_bounds__(256) k_rcd_update_mfma(RCtx c) {
    using V2 = typename C2<T>::t;
    using v4 = typename RMf<T>::v4;
    constexpr int NC = 128;      // real columns per chunk: 64 modes
    constexpr int SA = MM + 4;   // row pitches padded so that the 64 lanes of an
    constexpr int SB = NC + 16;  // operand read fall on distinct LDS banks
    __shared__ T vtl[MM * SA];  // V^T (row j, column i)
    __shared__ T vl[MM * SA];   // V (row m, column j)
    __shared__ T bs[MM * SB];   // B, then X
    __shared__ T ws[MM * SB];   // W
    __shared__ T laml[MM];
    __shared__ T dks[NC / 2];
    __shared__ double red[4];
    const T *vsrc = reinterpret_cast<const T *>(c.vt);  // V^T, zero-padded
    for (int k = threadIdx.x; k < MM * MM; k += blockDim.x) {
        const int r = k / MM, q2 = k - r * MM;
        vtl[r * SA + q2] = vsrc[k];
        vl[q2 * SA + r] = vsrc[k];
    }
    for (int k = threadIdx.x; k < MM; k += blockDim.x) laml[k] = reinterpret_cast<const T *>(c.lam)[k];
    __syncthreads();
    V2 *q = reinterpret_cast<V2 *>(c.state);
    const V2 *rh = reinterpret_cast<const V2 *>(c.rhs);
    const int M = c.M, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t N = c.g.N;
    const T dt = (T)c.dt;
    const int64_t total = c.dense ? c.g.nb : (int64_t)*c.count;
    const int xcd = blockIdx.x & 7, per = gridDim.x >> 3;
    const int64_t seg = (total + 7) >> 3;
    const int64_t lo = std::min<int64_t>(total, seg * xcd), hi = std::min<int64_t>(total, seg * (xcd + 1));
    const int row = lane & 15, kq = lane >> 4;  // MFMA operand position of this lane
    // The chunks of the workgroup's blocks run as one sequence, and the
    // global loads of the next chunk are issued before the current chunk's
    // two products, so the memory traffic overlaps the matrix-core work.
    // Thread t holds mode t % 64 of the chunk (its offset and dt k^2 in
    // registers) for components t / 64 + 4 j.
    constexpr int PT = MM / 4;
    V2 pv[PT], pf[PT];
    int64_t pb = 0, pe = 0;
    int pnm = 0;
    T pdk = (T)0;
    auto fetch = [&](int64_t en, int s) {  // workgroup-uniform arguments
        pb = c.dense ? en : (int64_t)c.list[en];
        pnm = min(NC / 2, c.g.bvol - s);
        double k2 = 0.0;
        pe = 0;
        if (lane < pnm) mode_of(c.g, pb, s + lane, pe, k2);
        pdk = (T)(c.dt * k2);
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int i = wave + 4 * j;
            V2 v, f;
            v.x = v.y = f.x = f.y = (T)0;
            if (i < M && lane < pnm) {
                v = q[i * N + pe];
                f = rh[i * N + pe];
            }
            pv[j] = v;
            pf[j] = f;
        }
    };
    int64_t ent = lo + (blockIdx.x >> 3);
    int s0 = 0;
    if (ent < hi) fetch(ent, 0);
    double amax = 0.0;
    while (ent < hi) {  // workgroup-uniform
        const int64_t b = pb, e = pe;
        const int nm = pnm;
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int i = wave + 4 * j;
            T bx = (T)0, by = (T)0;
            if (i < M && lane < nm) {
                bx = fma(dt, pf[j].x, pv[j].x);
                by = fma(dt, pf[j].y, pv[j].y);
            }
            bs[i * SB + 2 * lane] = bx;
            bs[i * SB + 2 * lane + 1] = by;
        }
        if (wave == 0) dks[lane] = pdk;
        __syncthreads();
        // the next chunk: its loads fly while this one is multiplied
        int s1 = s0 + NC / 2;
        int64_t ent1 = ent;
        const bool last = s1 >= c.g.bvol;  // the block's last chunk
        if (last) {
            s1 = 0;
            ent1 += per;
        }
        if (ent1 < hi) fetch(ent1, s1);
        // W = V^T B, scaled; tiles (jt, ct) dealt to the four waves
        for (int tile = wave; tile < (MM / 16) * (NC / 16); tile += 4) {
            const int jt = tile / (NC / 16), ct = tile - jt * (NC / 16);
            v4 acc = {(T)0, (T)0, (T)0, (T)0};
            for (int k0 = 0; k0 < MM; k0 += 4) {
                const T av = vtl[(jt * 16 + row) * SA + k0 + kq];
                const T bv = bs[(k0 + kq) * SB + ct * 16 + row];
                acc = RMf<T>::mac(av, bv, acc);
            }
            const int col = ct * 16 + row;
            const T dk = dks[col >> 1];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = jt * 16 + RMf<T>::drow(kq, r);
                ws[j * SB + col] = acc[r] * ((T)1 / ((T)1 + dk * laml[j]));
            }
        }
        __syncthreads();
        // X = V W into bs
        for (int tile = wave; tile < (MM / 16) * (NC / 16); tile += 4) {
            const int mt = tile / (NC / 16), ct = tile - mt * (NC / 16);
            v4 acc = {(T)0, (T)0, (T)0, (T)0};
            for (int k0 = 0; k0 < MM; k0 += 4) {
                const T av = vl[(mt * 16 + row) * SA + k0 + kq];
                const T bv = ws[(k0 + kq) * SB + ct * 16 + row];
                acc = RMf<T>::mac(av, bv, acc);
            }
            const int col = ct * 16 + row;
#pragma unroll
            for (int r = 0; r < 4; ++r) bs[(mt * 16 + RMf<T>::drow(kq, r)) * SB + col] = acc[r];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int i = wave + 4 * j;
            if (i < M && lane < nm) {
                V2 o;
                o.x = bs[i * SB + 2 * lane];
                o.y = bs[i * SB + 2 * lane + 1];
                q[i * N + e] = o;
            }
        }
        if (c.keep && t < nm) {  // the measure of what is stored, components in order
            double acc = 0.0;
            for (int i = 0; i < M; ++i) acc = acc + rsq2((double)bs[i * SB + 2 * t], (double)bs[i * SB + 2 * t + 1]);
            if (e == 0) acc = 0.0;
            amax = fmax(amax, acc);
        }
        if (c.keep && last) {  // workgroup-uniform
            amax = rwave_max(amax);
            if (lane == 0) red[wave] = amax;
            __syncthreads();
            if (t == 0) c.anext[b] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            amax = 0.0;
        }
        __syncthreads();  // bs, dks and red are free for the next chunk
        ent = ent1;
        s0 = s1;
    }
}

template <typename T>
__global__ void k_rcd_real_in(int64_t n, const T *re, typename C2<T>::t *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        typename C2<T>::t o;
        o.x = re[i];
        o.y = (T)0;
        out[i] = o;
    }
}

template <typename T>
__global__ void k_rcd_real_out(int64_t n, const typename C2<T>::t *in, T *re, T invN) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        re[i] = in[i].x * invN;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) { int l = 0; while ((int64_t(1) << l) < v) ++l; return l; }

// FP64 cyclic Jacobi for the symmetric D: D = V diag(lam) V^T, V[i*M + j] = V_ij
void jacobi(int M, std::vector<double> A, std::vector<double> &V, std::vector<double> &lam) {
    V.assign((size_t)M * M, 0.0);
    for (int i = 0; i < M; ++i) V[(size_t)i * M + i] = 1.0;
    auto at = [&](int i, int j) -> double & { return A[(size_t)i * M + j]; };
    double diag = 0.0;
    for (int i = 0; i < M; ++i) diag += at(i, i) * at(i, i);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < M; ++p)
            for (int q = p + 1; q < M; ++q) off += at(p, q) * at(p, q);
        if (off <= 1e-32 * std::max(diag, 1e-300)) break;
        for (int p = 0; p < M; ++p)
            for (int q = p + 1; q < M; ++q) {
                if (at(p, q) == 0.0) continue;
                const double th = (at(q, q) - at(p, p)) / (2.0 * at(p, q));
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < M; ++k) {
                    const double kp = at(k, p), kq = at(k, q);
                    at(k, p) = cs * kp - sn * kq;
                    at(k, q) = sn * kp + cs * kq;
                }
                for (int k = 0; k < M; ++k) {
                    const double pk = at(p, k), qk = at(q, k);
                    at(p, k) = cs * pk - sn * qk;
                    at(q, k) = sn * pk + cs * qk;
                }
                for (int k = 0; k < M; ++k) {
                    const double vp = V[(size_t)k * M + p], vq = V[(size_t)k * M + q];
                    V[(size_t)k * M + p] = cs * vp - sn * vq;
                    V[(size_t)k * M + q] = sn * vp + cs * vq;
                }
            }
    }
    lam.resize(M);
    for (int i = 0; i < M; ++i) lam[i] = at(i, i);
}

std::vector<double> diffusion(int M, double dd, double dc) {
    std::vector<double> D((size_t)M * M, 0.0);
    for (int i = 0; i < M; ++i) {
        D[(size_t)i * M + i] = dd + 2.0 * dc;
        D[(size_t)i * M + (i + 1) % M] = -dc;
        D[(size_t)i * M + (i + M - 1) % M] = -dc;
    }
    return D;
}

// register tiles 2, 4, 8, 16; matrix-core tiles 32, 48, 64 (multiples of the 16-row MFMA tile)
int tile_of(int M) {
    if (M > 32) return M > 48 ? 64 : 48;
    int mm = 2;
    while (mm < M) mm <<= 1;
    return mm;
}

}  // namespace

struct spdba_rcd_s {
    spdba_rcd_desc d{};
    RCtx c{};
    bool dbl = false, timing = false, bound = false;
    int nd = 0, esize = 8;
    hipStream_t stream = nullptr;
    size_t state_bytes = 0, work_bytes = 0;
    size_t o_rhs = 0, o_fft = 0, o_ab = 0, o_anext = 0, o_mask = 0, o_list = 0, o_ctl = 0, o_vt = 0, o_lam = 0,
           o_dm = 0, o_stage = 0;
    spdba::BlockStage stage{};  // G, threshold and ordered compaction (the main plan's kernels)
    size_t fft_work = 0;
    rocfft_plan fwd = nullptr, inv = nullptr, inv_oop = nullptr;
    bool inv_keeps = false;  // the out-of-place inverse leaves its input intact (probed at bind)
    bool ab_valid = false;   // a_b and anext describe the current state (no load since the last update)
    rocfft_execution_info info = nullptr;
    std::vector<double> V, lam;
    char *d_state = nullptr, *d_work = nullptr;
    int cu = 256;
    hipEvent_t ev[5] = {};
    bool ev_valid = false;
};

namespace {

#define RTRY_HIP(x)                                   \
    do {                                              \
        if ((x) != hipSuccess) return SPDBA_EDEVICE;  \
    } while (0)
#define RTRY(x)                                       \
    do {                                              \
        spdba_status s_ = (x);                        \
        if (s_ != SPDBA_OK) return s_;                \
    } while (0)

spdba_status validate(const spdba_rcd_desc *d) {
    if (!d) return SPDBA_EINVAL;
    if (d->ndim < 1 || d->ndim > 3 || d->M < 2) return SPDBA_EINVAL;
    if (d->dtype != SPDBA_F32 && d->dtype != SPDBA_F64) return SPDBA_EINVAL;
    if (d->flags & ~(uint32_t)(SPDBA_RCD_DENSE | SPDBA_RCD_PIN_K0 | SPDBA_RCD_TIMING | SPDBA_RCD_DIRECT))
        return SPDBA_EINVAL;
    for (int a = 0; a < 3; ++a) {
        const bool used = a >= 3 - d->ndim;
        if (!used && (d->dims[a] != 1 || d->block[a] != 1)) return SPDBA_EINVAL;
        if (!pow2(d->dims[a]) || !pow2(d->block[a]) || d->block[a] > d->dims[a]) return SPDBA_EINVAL;
        if (d->dims[a] > (int64_t(1) << 24)) return SPDBA_EINVAL;
    }
    const double vals[] = {d->tau, d->dt, d->dx, d->d_diag, d->d_cross, d->alpha, d->beta, d->r, d->a};
    for (double v : vals)
        if (!std::isfinite(v)) return SPDBA_EINVAL;
    if (d->tau < 0 || d->dt <= 0 || d->dx <= 0 || d->d_diag <= 0 || d->d_cross < 0) return SPDBA_EINVAL;
    const int64_t N = d->dims[0] * d->dims[1] * d->dims[2];
    if (N > (int64_t(1) << 31) || (int64_t)d->M * N > (int64_t(1) << 36)) return SPDBA_EINVAL;
    if (d->M > (d->dtype == SPDBA_F64 ? kMaxMF64 : kMaxMF32)) return SPDBA_EUNSUPPORTED;
    return SPDBA_OK;
}

template <typename T, bool DIRECT>
void launch_update_d(const RCtx &c, int grid, hipStream_t s) {
    switch (c.mm) {
        case 2: hipLaunchKernelGGL((k_rcd_update<T, 2, DIRECT>), dim3(grid), dim3(256), 0, s, c); break;
        case 4: hipLaunchKernelGGL((k_rcd_update<T, 4, DIRECT>), dim3(grid), dim3(256), 0, s, c); break;
        case 8: hipLaunchKernelGGL((k_rcd_update<T, 8, DIRECT>), dim3(grid), dim3(256), 0, s, c); break;
        default:  // tile 16: FP32 eigen form only (validated at creation)
            if constexpr (sizeof(T) == 4 && !DIRECT)
                hipLaunchKernelGGL((k_rcd_update<T, 16, false>), dim3(grid), dim3(256), 0, s, c);
            break;
    }
}
// the eigen form: register tiles (FP32 2..16, FP64 2..8) on the vector units,
// wider tiles (FP64 16; 32, 48; FP32 64) as matrix-core GEMMs; the direct
// form: the factor in registers to tile 8, one wave per mode beyond
template <typename T>
void launch_update_t(const RCtx &c, int grid, hipStream_t s) {
    if (c.direct && c.mm <= kMaxMReg) {
        launch_update_d<T, true>(c, grid, s);
        return;
    }
    if (c.direct) {  // wide systems: one wave per mode
        switch (c.mm) {
            case 16: hipLaunchKernelGGL((k_rcd_update_direct<T, 16>), dim3(grid), dim3(256), 0, s, c); break;
            case 32: hipLaunchKernelGGL((k_rcd_update_direct<T, 32>), dim3(grid), dim3(256), 0, s, c); break;
            case 48: hipLaunchKernelGGL((k_rcd_update_direct<T, 48>), dim3(grid), dim3(256), 0, s, c); break;
            default:  // tile 64: FP32 only (validated at creation)
                if constexpr (sizeof(T) == 4)
                    hipLaunchKernelGGL((k_rcd_update_direct<T, 64>), dim3(grid), dim3(256), 0, s, c);
                break;
        }
        return;
    }
    const bool mfma = c.mm >= 32 || (sizeof(T) == 8 && c.mm == 16);
    if (!mfma) {
        launch_update_d<T, false>(c, grid, s);
        return;
    }
    switch (c.mm) {
        case 16: hipLaunchKernelGGL((k_rcd_update_mfma<T, 16>), dim3(grid), dim3(256), 0, s, c); break;
        case 32: hipLaunchKernelGGL((k_rcd_update_mfma<T, 32>), dim3(grid), dim3(256), 0, s, c); break;
        case 48: hipLaunchKernelGGL((k_rcd_update_mfma<T, 48>), dim3(grid), dim3(256), 0, s, c); break;
        default:  // tile 64: FP32 only (its FP64 LDS would exceed 160 KB; validated at creation)
            if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_rcd_update_mfma<T, 64>), dim3(grid), dim3(256), 0, s, c);
            break;
    }
}

template <typename T>
void launch_reaction_t(const RCtx &c, void *w, int grid, hipStream_t s) {
    auto *p = reinterpret_cast<typename C2<T>::t *>(w);
    switch (c.mm) {
        case 2: hipLaunchKernelGGL((k_rcd_reaction<T, 2>), dim3(grid), dim3(256), 0, s, c, p); break;
        case 4: hipLaunchKernelGGL((k_rcd_reaction<T, 4>), dim3(grid), dim3(256), 0, s, c, p); break;
        case 8: hipLaunchKernelGGL((k_rcd_reaction<T, 8>), dim3(grid), dim3(256), 0, s, c, p); break;
        case 16: hipLaunchKernelGGL((k_rcd_reaction<T, 16>), dim3(grid), dim3(256), 0, s, c, p); break;
        case 32: hipLaunchKernelGGL((k_rcd_reaction<T, 32>), dim3(grid), dim3(256), 0, s, c, p); break;
        case 48: hipLaunchKernelGGL((k_rcd_reaction<T, 48>), dim3(grid), dim3(256), 0, s, c, p); break;
        default:  // tile 64: FP32 only (validated at creation)
            if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_rcd_reaction<T, 64>), dim3(grid), dim3(256), 0, s, c, p);
            break;
    }
}

void rec(spdba_rcd_plan p, int i) {
    if (p->timing) (void)hipEventRecord(p->ev[i], p->stream);
}

spdba_status exec(spdba_rcd_plan p, rocfft_plan f, void *buf, void *out = nullptr) {
    void *ib[1] = {buf}, *ob[1] = {out};
    return rocfft_execute(f, ib, out ? ob : nullptr, p->info) == rocfft_status_success ? SPDBA_OK : SPDBA_EFFT;
}

// inverse transforms of the state into the work spectra, the state kept
spdba_status inverse_into(spdba_rcd_plan p, char *dst) {
    if (p->inv_keeps) return exec(p, p->inv_oop, p->d_state, dst);
    RTRY_HIP(hipMemcpyAsync(dst, p->d_state, p->state_bytes, hipMemcpyDeviceToDevice, p->stream));
    return exec(p, p->inv, dst);
}

// measure, threshold and compaction, update; rhs: device spectra of R
spdba_status update_stage(spdba_rcd_plan p, const void *rhs) {
    RCtx c = p->c;
    c.rhs = rhs;
    const int nbg = (int)(((c.g.nb + 7) >> 3) << 3);  // k_rcd_measure: eight XCD ranges
    if (!c.dense) {
        hipLaunchKernelGGL(k_rcd_reset, dim3(1), dim3(64), 0, p->stream, c);
        // the state entering this update is what the last one stored (frozen
        // blocks unchanged), so its measure is the kept one; after a load, a
        // full pass
        if (!p->ab_valid) {
            if (p->dbl) hipLaunchKernelGGL(k_rcd_measure<double>, dim3(nbg), dim3(256), 0, p->stream, c);
            else hipLaunchKernelGGL(k_rcd_measure<float>, dim3(nbg), dim3(256), 0, p->stream, c);
        }
        RTRY_HIP(hipGetLastError());
        rec(p, 2);
        RTRY_HIP(spdba::launch_block_stage(p->stage, p->stream));
        RTRY_HIP(hipGetLastError());
    } else {
        rec(p, 2);
    }
    rec(p, 3);
    // persistent: a few workgroups per compute unit, a multiple of 8 (one list
    // segment per XCD)
    const int grid = (int)(std::max<int64_t>(8, std::min<int64_t>(c.g.nb, (int64_t)p->cu * 8)) + 7) / 8 * 8;
    c.keep = c.dense ? 0 : 1;
    if (p->dbl) launch_update_t<double>(c, grid, p->stream);
    else launch_update_t<float>(c, grid, p->stream);
    RTRY_HIP(hipGetLastError());
    p->ab_valid = !c.dense;
    rec(p, 4);
    p->ev_valid = p->timing;
    return SPDBA_OK;
}

spdba_status one_step(spdba_rcd_plan p) {
    const RCtx &c = p->c;
    char *rhs = p->d_work + p->o_rhs;
    rec(p, 0);
    RTRY(inverse_into(p, rhs));
    const int grid = (int)std::min<int64_t>((c.g.N + 255) / 256, (int64_t)p->cu * 16);
    if (p->dbl) launch_reaction_t<double>(c, rhs, grid, p->stream);
    else launch_reaction_t<float>(c, rhs, grid, p->stream);
    RTRY_HIP(hipGetLastError());
    RTRY(exec(p, p->fwd, rhs));
    rec(p, 1);
    return update_stage(p, rhs);
}

}  // namespace

extern "C" {

spdba_status spdba_rcd_eigen(int32_t M, double d_diag, double d_cross, double *V, double *lam) {
    if (M < 2 || M > 1024 || !V || !lam || !std::isfinite(d_diag) || !std::isfinite(d_cross)) return SPDBA_EINVAL;
    std::vector<double> v, l;
    jacobi(M, diffusion(M, d_diag, d_cross), v, l);
    std::memcpy(V, v.data(), sizeof(double) * v.size());
    std::memcpy(lam, l.data(), sizeof(double) * l.size());
    return SPDBA_OK;
}

spdba_status spdba_rcd_create(const spdba_rcd_desc *desc, void *stream, spdba_rcd_plan *out) {
    if (!out) return SPDBA_EINVAL;
    *out = nullptr;
    RTRY(validate(desc));
    spdba_rcd_plan p = new (std::nothrow) spdba_rcd_s();
    if (!p) return SPDBA_EDEVICE;
    p->d = *desc;
    p->dbl = desc->dtype == SPDBA_F64;
    p->esize = p->dbl ? 16 : 8;
    p->timing = (desc->flags & SPDBA_RCD_TIMING) != 0;
    p->nd = desc->ndim;
    p->stream = reinterpret_cast<hipStream_t>(stream);
    RCtx &c = p->c;
    RGeo &g = c.g;
    g.N = 1;
    g.nb = 1;
    g.bvol = 1;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = (int)desc->dims[a];
        g.b[a] = desc->block[a];
        g.nbk[a] = g.n[a] / g.b[a];
        g.ln[a] = ilog2(g.n[a]);
        g.lb[a] = ilog2(g.b[a]);
        g.lnbk[a] = ilog2(g.nbk[a]);
        g.kf[a] = kTwoPiR / ((double)g.n[a] * desc->dx);
        g.N *= g.n[a];
        g.nb *= g.nbk[a];
        g.bvol *= g.b[a];
    }
    g.lbvol = ilog2(g.bvol);
    c.M = desc->M;
    c.mm = tile_of(desc->M);
    c.tau2 = desc->tau * desc->tau;
    c.dt = desc->dt;
    c.invN = 1.0 / (double)g.N;
    c.alpha = desc->alpha;
    c.beta = desc->beta;
    c.r = desc->r;
    c.a = desc->a;
    c.pin = (desc->flags & SPDBA_RCD_PIN_K0) ? 1 : 0;
    c.dense = (desc->flags & SPDBA_RCD_DENSE) ? 1 : 0;
    c.direct = (desc->flags & SPDBA_RCD_DIRECT) ? 1 : 0;
    jacobi(c.M, diffusion(c.M, desc->d_diag, desc->d_cross), p->V, p->lam);

    auto fail = [&](spdba_status s) {
        spdba_rcd_destroy(p);
        return s;
    };
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(SPDBA_EDEVICE);
    p->cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (spdba::fft_setup() != SPDBA_OK) return fail(SPDBA_EFFT);
    size_t len[3];
    for (int a = 0; a < p->nd; ++a) len[a] = (size_t)g.n[2 - a];  // fastest first
    const rocfft_precision prec = p->dbl ? rocfft_precision_double : rocfft_precision_single;
    if (rocfft_plan_create(&p->fwd, rocfft_placement_inplace, rocfft_transform_type_complex_forward, prec,
                           (size_t)p->nd, len, (size_t)c.M, nullptr) != rocfft_status_success ||
        rocfft_plan_create(&p->inv, rocfft_placement_inplace, rocfft_transform_type_complex_inverse, prec,
                           (size_t)p->nd, len, (size_t)c.M, nullptr) != rocfft_status_success ||
        rocfft_plan_create(&p->inv_oop, rocfft_placement_notinplace, rocfft_transform_type_complex_inverse, prec,
                           (size_t)p->nd, len, (size_t)c.M, nullptr) != rocfft_status_success)
        return fail(SPDBA_EFFT);
    size_t w1 = 0, w2 = 0, w3 = 0;
    if (rocfft_plan_get_work_buffer_size(p->fwd, &w1) != rocfft_status_success ||
        rocfft_plan_get_work_buffer_size(p->inv, &w2) != rocfft_status_success ||
        rocfft_plan_get_work_buffer_size(p->inv_oop, &w3) != rocfft_status_success)
        return fail(SPDBA_EFFT);
    p->fft_work = std::max(w1, std::max(w2, w3));
    if (rocfft_execution_info_create(&p->info) != rocfft_status_success ||
        rocfft_execution_info_set_stream(p->info, p->stream) != rocfft_status_success)
        return fail(SPDBA_EFFT);
    if (p->timing)
        for (auto &e : p->ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(SPDBA_EDEVICE);

    const size_t spec = (size_t)c.M * g.N * p->esize;
    const size_t tsz = p->dbl ? 8 : 4;
    p->state_bytes = spec;
    size_t o = 0;
    p->o_rhs = o;
    o = al256(o + spec);
    p->o_fft = o;
    o = al256(o + p->fft_work);
    p->o_ab = o;
    o = al256(o + sizeof(double) * g.nb);
    p->o_anext = o;
    o = al256(o + sizeof(double) * g.nb);
    p->o_mask = o;
    o = al256(o + g.nb);
    p->o_list = o;
    o = al256(o + sizeof(uint32_t) * g.nb);
    p->o_ctl = o;
    o = al256(o + 16);
    p->o_vt = o;
    o = al256(o + tsz * c.mm * c.mm);
    p->o_lam = o;
    o = al256(o + tsz * c.mm);
    p->o_dm = o;
    o = al256(o + tsz * c.mm * c.mm);
    p->o_stage = o;
    o = al256(o + spdba::block_stage_bytes(g.nb));
    p->work_bytes = o;
    *out = p;
    return SPDBA_OK;
}

spdba_status spdba_rcd_buffer_sizes(spdba_rcd_plan p, size_t *state_bytes, size_t *work_bytes) {
    if (!p || !state_bytes || !work_bytes) return SPDBA_EINVAL;
    *state_bytes = p->state_bytes;
    *work_bytes = p->work_bytes;
    return SPDBA_OK;
}

spdba_status spdba_rcd_bind(spdba_rcd_plan p, void *d_state, void *d_work) {
    if (!p || !d_state || !d_work) return SPDBA_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_state) & 255) || (reinterpret_cast<uintptr_t>(d_work) & 255))
        return SPDBA_EINVAL;
    p->d_state = static_cast<char *>(d_state);
    p->d_work = static_cast<char *>(d_work);
    RCtx &c = p->c;
    c.state = p->d_state;
    c.ab = reinterpret_cast<double *>(p->d_work + p->o_ab);
    c.anext = reinterpret_cast<double *>(p->d_work + p->o_anext);
    c.mask = reinterpret_cast<uint8_t *>(p->d_work + p->o_mask);
    c.list = reinterpret_cast<uint32_t *>(p->d_work + p->o_list);
    c.G = reinterpret_cast<unsigned long long *>(p->d_work + p->o_ctl);
    c.count = reinterpret_cast<uint32_t *>(p->d_work + p->o_ctl + 8);
    c.vt = p->d_work + p->o_vt;
    c.lam = p->d_work + p->o_lam;
    c.dm = p->d_work + p->o_dm;
    if (p->fft_work &&
        rocfft_execution_info_set_work_buffer(p->info, p->d_work + p->o_fft, p->fft_work) != rocfft_status_success)
        return SPDBA_EFFT;
    // V^T and lambda, zero-padded to the register tile, in the kernels' precision
    const int M = c.M, mm = c.mm;
    std::vector<double> vt((size_t)mm * mm, 0.0), lam(mm, 0.0), dm((size_t)mm * mm, 0.0);
    const std::vector<double> D = diffusion(M, p->d.d_diag, p->d.d_cross);
    for (int j = 0; j < M; ++j) {
        lam[j] = p->lam[j];
        for (int i = 0; i < M; ++i) {
            vt[(size_t)j * mm + i] = p->V[(size_t)i * M + j];
            dm[(size_t)j * mm + i] = D[(size_t)j * M + i];
        }
    }
    if (p->dbl) {
        RTRY_HIP(hipMemcpy(p->d_work + p->o_vt, vt.data(), 8 * vt.size(), hipMemcpyHostToDevice));
        RTRY_HIP(hipMemcpy(p->d_work + p->o_lam, lam.data(), 8 * lam.size(), hipMemcpyHostToDevice));
        RTRY_HIP(hipMemcpy(p->d_work + p->o_dm, dm.data(), 8 * dm.size(), hipMemcpyHostToDevice));
    } else {
        std::vector<float> vf(vt.begin(), vt.end()), lf(lam.begin(), lam.end()), df(dm.begin(), dm.end());
        RTRY_HIP(hipMemcpy(p->d_work + p->o_vt, vf.data(), 4 * vf.size(), hipMemcpyHostToDevice));
        RTRY_HIP(hipMemcpy(p->d_work + p->o_lam, lf.data(), 4 * lf.size(), hipMemcpyHostToDevice));
        RTRY_HIP(hipMemcpy(p->d_work + p->o_dm, df.data(), 4 * df.size(), hipMemcpyHostToDevice));
    }
    // the tables read back before any update: zero a_b, mask, G and the count
    RTRY_HIP(hipMemsetAsync(p->d_work + p->o_ab, 0, p->o_vt - p->o_ab, p->stream));
    p->stage.nb = c.g.nb;
    p->stage.a_b = c.ab;
    p->stage.a_next = c.anext;
    p->stage.mask = c.mask;
    p->stage.list = c.list;
    p->stage.count = c.count;
    p->stage.G = c.G;
    p->stage.aux = p->d_work + p->o_stage;
    RTRY_HIP(spdba::block_stage_init(p->stage, c.tau2, c.pin, p->stream));
    // does the out-of-place inverse keep its input?  A pattern in the state,
    // one transform, a check (the state's contents are undefined until loaded)
    uint32_t *bad = reinterpret_cast<uint32_t *>(p->d_work + p->o_ctl + 12);
    const int64_t ne = (int64_t)M * c.g.N;
    RTRY_HIP(spdba::launch_fill_pattern(p->d_state, ne, p->dbl, p->stream));
    RTRY(exec(p, p->inv_oop, p->d_state, p->d_work + p->o_rhs));
    RTRY_HIP(spdba::launch_check_pattern(p->d_state, ne, p->dbl, bad, p->stream));
    uint32_t h = 1;
    RTRY_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, p->stream));
    RTRY_HIP(hipStreamSynchronize(p->stream));
    p->inv_keeps = (h == 0);
    p->bound = true;
    return SPDBA_OK;
}

spdba_status spdba_rcd_set_spectrum(spdba_rcd_plan p, const void *src) {
    if (!p || !src) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    p->ab_valid = false;
    RTRY_HIP(hipMemcpyAsync(p->d_state, src, p->state_bytes, hipMemcpyDeviceToDevice, p->stream));
    return SPDBA_OK;
}

spdba_status spdba_rcd_get_spectrum(spdba_rcd_plan p, void *dst) {
    if (!p || !dst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    RTRY_HIP(hipMemcpyAsync(dst, p->d_state, p->state_bytes, hipMemcpyDeviceToDevice, p->stream));
    return SPDBA_OK;
}

spdba_status spdba_rcd_set_field(spdba_rcd_plan p, const void *re) {
    if (!p || !re) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    p->ab_valid = false;
    const int64_t n = (int64_t)p->c.M * p->c.g.N;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, (int64_t)p->cu * 16);
    if (p->dbl)
        hipLaunchKernelGGL(k_rcd_real_in<double>, dim3(grid), dim3(256), 0, p->stream, n,
                           static_cast<const double *>(re), reinterpret_cast<double2 *>(p->d_state));
    else
        hipLaunchKernelGGL(k_rcd_real_in<float>, dim3(grid), dim3(256), 0, p->stream, n,
                           static_cast<const float *>(re), reinterpret_cast<float2 *>(p->d_state));
    RTRY_HIP(hipGetLastError());
    return exec(p, p->fwd, p->d_state);
}

spdba_status spdba_rcd_get_field(spdba_rcd_plan p, void *re) {
    if (!p || !re) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    char *w = p->d_work + p->o_rhs;
    RTRY(inverse_into(p, w));
    const int64_t n = (int64_t)p->c.M * p->c.g.N;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, (int64_t)p->cu * 16);
    if (p->dbl)
        hipLaunchKernelGGL(k_rcd_real_out<double>, dim3(grid), dim3(256), 0, p->stream, n,
                           reinterpret_cast<const double2 *>(w), static_cast<double *>(re), p->c.invN);
    else
        hipLaunchKernelGGL(k_rcd_real_out<float>, dim3(grid), dim3(256), 0, p->stream, n,
                           reinterpret_cast<const float2 *>(w), static_cast<float *>(re), (float)p->c.invN);
    RTRY_HIP(hipGetLastError());
    return SPDBA_OK;
}

spdba_status spdba_rcd_apply(spdba_rcd_plan p, const void *rhs) {
    if (!p || !rhs) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    rec(p, 0);
    rec(p, 1);
    return update_stage(p, rhs);
}

spdba_status spdba_rcd_step(spdba_rcd_plan p, int32_t n) {
    if (!p || n < 0) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    for (int32_t i = 0; i < n; ++i) RTRY(one_step(p));
    return SPDBA_OK;
}

spdba_status spdba_rcd_indicator(spdba_rcd_plan p, double *ab, size_t n, double *G) {
    if (!p || (ab && n < (size_t)p->c.g.nb)) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    RTRY_HIP(hipStreamSynchronize(p->stream));
    if (ab) RTRY_HIP(hipMemcpy(ab, p->c.ab, sizeof(double) * p->c.g.nb, hipMemcpyDeviceToHost));
    if (G) {
        unsigned long long bits = 0;
        RTRY_HIP(hipMemcpy(&bits, p->c.G, 8, hipMemcpyDeviceToHost));
        std::memcpy(G, &bits, 8);
    }
    return SPDBA_OK;
}

spdba_status spdba_rcd_active_mask(spdba_rcd_plan p, uint8_t *mask, size_t n, int64_t *count) {
    if (!p || (mask && n < (size_t)p->c.g.nb)) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    RTRY_HIP(hipStreamSynchronize(p->stream));
    if (p->c.dense) {
        if (mask) std::memset(mask, 1, p->c.g.nb);
        if (count) *count = p->c.g.nb;
        return SPDBA_OK;
    }
    if (mask) RTRY_HIP(hipMemcpy(mask, p->c.mask, p->c.g.nb, hipMemcpyDeviceToHost));
    if (count) {
        uint32_t c = 0;
        RTRY_HIP(hipMemcpy(&c, p->c.count, 4, hipMemcpyDeviceToHost));
        *count = c;
    }
    return SPDBA_OK;
}

spdba_status spdba_rcd_stats(spdba_rcd_plan p, spdba_rcd_stats_t *out) {
    if (!p || !out) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    std::memset(out, 0, sizeof(*out));
    out->n_blocks = p->c.g.nb;
    RTRY(spdba_rcd_active_mask(p, nullptr, 0, &out->active_blocks));
    if (!p->c.dense) RTRY(spdba_rcd_indicator(p, nullptr, 0, &out->G));
    if (p->timing && p->ev_valid)
        for (int i = 0; i < 4; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p->ev[i], p->ev[i + 1]) == hipSuccess) out->stage_ms[i] = ms;
        }
    return SPDBA_OK;
}

spdba_status spdba_rcd_destroy(spdba_rcd_plan p) {
    if (!p) return SPDBA_OK;
    if (p->fwd) rocfft_plan_destroy(p->fwd);
    if (p->inv) rocfft_plan_destroy(p->inv);
    if (p->inv_oop) rocfft_plan_destroy(p->inv_oop);
    if (p->info) rocfft_execution_info_destroy(p->info);
    for (auto &e : p->ev)
        if (e) (void)hipEventDestroy(e);
    delete p;
    return SPDBA_OK;
}

}  // extern "C"
