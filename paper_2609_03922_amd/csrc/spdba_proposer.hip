// spdba_proposer.hip -- learned activation proposer kernels for gfx950:
// block features, the fused MLP forward pass (8 -> 64 -> 64 -> 1) on bf16
// MFMA, its backward pass (split-K bf16 MFMA GEMMs with fixed-order
// reductions), weighted BCE, Adam, labels and skip sets.
//
// MFMA v_mfma_f32_16x16x32_bf16, wave64 operand layout (lane l, g = l >> 4,
// c = l & 15): A[16 x 32] lane holds row c, k = 8g..8g+7; B[32 x 16] lane holds
// column c, k = 8g..8g+7; D[16 x 16] lane holds column c, rows 4g..4g+3.
//
// Built with -ffp-contract=off; rounding to bf16 is round-to-nearest-even.

#include "spdba_internal.h"
#include "spdba_proposer.h"

#include <float.h>

namespace spdba {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int OW1 = 0, OB1 = 512, OW2 = 576, OB2 = 4672, OW3 = 4736, OB3 = 4800;
constexpr int NPARAM = SPDBA_MLP_NPARAM;

__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }
__device__ __forceinline__ float rbf(float f) { return bf2f(f2bf(f)); }
__device__ __forceinline__ int sidx_f(int i, int n) { return (2 * i < n) ? i : i - n; }

__device__ __forceinline__ f32x4 mfma(u16x8 a, u16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// fused forward pass: one wave per 16-sample tile, weights held in registers
// as B fragments, the hidden activations re-laid out through LDS
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_mlp_forward(const float *x, int64_t n, const uint16_t *w,
                                                     float *prob, float *logit, float *h1o,
                                                     float *h2o) {
    __shared__ unsigned short T[4][16][72];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    u16x8 B1[4], B2[2][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * grp + j;
            B1[nt][j] = k < 8 ? w[OW1 + k * 64 + nt * 16 + col] : (unsigned short)0;
            B2[0][nt][j] = w[OW2 + k * 64 + nt * 16 + col];
            B2[1][nt][j] = w[OW2 + (32 + k) * 64 + nt * 16 + col];
        }
    float bias1[4], bias2[4], w3[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        bias1[nt] = bf2f(w[OB1 + nt * 16 + col]);
        bias2[nt] = bf2f(w[OB2 + nt * 16 + col]);
        w3[nt] = bf2f(w[OW3 + nt * 16 + col]);
    }
    const float b3 = bf2f(w[OB3]);
    const int64_t ntiles = (n + 15) / 16;
    // the loop bound is uniform over the workgroup (barriers inside)
    for (int64_t base = (int64_t)blockIdx.x * 4; base < ntiles; base += (int64_t)gridDim.x * 4) {
        const int64_t tile = base + wv;
        const int64_t r0 = tile * 16;
        u16x8 a1;
#pragma unroll
        for (int j = 0; j < 8; ++j) a1[j] = 0;
        if (grp == 0 && tile < ntiles && r0 + col < n) {
            const float4 lo = *reinterpret_cast<const float4 *>(x + (r0 + col) * 8);
            const float4 hi = *reinterpret_cast<const float4 *>(x + (r0 + col) * 8 + 4);
            a1[0] = f2bf(lo.x); a1[1] = f2bf(lo.y); a1[2] = f2bf(lo.z); a1[3] = f2bf(lo.w);
            a1[4] = f2bf(hi.x); a1[5] = f2bf(hi.y); a1[6] = f2bf(hi.z); a1[7] = f2bf(hi.w);
        }
        f32x4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 z = {0.f, 0.f, 0.f, 0.f};
            acc[nt] = mfma(a1, B1[nt], z);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 4 * grp + j;
                const float h = fmaxf(acc[nt][j] + bias1[nt], 0.f);
                if (h1o && tile < ntiles && r0 + row < n) h1o[(r0 + row) * 64 + nt * 16 + col] = h;
                T[wv][row][nt * 16 + col] = f2bf(h);
            }
        __syncthreads();
        u16x8 a2[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int j = 0; j < 8; ++j) a2[ks][j] = T[wv][col][32 * ks + 8 * grp + j];
        __syncthreads();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 z = {0.f, 0.f, 0.f, 0.f};
            acc[nt] = mfma(a2[0], B2[0][nt], z);
            acc[nt] = mfma(a2[1], B2[1][nt], acc[nt]);
        }
        float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 4 * grp + j;
                const float h = fmaxf(acc[nt][j] + bias2[nt], 0.f);
                if (h2o && tile < ntiles && r0 + row < n) h2o[(r0 + row) * 64 + nt * 16 + col] = h;
                s[j] = __builtin_fmaf(rbf(h), w3[nt], s[j]);
            }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) s[j] += __shfl_xor(s[j], off, 64);
        if (col == 0 && tile < ntiles)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t r = r0 + 4 * grp + j;
                if (r < n) {
                    const float z = s[j] + b3;
                    if (logit) logit[r] = z;
                    if (prob) prob[r] = 1.f / (1.f + expf(-z));
                }
            }
    }
}

// ---------------------------------------------------------------------------
// split-K bf16 GEMM for the backward pass:
//   P[split][m][n] = sum_{k in split} A(m, k) B(k, n),  A(m,k) = A[m*sam + k*sak],
//   B(k,n) = B[k*sbk + n*sbn]; FP32 operands rounded to bf16, FP32 accumulate.
// One wave per (16 x 16 tile, split).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(64) k_gemm_bf16(const float *A, int64_t sam, int64_t sak,
                                                  const float *B, int64_t sbk, int64_t sbn,
                                                  float *P, int M, int N, int64_t K, int splits,
                                                  int64_t kchunk) {
    const int lane = threadIdx.x;
    const int col = lane & 15, grp = lane >> 4;
    const int tn = (N + 15) / 16;
    const int64_t t = blockIdx.x / splits;
    const int sp = (int)(blockIdx.x % splits);
    const int m0 = (int)(t / tn) * 16, n0 = (int)(t % tn) * 16;
    const int64_t k_lo = (int64_t)sp * kchunk, k_hi = k_lo + kchunk < K ? k_lo + kchunk : K;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int am = m0 + col, bn = n0 + col;
    for (int64_t k0 = k_lo; k0 < k_hi; k0 += 32) {
        u16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t k = k0 + 8 * grp + j;
            const bool kin = k < k_hi;
            a[j] = (kin && am < M) ? f2bf(A[am * sam + k * sak]) : (unsigned short)0;
            b[j] = (kin && bn < N) ? f2bf(B[k * sbk + bn * sbn]) : (unsigned short)0;
        }
        acc = mfma(a, b, acc);
    }
    float *out = P + (int64_t)sp * M * N;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = m0 + 4 * grp + j, nn = n0 + col;
        if (m < M && nn < N) out[(int64_t)m * N + nn] = acc[j];
    }
}

// C[i] = sum over splits (in order) of P[s][i]; optional ReLU gate: C *= (gate[i] > 0)
__global__ void k_sum_splits(const float *P, int64_t mn, int splits, float *C, const float *gate) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < mn;
         i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int sp = 0; sp < splits; ++sp) s += P[(int64_t)sp * mn + i];
        if (gate) s = gate[i] > 0.f ? s : 0.f;
        C[i] = s;
    }
}

// dh2[r][c] = dlogit[r] * bf16(W3[c]) * (h2[r][c] > 0)
__global__ void k_dh2(const float *dlogit, const float *h2, const float *wm, float *dh2, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * 64;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i >> 6;
        const int c = (int)(i & 63);
        dh2[i] = h2[i] > 0.f ? dlogit[r] * rbf(wm[OW3 + c]) : 0.f;
    }
}

// column sums of X[n][ncol] in a fixed order: per-chunk partials, then in order
__global__ void __launch_bounds__(256) k_colsum_part(const float *X, int64_t n, int ncol,
                                                     int64_t rows_per, float *part) {
    const int c = threadIdx.x % ncol;
    const int lanes = blockDim.x / ncol;  // row lanes per column
    const int rl = threadIdx.x / ncol;
    __shared__ float red[256];
    const int64_t r_lo = (int64_t)blockIdx.x * rows_per;
    float s = 0.f;
    if (rl < lanes)
        for (int64_t r = r_lo + rl; r < r_lo + rows_per && r < n; r += lanes) s += X[r * ncol + c];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < ncol) {
        float t = 0.f;
        for (int l = 0; l < lanes; ++l) t += red[l * ncol + threadIdx.x];
        part[(int64_t)blockIdx.x * ncol + threadIdx.x] = t;
    }
}
__global__ void k_colsum_final(const float *part, int64_t nparts, int ncol, float *out) {
    const int c = threadIdx.x;
    if (c >= ncol) return;
    float t = 0.f;
    for (int64_t p = 0; p < nparts; ++p) t += part[p * ncol + c];
    out[c] = t;
}

// ---------------------------------------------------------------------------
// loss, optimiser, labels, skip sets
// ---------------------------------------------------------------------------

__device__ __forceinline__ float softplus(float z) { return z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z)); }

__global__ void __launch_bounds__(256) k_bce(const float *logit, const float *y, int64_t n, float pw,
                                             float *dlogit, double *part) {
    __shared__ double red[256];
    double acc = 0.0;
    const float inv_n = 1.f / (float)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float z = logit[i], t = y[i];
        const float p = 1.f / (1.f + expf(-z));
        dlogit[i] = (pw * t * (p - 1.f) + (1.f - t) * p) * inv_n;
        acc += (double)(pw * t * softplus(-z) + (1.f - t) * softplus(z));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) s += red[i];
        part[blockIdx.x] = s;
    }
}
__global__ void k_bce_final(const double *part, int nparts, int64_t n, double *loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[i];
    loss[0] = s / (double)n;
}

__global__ void k_adam(float *w, float *m, float *v, const float *g, uint16_t *wb, int64_t np, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        wb[i] = f2bf(wi);
    }
}

__global__ void k_to_bf16(const float *w, uint16_t *wb, int64_t np) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x)
        wb[i] = f2bf(w[i]);
}

__global__ void k_labels(const uint8_t *masks, int nm, int64_t nb, float *y) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        uint8_t any = 0;
        for (int j = 0; j < nm; ++j) any |= masks[(int64_t)j * nb + b];
        y[b] = any ? 1.f : 0.f;
    }
}

__global__ void k_miss(const uint8_t *skip, const uint8_t *mask, int64_t nb, uint32_t *count) {
    uint32_t n = 0;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x)
        n += (skip[b] && mask[b]) ? 1u : 0u;
    for (int off = 32; off >= 1; off >>= 1) n += __shfl_xor(n, off, 64);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(count, n);
}

// skip[b] = prob[b] < thr, or all zero when the gate (a miss count) is set;
// optionally adds the number of skipped blocks to *count
__global__ void k_skip(const float *prob, int64_t nb, float thr, const uint32_t *gate, uint8_t *skip,
                       uint32_t *count) {
    const bool off = gate != nullptr && *gate != 0u;
    uint32_t n = 0;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        const bool s = !off && prob[b] < thr;
        skip[b] = s ? 1 : 0;
        n += s ? 1u : 0u;
    }
    if (count) {
        for (int off2 = 32; off2 >= 1; off2 >>= 1) n += __shfl_xor(n, off2, 64);
        if ((threadIdx.x & 63) == 0 && n) atomicAdd(count, n);
    }
}

// ---------------------------------------------------------------------------
// block features
// ---------------------------------------------------------------------------

constexpr int EB_SPLIT = 64;  // fixed partition of each instance's blocks

// per-instance E_tot in two fixed-order levels: partial over one of EB_SPLIT
// contiguous ranges of the instance's blocks, then the sum of the partials
__global__ void __launch_bounds__(256) k_eb_part(const InstDev *ins, const double *eb, double *part) {
    __shared__ double red[256];
    const int ii = blockIdx.x / EB_SPLIT, sp = blockIdx.x % EB_SPLIT;
    const InstDev &I = ins[ii];
    const int64_t per = (I.nb + EB_SPLIT - 1) / EB_SPLIT;
    const int64_t lo = sp * per, hi = lo + per < I.nb ? lo + per : I.nb;
    double s = 0.0;
    for (int64_t b = lo + threadIdx.x; b < hi; b += blockDim.x) s += eb[I.blk_off + b];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += red[i];
        part[blockIdx.x] = t;
    }
}
__global__ void k_eb_total(const double *part, int n_inst, double *tot) {
    const int ii = blockIdx.x * blockDim.x + threadIdx.x;
    if (ii >= n_inst) return;
    double t = 0.0;
    for (int sp = 0; sp < EB_SPLIT; ++sp) t += part[ii * EB_SPLIT + sp];
    tot[ii] = t;
}

struct FeatArgs {
    const double *ab0, *ab1, *ab2;
    const double *G0, *G1, *G2;
};

__device__ __forceinline__ float log_feature(double a, double G) {
    if (!(G > 0.0) || !(a > 0.0)) return 0.f;  // log10 clamped at -40 -> scaled 0
    double l = log10(a / G);
    l = l < -40.0 ? -40.0 : (l > 0.0 ? 0.0 : l);
    return (float)(1.0 + l / 40.0);
}

__global__ void k_features(Ctx c, FeatArgs fa, const uint8_t *mask, const double *eb,
                           const double *etot, float frac, float *x) {
    for (int64_t gb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gb < c.nb_total;
         gb += (int64_t)gridDim.x * blockDim.x) {
        const int ii = c.blk_inst[gb];
        const InstDev &I = c.inst[ii];
        const int64_t lb = gb - I.blk_off;
        const int bx = (int)(lb & (I.nbk[2] - 1));
        const int64_t t = lb >> I.lnbk[2];
        const int by = (int)(t & (I.nbk[1] - 1));
        const int bz = (int)(t >> I.lnbk[1]);
        float f[8];
        f[0] = log_feature(fa.ab0[gb], fa.G0[ii]);
        f[1] = log_feature(fa.ab1[gb], fa.G1[ii]);
        f[2] = log_feature(fa.ab2[gb], fa.G2[ii]);
        // mean |k| over the block, relative to |k| at the Nyquist index
        double ks = 0.0;
        for (int iz = 0; iz < I.b[0]; ++iz) {
            const int mz = sidx_f(bz * I.b[0] + iz, I.n[0]);
            for (int iy = 0; iy < I.b[1]; ++iy) {
                const int my = sidx_f(by * I.b[1] + iy, I.n[1]);
                for (int ix = 0; ix < I.b[2]; ++ix) {
                    const int mx = sidx_f(bx * I.b[2] + ix, I.n[2]);
                    ks += sqrt((double)mz * mz + (double)my * my + (double)mx * mx);
                }
            }
        }
        const double nmodes = (double)I.b[0] * I.b[1] * I.b[2];
        f[3] = (float)(ks / nmodes / (0.5 * (double)I.n[2]));
        // active face neighbours on the periodic block grid
        int act = 0;
        const int nb3[3] = {I.nbk[0], I.nbk[1], I.nbk[2]};
        const int bc[3] = {bz, by, bx};
        for (int a = 0; a < 3; ++a) {
            if (nb3[a] < 2) continue;
            for (int d = -1; d <= 1; d += 2) {
                int q[3] = {bc[0], bc[1], bc[2]};
                q[a] = (q[a] + d + nb3[a]) % nb3[a];
                const int64_t nl = (((int64_t)q[0] * nb3[1]) + q[1]) * nb3[2] + q[2];
                act += mask[I.blk_off + nl] ? 1 : 0;
            }
        }
        f[4] = (float)act / 6.f;
        f[5] = frac;
        double e = etot[ii] > 0.0 ? eb[gb] * (double)I.nb / etot[ii] : 0.0;
        double le = e > 0.0 ? log10(e) : -40.0;
        le = le < -40.0 ? -40.0 : (le > 40.0 ? 40.0 : le);
        f[6] = (float)(le / 40.0);
        f[7] = mask[gb] ? 1.f : 0.f;
        float4 *o = reinterpret_cast<float4 *>(x + gb * 8);
        o[0] = make_float4(f[0], f[1], f[2], f[3]);
        o[1] = make_float4(f[4], f[5], f[6], f[7]);
    }
}

static unsigned grid_n(int64_t n, int per = 256) {
    int64_t g = (n + per - 1) / per;
    return (unsigned)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

}  // namespace spdba

using namespace spdba;

namespace {
spdba_status st(hipError_t e) { return e == hipSuccess ? SPDBA_OK : SPDBA_EDEVICE; }
int64_t bwd_splits(int64_t n) {
    int64_t s = (n + 511) / 512;
    return s < 1 ? 1 : (s > 64 ? 64 : s);
}
}  // namespace

extern "C" {

spdba_status spdba_mlp_forward(const float *x, int64_t n, const uint16_t *w_bf16, float *prob,
                               float *logit, float *h1, float *h2, void *stream) {
    if (!x || !w_bf16 || n < 0) return SPDBA_EINVAL;
    if (n == 0) return SPDBA_OK;
    const int64_t tiles = (n + 15) / 16;
    int64_t g = (tiles + 3) / 4;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream, x, n,
                       w_bf16, prob, logit, h1, h2);
    return st(hipGetLastError());
}

size_t spdba_mlp_backward_scratch(int64_t n) {
    const int64_t S = bwd_splits(n);
    const int64_t nparts = (n + 1023) / 1024 + 1;
    size_t b = 0;
    b += (size_t)n * 64 * 4 * 2;           // dh2, dh1
    b += (size_t)S * 64 * 64 * 4;          // split-K partials
    b += (size_t)nparts * 64 * 4 + 256;    // column-sum partials
    b += (size_t)grid_n(n) * 8 + 256;      // loss partials
    return b + 4096;
}

spdba_status spdba_mlp_backward(const float *x, const float *h1, const float *h2,
                                const float *dlogit, int64_t n, const float *w, float *grad,
                                void *scratch, void *stream) {
    if (!x || !h1 || !h2 || !dlogit || !w || !grad || !scratch || n <= 0) return SPDBA_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t S = bwd_splits(n);
    int64_t kchunk = (n + S - 1) / S;
    kchunk = (kchunk + 31) / 32 * 32;
    char *p = static_cast<char *>(scratch);
    float *dh2 = reinterpret_cast<float *>(p);
    float *dh1 = dh2 + n * 64;
    float *P = dh1 + n * 64;
    float *cpart = P + S * 64 * 64;
    const int64_t rows_per = 1024, nparts = (n + rows_per - 1) / rows_per;
    auto gemm = [&](const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk,
                    int64_t sbn, float *out, int M, int N, int64_t K, int splits, int64_t kc) {
        const int64_t tiles = (int64_t)((M + 15) / 16) * ((N + 15) / 16);
        hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)(tiles * splits)), dim3(64), 0, s, A, sam, sak,
                           B, sbk, sbn, out, M, N, K, splits, kc);
        return hipGetLastError();
    };
    auto sum_splits = [&](const float *Pp, int64_t mn, int splits, float *C, const float *gate) {
        hipLaunchKernelGGL(k_sum_splits, dim3(grid_n(mn)), dim3(256), 0, s, Pp, mn, splits, C, gate);
        return hipGetLastError();
    };
    auto colsum = [&](const float *X, int ncol, float *out) {
        hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)nparts), dim3(256), 0, s, X, n, ncol,
                           rows_per, cpart);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(64), 0, s, cpart, nparts, ncol, out);
        return hipGetLastError();
    };
#define CK(e)                                          \
    do {                                               \
        if ((e) != hipSuccess) return SPDBA_EDEVICE;   \
    } while (0)
    // layer 3: dW3 = bf16(h2)^T bf16(dlogit), db3 = sum dlogit
    CK(gemm(dlogit, 0, 1, h2, 64, 1, P, 1, 64, n, (int)S, kchunk));
    CK(sum_splits(P, 64, (int)S, grad + OW3, nullptr));
    CK(colsum(dlogit, 1, grad + OB3));
    // back through layer 3 and the second ReLU
    hipLaunchKernelGGL(k_dh2, dim3(grid_n(n * 64)), dim3(256), 0, s, dlogit, h2, w, dh2, n);
    CK(hipGetLastError());
    // layer 2: dW2 = bf16(h1)^T bf16(dh2), db2 = column sums of dh2
    CK(gemm(h1, 1, 64, dh2, 64, 1, P, 64, 64, n, (int)S, kchunk));
    CK(sum_splits(P, 64 * 64, (int)S, grad + OW2, nullptr));
    CK(colsum(dh2, 64, grad + OB2));
    // back through layer 2 and the first ReLU: dh1 = (bf16(dh2) bf16(W2)^T) * (h1 > 0)
    CK(gemm(dh2, 64, 1, w + OW2, 1, 64, dh1, (int)n, 64, 64, 1, 64));
    CK(sum_splits(dh1, n * 64, 1, dh1, h1));
    // layer 1: dW1 = bf16(x)^T bf16(dh1), db1 = column sums of dh1
    CK(gemm(x, 1, 8, dh1, 64, 1, P, 8, 64, n, (int)S, kchunk));
    CK(sum_splits(P, 8 * 64, (int)S, grad + OW1, nullptr));
    CK(colsum(dh1, 64, grad + OB1));
#undef CK
    return SPDBA_OK;
}

spdba_status spdba_mlp_bce(const float *logit, const float *y, int64_t n, float pos_weight,
                           float *dlogit, double *loss, void *scratch, void *stream) {
    if (!logit || !y || !dlogit || !scratch || n <= 0) return SPDBA_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const unsigned g = grid_n(n) > 1024 ? 1024 : grid_n(n);
    double *part = reinterpret_cast<double *>(scratch);
    hipLaunchKernelGGL(k_bce, dim3(g), dim3(256), 0, s, logit, y, n, pos_weight, dlogit, part);
    if (hipGetLastError() != hipSuccess) return SPDBA_EDEVICE;
    if (loss) {
        hipLaunchKernelGGL(k_bce_final, dim3(1), dim3(64), 0, s, part, (int)g, n, loss);
        return st(hipGetLastError());
    }
    return SPDBA_OK;
}

spdba_status spdba_proposer_features(spdba_plan plan, const double *const ab[3],
                                     const double *const G[3], const uint8_t *mask,
                                     const double *eb, float step_fraction, float *x,
                                     void *scratch, void *stream) {
    if (!plan || !ab || !G || !mask || !eb || !x || !scratch) return SPDBA_EINVAL;
    for (int j = 0; j < 3; ++j)
        if (!ab[j] || !G[j]) return SPDBA_EINVAL;
    const Ctx *c = plan_ctx(plan);
    if (!c) return SPDBA_ESTATE;
    if (c->half) return SPDBA_EUNSUPPORTED;  // features read the full layout's block grid
    hipStream_t s = (hipStream_t)stream;
    double *part = reinterpret_cast<double *>(scratch);
    double *etot = part + (int64_t)c->n_inst * EB_SPLIT;
    hipLaunchKernelGGL(k_eb_part, dim3((unsigned)(c->n_inst * EB_SPLIT)), dim3(256), 0, s, c->inst, eb, part);
    if (hipGetLastError() != hipSuccess) return SPDBA_EDEVICE;
    hipLaunchKernelGGL(k_eb_total, dim3((c->n_inst + 63) / 64), dim3(64), 0, s, part, c->n_inst, etot);
    if (hipGetLastError() != hipSuccess) return SPDBA_EDEVICE;
    FeatArgs fa{ab[0], ab[1], ab[2], G[0], G[1], G[2]};
    hipLaunchKernelGGL(k_features, dim3(grid_n(c->nb_total)), dim3(256), 0, s, *c, fa, mask, eb, etot,
                       step_fraction, x);
    return st(hipGetLastError());
}

spdba_status spdba_mlp_adam(float *w, float *m, float *v, const float *g, uint16_t *w_bf16,
                            int64_t np, float lr, float b1, float b2, float eps, int64_t t,
                            void *stream) {
    if (!w || !m || !v || !g || !w_bf16 || np <= 0 || t < 1) return SPDBA_EINVAL;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid_n(np)), dim3(256), 0, (hipStream_t)stream, w, m, v, g,
                       w_bf16, np, lr, b1, b2, eps, c1, c2);
    return st(hipGetLastError());
}

spdba_status spdba_mlp_to_bf16(const float *w, uint16_t *w_bf16, int64_t np, void *stream) {
    if (!w || !w_bf16 || np <= 0) return SPDBA_EINVAL;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_n(np)), dim3(256), 0, (hipStream_t)stream, w, w_bf16, np);
    return st(hipGetLastError());
}

spdba_status spdba_proposer_labels(const uint8_t *masks, int32_t nm, int64_t nb, float *y,
                                   void *stream) {
    if (!masks || !y || nm < 1 || nb < 1) return SPDBA_EINVAL;
    hipLaunchKernelGGL(k_labels, dim3(grid_n(nb)), dim3(256), 0, (hipStream_t)stream, masks, nm, nb, y);
    return st(hipGetLastError());
}

spdba_status spdba_proposer_miss(const uint8_t *skip, const uint8_t *mask, int64_t nb, uint32_t *count,
                                 void *stream) {
    if (!skip || !mask || !count || nb < 1) return SPDBA_EINVAL;
    hipLaunchKernelGGL(k_miss, dim3(grid_n(nb)), dim3(256), 0, (hipStream_t)stream, skip, mask, nb, count);
    return st(hipGetLastError());
}

spdba_status spdba_proposer_skip(const float *prob, int64_t nb, float thr, const uint32_t *gate,
                                 uint8_t *skip, uint32_t *count, void *stream) {
    if (!prob || !skip || nb < 1 || !(thr == thr)) return SPDBA_EINVAL;
    hipLaunchKernelGGL(k_skip, dim3(grid_n(nb)), dim3(256), 0, (hipStream_t)stream, prob, nb, thr, gate, skip,
                       count);
    return st(hipGetLastError());
}

}  // extern "C"
