// sp-DBA for multimode digital backpropagation (Supplementary S5): kernels
// and the C ABI of include/spdba_mdbp.h.
//
//   k_md_measure   per block of bins: a_b = max of sum_m |E_m|^2 (FP64, modes
//                  in order, omega = 0 left out); blocks dealt to the XCDs in
//                  eight contiguous ranges (k_md_measure_small for blocks of
//                  at most 64 bins: a thread per bin, a max over lane groups);
//                  both clear the mask of the blocks they measure
//   G, the threshold, the mask and the list of active blocks: the
//                  block-activity stage of the main plan (spdba::launch_block_stage)
//   k_md_update    persistent walk of the list, one list segment per XCD; per
//                  bin the M modes in registers, then E'_m = h(omega) sum_j
//                  W_mj E_j row by row with W in LDS (read as broadcasts);
//                  FP32 with M > 16: k_md_update_mfma, one real GEMM per chunk
//                  of 64 bins on the matrix cores
//   k_md_kerr      time domain: E_m <- E_m / n exp(i gamma 8/9 P dz), P the
//                  total power of the sample (the phase in FP64)
//
// Per bin the update moves 16 M bytes (FP32) for 4 M^2 FMAs: up to M = 16
// below the FP32 vector balance point against HBM, above it compute-heavy;
// the matrix W stays in LDS, the modes in registers.

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <vector>

#include "spdba_internal.h"
#include "spdba_mdbp.h"

namespace {

constexpr int kMaxF32 = 64, kMaxF64 = 32;

struct MCtx {
    int M, mm;
    int64_t n, nb;
    int B, lB;
    void *E;             // M x n complex (the state)
    double *ab;
    uint8_t *mask;
    uint32_t *list;
    uint32_t *count;
    unsigned long long *G;
    const void *W;       // [mm][mm] complex, zero-padded
    double tau2, T, dz, alpha, beta2, gamma, invn;
    int pin, dense;
};

template <typename T> struct V2T;
template <> struct V2T<float> { using t = float2; };
template <> struct V2T<double> { using t = double2; };

__device__ __forceinline__ double msq2(double x, double y) { return x * x + y * y; }

__device__ __forceinline__ double mwave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__global__ void k_md_reset(MCtx c) {
    if (threadIdx.x == 0) {
        *c.G = 0ull;
        *c.count = 0u;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_md_measure(MCtx c) {
    __shared__ double red[4];
    using V2 = typename V2T<T>::t;
    const V2 *E = reinterpret_cast<const V2 *>(c.E);
    const int64_t per = (c.nb + 7) >> 3;
    const int64_t b = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (b >= c.nb) return;  // workgroup-uniform, before any barrier
    double amax = 0.0;
    for (int s = threadIdx.x; s < c.B; s += blockDim.x) {
        const int64_t e = (b << c.lB) + s;
        double acc = 0.0;
        for (int m = 0; m < c.M; ++m) {
            const V2 v = E[m * c.n + e];
            acc = acc + msq2((double)v.x, (double)v.y);
        }
        if (e == 0) acc = 0.0;
        amax = fmax(amax, acc);
    }
    amax = mwave_max(amax);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = fmax(m, red[k]);
        c.ab[b] = m;
        c.mask[b] = 0;  // a fresh measure: nothing for the stage's G pass to merge
    }
}

// blocks of at most 64 bins: one thread per bin, the block maximum a max over
// groups of B lanes (n is a multiple of 64, so every wave runs whole)
__global__ void __launch_bounds__(256) k_md_measure_small(MCtx c, int fp64) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < c.n; e += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        if (fp64) {
            const double2 *E = reinterpret_cast<const double2 *>(c.E);
#pragma unroll 8
            for (int m = 0; m < c.M; ++m) {
                const double2 v = E[m * c.n + e];
                acc = acc + msq2(v.x, v.y);
            }
        } else {
            const float2 *E = reinterpret_cast<const float2 *>(c.E);
#pragma unroll 8
            for (int m = 0; m < c.M; ++m) {
                const float2 v = E[m * c.n + e];
                acc = acc + msq2((double)v.x, (double)v.y);
            }
        }
        if (e == 0) acc = 0.0;
        for (int off = c.B >> 1; off >= 1; off >>= 1) acc = fmax(acc, __shfl_xor(acc, off, 64));
        if ((e & (c.B - 1)) == 0) {
            c.ab[e >> c.lB] = acc;
            c.mask[e >> c.lB] = 0;
        }
    }
}

template <typename T, int MM>
__global__ void __launch_bounds__(256) k_md_update(MCtx c) {
    using V2 = typename V2T<T>::t;
    __shared__ V2 w[MM * MM];
    for (int i = threadIdx.x; i < MM * MM; i += blockDim.x) w[i] = reinterpret_cast<const V2 *>(c.W)[i];
    __syncthreads();
    V2 *E = reinterpret_cast<V2 *>(c.E);
    const int M = c.M;
    const int64_t n = c.n;
    const int64_t total = c.dense ? c.nb : (int64_t)*c.count;
    const int xcd = blockIdx.x & 7, per = gridDim.x >> 3;
    const int64_t seg = (total + 7) >> 3;
    const int64_t lo = std::min<int64_t>(total, seg * xcd), hi = std::min<int64_t>(total, seg * (xcd + 1));
    const double att = exp(-c.alpha * c.dz / 4.0);
    // blocks narrower than the workgroup: several list entries per iteration
    const int lanes = c.B < (int)blockDim.x ? c.B : (int)blockDim.x;
    const int epi = (int)blockDim.x / lanes, sub = (int)threadIdx.x / lanes, s0 = (int)threadIdx.x - sub * lanes;
    for (int64_t base = lo + (int64_t)(blockIdx.x >> 3) * epi; base < hi; base += (int64_t)per * epi) {
        const int64_t ent = base + sub;
        if (ent >= hi) continue;
        const int64_t b = c.dense ? ent : (int64_t)c.list[ent];
        for (int s = s0; s < c.B; s += lanes) {
            const int64_t e = (b << c.lB) + s;
            const int64_t si = e <= ((n - 1) >> 1) ? e : e - n;
            const double om = 6.283185307179586476925286766559 * (double)si / c.T;
            const double ph = c.beta2 * 0.5 * om * om * c.dz * 0.5;
            double sp, cp;
            sincos(ph, &sp, &cp);
            const T hr = (T)(att * cp), hi2 = (T)(att * sp);
            T br[MM], bi[MM];
#pragma unroll
            for (int j = 0; j < MM; ++j) {
                br[j] = bi[j] = (T)0;
                if (j < M) {
                    const V2 v = E[j * n + e];
                    br[j] = v.x;
                    bi[j] = v.y;
                }
            }
            for (int m = 0; m < M; ++m) {
                T xr = (T)0, xi = (T)0;
#pragma unroll
                for (int j = 0; j < MM; ++j) {
                    const V2 wv = w[m * MM + j];
                    xr = fma(wv.x, br[j], xr);
                    xr = fma(-wv.y, bi[j], xr);
                    xi = fma(wv.x, bi[j], xi);
                    xi = fma(wv.y, br[j], xi);
                }
                V2 o;
                o.x = hr * xr - hi2 * xi;
                o.y = hr * xi + hi2 * xr;
                E[m * n + e] = o;
            }
        }
    }
}

// Wide modes (FP32, M > 16): the coupled half-step as one real GEMM per chunk
// of 64 bins on the matrix cores.  With W = Wr + i Wi and b = br + i bi,
// [xr; xi] = [[Wr, -Wi], [Wi, Wr]] [br; bi]; B holds the chunk's bins as 64
// columns over 2 MM rows (re rows, then im rows), the product goes to LDS
// and the stores apply h(omega) in the loads' coalesced pattern.  LDS pitches
// padded so that an operand read falls on distinct banks.
typedef float md_f4 __attribute__((ext_vector_type(4)));

template <int MM>
__global__ void __launch_bounds__(256) k_md_update_mfma(MCtx c) {
    constexpr int R = 2 * MM, NC = 64, SA = R + 4, SB = NC + 16;
    __shared__ float wa[R * SA];  // the real form of W
    __shared__ float bs[R * SB];  // B, then X
    const float2 *wsrc = reinterpret_cast<const float2 *>(c.W);  // [MM][MM] complex, zero-padded
    for (int k = threadIdx.x; k < MM * MM; k += blockDim.x) {
        const int i = k / MM, j = k - i * MM;
        const float2 v = wsrc[k];
        wa[i * SA + j] = v.x;
        wa[i * SA + MM + j] = -v.y;
        wa[(MM + i) * SA + j] = v.y;
        wa[(MM + i) * SA + MM + j] = v.x;
    }
    __syncthreads();
    float2 *E = reinterpret_cast<float2 *>(c.E);
    const int M = c.M, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t n = c.n;
    const int64_t total = c.dense ? c.nb : (int64_t)*c.count;
    const int xcd = blockIdx.x & 7, per = gridDim.x >> 3;
    const int64_t seg = (total + 7) >> 3;
    const int64_t lo = std::min<int64_t>(total, seg * xcd), hi = std::min<int64_t>(total, seg * (xcd + 1));
    const int row = lane & 15, kq = lane >> 4;
    const double att = exp(-c.alpha * c.dz / 4.0);
    // chunks of 64 bins: NC / B blocks of the list per chunk when B < 64.
    // The chunks of the workgroup run as one sequence, and the global loads
    // of the next chunk are issued before the current chunk's product.
    // Thread t holds bin t % 64 of the chunk (its offset and h(omega) in
    // registers) for the modes t / 64 + 4 j.
    const int bpc = c.B < NC ? NC / c.B : 1;
    constexpr int PT = MM / 4;
    float2 pv[PT];
    int64_t pe = 0;
    int pnm = 0;
    float2 ph = make_float2(0.f, 0.f);
    auto fetch = [&](int64_t bs0, int s) {  // workgroup-uniform arguments
        const int nblk = (int)std::min<int64_t>(bpc, hi - bs0);
        pnm = bpc > 1 ? nblk * c.B : min(NC, c.B - s);
        pe = 0;
        if (lane < pnm) {
            const int64_t b = bpc > 1 ? (c.dense ? bs0 + lane / c.B : (int64_t)c.list[bs0 + lane / c.B]) :
                                        (c.dense ? bs0 : (int64_t)c.list[bs0]);
            pe = (b << c.lB) + (bpc > 1 ? (lane & (c.B - 1)) : s + lane);
        }
        const int64_t si = pe <= ((n - 1) >> 1) ? pe : pe - n;
        const double om = 6.283185307179586476925286766559 * (double)si / c.T;
        double sp, cp;
        sincos(c.beta2 * 0.5 * om * om * c.dz * 0.5, &sp, &cp);
        ph = make_float2((float)(att * cp), (float)(att * sp));
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int i = wave + 4 * j;
            pv[j] = (i < M && lane < pnm) ? E[i * n + pe] : make_float2(0.f, 0.f);
        }
    };
    int64_t base = lo + (int64_t)(blockIdx.x >> 3) * bpc;
    int s0 = 0;
    if (base < hi) fetch(base, 0);
    while (base < hi) {  // workgroup-uniform
        const int nm = pnm;
        const int64_t e = pe;
        const float2 h = ph;
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int i = wave + 4 * j;
            bs[i * SB + lane] = pv[j].x;
            bs[(MM + i) * SB + lane] = pv[j].y;
        }
        __syncthreads();
        // the next chunk (blocks of at least 64 bins go in chunks): its loads
        // fly while this one is multiplied
        int s1 = s0 + NC;
        int64_t base1 = base;
        if (bpc > 1 || s1 >= c.B) {
            s1 = 0;
            base1 += (int64_t)per * bpc;
        }
        if (base1 < hi) fetch(base1, s1);
        // X = Wa B: (R / 16) x (NC / 16) tiles over the four waves; the
        // results wait in registers until every wave has read B
        md_f4 acc[(R / 16) * (NC / 16) / 4];
#pragma unroll
        for (int q = 0; q < (R / 16) * (NC / 16) / 4; ++q) {
            const int tile = wave + 4 * q;
            const int rt = tile / (NC / 16), ct = tile - rt * (NC / 16);
            md_f4 a4 = {0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < R; k0 += 4) {
                const float av = wa[(rt * 16 + row) * SA + k0 + kq];
                const float bv = bs[(k0 + kq) * SB + ct * 16 + row];
                a4 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, a4, 0, 0, 0);
            }
            acc[q] = a4;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < (R / 16) * (NC / 16) / 4; ++q) {
            const int tile = wave + 4 * q;
            const int rt = tile / (NC / 16), ct = tile - rt * (NC / 16);
#pragma unroll
            for (int r = 0; r < 4; ++r) bs[(rt * 16 + kq * 4 + r) * SB + ct * 16 + row] = acc[q][r];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int i = wave + 4 * j;
            if (i < M && lane < nm) {
                const float xr = bs[i * SB + lane], xi = bs[(MM + i) * SB + lane];
                E[i * n + e] = make_float2(h.x * xr - h.y * xi, h.x * xi + h.y * xr);
            }
        }
        __syncthreads();  // bs is free for the next chunk
        base = base1;
        s0 = s1;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_md_kerr(MCtx c) {
    using V2 = typename V2T<T>::t;
    V2 *E = reinterpret_cast<V2 *>(c.E);
    const double k = c.gamma * (8.0 / 9.0) * c.dz;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < c.n; p += (int64_t)gridDim.x * blockDim.x) {
        double P = 0.0;
        for (int m = 0; m < c.M; ++m) {
            const V2 v = E[m * c.n + p];
            P = P + msq2((double)v.x * c.invn, (double)v.y * c.invn);
        }
        double sp, cp;
        sincos(k * P, &sp, &cp);
        const T cr = (T)(cp * c.invn), ci = (T)(sp * c.invn);
        for (int m = 0; m < c.M; ++m) {
            const V2 v = E[m * c.n + p];
            V2 o;
            o.x = cr * v.x - ci * v.y;
            o.y = cr * v.y + ci * v.x;
            E[m * c.n + p] = o;
        }
    }
}

template <typename T>
__global__ void k_md_scale(int64_t cnt, const typename V2T<T>::t *in, typename V2T<T>::t *out, T s) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        typename V2T<T>::t o = in[i];
        o.x *= s;
        o.y *= s;
        out[i] = o;
    }
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) { int l = 0; while ((int64_t(1) << l) < v) ++l; return l; }

using cd = std::complex<double>;

// exp(i delta K) by scaling and squaring of the Taylor series (FP64)
std::vector<cd> expm_i(int M, const double *K, double delta) {
    std::vector<cd> A((size_t)M * M), R((size_t)M * M, 0.0), term, tmp((size_t)M * M);
    double nrm = 0.0;
    for (int i = 0; i < M; ++i) {
        double row = 0.0;
        for (int j = 0; j < M; ++j) {
            A[(size_t)i * M + j] = cd(0.0, delta) * cd(K[2 * ((size_t)i * M + j)], K[2 * ((size_t)i * M + j) + 1]);
            row += std::abs(A[(size_t)i * M + j]);
        }
        nrm = std::max(nrm, row);
    }
    int sq = 0;
    while (nrm > 0.25) {
        nrm *= 0.5;
        ++sq;
    }
    const double sc = std::ldexp(1.0, -sq);
    for (auto &v : A) v *= sc;
    auto mul = [&](const std::vector<cd> &X, const std::vector<cd> &Y, std::vector<cd> &Z) {
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                cd s = 0.0;
                for (int k = 0; k < M; ++k) s += X[(size_t)i * M + k] * Y[(size_t)k * M + j];
                Z[(size_t)i * M + j] = s;
            }
    };
    term.assign((size_t)M * M, 0.0);
    for (int i = 0; i < M; ++i) term[(size_t)i * M + i] = R[(size_t)i * M + i] = 1.0;
    for (int k = 1; k <= 24; ++k) {  // |A| <= 1/4: the remainder is below 1e-30
        mul(term, A, tmp);
        for (auto &v : tmp) v /= (double)k;
        term.swap(tmp);
        for (size_t i = 0; i < R.size(); ++i) R[i] += term[i];
    }
    for (int s = 0; s < sq; ++s) {
        mul(R, R, tmp);
        R.swap(tmp);
    }
    return R;
}

int tile_of(int M) {
    int mm = 2;
    while (mm < M) mm <<= 1;
    return mm;
}

}  // namespace

struct spdba_mdbp_s {
    spdba_mdbp_desc d{};
    MCtx c{};
    bool dbl = false, timing = false, bound = false;
    int esize = 8, cu = 256;
    hipStream_t stream = nullptr;
    size_t state_bytes = 0, work_bytes = 0, fft_work = 0;
    size_t o_fft = 0, o_ab = 0, o_mask = 0, o_list = 0, o_ctl = 0, o_w = 0, o_tmp = 0, o_stage = 0;
    spdba::BlockStage stage{};  // G, threshold and ordered compaction (the main plan's kernels)
    rocfft_plan fwd = nullptr, inv = nullptr;
    rocfft_execution_info info = nullptr;
    std::vector<cd> W;
    char *d_state = nullptr, *d_work = nullptr;
    hipEvent_t ev[6] = {};
    bool ev_valid = false;
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
};

namespace {

#define MTRY_HIP(x)                                   \
    do {                                              \
        if ((x) != hipSuccess) return SPDBA_EDEVICE;  \
    } while (0)
#define MTRY(x)                                       \
    do {                                              \
        spdba_status s_ = (x);                        \
        if (s_ != SPDBA_OK) return s_;                \
    } while (0)

spdba_status validate(const spdba_mdbp_desc *d, const double *K) {
    if (!d || !K) return SPDBA_EINVAL;
    if (d->M < 1 || d->dtype < SPDBA_F32 || d->dtype > SPDBA_F64) return SPDBA_EINVAL;
    if (d->flags & ~(uint32_t)(SPDBA_MDBP_DENSE | SPDBA_MDBP_PIN_K0 | SPDBA_MDBP_TIMING | SPDBA_MDBP_GRAPH))
        return SPDBA_EINVAL;
    if ((d->flags & SPDBA_MDBP_GRAPH) && (d->flags & SPDBA_MDBP_TIMING)) return SPDBA_EUNSUPPORTED;
    if (!pow2(d->n) || d->n < 16 || d->n > (int64_t(1) << 28)) return SPDBA_EINVAL;
    if (!pow2(d->block) || d->block > d->n) return SPDBA_EINVAL;
    const double vals[] = {d->tau, d->T, d->dz, d->alpha, d->beta2, d->gamma};
    for (double v : vals)
        if (!std::isfinite(v)) return SPDBA_EINVAL;
    if (d->tau < 0 || d->T <= 0 || d->dz <= 0) return SPDBA_EINVAL;
    if ((int64_t)d->M * d->n > (int64_t(1) << 34)) return SPDBA_EINVAL;
    if (d->M > (d->dtype == SPDBA_F64 ? kMaxF64 : kMaxF32)) return SPDBA_EUNSUPPORTED;
    double scale = 0.0;
    for (int i = 0; i < d->M * d->M * 2; ++i) {
        if (!std::isfinite(K[i])) return SPDBA_EINVAL;
        scale = std::max(scale, std::fabs(K[i]));
    }
    for (int i = 0; i < d->M; ++i)
        for (int j = 0; j < d->M; ++j) {
            const double *a = K + 2 * ((size_t)i * d->M + j), *b = K + 2 * ((size_t)j * d->M + i);
            if (std::fabs(a[0] - b[0]) > 1e-12 * scale || std::fabs(a[1] + b[1]) > 1e-12 * scale) return SPDBA_EINVAL;
        }
    return SPDBA_OK;
}

template <typename T>
void launch_upd(const MCtx &c, int grid, hipStream_t s) {
    // wide modes, sparse walk: the matrix cores (two blocks of 32 bins per
    // workgroup keep many workgroups busy at low activity); the Regular
    // update of every block is faster on the vector units (its 109 KB of LDS
    // at M = 64 would leave one workgroup per compute unit)
    if constexpr (sizeof(T) == 4) {
        if (c.dense) goto vector;
        if (c.mm == 32) {
            hipLaunchKernelGGL((k_md_update_mfma<32>), dim3(grid), dim3(256), 0, s, c);
            return;
        }
        if (c.mm == 64) {
            hipLaunchKernelGGL((k_md_update_mfma<64>), dim3(grid), dim3(256), 0, s, c);
            return;
        }
    }
vector:
    switch (c.mm) {
        case 2: hipLaunchKernelGGL((k_md_update<T, 2>), dim3(grid), dim3(256), 0, s, c); break;
        case 4: hipLaunchKernelGGL((k_md_update<T, 4>), dim3(grid), dim3(256), 0, s, c); break;
        case 8: hipLaunchKernelGGL((k_md_update<T, 8>), dim3(grid), dim3(256), 0, s, c); break;
        case 16: hipLaunchKernelGGL((k_md_update<T, 16>), dim3(grid), dim3(256), 0, s, c); break;
        case 32: hipLaunchKernelGGL((k_md_update<T, 32>), dim3(grid), dim3(256), 0, s, c); break;
        default:  // tile 64: FP32 only (validated at creation)
            if constexpr (sizeof(T) == 4) hipLaunchKernelGGL((k_md_update<T, 64>), dim3(grid), dim3(256), 0, s, c);
            break;
    }
}

spdba_status exec(spdba_mdbp_plan p, rocfft_plan f, void *buf) {
    void *ib[1] = {buf};
    return rocfft_execute(f, ib, nullptr, p->info) == rocfft_status_success ? SPDBA_OK : SPDBA_EFFT;
}

spdba_status linear_half(spdba_mdbp_plan p) {
    const MCtx &c = p->c;
    if (!c.dense) {
        hipLaunchKernelGGL(k_md_reset, dim3(1), dim3(64), 0, p->stream, c);
        if (c.B <= 64 && c.n >= 64) {
            const int g = (int)std::min<int64_t>((c.n + 255) / 256, (int64_t)p->cu * 16);
            hipLaunchKernelGGL(k_md_measure_small, dim3(g), dim3(256), 0, p->stream, c, p->dbl ? 1 : 0);
        } else {
            const int nbg = (int)(((c.nb + 7) >> 3) << 3);
            if (p->dbl) hipLaunchKernelGGL(k_md_measure<double>, dim3(nbg), dim3(256), 0, p->stream, c);
            else hipLaunchKernelGGL(k_md_measure<float>, dim3(nbg), dim3(256), 0, p->stream, c);
        }
        MTRY_HIP(hipGetLastError());
        MTRY_HIP(spdba::launch_block_stage(p->stage, p->stream));
    }
    const int64_t epi = c.B < 256 ? 256 / c.B : 1;  // list entries per workgroup iteration
    const int grid = (int)(std::max<int64_t>(8, std::min<int64_t>((c.nb + epi - 1) / epi, (int64_t)p->cu * 8)) + 7) / 8 * 8;
    if (p->dbl) launch_upd<double>(c, grid, p->stream);
    else launch_upd<float>(c, grid, p->stream);
    MTRY_HIP(hipGetLastError());
    return SPDBA_OK;
}

void rec(spdba_mdbp_plan p, int i) {
    if (p->timing) (void)hipEventRecord(p->ev[i], p->stream);
}

spdba_status one_step(spdba_mdbp_plan p) {
    const MCtx &c = p->c;
    rec(p, 0);
    MTRY(linear_half(p));
    rec(p, 1);
    MTRY(exec(p, p->inv, p->d_state));
    rec(p, 2);
    const int grid = (int)std::min<int64_t>((c.n + 255) / 256, (int64_t)p->cu * 16);
    if (p->dbl) hipLaunchKernelGGL(k_md_kerr<double>, dim3(grid), dim3(256), 0, p->stream, c);
    else hipLaunchKernelGGL(k_md_kerr<float>, dim3(grid), dim3(256), 0, p->stream, c);
    MTRY_HIP(hipGetLastError());
    rec(p, 3);
    MTRY(exec(p, p->fwd, p->d_state));
    rec(p, 4);
    MTRY(linear_half(p));
    rec(p, 5);
    p->ev_valid = p->timing;
    return SPDBA_OK;
}

}  // namespace

extern "C" {

spdba_status spdba_mdbp_coupling(int32_t M, const double *K, double delta, double *out) {
    if (M < 1 || M > 1024 || !K || !out || !std::isfinite(delta)) return SPDBA_EINVAL;
    const std::vector<cd> W = expm_i(M, K, delta);
    for (size_t i = 0; i < W.size(); ++i) {
        out[2 * i] = W[i].real();
        out[2 * i + 1] = W[i].imag();
    }
    return SPDBA_OK;
}

spdba_status spdba_mdbp_create(const spdba_mdbp_desc *desc, const double *K, void *stream, spdba_mdbp_plan *out) {
    if (!out) return SPDBA_EINVAL;
    *out = nullptr;
    MTRY(validate(desc, K));
    spdba_mdbp_plan p = new (std::nothrow) spdba_mdbp_s();
    if (!p) return SPDBA_EDEVICE;
    p->d = *desc;
    p->dbl = desc->dtype == SPDBA_F64;
    p->esize = p->dbl ? 16 : 8;
    p->timing = (desc->flags & SPDBA_MDBP_TIMING) != 0;
    p->use_graph = (desc->flags & SPDBA_MDBP_GRAPH) != 0;
    p->stream = reinterpret_cast<hipStream_t>(stream);
    MCtx &c = p->c;
    c.M = desc->M;
    c.mm = tile_of(desc->M);
    c.n = desc->n;
    c.B = desc->block;
    c.lB = ilog2(desc->block);
    c.nb = desc->n / desc->block;
    c.tau2 = desc->tau * desc->tau;
    c.T = desc->T;
    c.dz = desc->dz;
    c.alpha = desc->alpha;
    c.beta2 = desc->beta2;
    c.gamma = desc->gamma;
    c.invn = 1.0 / (double)desc->n;
    c.pin = (desc->flags & SPDBA_MDBP_PIN_K0) ? 1 : 0;
    c.dense = (desc->flags & SPDBA_MDBP_DENSE) ? 1 : 0;
    p->W = expm_i(c.M, K, desc->dz / 2.0);
    auto fail = [&](spdba_status s) {
        spdba_mdbp_destroy(p);
        return s;
    };
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(SPDBA_EDEVICE);
    p->cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (spdba::fft_setup() != SPDBA_OK) return fail(SPDBA_EFFT);
    size_t len[1] = {(size_t)c.n};
    const rocfft_precision prec = p->dbl ? rocfft_precision_double : rocfft_precision_single;
    if (rocfft_plan_create(&p->fwd, rocfft_placement_inplace, rocfft_transform_type_complex_forward, prec, 1, len,
                           (size_t)c.M, nullptr) != rocfft_status_success ||
        rocfft_plan_create(&p->inv, rocfft_placement_inplace, rocfft_transform_type_complex_inverse, prec, 1, len,
                           (size_t)c.M, nullptr) != rocfft_status_success)
        return fail(SPDBA_EFFT);
    size_t w1 = 0, w2 = 0;
    if (rocfft_plan_get_work_buffer_size(p->fwd, &w1) != rocfft_status_success ||
        rocfft_plan_get_work_buffer_size(p->inv, &w2) != rocfft_status_success)
        return fail(SPDBA_EFFT);
    p->fft_work = std::max(w1, w2);
    if (rocfft_execution_info_create(&p->info) != rocfft_status_success ||
        rocfft_execution_info_set_stream(p->info, p->stream) != rocfft_status_success)
        return fail(SPDBA_EFFT);
    if (p->timing)
        for (auto &e : p->ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(SPDBA_EDEVICE);
    const size_t spec = (size_t)c.M * c.n * p->esize;
    p->state_bytes = spec;
    size_t o = 0;
    p->o_fft = o;
    o = al256(o + p->fft_work);
    p->o_ab = o;
    o = al256(o + sizeof(double) * c.nb);
    p->o_mask = o;
    o = al256(o + c.nb);
    p->o_list = o;
    o = al256(o + sizeof(uint32_t) * c.nb);
    p->o_ctl = o;
    o = al256(o + 16);
    p->o_w = o;
    o = al256(o + (size_t)p->esize * c.mm * c.mm);
    p->o_tmp = o;  // get_field's copy
    o = al256(o + spec);
    p->o_stage = o;
    o = al256(o + spdba::block_stage_bytes(c.nb));
    p->work_bytes = o;
    *out = p;
    return SPDBA_OK;
}

spdba_status spdba_mdbp_buffer_sizes(spdba_mdbp_plan p, size_t *sb, size_t *wb) {
    if (!p || !sb || !wb) return SPDBA_EINVAL;
    *sb = p->state_bytes;
    *wb = p->work_bytes;
    return SPDBA_OK;
}

spdba_status spdba_mdbp_bind(spdba_mdbp_plan p, void *d_state, void *d_work) {
    if (!p || !d_state || !d_work) return SPDBA_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_state) & 255) || (reinterpret_cast<uintptr_t>(d_work) & 255))
        return SPDBA_EINVAL;
    p->d_state = static_cast<char *>(d_state);
    p->d_work = static_cast<char *>(d_work);
    MCtx &c = p->c;
    c.E = p->d_state;
    c.ab = reinterpret_cast<double *>(p->d_work + p->o_ab);
    c.mask = reinterpret_cast<uint8_t *>(p->d_work + p->o_mask);
    c.list = reinterpret_cast<uint32_t *>(p->d_work + p->o_list);
    c.G = reinterpret_cast<unsigned long long *>(p->d_work + p->o_ctl);
    c.count = reinterpret_cast<uint32_t *>(p->d_work + p->o_ctl + 8);
    c.W = p->d_work + p->o_w;
    if (p->fft_work &&
        rocfft_execution_info_set_work_buffer(p->info, p->d_work + p->o_fft, p->fft_work) != rocfft_status_success)
        return SPDBA_EFFT;
    const int M = c.M, mm = c.mm;
    std::vector<double> wd((size_t)2 * mm * mm, 0.0);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            wd[2 * ((size_t)i * mm + j)] = p->W[(size_t)i * M + j].real();
            wd[2 * ((size_t)i * mm + j) + 1] = p->W[(size_t)i * M + j].imag();
        }
    if (p->dbl) {
        MTRY_HIP(hipMemcpy(p->d_work + p->o_w, wd.data(), 8 * wd.size(), hipMemcpyHostToDevice));
    } else {
        std::vector<float> wf(wd.begin(), wd.end());
        MTRY_HIP(hipMemcpy(p->d_work + p->o_w, wf.data(), 4 * wf.size(), hipMemcpyHostToDevice));
    }
    MTRY_HIP(hipMemsetAsync(p->d_work + p->o_ab, 0, p->o_w - p->o_ab, p->stream));
    p->stage.nb = c.nb;
    p->stage.a_b = c.ab;
    p->stage.a_next = c.ab;  // no kept measure: the measure pass clears the mask every update
    p->stage.mask = c.mask;
    p->stage.list = c.list;
    p->stage.count = c.count;
    p->stage.G = c.G;
    p->stage.aux = p->d_work + p->o_stage;
    MTRY_HIP(spdba::block_stage_init(p->stage, c.tau2, c.pin, p->stream));
    MTRY_HIP(hipStreamSynchronize(p->stream));
    p->bound = true;
    return SPDBA_OK;
}

spdba_status spdba_mdbp_set_spectrum(spdba_mdbp_plan p, const void *src) {
    if (!p || !src) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    MTRY_HIP(hipMemcpyAsync(p->d_state, src, p->state_bytes, hipMemcpyDeviceToDevice, p->stream));
    return SPDBA_OK;
}

spdba_status spdba_mdbp_get_spectrum(spdba_mdbp_plan p, void *dst) {
    if (!p || !dst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    MTRY_HIP(hipMemcpyAsync(dst, p->d_state, p->state_bytes, hipMemcpyDeviceToDevice, p->stream));
    return SPDBA_OK;
}

spdba_status spdba_mdbp_set_field(spdba_mdbp_plan p, const void *src) {
    MTRY(spdba_mdbp_set_spectrum(p, src));
    return exec(p, p->fwd, p->d_state);
}

spdba_status spdba_mdbp_get_field(spdba_mdbp_plan p, void *dst) {
    if (!p || !dst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    char *tmp = p->d_work + p->o_tmp;
    MTRY_HIP(hipMemcpyAsync(tmp, p->d_state, p->state_bytes, hipMemcpyDeviceToDevice, p->stream));
    MTRY(exec(p, p->inv, tmp));
    const int64_t cnt = (int64_t)p->c.M * p->c.n;
    const int grid = (int)std::min<int64_t>((cnt + 255) / 256, (int64_t)p->cu * 16);
    if (p->dbl)
        hipLaunchKernelGGL(k_md_scale<double>, dim3(grid), dim3(256), 0, p->stream, cnt,
                           reinterpret_cast<const double2 *>(tmp), static_cast<double2 *>(dst), p->c.invn);
    else
        hipLaunchKernelGGL(k_md_scale<float>, dim3(grid), dim3(256), 0, p->stream, cnt,
                           reinterpret_cast<const float2 *>(tmp), static_cast<float2 *>(dst), (float)p->c.invn);
    MTRY_HIP(hipGetLastError());
    return SPDBA_OK;
}

spdba_status spdba_mdbp_apply(spdba_mdbp_plan p) {
    if (!p) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    return linear_half(p);
}

spdba_status spdba_mdbp_step(spdba_mdbp_plan p, int32_t n) {
    if (!p || n < 0) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    if (!p->use_graph || n == 0) {
        for (int32_t i = 0; i < n; ++i) MTRY(one_step(p));
        return SPDBA_OK;
    }
    if (!p->gexec) {  // one whole step captured once (kernels and rocFFT launches, no memset nodes)
        MTRY_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
        const spdba_status st = one_step(p);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(p->stream, &g);
        if (st != SPDBA_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        MTRY_HIP(ec);
        p->graph = g;
        MTRY_HIP(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
    }
    for (int32_t i = 0; i < n; ++i) MTRY_HIP(hipGraphLaunch(p->gexec, p->stream));
    return SPDBA_OK;
}

spdba_status spdba_mdbp_indicator(spdba_mdbp_plan p, double *ab, size_t n, double *G) {
    if (!p || (ab && n < (size_t)p->c.nb)) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    MTRY_HIP(hipStreamSynchronize(p->stream));
    if (ab) MTRY_HIP(hipMemcpy(ab, p->c.ab, sizeof(double) * p->c.nb, hipMemcpyDeviceToHost));
    if (G) {
        unsigned long long bits = 0;
        MTRY_HIP(hipMemcpy(&bits, p->c.G, 8, hipMemcpyDeviceToHost));
        std::memcpy(G, &bits, 8);
    }
    return SPDBA_OK;
}

spdba_status spdba_mdbp_active_mask(spdba_mdbp_plan p, uint8_t *mask, size_t n, int64_t *count) {
    if (!p || (mask && n < (size_t)p->c.nb)) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    MTRY_HIP(hipStreamSynchronize(p->stream));
    if (p->c.dense) {
        if (mask) std::memset(mask, 1, p->c.nb);
        if (count) *count = p->c.nb;
        return SPDBA_OK;
    }
    if (mask) MTRY_HIP(hipMemcpy(mask, p->c.mask, p->c.nb, hipMemcpyDeviceToHost));
    if (count) {
        uint32_t v = 0;
        MTRY_HIP(hipMemcpy(&v, p->c.count, 4, hipMemcpyDeviceToHost));
        *count = v;
    }
    return SPDBA_OK;
}

spdba_status spdba_mdbp_stats(spdba_mdbp_plan p, spdba_mdbp_stats_t *out) {
    if (!p || !out) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    std::memset(out, 0, sizeof(*out));
    out->n_blocks = p->c.nb;
    MTRY(spdba_mdbp_active_mask(p, nullptr, 0, &out->active_blocks));
    if (!p->c.dense) MTRY(spdba_mdbp_indicator(p, nullptr, 0, &out->G));
    if (p->timing && p->ev_valid) {
        float a = 0.f, b = 0.f, t1 = 0.f, t2 = 0.f, k = 0.f;
        (void)hipEventElapsedTime(&a, p->ev[0], p->ev[1]);
        (void)hipEventElapsedTime(&t1, p->ev[1], p->ev[2]);
        (void)hipEventElapsedTime(&k, p->ev[2], p->ev[3]);
        (void)hipEventElapsedTime(&t2, p->ev[3], p->ev[4]);
        (void)hipEventElapsedTime(&b, p->ev[4], p->ev[5]);
        out->stage_ms[0] = a + b;
        out->stage_ms[1] = t1 + t2;
        out->stage_ms[2] = k;
    }
    return SPDBA_OK;
}

spdba_status spdba_mdbp_destroy(spdba_mdbp_plan p) {
    if (!p) return SPDBA_OK;
    if (p->fwd) rocfft_plan_destroy(p->fwd);
    if (p->inv) rocfft_plan_destroy(p->inv);
    if (p->info) rocfft_execution_info_destroy(p->info);
    for (auto &e : p->ev)
        if (e) (void)hipEventDestroy(e);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
    return SPDBA_OK;
}

}  // extern "C"
