// spdba_static.hip -- the update stage of one instance with no allocation.
//
// spdba_apply_noalloc runs what spdba_apply runs for a one-instance plan
// (indicator pass, compaction, active update or the dense update), with the
// same kernels, but without a plan: its scratch memory (instance table, a_b,
// list, counters, G, per-strip and per-tile partial sums) is the file-scope
// device array `scratch`, whose address is taken once per device with
// hipGetSymbolAddress.  Every call on a device shares that array; calls that
// overlap on one device race.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "spdba.h"
#include "spdba_internal.h"

namespace {

using spdba::Ctx;
using spdba::CtlDev;
using spdba::InstDev;

constexpr int64_t kMaxBlocks = int64_t(1) << 18;  // blocks of one call
constexpr int64_t kMaxTiles = int64_t(1) << 17;   // elementwise tiles of the dense update
// byte offsets into the scratch array (each region 256-byte aligned)
constexpr size_t kOffTable = 0;     // InstDev
constexpr size_t kOffCtl = 1024;    // CtlDev (never advanced: no consistency control here)
constexpr size_t kOffCnt = 1536;    // count, nonfinite, done
constexpr size_t kOffG = 1792;      // G, G_last
constexpr size_t kOffK0 = 2048;     // FP64 k = 0 stand-ins of the FP64 path (never read)
constexpr size_t kOffAb = 4096;
constexpr size_t kOffWl = kOffAb + 8 * kMaxBlocks;
constexpr size_t kOffBinst = kOffWl + 4 * kMaxBlocks;
constexpr size_t kOffChunk = kOffBinst + 2 * kMaxBlocks;
constexpr size_t kOffInd = kOffChunk + 4 * (kMaxBlocks / spdba::CHUNK_BLOCKS);
constexpr size_t kOffSmax = kOffInd + 8 * kMaxBlocks;  // strips never outnumber blocks
constexpr size_t kOffDense = kOffSmax + 8 * kMaxBlocks;
constexpr size_t kScratchBytes = kOffDense + 8 * kMaxTiles;  // about 8.9 MB
static_assert(sizeof(InstDev) <= kOffCtl - kOffTable && sizeof(CtlDev) <= kOffCnt - kOffCtl,
              "scratch regions");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Table, control record, counters and G of the call; every block owned by
// instance 0; Regular mode: every block active.
__global__ void __launch_bounds__(256) k_static_init(Ctx c, InstDev I, int dense) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        *const_cast<InstDev *>(c.inst) = I;
        std::memset(static_cast<void *>(c.ctl), 0, sizeof(CtlDev));
        c.ctl->tau = I.tau0;
        c.ctl->tau2 = I.tau2;
        c.count[0] = dense ? (uint32_t)c.nb_total : 0u;
        c.nonfinite[0] = 0u;
        c.done[0] = 0u;
        c.G[0] = 0ull;
        c.G_last[0] = 0ull;
    }
    for (int64_t b = t; b < c.nb_total; b += (int64_t)gridDim.x * blockDim.x) {
        const_cast<uint16_t *>(c.blk_inst)[b] = 0;
        if (dense) {
            c.mask[b] = 1;
            c.worklist[b] = (uint32_t)b;
        }
    }
}

// the device address of `scratch` on the current device, taken once
spdba_status scratch_ptr(unsigned char **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SPDBA_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPDBA_EDEVICE;
        g_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_ptr[dev]);
    return SPDBA_OK;
}

}  // namespace

extern "C" spdba_status spdba_apply_noalloc(const spdba_instance_desc *desc, void *d_state, const void *d_rhs_hat,
                                            double *d_k0, const double *d_rhs_k0, uint8_t *d_mask, void *stream) {
    if (!desc || !d_state || !d_rhs_hat || !d_mask) return SPDBA_EINVAL;
    const spdba_status vs = spdba::validate_desc(desc, 1);
    if (vs != SPDBA_OK) return vs;
    const spdba_instance_desc &x = *desc;
    // CH and GS on the full layout, without consistency control or a kept
    // measure across calls (each call evaluates its measure in full)
    if (x.op != SPDBA_OP_CAHN_HILLIARD && x.op != SPDBA_OP_GRAY_SCOTT) return SPDBA_EUNSUPPORTED;
    if (x.flags & (SPDBA_FLAG_HALF_SPECTRUM | SPDBA_FLAG_TRANSITION | SPDBA_FLAG_REFRESH |
                   SPDBA_FLAG_DYN_THRESHOLD | SPDBA_FLAG_GRAPH))
        return SPDBA_EUNSUPPORTED;
    if (x.full_steps > 0) return SPDBA_EUNSUPPORTED;
    const bool dbl = x.dtype == SPDBA_F64;
    const int op = x.op;
    InstDev I;
    spdba::fill_inst(x, op, dbl, (x.flags & SPDBA_FLAG_PIN_K0) != 0, false, x.dims[2], I);
    // the scratch array's limits
    if (I.nb > kMaxBlocks || I.nstrips > kMaxBlocks || I.ntiles > kMaxTiles) return SPDBA_EUNSUPPORTED;
    if (I.k0path && (!d_k0 || !d_rhs_k0)) return SPDBA_EINVAL;
    unsigned char *sp = nullptr;
    const spdba_status ss = scratch_ptr(&sp);
    if (ss != SPDBA_OK) return ss;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess) return SPDBA_EDEVICE;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;

    const bool dense = (x.flags & SPDBA_FLAG_DENSE) != 0;
    Ctx c;
    std::memset(&c, 0, sizeof(c));
    c.inst = reinterpret_cast<const InstDev *>(sp + kOffTable);
    c.n_inst = 1;
    c.nspec = op == SPDBA_OP_GRAY_SCOTT ? 2 : 1;
    c.op = op;
    c.dense = dense ? 1 : 0;
    c.state = d_state;
    c.work = d_state;  // no transforms here
    c.rhs = const_cast<void *>(d_rhs_hat);
    c.k0 = I.k0path ? d_k0 : reinterpret_cast<double *>(sp + kOffK0);
    c.rhs_k0 = I.k0path ? const_cast<double *>(d_rhs_k0) : reinterpret_cast<double *>(sp + kOffK0 + 16);
    c.a_b = reinterpret_cast<double *>(sp + kOffAb);
    c.a_next = nullptr;
    c.G = reinterpret_cast<unsigned long long *>(sp + kOffG);
    c.G_last = reinterpret_cast<unsigned long long *>(sp + kOffG + 8);
    c.mask = d_mask;
    c.worklist = reinterpret_cast<uint32_t *>(sp + kOffWl);
    c.chunk_cnt = reinterpret_cast<uint32_t *>(sp + kOffChunk);
    c.count = reinterpret_cast<uint32_t *>(sp + kOffCnt);
    c.nonfinite = reinterpret_cast<uint32_t *>(sp + kOffCnt + 4);
    c.done = reinterpret_cast<uint32_t *>(sp + kOffCnt + 8);
    c.nl_part = reinterpret_cast<double *>(sp + kOffDense);  // no nonlinear stage here
    c.ind_part = reinterpret_cast<double *>(sp + kOffInd);
    c.strip_max = reinterpret_cast<double *>(sp + kOffSmax);
    c.dense_part = reinterpret_cast<double *>(sp + kOffDense);
    c.blk_inst = reinterpret_cast<const uint16_t *>(sp + kOffBinst);
    c.skip = nullptr;
    c.e_b = nullptr;
    c.ctl = reinterpret_cast<CtlDev *>(sp + kOffCtl);
    c.htab = nullptr;
    c.ltab = reinterpret_cast<const double *>(sp + kOffK0);
    c.hist1 = c.hist2 = c.hist3 = c.rhs;
    c.taper = nullptr;
    c.taper_bs = 0;
    c.state_ind = (x.flags & SPDBA_FLAG_STATE_INDICATOR) ? 1 : 0;
    c.ab_inc = 0;
    c.trans = 0;
    c.sig_bytes = 0;
    c.half = 0;
    c.half_nb = 0;
    c.ab_sum = (x.flags & SPDBA_FLAG_BLOCK_ENERGY) ? 1 : 0;
    c.run_lmax = 0;
    c.run_ub = 0;
    c.htab_all = 0;
    c.wave_ind = I.chunks > 1 ? 1 : 0;  // block rows wider than a wave row: one wave per strip
    c.nb_total = I.nb;
    c.n_strips = I.nstrips;
    c.n_tiles = I.ntiles;
    c.n_chunks = (I.nb + spdba::CHUNK_BLOCKS - 1) / spdba::CHUNK_BLOCKS;

    const int init_grid = (int)std::min<int64_t>(1024, (I.nb + 255) / 256);
    hipLaunchKernelGGL(k_static_init, dim3(init_grid), dim3(256), 0, s, c, I, dense ? 1 : 0);
    if (hipGetLastError() != hipSuccess) return SPDBA_EDEVICE;
    if (dense) {
        if (spdba::launch_dense(c, dbl, 256, s) != hipSuccess) return SPDBA_EDEVICE;
        return SPDBA_OK;
    }
    if (spdba::launch_indicator(c, dbl, 4, s) != hipSuccess) return SPDBA_EDEVICE;
    if (spdba::launch_compact_append(c, s) != hipSuccess) return SPDBA_EDEVICE;
    const int grid = ((cus * 4 + 7) / 8) * 8;  // a multiple of 8: one list segment per XCD
    if (spdba::launch_update(c, dbl, grid, 0, s) != hipSuccess) return SPDBA_EDEVICE;
    return SPDBA_OK;
}
