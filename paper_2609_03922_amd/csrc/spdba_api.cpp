// spdba_api.cpp -- host side of the sp-DBA library: descriptor validation,
// buffer layout, rocFFT plans, stage sequencing, HIP-graph replay and
// read-backs.  Implements the C ABI declared in include/spdba.h.
//
// The host never touches field data: every step of the method runs in the HIP
// kernels of spdba_kernels.hip or in rocFFT.

#include "spdba.h"
#include "spdba_internal.h"
#include "spdba_proposer.h"

#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

using namespace spdba;

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int64_t kMaxSigBytes = 65536;  // LDS of the transition update per workgroup
constexpr int64_t kMaxHalfPoints = int64_t(1) << 18;  // largest half-layout grid accepted

std::once_flag g_rocfft_once;
rocfft_status g_rocfft_setup = rocfft_status_success;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// One rocFFT plan with its input-preservation property.
struct Fft {
    rocfft_plan plan = nullptr;
    bool preserves = true;  // out-of-place plans: input survives execution
};

// Instances of one grid size, contiguous in memory (transform batch).
struct Group {
    int64_t N = 0;
    int count = 0;
    int64_t off = 0;       // first complex element of the group
    Fft inv_oop, fwd_ip;   // batched: CH/GS inverse state->work; NLSE forward in place
    Fft fwd_oop;           // batched: CH/GS forward work->rhs
    Fft inv_ip;            // batched in-place inverse (NLSE, or CH/GS copy fallback)
    Fft inv1_oop, fwd1_ip, inv1_ip;  // one instance (nspec transforms)
    Fft fwd1_oop;                    // half layout: one instance, real W -> R
};

}  // namespace

struct spdba_plan_s {
    std::vector<spdba_instance_desc> desc;
    std::vector<InstDev> hinst;      // host copy of the device table (original order)
    std::vector<uint16_t> blk_inst;  // owning instance per global block
    std::vector<int> group_of;       // instance -> group
    std::vector<Group> groups;
    int n_inst = 0, op = 0, nspec = 1, ndim = 1;
    bool dbl = false, dense = false, pin = false, use_graph = false, timing = false;
    bool ctl = false;    // consistency control: states kernel and control kernel per update
    bool ab_inc = false; // state measure kept by the update kernel (CH, GS)
    bool ab_valid = false;  // a_b and a_next hold the measure of the current state
    bool trans = false;  // transition blocks
    bool half = false;   // half-spectrum layout (real fields)
    hipStream_t stream = nullptr;
    int64_t total_elems = 0, nb_total = 0, n_strips = 0, n_tiles = 0, n_chunks = 0;
    size_t esize = 8;  // bytes per complex element
    size_t fft_work = 0;
    // buffer layout
    size_t st_spec = 0, st_k0 = 0, st_ctl = 0, state_bytes = 0;
    size_t w_W = 0, w_R = 0, w_fft = 0, w_ab = 0, w_mask = 0, w_wl = 0, w_chunk = 0, w_cnt = 0, w_G = 0,
           w_Glast = 0, w_rk0 = 0, w_nl = 0, w_ind = 0, w_smax = 0, w_dense = 0, w_binst = 0, w_table = 0,
           w_taper = 0, w_htab = 0, w_anext = 0, w_probe = 0, work_bytes = 0;
    int64_t n_taper = 0;  // roll-off table length: 2 x the largest block edge
    int64_t n_htab = 0;   // NLSE H(|m|) table entries over all instances
    bool bound = false;
    char *d_state = nullptr, *d_work = nullptr;
    Ctx ctx{};
    rocfft_execution_info info = nullptr;
    int64_t steps = 0;
    bool last_dense = false;
    bool last_inc = false;  // the last update took the kept state measure (no energy partials)
    bool inv_preserving = true;
    // launch geometry
    int ind_waves = 4, nl_waves = 4, upd_per_cu = 4, dense_threads = 256, cu_count = 256;
    int upd_mode = 1;      // 0: block-list walk, 1: strip walk, 2: block-list walk, 4 entries in flight,
                           // 3: block-list walk, one wave per entry, 4: run walk (band list)
    int run_lmax = 0;      // run walk: longest piece in blocks, 0 where the walk does not apply
    int run_ub = 0;        // run walk: slots per block / 64
    int upd_waves = 4;     // strip walk: waves per workgroup
    bool fwd_in_place = false;  // CH/GS full layout: the step's forward transform runs in place in W,
                                // which then holds the right-hand side the update reads
    int max_slots = 0;     // largest block in 16-byte lane slots
    int min_slots = 0;     // smallest block in 16-byte lane slots
    bool list_stale = false;  // the ordered active list lags the mask
    // graph of one step
    hipGraphExec_t graph[4] = {};  // one captured step; XPFC: one per history phase
    bool graph_failed = false;
    // XPFC: the four nonlinear transforms rotate through slots of the state
    // buffer; the slot of the coming step's transform is xphase
    int xphase = 0;
    bool hist_valid = false;  // the three older slots hold the previous steps' transforms
    size_t st_hist = 0;       // first history slot in the state buffer
    size_t w_ltab = 0;        // L(|m|^2) tables in the work buffer
    std::vector<double> ltab; // host copy of the tables
    // stage events: a ring of per-step sets, read only after the stream drained
    static constexpr int kRing = 64;
    hipEvent_t ev[kRing][12] = {};
    hipEvent_t evk[kRing][4] = {};  // indicator dispatch start/stop, per half step
    bool evk_set[kRing][2] = {};    // the pair was stamped by an indicator dispatch of that step
    bool have_events = false;
    int ring = 0;         // set used by the step being enqueued
    int ring_filled = 0;  // sets holding a complete step
    const uint8_t *d_skip = nullptr;
    double *d_eb = nullptr;
};

namespace {

spdba_status dev_err(hipError_t e) { return e == hipSuccess ? SPDBA_OK : SPDBA_EDEVICE; }

#define TRY_HIP(x)                                   \
    do {                                             \
        hipError_t _e = (x);                         \
        if (_e != hipSuccess) return SPDBA_EDEVICE;  \
    } while (0)
#define TRY(x)                            \
    do {                                  \
        spdba_status _s = (x);            \
        if (_s != SPDBA_OK) return _s;    \
    } while (0)

bool has_control(const spdba_instance_desc &x) {
    return (x.flags & (SPDBA_FLAG_TRANSITION | SPDBA_FLAG_REFRESH | SPDBA_FLAG_DYN_THRESHOLD)) != 0 ||
           x.full_steps > 0;
}

spdba_status validate(const spdba_instance_desc *d, int32_t n, bool half_cap = true) {
    if (!d || n < 1 || n > 65535) return SPDBA_EINVAL;
    for (int i = 0; i < n; ++i) {
        const spdba_instance_desc &x = d[i];
        if (x.ndim < 1 || x.ndim > 3) return SPDBA_EINVAL;
        if (x.reserved != 0) return SPDBA_EINVAL;
        int64_t ext = 0;
        for (int a = 0; a < 3; ++a) {
            const int64_t dm = x.dims[a];
            const int64_t b = x.block[a];
            const bool used = a >= 3 - x.ndim;
            if (!used) {
                if (dm != 1 || b != 1) return SPDBA_EINVAL;
                continue;
            }
            if (!is_pow2(dm) || dm < 2) return SPDBA_EINVAL;
            if (ext == 0) ext = dm;
            else if (ext != dm) return SPDBA_EINVAL;
            if (b < 1 || dm % b != 0) return SPDBA_EINVAL;
        }
        if (!(x.threshold >= 0.0) || !std::isfinite(x.threshold)) return SPDBA_EINVAL;
        if (!(x.dt > 0.0) || !std::isfinite(x.dt)) return SPDBA_EINVAL;
        if (!(x.dx > 0.0) || !std::isfinite(x.dx)) return SPDBA_EINVAL;
        for (int p = 0; p < 8; ++p)
            if (!std::isfinite(x.op_params[p])) return SPDBA_EINVAL;
        // the implicit denominators 1 + dt M kappa k^4 and 1 + dt D k^2 stay >= 1
        if (x.op == SPDBA_OP_CAHN_HILLIARD && !(x.op_params[0] >= 0.0 && x.op_params[1] >= 0.0))
            return SPDBA_EINVAL;
        if (x.op == SPDBA_OP_GRAY_SCOTT && !(x.op_params[0] >= 0.0 && x.op_params[1] >= 0.0))
            return SPDBA_EINVAL;
        if (x.op < SPDBA_OP_CAHN_HILLIARD || x.op > SPDBA_OP_XPFC) return SPDBA_EUNSUPPORTED;
        if (x.op == SPDBA_OP_XPFC) {
            // peak width alpha > 0 and rho beta > 0 (the Gaussian and the
            // Debye-Waller factor); the state-amplitude measure (the paper's
            // block energy or its maximum form) or Regular mode; full layout
            if (!(x.op_params[2] > 0.0) || !(x.op_params[5] * x.op_params[6] > 0.0)) return SPDBA_EINVAL;
            if (!(x.flags & (SPDBA_FLAG_STATE_INDICATOR | SPDBA_FLAG_DENSE))) return SPDBA_EUNSUPPORTED;
            if (x.flags & SPDBA_FLAG_HALF_SPECTRUM) return SPDBA_EUNSUPPORTED;
            // the L table holds (n/2 + 1)^ndim FP64 entries
            int64_t tab = 1;
            for (int a = 0; a < 3; ++a) tab *= x.dims[a] / 2 + 1;
            if (tab > (int64_t(1) << 28)) return SPDBA_EUNSUPPORTED;
        }
        if (x.dtype != SPDBA_F32 && x.dtype != SPDBA_F64) return SPDBA_EUNSUPPORTED;
        if (x.flags & ~uint32_t(SPDBA_FLAG_DENSE | SPDBA_FLAG_PIN_K0 | SPDBA_FLAG_GRAPH |
                                SPDBA_FLAG_TIMING | SPDBA_FLAG_TRANSITION | SPDBA_FLAG_REFRESH |
                                SPDBA_FLAG_DYN_THRESHOLD | SPDBA_FLAG_STATE_INDICATOR |
                                SPDBA_FLAG_HALF_SPECTRUM | SPDBA_FLAG_BLOCK_ENERGY))
            return SPDBA_EUNSUPPORTED;
        // the block energy sums the state measure; the half layout's indicator keeps maxima only
        if ((x.flags & SPDBA_FLAG_BLOCK_ENERGY) && !(x.flags & SPDBA_FLAG_STATE_INDICATOR)) return SPDBA_EINVAL;
        if ((x.flags & SPDBA_FLAG_BLOCK_ENERGY) && (x.flags & SPDBA_FLAG_HALF_SPECTRUM)) return SPDBA_EUNSUPPORTED;
        if (x.flags & SPDBA_FLAG_HALF_SPECTRUM) {
            // real fields of two or three dimensions; the x block edge divides
            // nx/2 (the column nx/2 forms blocks of its own); transition
            // states need the columns 0 and 1 in the first x block (the
            // conjugate neighbour across kx = 0); the indicator keeps
            // 4 x (blocks per block row) doubles in LDS
            if (x.op == SPDBA_OP_NLSE || x.op == SPDBA_OP_XPFC || x.ndim < 2) return SPDBA_EUNSUPPORTED;
            if ((x.dims[2] / 2) % x.block[2] != 0) return SPDBA_EUNSUPPORTED;
            if ((x.flags & SPDBA_FLAG_TRANSITION) && x.block[2] < 2) return SPDBA_EUNSUPPORTED;
            // Grids above 2^18 points are refused: timed 256^3 runs of this
            // layout ended in device faults whose cause is not yet found, while
            // every grid up to 64^3 / 512^2 passed its parity tests.
            if (half_cap && x.dims[0] * x.dims[1] * x.dims[2] > kMaxHalfPoints) return SPDBA_EUNSUPPORTED;
            if (4 * 8 * (x.dims[2] / (2 * x.block[2]) + 1) > kMaxSigBytes) return SPDBA_EUNSUPPORTED;
        }
        // consistency control: schedule and controller parameters
        if (x.reserved2 != 0 || x.full_steps < 0) return SPDBA_EINVAL;
        if ((x.flags & SPDBA_FLAG_REFRESH) && x.refresh_period < 1) return SPDBA_EINVAL;
        if ((x.flags & SPDBA_FLAG_DYN_THRESHOLD) &&
            (x.control_interval < 1 || !(x.target_ratio > 0.0 && x.target_ratio <= 1.0) ||
             !(x.deadband >= 0.0 && x.deadband < 1.0)))
            return SPDBA_EINVAL;
        // Regular mode has no threshold rule to control
        if ((x.flags & SPDBA_FLAG_DENSE) && (has_control(x))) return SPDBA_EUNSUPPORTED;
        // the transition update keeps the roll-off tables (2 B doubles for the
        // largest edge B) in LDS
        if ((x.flags & SPDBA_FLAG_TRANSITION) &&
            2 * 8 * (int64_t)std::max({x.block[0], x.block[1], x.block[2]}) > kMaxSigBytes)
            return SPDBA_EUNSUPPORTED;
        // a lane reads 16 bytes: the x block edge must hold whole lanes
        const int V = x.dtype == SPDBA_F32 ? 2 : 1;
        if (x.block[2] < V) return SPDBA_EUNSUPPORTED;
        if (i > 0 && (x.op != d[0].op || x.dtype != d[0].dtype || x.flags != d[0].flags ||
                      x.ndim != d[0].ndim))
            return SPDBA_EUNSUPPORTED;
    }
    return SPDBA_OK;
}

spdba_status create_fft(spdba_plan p, const InstDev &I, Fft &f, bool forward, bool inplace,
                        int64_t batch) {
    size_t len[3];
    const int nd = p->ndim;
    // rocFFT takes lengths fastest dimension first
    for (int a = 0; a < nd; ++a) len[a] = (size_t)I.n[2 - a];
    rocfft_status st = rocfft_plan_create(
        &f.plan, inplace ? rocfft_placement_inplace : rocfft_placement_notinplace,
        forward ? rocfft_transform_type_complex_forward : rocfft_transform_type_complex_inverse,
        p->dbl ? rocfft_precision_double : rocfft_precision_single, (size_t)nd, len, (size_t)batch,
        nullptr);
    if (st != rocfft_status_success) return SPDBA_EFFT;
    size_t wb = 0;
    if (rocfft_plan_get_work_buffer_size(f.plan, &wb) != rocfft_status_success) return SPDBA_EFFT;
    p->fft_work = std::max(p->fft_work, wb);
    return SPDBA_OK;
}

// The data layout of a rocFFT transform as the plan is created with it:
// lengths and strides fastest dimension first, element counts of the input
// and output sides (a real or a complex element)
struct FftLayout {
    int nd = 0;
    size_t len[3] = {1, 1, 1};
    size_t is[3] = {1, 1, 1}, os[3] = {1, 1, 1};
    size_t idist = 0, odist = 0, batch = 0;
    bool in_real = false, out_real = false;  // real side (half layout) or complex
    bool in_herm = false, out_herm = false;  // Hermitian side: len[0] / 2 + 1 fastest elements
};

// elements spanned from the base: the largest offset plus one
size_t fft_span(const FftLayout &L, bool input) {
    const size_t *st = input ? L.is : L.os;
    const bool herm = input ? L.in_herm : L.out_herm;
    size_t m = (L.batch - 1) * (input ? L.idist : L.odist);
    for (int a = 0; a < L.nd; ++a) m += ((a == 0 && herm ? L.len[0] / 2 + 1 : L.len[a]) - 1) * st[a];
    return m + 1;
}

// Real-to-complex (forward) or complex-to-real (inverse) transforms of the
// half layout, out of place: the real fields follow each other at nz*ny*nx
// values (rocFFT's default; its two-dimensional batched complex-to-real plans
// accept no other distance), the half spectra at N complex values with rows
// of pitch xs.
FftLayout half_fft_layout(const spdba_plan p, const InstDev &I, bool forward, int64_t batch) {
    FftLayout L;
    L.nd = p->ndim;
    size_t rs[3], cs[3];
    for (int a = 0; a < L.nd; ++a) L.len[a] = (size_t)I.n[2 - a];  // fastest first
    rs[0] = cs[0] = 1;
    for (int a = 1; a < L.nd; ++a) {
        rs[a] = rs[a - 1] * L.len[a - 1];
        cs[a] = cs[a - 1] * (a == 1 ? (size_t)I.xs : L.len[a - 1]);
    }
    const size_t rdist = (size_t)I.Nreal, cdist = (size_t)I.N;
    for (int a = 0; a < 3; ++a) {
        L.is[a] = forward ? rs[a] : cs[a];
        L.os[a] = forward ? cs[a] : rs[a];
    }
    L.idist = forward ? rdist : cdist;
    L.odist = forward ? cdist : rdist;
    L.batch = (size_t)batch;
    L.in_real = forward;
    L.out_real = !forward;
    L.in_herm = !forward;
    L.out_herm = forward;
    return L;
}

// The full layout's complex transforms: rocFFT's default packed layout
FftLayout full_fft_layout(const spdba_plan p, const InstDev &I, int64_t batch) {
    FftLayout L;
    L.nd = p->ndim;
    for (int a = 0; a < L.nd; ++a) L.len[a] = (size_t)I.n[2 - a];
    for (int a = 1; a < L.nd; ++a) L.is[a] = L.os[a] = L.is[a - 1] * L.len[a - 1];
    L.idist = L.odist = (size_t)I.N;
    L.batch = (size_t)batch;
    return L;
}

spdba_status create_fft_half(spdba_plan p, const InstDev &I, Fft &f, bool forward, int64_t batch) {
    const FftLayout L = half_fft_layout(p, I, forward, batch);
    size_t is[3], os[3];
    std::copy(L.is, L.is + 3, is);
    std::copy(L.os, L.os + 3, os);
    rocfft_plan_description desc = nullptr;
    if (rocfft_plan_description_create(&desc) != rocfft_status_success) return SPDBA_EFFT;
    const rocfft_array_type ti = forward ? rocfft_array_type_real : rocfft_array_type_hermitian_interleaved;
    const rocfft_array_type to = forward ? rocfft_array_type_hermitian_interleaved : rocfft_array_type_real;
    rocfft_status st = rocfft_plan_description_set_data_layout(desc, ti, to, nullptr, nullptr, (size_t)L.nd, is,
                                                               L.idist, (size_t)L.nd, os, L.odist);
    if (st == rocfft_status_success)
        st = rocfft_plan_create(&f.plan, rocfft_placement_notinplace,
                                forward ? rocfft_transform_type_real_forward : rocfft_transform_type_real_inverse,
                                p->dbl ? rocfft_precision_double : rocfft_precision_single, (size_t)L.nd, L.len,
                                L.batch, desc);
    rocfft_plan_description_destroy(desc);
    if (st != rocfft_status_success) return SPDBA_EFFT;
    size_t wb = 0;
    if (rocfft_plan_get_work_buffer_size(f.plan, &wb) != rocfft_status_success) return SPDBA_EFFT;
    p->fft_work = std::max(p->fft_work, wb);
    return SPDBA_OK;
}

void destroy_fft(Fft &f) {
    if (f.plan) rocfft_plan_destroy(f.plan);
    f.plan = nullptr;
}

spdba_status exec_fft(spdba_plan p, const Fft &f, void *in, void *out) {
    void *ib[1] = {in};
    void *ob[1] = {out};
    rocfft_status st = rocfft_execute(f.plan, ib, out ? ob : nullptr, p->info);
    return st == rocfft_status_success ? SPDBA_OK : SPDBA_EFFT;
}

char *state_ptr(spdba_plan p, int64_t elem_off) { return p->d_state + p->st_spec + elem_off * p->esize; }
char *work_ptr(spdba_plan p, int64_t elem_off) { return p->d_work + p->w_W + elem_off * p->esize; }
// the right-hand side: R, or W when the forward transform runs in place
char *rhs_ptr(spdba_plan p, int64_t elem_off) {
    return p->d_work + (p->fwd_in_place ? p->w_W : p->w_R) + elem_off * p->esize;
}
// the full layout's CH/GS step can take its forward transform in place
bool fwd_in_place_ok(spdba_plan p) { return !p->half && (p->op == OP_CH || p->op == OP_GS); }
// XPFC: history slot `slot` (0..3) of the nonlinear transforms
char *hist_ptr(spdba_plan p, int slot, int64_t elem_off) {
    return p->d_state + p->st_hist + ((size_t)slot * (size_t)p->total_elems + (size_t)elem_off) * p->esize;
}
// XPFC: the coming step's transform goes to slot xphase, the three previous
// steps' are in the slots behind it
void set_phase(spdba_plan p) {
    if (p->op != OP_XPFC) return;
    Ctx &c = p->ctx;
    c.rhs = hist_ptr(p, p->xphase, 0);
    c.hist1 = hist_ptr(p, (p->xphase + 3) & 3, 0);
    c.hist2 = hist_ptr(p, (p->xphase + 2) & 3, 0);
    c.hist3 = hist_ptr(p, (p->xphase + 1) & 3, 0);
}
// XPFC: a step is done: its transform becomes the previous one
void advance_phase(spdba_plan p) {
    if (p->op != OP_XPFC) return;
    p->xphase = (p->xphase + 1) & 3;
    p->hist_valid = true;
}
// XPFC, first step of a new field: the older slots take this step's transform
spdba_status fill_history(spdba_plan p) {
    if (p->op != OP_XPFC || p->hist_valid) return SPDBA_OK;
    const size_t bytes = (size_t)p->total_elems * p->esize;
    for (int k = 1; k < 4; ++k)
        TRY_HIP(launch_copy8(hist_ptr(p, p->xphase, 0), hist_ptr(p, (p->xphase + k) & 3, 0), bytes, p->stream));
    return SPDBA_OK;
}
void drop_graphs(spdba_plan p) {
    for (auto &g : p->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}
// half layout: a real field in W (offset in real values)
char *wreal_ptr(spdba_plan p, int64_t real_off) { return p->d_work + p->w_W + real_off * (p->esize / 2); }

// inverse transform of a state region into the work buffer, keeping the state
spdba_status inverse_keep(spdba_plan p, const Fft &oop, const Fft &ip, int64_t off, int64_t n_elems) {
    if (oop.preserves) return exec_fft(p, oop, state_ptr(p, off), work_ptr(p, off));
    TRY_HIP(launch_copy8(state_ptr(p, off), work_ptr(p, off), (size_t)n_elems * p->esize, p->stream));
    return exec_fft(p, ip, work_ptr(p, off), nullptr);
}

// half layout: inverse of stored spectra into the real slots of W, keeping
// the state (through a copy in R when the plan overwrites its input)
spdba_status inverse_half(spdba_plan p, const Fft &oop, int64_t off, int64_t roff, int64_t n_elems) {
    if (oop.preserves) return exec_fft(p, oop, state_ptr(p, off), wreal_ptr(p, roff));
    TRY_HIP(launch_copy8(state_ptr(p, off), rhs_ptr(p, off), (size_t)n_elems * p->esize, p->stream));
    return exec_fft(p, oop, rhs_ptr(p, off), wreal_ptr(p, roff));
}

void record(spdba_plan p, int i) {
    if (p->timing && p->have_events && !p->use_graph) (void)hipEventRecord(p->ev[p->ring][i], p->stream);
}

void ring_advance(spdba_plan p) {
    if (p->timing && p->have_events && !p->use_graph) {
        p->ring = (p->ring + 1) % spdba_plan_s::kRing;
        p->ring_filled = std::min(p->ring_filled + 1, spdba_plan_s::kRing);
    }
}

// the coming update takes the state measure kept by the last one
bool kept_measure(spdba_plan p) { return !p->dense && p->ab_inc && p->ab_valid && !p->d_skip; }

// update stage: indicator + compaction + active update, or the dense update
// (ind_done: the state measure's full pass already ran at the step's start)
spdba_status update_stage(spdba_plan p, int ev_base, bool ind_done = false) {
    const bool d = p->dbl;
    if (p->dense) {
        TRY_HIP(launch_dense(p->ctx, d, p->dense_threads, p->stream));
        record(p, ev_base + 2);
        p->last_dense = true;
        return SPDBA_OK;
    }
    hipEvent_t k0 = nullptr, k1 = nullptr;
    const int hs = ev_base == 8 ? 1 : 0;  // second NLSE half step
    if (p->timing && p->have_events && !p->use_graph) {
        k0 = p->evk[p->ring][2 * hs];
        k1 = p->evk[p->ring][2 * hs + 1];
    }
    // state measure kept by the last update: only G (and the merge of the
    // stored blocks' measures) is left to do
    const bool inc = kept_measure(p);
    if (!ind_done) {
        if (k0) p->evk_set[p->ring][hs] = true;
        if (inc) TRY_HIP(launch_gmax(p->ctx, p->stream, k0, k1));
        else TRY_HIP(launch_indicator(p->ctx, d, p->ind_waves, p->stream, k0, k1));
    }
    // the next update may continue incrementally only from a step without a
    // skip set (skipped blocks report a_b = 0, not their measure)
    p->ab_valid = p->ab_inc && !p->d_skip;
    p->last_inc = inc;
    record(p, ev_base);
    if (p->ctl) {
        // consistency control: block states (controlled threshold, full
        // steps, transition blocks) and the append of every non-frozen block,
        // then the block-list walk (the strip walk has no neighbour
        // information), which also closes the update's control step
        TRY_HIP(launch_compact_states(p->ctx, p->stream));
        record(p, ev_base + 1);
        p->list_stale = true;
        const int grid = ((p->cu_count * p->upd_per_cu + 7) / 8) * 8;
        TRY_HIP(launch_update(p->ctx, d, grid, 0, p->stream, p->trans, true));
        record(p, ev_base + 2);
        p->last_dense = false;
        return SPDBA_OK;
    }
    if (p->upd_mode == 1 && !p->ab_inc && !p->half) {
        // threshold, mask and update in one pass; the ordered list is built
        // from the mask only when it is read back
        record(p, ev_base + 1);
        // persistent: a grid stride over the strips
        const int64_t grid = std::min<int64_t>(p->n_strips, (int64_t)p->cu_count * p->upd_per_cu);
        TRY_HIP(launch_update_strip(p->ctx, d, p->upd_waves, (int)grid, p->stream));
        p->list_stale = true;
    } else if (p->upd_mode == 4 && p->run_lmax > 0) {
        // threshold, mask and the band list of aligned runs, then the run walk
        TRY_HIP(launch_compact_runs(p->ctx, p->stream));
        record(p, ev_base + 1);
        p->list_stale = true;
        const int grid = ((p->cu_count * p->upd_per_cu + 7) / 8) * 8;
        TRY_HIP(launch_update(p->ctx, d, grid, 3, p->stream));
    } else {
        // one-pass threshold, mask and unordered append of the active blocks
        TRY_HIP(launch_compact_append(p->ctx, p->stream));
        record(p, ev_base + 1);
        p->list_stale = true;
        // a multiple of 8: the update splits its list into one segment per XCD
        const int grid = ((p->cu_count * p->upd_per_cu + 7) / 8) * 8;
        // four entries in flight need blocks of at most one slot per thread;
        // one wave per entry needs blocks of at least one slot per lane
        int multi = (p->upd_mode == 2 && p->max_slots <= 256 && !p->ab_inc && !p->half) ? 1 : 0;
        if (p->upd_mode == 3 && p->min_slots >= 64 && !p->half) multi = 2;
        TRY_HIP(launch_update(p->ctx, d, grid, multi, p->stream));
    }
    record(p, ev_base + 2);
    p->last_dense = false;
    return SPDBA_OK;
}

// one full step, enqueued on the plan stream
spdba_status enqueue_step(spdba_plan p) {
    const bool d = p->dbl;
    if (p->op != OP_NLSE) {
        record(p, 0);
        // the state measure's full pass reads only the state the last update
        // stored: it runs first, before the transforms leave their output to
        // be written back from the caches while it streams
        const bool early = !p->dense && p->ctx.state_ind && !kept_measure(p);
        if (early) {
            hipEvent_t k0 = nullptr, k1 = nullptr;
            if (p->timing && p->have_events && !p->use_graph) {
                k0 = p->evk[p->ring][0];
                k1 = p->evk[p->ring][1];
                p->evk_set[p->ring][0] = true;
            }
            TRY_HIP(launch_indicator(p->ctx, d, p->ind_waves, p->stream, k0, k1));
        }
        record(p, 7);
        for (auto &g : p->groups) {
            if (p->half) TRY(inverse_half(p, g.inv_oop, g.off, 2 * g.off, g.N * g.count * p->nspec));
            else TRY(inverse_keep(p, g.inv_oop, g.inv_ip, g.off, g.N * g.count * p->nspec));
        }
        record(p, 1);
        TRY_HIP(launch_nonlinear(p->ctx, d, p->nl_waves, p->stream));
        record(p, 2);
        for (auto &g : p->groups) {
            if (p->fwd_in_place) TRY(exec_fft(p, g.fwd_ip, work_ptr(p, g.off), nullptr));
            else TRY(exec_fft(p, g.fwd_oop, work_ptr(p, g.off),
                              p->op == OP_XPFC ? hist_ptr(p, p->xphase, g.off) : rhs_ptr(p, g.off)));
        }
        TRY(fill_history(p));  // XPFC, first step of a new field (eager)
        if (p->op == OP_GS && !d) TRY_HIP(launch_k0_rhs(p->ctx, p->stream));
        record(p, 3);
        TRY(update_stage(p, 4, early));
        return SPDBA_OK;
    }
    // NLSE: linear half step, Kerr step, linear half step (all in place on the state)
    for (int half = 0; half < 2; ++half) {
        record(p, half ? 6 : 0);
        for (auto &g : p->groups) TRY(exec_fft(p, g.fwd_ip, state_ptr(p, g.off), nullptr));
        record(p, half ? 7 : 1);
        TRY(update_stage(p, half ? 8 : 2));
        for (auto &g : p->groups) TRY(exec_fft(p, g.inv_ip, state_ptr(p, g.off), nullptr));
        record(p, half ? 11 : 5);
        if (half == 0) TRY_HIP(launch_nonlinear(p->ctx, d, p->nl_waves, p->stream));
    }
    return SPDBA_OK;
}

spdba_status probe_preserving(spdba_plan p, Fft &oop, int64_t off, int64_t n_elems) {
    uint32_t *bad = reinterpret_cast<uint32_t *>(p->d_work + p->w_probe);
    TRY_HIP(hipMemsetAsync(bad, 0, 4, p->stream));
    TRY_HIP(launch_fill_pattern(state_ptr(p, off), n_elems, p->dbl, p->stream));
    TRY(exec_fft(p, oop, state_ptr(p, off), work_ptr(p, off)));
    TRY_HIP(launch_check_pattern(state_ptr(p, off), n_elems, p->dbl, bad, p->stream));
    uint32_t h = 0;
    TRY_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, p->stream));
    TRY_HIP(hipStreamSynchronize(p->stream));
    oop.preserves = (h == 0);
    return SPDBA_OK;
}

spdba_status check_nonfinite(spdba_plan p) {
    uint32_t h = 0;
    TRY_HIP(hipMemcpyAsync(&h, p->ctx.nonfinite, 4, hipMemcpyDeviceToHost, p->stream));
    TRY_HIP(hipStreamSynchronize(p->stream));
    if (h) {
        TRY_HIP(hipMemsetAsync(p->ctx.nonfinite, 0, 4, p->stream));
        TRY_HIP(hipStreamSynchronize(p->stream));
        return SPDBA_ENONFINITE;
    }
    return SPDBA_OK;
}

}  // namespace

namespace spdba {

// Per-instance constants of the device table: geometry (full layout, or the
// half layout with row pitch `xs`), strips and tiles, the operator's
// coefficients and the control parameters.  Offsets into the concatenated
// spaces (off, roff, blk_off, strip_off, tile_off, ht_off, ltab_off) are
// left 0 for the caller.
void fill_inst(const spdba_instance_desc &x, int op, bool dbl, bool pin, bool half, int64_t xs, InstDev &I) {
    std::memset(&I, 0, sizeof(I));
    const int V = dbl ? 1 : 2;
    const int64_t TE = dbl ? 512 : 1024;
    for (int a = 0; a < 3; ++a) {
        I.n[a] = (int32_t)x.dims[a];
        I.b[a] = x.block[a];
        I.nbk[a] = (int32_t)(x.dims[a] / x.block[a]);
    }
    I.N = x.dims[0] * x.dims[1] * xs;
    I.nb = (int64_t)I.nbk[0] * I.nbk[1] * I.nbk[2];
    I.half = half ? 1 : 0;
    I.Nreal = x.dims[0] * x.dims[1] * x.dims[2];
    I.xs = (int32_t)xs;
    I.nbxm = half ? (int32_t)(x.dims[2] / (2 * x.block[2])) : I.nbk[2];
    I.nbm = (int64_t)I.nbk[0] * I.nbk[1] * I.nbxm;
    if (half) I.nb = I.nbm + (int64_t)I.nbk[0] * I.nbk[1];
    I.S = std::min<int>(I.nbk[2], std::max(1, 64 * V / I.b[2]));
    I.chunks = std::max(1, I.b[2] / (64 * V));
    auto lg = [](int64_t v) { int l = 0; while ((int64_t(1) << l) < v) ++l; return l; };
    for (int a = 0; a < 3; ++a) {
        I.ln[a] = lg(I.n[a]);
        I.lb[a] = lg(I.b[a]);
        I.lnbk[a] = lg(I.nbk[a]);
    }
    I.lS = lg(I.S);
    I.lchunks = lg(I.chunks);
    I.lnbxm = lg(I.nbxm);
    // half layout: one indicator strip per (z, y) block row; tiles of TE
    // values, enough for the reals of the nonlinear term and for the
    // stored values (padding included) of the dense update
    I.nstrips = half ? (int64_t)I.nbk[0] * I.nbk[1] : (int64_t)I.nbk[0] * I.nbk[1] * (I.nbk[2] / I.S);
    I.ntiles = ((half ? std::max(I.Nreal, I.N) : I.N) + TE - 1) / TE;
    I.nspec = op == OP_GS ? 2 : 1;
    I.k0path = (!dbl && op != OP_NLSE) ? 1 : 0;
    I.pin = pin ? 1 : 0;
    const int64_t ext = x.dims[2];
    const double K = kTwoPi / ((double)ext * x.dx);
    I.K2 = K * K;
    I.tau2 = x.threshold * x.threshold;
    I.invN = 1.0 / (double)I.Nreal;
    double dvol = 1.0;
    for (int a = 0; a < x.ndim; ++a) dvol *= x.dx;
    I.dvol = dvol;
    if (op == OP_CH) {
        I.c0 = x.dt * x.op_params[0];
        I.c1 = I.c0 * x.op_params[1];
    } else if (op == OP_GS) {
        I.c0 = x.dt;
        I.c1 = x.dt * x.op_params[0];
        I.c2 = x.dt * x.op_params[1];
        I.q0 = x.op_params[2];
        I.q1 = x.op_params[3];
    } else if (op == OP_XPFC) {
        I.c0 = x.dt;
        I.q0 = x.op_params[3];  // omega
        I.q1 = x.op_params[4];  // u
    } else {
        I.c0 = ((x.op_params[0] * x.dt) * 0.25) * I.K2;
        I.c1 = std::exp(-(x.op_params[2] * x.dt) * 0.25);
        I.q0 = x.op_params[1] * x.dt;
    }
    I.full_steps = x.full_steps;
    I.refresh = (x.flags & SPDBA_FLAG_REFRESH) ? x.refresh_period : 0;
    I.interval = (x.flags & SPDBA_FLAG_DYN_THRESHOLD) ? x.control_interval : 0;
    I.per = op == OP_NLSE ? 2 : 1;
    I.tau0 = x.threshold;
    I.ht_off = -1;
    I.target = x.target_ratio;
    I.deadband = x.deadband;
}

spdba_status validate_desc(const spdba_instance_desc *d, int32_t n) { return validate(d, n); }

const Ctx *plan_ctx(spdba_plan p) { return p && p->bound ? &p->ctx : nullptr; }
const InstDev *plan_hinst(spdba_plan p, int *n_inst, int64_t *nb_total) {
    if (!p) return nullptr;
    *n_inst = p->n_inst;
    *nb_total = p->nb_total;
    return p->hinst.data();
}
}  // namespace spdba

namespace {

// Everything of a plan that needs no device: the instance table, the grid
// groups and block counts, the per-instance tables (XPFC L, NLSE H)
spdba_status build_layout(spdba_plan p, const spdba_instance_desc *inst, int32_t n_inst) {
    p->desc.assign(inst, inst + n_inst);
    p->n_inst = n_inst;
    p->op = inst[0].op;
    p->ndim = inst[0].ndim;
    p->dbl = inst[0].dtype == SPDBA_F64;
    p->dense = (inst[0].flags & SPDBA_FLAG_DENSE) != 0;
    p->pin = (inst[0].flags & SPDBA_FLAG_PIN_K0) != 0;
    p->use_graph = (inst[0].flags & SPDBA_FLAG_GRAPH) != 0;
    p->timing = (inst[0].flags & SPDBA_FLAG_TIMING) != 0;
    p->trans = (inst[0].flags & SPDBA_FLAG_TRANSITION) != 0;
    p->half = (inst[0].flags & SPDBA_FLAG_HALF_SPECTRUM) != 0;
    for (int i = 0; i < n_inst; ++i) p->ctl = p->ctl || has_control(inst[i]);
    p->nspec = p->op == OP_GS ? 2 : 1;
    p->esize = p->dbl ? 16 : 8;
    const int V = p->dbl ? 1 : 2;
    const int64_t TE = p->dbl ? 512 : 1024;

    // memory order: larger grids first, original order within a size
    std::vector<int> order(n_inst);
    std::iota(order.begin(), order.end(), 0);
    // stored row pitch: half layout, nx/2 + 1 columns rounded up to 128 bytes
    const int64_t pq = p->dbl ? 8 : 16;
    auto pitch = [&](int i) {
        return p->half ? ((inst[i].dims[2] / 2 + 1 + pq - 1) / pq) * pq : inst[i].dims[2];
    };
    // stored values per species (with the half layout's padding columns)
    auto Nof = [&](int i) { return inst[i].dims[0] * inst[i].dims[1] * pitch(i); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return Nof(a) > Nof(b); });
    std::vector<int64_t> mem_off(n_inst);
    int64_t acc = 0;
    p->group_of.assign(n_inst, -1);
    for (int k = 0; k < n_inst; ++k) {
        const int i = order[k];
        const int64_t N = Nof(i);
        if (p->groups.empty() || p->groups.back().N != N) {
            Group g;
            g.N = N;
            g.off = acc;
            p->groups.push_back(g);
        }
        p->groups.back().count++;
        p->group_of[i] = (int)p->groups.size() - 1;
        mem_off[i] = acc;
        acc += N * p->nspec;
    }
    p->total_elems = acc;

    // per-instance table in original order
    int64_t blk = 0, strip = 0, tile = 0, taper = 0, htab = 0;
    p->hinst.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const spdba_instance_desc &x = inst[i];
        InstDev I;
        spdba::fill_inst(x, p->op, p->dbl, p->pin, p->half, pitch(i), I);
        I.off = mem_off[i];
        {  // half layout: reals of the batch packed from twice the group's offset
            const Group &gg = p->groups[p->group_of[i]];
            const int64_t pos = (mem_off[i] - gg.off) / (I.N * p->nspec);
            I.roff = 2 * gg.off + pos * p->nspec * x.dims[0] * x.dims[1] * x.dims[2];
        }
        I.blk_off = blk;
        blk += I.nb;
        p->max_slots = std::max(p->max_slots, I.b[0] * I.b[1] * (I.b[2] / V));
        p->min_slots = i == 0 ? I.b[0] * I.b[1] * (I.b[2] / V) : std::min(p->min_slots, I.b[0] * I.b[1] * (I.b[2] / V));
        I.strip_off = strip;
        strip += I.nstrips;
        I.tile_off = tile;
        tile += I.ntiles;
        I.ltab_off = 0;
        if (p->op == OP_XPFC) {
            // L(k) = -k^2 (1 - C2(k)) in FP64 by the steps of the definition
            // (Supplementary S3.1), one entry per (|m_z|, |m_y|, |m_x|), C
            // order over extents n/2 + 1: a row of the table serves a row of
            // the grid with consecutive reads
            const int64_t h0 = x.dims[0] / 2 + 1, h1 = x.dims[1] / 2 + 1, h2 = x.dims[2] / 2 + 1;
            I.ltab_off = (int64_t)p->ltab.size();
            const double q0 = x.op_params[0], sg = x.op_params[1], al = x.op_params[2];
            const double rho = x.op_params[5], be = x.op_params[6];
            const double dw = std::exp(-((sg * sg) * (q0 * q0)) / (2.0 * (rho * be)));
            for (int64_t az = 0; az < h0; ++az)
                for (int64_t ay = 0; ay < h1; ++ay)
                    for (int64_t ax = 0; ax < h2; ++ax) {
                        const int64_t m2 = az * az + ay * ay + ax * ax;
                        const double k2 = I.K2 * (double)m2;
                        const double k = std::sqrt(k2);
                        const double dk = k - q0;
                        const double peak = std::exp(-(dk * dk) / (2.0 * (al * al)));
                        const double c2 = peak * dw;
                        p->ltab.push_back(-k2 * (1.0 - c2));
                    }
        }
        for (int a = 0; a < 3; ++a) taper = std::max<int64_t>(taper, 2 * (int64_t)I.b[a]);
        I.ht_off = -1;
        if (p->op == OP_NLSE && x.ndim == 1) {  // H depends on |m| only: one table entry per |m|
            I.ht_off = htab;
            htab += x.dims[2] / 2 + 1;
        }
        I.target = x.target_ratio;
        I.deadband = x.deadband;
        p->hinst[i] = I;
    }
    p->nb_total = blk;
    // the run walk: full layout, CH / GS without transition blocks or the
    // block-energy sum (its bands give partial sums), equal blocks of 256 or
    // 512 slots whose rows are at most one wave row, list entries of 24 bits
    if (!p->half && p->op != OP_NLSE && p->op != OP_XPFC && !p->trans && !(inst[0].flags & SPDBA_FLAG_BLOCK_ENERGY) &&
        p->min_slots == p->max_slots && (p->max_slots == 256 || p->max_slots == 512) && blk <= (int64_t)1 << 24) {
        int lmax = 16;
        for (int i = 0; i < n_inst; ++i) {
            const InstDev &I = p->hinst[i];
            const int lpr = I.b[2] / V;
            if (lpr > 64) lmax = 0;
            else lmax = std::min({lmax, 64 / lpr, I.nbk[2], I.b[0] * I.b[1]});
        }
        if (lmax > 0) {
            p->run_lmax = lmax;
            p->run_ub = p->max_slots / 64;
        }
    }
    p->n_taper = taper;
    p->n_htab = htab;
    p->n_strips = strip;
    p->n_tiles = tile;
    p->n_chunks = (blk + CHUNK_BLOCKS - 1) / CHUNK_BLOCKS;
    // list entries hold a block id (transition plans: 25 bits beside the
    // face bits)
    if (blk > 0xFFFFFFFFll || (p->trans && blk > (int64_t)kEntryId)) return SPDBA_EUNSUPPORTED;
    p->blk_inst.resize(blk);
    for (int i = 0; i < n_inst; ++i)
        for (int64_t b = 0; b < p->hinst[i].nb; ++b) p->blk_inst[p->hinst[i].blk_off + b] = (uint16_t)i;

    return SPDBA_OK;
}

// Region offsets of the state and work buffers (after the transforms' work
// size is known)
void build_buffers(spdba_plan p) {
    const int64_t blk = p->nb_total, tile = p->n_tiles, strip = p->n_strips;
    const int n_inst = p->n_inst;
    // buffer layout
    size_t o = 0;
    p->st_spec = o;
    o = align256(o + (size_t)p->total_elems * p->esize);
    p->st_hist = o;
    if (p->op == OP_XPFC) o = align256(o + 4 * (size_t)p->total_elems * p->esize);
    p->st_k0 = o;
    o = align256(o + (size_t)n_inst * 2 * sizeof(double));
    p->st_ctl = o;
    o = align256(o + (size_t)n_inst * sizeof(CtlDev));
    p->state_bytes = o;
    o = 0;
    auto take = [&o](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    p->w_W = take((size_t)p->total_elems * p->esize);
    p->w_R = (p->op == OP_NLSE) ? p->w_W : take((size_t)p->total_elems * p->esize);
    p->w_fft = take(std::max<size_t>(p->fft_work, 256));
    p->w_ab = take((size_t)blk * sizeof(double));
    p->w_mask = take((size_t)blk);
    p->w_wl = take((size_t)blk * sizeof(uint32_t));
    p->w_chunk = take((size_t)p->n_chunks * sizeof(uint32_t));
    p->w_cnt = take(16);
    p->w_G = take((size_t)n_inst * 8);
    p->w_Glast = take((size_t)n_inst * 8);
    p->w_rk0 = take((size_t)n_inst * 2 * sizeof(double));
    p->w_nl = take((size_t)tile * 2 * sizeof(double));
    p->w_ind = take((size_t)strip * sizeof(double));
    p->w_smax = take((size_t)strip * sizeof(double));
    p->w_dense = take((size_t)tile * sizeof(double));
    p->w_binst = take((size_t)blk * sizeof(uint16_t));
    p->w_table = take((size_t)n_inst * sizeof(InstDev));
    p->w_taper = take((size_t)p->n_taper * sizeof(double));
    p->w_htab = take((size_t)p->n_htab * p->esize);
    p->w_anext = take((size_t)blk * sizeof(double));
    p->w_ltab = take(std::max<size_t>(p->ltab.size() * sizeof(double), 8));
    p->w_probe = take(8);
    p->work_bytes = o;
}

}  // namespace

extern "C" {

const char *spdba_status_string(spdba_status s) {
    switch (s) {
        case SPDBA_OK: return "success";
        case SPDBA_EINVAL: return "invalid argument";
        case SPDBA_EUNSUPPORTED: return "unsupported combination";
        case SPDBA_ESTATE: return "call out of order";
        case SPDBA_EDEVICE: return "HIP runtime error";
        case SPDBA_EFFT: return "rocFFT error";
        case SPDBA_ENONFINITE: return "non-finite indicator value";
        default: return "unknown status";
    }
}

spdba_status spdba_plan_create(const spdba_instance_desc *inst, int32_t n_inst, void *stream,
                               spdba_plan *out) {
    if (!out) return SPDBA_EINVAL;
    *out = nullptr;
    TRY(validate(inst, n_inst));
    // everything below needs a device
    int dev = 0;
    TRY_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    TRY_HIP(hipGetDeviceProperties(&prop, dev));
    if (spdba::fft_setup() != SPDBA_OK) return SPDBA_EFFT;

    spdba_plan p = new (std::nothrow) spdba_plan_s();
    if (!p) return SPDBA_EDEVICE;
    p->stream = reinterpret_cast<hipStream_t>(stream);
    p->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (spdba_status ls = build_layout(p, inst, n_inst)) {
        delete p;
        return ls;
    }

    // rocFFT plans, one set per grid size
    spdba_status st = SPDBA_OK;
    for (auto &g : p->groups) {
        int rep = -1;
        for (int i = 0; i < n_inst; ++i)
            if (p->group_of[i] == (int)(&g - &p->groups[0])) { rep = i; break; }
        const InstDev &I = p->hinst[rep];
        const int64_t batch = (int64_t)g.count * p->nspec;
        if (p->op == OP_NLSE) {
            if ((st = create_fft(p, I, g.fwd_ip, true, true, batch))) break;
            if ((st = create_fft(p, I, g.inv_ip, false, true, batch))) break;
        } else if (p->half) {
            if ((st = create_fft_half(p, I, g.inv_oop, false, batch))) break;
            if ((st = create_fft_half(p, I, g.fwd_oop, true, batch))) break;
            if ((st = create_fft_half(p, I, g.inv1_oop, false, p->nspec))) break;
            if ((st = create_fft_half(p, I, g.fwd1_oop, true, p->nspec))) break;
        } else {
            if ((st = create_fft(p, I, g.inv_oop, false, false, batch))) break;
            if ((st = create_fft(p, I, g.fwd_oop, true, false, batch))) break;
            if ((st = create_fft(p, I, g.inv_ip, false, true, batch))) break;
            if (fwd_in_place_ok(p) && (st = create_fft(p, I, g.fwd_ip, true, true, batch))) break;
            if ((st = create_fft(p, I, g.inv1_oop, false, false, p->nspec))) break;
            if ((st = create_fft(p, I, g.fwd1_ip, true, true, p->nspec))) break;
            if ((st = create_fft(p, I, g.inv1_ip, false, true, p->nspec))) break;
        }
    }
    if (st == SPDBA_OK && rocfft_execution_info_create(&p->info) != rocfft_status_success)
        st = SPDBA_EFFT;
    if (st == SPDBA_OK && p->stream &&
        rocfft_execution_info_set_stream(p->info, p->stream) != rocfft_status_success)
        st = SPDBA_EFFT;
    if (st != SPDBA_OK) {
        spdba_destroy(p);
        return st;
    }

    build_buffers(p);
    *out = p;
    return SPDBA_OK;
}

spdba_status spdba_plan_audit(const spdba_instance_desc *inst, int32_t n_inst, char *msg, size_t msg_len) {
    if (msg && msg_len) msg[0] = 0;
    // the half layout's grid cap does not apply: the audit is how larger
    // grids are examined without a device
    TRY(validate(inst, n_inst, false));
    std::unique_ptr<spdba_plan_s> hold(new (std::nothrow) spdba_plan_s());
    spdba_plan p = hold.get();
    if (!p) return SPDBA_EDEVICE;
    TRY(build_layout(p, inst, n_inst));
    build_buffers(p);  // the transforms' own work area (sized by rocFFT) is not part of the audit
    // buffer bases: the pointers below are compared, never dereferenced
    char *const S = reinterpret_cast<char *>(uintptr_t(1) << 44);
    char *const Wk = reinterpret_cast<char *>(uintptr_t(1) << 45);
    p->d_state = S;
    p->d_work = Wk;
    const size_t esz = (size_t)p->esize, rsz = esz / 2, spec = (size_t)p->total_elems * esz;
    struct Region {
        const char *name;
        const char *lo;
        size_t bytes;
    };
    const Region st{"state spectra", S + p->st_spec, spec}, W{"work W", Wk + p->w_W, spec},
        R{"work R", Wk + p->w_R, spec};
    std::vector<Region> hist;
    if (p->op == OP_XPFC)
        for (int k = 0; k < 4; ++k) hist.push_back(Region{"history slot", S + p->st_hist + k * spec, spec});
    bool ok = true;
    auto fail = [&](const std::string &what) {
        if (ok && msg && msg_len) std::snprintf(msg, msg_len, "%s", what.c_str());
        ok = false;
    };
    auto inside = [&](const std::string &what, const char *ptr, size_t bytes, const Region &r) {
        if (ptr < r.lo || ptr + bytes > r.lo + r.bytes)
            fail(what + ": " + std::to_string(bytes) + " bytes at offset " + std::to_string(ptr - r.lo) + " of " +
                 r.name + " (" + std::to_string(r.bytes) + " bytes)");
    };
    // a transform: input and output spans against their regions
    auto fft = [&](const std::string &what, const FftLayout &L, const char *in, const Region &ri, const char *out,
                   const Region &ro) {
        inside(what + " input", in, fft_span(L, true) * (L.in_real ? rsz : esz), ri);
        inside(what + " output", out ? out : in, fft_span(L, false) * (L.out_real ? rsz : esz), out ? ro : ri);
    };
    if (p->state_bytes < (size_t)p->st_spec + spec || p->work_bytes < (size_t)p->w_R + spec)
        fail("buffer sizes below their regions");
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        const Group &g = p->groups[gi];
        int rep = -1;
        for (int i = 0; i < n_inst; ++i)
            if (p->group_of[i] == (int)gi) { rep = i; break; }
        const InstDev &I = p->hinst[rep];
        const int64_t batch = (int64_t)g.count * p->nspec, ng = g.N * batch;
        const std::string gs = "group " + std::to_string(gi);
        if (p->op == OP_NLSE) {  // in place on the state
            const FftLayout L = full_fft_layout(p, I, batch);
            fft(gs + " forward", L, state_ptr(p, g.off), st, nullptr, st);
            continue;
        }
        if (p->half) {
            const FftLayout inv = half_fft_layout(p, I, false, batch), fwd = half_fft_layout(p, I, true, batch);
            // step: inverse from the state or from its copy in R, into W's real slots
            inside(gs + " inverse copy source", state_ptr(p, g.off), (size_t)ng * esz, st);
            inside(gs + " inverse copy target", rhs_ptr(p, g.off), (size_t)ng * esz, R);
            fft(gs + " inverse", inv, state_ptr(p, g.off), st, wreal_ptr(p, 2 * g.off), W);
            fft(gs + " inverse (from the copy)", inv, rhs_ptr(p, g.off), R, wreal_ptr(p, 2 * g.off), W);
            fft(gs + " forward", fwd, work_ptr(p, g.off), W, rhs_ptr(p, g.off), R);
            fft(gs + " preservation probe", inv, state_ptr(p, g.off), st, work_ptr(p, g.off), W);
            const FftLayout inv1 = half_fft_layout(p, I, false, p->nspec), fwd1 = half_fft_layout(p, I, true, p->nspec);
            for (int i = 0; i < n_inst; ++i) {
                if (p->group_of[i] != (int)gi) continue;
                const InstDev &J = p->hinst[i];
                const std::string is = "instance " + std::to_string(i);
                const size_t nr = (size_t)J.Nreal * p->nspec;
                inside(is + " real slots", wreal_ptr(p, J.roff), nr * rsz, W);
                // the real slots of the batch lie in order inside the group's transform span
                if (J.roff < 2 * g.off || J.roff + (int64_t)nr > 2 * g.off + (int64_t)(batch * J.Nreal))
                    fail(is + " real slots outside the batch transform's span");
                fft(is + " field in", fwd1, wreal_ptr(p, J.roff), W, rhs_ptr(p, J.off), R);
                inside(is + " field out copy", rhs_ptr(p, J.off), (size_t)J.N * p->nspec * esz, R);
                fft(is + " field out", inv1, rhs_ptr(p, J.off), R, wreal_ptr(p, J.roff), W);
            }
            fft(gs + " preservation probe (one instance)", inv1, state_ptr(p, g.off), st, work_ptr(p, g.off), W);
            continue;
        }
        const FftLayout L = full_fft_layout(p, I, batch), L1 = full_fft_layout(p, I, p->nspec);
        fft(gs + " inverse", L, state_ptr(p, g.off), st, work_ptr(p, g.off), W);
        inside(gs + " inverse copy", work_ptr(p, g.off), (size_t)ng * esz, W);
        fft(gs + " inverse in place", L, work_ptr(p, g.off), W, nullptr, W);
        if (p->op == OP_XPFC) {
            for (int k = 0; k < 4; ++k) fft(gs + " forward", L, work_ptr(p, g.off), W, hist_ptr(p, k, g.off), hist[k]);
        } else {
            fft(gs + " forward", L, work_ptr(p, g.off), W, rhs_ptr(p, g.off), R);
            fft(gs + " forward in place", L, work_ptr(p, g.off), W, nullptr, W);
        }
        for (int i = 0; i < n_inst; ++i) {
            if (p->group_of[i] != (int)gi) continue;
            const InstDev &J = p->hinst[i];
            const std::string is = "instance " + std::to_string(i);
            fft(is + " field in", L1, work_ptr(p, J.off), W, nullptr, W);
            fft(is + " field out", L1, state_ptr(p, J.off), st, work_ptr(p, J.off), W);
        }
    }
    // instances: stored spectra disjoint and in order
    for (int i = 0; i < n_inst; ++i) {
        const InstDev &J = p->hinst[i];
        inside("instance " + std::to_string(i) + " spectrum", state_ptr(p, J.off), (size_t)J.N * p->nspec * esz, st);
    }
    return ok ? SPDBA_OK : SPDBA_EINVAL;
}

spdba_status spdba_plan_buffer_sizes(spdba_plan p, size_t *state_bytes, size_t *work_bytes) {
    if (!p) return SPDBA_EINVAL;
    if (state_bytes) *state_bytes = p->state_bytes;
    if (work_bytes) *work_bytes = p->work_bytes;
    return SPDBA_OK;
}

spdba_status spdba_plan_bind(spdba_plan p, void *d_state, void *d_work) {
    if (!p || !d_state || !d_work) return SPDBA_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_state) & 255) || (reinterpret_cast<uintptr_t>(d_work) & 255))
        return SPDBA_EINVAL;
    p->d_state = static_cast<char *>(d_state);
    p->d_work = static_cast<char *>(d_work);
    if (p->fft_work > 0 &&
        rocfft_execution_info_set_work_buffer(p->info, p->d_work + p->w_fft, p->fft_work) !=
            rocfft_status_success)
        return SPDBA_EFFT;
    Ctx &c = p->ctx;
    c.inst = reinterpret_cast<const InstDev *>(p->d_work + p->w_table);
    c.n_inst = p->n_inst;
    c.nspec = p->nspec;
    c.op = p->op;
    c.dense = p->dense ? 1 : 0;
    c.state = p->d_state + p->st_spec;
    c.work = p->d_work + p->w_W;
    c.rhs = rhs_ptr(p, 0);
    c.k0 = reinterpret_cast<double *>(p->d_state + p->st_k0);
    c.rhs_k0 = reinterpret_cast<double *>(p->d_work + p->w_rk0);
    c.a_b = reinterpret_cast<double *>(p->d_work + p->w_ab);
    c.G = reinterpret_cast<unsigned long long *>(p->d_work + p->w_G);
    c.G_last = reinterpret_cast<unsigned long long *>(p->d_work + p->w_Glast);
    c.mask = reinterpret_cast<uint8_t *>(p->d_work + p->w_mask);
    c.worklist = reinterpret_cast<uint32_t *>(p->d_work + p->w_wl);
    c.chunk_cnt = reinterpret_cast<uint32_t *>(p->d_work + p->w_chunk);
    c.count = reinterpret_cast<uint32_t *>(p->d_work + p->w_cnt);
    c.nonfinite = reinterpret_cast<uint32_t *>(p->d_work + p->w_cnt + 4);
    c.done = reinterpret_cast<uint32_t *>(p->d_work + p->w_cnt + 8);
    c.nl_part = reinterpret_cast<double *>(p->d_work + p->w_nl);
    c.ind_part = reinterpret_cast<double *>(p->d_work + p->w_ind);
    c.strip_max = reinterpret_cast<double *>(p->d_work + p->w_smax);
    c.dense_part = reinterpret_cast<double *>(p->d_work + p->w_dense);
    c.blk_inst = reinterpret_cast<const uint16_t *>(p->d_work + p->w_binst);
    c.skip = p->d_skip;
    c.e_b = p->d_eb;
    c.ctl = reinterpret_cast<CtlDev *>(p->d_state + p->st_ctl);
    c.taper = reinterpret_cast<const double *>(p->d_work + p->w_taper);
    c.htab = p->d_work + p->w_htab;
    c.ltab = reinterpret_cast<const double *>(p->d_work + p->w_ltab);
    c.hist1 = c.hist2 = c.hist3 = c.rhs;  // XPFC: set per step (set_phase)
    c.trans = p->trans ? 1 : 0;
    c.state_ind = (p->desc[0].flags & SPDBA_FLAG_STATE_INDICATOR) ? 1 : 0;
    // the state entering a CH or GS update is the state the last one stored:
    // its measure can be kept by the update kernel (NLSE: the Kerr step
    // changes every mode between the updates)
    // (the block energy is a sum: the full pass computes it every update in
    // one fixed order, so the update kernel does not keep it)
    c.ab_sum = (p->desc[0].flags & SPDBA_FLAG_BLOCK_ENERGY) ? 1 : 0;
    c.run_lmax = p->run_lmax;
    c.run_ub = p->run_ub;
    p->ab_inc = c.state_ind && p->op != OP_NLSE && !p->dense;
    c.ab_inc = p->ab_inc ? 1 : 0;
    c.a_next = reinterpret_cast<double *>(p->d_work + p->w_anext);
    p->ab_valid = false;
    c.htab_all = 1;
    for (const InstDev &I : p->hinst) c.htab_all = c.htab_all && I.ht_off >= 0;
    // the wave-per-strip indicator, for block rows wider than a wave row (NLSE
    // only with its H tables: the evaluated propagator needs the registers of
    // the workgroup-per-strip kernel)
    c.wave_ind = (p->op != OP_NLSE || c.htab_all) && !p->half ? 1 : 0;
    c.half = p->half ? 1 : 0;
    c.half_nb = 0;
    for (const InstDev &I : p->hinst) c.half_nb = std::max(c.half_nb, I.nbxm + 1);
    for (const InstDev &I : p->hinst) c.wave_ind = c.wave_ind && I.chunks > 1;
    // the workgroup walk serves blocks of at most 128 (64) slots two (four)
    // at a time, so that its 256 threads are busy
    c.upd_group = p->max_slots <= 64 ? 4 : p->max_slots <= 128 ? 2 : 1;
    c.sig_bytes = (int32_t)(p->n_taper * sizeof(double));
    c.taper_bs = 0;
    for (const InstDev &I : p->hinst)
        for (int a = 0; a < 3; ++a) c.taper_bs |= 1u << I.lb[a];
    if (p->half) c.taper_bs |= 1u;  // the one-column blocks of nx/2: edge 1
    c.nb_total = p->nb_total;
    c.n_strips = p->n_strips;
    c.n_tiles = p->n_tiles;
    c.n_chunks = p->n_chunks;
    TRY_HIP(hipMemcpyAsync(p->d_work + p->w_table, p->hinst.data(), p->hinst.size() * sizeof(InstDev),
                           hipMemcpyHostToDevice, p->stream));
    TRY_HIP(hipMemcpyAsync(p->d_work + p->w_binst, p->blk_inst.data(),
                           p->blk_inst.size() * sizeof(uint16_t), hipMemcpyHostToDevice, p->stream));
    if (!p->ltab.empty())
        TRY_HIP(hipMemcpyAsync(p->d_work + p->w_ltab, p->ltab.data(), p->ltab.size() * sizeof(double),
                               hipMemcpyHostToDevice, p->stream));
    p->hist_valid = false;
    TRY_HIP(hipMemsetAsync(p->d_state + p->st_k0, 0, (size_t)p->n_inst * 2 * sizeof(double), p->stream));
    TRY_HIP(hipMemsetAsync(c.rhs_k0, 0, (size_t)p->n_inst * 2 * sizeof(double), p->stream));
    TRY_HIP(hipMemsetAsync(c.count, 0, 16, p->stream));
    TRY_HIP(hipMemsetAsync(c.mask, 0, (size_t)p->nb_total, p->stream));
    TRY_HIP(hipMemsetAsync(c.a_b, 0, (size_t)p->nb_total * sizeof(double), p->stream));
    TRY_HIP(launch_reset(c, p->stream));
    TRY_HIP(launch_tapers(c, p->stream));
    if (p->n_htab > 0) TRY_HIP(launch_htable(c, p->dbl, p->stream));
    TRY_HIP(launch_ctl_reset(c, -1, p->stream));
    if (p->dense) {  // Regular mode: every block active, the list is every block
        std::vector<uint32_t> all((size_t)p->nb_total);
        std::iota(all.begin(), all.end(), 0u);
        const uint32_t cnt = (uint32_t)p->nb_total;
        TRY_HIP(hipMemsetAsync(c.mask, 1, (size_t)p->nb_total, p->stream));
        TRY_HIP(hipMemcpyAsync(c.worklist, all.data(), all.size() * 4, hipMemcpyHostToDevice, p->stream));
        TRY_HIP(hipMemcpyAsync(c.count, &cnt, 4, hipMemcpyHostToDevice, p->stream));
        TRY_HIP(hipStreamSynchronize(p->stream));
    }
    TRY_HIP(hipStreamSynchronize(p->stream));
    p->bound = true;
    // out-of-place inverse transforms: does the input survive?
    p->inv_preserving = true;
    if (p->op != OP_NLSE) {
        for (auto &g : p->groups) {
            TRY(probe_preserving(p, g.inv_oop, g.off, g.N * g.count * p->nspec));
            TRY(probe_preserving(p, g.inv1_oop, g.off, g.N * p->nspec));
            p->inv_preserving = p->inv_preserving && g.inv_oop.preserves && g.inv1_oop.preserves;
        }
        TRY_HIP(hipMemsetAsync(p->d_state + p->st_spec, 0, (size_t)p->total_elems * p->esize, p->stream));
        TRY_HIP(hipStreamSynchronize(p->stream));
    }
    if (p->timing && !p->have_events) {
        for (auto &set : p->ev)
            for (auto &e : set) TRY_HIP(hipEventCreate(&e));
        for (auto &set : p->evk)
            for (auto &e : set) TRY_HIP(hipEventCreate(&e));
        p->have_events = true;
    }
    return SPDBA_OK;
}

spdba_status spdba_set_field(spdba_plan p, int32_t inst, const void *d_real) {
    if (!p || !d_real || inst < 0 || inst >= p->n_inst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    const InstDev &I = p->hinst[inst];
    const int64_t n = I.N * p->nspec;
    TRY_HIP(launch_ctl_reset(p->ctx, inst, p->stream));
    p->ab_valid = false;
    p->hist_valid = false;
    if (p->op == OP_NLSE) {
        TRY_HIP(launch_scale_copy(p->dbl, d_real, state_ptr(p, I.off), n, (double)I.N, p->stream));
        return SPDBA_OK;
    }
    const Group &g = p->groups[p->group_of[inst]];
    if (p->half) {  // real slots of W, forward into R, then the state
        TRY_HIP(launch_real_to_complex(p->ctx, p->dbl, inst, d_real, I.Nreal * p->nspec, p->stream));
        TRY(exec_fft(p, g.fwd1_oop, wreal_ptr(p, I.roff), rhs_ptr(p, I.off)));
        TRY_HIP(launch_copy_spectrum(p->ctx, p->dbl, inst, rhs_ptr(p, I.off), state_ptr(p, I.off), n,
                                     I.k0path, nullptr, p->stream));
        if (I.k0path) TRY_HIP(launch_real_sums_to_k0(p->ctx, p->dbl, inst, d_real, I.ntiles, p->stream));
        return SPDBA_OK;
    }
    TRY_HIP(launch_real_to_complex(p->ctx, p->dbl, inst, d_real, n, p->stream));
    TRY(exec_fft(p, g.fwd1_ip, work_ptr(p, I.off), nullptr));
    TRY_HIP(launch_copy_spectrum(p->ctx, p->dbl, inst, work_ptr(p, I.off), state_ptr(p, I.off), n,
                                 I.k0path, nullptr, p->stream));
    if (I.k0path) TRY_HIP(launch_real_sums_to_k0(p->ctx, p->dbl, inst, d_real, I.ntiles, p->stream));
    return SPDBA_OK;
}

spdba_status spdba_get_field(spdba_plan p, int32_t inst, void *d_out) {
    if (!p || !d_out || inst < 0 || inst >= p->n_inst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    const InstDev &I = p->hinst[inst];
    const int64_t n = I.N * p->nspec;
    if (p->op == OP_NLSE) {
        TRY_HIP(launch_scale_copy(p->dbl, state_ptr(p, I.off), d_out, n, I.invN, p->stream));
        return SPDBA_OK;
    }
    const Group &g = p->groups[p->group_of[inst]];
    if (p->half) {
        TRY(inverse_half(p, g.inv1_oop, I.off, I.roff, n));
        TRY_HIP(launch_work_to_real(p->ctx, p->dbl, inst, d_out, I.Nreal * p->nspec, p->stream));
        return SPDBA_OK;
    }
    TRY(inverse_keep(p, g.inv1_oop, g.inv1_ip, I.off, n));
    TRY_HIP(launch_work_to_real(p->ctx, p->dbl, inst, d_out, n, p->stream));
    return SPDBA_OK;
}

spdba_status spdba_set_spectrum(spdba_plan p, int32_t inst, const void *d_hat, const double *h_k0) {
    if (!p || !d_hat || inst < 0 || inst >= p->n_inst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    const InstDev &I = p->hinst[inst];
    const int64_t n = I.N * p->nspec;
    double *k0 = p->ctx.k0 + 2 * inst;
    TRY_HIP(launch_ctl_reset(p->ctx, inst, p->stream));
    p->ab_valid = false;
    p->hist_valid = false;
    if (p->half)  // compact rows of nx/2 + 1 into the pitched rows
        TRY_HIP(launch_copy_half(p->ctx, p->dbl, inst, d_hat, state_ptr(p, I.off), true, I.k0path,
                                 (I.k0path && !h_k0) ? k0 : nullptr, p->stream));
    else
        TRY_HIP(launch_copy_spectrum(p->ctx, p->dbl, inst, d_hat, state_ptr(p, I.off), n, I.k0path,
                                     (I.k0path && !h_k0) ? k0 : nullptr, p->stream));
    if (I.k0path && h_k0) {
        TRY_HIP(hipMemcpyAsync(k0, h_k0, (size_t)p->nspec * sizeof(double), hipMemcpyHostToDevice,
                               p->stream));
        TRY_HIP(hipStreamSynchronize(p->stream));
    }
    return SPDBA_OK;
}

spdba_status spdba_get_spectrum(spdba_plan p, int32_t inst, void *d_hat, double *h_k0) {
    if (!p || !d_hat || inst < 0 || inst >= p->n_inst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    const InstDev &I = p->hinst[inst];
    if (p->half)
        TRY_HIP(launch_copy_half(p->ctx, p->dbl, inst, state_ptr(p, I.off), d_hat, false, 0, nullptr, p->stream));
    else
        TRY_HIP(hipMemcpyAsync(d_hat, state_ptr(p, I.off), (size_t)(I.N * p->nspec) * p->esize,
                               hipMemcpyDeviceToDevice, p->stream));
    if (h_k0) {
        double tmp[2] = {0.0, 0.0};
        TRY_HIP(hipMemcpyAsync(tmp, p->ctx.k0 + 2 * inst, 2 * sizeof(double), hipMemcpyDeviceToHost,
                               p->stream));
        TRY_HIP(hipStreamSynchronize(p->stream));
        for (int s = 0; s < p->nspec; ++s) h_k0[s] = I.k0path ? tmp[s] : 0.0;
    }
    TRY_HIP(hipStreamSynchronize(p->stream));
    return check_nonfinite(p);
}

spdba_status spdba_step(spdba_plan p, int32_t n_steps) {
    if (!p || n_steps < 0) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    if (n_steps == 0) return SPDBA_OK;
    // a graph holds the kept-measure update stage and (XPFC) a filled
    // history: after a field load the measure is first evaluated in full,
    // and the history filled, by one eager step
    while (n_steps > 0 && p->use_graph && ((p->ab_inc && !p->ab_valid) || (p->op == OP_XPFC && !p->hist_valid))) {
        set_phase(p);
        TRY(enqueue_step(p));
        advance_phase(p);
        p->steps++;
        --n_steps;
    }
    if (n_steps == 0) return SPDBA_OK;
    if (p->use_graph && !p->graph_failed) {
        while (n_steps > 0) {
            const int gi = p->op == OP_XPFC ? p->xphase : 0;
            if (!p->graph[gi]) {
                set_phase(p);
                hipGraph_t gr = nullptr;
                hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeRelaxed);
                spdba_status st = SPDBA_OK;
                if (e == hipSuccess) st = enqueue_step(p);
                hipError_t e2 = hipStreamEndCapture(p->stream, &gr);
                if (e != hipSuccess || st != SPDBA_OK || e2 != hipSuccess || !gr ||
                    hipGraphInstantiate(&p->graph[gi], gr, nullptr, nullptr, 0) != hipSuccess) {
                    p->graph[gi] = nullptr;
                    p->graph_failed = true;
                    (void)hipGetLastError();
                }
                if (gr) (void)hipGraphDestroy(gr);
                if (!p->graph[gi]) break;  // eager from here on
            }
            TRY_HIP(hipGraphLaunch(p->graph[gi], p->stream));
            advance_phase(p);
            p->steps++;
            --n_steps;
        }
        if (n_steps == 0) return SPDBA_OK;
    }
    for (int i = 0; i < n_steps; ++i) {
        set_phase(p);
        TRY(enqueue_step(p));
        advance_phase(p);
        ring_advance(p);
        p->steps++;
    }
    return SPDBA_OK;
}

spdba_status spdba_apply(spdba_plan p, const void *d_rhs_hat, const double *h_rhs_k0) {
    if (!p) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    if (p->op != OP_NLSE) {
        if (!d_rhs_hat) return SPDBA_EINVAL;
        int64_t src = 0;
        for (int i = 0; i < p->n_inst; ++i) {
            const InstDev &I = p->hinst[i];
            const char *sp = static_cast<const char *>(d_rhs_hat) + src * p->esize;
            double *rk0 = (I.k0path && !h_rhs_k0) ? p->ctx.rhs_k0 + 2 * i : nullptr;
            if (p->half) {  // compact rows of nx/2 + 1
                TRY_HIP(launch_copy_half(p->ctx, p->dbl, i, sp, rhs_ptr(p, I.off), true, 0, rk0, p->stream));
                src += (int64_t)I.n[0] * I.n[1] * (I.n[2] / 2 + 1) * p->nspec;
            } else {
                const int64_t n = I.N * p->nspec;
                char *dst = p->op == OP_XPFC ? hist_ptr(p, p->xphase, I.off) : rhs_ptr(p, I.off);
                TRY_HIP(launch_copy_spectrum(p->ctx, p->dbl, i, sp, dst, n, 0, rk0, p->stream));
                src += n;
            }
        }
        if (h_rhs_k0 && !p->dbl) {
            std::vector<double> tmp((size_t)p->n_inst * 2, 0.0);
            for (int i = 0; i < p->n_inst; ++i)
                for (int s = 0; s < p->nspec; ++s) tmp[2 * i + s] = h_rhs_k0[i * p->nspec + s];
            TRY_HIP(hipMemcpyAsync(p->ctx.rhs_k0, tmp.data(), tmp.size() * sizeof(double),
                                   hipMemcpyHostToDevice, p->stream));
            TRY_HIP(hipStreamSynchronize(p->stream));
        }
    }
    // the update stage alone: events 3..6 of a CH/GS step
    TRY(fill_history(p));  // XPFC: a new field's history starts from this transform
    set_phase(p);
    record(p, 3);
    TRY(update_stage(p, p->op == OP_NLSE ? 2 : 4));
    advance_phase(p);
    return SPDBA_OK;
}

spdba_status spdba_set_skip(spdba_plan p, const uint8_t *d_skip) {
    if (!p) return SPDBA_EINVAL;
    p->d_skip = d_skip;
    p->ctx.skip = d_skip;
    p->ab_valid = false;
    drop_graphs(p);  // a captured graph holds the old pointers
    return SPDBA_OK;
}

spdba_status spdba_set_block_energy(spdba_plan p, double *d_eb) {
    if (!p) return SPDBA_EINVAL;
    if (p->half && d_eb) return SPDBA_EUNSUPPORTED;
    p->d_eb = d_eb;
    p->ctx.e_b = d_eb;
    drop_graphs(p);  // a captured graph holds the old pointers
    return SPDBA_OK;
}

spdba_status spdba_active_mask(spdba_plan p, int32_t inst, uint8_t *host_out, size_t n) {
    if (!p || !host_out || inst < 0 || inst >= p->n_inst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    const InstDev &I = p->hinst[inst];
    if (n < (size_t)I.nb) return SPDBA_EINVAL;
    TRY_HIP(hipMemcpyAsync(host_out, p->ctx.mask + I.blk_off, (size_t)I.nb, hipMemcpyDeviceToHost,
                           p->stream));
    return check_nonfinite(p);
}

spdba_status spdba_indicator(spdba_plan p, int32_t inst, double *host_ab, size_t n, double *host_G) {
    if (!p || inst < 0 || inst >= p->n_inst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    const InstDev &I = p->hinst[inst];
    if (host_ab) {
        if (n < (size_t)I.nb) return SPDBA_EINVAL;
        TRY_HIP(hipMemcpyAsync(host_ab, p->ctx.a_b + I.blk_off, (size_t)I.nb * sizeof(double),
                               hipMemcpyDeviceToHost, p->stream));
    }
    if (host_G) {
        unsigned long long g = 0;
        TRY_HIP(hipMemcpyAsync(&g, p->ctx.G_last + inst, 8, hipMemcpyDeviceToHost, p->stream));
        TRY_HIP(hipStreamSynchronize(p->stream));
        double v;
        std::memcpy(&v, &g, 8);
        *host_G = v;
    }
    return check_nonfinite(p);
}

spdba_status spdba_worklist(spdba_plan p, int32_t inst, uint32_t *host_out, size_t n, int64_t *count) {
    if (!p || !host_out || !count || inst < 0 || inst >= p->n_inst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    const InstDev &I = p->hinst[inst];
    if (n < (size_t)I.nb) return SPDBA_EINVAL;
    if (p->list_stale) {  // build the ordered list from the current mask
        TRY_HIP(launch_compact(p->ctx, p->stream, 1));
        p->list_stale = false;
    }
    uint32_t total = 0;
    TRY_HIP(hipMemcpyAsync(&total, p->ctx.count, 4, hipMemcpyDeviceToHost, p->stream));
    TRY_HIP(hipStreamSynchronize(p->stream));
    std::vector<uint32_t> all(total);
    if (total)
        TRY_HIP(hipMemcpyAsync(all.data(), p->ctx.worklist, (size_t)total * 4, hipMemcpyDeviceToHost,
                               p->stream));
    TRY_HIP(hipStreamSynchronize(p->stream));
    int64_t k = 0;
    for (uint32_t v : all)
        if ((int64_t)v >= I.blk_off && (int64_t)v < I.blk_off + I.nb) host_out[k++] = (uint32_t)(v - I.blk_off);
    *count = k;
    return check_nonfinite(p);
}

spdba_status spdba_device_views(spdba_plan p, const double **d_ab, const uint8_t **d_mask,
                                const double **d_G, int64_t *total_blocks) {
    if (!p) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    if (d_ab) *d_ab = p->ctx.a_b;
    if (d_mask) *d_mask = p->ctx.mask;
    if (d_G) *d_G = reinterpret_cast<const double *>(p->ctx.G_last);
    if (total_blocks) *total_blocks = p->nb_total;
    return SPDBA_OK;
}

spdba_status spdba_stats(spdba_plan p, int32_t inst, spdba_stats_t *out) {
    if (!p || !out || inst < 0 || inst >= p->n_inst) return SPDBA_EINVAL;
    if (!p->bound) return SPDBA_ESTATE;
    std::memset(out, 0, sizeof(*out));
    const InstDev &I = p->hinst[inst];
    std::vector<uint8_t> mk((size_t)I.nb);
    TRY_HIP(hipMemcpyAsync(mk.data(), p->ctx.mask + I.blk_off, (size_t)I.nb, hipMemcpyDeviceToHost,
                           p->stream));
    unsigned long long g = 0;
    TRY_HIP(hipMemcpyAsync(&g, p->ctx.G_last + inst, 8, hipMemcpyDeviceToHost, p->stream));
    double k0[2] = {0.0, 0.0};
    TRY_HIP(hipMemcpyAsync(k0, p->ctx.k0 + 2 * inst, 16, hipMemcpyDeviceToHost, p->stream));
    CtlDev C;
    TRY_HIP(hipMemcpyAsync(&C, p->ctx.ctl + inst, sizeof(CtlDev), hipMemcpyDeviceToHost, p->stream));
    double slot0[2][2] = {{0, 0}, {0, 0}};
    if (p->dbl && p->op != OP_NLSE)
        for (int s = 0; s < p->nspec; ++s)
            TRY_HIP(hipMemcpyAsync(slot0[s], state_ptr(p, I.off + s * I.N), 16, hipMemcpyDeviceToHost,
                                   p->stream));
    std::vector<double> nlp, egp;
    if (p->op == OP_CH && p->steps > 0 && !p->last_inc) {
        nlp.resize((size_t)I.ntiles * 2);
        TRY_HIP(hipMemcpyAsync(nlp.data(), p->ctx.nl_part + 2 * I.tile_off, nlp.size() * 8,
                               hipMemcpyDeviceToHost, p->stream));
        if (p->last_dense) {
            egp.resize((size_t)I.ntiles);
            TRY_HIP(hipMemcpyAsync(egp.data(), p->ctx.dense_part + I.tile_off, egp.size() * 8,
                                   hipMemcpyDeviceToHost, p->stream));
        } else {
            egp.resize((size_t)I.nstrips);
            TRY_HIP(hipMemcpyAsync(egp.data(), p->ctx.ind_part + I.strip_off, egp.size() * 8,
                                   hipMemcpyDeviceToHost, p->stream));
        }
    }
    TRY_HIP(hipStreamSynchronize(p->stream));
    out->steps = p->steps;
    out->total_blocks = I.nb;
    int64_t a = 0, tr = 0;
    for (uint8_t v : mk) {
        a += v == 1;
        tr += v == 2;
    }
    out->active_blocks = a;
    out->transition_blocks = tr;
    out->tau = C.tau;
    out->control_step = C.step;
    const int64_t updates = C.step * I.per + C.upd;
    out->nonfrozen_ratio_mean = (p->ctl && updates > 0) ? (double)C.nf_total / ((double)I.nb * (double)updates) : NAN;
    std::memcpy(&out->G, &g, 8);
    for (int s = 0; s < p->nspec; ++s)
        out->mean[s] = p->op == OP_NLSE ? 0.0 : (I.k0path ? k0[s] : slot0[s][0]) * I.invN;
    out->energy = NAN;
    if (!nlp.empty() && p->op == OP_CH) {
        double bulk = 0.0, grad = 0.0;
        for (int64_t t = 0; t < I.ntiles; ++t) bulk += nlp[2 * t];
        for (double v : egp) grad += v;
        out->energy = I.dvol * bulk + 0.5 * p->desc[inst].op_params[1] * (I.dvol * I.invN) * grad;
    }
    if (p->timing && p->have_events && p->ring_filled > 0) {
        // mean over the completed steps held in the ring (the stream has drained)
        const int nset = p->ring_filled;
        double acc6[6] = {0, 0, 0, 0, 0, 0};
        double ind_k = 0.0;
        for (int k = 1; k <= nset; ++k) {
            hipEvent_t *ev = p->ev[(p->ring - k + spdba_plan_s::kRing) % spdba_plan_s::kRing];
            auto el = [&](int a0, int b0) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[a0], ev[b0]) != hipSuccess) return 0.0;
                return (double)ms;
            };
            double st[6] = {0, 0, 0, 0, 0, 0};
            if (p->op != OP_NLSE) {
                st[0] = el(7, 1) + el(2, 3);
                st[1] = el(1, 2);
                if (!p->last_dense) {
                    st[2] = el(0, 7) + el(3, 4);  // a state-measure full pass runs first
                    st[3] = el(4, 5);
                    st[4] = el(5, 6);
                } else {
                    st[4] = el(3, 6);
                }
                st[5] = el(0, 6);
            } else {
                st[0] = el(0, 1) + el(6, 7) + el(4, 5) + el(10, 11);
                if (!p->last_dense) {
                    st[2] = el(1, 2) + el(7, 8);
                    st[3] = el(2, 3) + el(8, 9);
                    st[4] = el(3, 4) + el(9, 10);
                } else {
                    st[4] = el(1, 4) + el(7, 10);
                }
                st[1] = el(5, 6);
                st[5] = el(0, 11);
            }
            for (int j = 0; j < 6; ++j) acc6[j] += st[j];
            const int slot = (p->ring - k + spdba_plan_s::kRing) % spdba_plan_s::kRing;
            auto pair = [](hipEvent_t a, hipEvent_t b) {
                float ms = 0.f;
                return hipEventElapsedTime(&ms, a, b) == hipSuccess ? (double)ms : 0.0;
            };
            for (int h = 0; h < (p->op == OP_NLSE ? 2 : 1); ++h)
                if (!p->last_dense && p->evk_set[slot][h]) ind_k += pair(p->evk[slot][2 * h], p->evk[slot][2 * h + 1]);
        }
        for (int j = 0; j < 6; ++j) out->stage_ms[j] = acc6[j] / nset;
        out->indicator_kernel_ms = ind_k / nset;
        // a failed read above must not surface at the next launch check
        (void)hipGetLastError();
    }
    out->input_preserving_fft = p->inv_preserving ? 1 : 0;
    out->graph_replay = (p->graph[0] || p->graph[1] || p->graph[2] || p->graph[3]) ? 1 : 0;
    return check_nonfinite(p);
}

spdba_status spdba_set_launch(spdba_plan p, int32_t kernel, int32_t value) {
    if (!p) return SPDBA_EINVAL;
    auto pow2_in = [](int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; };
    switch (kernel) {
        case 0: if (!pow2_in(value, 1, 16)) return SPDBA_EINVAL; p->ind_waves = value; break;
        case 1: if (value < 1 || value > 64) return SPDBA_EINVAL; p->upd_per_cu = value; break;
        case 2: if (!pow2_in(value, 64, 1024)) return SPDBA_EINVAL; p->dense_threads = value; break;
        case 3: if (value < 0 || value > 4) return SPDBA_EINVAL; p->upd_mode = value; break;
        case 4: if (!pow2_in(value, 1, 16)) return SPDBA_EINVAL; p->upd_waves = value; break;
        case 5:
            if (value != 0 && value != 1) return SPDBA_EINVAL;
            if (value && !fwd_in_place_ok(p)) return SPDBA_EUNSUPPORTED;
            p->fwd_in_place = value != 0;
            if (p->bound) p->ctx.rhs = rhs_ptr(p, 0);
            break;
        default: return SPDBA_EINVAL;
    }
    p->ring_filled = 0;  // timings of the previous geometry are stale
    drop_graphs(p);  // a captured graph holds the old pointers
    return SPDBA_OK;
}

spdba_status spdba_destroy(spdba_plan p) {
    if (!p) return SPDBA_OK;
    drop_graphs(p);
    for (auto &g : p->groups) {
        destroy_fft(g.inv_oop);
        destroy_fft(g.fwd_ip);
        destroy_fft(g.fwd_oop);
        destroy_fft(g.inv_ip);
        destroy_fft(g.inv1_oop);
        destroy_fft(g.fwd1_ip);
        destroy_fft(g.inv1_ip);
        destroy_fft(g.fwd1_oop);
    }
    if (p->info) rocfft_execution_info_destroy(p->info);
    if (p->have_events) {
        for (auto &set : p->ev)
            for (auto &e : set) (void)hipEventDestroy(e);
        for (auto &set : p->evk)
            for (auto &e : set) (void)hipEventDestroy(e);
    }
    delete p;
    return SPDBA_OK;
}

}  // extern "C"

// rocFFT's library set-up, once per process, shared by every plan type
int32_t spdba::fft_setup() {
    std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
    return g_rocfft_setup == rocfft_status_success ? SPDBA_OK : SPDBA_EFFT;
}
