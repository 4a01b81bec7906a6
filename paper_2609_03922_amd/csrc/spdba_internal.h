// spdba_internal.h -- device-side instance table and kernel launchers shared by
// the host API (spdba_api.cpp) and the HIP kernels (spdba_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spdba.h"

struct spdba_plan_s;

namespace spdba {

enum Op : int { OP_CH = 1, OP_GS = 2, OP_NLSE = 3, OP_XPFC = 4 };

// Per-instance constants, uploaded once at bind.  Offsets are in complex
// elements (state and transform buffers share one layout) or block / strip /
// tile ids in the concatenated spaces of all instances.
struct InstDev {
    int64_t off;        // first complex element of species 0 in state / work
    int64_t N;          // modes per species
    int64_t blk_off;    // first global block id
    int64_t nb;         // blocks
    int64_t strip_off;  // first global indicator strip id
    int64_t nstrips;
    int64_t tile_off;   // first global elementwise tile id
    int64_t ntiles;
    int32_t n[3];       // nz, ny, nx
    int32_t b[3];       // block edges
    int32_t nbk[3];     // blocks per axis
    int32_t S;          // blocks per strip along x
    int32_t chunks;     // 64-lane chunks per block row (when a block row is wider than a wave row)
    int32_t nspec;
    int32_t k0path;     // 1: FP32 real field, k = 0 kept in FP64
    int32_t pin;        // PIN_K0
    int32_t ln[3];      // log2 of n[] (all extents and block edges are powers of two)
    int32_t lb[3];      // log2 of b[]
    int32_t lnbk[3];    // log2 of nbk[]
    int32_t lS, lchunks;
    double K2;          // (2 pi / (n dx))^2
    double c0, c1, c2;  // CH: dt*M, dt*M*kappa, -; GS: dt, dt*Du, dt*Dv; NLSE: theta/m^2, A, -
    double tau2;        // fl(tau*tau)
    double invN;        // 1/N (exact power of two)
    double q0, q1;      // nonlinear parameters: GS F, k; NLSE gamma*h, -
    double dvol;        // dx^d
    // consistency control (schedule and threshold controller)
    int32_t full_steps; // steps 0..full_steps-1 update every block
    int32_t refresh;    // period of full steps (0: off)
    int32_t interval;   // controller interval in steps (0: fixed threshold)
    int32_t per;        // updates per step (NLSE: two half steps)
    double tau0;        // threshold after a reset
    double target, deadband;
    int64_t ht_off;     // NLSE in one dimension: first entry of the H(|m|) table (complex); else -1
    int64_t ltab_off;   // XPFC: first entry of the L(|m|^2) table (FP64, one per integer |m|^2)
    // half-spectrum layout (real fields): rows of xs = nx/2 + 1 stored columns;
    // the blocks of the columns below nx/2 first (nbm of them, nbxm along x),
    // then one block per (z, y) block row for the column nx/2
    int32_t half;
    int32_t xs;         // stored row pitch: nx in the full layout; half: nx/2 + 1
                        // rounded up to 128 bytes (the columns beyond nx/2 are
                        // never read or written; rocFFT's passes across rows
                        // then run on aligned lines)
    int32_t nbxm;       // blocks along x below the column nx/2
    int32_t lnbxm;      // log2 nbxm
    int64_t nbm;        // blocks of the columns below nx/2 (nb in the full layout)
    int64_t Nreal;      // grid points per species (N in the full layout)
    int64_t roff;       // half: first real of species 0 in W; the species and
                        // the instances of one transform batch follow each
                        // other at Nreal values (the real transforms' default)
};

// Per-instance control state, in the state buffer: it persists across steps
// (and graph replays) and is reset with the field.
struct CtlDev {
    double tau, tau2;   // threshold of the current step and fl(tau*tau)
    double sum;         // controller: sum of the per-step ratios of the interval
    int64_t step;       // completed steps since the reset
    int32_t full;       // the current step updates every block
    int32_t upd;        // updates done in the current step
    int32_t n;          // steps accumulated in sum
    int32_t pad0;
    uint32_t nf_step;   // non-frozen blocks over the current step's updates
    uint32_t nf_upd;    // non-frozen blocks of the update in flight
    uint64_t nf_total;  // non-frozen blocks summed over every update since the reset
};

// Everything a kernel needs, passed by value.
struct Ctx {
    const InstDev *inst;
    int32_t n_inst;
    int32_t nspec;
    int32_t op;
    int32_t dense;
    void *state;               // complex T
    void *work;                // complex T: inverse transform / nonlinear term
    void *rhs;                 // complex T: forward transform of the nonlinear term
    double *k0;                // [n_inst][2] FP64 k = 0 state
    double *rhs_k0;            // [n_inst][2]
    double *a_b;               // [nb_total]
    double *a_next;            // [nb_total] state measure of the blocks the last update stored (ab_inc)
    unsigned long long *G;     // [n_inst] bits of a non-negative double
    unsigned long long *G_last;// [n_inst] G of the last completed update
    uint8_t *mask;             // [nb_total]
    uint32_t *worklist;        // [nb_total] global block ids, ascending
    uint32_t *chunk_cnt;       // [n_chunks]
    uint32_t *count;           // [1] active blocks over all instances
    uint32_t *done;            // [1] workgroup arrival counter (self-resetting)
    double *nl_part;           // [n_tiles][2] per-tile FP64 sums of the nonlinear stage
    double *ind_part;          // [n_strips] per-strip FP64 sums (CH gradient energy)
    double *strip_max;         // [n_strips] largest block value a_b of each strip
    double *dense_part;        // [n_tiles] per-tile FP64 sums of the dense update
    uint32_t *nonfinite;       // [1]
    const uint16_t *blk_inst;  // [nb_total] owning instance of each block
    const uint8_t *skip;       // [nb_total] or nullptr
    double *e_b;               // [nb_total] per-block energies or nullptr
    CtlDev *ctl;               // [n_inst] control state
    const void *htab;          // NLSE H(|m|) tables (complex, working precision)
    const double *ltab;        // XPFC L(|m|^2) tables (FP64)
    const void *hist1, *hist2, *hist3;  // XPFC: transforms of the three previous steps (rhs: this step's)
    const double *taper;       // roll-off tables: edge B at [B, 2B)
    uint32_t taper_bs;         // bit k: block edge 2^k in use
    int32_t wave_ind;          // every block row spans several wave rows: one wave per strip
    int32_t htab_all;          // every instance has an NLSE H table
    int32_t state_ind;         // state-amplitude activity measure
    int32_t ab_inc;            // the update rewrites a_b of the blocks it stores (state measure, CH/GS)
    int32_t trans;             // transition blocks on
    int32_t sig_bytes;         // LDS of the transition update: the tables, 2 B_max doubles
    int32_t half;              // half-spectrum layout
    int32_t half_nb;           // half: largest number of blocks of one (z, y) block row
    int32_t ab_sum;            // state measure: a_b is the block's sum (block energy), not its maximum
    int32_t run_lmax;          // run walk: longest piece in blocks (power of two), 0 = not available
    int32_t run_ub;            // run walk: 16-byte loads per lane and array (slots per block / 64)
    int32_t upd_group;         // workgroup walk: list entries per iteration (1, 2, 4; blocks of at
                               // most 256 / upd_group slots); 0 = 1
    int64_t nb_total;
    int64_t n_strips;
    int64_t n_tiles;
    int64_t n_chunks;
};

constexpr int TILE_THREADS = 256;
constexpr uint32_t kEntryId = (1u << 25) - 1;  // block-id field of a transition plan's list entry
constexpr int CHUNK_BLOCKS = 1024;  // compaction chunk

// elementwise tile size in complex elements per dtype (FP32: 4 per thread, FP64: 2)
template <typename T> constexpr int tile_elems() { return sizeof(T) == 4 ? 1024 : 512; }

// Launchers (return hipError_t of the launch).  `dbl` selects FP64.
hipError_t launch_nonlinear(const Ctx &c, bool dbl, int waves, hipStream_t s);
hipError_t launch_k0_rhs(const Ctx &c, hipStream_t s);
hipError_t launch_indicator(const Ctx &c, bool dbl, int waves, hipStream_t s, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr);
hipError_t launch_compact(const Ctx &c, hipStream_t s, int from_mask = 0);
hipError_t launch_compact_append(const Ctx &c, hipStream_t s);
// run walk: threshold, mask and the band list of aligned runs of active blocks
hipError_t launch_compact_runs(const Ctx &c, hipStream_t s);
// consistency control: block states and list; reset; roll-off tables
hipError_t launch_compact_states(const Ctx &c, hipStream_t s);
hipError_t launch_gmax(const Ctx &c, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_ctl_reset(const Ctx &c, int only_inst, hipStream_t s);
hipError_t launch_tapers(const Ctx &c, hipStream_t s);
hipError_t launch_htable(const Ctx &c, bool dbl, hipStream_t s);
// multi: 0 block-list walk, 1 four entries in flight, 2 one wave per entry, 3 run walk (band list);
// tr: transition weights; ctl: end-of-update control in the last workgroup
hipError_t launch_update(const Ctx &c, bool dbl, int grid, int multi, hipStream_t s, bool tr = false,
                         bool ctl = false);
hipError_t launch_update_strip(const Ctx &c, bool dbl, int waves, int grid, hipStream_t s);
hipError_t launch_dense(const Ctx &c, bool dbl, int threads, hipStream_t s);
hipError_t launch_reset(const Ctx &c, hipStream_t s);
// set_field / get_field helpers on one instance (sizes from the host table)
hipError_t launch_real_to_complex(const Ctx &c, bool dbl, int inst, const void *real, int64_t n,
                                  hipStream_t s);
hipError_t launch_real_sums_to_k0(const Ctx &c, bool dbl, int inst, const void *real,
                                  int64_t ntiles, hipStream_t s);
hipError_t launch_work_to_real(const Ctx &c, bool dbl, int inst, void *out, int64_t n,
                               hipStream_t s);
hipError_t launch_scale_copy(bool dbl, const void *src, void *dst, int64_t n_complex, double scale,
                             hipStream_t s);
hipError_t launch_copy_spectrum(const Ctx &c, bool dbl, int inst, const void *src, void *dst,
                                int64_t n, int zero_slot0, double *k0_dst, hipStream_t s);
// half layout: a compact spectrum (rows of nx/2 + 1) to the pitched stored layout
// (to_pitched, optionally moving slot 0 of each species to k0_dst and zeroing it) or back
hipError_t launch_copy_half(const Ctx &c, bool dbl, int inst, const void *src, void *dst, bool to_pitched,
                            int zero_slot0, double *k0_dst, hipStream_t s);
// probe helpers
hipError_t launch_fill_pattern(void *buf, int64_t n_elems, bool dbl, hipStream_t s);
// bytes a multiple of 8, both pointers 8-byte aligned
hipError_t launch_copy8(const void *src, void *dst, size_t bytes, hipStream_t s);
hipError_t launch_check_pattern(const void *buf, int64_t n_elems, bool dbl, uint32_t *bad, hipStream_t s);

// The block-activity stage that every plan type runs with the same kernels
// (k_gmax, k_compact_append): G = max_b a_b, where the blocks the last update
// stored (mask nonzero) first take the measure it kept (a_next); then the
// threshold rule a_b > fl(tau^2) G (block 0 always active when pinned), the
// mask and the list of active blocks (ascending within chunks of 1024 blocks,
// chunks in arrival order) with its count.  One instance, no skip set.  A
// caller whose measure pass rewrites every a_b clears the mask in that pass,
// so nothing is merged; without a kept measure a_next may alias a_b.
struct BlockStage {
    int64_t nb;
    double *a_b;
    const double *a_next;
    uint8_t *mask;             // 8-byte aligned
    uint32_t *list, *count;
    unsigned long long *G;     // zero before the stage (the caller clears it)
    void *aux;                 // block_stage_bytes(nb) bytes of device memory, 256-byte aligned:
                               // the instance record and the block owner table
};
size_t block_stage_bytes(int64_t nb);
// fills aux (instance record with tau^2 and the pin flag, owner table) on s
// and waits for it; outside any graph capture
hipError_t block_stage_init(const BlockStage &b, double tau2, int pin, hipStream_t s);
hipError_t launch_block_stage(const BlockStage &b, hipStream_t s);

// rocFFT's library set-up, once per process (spdba_api.cpp)
int32_t fft_setup();  // an spdba_status

// per-instance constants of the device table (spdba_api.cpp): everything but
// the offsets into the concatenated spaces, which are left 0
void fill_inst(const spdba_instance_desc &x, int op, bool dbl, bool pin, bool half, int64_t xs, InstDev &I);
// descriptor validation of spdba_plan_create (an spdba_status)
int32_t validate_desc(const spdba_instance_desc *d, int32_t n);

// plan internals for the proposer kernels (spdba_api.cpp)
const Ctx *plan_ctx(::spdba_plan_s *p);
const InstDev *plan_hinst(::spdba_plan_s *p, int *n_inst, int64_t *nb_total);

}  // namespace spdba
