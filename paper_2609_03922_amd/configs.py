"""The five synthetic workloads, as plain parameter records.

Each workload is named by what it is.  Operator parameter order follows the
library's descriptor: CH (M, kappa); GS (Du, Dv, F, k); NLSE (beta2, gamma, alpha).
``measure`` is the activity measure of the timed sp-DBA runs: the candidate
increment |dq|^2 where the workload prescribes it, else the state amplitude
|q|^2 (the paper's own state-based measures).  ``layout`` is the stored
spectrum of the timed runs: "full" (the natural c2c spectrum) or "half" (the
non-redundant half of a real field's transform, columns 0 .. n/2,
Supplementary S1.2; ``bench.py --layout half``).
Sizes of batched workloads are drawn from the workload's seed by
``inputs.instance_sizes``.
"""
from __future__ import annotations

CH2D_128_F64 = dict(
    name="ch2d_128_f64",
    op="ch", dtype="f64", ndim=2, n=128, block=16, tau=1e-6,
    dx=1.0, dt=0.01, params=(1.0, 1.0), steps=2000, seed=1001, measure="increment",
    layout="full",
    ic=dict(kind="uniform", mean=0.0, half_width=0.05),
)

CH3D_256_F32 = dict(
    name="ch3d_256_f32",
    op="ch", dtype="f32", ndim=3, n=256, block=8, tau=1e-6,
    dx=1.0, dt=0.01, params=(1.0, 1.0), steps=500, seed=1002, measure="state",
    layout="full",
    ic=dict(kind="uniform", mean=0.1, half_width=0.02),
)

NLSE1D_BATCH48_F32 = dict(
    name="nlse1d_batch48_f32",
    op="nlse", dtype="f32", ndim=1, n_instances=48, log2_min=14, log2_max=20, block=1024,
    tau=1e-6, dx=15.625, dt=0.8, params=(-21.7, 1.3, 0.0), steps=100, seed=1003, measure="state",
    layout="full",
    ic=dict(kind="qam16_rrc", sps=2, rolloff=0.1, power_w=1e-3),
)

GS2D_BATCH32_F32 = dict(
    name="gs2d_batch32_f32",
    op="gs", dtype="f32", ndim=2, n_instances=32, sizes=(256, 512, 1024), block=32,
    tau=1e-6, dx=1.0, dt=1.0, params=(0.16, 0.08, 0.035, 0.060), steps=5000, seed=1004, measure="state",
    layout="full",
    ic=dict(kind="gs_patches", patches=10, patch=8, u=0.5, v=0.25),
)

CH3D_512_F32_PROPOSER = dict(
    name="ch3d_512_f32_proposer",
    op="ch", dtype="f32", ndim=3, n=512, block=8, tau=1e-6,
    dx=1.0, dt=0.01, params=(1.0, 1.0), steps=500, seed=1005, measure="increment",
    layout="full",
    ic=dict(kind="uniform", mean=0.1, half_width=0.02),
    proposer=dict(K=10, audit_steps=3, train_n=256, train_seeds=tuple(range(2001, 2009))),
)

# XPFC polycrystalline coarsening (Supplementary S3.2): the paper's model and
# sp-DBA settings (dx, dt, q0, sigma, alpha, omega, u, psi_c, A_h; 16^2
# blocks, block energy, transition smoothing, threshold control with
# adjustment factor 0.05 every 50 steps from tau = 5e-5, an initial
# full-activation stage) on a 4096^2 grid in FP32, grown from seeded crystals
# for `full_steps` steps, the controller settling for `settle_steps`, then
# `window` timed steps at each target active ratio.
XPFC2D_4096_F32 = dict(
    name="xpfc2d_4096_f32",
    op="xpfc", dtype="f32", ndim=2, n=4096, block=16, tau=5e-5,
    dx=0.7854, dt=0.01, params=(1.0, 0.02, 0.1, 1.0, 1.0, 1.0, 1.0), seed=1010,
    full_steps=3000, settle_steps=1000, window=200, control_interval=50, deadband=0.05,
    targets=(0.05, 0.10, 0.20), taus=(1e-3, 3e-4, 1e-4, 3e-5, 1e-5), measure="energy", layout="full",
    ic=dict(kind="xpfc_seeds", mean=0.12, amp=0.25, seeds=400, radius_frac=0.02),
)

ALL = [CH2D_128_F64, CH3D_256_F32, NLSE1D_BATCH48_F32, GS2D_BATCH32_F32, CH3D_512_F32_PROPOSER, XPFC2D_4096_F32]


def lv_equilibrium(M: int, alpha: float, beta: float, r: float = 1.0, a: float = 1.0) -> float:
    """Homogeneous coexistence state of the Lotka--Volterra reaction with the
    circulant interactions of Supplementary S4.1 (neighbours beta + alpha,
    others beta): r / (a + 2 (beta + alpha) + (M - 3) beta), or
    r / (a + beta + alpha) for M = 2 -- the reference state the initial
    condition perturbs."""
    others = (beta + alpha) if M == 2 else 2.0 * (beta + alpha) + (M - 3) * beta
    return r / (a + others)


# Reaction--cross-diffusion (Supplementary S4.2): 256^3, M = 8 components,
# 8^3 blocks, dx = 0.5, dt = 0.01, D_diag = 0.5, D_cross = 0.05, alpha = 1,
# beta = 0.3, r_i = a_i = 1; a nearly homogeneous start with random
# perturbation of amplitude 0.1.  The relative thresholds of the sweep stand in
# for the paper's absolute threshold with its controller (target active ratio
# 3 to 20 %).
RCD3D_256_M8_F32 = dict(
    name="rcd3d_256_m8_f32",
    op="rcd", dtype="f32", ndim=3, n=256, block=8, M=8, steps=200, seed=1006,
    dt=0.01, dx=0.5, d_diag=0.5, d_cross=0.05, alpha=1.0, beta=0.3, r=1.0, a=1.0,
    ic=dict(kind="perturbed", amp=0.1),
    taus=(1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7),
)

# the paper's wide-component point (Fig. 3d: M = 48, 128^3 with 4^3 blocks);
# the FP64 Regular run on the GPU (matrix cores) is the truth.
RCD3D_128_M48_F32 = dict(
    name="rcd3d_128_m48_f32",
    op="rcd", dtype="f32", ndim=3, n=128, block=4, M=48, steps=200, seed=1007,
    dt=0.01, dx=0.5, d_diag=0.5, d_cross=0.05, alpha=1.0, beta=0.3, r=1.0, a=1.0,
    ic=dict(kind="perturbed", amp=0.1),
    taus=(1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7),
    err_bar=1e-4,  # used only where the FP64 path stops (M > 48)
)

# the paper's widest point (M = 64): no FP64 path, so the FP32 Regular run is
# the reference and err_bar the tolerance
RCD3D_128_M64_F32 = dict(RCD3D_128_M48_F32, name="rcd3d_128_m64_f32", M=64, seed=1008)

RCD = [RCD3D_256_M8_F32, RCD3D_128_M48_F32, RCD3D_128_M64_F32]

# Multimode digital backpropagation (Supplementary S5.3), the large end of the
# paper's scaling tests: M = 32 coupled modes (the widest with an FP64 path
# for the truth), 262,144 samples over T = 1000, 32-bin blocks, dz = 0.1 over
# 500 (5000 steps),
# beta2 = -21, alpha = 0.1, gamma = 1.3; three Gaussian packets (width 10,
# offsets -20/0/20, carriers -0.15/0/0.15 of 2 pi N/T) on every mode; K a
# seeded Hermitian matrix with mean |K_ij|^2 = 1.  P0 = 0.1 instead of the
# printed 1000: at 1000 the Kerr phase is tens of radians per step and the
# spectrum fills every block within twenty steps (the oracle shows it), which
# contradicts the localized bands the paper reports; 0.1 keeps them localized.
MDBP1D_262144_M32_F32 = dict(
    name="mdbp1d_262144_m32_f32",
    op="mdbp", dtype="f32", M=32, n=262144, block=32, steps=5000, seed=1234,
    T=1000.0, dz=0.1, alpha=0.1, beta2=-21.0, gamma=1.3, P0=0.1,
    taus=(1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5),
)

# M = 64, the paper's widest: no FP64 path above M = 32, so the reference is
# the FP32 Regular back-propagation and the threshold is the largest whose
# recovered field stays within err_bar of it
MDBP1D_262144_M64_F32 = dict(MDBP1D_262144_M32_F32, name="mdbp1d_262144_m64_f32", M=64, err_bar=1e-3)

# the printed peak-power parameter P0 = 1000, run to measure what it does to
# the activity (every other parameter as above)
MDBP1D_262144_M32_F32_P1000 = dict(MDBP1D_262144_M32_F32, name="mdbp1d_262144_m32_f32_p1000", P0=1000.0)

MDBP = [MDBP1D_262144_M32_F32, MDBP1D_262144_M64_F32, MDBP1D_262144_M32_F32_P1000]
BY_NAME = {c["name"]: c for c in ALL + RCD + MDBP}
