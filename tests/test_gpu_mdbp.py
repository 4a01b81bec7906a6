"""Multimode DBP (Supplementary S5) on the GPU through the C ABI against the
oracle.

Bar: the measure, G, the mask and the active count bit-exact (the same FP64
sums of the same values, modes in order); frozen blocks keep their bins bit
for bit; an updated bin agrees with the oracle's U_c(dz/4) h U_c(dz/4) within
(4 M + 16) u ||E|| in FP32 and 16 (M + 4) u ||E|| in FP64 (||E|| the bin's
mode-vector norm, u the unit roundoff): one product with the unitary W of M
terms per row, the scalar h(omega) (|h| <= 1, computed in FP64 and rounded
once), and W rounded once; the oracle's two products with U_c are within a
few u each.
"""
import numpy as np
import pytest

from _parity import assert_bits_equal
from oracle import mdbp as OM
from paper_2609_03922_amd import inputs, mdbp

pytestmark = pytest.mark.gpu

PHYS = dict(T=1000.0, dz=0.1, alpha=0.1, beta2=-21.0, gamma=1.3)


def tol_of(M, dtype):
    return (4 * M + 16) * 2.0 ** -24 if dtype == "f32" else 16 * (M + 4) * 2.0 ** -53


def spectra(seed, M, n, dtype):
    cd = np.complex64 if dtype == "f32" else np.complex128
    return np.stack([inputs.shaped_spectrum(seed, m, (n,), width=n / 64) for m in range(M)]).astype(cd)


CASES = [
    (2, "f32", 4096, 32, 0.05, {}),
    (5, "f32", 8192, 32, 0.05, {}),
    (8, "f32", 16384, 32, 0.03, {}),
    (16, "f32", 4096, 64, 0.05, {}),
    (33, "f32", 4096, 32, 0.05, {}),
    (64, "f32", 2048, 32, 0.05, {}),
    (8, "f32", 4096, 32, 0.05, {"pin_k0": False}),
    (8, "f32", 4096, 32, 0.0, {"dense": True}),
    (64, "f32", 2048, 32, 0.0, {"dense": True}),   # Regular at tile 64: the vector path
    (4, "f64", 4096, 32, 0.05, {}),
    (16, "f64", 4096, 32, 0.05, {}),
    (32, "f64", 2048, 32, 0.05, {}),
]


@pytest.mark.parametrize("case", CASES, ids=[f"M{c[0]}-{c[1]}-n{c[2]}-{i}" for i, c in enumerate(CASES)])
def test_mdbp_half_step_matches_oracle(case):
    import torch

    M, dtype, n, B, tau, extra = case
    print(f"mdbp half-step M={M} {dtype} n={n} B={B} tau={tau} {extra}", flush=True)
    K = inputs.hermitian_coupling(20 + M, M)
    E = spectra(30 + M, M, n, dtype)
    plan = mdbp.MdbpPlan(mdbp.make_desc(M, n, B, dtype=dtype, tau=tau, **PHYS, **extra), K)
    plan.set_spectrum(torch.from_numpy(E.ravel()))
    plan.apply()
    ref = OM.linear_half(E, K, PHYS["T"], PHYS["dz"], PHYS["alpha"], PHYS["beta2"], B, tau,
                         pin_k0=extra.get("pin_k0", True), dense=extra.get("dense", False))
    mask, count = plan.active_mask()
    assert_bits_equal(mask, ref["mask"], "mask")
    assert count == ref["count"]
    if not extra.get("dense"):
        ab, G = plan.indicator()
        assert_bits_equal(ab, ref["a_b"], "a_b")
        assert G == ref["G"]
        assert 0 < count < plan.n_blocks
    got = plan.get_spectrum().cpu().numpy().reshape(M, n)
    plan.destroy()
    act = np.repeat(ref["mask"].astype(bool), B)
    assert_bits_equal(np.ascontiguousarray(got[:, ~act]), np.ascontiguousarray(E[:, ~act]), "frozen bins")
    nrm = np.sqrt(np.sum(np.abs(E[:, act].astype(np.complex128)) ** 2, axis=0))
    err = np.max(np.abs(got[:, act].astype(np.complex128) - ref["E"][:, act]), axis=0)
    ratio = err / np.maximum(nrm, 1e-300)
    assert np.all(ratio <= tol_of(M, dtype)), (float(ratio.max()), tol_of(M, dtype))


@pytest.mark.parametrize("dtype,M,n,steps,tau,bar", [("f64", 4, 1024, 20, 0.01, 1e-11),
                                                     ("f32", 8, 4096, 20, 0.01, 2e-5)])
def test_mdbp_trajectory_matches_oracle(dtype, M, n, steps, tau, bar):
    import torch

    print(f"mdbp trajectory {dtype} M={M} n={n}", flush=True)
    K = inputs.hermitian_coupling(40, M)
    Et = inputs.gaussian_packets(n, PHYS["T"], M, P0=0.1)
    plan = mdbp.MdbpPlan(mdbp.make_desc(M, n, 32, dtype=dtype, tau=tau, **PHYS), K)
    plan.set_field(torch.from_numpy(Et.astype(np.complex64 if dtype == "f32" else np.complex128).ravel()))
    E0 = np.fft.fft(Et.astype(np.complex64).astype(np.complex128) if dtype == "f32" else Et, axis=1)
    ref = OM.step(E0, steps, K, PHYS["T"], PHYS["dz"], PHYS["alpha"], PHYS["beta2"], PHYS["gamma"], 32, tau,
                  masks=True)
    counts, ties = [], 0
    for st in range(steps):
        plan.step(1)
        m, c = plan.active_mask()   # the second half-step of the step
        counts.append(c)
        if not np.array_equal(m, ref["masks"][2 * st + 1]):
            ties += int(np.sum(m != ref["masks"][2 * st + 1]))
    assert ties <= 2
    got = plan.get_spectrum().cpu().numpy().reshape(M, n).astype(np.complex128)
    err = np.linalg.norm(got - ref["state"]) / np.linalg.norm(ref["state"])
    print(f"mdbp trajectory {dtype}: rel-L2 {err:.3e}, active {min(counts)}..{max(counts)} of {plan.n_blocks}",
          flush=True)
    assert err <= bar and min(counts) < plan.n_blocks
    plan.destroy()


def test_mdbp_backpropagation_recovers_the_field():
    """Forward propagation, then back-propagation with reversed parameters
    (-alpha, -beta2, -gamma, -K) on the GPU, FP64, every block updated."""
    import torch

    M, n, steps = 4, 2048, 30
    K = inputs.hermitian_coupling(41, M)
    Et = inputs.gaussian_packets(n, PHYS["T"], M, P0=0.1)
    fwd = mdbp.MdbpPlan(mdbp.make_desc(M, n, 32, dtype="f64", dense=True, **PHYS), K)
    fwd.set_field(torch.from_numpy(Et.ravel()))
    fwd.step(steps)
    rx = fwd.get_spectrum()
    fwd.destroy()
    back = {k: -v for k, v in PHYS.items() if k in ("alpha", "beta2", "gamma")}
    bwd = mdbp.MdbpPlan(mdbp.make_desc(M, n, 32, dtype="f64", dense=True, T=PHYS["T"], dz=PHYS["dz"], **back), -K)
    bwd.set_spectrum(rx)
    bwd.step(steps)
    rec = bwd.get_field().cpu().numpy().reshape(M, n)
    bwd.destroy()
    assert np.linalg.norm(rx.cpu().numpy() - np.fft.fft(Et, axis=1).ravel()) > 0.1 * np.linalg.norm(np.fft.fft(Et, axis=1))
    assert OM.nmse_db(rec, Et) < -200.0


def test_mdbp_dense_equals_threshold_zero():
    import torch

    M, n = 8, 4096
    K = inputs.hermitian_coupling(42, M)
    Et = inputs.gaussian_packets(n, PHYS["T"], M, P0=0.1).astype(np.complex64)
    out = []
    for kw in ({"dense": True}, {"tau": 0.0}):
        p = mdbp.MdbpPlan(mdbp.make_desc(M, n, 32, **{**PHYS, **kw}), K)
        p.set_field(torch.from_numpy(Et.ravel()))
        p.step(5)
        out.append(p.get_spectrum().cpu().numpy())
        p.destroy()
    assert_bits_equal(out[0], out[1], "dense vs tau = 0")


def test_mdbp_graph_replay_equals_eager():
    """Whole steps replayed as a HIP graph give the eager steps' bits (the
    graph is replayed several times, with reads between the replays)."""
    import torch

    M, n = 8, 4096
    K = inputs.hermitian_coupling(43, M)
    Et = inputs.gaussian_packets(n, PHYS["T"], M, P0=0.1).astype(np.complex64)
    plans = [mdbp.MdbpPlan(mdbp.make_desc(M, n, 32, tau=1e-3, graph=g, **PHYS), K) for g in (False, True)]
    for p in plans:
        p.set_field(torch.from_numpy(Et.ravel()))
    for rep in range(3):
        for p in plans:
            p.step(4)
        a, b = (p.get_spectrum().cpu().numpy() for p in plans)
        assert_bits_equal(b, a, f"graph vs eager after {4 * (rep + 1)} steps")
        assert np.array_equal(plans[0].active_mask()[0], plans[1].active_mask()[0])
    for p in plans:
        p.destroy()
