"""RCD (Supplementary S4) on the GPU through the C ABI against the oracle.

Bar: the measure, G, the mask and the active count are bit-exact (the same FP64
sums of FP64-converted inputs in component order); frozen blocks keep their
coefficients bit for bit; an updated mode agrees with the oracle's direct FP64
solve within 4 (M + 2) u ||b|| in FP32 and 16 (M + 2) u ||b|| in FP64, where
b = q + dt R is the mode's component vector and u the unit roundoff.  The
bound follows the eigen form: two contractions with an orthonormal V of M
terms each (|V_j| = 1, so each is within (M + 1) u ||b||), one scaling at most
1, and V rounded to the kernel's precision; the oracle's direct solve is
within a few u (the system's condition number is below 2 here).  The direct
form (Cholesky to M = 8, elimination without pivoting beyond; both backward
stable for a symmetric positive definite matrix, with error of order
(M + 1) u |L||L^T| against a matrix at least I, so that ||x|| <= ||b||)
meets the same bound.
"""
import numpy as np
import pytest

from _parity import assert_bits_equal
from oracle import rcd as OR
from paper_2609_03922_amd import inputs
from paper_2609_03922_amd import rcd

pytestmark = pytest.mark.gpu

P = dict(dt=0.01, dx=0.5, d_diag=0.5, d_cross=0.05, alpha=1.0, beta=0.3)


def dims_of(ndim, n):
    return tuple([1] * (3 - ndim) + [n] * ndim)


def block_of(ndim, b):
    return tuple([1] * (3 - ndim) + [b] * ndim)


def draw(seed, M, dims, dtype, width=3.0, floor=1e-4):
    cd = np.complex128 if dtype == "f64" else np.complex64
    q = np.stack([inputs.shaped_spectrum(seed, m, dims, width=width, floor=floor).ravel() for m in range(M)]).astype(cd)
    r = np.stack([inputs.shaped_spectrum(seed + 50, m, dims, width=width, floor=floor).ravel() for m in range(M)]).astype(cd)
    return q, r


def tol_of(M, dtype):
    return (4.0 * (M + 2) * 2.0 ** -24) if dtype == "f32" else (16.0 * (M + 2) * 2.0 ** -53)


def check_update(got, q, r, ref, M, dtype, tag):
    """Frozen modes bit for bit; updated modes within the bound."""
    bid_mask = ref["mask_modes"]
    assert_bits_equal(np.ascontiguousarray(got[:, ~bid_mask]), np.ascontiguousarray(q[:, ~bid_mask]),
                      tag + " frozen coefficients")
    if bid_mask.any():
        b = q[:, bid_mask].astype(np.complex128) + P["dt"] * r[:, bid_mask].astype(np.complex128)
        nb = np.sqrt(np.sum(np.abs(b) ** 2, axis=0))
        err = np.max(np.abs(got[:, bid_mask].astype(np.complex128) - ref["q"][:, bid_mask]), axis=0)
        ratio = err / np.maximum(nb, 1e-300)
        assert np.all(ratio <= tol_of(M, dtype)), (tag, float(ratio.max()), tol_of(M, dtype))


CASES = [
    # (M, dtype, ndim, n, block, tau, extra)
    (2, "f32", 3, 32, 8, 0.05, {}),
    (3, "f32", 3, 32, 4, 0.05, {}),
    (8, "f32", 3, 32, 8, 0.03, {}),
    (16, "f32", 2, 64, 8, 0.05, {}),
    (5, "f32", 1, 4096, 256, 0.05, {}),
    (8, "f32", 3, 32, 8, 0.03, {"pin_k0": False}),
    (8, "f32", 3, 32, 8, 0.0, {"dense": True}),
    (5, "f64", 3, 16, 4, 0.05, {}),
    (8, "f64", 2, 64, 16, 0.05, {}),
    (2, "f64", 1, 2048, 128, 0.05, {}),
    # wide components (FP32, b staged in LDS): tiles 32 and 64
    (24, "f32", 3, 16, 4, 0.05, {}),
    (33, "f32", 2, 32, 8, 0.05, {}),
    (48, "f32", 3, 16, 4, 0.05, {}),
    (64, "f32", 3, 16, 4, 0.05, {}),
    (48, "f32", 3, 16, 4, 0.0, {"dense": True}),
    # FP64 on the matrix cores: tiles 16, 32, 48
    (12, "f64", 3, 16, 4, 0.05, {}),
    (24, "f64", 3, 16, 4, 0.05, {}),
    (48, "f64", 3, 16, 4, 0.05, {}),
    # the direct form of S4.2 (per-mode Cholesky of I + dt k^2 D)
    (2, "f32", 3, 32, 8, 0.05, {"direct": True}),
    (3, "f32", 3, 32, 4, 0.05, {"direct": True}),
    (8, "f32", 3, 32, 8, 0.03, {"direct": True}),
    (8, "f32", 3, 32, 8, 0.0, {"direct": True, "dense": True}),
    (5, "f64", 3, 16, 4, 0.05, {"direct": True}),
    (8, "f64", 2, 64, 16, 0.05, {"direct": True}),
    # wide systems: one wave's elimination per mode (tiles 16, 32, 48, 64)
    (12, "f32", 3, 16, 4, 0.05, {"direct": True}),
    (24, "f32", 3, 16, 4, 0.05, {"direct": True}),
    (33, "f32", 2, 32, 8, 0.05, {"direct": True}),
    (48, "f32", 3, 16, 4, 0.05, {"direct": True}),
    (64, "f32", 3, 16, 4, 0.05, {"direct": True}),
    (48, "f32", 3, 16, 4, 0.0, {"direct": True, "dense": True}),
    (16, "f64", 2, 64, 8, 0.05, {"direct": True}),
    (24, "f64", 3, 16, 4, 0.05, {"direct": True}),
    (48, "f64", 3, 16, 4, 0.05, {"direct": True}),
    # tile edges of the wave form: identity rows from lane M on (17 in tile
    # 32, 49 in tile 64), a full tile (32), one row short of it (31, FP64)
    (17, "f32", 3, 16, 4, 0.05, {"direct": True}),
    (32, "f32", 2, 32, 8, 0.05, {"direct": True}),
    (49, "f32", 3, 16, 4, 0.05, {"direct": True}),
    (31, "f64", 3, 16, 4, 0.05, {"direct": True, "pin_k0": False}),
]


@pytest.mark.parametrize("case", CASES, ids=[f"M{c[0]}-{c[1]}-{c[2]}d{c[3]}-b{c[4]}-{i}" for i, c in enumerate(CASES)])
def test_rcd_apply_matches_oracle(case):
    import torch

    M, dtype, ndim, n, bl, tau, extra = case
    print(f"rcd apply M={M} {dtype} {ndim}-D n={n} block={bl} tau={tau} {extra}", flush=True)
    dims, block = dims_of(ndim, n), block_of(ndim, bl)
    q, r = draw(200 + M + n, M, dims, dtype)
    plan = rcd.RcdPlan(rcd.make_desc(M, ndim, n, bl, dtype=dtype, tau=tau, **P, **extra))
    plan.set_spectrum(torch.from_numpy(q.ravel()))
    plan.apply(torch.from_numpy(r.ravel()))
    ref = OR.apply(q, r, dims, block, tau, P["dt"], P["dx"], P["d_diag"], P["d_cross"],
                   pin_k0=extra.get("pin_k0", True), dense=extra.get("dense", False))
    mask, count = plan.active_mask()
    assert_bits_equal(mask, ref["mask"], "mask")
    assert count == ref["count"]
    if not extra.get("dense"):
        ab, G = plan.indicator()
        assert_bits_equal(ab, ref["a_b"], "a_b")
        assert G == ref["G"]
        assert 0 < count < plan.n_blocks, (count, plan.n_blocks)
    ref["mask_modes"] = ref["mask"][OR.block_ids(dims, block)].astype(bool)
    got = plan.get_spectrum().cpu().numpy().reshape(M, -1)
    check_update(got, q, r, ref, M, dtype, f"M={M} {dtype}")
    plan.destroy()


@pytest.mark.parametrize("M,direct", [(4, False), (4, True), (24, True)])
def test_rcd_no_active_block_leaves_state_unchanged(M, direct):
    import torch

    dims = (32, 32, 32)
    q, r = draw(301, M, dims, "f32")
    plan = rcd.RcdPlan(rcd.make_desc(M, 3, 32, 8, tau=2.0, pin_k0=False, direct=direct, **P))  # tau^2 G > every a_b
    plan.set_spectrum(torch.from_numpy(q.ravel()))
    plan.apply(torch.from_numpy(r.ravel()))
    mask, count = plan.active_mask()
    assert count == 0 and not mask.any()
    assert_bits_equal(plan.get_spectrum().cpu().numpy(), q.ravel(), "untouched state")
    plan.destroy()


def test_rcd_dense_equals_threshold_zero():
    import torch

    M, n = 8, 32
    u0 = inputs.perturbed_components(302, M, (n, n, n), OR.equilibrium(M, 1.0, 0.3), 0.1, dtype=np.float32)
    out = []
    for kw in ({"dense": True}, {"tau": 0.0}):
        plan = rcd.RcdPlan(rcd.make_desc(M, 3, n, 8, **{**P, **kw}))
        plan.set_field(torch.from_numpy(u0.ravel()))
        plan.step(5)
        out.append(plan.get_spectrum().cpu().numpy())
        plan.destroy()
    assert_bits_equal(out[0], out[1], "dense vs tau = 0")


def test_rcd_field_round_trip():
    import torch

    M, n = 3, 32
    u0 = inputs.perturbed_components(303, M, (n, n), 0.2, 0.1)
    plan = rcd.RcdPlan(rcd.make_desc(M, 2, n, 8, dtype="f64", **P))
    plan.set_field(torch.from_numpy(u0.ravel()))
    back = plan.get_field().cpu().numpy()
    assert np.max(np.abs(back - u0.ravel())) <= 1e-15
    hat = plan.get_spectrum().cpu().numpy().reshape(M, -1)
    want = np.stack([np.fft.fftn(u0[m]).ravel() for m in range(M)])
    assert np.max(np.abs(hat - want)) <= 1e-12 * np.max(np.abs(want))
    plan.destroy()


@pytest.mark.parametrize("dtype,M,n,steps,tau,direct", [
    ("f64", 4, 16, 25, 0.02, False), ("f32", 8, 32, 10, 0.1, False), ("f32", 24, 16, 25, 0.1, False),
    ("f32", 40, 16, 25, 0.1, False), ("f32", 64, 16, 25, 0.1, False), ("f64", 24, 16, 25, 0.1, False),
    ("f32", 48, 16, 25, 0.1, True), ("f64", 24, 16, 25, 0.1, True)])
def test_rcd_trajectory_matches_oracle(dtype, M, n, steps, tau, direct):
    """Full steps (transforms, Lotka--Volterra reaction, measure, update) from a
    perturbed homogeneous state: masks of every step agree with the oracle's
    except at near-ties; the final field within the precision's bar."""
    import torch

    print(f"rcd trajectory {dtype} M={M} n={n} steps={steps} tau={tau} direct={direct}", flush=True)
    dims = (n, n, n)
    u0 = inputs.perturbed_components(304, M, dims, OR.equilibrium(M, 1.0, 0.3), 0.1)
    if dtype == "f32":
        u0 = u0.astype(np.float32)
    plan = rcd.RcdPlan(rcd.make_desc(M, 3, n, 4, dtype=dtype, tau=tau, direct=direct, **P))
    plan.set_field(torch.from_numpy(u0.ravel()))
    q0 = np.stack([np.fft.fftn(u0[m].astype(np.float64)).ravel() for m in range(M)])
    ref = OR.step(q0, steps, dims, (4, 4, 4), tau, P["dt"], P["dx"], P["d_diag"], P["d_cross"], 1.0, 0.3,
                  masks=True)
    ties, seen = 0, set()
    for st in range(steps):
        plan.step(1)
        m, c = plan.active_mask()
        seen.add(c)
        if not np.array_equal(m, ref["masks"][st]):
            ab, G = plan.indicator()
            bad = np.flatnonzero(m != ref["masks"][st])
            thr = tau * tau * G
            assert np.all(np.abs(ab[bad] - thr) <= 1e-6 * thr), (st, bad[:8])
            ties += bad.size
    assert ties <= 2
    got = plan.get_spectrum().cpu().numpy().reshape(M, -1).astype(np.complex128)
    err = np.linalg.norm(got - ref["state"]) / np.linalg.norm(ref["state"])
    print(f"rcd trajectory {dtype}: rel-L2 {err:.3e}, active counts {sorted(seen)[:5]}..{max(seen)}", flush=True)
    assert err <= (1e-12 if dtype == "f64" else 1e-5)
    assert min(seen) < plan.n_blocks
    plan.destroy()


def test_rcd_full_size_sampled():
    """256^3, M = 8, FP32, 8^3 blocks (the size of the paper's three-layer
    figure): the measure, mask and count over the whole grid bit-exact against
    the oracle's measure; 4096 sampled modes of active blocks within the bar;
    4096 sampled modes of frozen blocks bit for bit."""
    import torch

    M, n, bl, tau = 8, 256, 8, 0.03
    print("rcd full size 256^3 M=8 apply", flush=True)
    dims, block = (n, n, n), (bl, bl, bl)
    q, r = draw(305, M, dims, "f32", width=6.0)
    plan = rcd.RcdPlan(rcd.make_desc(M, 3, n, bl, tau=tau, **P))
    plan.set_spectrum(torch.from_numpy(q.ravel()))
    plan.apply(torch.from_numpy(r.ravel()))
    mask, count = plan.active_mask()
    ab, G = plan.indicator()
    got = plan.get_spectrum().cpu().numpy().reshape(M, -1)
    plan.destroy()
    a = OR.measure(q)
    bid = OR.block_ids(dims, block)
    want_ab = np.zeros(plan.n_blocks)
    np.maximum.at(want_ab, bid, a)
    assert_bits_equal(ab, want_ab, "a_b")
    assert G == want_ab.max()
    want_mask = (want_ab > (tau * tau) * G).astype(np.uint8)
    want_mask[0] = 1
    assert_bits_equal(mask, want_mask, "mask")
    assert count == int(want_mask.sum()) and 0 < count < plan.n_blocks
    act = want_mask[bid].astype(bool)
    rng = np.random.default_rng(9)
    ia = rng.choice(np.flatnonzero(act), 4096, replace=False)
    ifz = rng.choice(np.flatnonzero(~act), 4096, replace=False)
    assert_bits_equal(np.ascontiguousarray(got[:, ifz]), np.ascontiguousarray(q[:, ifz]), "frozen sample")
    x = OR.update_modes(q[:, ia].astype(np.complex128), r[:, ia].astype(np.complex128), OR.k2(dims, P["dx"])[ia],
                        P["dt"], OR.diffusion_matrix(M, P["d_diag"], P["d_cross"]))
    b = q[:, ia].astype(np.complex128) + P["dt"] * r[:, ia].astype(np.complex128)
    ratio = np.max(np.abs(got[:, ia] - x), axis=0) / np.sqrt(np.sum(np.abs(b) ** 2, axis=0))
    assert np.all(ratio <= tol_of(M, "f32")), float(ratio.max())


@pytest.mark.parametrize("M,dtype,ndim,n,bl,tau,direct", [
    (8, "f32", 3, 32, 8, 0.03, False), (4, "f64", 2, 64, 8, 0.05, False), (16, "f32", 2, 64, 16, 0.05, False),
    (48, "f32", 3, 16, 4, 0.05, False), (8, "f32", 3, 32, 8, 0.03, True), (48, "f32", 3, 16, 4, 0.05, True),
    (24, "f64", 3, 16, 4, 0.05, True)])
def test_rcd_kept_measure_over_a_sequence(M, dtype, ndim, n, bl, tau, direct):
    """From the second update on, the measure is the one the last update kept
    for the blocks it stored (frozen blocks unchanged): before every update the
    oracle gets the GPU's current state, and a_b, G, mask and count agree bit
    for bit; a reload in the middle forces a full pass."""
    import torch

    print(f"rcd kept-measure sequence M={M} {dtype} {ndim}-D n={n} direct={direct}", flush=True)
    dims, block = dims_of(ndim, n), block_of(ndim, bl)
    q, _ = draw(400 + M, M, dims, dtype)
    plan = rcd.RcdPlan(rcd.make_desc(M, ndim, n, bl, dtype=dtype, tau=tau, direct=direct, **P))
    plan.set_spectrum(torch.from_numpy(q.ravel()))
    counts = []
    for step in range(6):
        if step == 3:  # reload the same state: the next update measures in full
            plan.set_spectrum(plan.get_spectrum())
        cur = plan.get_spectrum().cpu().numpy().reshape(M, -1)
        _, r = draw(500 + 10 * M + step, M, dims, dtype)
        plan.apply(torch.from_numpy(r.ravel()))
        ref = OR.apply(cur, r, dims, block, tau, P["dt"], P["dx"], P["d_diag"], P["d_cross"])
        mask, count = plan.active_mask()
        ab, G = plan.indicator()
        tag = f"update {step}"
        assert_bits_equal(ab, ref["a_b"], tag + " a_b")
        assert G == ref["G"], tag
        assert_bits_equal(mask, ref["mask"], tag + " mask")
        assert count == ref["count"]
        counts.append(count)
        ref["mask_modes"] = ref["mask"][OR.block_ids(dims, block)].astype(bool)
        check_update(plan.get_spectrum().cpu().numpy().reshape(M, -1), cur, r, ref, M, dtype, tag)
    assert any(0 < c < plan.n_blocks for c in counts), counts
    plan.destroy()
