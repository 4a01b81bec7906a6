"""Pins of the oracle's state-amplitude activity measure (the paper's
state-based indicators: block energy in the main text's XPFC section, the
component RMS amplitude with "any mode above" of Supplementary S4.2, the modal
spectral power of S5.3): a(k) = sum over species of |q(k)|^2 of the state
entering the update, block maximum, k = 0 left out.

The pins rest on properties the definition fixes: the measure does not see
the right-hand side; a single mode gives exactly one active block with its
squared modulus; an exact power-of-two rescaling changes nothing; k = 0 is
excluded; at threshold zero the rule reduces to the dense update; the update
itself is the candidate of the plain rule.
"""
import numpy as np
import pytest

from paper_2609_03922_amd import inputs


def _ch(o, n, B, tau, state=True, pin=True, ndim=2):
    fl = (o.FLAG_STATE if state else 0) | (o.FLAG_PIN_K0 if pin else 0)
    dims = tuple([1] * (3 - ndim) + [n] * ndim)
    blk = tuple([1] * (3 - ndim) + [B] * ndim)
    return o.Inst(op=o.OP_CH, dims=dims, block=blk, tau=tau, dx=1.0, dt=0.01, p=(1.0, 1.0), flags=fl)


def _block_of(n, B, iy, ix):
    return (iy // B) * (n // B) + ix // B


def test_state_measure_ignores_rhs(oracle_mod):
    o = oracle_mod
    n, B = 32, 8
    q = inputs.shaped_spectrum(51, 0, (n, n), width=3.0).ravel()
    r1 = inputs.shaped_spectrum(51, 1, (n, n), width=2.0, scale=3.0).ravel()
    r2 = inputs.shaped_spectrum(51, 2, (n, n), width=9.0, scale=0.1).ravel()
    a = o.apply(_ch(o, n, B, 0.05), q, r1)
    b = o.apply(_ch(o, n, B, 0.05), q, r2)
    assert np.array_equal(a["a_b"], b["a_b"]) and np.array_equal(a["mask"], b["mask"])
    assert a["G"] == b["G"]
    # the increment rule does see it
    c = o.apply(_ch(o, n, B, 0.05, state=False), q, r1)
    d = o.apply(_ch(o, n, B, 0.05, state=False), q, r2)
    assert not np.array_equal(c["a_b"], d["a_b"])


@pytest.mark.parametrize("f32", [False, True])
def test_single_mode_activates_exactly_its_block(oracle_mod, f32):
    o = oracle_mod
    n, B = 32, 4
    q = np.zeros(n * n, np.complex128)
    iy, ix = 9, 27  # block (2, 6)
    z = 3.0 - 4.0j  # |z|^2 = 25 exactly
    q[iy * n + ix] = z
    rhs = np.zeros_like(q)
    inst = _ch(o, n, B, 1e-3, pin=False)
    if f32:
        res = o.apply(inst, q.astype(np.complex64), rhs.astype(np.complex64), dtype="f32",
                      k0=np.array([0.0]), rhs_k0=np.array([0.0]))
    else:
        res = o.apply(inst, q, rhs)
    b = _block_of(n, B, iy, ix)
    want_ab = np.zeros((n // B) ** 2)
    want_ab[b] = 25.0
    assert np.array_equal(res["a_b"], want_ab)
    assert res["G"] == 25.0
    assert np.flatnonzero(res["mask"]).tolist() == [b]


def test_power_of_two_rescaling_keeps_the_mask(oracle_mod):
    """a scales by exactly 4^k under q -> 2^k q, and so do G and fl(tau^2 G):
    every decision is unchanged bit for bit (also for GS, two species)."""
    o = oracle_mod
    n, B = 32, 8
    q = inputs.shaped_spectrum(52, 0, (n, n), width=4.0, floor=1e-3).ravel()
    r = inputs.shaped_spectrum(52, 1, (n, n), width=3.0).ravel()
    base = o.apply(_ch(o, n, B, 0.02), q, r)
    for k in (-3, 5):
        s = o.apply(_ch(o, n, B, 0.02), q * 2.0 ** k, r)
        assert np.array_equal(s["mask"], base["mask"])
        assert np.array_equal(s["a_b"], base["a_b"] * 4.0 ** k)
    assert 1 < base["count"] < (n // B) ** 2
    gs = lambda: o.Inst(op=o.OP_GS, dims=(1, n, n), block=(1, B, B), tau=0.02, dx=1.0, dt=1.0,
                        p=(0.16, 0.08, 0.035, 0.06), flags=o.FLAG_STATE | o.FLAG_PIN_K0)
    q2 = np.concatenate([q, inputs.shaped_spectrum(52, 2, (n, n), width=2.0).ravel()])
    r2 = np.concatenate([r, r])
    g0 = o.apply(gs(), q2, r2)
    g1 = o.apply(gs(), q2 * 2.0 ** 7, r2)
    assert np.array_equal(g0["mask"], g1["mask"])
    assert np.array_equal(g1["a_b"], g0["a_b"] * 4.0 ** 7)


def test_gs_state_measure_sums_both_species(oracle_mod):
    """A mode carried by v alone counts as much as the same mode in u."""
    o = oracle_mod
    n, B = 16, 4
    q = np.zeros(2 * n * n, np.complex128)
    q[3 * n + 5] = 2.0            # u at (3, 5), block (0, 1)
    q[n * n + 13 * n + 6] = 2.0j  # v at (13, 6), block (3, 1)
    rhs = np.zeros_like(q)
    inst = o.Inst(op=o.OP_GS, dims=(1, n, n), block=(1, B, B), tau=0.5, dx=1.0, dt=1.0,
                  p=(0.16, 0.08, 0.035, 0.06), flags=o.FLAG_STATE)
    res = o.apply(inst, q, rhs)
    assert res["a_b"][_block_of(n, B, 3, 5)] == 4.0
    assert res["a_b"][_block_of(n, B, 13, 6)] == 4.0
    assert sorted(np.flatnonzero(res["mask"]).tolist()) == sorted([_block_of(n, B, 3, 5), _block_of(n, B, 13, 6)])


def test_k0_left_out_of_the_measure(oracle_mod):
    """A dominant k = 0 coefficient (the mean) neither enters a_b of block 0
    nor sets G; block 0 stays active through the pin."""
    o = oracle_mod
    n, B = 16, 4
    q = np.zeros(n * n, np.complex128)
    q[0] = 1e6
    q[1] = 1.0      # block 0, |q|^2 = 1
    q[7 * n + 9] = 0.5  # block (1, 2), |q|^2 = 0.25
    res = o.apply(_ch(o, n, B, 0.6), q, np.zeros_like(q))
    assert res["a_b"][0] == 1.0 and res["G"] == 1.0
    # 0.25 <= fl(0.36 * 1): only the pinned block
    assert np.flatnonzero(res["mask"]).tolist() == [0]
    res = o.apply(_ch(o, n, B, 0.4), q, np.zeros_like(q))
    assert sorted(np.flatnonzero(res["mask"]).tolist()) == [0, _block_of(n, B, 7, 9)]


def test_state_threshold_zero_equals_dense_trajectory(oracle_mod):
    """With tau = 0 every block holding a nonzero mode is active: a generic
    state reproduces the dense trajectory bit for bit."""
    o = oracle_mod
    n = 64
    c0 = inputs.uniform_field(1001, 3, (n, n), 0.0, 0.05)
    chat = np.fft.fft2(c0)
    dense = o.step(_ch(o, n, 16, 0.0, state=False, pin=True), chat, 30)["state"]
    dflag = o.Inst(op=o.OP_CH, dims=(1, n, n), block=(1, 16, 16), tau=0.0, dx=1.0, dt=0.01,
                   p=(1.0, 1.0), flags=o.FLAG_DENSE)
    ref = o.step(dflag, chat, 30)["state"]
    st = o.step(_ch(o, n, 16, 0.0), chat, 30, masks=True)
    assert np.array_equal(st["state"], ref) and np.array_equal(dense, ref)
    assert st["masks"].all()


def test_state_rule_updates_active_blocks_with_the_plain_candidate(oracle_mod):
    """The measure changes only the selection: on the blocks it activates the
    coefficients equal those of the increment rule at threshold zero (every
    block active), elsewhere the input."""
    o = oracle_mod
    n, B = 32, 8
    q = inputs.shaped_spectrum(53, 0, (n, n), width=3.0, floor=1e-4).ravel()
    r = inputs.shaped_spectrum(53, 1, (n, n), width=2.0, scale=3.0).ravel()
    st = o.apply(_ch(o, n, B, 0.01), q, r)
    full = o.apply(_ch(o, n, B, 0.0, state=False), q, r)
    assert full["mask"].all() and 1 < st["count"] < (n // B) ** 2
    for i in range(n * n):
        b = _block_of(n, B, i // n, i % n)
        want = full["q"][i] if st["mask"][b] else q[i]
        assert st["q"][i] == want
