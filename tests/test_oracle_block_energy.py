"""Pins of the oracle's block-energy measure (the state-based indicator of the
main text's XPFC section, E_B = sum over the block of |q(k)|^2, and the modal
spectral power of S5.3): with the state measure, a_b is the block's sum of
a(k) = sum over species of |q(k)|^2 (k = 0 left out) instead of its maximum.

What fixes it independently of the oracle's code: Parseval (the block sums
add up to N times the real-space variance of the field), exact small-integer
cases (one mode, two modes in one block, both GS species), the relation to
the maximum form (never smaller, equal where a block holds one mode), exact
invariance under power-of-two rescaling, and threshold zero equal to dense.
"""
import numpy as np
import pytest

from paper_2609_03922_amd import inputs


def _ch(o, n, B, tau, ndim=2, energy=True, pin=True, half=False):
    fl = o.FLAG_STATE | (o.FLAG_ENERGY if energy else 0) | (o.FLAG_PIN_K0 if pin else 0) | (o.FLAG_HALF if half else 0)
    dims = tuple([1] * (3 - ndim) + [n] * ndim)
    blk = tuple([1] * (3 - ndim) + [B] * ndim)
    return o.Inst(op=o.OP_CH, dims=dims, block=blk, tau=tau, dx=1.0, dt=0.01, p=(1.0, 1.0), flags=fl)


@pytest.mark.parametrize("ndim,half", [(2, False), (3, False), (2, True)])
def test_block_energies_add_up_to_the_real_space_variance(oracle_mod, ndim, half):
    o = oracle_mod
    n = 32 if ndim == 2 else 16
    c = inputs.uniform_field(1101, ndim, (n,) * ndim, 0.3, 0.1)
    N = c.size
    if half:
        q = o.rfft(c).ravel()
        res = o.apply(_ch(o, n, 8 if ndim == 2 else 4, 0.1, ndim, half=True), q, np.zeros_like(q))
        # the stored columns 1 .. n/2 - 1 stand for their conjugate partners as well
        xs = n // 2 + 1
        nb = res["a_b"]
        rows = (n // 8) ** (ndim - 1)
        # recompute with weights from the stored modes' own |q|^2 (not the oracle's sums)
        a = np.abs(q.reshape(-1, xs)) ** 2
        a[0, 0] = 0.0
        w = np.full(xs, 2.0)
        w[0] = w[-1] = 1.0
        total = float(np.sum(a * w))
        assert abs(total - N * np.sum((c - c.mean()) ** 2)) <= 1e-10 * total
        assert nb.size == rows * (n // 16 + 1)
        assert abs(float(np.sum(nb)) - float(np.sum(a))) <= 1e-12 * float(np.sum(a))
    else:
        q = np.fft.fftn(c).ravel()
        res = o.apply(_ch(o, n, 8 if ndim == 2 else 4, 0.1, ndim), q, np.zeros_like(q))
        var = N * float(np.sum((c - c.mean()) ** 2))
        assert abs(float(np.sum(res["a_b"])) - var) <= 1e-11 * var


def test_one_and_two_modes_exact(oracle_mod):
    o = oracle_mod
    n, B = 16, 4
    q = np.zeros((n, n), np.complex128)
    q[5, 6] = 3.0 - 4.0j          # block (1, 1): 25
    q[6, 7] = 1.0 + 2.0j          # same block: + 5
    q[13, 2] = 2.0                # block (3, 0): 4
    res = o.apply(_ch(o, n, B, 0.2, pin=False), q.ravel(), np.zeros(n * n, np.complex128))
    want = np.zeros((n // B) ** 2)
    want[1 * 4 + 1] = 30.0
    want[3 * 4 + 0] = 4.0
    assert np.array_equal(res["a_b"], want) and res["G"] == 30.0
    # the maximum form keeps 25 for the shared block
    mx = o.apply(_ch(o, n, B, 0.2, energy=False, pin=False), q.ravel(), np.zeros(n * n, np.complex128))
    assert mx["a_b"][5] == 25.0 and mx["a_b"][12] == 4.0
    # fl(0.04 * 30) = 1.2 < 4: both blocks active; at tau = 0.4 (0.16 * 30 = 4.8) only the pair
    assert sorted(np.flatnonzero(res["mask"]).tolist()) == [5, 12]
    res4 = o.apply(_ch(o, n, B, 0.4, pin=False), q.ravel(), np.zeros(n * n, np.complex128))
    assert np.flatnonzero(res4["mask"]).tolist() == [5]


def test_gs_sums_both_species_and_never_below_the_maximum(oracle_mod):
    o = oracle_mod
    n, B = 32, 8
    q = np.concatenate([inputs.shaped_spectrum(61, s, (n, n), width=3.0, floor=1e-3).ravel() for s in range(2)])
    r = np.zeros_like(q)
    mk = lambda fl: o.Inst(op=o.OP_GS, dims=(1, n, n), block=(1, B, B), tau=0.05, dx=1.0, dt=1.0,
                           p=(0.16, 0.08, 0.035, 0.06), flags=fl)
    e = o.apply(mk(o.FLAG_STATE | o.FLAG_ENERGY), q, r)
    m = o.apply(mk(o.FLAG_STATE), q, r)
    assert np.all(e["a_b"] >= m["a_b"]) and np.all(e["a_b"] <= m["a_b"] * B * B)
    u, v = q[: n * n].reshape(n, n), q[n * n:].reshape(n, n)
    tot = np.abs(u) ** 2 + np.abs(v) ** 2
    tot[0, 0] = 0.0
    blocks = tot.reshape(n // B, B, n // B, B).sum(axis=(1, 3)).ravel()
    assert np.allclose(e["a_b"], blocks, rtol=1e-13, atol=0)


def test_power_of_two_rescaling_and_threshold_zero(oracle_mod):
    o = oracle_mod
    n = 32
    q = inputs.shaped_spectrum(62, 0, (n, n), width=4.0, floor=1e-3).ravel()
    r = np.zeros_like(q)
    base = o.apply(_ch(o, n, 8, 0.3), q, r)
    for k in (-4, 3):
        s = o.apply(_ch(o, n, 8, 0.3), q * 2.0 ** k, r)
        assert np.array_equal(s["mask"], base["mask"]) and np.array_equal(s["a_b"], base["a_b"] * 4.0 ** k)
    assert 1 < base["count"] < 16
    c0 = inputs.uniform_field(1001, 4, (n, n), 0.0, 0.05)
    dense = o.step(o.Inst(op=o.OP_CH, dims=(1, n, n), block=(1, 8, 8), tau=0.0, dx=1.0, dt=0.01, p=(1.0, 1.0),
                          flags=o.FLAG_DENSE), o.fft(c0, -1), 20)["state"]
    st = o.step(_ch(o, n, 8, 0.0), o.fft(c0, -1), 20, masks=True)
    assert st["masks"].all() and np.array_equal(st["state"], dense)


def test_energy_needs_the_state_measure(oracle_mod):
    o = oracle_mod
    inst = o.Inst(op=o.OP_CH, dims=(1, 16, 16), block=(1, 4, 4), tau=0.1, dx=1.0, dt=0.01, p=(1.0, 1.0),
                  flags=o.FLAG_ENERGY)
    with pytest.raises(o.OracleError):
        o.apply(inst, np.zeros(256, np.complex128), np.zeros(256, np.complex128))
