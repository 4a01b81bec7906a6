"""Pins of the CPU oracle against facts fixed by the mathematics, not by itself.

Each test names the passage of the paper (or the textbook fact) it rests on.
A plausible slip anywhere in the oracle -- a dropped term, a wrong sign, a
transposed operand, a wrong wavenumber scale, a wrong block index, a
mis-ordered threshold -- fails at least one of these.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2609_03922_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def brute_dft(a, sign):
    """Direct O(N^2) DFT along every axis (textbook definition)."""
    out = np.asarray(a, np.complex128)
    for ax in range(out.ndim):
        n = out.shape[ax]
        j = np.arange(n)
        W = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
        out = np.moveaxis(np.tensordot(W, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    if sign > 0:
        out = out / out.size
    return out


# ---------------------------------------------------------------------------
# FFT
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(2,), (8,), (256,), (16, 16), (4, 32), (8, 8, 8)])
def test_fft_matches_brute_dft(oracle_mod, shape):
    r = np.random.default_rng(7)
    a = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    for sign in (-1, 1):
        ref = brute_dft(a, sign)
        got = oracle_mod.fft(a, sign)
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()) * 10


def test_fft_roundtrip_parseval_and_numpy(oracle_mod):
    r = np.random.default_rng(8)
    a = r.standard_normal((16, 32, 8)) + 1j * r.standard_normal((16, 32, 8))
    A = oracle_mod.fft(a, -1)
    assert np.allclose(A, np.fft.fftn(a), rtol=0, atol=1e-11)
    back = oracle_mod.fft(A, +1)
    assert np.abs(back - a).max() < 1e-13
    assert abs(np.sum(np.abs(A) ** 2) / a.size - np.sum(np.abs(a) ** 2)) < 1e-10


# ---------------------------------------------------------------------------
# sin/cos used for the split-step factor
# ---------------------------------------------------------------------------

def test_sincos_within_two_ulp_of_libm(oracle_mod):
    xs = np.concatenate([np.linspace(-0.3, 0.3, 601), np.linspace(-40, 40, 2001),
                         [1e-300, 1e-9, -1e-9, math.pi / 4, math.pi / 2, 3 * math.pi]])
    for x in xs:
        s, c = oracle_mod.sincos(float(x))
        for got, ref in ((s, math.sin(x)), (c, math.cos(x))):
            ulp = math.ulp(max(abs(ref), 1e-300))
            # near zeros of sin/cos the absolute error is bounded by ulp(1)*|x|-ish
            tol = 2 * ulp if abs(ref) > 1e-3 else 4 * math.ulp(1.0) * max(1.0, abs(x)) / 4
            assert abs(got - ref) <= tol, (x, got, ref)


# ---------------------------------------------------------------------------
# Cahn-Hilliard step: linearised growth, pure relaxation, mass, energy
# ---------------------------------------------------------------------------

def _ch_inst(oracle_mod, n, ndim=2, block=8, dx=1.0, dt=0.01, tau=0.0, flags=None, M=1.0, kap=1.0):
    o = oracle_mod
    return o.Inst(op=o.OP_CH, dims=inputs.dims3(ndim, n), block=inputs.block3(ndim, block),
                  tau=tau, dx=dx, dt=dt, p=(M, kap), flags=o.FLAG_DENSE if flags is None else flags)


def _load_growth():
    rows = []
    with open(os.path.join(GOLD, "ch_linear_growth.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, dx, m, k, g = line.split()
                rows.append((int(n), float(dx), int(m), float(k), float(g)))
    return rows


@pytest.mark.parametrize("row", _load_growth())
def test_ch_linear_growth_golden(oracle_mod, row):
    """A small single mode grows by g(k) per step (golden values, closed form)."""
    n, dx, m, k, g = row
    inst = _ch_inst(oracle_mod, n, ndim=2, dx=dx)
    eps = 1e-7
    x = np.arange(n)
    c = eps * np.cos(2 * np.pi * m * x / n)[None, :] * np.ones((n, 1))
    chat = np.fft.fft2(c)
    res = oracle_mod.step(inst, chat, 3)
    ratio = res["state"].reshape(n, n)[0, m].real / chat[0, m].real
    assert abs(ratio - g ** 3) <= 1e-10 * g ** 3
    # the grid wavenumber the golden row assumes
    assert abs(2 * np.pi * m / (n * dx) - k) < 1e-12


def test_ch_pure_relaxation_closed_form(oracle_mod):
    """Zero nonlinear right-hand side: c-hat^n = c-hat^0 (1 + dt M kappa k^4)^-n."""
    n, steps = 32, 7
    inst = _ch_inst(oracle_mod, n, ndim=2, block=8, dx=0.7, M=1.3, kap=0.8, dt=0.05)
    q = inputs.shaped_spectrum(11, 0, (n, n), width=6.0)
    zero = np.zeros_like(q)
    cur = q.copy()
    for _ in range(steps):
        cur = oracle_mod.apply(inst, cur, zero)["q"]
    m = np.fft.fftfreq(n, 1.0 / n)
    k2 = (2 * np.pi / (n * 0.7)) ** 2 * (m[:, None] ** 2 + m[None, :] ** 2)
    ref = q * (1 + 0.05 * 1.3 * 0.8 * k2 ** 2) ** (-steps)
    assert np.abs(cur.reshape(n, n) - ref).max() <= 1e-13 * steps * np.abs(q).max()


def test_ch_linear_response_to_rhs(oracle_mod):
    """c' = (c - dt M k^2 N)/(1 + dt M kappa k^4) for an arbitrary N (one step)."""
    n = 16
    inst = _ch_inst(oracle_mod, n, ndim=3, block=4, dx=1.1, M=0.7, kap=1.9, dt=0.02)
    q = inputs.shaped_spectrum(12, 0, (n, n, n), width=4.0)
    N = inputs.shaped_spectrum(12, 1, (n, n, n), width=3.0)
    got = oracle_mod.apply(inst, q, N)["q"].reshape(n, n, n)
    m = np.fft.fftfreq(n, 1.0 / n)
    K = 2 * np.pi / (n * 1.1)
    k2 = K * K * (m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2)
    ref = (q - 0.02 * 0.7 * k2 * N) / (1 + 0.02 * 0.7 * 1.9 * k2 ** 2)
    assert np.abs(got - ref).max() <= 4e-16 * np.abs(ref).max() * 8


@pytest.mark.parametrize("tau", [0.0, 1e-3])
def test_ch_mass_bit_exact_and_energy_decreases(oracle_mod, tau):
    """Mean density conserved exactly (S6.1 keeps the k=0 block active); free
    energy does not increase for the dense update at these parameters."""
    n = 64
    o = oracle_mod
    flags = o.FLAG_DENSE if tau == 0.0 else o.FLAG_PIN_K0
    inst = _ch_inst(o, n, ndim=2, block=16, tau=tau, flags=flags)
    c0 = inputs.uniform_field(1001, 0, (n, n), 0.0, 0.05)
    chat = np.fft.fft2(c0)
    res = o.step(inst, chat, 150, diag=True)
    mass = res["diag"][:, 0]
    assert np.all(mass == mass[0])
    assert res["state"][0] == chat[0, 0]
    if tau == 0.0:
        F = res["diag"][:, 1]
        assert np.all(F[1:] <= F[:-1] * (1 + 1e-12) + 1e-15)


def test_ch_energy_single_mode_closed_form(oracle_mod):
    """F for c = cbar + A cos(k x): bulk term by quadrature of (c^2-1)^2/4 and
    gradient term kappa/2 * A^2 k^2 / 2 per unit area (exact for one mode)."""
    n, dx, A, cbar, kap = 64, 0.5, 0.3, 0.1, 1.7
    inst = _ch_inst(oracle_mod, n, ndim=2, dx=dx, kap=kap)
    m = 3
    x = np.arange(n)
    c = cbar + A * np.cos(2 * np.pi * m * x / n)[None, :] * np.ones((n, 1))
    F, mass = oracle_mod.ch_energy(inst, np.fft.fft2(c))
    k = 2 * np.pi * m / (n * dx)
    area = (n * dx) ** 2
    bulk = dx * dx * np.sum(0.25 * (c ** 2 - 1) ** 2)
    assert abs(F - (bulk + 0.5 * kap * A * A * k * k / 2 * area)) < 1e-10 * abs(F)
    assert abs(mass - cbar) < 1e-15


# ---------------------------------------------------------------------------
# Threshold 0 equals dense; the adaptive bookkeeping
# ---------------------------------------------------------------------------

def test_threshold_zero_equals_dense_ch(oracle_mod):
    o = oracle_mod
    n = 64
    c0 = inputs.uniform_field(1001, 0, (n, n), 0.0, 0.05)
    chat = np.fft.fft2(c0)
    dense = o.step(_ch_inst(o, n, 2, 16, tau=0.0, flags=o.FLAG_DENSE), chat, 40)["state"]
    ad = o.step(_ch_inst(o, n, 2, 16, tau=0.0, flags=o.FLAG_PIN_K0), chat, 40, masks=True)
    assert np.array_equal(dense, ad["state"])


def test_threshold_zero_equals_dense_gs_and_nlse(oracle_mod):
    o = oracle_mod
    n = 64
    u, v = inputs.gs_patch_field(1004, 0, n, dtype=np.float64)
    st = np.concatenate([np.fft.fft2(u).ravel(), np.fft.fft2(v).ravel()])
    mk = lambda fl: o.Inst(op=o.OP_GS, dims=(1, n, n), block=(1, 16, 16), tau=0.0, dx=1.0,
                           dt=1.0, p=(0.16, 0.08, 0.035, 0.06), flags=fl)
    a = o.step(mk(o.FLAG_DENSE), st, 30)["state"]
    b = o.step(mk(o.FLAG_PIN_K0), st, 30)["state"]
    assert np.array_equal(a, b)
    E = inputs.qam16_rrc_signal(1003, 0, 4096).astype(np.complex128)
    mk2 = lambda fl: o.Inst(op=o.OP_NLSE, dims=(1, 1, 4096), block=(1, 1, 256), tau=0.0,
                            dx=15.625, dt=0.8, p=(-21.7, 1.3, 0.0), flags=fl)
    a = o.step(mk2(o.FLAG_DENSE), E, 10)["state"]
    b = o.step(mk2(o.FLAG_PIN_K0), E, 10)["state"]
    assert np.array_equal(a, b)


def _nlse_H(n, dx, h, beta2, alpha):
    w = 2 * np.pi * np.fft.fftfreq(n, 1.0 / n) / (n * dx)
    return np.exp((-alpha / 2 + 1j * beta2 * w * w / 2) * h / 2)


def test_nlse_linear_adaptive_bookkeeping(oracle_mod):
    """gamma = 0: every half step is linear, so E-hat^n(k) = H(k)^A(b) E-hat^0(k)
    with A(b) the number of half steps block b was active (frozen = identity)."""
    o = oracle_mod
    n, h, beta2, alpha, dx = 8192, 0.8, -21.7, 0.05, 15.625
    inst = o.Inst(op=o.OP_NLSE, dims=(1, 1, n), block=(1, 1, 512), tau=3e-3, dx=dx, dt=h,
                  p=(beta2, 0.0, alpha), flags=o.FLAG_PIN_K0)
    E0 = inputs.qam16_rrc_signal(1003, 1, n).astype(np.complex128)
    res = o.step(inst, E0, 12, masks=True)
    A = res["active_steps"]
    assert 0 < A.sum() < 24 * inst.n_blocks  # some blocks were frozen some of the time
    H = _nlse_H(n, dx, h, beta2, alpha)
    blk = np.arange(n) // 512
    ref = np.fft.ifft(np.fft.fft(E0) * H ** A[blk])
    assert np.abs(res["state"] - ref).max() <= 1e-13 * 24 * np.abs(E0).max()


def test_nlse_dispersion_only_dense_closed_form(oracle_mod):
    o = oracle_mod
    n, h, beta2, alpha, dx, steps = 4096, 0.8, -21.7, 0.1, 15.625, 9
    inst = o.Inst(op=o.OP_NLSE, dims=(1, 1, n), block=(1, 1, 256), tau=0.0, dx=dx, dt=h,
                  p=(beta2, 0.0, alpha), flags=o.FLAG_DENSE)
    E0 = inputs.qam16_rrc_signal(1003, 2, n).astype(np.complex128)
    got = o.step(inst, E0, steps)["state"]
    w = 2 * np.pi * np.fft.fftfreq(n, 1.0 / n) / (n * dx)
    ref = np.fft.ifft(np.fft.fft(E0) * np.exp(1j * beta2 * w * w * steps * h / 2)
                      * np.exp(-alpha * steps * h / 2))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(E0).max()


def test_nlse_kerr_only_and_power_conservation(oracle_mod):
    """beta2 = 0: |E| invariant, phase gamma |E|^2 n h.  alpha = 0: sum |E|^2
    conserved by dense and adaptive runs (each half step unitary or identity)."""
    o = oracle_mod
    n, h, gam = 2048, 0.8, 1.3
    E0 = inputs.qam16_rrc_signal(1003, 3, n).astype(np.complex128) * 30
    inst = o.Inst(op=o.OP_NLSE, dims=(1, 1, n), block=(1, 1, 128), tau=0.0, dx=15.625, dt=h,
                  p=(0.0, gam, 0.0), flags=o.FLAG_DENSE)
    got = o.step(inst, E0, 5)["state"]
    ref = E0 * np.exp(1j * gam * np.abs(E0) ** 2 * 5 * h)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(E0).max()
    P0 = np.sum(np.abs(E0) ** 2)
    for fl, tau in ((o.FLAG_DENSE, 0.0), (o.FLAG_PIN_K0, 1e-2)):
        inst = o.Inst(op=o.OP_NLSE, dims=(1, 1, n), block=(1, 1, 128), tau=tau, dx=15.625,
                      dt=h, p=(-21.7, gam, 0.0), flags=fl)
        res = o.step(inst, E0, 8, diag=True)
        P = np.sum(np.abs(res["state"]) ** 2)
        assert abs(P - P0) <= 1e-12 * P0
        assert np.all(np.abs(res["diag"][:, 0] - P0) <= 1e-12 * P0)


def test_nlse_fundamental_soliton_shape(oracle_mod):
    """Fundamental soliton of the focusing NLSE (beta2 < 0): A sech(t/T0) with
    gamma A^2 T0^2 / |beta2| = 1 keeps |E| to O(h^2) over a dispersion length."""
    o = oracle_mod
    n, dt_s, beta2, gam, T0 = 2048, 0.25, -1.0, 1.0, 4.0
    A = math.sqrt(abs(beta2) / (gam * T0 * T0))
    t = (np.arange(n) - n / 2) * dt_s
    E0 = A / np.cosh(t / T0) + 0j
    LD = T0 * T0 / abs(beta2)
    errs = []
    for steps in (40, 80):
        h = LD / steps
        inst = o.Inst(op=o.OP_NLSE, dims=(1, 1, n), block=(1, 1, 64), tau=0.0, dx=dt_s,
                      dt=h, p=(beta2, gam, 0.0), flags=o.FLAG_DENSE)
        E = o.step(inst, E0, steps)["state"]
        errs.append(np.abs(np.abs(E) - np.abs(E0)).max() / A)
    assert errs[0] < 2e-3
    assert errs[1] < errs[0] / 3.0  # second-order convergence in h


# ---------------------------------------------------------------------------
# Gray-Scott: fixed point, uniform state, diffusion only
# ---------------------------------------------------------------------------

def _gs_inst(o, n, tau=0.0, flags=None, p=(0.16, 0.08, 0.035, 0.06), dt=1.0):
    return o.Inst(op=o.OP_GS, dims=(1, n, n), block=(1, 8, 8), tau=tau, dx=1.0, dt=dt, p=p,
                  flags=o.FLAG_DENSE if flags is None else flags)


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_gs_uniform_state_follows_scalar_euler_bit_exact(oracle_mod):
    o = oracle_mod
    n = 32
    u0, v0 = 0.7, 0.2
    st = np.zeros(2 * n * n, np.complex128)
    st[0] = u0 * n * n
    st[n * n] = v0 * n * n
    F, k = 0.035, 0.06
    res = o.step(_gs_inst(o, n), st, 20)
    u, v = u0, v0
    for _ in range(20):
        uvv = u * v * v
        ru = -uvv + F * (1.0 - u)
        rv = uvv - (F + k) * v
        u, v = _fma(1.0, ru, u), _fma(1.0, rv, v)
    out = res["state"]
    assert out[0] == u * n * n and out[n * n] == v * n * n
    assert np.all(out[1:n * n] == 0) and np.all(out[n * n + 1:] == 0)
    # (u, v) = (1, 0) is an exact fixed point
    st[0], st[n * n] = n * n, 0
    assert np.array_equal(o.step(_gs_inst(o, n), st, 5)["state"], st)


def test_gs_diffusion_only_closed_form(oracle_mod):
    o = oracle_mod
    n, steps, Du, Dv, dt = 32, 6, 0.16, 0.08, 0.5
    # F = k = 0 and v = 0: R_u = R_v = 0, pure implicit diffusion of u
    u = inputs.uniform_field(5, 0, (n, n), 0.5, 0.2)
    st = np.concatenate([np.fft.fft2(u).ravel(), np.zeros(n * n, np.complex128)])
    got = o.step(_gs_inst(o, n, p=(Du, Dv, 0.0, 0.0), dt=dt), st, steps)["state"][:n * n]
    m = np.fft.fftfreq(n, 1.0 / n)
    k2 = (2 * np.pi / n) ** 2 * (m[:, None] ** 2 + m[None, :] ** 2)
    ref = np.fft.fft2(u) * (1 + dt * Du * k2) ** (-steps)
    assert np.abs(got.reshape(n, n) - ref).max() <= 1e-13 * steps * np.abs(ref).max()


# ---------------------------------------------------------------------------
# Indicator, threshold, mask and worklist against a brute-force rational
# re-evaluation on a tiny grid (FP32 and FP64 working precision)
# ---------------------------------------------------------------------------

def _f32(x):
    return float(np.float32(x))


def _fmaf(a, b, c):
    return _f32(Fraction(a) * Fraction(b) + Fraction(c))


def _brute_ch(q, N, n, B, dx, dt, M, kap, tau, f32, k0=None, rk0=None):
    """Plain-Python evaluation of the adaptive rule on an n x n grid."""
    K = 2 * math.pi / (n * dx)
    K2 = K * K
    nb = n // B
    ab = np.zeros(nb * nb)
    cand = {}
    for iy in range(n):
        for ix in range(n):
            my = iy if iy < n // 2 else iy - n
            mx = ix if ix < n // 2 else ix - n
            k2 = K2 * float(my * my + mx * mx)
            s = (dt * M) * k2
            a = 1.0 / (1.0 + ((dt * M) * kap) * (k2 * k2))
            i = iy * n + ix
            if f32 and i == 0:
                c0 = _fma(-s, rk0, k0) * a
                cand[i] = (c0, 0.0)
                d = (c0 - k0) ** 2 + 0.0
            elif f32:
                sf, af = _f32(s), _f32(a)
                cr = _f32(_fmaf(-sf, float(N[i].real), float(q[i].real)) * af)
                ci = _f32(_fmaf(-sf, float(N[i].imag), float(q[i].imag)) * af)
                cand[i] = (cr, ci)
                dr, di = cr - float(q[i].real), ci - float(q[i].imag)
                d = dr * dr + di * di
            else:
                cr = _fma(-s, N[i].real, q[i].real) * a
                ci = _fma(-s, N[i].imag, q[i].imag) * a
                cand[i] = (cr, ci)
                dr, di = cr - q[i].real, ci - q[i].imag
                d = dr * dr + di * di
            b = (iy // B) * nb + ix // B
            ab[b] = max(ab[b], d)
    G = ab.max()
    thr = (tau * tau) * G
    mask = (ab > thr).astype(np.uint8)
    mask[0] = 1
    return ab, G, mask, cand


@pytest.mark.parametrize("f32", [False, True])
def test_indicator_mask_worklist_brute_force(oracle_mod, f32):
    o = oracle_mod
    n, B, dx, dt, M, kap, tau = 16, 4, 1.0, 0.01, 1.0, 1.0, 0.3
    q = inputs.shaped_spectrum(21, 0, (n, n), width=2.5).ravel()
    N = inputs.shaped_spectrum(21, 1, (n, n), width=2.0, scale=3.0).ravel()
    if f32:
        q = q.astype(np.complex64)
        N = N.astype(np.complex64)
    inst = o.Inst(op=o.OP_CH, dims=(1, n, n), block=(1, B, B), tau=tau, dx=dx, dt=dt,
                  p=(M, kap), flags=o.FLAG_PIN_K0)
    k0, rk0 = 3.25, -0.75
    if f32:
        res = o.apply(inst, q, N, dtype="f32", k0=np.array([k0]), rhs_k0=np.array([rk0]))
    else:
        res = o.apply(inst, q, N)
    ab, G, mask, cand = _brute_ch(q, N, n, B, dx, dt, M, kap, tau, f32, k0, rk0)
    assert np.array_equal(res["a_b"], ab)
    assert res["G"] == G
    assert np.array_equal(res["mask"], mask)
    assert np.array_equal(res["worklist"], np.flatnonzero(mask))
    assert 1 < res["count"] < (n // B) ** 2
    out = res["q"]
    for i in range(n * n):
        b = (i // n // B) * (n // B) + (i % n) // B
        if f32 and i == 0:
            assert out[0] == 0 and res["k0"][0] == cand[0][0]
        elif mask[b]:
            assert (out[i].real, out[i].imag) == cand[i]
        else:
            assert out[i] == q[i]


def test_skip_set_freezes_without_evaluation(oracle_mod):
    """Proposer mode: skipped blocks are frozen and excluded from G; an empty
    skip set reproduces the plain rule."""
    o = oracle_mod
    n = 32
    inst = _ch_inst(o, n, ndim=2, block=8, tau=1e-2, flags=o.FLAG_PIN_K0)
    q = inputs.shaped_spectrum(31, 0, (n, n), width=4.0)
    N = inputs.shaped_spectrum(31, 1, (n, n), width=3.0)
    plain = o.apply(inst, q, N)
    empty = o.apply(inst, q, N, skip=np.zeros(inst.n_blocks, np.uint8))
    for k in ("a_b", "mask", "q"):
        assert np.array_equal(plain[k], empty[k])
    skip = np.zeros(inst.n_blocks, np.uint8)
    top = int(np.argmax(np.where(np.arange(inst.n_blocks) == 0, -1, plain["a_b"])))
    skip[top] = 1
    res = o.apply(inst, q, N, skip=skip)
    assert res["mask"][top] == 0 and res["a_b"][top] == 0.0
    assert res["G"] == max(v for b, v in enumerate(plain["a_b"]) if b != top)
    blk = (np.arange(n)[:, None] // 8) * 4 + np.arange(n)[None, :] // 8
    assert np.array_equal(res["q"].reshape(n, n)[blk == top], q[blk == top])


def test_nonfinite_indicator_raises(oracle_mod):
    o = oracle_mod
    n = 16
    inst = _ch_inst(o, n, ndim=2, block=4, tau=1e-3, flags=o.FLAG_PIN_K0)
    q = inputs.shaped_spectrum(41, 0, (n, n), width=3.0)
    N = inputs.shaped_spectrum(41, 1, (n, n), width=3.0)
    N[5, 7] = np.nan
    with pytest.raises(o.OracleError):
        o.apply(inst, q, N)


def test_invalid_descriptor_rejected(oracle_mod):
    o = oracle_mod
    bad = o.Inst(op=o.OP_CH, dims=(1, 16, 16), block=(1, 5, 5), tau=1e-3, dx=1.0, dt=0.01,
                 p=(1.0, 1.0))
    with pytest.raises(o.OracleError):
        o.apply(bad, np.zeros(256, np.complex128), np.zeros(256, np.complex128))
