"""Pins of the XPFC oracle (Supplementary S3.1-S3.2) against what the
mathematics fixes independently of its code:

* the ETD coefficient functions phi_l(z) against their defining series summed
  exactly in rational arithmetic, on both branches (series for |z| <= 1,
  closed form beyond), and their values at z = 0;
* fourth-order convergence of the ETD4 multistep update, with the oracle's
  coefficients, on a scalar ODE with a closed-form solution (a wrong Phi_3 or
  Phi_4 combination lowers the order);
* the linear operator in closed form at k = q0, at k = 0 and far from the
  peak, and the symmetry of the correlation peak;
* exact exponential decay of every mode when the nonlinear terms vanish;
* exact conservation of the mean density and decay of the free energy along
  a dense FP64 run;
* threshold zero equal to dense, a split run equal to one run, and the
  history start rule (the three older transforms set to the first one)."""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle as O
from paper_2609_03922_amd import inputs

P = (1.0, 0.02, 0.1, 1.0, 1.0, 1.0, 1.0)  # q0, sigma, alpha, omega, u, rho, beta
DX, DT = math.pi / 4, 0.01


def inst(n=32, block=8, tau=0.0, flags=O.FLAG_PIN_K0 | O.FLAG_STATE, p=P, dx=DX, dt=DT, **kw):
    return O.Inst(op=O.OP_XPFC, dims=(1, n, n), block=(1, block, block), tau=tau, dx=dx, dt=dt, p=p,
                  flags=flags, **kw)


def phi_exact(z: float, terms: int = 160):
    """phi_l(z) = sum_j z^j / (l + j)! in exact rational arithmetic."""
    zf = Fraction(z)
    out = []
    for l in range(5):
        s = Fraction(0)
        t = Fraction(1, math.factorial(l))
        for j in range(terms):
            s += t
            t = t * zf / (l + j + 1)
        out.append(float(s))
    return out  # e^z = phi_0


@pytest.mark.parametrize("z", [0.0, -1e-6, -0.3, -0.999, -1.0, 0.7, -1.001, -1.5, -2.0, -5.0, -20.0, 3.0])
def test_phi_functions_against_the_exact_series(z):
    got = O.etd4_phi(z)
    want = phi_exact(z)
    # series branch: a few ulp; closed form: the divisions by z amplify the
    # rounding of e^z - 1 - ... by at most about l!/(|z| phi_l) (below 1e3 here)
    tol = 4e-16 if abs(z) <= 1.0 else 2e-13
    for l in range(5):
        assert abs(got[l] - want[l]) <= tol * abs(want[l]), (z, l, got[l], want[l])
    if z == 0.0:
        assert list(got) == [1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0]


def test_phi_branches_meet_at_one():
    a, b = O.etd4_phi(-1.0), O.etd4_phi(-1.0 - 2.0 ** -40)
    assert np.allclose(a, b, rtol=1e-11, atol=0)


def _etd4_ode_error(h, T=2.0):
    """y' = -y + y^2, y(0) = 1/2: y(t) = 1 / (1 + e^t).  ETD4 with the oracle's
    coefficients (mk2 = 1: B_l = Phi_l), exact starting history."""
    lam = -1.0
    y_ex = lambda t: 1.0 / (1.0 + math.exp(t))
    N = lambda y: y * y
    co = O.etd4_coef(lam * h, h, 1.0)
    hist = [N(y_ex(-k * h)) for k in range(4)]  # N at t = 0, -h, -2h, -3h
    y = y_ex(0.0)
    steps = int(round(T / h))
    for _ in range(steps):
        n0, n1, n2, n3 = hist
        y = (co[0] * y + co[1] * n0 + co[2] * (n0 - n1) + co[3] * (n0 - 2 * n1 + n2)
             + co[4] * (n0 - 3 * n1 + 3 * n2 - n3))
        hist = [N(y), n0, n1, n2]
    return abs(y - y_ex(T))


def test_etd4_is_fourth_order():
    e = [_etd4_ode_error(h) for h in (0.1, 0.05, 0.025, 0.0125)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(3)]
    # the observed order approaches 4 from above as h shrinks
    assert all(3.9 < r < 4.3 for r in rates) and abs(rates[-1] - 4.0) < 0.1, (e, rates)


def test_the_order_pin_sees_a_wrong_combination():
    """The same integration with Phi_3 = dt phi_3 (the phi_2 / 2 term dropped)
    is only third order: the pin above would catch such a slip."""
    def err(h, T=2.0):
        y_ex = lambda t: 1.0 / (1.0 + math.exp(t))
        ph = O.etd4_phi(-h)
        co = [ph[0], h * ph[1], h * ph[2], h * ph[3], h * (ph[2] / 3 + ph[3] + ph[4])]
        hist = [y_ex(-k * h) ** 2 for k in range(4)]
        y = 0.5
        for _ in range(int(round(T / h))):
            n0, n1, n2, n3 = hist
            y = (co[0] * y + co[1] * n0 + co[2] * (n0 - n1) + co[3] * (n0 - 2 * n1 + n2)
                 + co[4] * (n0 - 3 * n1 + 3 * n2 - n3))
            hist = [y * y, n0, n1, n2]
        return abs(y - y_ex(T))
    e = [err(h) for h in (0.05, 0.025, 0.0125)]
    assert math.log2(e[-2] / e[-1]) < 3.3


def test_linear_operator_closed_forms():
    d = inst()
    q0, sg, al = P[0], P[1], P[2]
    dw = math.exp(-(sg * sg * q0 * q0) / 2.0)
    assert O.xpfc_linear(d, q0 * q0) == pytest.approx(-q0 * q0 * (1.0 - dw), rel=1e-12)
    assert O.xpfc_linear(d, 0.0) == 0.0
    k = q0 + 40 * al  # the peak has decayed to exp(-800): L = -k^2
    assert O.xpfc_linear(d, k * k) == -k * k
    for delta in (0.05, 0.1, 0.2):
        kp, km = q0 + delta, q0 - delta
        cp = 1.0 + O.xpfc_linear(d, kp * kp) / (kp * kp)
        cm = 1.0 + O.xpfc_linear(d, km * km) / (km * km)
        assert cp == pytest.approx(cm, rel=1e-12)
        assert cp == pytest.approx(dw * math.exp(-delta * delta / (2 * al * al)), rel=1e-12)


def test_the_grid_wavenumber_that_hits_the_peak():
    # n = 16, dx = pi/2: k(m = 4) = 2 pi 4 / (16 pi/2) = 1 = q0 exactly
    d = inst(n=16, block=4, dx=math.pi / 2, p=(1.0, 0.3, 0.1, 0.0, 0.0, 1.0, 1.0), flags=O.FLAG_DENSE)
    q = np.zeros((16, 16), np.complex128)
    q[0, 4] = 1.0
    h = np.zeros(4 * 256, np.complex128)
    out = O.apply(d, q.ravel(), h)["q"].reshape(16, 16)
    L = -1.0 * (1.0 - math.exp(-0.09 / 2.0))
    assert out[0, 4] == pytest.approx(math.exp(L * d.dt), rel=1e-15)


def test_linear_run_decays_every_mode_exactly():
    # omega = u = 0: no nonlinear term, each mode decays as exp(n L dt)
    p0 = (P[0], P[1], P[2], 0.0, 0.0, 1.0, 1.0)
    d = inst(n=16, block=4, p=p0, flags=O.FLAG_DENSE)
    f = inputs.xpfc_seed_field(3, 0, 16, DX)
    psi = O.fft(f, -1).ravel()
    n = 25
    st = O.step(d, np.concatenate([psi, np.zeros(3 * psi.size)]), n)["state"][:psi.size]
    m = np.where(np.arange(16) < 8, np.arange(16), np.arange(16) - 16)
    K2 = (2 * np.pi / (16 * DX)) ** 2
    k2 = K2 * (m[:, None] ** 2 + m[None, :] ** 2).ravel()
    z = np.array([O.xpfc_linear(d, v) for v in k2]) * DT
    assert np.allclose(st, psi * np.exp(n * z), rtol=1e-13, atol=1e-13 * np.abs(psi).max())


def _run(d, f, n, **kw):
    psi = O.fft(f, -1).ravel()
    return O.step(d, np.concatenate([psi, np.zeros(3 * psi.size)]), n, **kw)


def test_mass_exact_and_free_energy_decays():
    n = 64
    d = inst(n=n, block=8, flags=O.FLAG_DENSE | O.FLAG_PIN_K0)
    f = inputs.xpfc_seed_field(5, 0, n, DX)
    r = _run(d, f, 200, diag=True)
    mass = r["diag"][:, 0]
    F = r["diag"][:, 1]
    N = n * n
    assert np.all(r["state"][0] == O.fft(f, -1).ravel()[0])  # k = 0 never changes
    assert np.allclose(mass, f.mean(), rtol=0, atol=1e-15)
    assert np.all(np.diff(F) <= 1e-12 * np.abs(F[:-1])), np.diff(F).max()
    assert F[-1] < F[0]


def test_threshold_zero_equals_dense_and_split_run():
    n = 32
    f = inputs.xpfc_seed_field(6, 0, n, DX)
    a = _run(inst(n=n, tau=0.0), f, 30)["state"]
    b = _run(inst(n=n, flags=O.FLAG_DENSE | O.FLAG_PIN_K0), f, 30)["state"]
    assert np.array_equal(a, b)
    d = inst(n=n, tau=3e-2)
    one = _run(d, f, 30, masks=True)
    half = _run(d, f, 12)
    d2 = inst(n=n, tau=3e-2, hist_valid=1)
    rest = O.step(d2, half["state"], 18)
    assert np.array_equal(one["state"], rest["state"])
    assert 0 < one["masks"][-1, 0].sum() < d.n_blocks


def test_history_starts_from_the_first_transform():
    n = 16
    f = inputs.xpfc_seed_field(7, 0, n, DX)
    st = _run(inst(n=n, block=4, flags=O.FLAG_DENSE | O.FLAG_PIN_K0), f, 1)["state"].reshape(4, -1)
    assert np.array_equal(st[1], st[2]) and np.array_equal(st[2], st[3])
    # and that transform is F[-(omega/2) psi^2 + (u/3) psi^3] of the start
    want = O.fft(-(P[3] / 2) * f ** 2 + (P[4] / 3) * f ** 3, -1).ravel()
    assert np.allclose(st[1], want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_wrong_array_sizes_are_refused_before_the_c_routines():
    """The C routines take extents from the descriptor; the wrappers refuse
    arrays of another size (an XPFC step needs psi-hat and three transforms)."""
    d = inst(n=16, block=4)
    psi = np.zeros(16 * 16, np.complex128)
    with pytest.raises(ValueError):
        O.step(d, psi, 1)
    with pytest.raises(ValueError):
        O.apply(d, psi, psi)  # the XPFC update takes four transforms
    with pytest.raises(ValueError):
        O.xpfc_energy(d, psi[:-1])
    O.step(d, np.concatenate([psi, np.zeros(3 * psi.size)]), 1)
