"""Pins of the multimode DBP oracle (Supplementary S5) against what the
mathematics fixes: the coupling propagator is unitary, a one-parameter group
and diagonal in closed form for a diagonal K; the dispersion factor in closed
form; with K = 0 the linear half-step is the scalar factor on every mode; the
Kerr step keeps |E_m| and rotates a constant field by gamma 8/9 P dz; the
paper's three-factor half-step equals h(omega) U_c(dz/2); back-propagation
with reversed parameters recovers the input; block geometry; threshold zero
equals dense; Parseval for the measure."""
import numpy as np
import pytest

from oracle import mdbp as O
from paper_2609_03922_amd import inputs

T, DZ, AL, B2, GA = 1000.0, 0.1, 0.1, -21.0, 1.3


@pytest.mark.parametrize("M", [2, 5, 8])
def test_coupling_unitary_group_and_diagonal(M):
    K = inputs.hermitian_coupling(3, M)
    assert abs(np.mean(np.abs(K) ** 2) - 1.0) < 1e-12 and np.allclose(K, K.conj().T)
    U = O.coupling(K, 0.37)
    assert np.allclose(U.conj().T @ U, np.eye(M), atol=1e-13)
    assert np.allclose(O.coupling(K, 0.2) @ O.coupling(K, 0.17), U, atol=1e-13)
    assert np.allclose(O.coupling(K, 0.0), np.eye(M), atol=1e-14)
    d = np.arange(M) * 0.5 - 1.0
    assert np.allclose(O.coupling(np.diag(d), 0.3), np.diag(np.exp(1j * 0.3 * d)), atol=1e-15)


def test_dispersion_closed_form():
    N = 64
    h = O.dispersion(N, T, DZ, AL, B2)
    w5 = 2 * np.pi * 5 / T          # bin 5
    wneg = 2 * np.pi * -3 / T       # bin N - 3
    assert np.isclose(h[5], np.exp(-AL * DZ / 4) * np.exp(1j * B2 / 2 * w5 ** 2 * DZ / 2), rtol=1e-14)
    assert np.isclose(h[N - 3], np.exp(-AL * DZ / 4) * np.exp(1j * B2 / 2 * wneg ** 2 * DZ / 2), rtol=1e-14)
    assert np.allclose(np.abs(h), np.exp(-AL * DZ / 4), rtol=1e-14)


def test_no_coupling_is_the_scalar_factor_and_three_factor_form():
    N, M = 256, 3
    E = np.stack([inputs.shaped_spectrum(5, m, (N,), width=20.0) for m in range(M)])
    r = O.linear_half(E, np.zeros((M, M)), T, DZ, AL, B2, 32, 0.0)
    assert np.allclose(r["E"], O.dispersion(N, T, DZ, AL, B2)[None, :] * E, rtol=1e-14, atol=0)
    K = inputs.hermitian_coupling(4, M)
    r = O.linear_half(E, K, T, DZ, AL, B2, 32, 0.0)
    want = O.dispersion(N, T, DZ, AL, B2)[None, :] * (O.coupling(K, DZ / 2) @ E)
    assert np.allclose(r["E"], want, rtol=0, atol=1e-12 * np.max(np.abs(E)))


def test_kerr_keeps_modulus_and_rotates_constant_field():
    M, N = 3, 16
    E = np.full((M, N), 2.0 + 1.0j)
    out = O.kerr(E, GA, DZ)
    P = M * 5.0
    assert np.allclose(out, E * np.exp(1j * GA * 8 / 9 * P * DZ), rtol=1e-15)
    Er = np.stack([inputs.shaped_spectrum(6, m, (N,), width=3.0) for m in range(M)])
    assert np.allclose(np.abs(O.kerr(Er, GA, DZ)), np.abs(Er), rtol=1e-14)


def test_backpropagation_recovers_the_input():
    N, M, steps = 1024, 4, 20
    E0 = np.fft.fft(inputs.gaussian_packets(N, T, M, P0=1.0), axis=1)
    K = inputs.hermitian_coupling(7, M)
    fwd = O.step(E0, steps, K, T, DZ, AL, B2, GA, 32, 0.0)["state"]
    assert np.linalg.norm(fwd - E0) > 0.1 * np.linalg.norm(E0)
    back = O.step(fwd, steps, -K, T, DZ, -AL, -B2, -GA, 32, 0.0)["state"]
    assert np.linalg.norm(back - E0) <= 1e-11 * np.linalg.norm(E0)


def test_blocks_single_mode_and_threshold_zero():
    N, M, B = 256, 2, 32
    E = np.zeros((M, N), np.complex128)
    E[1, 70] = 3 - 4j               # block 2, P = 25
    E[0, 70] = 1.0                  # same bin: 26
    E[0, 0] = 100.0                 # omega = 0 left out
    r = O.linear_half(E, np.zeros((M, M)), T, DZ, AL, B2, B, 0.5)
    assert r["G"] == 26.0 and r["a_b"][2] == 26.0 and r["a_b"].sum() == 26.0
    assert sorted(np.flatnonzero(r["mask"]).tolist()) == [0, 2]
    E0 = np.fft.fft(inputs.gaussian_packets(N, T, M, P0=1.0), axis=1)
    K = inputs.hermitian_coupling(8, M)
    a = O.step(E0, 3, K, T, DZ, AL, B2, GA, B, 0.0)["state"]
    b = O.step(E0, 3, K, T, DZ, AL, B2, GA, B, 0.0, dense=True)["state"]
    assert np.array_equal(a, b)


def test_measure_parseval_and_packets():
    N, M = 512, 3
    Et = inputs.gaussian_packets(N, T, M, P0=9.0)
    E = np.fft.fft(Et, axis=1)
    a = O.measure(E)
    want = N * np.sum(np.abs(Et) ** 2) - np.sum(np.abs(E[:, 0]) ** 2)
    assert abs(a.sum() - want) <= 1e-11 * want
    # three packets of amplitude sqrt(P0/3) = sqrt(3): at t = 0 the middle one
    # plus the tails of the two at +-20 (exp(-400/200) each, carrier phase 0)
    assert np.isclose(abs(Et[0, N // 2]), np.sqrt(3.0) * (1 + 2 * np.exp(-2.0)), rtol=1e-12)


@pytest.mark.parametrize("delta", [0.3, 2.5, 40.0])
def test_expm_closed_form_two_modes(delta):
    """exp(i d sigma_x) = cos d I + i sin d sigma_x, and for a Hermitian K with
    K^2 = I (a reflection) the same form; the large argument exercises the
    squaring steps."""
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    want = np.cos(delta) * np.eye(2) + 1j * np.sin(delta) * sx
    assert np.allclose(O.expm_i(sx, delta), want, rtol=0, atol=1e-12)
    v = np.array([1.0, 1j]) / np.sqrt(2.0)
    R = 2.0 * np.outer(v, v.conj()) - np.eye(2)     # Hermitian, R^2 = I
    want = np.cos(delta) * np.eye(2) + 1j * np.sin(delta) * R
    assert np.allclose(O.expm_i(R, delta), want, rtol=0, atol=1e-12)


def test_omega_signed_bins():
    w = O.omega(8, 2.0)
    assert np.allclose(w, 2 * np.pi * np.array([0, 1, 2, 3, -4, -3, -2, -1]) / 2.0, rtol=0, atol=0)
