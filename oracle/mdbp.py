"""CPU reference of multimode digital backpropagation (DBP), Supplementary S5.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain FP64 numpy,
written from the definitions.

* Model (S5.1): dE/dz = (D + N) E for M coupled modes; D = -alpha/2 I
  - i beta2/2 d^2/dt^2 I + i K with a constant Hermitian coupling K; the
  Manakov-averaged Kerr term N = i gamma 8/9 (sum_m |E_m|^2) I.
* Step (S5.2): symmetric split step -- a linear half-step in the frequency
  domain, the nonlinear step in the time domain, a linear half-step.  Each
  linear half-step is the paper's factorisation
  U_c(dz/4) exp[(-alpha/2 + i beta2/2 omega^2) dz/2] U_c(dz/4) per bin, with
  U_c(delta) = exp(i delta K) (= V exp(i delta Lambda) V^H for K = V Lambda
  V^H), here from its power series with scaling and squaring (``expm_i``,
  written out: no eigen-solver).
  Over a step the Kerr intensity is taken at the start of the step (the
  integral of N over dz with |E| constant, since the rotation keeps |E_m|).
* Activation (S5.3): the total modal spectral power P(omega) = sum_m |E_m|^2
  (re^2 + im^2 per mode in FP64, modes in order); with the package's relative
  rule a frequency block is active iff its maximum exceeds fl(tau^2 G); the
  bin omega = 0 is left out and its block pinned (as everywhere in this
  package).  Active blocks update all M modes; frozen blocks keep theirs.

Spectra: shape (M, N), each mode in natural FFT order; the time window is T
with N samples, omega = 2 pi m / T with m the signed index (i below N/2,
i - N from N/2 on).  Transforms: the package's own radix-2 FFT
(``oracle.fft``).
"""
from __future__ import annotations

import numpy as np

from . import fft as _fft


def expm_i(K: np.ndarray, delta: float) -> np.ndarray:
    """exp(i delta K) from the exponential series: X = i delta K / 2^s with
    s chosen so that the largest absolute row sum of X is at most 1/2, the
    series summed to 30 terms (remainder below 2^-30 / 30!), then squared s
    times."""
    K = np.asarray(K, dtype=np.complex128)
    M = K.shape[0]
    X = 1j * float(delta) * K
    norm = float(np.max(np.sum(np.abs(X), axis=1))) if M else 0.0
    s = 0
    while norm > 0.5:
        norm *= 0.5
        s += 1
    X = X / (2.0 ** s)
    U = np.eye(M, dtype=np.complex128)
    term = np.eye(M, dtype=np.complex128)
    for j in range(1, 31):
        term = term @ X / j
        U = U + term
    for _ in range(s):
        U = U @ U
    return U


def coupling(K: np.ndarray, delta: float) -> np.ndarray:
    """U_c(delta) = exp(i delta K) (S5.2)."""
    return expm_i(K, delta)


def omega(N: int, T: float) -> np.ndarray:
    i = np.arange(N)
    return 2.0 * np.pi * np.where(2 * i < N, i, i - N).astype(np.float64) / T


def dispersion(N: int, T: float, dz: float, alpha: float, beta2: float) -> np.ndarray:
    """The scalar factor exp[(-alpha/2 + i beta2/2 omega^2) dz/2] per bin."""
    w = omega(N, T)
    return np.exp((-alpha / 2.0 + 1j * beta2 / 2.0 * w * w) * dz / 2.0)


def measure(E: np.ndarray) -> np.ndarray:
    E = np.asarray(E, dtype=np.complex128)
    a = np.zeros(E.shape[1])
    for m in range(E.shape[0]):
        a = a + (E[m].real * E[m].real + E[m].imag * E[m].imag)
    a[0] = 0.0
    return a


def linear_half(E, K, T, dz, alpha, beta2, block, tau, pin_k0=True, dense=False) -> dict:
    """One sp-DBA linear half-step on the spectra E (M, N)."""
    E = np.asarray(E, dtype=np.complex128)
    M, N = E.shape
    nb = N // block
    a = measure(E)
    a_b = a.reshape(nb, block).max(axis=1)
    G = float(a_b.max())
    mask = np.ones(nb, np.uint8) if dense else (a_b > (tau * tau) * G).astype(np.uint8)
    if pin_k0:
        mask[0] = 1
    act = np.repeat(mask.astype(bool), block)
    U = coupling(K, dz / 4.0)
    h = dispersion(N, T, dz, alpha, beta2)
    out = E.copy()
    if act.any():
        x = U @ E[:, act]
        x = h[act][None, :] * x
        out[:, act] = U @ x
    return {"a_b": a_b, "G": G, "mask": mask, "E": out, "count": int(mask.sum())}


def kerr(Et: np.ndarray, gamma: float, dz: float) -> np.ndarray:
    """Time domain: E_m <- E_m exp(i gamma 8/9 P dz), P = sum_m |E_m|^2."""
    Et = np.asarray(Et, dtype=np.complex128)
    P = np.sum(Et.real ** 2 + Et.imag ** 2, axis=0)
    return Et * np.exp(1j * gamma * (8.0 / 9.0) * P * dz)[None, :]


def step(E, steps, K, T, dz, alpha, beta2, gamma, block, tau, pin_k0=True, dense=False, masks=False) -> dict:
    """Symmetric split steps on the spectra: linear half, Kerr, linear half."""
    E = np.asarray(E, dtype=np.complex128).copy()
    log = []
    for _ in range(steps):
        for half in range(2):
            r = linear_half(E, K, T, dz, alpha, beta2, block, tau, pin_k0, dense)
            E = r["E"]
            if masks:
                log.append(r["mask"])
            if half == 0:
                Et = np.stack([_fft(E[m], +1) for m in range(E.shape[0])])
                Ek = kerr(Et, gamma, dz)
                E = np.stack([_fft(Ek[m], -1) for m in range(E.shape[0])])
    out = {"state": E}
    if masks:
        out["masks"] = np.array(log)
    return out


def nmse_db(rec: np.ndarray, ref: np.ndarray) -> float:
    """Normalised mean-squared error over the whole multimode field, in dB."""
    return float(10.0 * np.log10(np.sum(np.abs(rec - ref) ** 2) / np.sum(np.abs(ref) ** 2)))
