"""CPU reference of the reaction--cross-diffusion (RCD) core (Supplementary S4).

TEST INFRASTRUCTURE ONLY (see the package docstring): plain FP64 numpy,
written from the definitions, no blocking or reordering beyond them.

* Model (S4.1): du/dt = D lap(u) + R(u) for M components, with the symmetric
  circulant cross-diffusion matrix D (diagonal d_diag + 2 d_cross, the two
  periodic neighbours -d_cross; for M = 2 the single off-diagonal entry is
  -d_cross) and the generalised Lotka--Volterra reaction
  R_i = u_i (r - a u_i - sum_{j != i} alpha_ij u_j), alpha_ij = beta + alpha
  for the periodic neighbours j = i +- 1 and beta otherwise.
* Update (S4.2): per stored mode, u'(k) = (I + dt k^2 D)^{-1} [u(k) + dt R(k)],
  solved here directly by Gaussian elimination (``solve``, written out; the
  matrix is symmetric positive definite, so no pivoting is needed), the plain
  definition; the eigen form of S4.3 gives the same values up to rounding.
* Transforms: the package's own radix-2 FFT (``oracle.fft``), unnormalised
  forward, inverse with 1/N.
* Activation (S4.2): the component RMS amplitude; a block is active when any
  of its modes exceeds the threshold.  As in the rest of this package the
  threshold is relative: a(k) = sum_m |u_m(k)|^2 in FP64 (components in
  order, re^2 + im^2 each, k = 0 left out), a_b = block maximum, G = max_b a_b,
  active iff a_b > fl(tau^2 G) or (pin_k0 and the block holds k = 0).  The
  1/M of the RMS and the square root are monotone and cancel in this rule.

Arrays: a spectrum q has shape (M, N) with N = prod(dims), each component in
natural FFT order, C order over dims (slowest .. fastest).  Blocks are in C
order over the block grid.
"""
from __future__ import annotations

import numpy as np

from . import fft as _fft


def diffusion_matrix(M: int, d_diag: float, d_cross: float) -> np.ndarray:
    """The constant cross-diffusion matrix of S4.1."""
    if M < 2:
        raise ValueError("M >= 2")
    D = np.zeros((M, M))
    for i in range(M):
        D[i, i] = d_diag + 2.0 * d_cross
        D[i, (i + 1) % M] = -d_cross
        D[i, (i - 1) % M] = -d_cross
    return D


def interaction_matrix(M: int, alpha: float, beta: float) -> np.ndarray:
    """alpha_ij of the Lotka--Volterra reaction (S4.1); the diagonal is unused."""
    A = np.full((M, M), beta)
    for i in range(M):
        A[i, (i + 1) % M] = beta + alpha
        A[i, (i - 1) % M] = beta + alpha
        A[i, i] = 0.0
    return A


def reaction(u: np.ndarray, alpha: float, beta: float, r: float = 1.0, a: float = 1.0) -> np.ndarray:
    """R_i(u) of S4.1 for u of shape (M, ...), by the explicit interaction sum."""
    u = np.asarray(u, dtype=np.float64)
    M = u.shape[0]
    A = interaction_matrix(M, alpha, beta)
    out = np.empty_like(u)
    for i in range(M):
        s = np.zeros_like(u[0])
        for j in range(M):
            if j != i:
                s = s + A[i, j] * u[j]
        out[i] = u[i] * (r - a * u[i] - s)
    return out


def signed_index(n: int) -> np.ndarray:
    """Wavenumber index of each position in natural FFT order: i below n/2,
    i - n from n/2 on (the Nyquist index maps to -n/2)."""
    i = np.arange(n)
    return np.where(2 * i < n, i, i - n).astype(np.float64)


def solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x with A x = b for a batch of symmetric positive definite systems:
    A (n, M, M), b (n, M).  Forward elimination column by column (the pivot
    stays on the diagonal, which positive definiteness keeps away from zero),
    then back substitution."""
    A = np.array(A, dtype=np.float64)
    x = np.array(b, dtype=np.float64)
    M = A.shape[1]
    for k in range(M):
        f = A[:, k + 1:, k] / A[:, k:k + 1, k]          # (n, M-k-1) multipliers
        A[:, k + 1:, k:] -= f[:, :, None] * A[:, k:k + 1, k:]
        x[:, k + 1:] -= f * x[:, k:k + 1]
    for k in range(M - 1, -1, -1):
        s = x[:, k] - np.sum(A[:, k, k + 1:] * x[:, k + 1:], axis=1)
        x[:, k] = s / A[:, k, k]
    return x


def k2(dims, dx: float) -> np.ndarray:
    """|k|^2 of every mode, natural FFT order, flattened in C order."""
    ks = [2.0 * np.pi * signed_index(n) / (n * dx) for n in dims]
    grids = np.meshgrid(*ks, indexing="ij")
    return sum(g * g for g in grids).ravel()


def measure(q: np.ndarray) -> np.ndarray:
    """a(k) = sum over components of re^2 + im^2, in component order; k = 0 -> 0."""
    q = np.asarray(q, dtype=np.complex128)
    a = np.zeros(q.shape[1])
    for m in range(q.shape[0]):
        a = a + (q[m].real * q[m].real + q[m].imag * q[m].imag)
    a[0] = 0.0
    return a


def block_ids(dims, block) -> np.ndarray:
    """Block index of every mode (C order over the block grid)."""
    idx = np.indices(dims).reshape(len(dims), -1)
    nbk = [n // b for n, b in zip(dims, block)]
    bid = np.zeros(idx.shape[1], dtype=np.int64)
    for ax in range(len(dims)):
        bid = bid * nbk[ax] + idx[ax] // block[ax]
    return bid


def update_modes(q, rhat, k2v, dt: float, D: np.ndarray) -> np.ndarray:
    """Direct coupled update of the given modes: columns of q, rhat (M, n)."""
    M, n = q.shape
    b = q + dt * rhat
    A = np.eye(M)[None, :, :] + dt * k2v[:, None, None] * D[None, :, :]
    xr = solve(A, b.real.T)
    xi = solve(A, b.imag.T)
    return (xr + 1j * xi).T


def apply(q, rhat, dims, block, tau: float, dt: float, dx: float, d_diag: float, d_cross: float,
          pin_k0: bool = True, dense: bool = False) -> dict:
    """One sp-DBA update of S4.2 (dense: every block, the Regular update)."""
    dims = tuple(int(n) for n in dims)
    q = np.asarray(q, dtype=np.complex128)
    rhat = np.asarray(rhat, dtype=np.complex128)
    M = q.shape[0]
    D = diffusion_matrix(M, d_diag, d_cross)
    bid = block_ids(dims, block)
    nb = int(np.prod([n // b for n, b in zip(dims, block)]))
    a = measure(q)
    a_b = np.zeros(nb)
    np.maximum.at(a_b, bid, a)
    G = float(a_b.max()) if nb else 0.0
    thr = (tau * tau) * G
    mask = np.ones(nb, dtype=np.uint8) if dense else (a_b > thr).astype(np.uint8)
    if pin_k0:
        mask[bid[0]] = 1
    act = mask[bid].astype(bool)
    out = q.copy()
    if act.any():
        out[:, act] = update_modes(q[:, act], rhat[:, act], k2(dims, dx)[act], dt, D)
    return {"a_b": a_b, "G": G, "mask": mask, "q": out, "count": int(mask.sum())}


def step(q, steps: int, dims, block, tau: float, dt: float, dx: float, d_diag: float, d_cross: float,
         alpha: float, beta: float, r: float = 1.0, a: float = 1.0, pin_k0: bool = True,
         dense: bool = False, masks: bool = False) -> dict:
    """Full steps: u = Re ifft(q) per component, R(u), its transform, the update."""
    dims = tuple(int(n) for n in dims)
    q = np.asarray(q, dtype=np.complex128).copy()
    M = q.shape[0]
    log = []
    for _ in range(steps):
        u = np.stack([_fft(q[m].reshape(dims), +1).real for m in range(M)])
        R = reaction(u, alpha, beta, r, a)
        rhat = np.stack([_fft(R[m].astype(np.complex128), -1).ravel() for m in range(M)])
        res = apply(q, rhat, dims, block, tau, dt, dx, d_diag, d_cross, pin_k0, dense)
        q = res["q"]
        if masks:
            log.append(res["mask"])
    out = {"state": q}
    if masks:
        out["masks"] = np.array(log)
    return out


def equilibrium(M: int, alpha: float, beta: float, r: float = 1.0, a: float = 1.0) -> float:
    """The homogeneous coexistence state u_i = u* of the reaction (all i equal)."""
    return r / (a + float(interaction_matrix(M, alpha, beta)[0].sum()))
