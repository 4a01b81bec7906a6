"""Seeded synthetic inputs shared by the library's tests, the oracle's tests and
the benchmark.

This module only draws random numbers and shapes them into initial fields and
test spectra; it contains none of the update method's arithmetic (no
wavenumbers, coefficients, indicators or time steps).  Every generator takes an
explicit seed and uses NumPy's PCG64 (``default_rng``), so both sides of a
parity test receive the same bytes.
"""
from __future__ import annotations

import numpy as np


def rng_for(seed: int, *stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), *[int(s) for s in stream]])


def dims3(ndim: int, n: int) -> tuple:
    """(nz, ny, nx) with unused leading axes set to 1."""
    return tuple([1] * (3 - ndim) + [n] * ndim)


def block3(ndim: int, b: int) -> tuple:
    return tuple([1] * (3 - ndim) + [b] * ndim)


# --------------------------------------------------------------------------
# batched workload sizes
# --------------------------------------------------------------------------

def instance_sizes(cfg: dict) -> list:
    """Per-instance grid extent of a batched workload, drawn from its seed."""
    r = rng_for(cfg["seed"], 0)
    if cfg["op"] == "nlse":
        e = r.integers(cfg["log2_min"], cfg["log2_max"] + 1, size=cfg["n_instances"])
        return [int(2 ** int(x)) for x in e]
    if cfg["op"] == "gs":
        return [int(x) for x in r.choice(np.array(cfg["sizes"]), size=cfg["n_instances"])]
    return [int(cfg["n"])]


# --------------------------------------------------------------------------
# initial fields (real space / time domain)
# --------------------------------------------------------------------------

def uniform_field(seed: int, inst: int, shape, mean: float, half_width: float,
                  dtype=np.float64) -> np.ndarray:
    """mean + U(-half_width, half_width), i.i.d. per grid point."""
    r = rng_for(seed, 1, inst)
    return (mean + r.uniform(-half_width, half_width, size=shape)).astype(dtype)


def gs_patch_field(seed: int, inst: int, n: int, patches: int = 10, patch: int = 8,
                   u_val: float = 0.5, v_val: float = 0.25, dtype=np.float32):
    """u = 1, v = 0 with `patches` square patches (periodic wrap, overwrite)."""
    r = rng_for(seed, 2, inst)
    u = np.ones((n, n), np.float64)
    v = np.zeros((n, n), np.float64)
    corners = r.integers(0, n, size=(patches, 2))
    idx = np.arange(patch)
    for cy, cx in corners:
        ys = (cy + idx) % n
        xs = (cx + idx) % n
        u[np.ix_(ys, xs)] = u_val
        v[np.ix_(ys, xs)] = v_val
    return u.astype(dtype), v.astype(dtype)


def qam16_rrc_signal(seed: int, inst: int, n: int, sps: int = 2, rolloff: float = 0.1,
                     power_w: float = 1e-3, dtype=np.complex64) -> np.ndarray:
    """Random 16-QAM symbols, zero-stuffed to `sps` samples/symbol, shaped by a
    root-raised-cosine response applied exactly in frequency (circular), then
    scaled to mean |E|^2 = power_w."""
    r = rng_for(seed, 3, inst)
    nsym = n // sps
    levels = np.array([-3.0, -1.0, 1.0, 3.0])
    sym = levels[r.integers(0, 4, nsym)] + 1j * levels[r.integers(0, 4, nsym)]
    x = np.zeros(n, np.complex128)
    x[::sps] = sym
    f = np.fft.fftfreq(n) * sps  # frequency in units of the symbol rate
    af = np.abs(f)
    f1, f2 = (1 - rolloff) / 2, (1 + rolloff) / 2
    h = np.zeros(n)
    h[af <= f1] = 1.0
    mid = (af > f1) & (af <= f2)
    h[mid] = np.sqrt(0.5 * (1 + np.cos(np.pi / rolloff * (af[mid] - f1))))
    y = np.fft.ifft(np.fft.fft(x) * h)
    y *= np.sqrt(power_w / np.mean(np.abs(y) ** 2))
    return y.astype(dtype)


# --------------------------------------------------------------------------
# spectra for kernel-level tests: structured random coefficients
# --------------------------------------------------------------------------

def shaped_spectrum(seed: int, stream: int, dims, width: float, floor: float = 1e-4,
                    scale: float = 1.0, dtype=np.complex128) -> np.ndarray:
    """Random complex coefficients whose magnitude falls off as a Gaussian in the
    distance from index 0 (periodic), plus a small floor -- a stand-in for the
    concentrated spectra of the workloads.  `width` is in index units."""
    r = rng_for(seed, 4, stream)
    shape = tuple(int(d) for d in dims)
    g = r.standard_normal(shape) + 1j * r.standard_normal(shape)
    dist2 = np.zeros(shape)
    for ax, n in enumerate(shape):
        i = np.arange(n)
        d = np.minimum(i, n - i).astype(np.float64)
        sh = [1] * len(shape)
        sh[ax] = n
        dist2 = dist2 + (d.reshape(sh)) ** 2
    amp = np.exp(-dist2 / (2.0 * width * width)) + floor
    return (scale * amp * g).astype(dtype)


def perturbed_components(seed: int, M: int, dims, base: float, amp: float, dtype=np.float64) -> np.ndarray:
    """M real fields of shape dims: base + a uniform perturbation in [-amp, amp)
    per point and component (a nearly homogeneous start with random
    perturbation), shape (M, *dims)."""
    r = rng_for(seed, 7, M)
    return (base + r.uniform(-amp, amp, (M, *dims))).astype(dtype)


def gaussian_packets(N: int, T: float, M: int, P0: float = 1000.0, w: float = 10.0,
                     offsets=(-20.0, 0.0, 20.0), carriers=(-0.15, 0.0, 0.15)) -> np.ndarray:
    """The transmitted field of the multimode tests: on the time grid of N
    samples over the window T (t from -T/2), a sum of Gaussian packets of width
    w at the given time offsets, each with amplitude sqrt(P0 / packets) and a
    carrier 2 pi N/T times the given fraction; the same waveform on all M
    modes.  Shape (M, N), complex128."""
    t = (np.arange(N) - N // 2) * (T / N)
    A0 = np.sqrt(P0 / len(offsets))
    e = np.zeros(N, np.complex128)
    for tq, cq in zip(offsets, carriers):
        e = e + A0 * np.exp(-((t - tq) ** 2) / (2.0 * w * w)) * np.exp(1j * 2.0 * np.pi * N / T * cq * t)
    return np.tile(e, (M, 1))


def hermitian_coupling(seed: int, M: int) -> np.ndarray:
    """A constant Hermitian mode-coupling matrix: real N(0,1) diagonal, real and
    imaginary parts of the upper triangle N(0,1), the lower triangle by
    Hermitian symmetry, scaled so that the mean of |K_ij|^2 is 1."""
    r = rng_for(seed, 9, M)
    K = np.zeros((M, M), np.complex128)
    for i in range(M):
        K[i, i] = r.standard_normal()
        for j in range(i + 1, M):
            K[i, j] = r.standard_normal() + 1j * r.standard_normal()
            K[j, i] = np.conj(K[i, j])
    return K / np.sqrt(np.mean(np.abs(K) ** 2))


def xpfc_seed_field(seed: int, inst: int, n: int, dx: float, q0: float = 1.0, mean: float = 0.12,
                    amp: float = 0.25, seeds: int = 12, radius_frac: float = 0.12, width: float = 2.0,
                    noise: float = 0.01, dtype=np.float64) -> np.ndarray:
    """Two-dimensional polycrystalline start of the density: a uniform mean
    with small noise, and `seeds` crystalline seeds of random centre and
    orientation, each a triangular (hexagonal-density) wave of three plane
    waves of wavenumber q0 at 120 degrees, `amp` each, faded out over
    `width` grid spacings at its radius (radius_frac of the domain edge).
    Where seeds overlap the nearest centre wins.  Each seed touches only the
    periodic window around its centre that its fade reaches."""
    r = rng_for(seed, inst, 17)
    L = n * dx
    cen = r.uniform(0.0, L, size=(seeds, 2))
    ang = r.uniform(0.0, np.pi / 3.0, size=seeds)
    rad = radius_frac * L
    f = mean + noise * r.uniform(-1.0, 1.0, size=(n, n))
    best = np.full((n, n), np.inf)
    reach = min(n // 2, int(np.ceil((rad + 8.0 * width * dx) / dx)) + 1)
    off = np.arange(-reach, reach + 1)
    for s in range(seeds):
        cx, cy = int(round(cen[s, 0] / dx)), int(round(cen[s, 1] / dx))
        ix, iy = np.unique((cx + off) % n), np.unique((cy + off) % n)
        x = (ix * dx)[None, :]
        y = (iy * dx)[:, None]
        # periodic distance to the centre
        dxs = (x - cen[s, 0] + 0.5 * L) % L - 0.5 * L
        dys = (y - cen[s, 1] + 0.5 * L) % L - 0.5 * L
        d = np.sqrt(dxs * dxs + dys * dys)
        wave = np.zeros(d.shape)
        for j in range(3):
            a = ang[s] + 2.0 * np.pi * j / 3.0
            wave = wave + np.cos(q0 * (np.cos(a) * dxs + np.sin(a) * dys))
        w = 0.5 * (1.0 - np.tanh((d - rad) / (width * dx)))
        sub = np.ix_(iy, ix)
        fb, bb = f[sub], best[sub]
        take = d < bb
        f[sub] = np.where(take & (w > 1e-3), mean + amp * w * wave + (1.0 - w) * (fb - mean), fb)
        best[sub] = np.where(take, d, bb)
    return f.astype(dtype)
