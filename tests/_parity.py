"""Shared helpers of the GPU parity tests: build matching oracle and library
descriptors from one record, draw seeded inputs, compare results."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_2609_03922_amd import inputs
from paper_2609_03922_amd import spdba as S

OPMAP = {"ch": O.OP_CH, "gs": O.OP_GS, "nlse": O.OP_NLSE, "xpfc": O.OP_XPFC}


def oracle_inst(d: S.Desc, full_now: int = 0) -> O.Inst:
    flags = ((O.FLAG_DENSE if d.dense else 0) | (O.FLAG_PIN_K0 if d.pin_k0 else 0)
             | (O.FLAG_TRANSITION if d.transition else 0) | (O.FLAG_REFRESH if d.refresh else 0)
             | (O.FLAG_DYN_TAU if d.target_ratio else 0) | (O.FLAG_STATE if d.state_indicator else 0)
             | (O.FLAG_HALF if d.half else 0) | (O.FLAG_ENERGY if d.block_energy else 0))
    return O.Inst(op=OPMAP[d.op], dims=d.dims3, block=d.block3, tau=d.tau, dx=d.dx, dt=d.dt,
                  p=tuple(d.params), flags=flags, refresh_period=d.refresh, full_steps=d.full_steps,
                  interval=d.control_interval, target_ratio=d.target_ratio, deadband=d.deadband,
                  full_now=full_now)


def k0path(d: S.Desc) -> bool:
    return d.dtype == "f32" and d.op != "nlse"


def draw_apply_inputs(d: S.Desc, seed: int, idx: int, width_frac: float = 1 / 12, floor: float = 0.0):
    """Seeded state and right-hand side spectra (species concatenated), plus
    FP64 k = 0 values for the FP32 real-field path."""
    cd = np.complex128 if d.dtype == "f64" else np.complex64
    shape = d.dims3[3 - d.ndim:]
    w = max(1.0, d.n * width_frac)
    xs = d.stored_dims[2]  # half layout: the stored columns of the full spectrum
    q = np.concatenate([inputs.shaped_spectrum(seed, 10 * idx + s, shape, w, floor=floor)[..., :xs].ravel()
                        for s in range(d.nspec)]).astype(cd)
    r = np.concatenate([inputs.shaped_spectrum(seed, 10 * idx + 5 + s, shape, 0.8 * w, floor=floor,
                                               scale=3.0)[..., :xs].ravel()
                        for s in range(d.nspec)]).astype(cd)
    rng = inputs.rng_for(seed, 99, idx)
    k0 = rng.uniform(-1.0, 1.0, d.nspec) * d.n_modes
    rk0 = rng.uniform(-1.0, 1.0, d.nspec) * d.n_modes
    return q, r, k0, rk0


def oracle_apply(d: S.Desc, q, r, k0, rk0, skip=None, full_now=0, tau=None):
    inst = oracle_inst(d, full_now)
    if tau is not None:
        inst.tau = tau
    if d.dtype == "f64":
        return O.apply(inst, q, None if d.op == "nlse" else r, skip=skip)
    if d.op == "nlse":
        return O.apply(inst, q, None, dtype="f32", skip=skip)
    return O.apply(inst, q, r, dtype="f32", k0=k0, rhs_k0=rk0, skip=skip)


def assert_bits_equal(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if a.dtype.kind == "c" or a.dtype.kind == "f":
        av = a.view(np.uint64 if a.dtype.itemsize in (8, 16) else np.uint32)
        bv = b.view(av.dtype)
        bad = np.flatnonzero(av.ravel() != bv.ravel())
    else:
        bad = np.flatnonzero(a.ravel() != b.ravel())
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:5]}"


def rel_l2(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
