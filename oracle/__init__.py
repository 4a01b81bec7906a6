"""CPU reference (oracle) for the sp-DBA transform-domain update.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The library in
``paper_2609_03922_amd`` never imports it and shares no code with it.

The arithmetic lives in ``spdba_oracle.c`` (plain C, FP64 unless the FP32
emulation entry point is used); this module only marshals numpy arrays through
ctypes.  ``mlp`` holds the FP64 / bf16-emulating reference of the activation
proposer's network.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OP_CH, OP_GS, OP_NLSE, OP_XPFC = 1, 2, 3, 4
FLAG_DENSE, FLAG_PIN_K0 = 1, 2
FLAG_TRANSITION, FLAG_REFRESH, FLAG_DYN_TAU = 4, 8, 16  # consistency control (S1.1, S1.3)
FLAG_STATE = 32  # state-amplitude activity measure (main text; S4.2; S5.3)
FLAG_HALF = 64  # half-spectrum layout of a real field (S1.2)
FLAG_ENERGY = 128  # with FLAG_STATE: block energy, the sum instead of the maximum (main text; S5.3)
OK, EINVAL, ENONFINITE = 0, 1, 6


class OracleError(RuntimeError):
    pass


class _Inst(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("dims", ctypes.c_int64 * 3),
        ("block", ctypes.c_int32 * 3),
        ("pad", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("p", ctypes.c_double * 8),
        ("refresh_period", ctypes.c_int32),
        ("full_steps", ctypes.c_int32),
        ("interval", ctypes.c_int32),
        ("full_now", ctypes.c_int32),
        ("target_ratio", ctypes.c_double),
        ("deadband", ctypes.c_double),
        ("hist_valid", ctypes.c_int32),
        ("pad2", ctypes.c_int32),
    ]


@dataclass
class Inst:
    """One grid instance: operator, grid, block shape, threshold, parameters.

    ``dims``/``block`` are 3-tuples (slowest..fastest), unused axes 1.
    ``p``: CH (M, kappa); GS (Du, Dv, F, k); NLSE (beta2, gamma, alpha).
    For NLSE, ``dx`` is the sample spacing and ``dt`` the propagation step.
    """

    op: int
    dims: tuple
    block: tuple
    tau: float
    dx: float
    dt: float
    p: tuple = ()
    flags: int = FLAG_PIN_K0
    # consistency control (Supplementary S1.1, S1.3); see spdba_oracle.h
    refresh_period: int = 0
    full_steps: int = 0
    interval: int = 0
    target_ratio: float = 0.0
    deadband: float = 0.0
    full_now: int = 0  # apply(): this update activates every block
    hist_valid: int = 0  # XPFC step(): the state carries the three older nonlinear transforms

    @property
    def half(self) -> bool:
        return bool(self.flags & FLAG_HALF)

    @property
    def stored_dims(self) -> tuple:
        """Extents of the stored spectrum (x keeps nx/2 + 1 columns in the half layout)."""
        d = tuple(int(v) for v in self.dims)
        return d[:2] + (d[2] // 2 + 1,) if self.half else d

    @property
    def n_modes(self) -> int:
        return int(np.prod(self.stored_dims))

    @property
    def n_blocks(self) -> int:
        nb = [d // b for d, b in zip(self.dims, self.block)]
        if self.half:  # columns below nx/2, then one block per (z, y) block row for nx/2
            return nb[0] * nb[1] * (self.dims[2] // (2 * self.block[2]) + 1)
        return int(np.prod(nb))

    @property
    def n_species(self) -> int:
        return 2 if self.op == OP_GS else 1

    def _c(self) -> _Inst:
        s = _Inst()
        s.op = self.op
        s.flags = self.flags
        for i in range(3):
            s.dims[i] = int(self.dims[i])
            s.block[i] = int(self.block[i])
        s.tau, s.dx, s.dt = float(self.tau), float(self.dx), float(self.dt)
        pp = list(self.p) + [0.0] * (8 - len(self.p))
        for i in range(8):
            s.p[i] = float(pp[i])
        s.refresh_period, s.full_steps = int(self.refresh_period), int(self.full_steps)
        s.interval, s.full_now = int(self.interval), int(self.full_now)
        s.target_ratio, s.deadband = float(self.target_ratio), float(self.deadband)
        s.hist_valid = int(self.hist_valid)
        return s


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b

            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.or_fft.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        lib.or_sincos.argtypes = [ctypes.c_double, P, P]
        lib.or_apply_f64.argtypes = [P, P, P, P, P, P, P, P, P]
        lib.or_apply_f32.argtypes = [P, P, P, P, P, P, P, P, P, P, P]
        lib.or_step_f64.argtypes = [P, ctypes.c_int64, P, P, P, P, P]
        lib.or_step_ctl_f64.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P]
        lib.or_taper.argtypes = [ctypes.c_int64, P]
        lib.or_ch_energy.argtypes = [P, P, P, P]
        lib.or_sizes.argtypes = [P, P, P]
        lib.or_r2c.argtypes = [ctypes.POINTER(ctypes.c_int64), P, P]
        lib.or_etd4_phi.argtypes = [ctypes.c_double, P]
        lib.or_etd4_coef.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        lib.or_xpfc_linear.argtypes = [P, ctypes.c_double]
        lib.or_xpfc_linear.restype = ctypes.c_double
        lib.or_xpfc_energy.argtypes = [P, P, P, P]
        lib.or_c2r.argtypes = [ctypes.POINTER(ctypes.c_int64), P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc):
    if rc == ENONFINITE:
        raise OracleError("non-finite indicator value")
    if rc != OK:
        raise OracleError(f"oracle error {rc}")


def fft(a: np.ndarray, sign: int) -> np.ndarray:
    """n-D FFT of a complex array (1..3 dims). sign=-1 forward, +1 inverse (1/N)."""
    a = np.ascontiguousarray(a, dtype=np.complex128).copy()
    shape = list(a.shape)
    dims = (ctypes.c_int64 * 3)(*([1] * (3 - len(shape)) + shape))
    _check(_load().or_fft(_ptr(a), dims, int(sign)))
    return a


def rfft(real: np.ndarray) -> np.ndarray:
    """Half spectrum (columns 0 .. nx/2 of the forward transform) of a real array."""
    a = np.ascontiguousarray(real, dtype=np.float64)
    shape = [1] * (3 - a.ndim) + list(a.shape)
    out = np.zeros(tuple(shape[:2]) + (shape[2] // 2 + 1,), np.complex128)
    _check(_load().or_r2c((ctypes.c_int64 * 3)(*shape), _ptr(a), _ptr(out)))
    return out.reshape(a.shape[:-1] + (a.shape[-1] // 2 + 1,))


def irfft(half: np.ndarray, shape) -> np.ndarray:
    """Real field of a half spectrum (the omitted columns by conjugate symmetry)."""
    shape = tuple(int(v) for v in shape)
    full = [1] * (3 - len(shape)) + list(shape)
    h = np.ascontiguousarray(half, dtype=np.complex128).reshape(-1)
    if h.size != full[0] * full[1] * (full[2] // 2 + 1):
        raise ValueError("half spectrum size does not match the shape")
    out = np.zeros(shape, np.float64)
    _check(_load().or_c2r((ctypes.c_int64 * 3)(*full), _ptr(h), _ptr(out)))
    return out


def sincos(x: float):
    s, c = ctypes.c_double(), ctypes.c_double()
    _load().or_sincos(float(x), ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def _sizes(c) -> tuple:
    """(stored modes per species, blocks) of a descriptor, after the C check."""
    nm, nb = ctypes.c_int64(), ctypes.c_int64()
    _check(_load().or_sizes(ctypes.byref(c), ctypes.byref(nm), ctypes.byref(nb)))
    return nm.value, nb.value


def _need(a, n: int, what: str):
    """The C routines take array extents from the instance: refuse a wrong size
    here rather than let them read or write past it."""
    if a is not None and a.size != n:
        raise ValueError(f"{what}: {a.size} values, the instance needs {n}")


def apply(inst: Inst, q, rhs=None, *, dtype="f64", k0=None, rhs_k0=None, skip=None):
    """One kernel-level update of one instance (candidate, indicator, mask, update).

    q, rhs: complex arrays of n_species * n_modes values (species concatenated).
    For dtype 'f32' with CH/GS, k0/rhs_k0 hold the FP64 k=0 values per species.
    Returns dict(q, a_b, G, mask, worklist, count, k0).
    """
    lib = _load()
    c = inst._c()
    nb = inst.n_blocks
    a_b = np.zeros(nb, np.float64)
    mask = np.zeros(nb, np.uint8)
    wl = np.zeros(max(nb, 1), np.uint32)
    G = ctypes.c_double()
    cnt = ctypes.c_int64()
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.uint8)
    if dtype == "f64":
        qq = np.ascontiguousarray(q, dtype=np.complex128).reshape(-1).copy()
        rr = None if rhs is None else np.ascontiguousarray(rhs, dtype=np.complex128).reshape(-1)
        _apply_sizes(inst, qq, rr, sk, None, None)
        rc = lib.or_apply_f64(ctypes.byref(c), _ptr(qq), _ptr(rr), _ptr(sk), _ptr(a_b),
                              ctypes.byref(G), _ptr(mask), _ptr(wl), ctypes.byref(cnt))
        k0o = None
    elif dtype == "f32":
        qq = np.ascontiguousarray(q, dtype=np.complex64).reshape(-1).copy()
        rr = None if rhs is None else np.ascontiguousarray(rhs, dtype=np.complex64).reshape(-1)
        k0o = None if k0 is None else np.ascontiguousarray(k0, dtype=np.float64).copy()
        rk = None if rhs_k0 is None else np.ascontiguousarray(rhs_k0, dtype=np.float64)
        _apply_sizes(inst, qq, rr, sk, k0o, rk)
        rc = lib.or_apply_f32(ctypes.byref(c), _ptr(qq), _ptr(rr), _ptr(k0o), _ptr(rk), _ptr(sk),
                              _ptr(a_b), ctypes.byref(G), _ptr(mask), _ptr(wl), ctypes.byref(cnt))
    else:
        raise ValueError(dtype)
    _check(rc)
    n = cnt.value
    return dict(q=qq, a_b=a_b, G=G.value, mask=mask, worklist=wl[:n].copy(), count=n, k0=k0o)


def _apply_sizes(inst: Inst, q, r, sk, k0, rk):
    nm, nb = _sizes(inst._c())
    ns = inst.n_species
    _need(q, ns * nm, "q")
    _need(r, (4 if inst.op == OP_XPFC else ns) * nm, "rhs")
    _need(sk, nb, "skip")
    _need(k0, ns, "k0")
    _need(rk, ns, "rhs_k0")


def step(inst: Inst, state, nsteps: int, *, masks=False, diag=False, ab=False):
    """nsteps full FP64 steps.  state: CH c-hat; GS u-hat|v-hat; NLSE E(t);
    XPFC psi-hat then the three older nonlinear transforms (4 n_modes values;
    with hist_valid = 0 the first step fills them).
    The consistency-control schedule of the instance (refresh, full steps,
    threshold control) applies.

    Returns dict(state, masks [nsteps, per, nb], diag [nsteps, 4], ab,
    active_steps (non-frozen updates per block), tau [nsteps]).
    """
    lib = _load()
    c = inst._c()
    nb = inst.n_blocks
    per = 2 if inst.op == OP_NLSE else 1
    st = np.ascontiguousarray(state, dtype=np.complex128).reshape(-1).copy()
    _need(st, (4 if inst.op == OP_XPFC else inst.n_species) * _sizes(c)[0], "state")
    mk = np.zeros((nsteps, per, nb), np.uint8) if masks else None
    dg = np.zeros((nsteps, 4), np.float64) if diag else None
    abv = np.zeros((nsteps, per, nb), np.float64) if ab else None
    act = np.zeros(nb, np.int64)
    tau = np.zeros(max(nsteps, 1), np.float64)
    _check(lib.or_step_ctl_f64(ctypes.byref(c), int(nsteps), _ptr(st), _ptr(mk), _ptr(dg),
                               _ptr(abv), _ptr(act), _ptr(tau)))
    return dict(state=st, masks=mk, diag=dg, ab=abv, active_steps=act, tau=tau[:nsteps])


def taper(B: int):
    """The transition taper w(i), i = 0 .. B-1 (Supplementary S1.1)."""
    w = np.zeros(max(int(B), 1), np.float64)
    _load().or_taper(int(B), _ptr(w))
    return w


def ch_energy(inst: Inst, chat):
    lib = _load()
    c = inst._c()
    ch = np.ascontiguousarray(chat, dtype=np.complex128).reshape(-1)
    _need(ch, _sizes(c)[0], "c-hat")
    e, m = ctypes.c_double(), ctypes.c_double()
    _check(lib.or_ch_energy(ctypes.byref(c), _ptr(ch), ctypes.byref(e), ctypes.byref(m)))
    return e.value, m.value


# ---------------------------------------------------------------------------
# XPFC (Supplementary S3.1-S3.2): ETD4 coefficients, linear operator, energy
# ---------------------------------------------------------------------------

def etd4_phi(z: float) -> np.ndarray:
    """(e^z, phi_1, phi_2, phi_3, phi_4) at z."""
    out = np.zeros(5, np.float64)
    _load().or_etd4_phi(float(z), _ptr(out))
    return out


def etd4_coef(z: float, dt: float, mk2: float) -> np.ndarray:
    """(e^z, B_1, .., B_4), B_l = mk2 Phi_l."""
    out = np.zeros(5, np.float64)
    _load().or_etd4_coef(float(z), float(dt), float(mk2), _ptr(out))
    return out


def xpfc_linear(inst: Inst, k2: float) -> float:
    c = inst._c()
    return float(_load().or_xpfc_linear(ctypes.byref(c), float(k2)))


def xpfc_energy(inst: Inst, psihat):
    """(free energy, mean density) of a spectrum."""
    c = inst._c()
    ph = np.ascontiguousarray(psihat, dtype=np.complex128).reshape(-1)
    _need(ph, _sizes(c)[0], "psi-hat")
    e, m = ctypes.c_double(), ctypes.c_double()
    _check(_load().or_xpfc_energy(ctypes.byref(c), _ptr(ph), ctypes.byref(e), ctypes.byref(m)))
    return e.value, m.value
