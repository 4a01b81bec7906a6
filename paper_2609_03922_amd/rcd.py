"""Python binding of the reaction--cross-diffusion entry points of libspdba.so
(include/spdba_rcd.h): argument marshalling only.

Every step runs in the library's HIP kernels and rocFFT; PyTorch provides the
device memory and the stream.  There is no fallback path: without the built
library the first call raises.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import spdba as S

SPDBA_RCD_DENSE, SPDBA_RCD_PIN_K0, SPDBA_RCD_TIMING, SPDBA_RCD_DIRECT = 1, 2, 4, 8

# every entry point include/spdba_rcd.h declares
RCD_EXPORTS = (
    "spdba_rcd_create", "spdba_rcd_buffer_sizes", "spdba_rcd_bind", "spdba_rcd_set_spectrum",
    "spdba_rcd_get_spectrum", "spdba_rcd_set_field", "spdba_rcd_get_field", "spdba_rcd_apply",
    "spdba_rcd_step", "spdba_rcd_indicator", "spdba_rcd_active_mask", "spdba_rcd_stats",
    "spdba_rcd_destroy", "spdba_rcd_eigen",
)


class RcdDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("M", ctypes.c_int32), ("dims", ctypes.c_int64 * 3),
        ("block", ctypes.c_int32 * 3), ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("tau", ctypes.c_double), ("dt", ctypes.c_double), ("dx", ctypes.c_double),
        ("d_diag", ctypes.c_double), ("d_cross", ctypes.c_double), ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double), ("r", ctypes.c_double), ("a", ctypes.c_double),
    ]


class RcdStats(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("active_blocks", ctypes.c_int64), ("G", ctypes.c_double),
                ("stage_ms", ctypes.c_float * 4)]


_ready = False


def load():
    global _ready
    lib = S.load()
    if not _ready:
        P, I32, SZ, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double
        sig = {
            "spdba_rcd_create": [ctypes.POINTER(RcdDesc), P, ctypes.POINTER(P)],
            "spdba_rcd_buffer_sizes": [P, ctypes.POINTER(SZ), ctypes.POINTER(SZ)],
            "spdba_rcd_bind": [P, P, P],
            "spdba_rcd_set_spectrum": [P, P], "spdba_rcd_get_spectrum": [P, P],
            "spdba_rcd_set_field": [P, P], "spdba_rcd_get_field": [P, P],
            "spdba_rcd_apply": [P, P], "spdba_rcd_step": [P, I32],
            "spdba_rcd_indicator": [P, P, SZ, P], "spdba_rcd_active_mask": [P, P, SZ, P],
            "spdba_rcd_stats": [P, ctypes.POINTER(RcdStats)], "spdba_rcd_destroy": [P],
            "spdba_rcd_eigen": [I32, D, D, P, P],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        _ready = True
    return lib


def eigen(M: int, d_diag: float, d_cross: float):
    """(V, lambda) of the plan's eigen form, computed by the library on the host."""
    V = np.zeros((M, M))
    lam = np.zeros(M)
    S._ck(load().spdba_rcd_eigen(M, d_diag, d_cross, V.ctypes.data, lam.ctypes.data), "spdba_rcd_eigen")
    return V, lam


def make_desc(M, ndim, n, block, dtype="f32", tau=1e-6, dt=0.01, dx=0.5, d_diag=0.5, d_cross=0.05,
              alpha=1.0, beta=0.3, r=1.0, a=1.0, dense=False, pin_k0=True, timing=False,
              direct=False) -> RcdDesc:
    c = RcdDesc()
    c.ndim, c.M = ndim, M
    for ax in range(3):
        used = ax >= 3 - ndim
        c.dims[ax] = n if used else 1
        c.block[ax] = block if used else 1
    c.dtype = S.DTYPES[dtype]
    c.flags = (SPDBA_RCD_DENSE if dense else 0) | (SPDBA_RCD_PIN_K0 if pin_k0 else 0) | \
              (SPDBA_RCD_TIMING if timing else 0) | (SPDBA_RCD_DIRECT if direct else 0)
    c.tau, c.dt, c.dx = tau, dt, dx
    c.d_diag, c.d_cross, c.alpha, c.beta, c.r, c.a = d_diag, d_cross, alpha, beta, r, a
    return c


def create_status(desc: RcdDesc) -> int:
    """Status of spdba_rcd_create (the plan, if any, is released)."""
    h = ctypes.c_void_p()
    st = load().spdba_rcd_create(ctypes.byref(desc), None, ctypes.byref(h))
    if h.value:
        load().spdba_rcd_destroy(h)
    return st


class RcdPlan:
    """A bound RCD plan with torch-owned buffers on a stream of its own."""

    def __init__(self, desc: RcdDesc, stream=None):
        import torch

        self.torch = torch
        self.desc = desc
        self.M = desc.M
        self.N = int(desc.dims[0] * desc.dims[1] * desc.dims[2])
        self.dbl = desc.dtype == S.SPDBA_F64
        self.n_blocks = int(np.prod([desc.dims[a] // desc.block[a] for a in range(3)]))
        lib = load()
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = ctypes.c_void_p()
        S._ck(lib.spdba_rcd_create(ctypes.byref(desc), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "spdba_rcd_create")
        self.h = h
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        S._ck(lib.spdba_rcd_buffer_sizes(h, ctypes.byref(sb), ctypes.byref(wb)), "spdba_rcd_buffer_sizes")
        self.d_state = torch.empty(sb.value + 256, dtype=torch.uint8, device="cuda")
        self.d_work = torch.empty(wb.value + 256, dtype=torch.uint8, device="cuda")
        S._ck(lib.spdba_rcd_bind(h, self._al(self.d_state), self._al(self.d_work)), "spdba_rcd_bind")

    @staticmethod
    def _al(t):
        p = t.data_ptr()
        return ctypes.c_void_p((p + 255) & ~255)

    def _enter(self):
        self.stream.wait_stream(self.torch.cuda.current_stream())

    def _real(self):
        return self.torch.float64 if self.dbl else self.torch.float32

    def _cplx(self):
        return self.torch.complex128 if self.dbl else self.torch.complex64

    def _dev(self, x, dtype):
        t = self.torch.as_tensor(x).to(device="cuda", dtype=dtype).contiguous().view(-1)
        if t.numel() != self.M * self.N:
            raise ValueError(f"expected {self.M * self.N} values, got {t.numel()}")
        return t

    def set_field(self, u):
        t = self._dev(u, self._real())
        self._enter()
        S._ck(load().spdba_rcd_set_field(self.h, ctypes.c_void_p(t.data_ptr())), "spdba_rcd_set_field")
        self.stream.synchronize()

    def get_field(self):
        out = self.torch.empty(self.M * self.N, dtype=self._real(), device="cuda")
        self._enter()
        S._ck(load().spdba_rcd_get_field(self.h, ctypes.c_void_p(out.data_ptr())), "spdba_rcd_get_field")
        self.stream.synchronize()
        return out

    def set_spectrum(self, q):
        t = self._dev(q, self._cplx())
        self._enter()
        S._ck(load().spdba_rcd_set_spectrum(self.h, ctypes.c_void_p(t.data_ptr())), "spdba_rcd_set_spectrum")
        self.stream.synchronize()

    def get_spectrum(self):
        out = self.torch.empty(self.M * self.N, dtype=self._cplx(), device="cuda")
        self._enter()
        S._ck(load().spdba_rcd_get_spectrum(self.h, ctypes.c_void_p(out.data_ptr())), "spdba_rcd_get_spectrum")
        self.stream.synchronize()
        return out

    def apply(self, rhs, sync=True):
        t = self._dev(rhs, self._cplx())
        self._enter()
        S._ck(load().spdba_rcd_apply(self.h, ctypes.c_void_p(t.data_ptr())), "spdba_rcd_apply")
        if sync:
            self.stream.synchronize()
        self._keep = t  # alive until the stream has consumed it

    def step(self, n=1):
        self._enter()
        S._ck(load().spdba_rcd_step(self.h, int(n)), "spdba_rcd_step")

    def indicator(self):
        ab = np.zeros(self.n_blocks)
        G = ctypes.c_double()
        S._ck(load().spdba_rcd_indicator(self.h, ab.ctypes.data, ab.size, ctypes.byref(G)), "spdba_rcd_indicator")
        return ab, G.value

    def active_mask(self):
        m = np.zeros(self.n_blocks, np.uint8)
        c = ctypes.c_int64()
        S._ck(load().spdba_rcd_active_mask(self.h, m.ctypes.data, m.size, ctypes.byref(c)), "spdba_rcd_active_mask")
        return m, c.value

    def stats(self):
        st = RcdStats()
        S._ck(load().spdba_rcd_stats(self.h, ctypes.byref(st)), "spdba_rcd_stats")
        return {"n_blocks": st.n_blocks, "active_blocks": st.active_blocks, "G": st.G,
                "stage_ms": [float(x) for x in st.stage_ms]}

    def destroy(self):
        if self.h:
            self.stream.synchronize()
            load().spdba_rcd_destroy(self.h)
            self.h = None
