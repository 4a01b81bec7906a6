"""Python binding of the multimode DBP entry points of libspdba.so
(include/spdba_mdbp.h): argument marshalling only.

Every step runs in the library's HIP kernels and rocFFT; PyTorch provides the
device memory and the stream.  There is no fallback path: without the built
library the first call raises.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import spdba as S

SPDBA_MDBP_DENSE, SPDBA_MDBP_PIN_K0, SPDBA_MDBP_TIMING, SPDBA_MDBP_GRAPH = 1, 2, 4, 8

# every entry point include/spdba_mdbp.h declares
MDBP_EXPORTS = (
    "spdba_mdbp_create", "spdba_mdbp_buffer_sizes", "spdba_mdbp_bind", "spdba_mdbp_set_spectrum",
    "spdba_mdbp_get_spectrum", "spdba_mdbp_set_field", "spdba_mdbp_get_field", "spdba_mdbp_apply",
    "spdba_mdbp_step", "spdba_mdbp_indicator", "spdba_mdbp_active_mask", "spdba_mdbp_stats",
    "spdba_mdbp_destroy", "spdba_mdbp_coupling",
)


class MdbpDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("block", ctypes.c_int32), ("n", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tau", ctypes.c_double), ("T", ctypes.c_double), ("dz", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta2", ctypes.c_double), ("gamma", ctypes.c_double)]


class MdbpStats(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("active_blocks", ctypes.c_int64), ("G", ctypes.c_double),
                ("stage_ms", ctypes.c_float * 4)]


_ready = False


def load():
    global _ready
    lib = S.load()
    if not _ready:
        P, I32, SZ, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double
        sig = {
            "spdba_mdbp_create": [ctypes.POINTER(MdbpDesc), P, P, ctypes.POINTER(P)],
            "spdba_mdbp_buffer_sizes": [P, ctypes.POINTER(SZ), ctypes.POINTER(SZ)],
            "spdba_mdbp_bind": [P, P, P],
            "spdba_mdbp_set_spectrum": [P, P], "spdba_mdbp_get_spectrum": [P, P],
            "spdba_mdbp_set_field": [P, P], "spdba_mdbp_get_field": [P, P],
            "spdba_mdbp_apply": [P], "spdba_mdbp_step": [P, I32],
            "spdba_mdbp_indicator": [P, P, SZ, P], "spdba_mdbp_active_mask": [P, P, SZ, P],
            "spdba_mdbp_stats": [P, ctypes.POINTER(MdbpStats)], "spdba_mdbp_destroy": [P],
            "spdba_mdbp_coupling": [I32, P, D, P],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        _ready = True
    return lib


def _kbuf(K):
    K = np.ascontiguousarray(np.asarray(K, dtype=np.complex128))
    return K, K.ctypes.data


def coupling(K, delta: float) -> np.ndarray:
    """exp(i delta K) as the library computes it (host)."""
    K, kp = _kbuf(K)
    out = np.zeros_like(K)
    S._ck(load().spdba_mdbp_coupling(K.shape[0], kp, float(delta), out.ctypes.data), "spdba_mdbp_coupling")
    return out


def make_desc(M, n, block, dtype="f32", tau=1e-6, T=1000.0, dz=0.1, alpha=0.1, beta2=-21.0, gamma=1.3,
              dense=False, pin_k0=True, timing=False, graph=False) -> MdbpDesc:
    d = MdbpDesc()
    d.M, d.block, d.n, d.dtype = M, block, n, S.DTYPES[dtype]
    d.flags = (SPDBA_MDBP_DENSE if dense else 0) | (SPDBA_MDBP_PIN_K0 if pin_k0 else 0) | \
              (SPDBA_MDBP_TIMING if timing else 0) | (SPDBA_MDBP_GRAPH if graph else 0)
    d.tau, d.T, d.dz, d.alpha, d.beta2, d.gamma = tau, T, dz, alpha, beta2, gamma
    return d


def create_status(desc: MdbpDesc, K) -> int:
    K, kp = _kbuf(K)
    h = ctypes.c_void_p()
    st = load().spdba_mdbp_create(ctypes.byref(desc), kp, None, ctypes.byref(h))
    if h.value:
        load().spdba_mdbp_destroy(h)
    return st


class MdbpPlan:
    """A bound multimode DBP plan with torch-owned buffers on a stream of its own."""

    def __init__(self, desc: MdbpDesc, K, stream=None):
        import torch

        self.torch = torch
        self.desc, self.M, self.n = desc, desc.M, int(desc.n)
        self.dbl = desc.dtype == S.SPDBA_F64
        self.n_blocks = self.n // desc.block
        lib = load()
        self.stream = stream if stream is not None else torch.cuda.Stream()
        K, kp = _kbuf(K)
        h = ctypes.c_void_p()
        S._ck(lib.spdba_mdbp_create(ctypes.byref(desc), kp, ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(h)), "spdba_mdbp_create")
        self.h = h
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        S._ck(lib.spdba_mdbp_buffer_sizes(h, ctypes.byref(sb), ctypes.byref(wb)), "spdba_mdbp_buffer_sizes")
        self.d_state = torch.empty(sb.value + 256, dtype=torch.uint8, device="cuda")
        self.d_work = torch.empty(wb.value + 256, dtype=torch.uint8, device="cuda")
        S._ck(lib.spdba_mdbp_bind(h, self._al(self.d_state), self._al(self.d_work)), "spdba_mdbp_bind")

    @staticmethod
    def _al(t):
        return ctypes.c_void_p((t.data_ptr() + 255) & ~255)

    def _cplx(self):
        return self.torch.complex128 if self.dbl else self.torch.complex64

    def _dev(self, x):
        t = self.torch.as_tensor(x).to(device="cuda", dtype=self._cplx()).contiguous().view(-1)
        if t.numel() != self.M * self.n:
            raise ValueError(f"expected {self.M * self.n} values, got {t.numel()}")
        return t

    def _call(self, name, *args):
        self.stream.wait_stream(self.torch.cuda.current_stream())
        S._ck(getattr(load(), name)(self.h, *args), name)

    def set_field(self, e):
        t = self._dev(e)
        self._call("spdba_mdbp_set_field", ctypes.c_void_p(t.data_ptr()))
        self.stream.synchronize()

    def set_spectrum(self, e):
        t = self._dev(e)
        self._call("spdba_mdbp_set_spectrum", ctypes.c_void_p(t.data_ptr()))
        self.stream.synchronize()

    def get_field(self):
        out = self.torch.empty(self.M * self.n, dtype=self._cplx(), device="cuda")
        self._call("spdba_mdbp_get_field", ctypes.c_void_p(out.data_ptr()))
        self.stream.synchronize()
        return out

    def get_spectrum(self):
        out = self.torch.empty(self.M * self.n, dtype=self._cplx(), device="cuda")
        self._call("spdba_mdbp_get_spectrum", ctypes.c_void_p(out.data_ptr()))
        self.stream.synchronize()
        return out

    def apply(self):
        self._call("spdba_mdbp_apply")

    def step(self, n=1):
        self._call("spdba_mdbp_step", int(n))

    def indicator(self):
        ab = np.zeros(self.n_blocks)
        G = ctypes.c_double()
        S._ck(load().spdba_mdbp_indicator(self.h, ab.ctypes.data, ab.size, ctypes.byref(G)), "spdba_mdbp_indicator")
        return ab, G.value

    def active_mask(self):
        m = np.zeros(self.n_blocks, np.uint8)
        c = ctypes.c_int64()
        S._ck(load().spdba_mdbp_active_mask(self.h, m.ctypes.data, m.size, ctypes.byref(c)), "spdba_mdbp_active_mask")
        return m, c.value

    def stats(self):
        st = MdbpStats()
        S._ck(load().spdba_mdbp_stats(self.h, ctypes.byref(st)), "spdba_mdbp_stats")
        return {"n_blocks": st.n_blocks, "active_blocks": st.active_blocks, "G": st.G,
                "stage_ms": [float(x) for x in st.stage_ms]}

    def destroy(self):
        if self.h:
            self.stream.synchronize()
            load().spdba_mdbp_destroy(self.h)
            self.h = None
