"""Python binding of libspdba.so (include/spdba.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels and rocFFT; this
module converts Python values to the C ABI and back.  PyTorch provides device
memory and the stream.  If the library is not built the import of any entry
point fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspdba.so")

SPDBA_OK, SPDBA_EINVAL, SPDBA_EUNSUPPORTED, SPDBA_ESTATE = 0, 1, 2, 3
SPDBA_EDEVICE, SPDBA_EFFT, SPDBA_ENONFINITE = 4, 5, 6
SPDBA_OP_CAHN_HILLIARD, SPDBA_OP_GRAY_SCOTT, SPDBA_OP_NLSE, SPDBA_OP_XPFC = 1, 2, 3, 4
SPDBA_F32, SPDBA_F64 = 0, 1
SPDBA_FLAG_DENSE, SPDBA_FLAG_PIN_K0, SPDBA_FLAG_GRAPH, SPDBA_FLAG_TIMING = 1, 2, 4, 8
SPDBA_FLAG_TRANSITION, SPDBA_FLAG_REFRESH, SPDBA_FLAG_DYN_THRESHOLD = 16, 32, 64
SPDBA_FLAG_STATE_INDICATOR = 128
SPDBA_FLAG_HALF_SPECTRUM = 256
SPDBA_FLAG_BLOCK_ENERGY = 512

OPS = {"ch": SPDBA_OP_CAHN_HILLIARD, "gs": SPDBA_OP_GRAY_SCOTT, "nlse": SPDBA_OP_NLSE, "xpfc": SPDBA_OP_XPFC}
DTYPES = {"f32": SPDBA_F32, "f64": SPDBA_F64}

# every entry point the header declares
EXPORTS = (
    "spdba_plan_create", "spdba_plan_buffer_sizes", "spdba_plan_bind", "spdba_set_field",
    "spdba_get_field", "spdba_set_spectrum", "spdba_get_spectrum", "spdba_step", "spdba_apply",
    "spdba_set_skip", "spdba_active_mask", "spdba_indicator", "spdba_worklist",
    "spdba_device_views", "spdba_stats", "spdba_set_launch", "spdba_destroy",
    "spdba_status_string", "spdba_apply_noalloc", "spdba_plan_audit",
)
# entry points of include/spdba_proposer.h
PROPOSER_EXPORTS = (
    "spdba_mlp_forward", "spdba_mlp_backward_scratch", "spdba_mlp_backward", "spdba_mlp_bce",
    "spdba_mlp_adam", "spdba_mlp_to_bf16", "spdba_proposer_features", "spdba_proposer_labels",
    "spdba_proposer_skip", "spdba_proposer_miss", "spdba_set_block_energy",
)


class SpdbaError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class InstanceDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("op", ctypes.c_int32),
        ("dims", ctypes.c_int64 * 3),
        ("block", ctypes.c_int32 * 3),
        ("dtype", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_int32),
        ("threshold", ctypes.c_double),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("op_params", ctypes.c_double * 8),
        ("refresh_period", ctypes.c_int32),
        ("full_steps", ctypes.c_int32),
        ("control_interval", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
        ("target_ratio", ctypes.c_double),
        ("deadband", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64),
        ("active_blocks", ctypes.c_int64),
        ("total_blocks", ctypes.c_int64),
        ("G", ctypes.c_double),
        ("mean", ctypes.c_double * 2),
        ("energy", ctypes.c_double),
        ("stage_ms", ctypes.c_double * 6),
        ("input_preserving_fft", ctypes.c_int32),
        ("graph_replay", ctypes.c_int32),
        ("indicator_kernel_ms", ctypes.c_double),
        ("transition_blocks", ctypes.c_int64),
        ("tau", ctypes.c_double),
        ("control_step", ctypes.c_int64),
        ("nonfrozen_ratio_mean", ctypes.c_double),
    ]


_lib = None


def load():
    """Load libspdba.so (import torch first so that one HIP runtime is shared)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)

    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "spdba_plan_create": [ctypes.POINTER(InstanceDesc), I32, P, ctypes.POINTER(P)],
        "spdba_plan_buffer_sizes": [P, ctypes.POINTER(SZ), ctypes.POINTER(SZ)],
        "spdba_plan_bind": [P, P, P],
        "spdba_set_field": [P, I32, P],
        "spdba_get_field": [P, I32, P],
        "spdba_set_spectrum": [P, I32, P, P],
        "spdba_get_spectrum": [P, I32, P, P],
        "spdba_step": [P, I32],
        "spdba_apply": [P, P, P],
        "spdba_set_skip": [P, P],
        "spdba_active_mask": [P, I32, P, SZ],
        "spdba_indicator": [P, I32, P, SZ, P],
        "spdba_worklist": [P, I32, P, SZ, ctypes.POINTER(I64)],
        "spdba_device_views": [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                               ctypes.POINTER(I64)],
        "spdba_stats": [P, I32, ctypes.POINTER(Stats)],
        "spdba_set_launch": [P, I32, I32],
        "spdba_destroy": [P],
        "spdba_status_string": [I32],
        "spdba_mlp_forward": [P, I64, P, P, P, P, P, P],
        "spdba_mlp_backward_scratch": [I64],
        "spdba_mlp_backward": [P, P, P, P, I64, P, P, P, P],
        "spdba_mlp_bce": [P, P, I64, ctypes.c_float, P, P, P, P],
        "spdba_mlp_adam": [P, P, P, P, P, I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, I64, P],
        "spdba_mlp_to_bf16": [P, P, I64, P],
        "spdba_proposer_features": [P, P, P, P, P, ctypes.c_float, P, P, P],
        "spdba_proposer_labels": [P, I32, I64, P, P],
        "spdba_proposer_skip": [P, I64, ctypes.c_float, P, P, P, P],
        "spdba_proposer_miss": [P, P, I64, P, P],
        "spdba_set_block_energy": [P, P],
        "spdba_apply_noalloc": [ctypes.POINTER(InstanceDesc), P, P, P, P, P, P],
        "spdba_plan_audit": [ctypes.POINTER(InstanceDesc), I32, ctypes.c_char_p, SZ],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = (ctypes.c_char_p if name == "spdba_status_string" else
                      ctypes.c_size_t if name == "spdba_mlp_backward_scratch" else ctypes.c_int32)
    _lib = lib
    return lib


def spdba_apply_noalloc(desc, state, rhs, k0=None, rhs_k0=None, mask=None, stream=None) -> int:
    """The allocation-free update stage of one instance (include/spdba.h):
    torch device tensors in and out (state updated in place, mask written);
    returns the status."""
    arr = descs_array([desc])
    ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
    return load().spdba_apply_noalloc(arr, ptr(state), ptr(rhs), ptr(k0), ptr(rhs_k0), ptr(mask), sp)


def plan_audit(descs) -> tuple:
    """The host-only layout audit (include/spdba.h): (status, message); no
    device is needed."""
    arr = descs_array(list(descs))
    buf = ctypes.create_string_buffer(512)
    st = load().spdba_plan_audit(arr, len(descs), buf, len(buf))
    return st, buf.value.decode()


def status_string(s: int) -> str:
    return load().spdba_status_string(int(s)).decode()


def _ck(status: int, where: str):
    if status != SPDBA_OK:
        raise SpdbaError(status, where)


@dataclass
class Desc:
    """One instance: operator, precision, grid, block shape, threshold, parameters."""

    op: str
    dtype: str
    ndim: int
    n: int
    block: int
    tau: float
    dx: float
    dt: float
    params: tuple
    dense: bool = False
    pin_k0: bool = True
    graph: bool = False
    timing: bool = False
    # consistency control (Supplementary S1.1, S1.3): transition blocks, a
    # full step every `refresh` steps (0: off), `full_steps` initial full
    # steps, and the threshold controller when target_ratio > 0
    transition: bool = False
    refresh: int = 0
    full_steps: int = 0
    target_ratio: float = 0.0
    control_interval: int = 0
    deadband: float = 0.0
    # activity measure from the state amplitude instead of the increment
    state_indicator: bool = False
    # half-spectrum layout of a real field (Supplementary S1.2)
    half: bool = False
    # with state_indicator: block energy (the block's sum of |q|^2) instead of the maximum
    block_energy: bool = False

    @property
    def dims3(self):
        return tuple([1] * (3 - self.ndim) + [self.n] * self.ndim)

    @property
    def block3(self):
        return tuple([1] * (3 - self.ndim) + [self.block] * self.ndim)

    @property
    def n_points(self):
        """Grid points per species (the real-space field)."""
        return self.n ** self.ndim

    @property
    def stored_dims(self):
        """Extents of the stored spectrum (x keeps n/2 + 1 columns in the half layout)."""
        d = self.dims3
        return d[:2] + (d[2] // 2 + 1,) if self.half else d

    @property
    def n_modes(self):
        """Stored modes per species."""
        return int(np.prod(self.stored_dims))

    @property
    def n_blocks(self):
        nb = self.n // self.block
        if self.half:  # columns below n/2, then one block per (z, y) block row for n/2
            rows = nb ** (self.ndim - 1)
            return rows * (self.n // (2 * self.block) + 1)
        return nb ** self.ndim

    @property
    def nspec(self):
        return 2 if self.op == "gs" else 1

    def to_c(self) -> InstanceDesc:
        d = InstanceDesc()
        d.ndim = self.ndim
        d.op = OPS[self.op]
        for a in range(3):
            d.dims[a] = self.dims3[a]
            d.block[a] = self.block3[a]
        d.dtype = DTYPES[self.dtype]
        d.flags = ((SPDBA_FLAG_DENSE if self.dense else 0) | (SPDBA_FLAG_PIN_K0 if self.pin_k0 else 0)
                   | (SPDBA_FLAG_GRAPH if self.graph else 0) | (SPDBA_FLAG_TIMING if self.timing else 0)
                   | (SPDBA_FLAG_TRANSITION if self.transition else 0)
                   | (SPDBA_FLAG_REFRESH if self.refresh else 0)
                   | (SPDBA_FLAG_DYN_THRESHOLD if self.target_ratio else 0)
                   | (SPDBA_FLAG_STATE_INDICATOR if self.state_indicator else 0)
                   | (SPDBA_FLAG_HALF_SPECTRUM if self.half else 0)
                   | (SPDBA_FLAG_BLOCK_ENERGY if self.block_energy else 0))
        d.reserved = 0
        d.threshold = float(self.tau)
        d.dx, d.dt = float(self.dx), float(self.dt)
        pp = list(self.params) + [0.0] * (8 - len(self.params))
        for i in range(8):
            d.op_params[i] = float(pp[i])
        d.refresh_period = int(self.refresh)
        d.full_steps = int(self.full_steps)
        d.control_interval = int(self.control_interval)
        d.reserved2 = 0
        d.target_ratio = float(self.target_ratio)
        d.deadband = float(self.deadband)
        return d


def descs_array(descs):
    arr = (InstanceDesc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d.to_c() if isinstance(d, Desc) else d
    return arr


def spdba_plan_create(descs, stream=None) -> ctypes.c_void_p:
    arr = descs_array(descs)
    h = ctypes.c_void_p()
    _ck(load().spdba_plan_create(arr, len(descs), stream, ctypes.byref(h)), "spdba_plan_create")
    return h


def spdba_plan_create_status(descs, stream=None) -> int:
    """Status of plan creation only (no plan kept); used by validation tests."""
    arr = descs_array(descs)
    h = ctypes.c_void_p()
    st = load().spdba_plan_create(arr, len(descs), stream, ctypes.byref(h))
    if st == SPDBA_OK:
        load().spdba_destroy(h)
    return st


class Plan:
    """A bound plan with torch-owned state and work buffers."""

    def __init__(self, descs, stream=None):
        import torch

        self.descs = list(descs)
        self.torch = torch
        # a stream of its own (default priority): HIP graphs cannot be captured
        # on the legacy default stream
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.h = spdba_plan_create(self.descs, ctypes.c_void_p(self.stream.cuda_stream))
        lib = load()
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _ck(lib.spdba_plan_buffer_sizes(self.h, ctypes.byref(sb), ctypes.byref(wb)), "buffer_sizes")
        self.state_bytes, self.work_bytes = sb.value, wb.value
        # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
        self.d_state = torch.empty(self.state_bytes + 256, dtype=torch.uint8, device="cuda")
        self.d_work = torch.empty(self.work_bytes + 256, dtype=torch.uint8, device="cuda")
        sp = self._aligned(self.d_state)
        wp = self._aligned(self.d_work)
        _ck(lib.spdba_plan_bind(self.h, sp, wp), "spdba_plan_bind")
        self._skip = None

    @staticmethod
    def _aligned(t):
        p = t.data_ptr()
        return ctypes.c_void_p((p + 255) & ~255)

    def _enter(self):
        # work already queued by torch (copies of inputs) precedes the library's
        self.stream.wait_stream(self.torch.cuda.current_stream())

    # ---- dtype helpers --------------------------------------------------
    def _real_dtype(self, i):
        return self.torch.float64 if self.descs[i].dtype == "f64" else self.torch.float32

    def _cplx_dtype(self, i):
        return self.torch.complex128 if self.descs[i].dtype == "f64" else self.torch.complex64

    # ---- field / spectrum -----------------------------------------------
    def set_field(self, i, field):
        d = self.descs[i]
        want = self._cplx_dtype(i) if d.op == "nlse" else self._real_dtype(i)
        field = field.to(device="cuda", dtype=want).contiguous()
        assert field.numel() == d.n_points * d.nspec
        self._enter()
        _ck(load().spdba_set_field(self.h, i, ctypes.c_void_p(field.data_ptr())), "spdba_set_field")
        self.stream.synchronize()

    def get_field(self, i):
        d = self.descs[i]
        want = self._cplx_dtype(i) if d.op == "nlse" else self._real_dtype(i)
        out = self.torch.empty(d.n_points * d.nspec, dtype=want, device="cuda")
        self._enter()
        _ck(load().spdba_get_field(self.h, i, ctypes.c_void_p(out.data_ptr())), "spdba_get_field")
        self.stream.synchronize()
        return out

    def set_spectrum(self, i, hat, k0=None):
        d = self.descs[i]
        hat = hat.to(device="cuda", dtype=self._cplx_dtype(i)).contiguous()
        assert hat.numel() == d.n_modes * d.nspec
        kk = None
        if k0 is not None:
            k0a = np.ascontiguousarray(k0, dtype=np.float64)
            kk = k0a.ctypes.data_as(ctypes.c_void_p)
        self._enter()
        _ck(load().spdba_set_spectrum(self.h, i, ctypes.c_void_p(hat.data_ptr()), kk), "set_spectrum")
        self.stream.synchronize()

    def get_spectrum(self, i):
        d = self.descs[i]
        out = self.torch.empty(d.n_modes * d.nspec, dtype=self._cplx_dtype(i), device="cuda")
        k0 = np.zeros(2, np.float64)
        self._enter()
        _ck(load().spdba_get_spectrum(self.h, i, ctypes.c_void_p(out.data_ptr()),
                                      k0.ctypes.data_as(ctypes.c_void_p)), "get_spectrum")
        self.stream.synchronize()
        return out, k0[: d.nspec].copy()

    # ---- stepping -------------------------------------------------------
    def step(self, n=1):
        _ck(load().spdba_step(self.h, int(n)), "spdba_step")

    def synchronize(self):
        self.stream.synchronize()

    def apply(self, rhs=None, rhs_k0=None):
        rp = None
        if rhs is not None:
            rhs = rhs.to(device="cuda", dtype=self._cplx_dtype(0)).contiguous()
            rp = ctypes.c_void_p(rhs.data_ptr())
        kp = None
        if rhs_k0 is not None:
            rk = np.ascontiguousarray(rhs_k0, dtype=np.float64)
            kp = rk.ctypes.data_as(ctypes.c_void_p)
        self._enter()
        _ck(load().spdba_apply(self.h, rp, kp), "spdba_apply")
        self.stream.synchronize()  # keeps rhs alive until the copies ran

    def set_skip(self, skip):
        self._skip = None if skip is None else skip.to(device="cuda", dtype=self.torch.uint8).contiguous()
        ptr = None if self._skip is None else ctypes.c_void_p(self._skip.data_ptr())
        self._enter()
        _ck(load().spdba_set_skip(self.h, ptr), "spdba_set_skip")

    def set_launch(self, kernel, value):
        _ck(load().spdba_set_launch(self.h, int(kernel), int(value)), "spdba_set_launch")

    # ---- read-backs -----------------------------------------------------
    def active_mask(self, i):
        nb = self.descs[i].n_blocks
        out = np.zeros(nb, np.uint8)
        _ck(load().spdba_active_mask(self.h, i, out.ctypes.data_as(ctypes.c_void_p), nb), "active_mask")
        return out

    def indicator(self, i):
        nb = self.descs[i].n_blocks
        ab = np.zeros(nb, np.float64)
        G = ctypes.c_double()
        _ck(load().spdba_indicator(self.h, i, ab.ctypes.data_as(ctypes.c_void_p), nb,
                                   ctypes.byref(G)), "indicator")
        return ab, G.value

    def worklist(self, i):
        nb = self.descs[i].n_blocks
        out = np.zeros(nb, np.uint32)
        cnt = ctypes.c_int64()
        _ck(load().spdba_worklist(self.h, i, out.ctypes.data_as(ctypes.c_void_p), nb,
                                  ctypes.byref(cnt)), "worklist")
        return out[: cnt.value].copy()

    def device_views(self):
        """(a_b, mask, G) device addresses and the number of blocks."""
        ab, mk, g, nb = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
        _ck(load().spdba_device_views(self.h, ctypes.byref(ab), ctypes.byref(mk), ctypes.byref(g),
                                      ctypes.byref(nb)), "device_views")
        return ab.value, mk.value, g.value, nb.value

    def set_block_energy(self, eb):
        """eb: torch float64 tensor with one value per block of the plan, or None."""
        self._eb = eb
        ptr = None if eb is None else ctypes.c_void_p(eb.data_ptr())
        _ck(load().spdba_set_block_energy(self.h, ptr), "spdba_set_block_energy")

    def total_blocks(self):
        return sum(d.n_blocks for d in self.descs)

    def stats(self, i):
        s = Stats()
        _ck(load().spdba_stats(self.h, i, ctypes.byref(s)), "spdba_stats")
        return dict(steps=s.steps, active_blocks=s.active_blocks, total_blocks=s.total_blocks,
                    G=s.G, mean=list(s.mean), energy=s.energy, stage_ms=list(s.stage_ms),
                    input_preserving_fft=s.input_preserving_fft, graph_replay=s.graph_replay,
                    indicator_kernel_ms=s.indicator_kernel_ms, transition_blocks=s.transition_blocks,
                    tau=s.tau, control_step=s.control_step, nonfrozen_ratio_mean=s.nonfrozen_ratio_mean)

    def destroy(self):
        if self.h is not None and self.h.value:
            self.stream.synchronize()  # the buffers go back to torch below
            load().spdba_destroy(self.h)
        self.h = None
        self.d_state = self.d_work = self._skip = None
        self._eb = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def desc_from_config(cfg: dict, n: int | None = None, **over) -> Desc:
    """Descriptor of one instance of a workload record (configs.py)."""
    from . import inputs  # noqa: F401  (kept beside the configs)

    d = Desc(op=cfg["op"], dtype=cfg["dtype"], ndim=cfg["ndim"], n=n if n is not None else cfg["n"],
             block=cfg["block"], tau=cfg["tau"], dx=cfg["dx"], dt=cfg["dt"], params=tuple(cfg["params"]),
             half=cfg.get("layout", "full") == "half")
    for k, v in over.items():
        setattr(d, k, v)
    return d


# ---------------------------------------------------------------------------
# proposer entry points (include/spdba_proposer.h), torch tensors in and out
# ---------------------------------------------------------------------------

def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _sp(stream):
    return ctypes.c_void_p(stream.cuda_stream) if stream is not None else None


def spdba_mlp_forward(x, w_bf16, prob=None, logit=None, h1=None, h2=None, stream=None):
    _ck(load().spdba_mlp_forward(_p(x), x.shape[0], _p(w_bf16), _p(prob), _p(logit), _p(h1), _p(h2),
                                 _sp(stream)), "spdba_mlp_forward")


def spdba_mlp_backward_scratch(n):
    return int(load().spdba_mlp_backward_scratch(int(n)))


def spdba_mlp_backward(x, h1, h2, dlogit, w, grad, scratch, stream=None):
    _ck(load().spdba_mlp_backward(_p(x), _p(h1), _p(h2), _p(dlogit), x.shape[0], _p(w), _p(grad),
                                  _p(scratch), _sp(stream)), "spdba_mlp_backward")


def spdba_mlp_bce(logit, y, pos_weight, dlogit, loss, scratch, stream=None):
    _ck(load().spdba_mlp_bce(_p(logit), _p(y), logit.shape[0], float(pos_weight), _p(dlogit), _p(loss),
                             _p(scratch), _sp(stream)), "spdba_mlp_bce")


def spdba_mlp_adam(w, m, v, g, w_bf16, lr, t, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _ck(load().spdba_mlp_adam(_p(w), _p(m), _p(v), _p(g), _p(w_bf16), w.numel(), float(lr), float(beta1),
                              float(beta2), float(eps), int(t), _sp(stream)), "spdba_mlp_adam")


def spdba_mlp_to_bf16(w, w_bf16, stream=None):
    _ck(load().spdba_mlp_to_bf16(_p(w), _p(w_bf16), w.numel(), _sp(stream)), "spdba_mlp_to_bf16")


def spdba_proposer_features(plan, ab3, G3, mask_addr, eb, step_fraction, x, scratch, stream=None):
    """ab3 / G3: three device addresses (ints) or tensors each; mask_addr: int or tensor."""
    addr = lambda t: t if isinstance(t, int) else t.data_ptr()
    abp = (ctypes.c_void_p * 3)(*[addr(t) for t in ab3])
    gp = (ctypes.c_void_p * 3)(*[addr(t) for t in G3])
    _ck(load().spdba_proposer_features(plan.h, abp, gp, ctypes.c_void_p(addr(mask_addr)), _p(eb),
                                       float(step_fraction), _p(x), _p(scratch), _sp(stream)),
        "spdba_proposer_features")


def spdba_proposer_labels(masks, y, stream=None):
    """masks: torch uint8 [n_masks, total_blocks]."""
    _ck(load().spdba_proposer_labels(_p(masks), masks.shape[0], masks.shape[1], _p(y), _sp(stream)),
        "spdba_proposer_labels")


def spdba_proposer_skip(prob, threshold, skip, gate=None, count=None, stream=None):
    _ck(load().spdba_proposer_skip(_p(prob), prob.numel(), float(threshold), _p(gate), _p(skip), _p(count),
                                   _sp(stream)), "spdba_proposer_skip")


def spdba_proposer_miss(skip, mask_addr, nb, count, stream=None):
    m = mask_addr if isinstance(mask_addr, int) else mask_addr.data_ptr()
    _ck(load().spdba_proposer_miss(_p(skip), ctypes.c_void_p(m), int(nb), _p(count), _sp(stream)),
        "spdba_proposer_miss")
