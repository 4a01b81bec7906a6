"""Host-side checks of libspdba.so that need no GPU: the library loads, exports
every entry point include/spdba.h declares, and rejects invalid descriptors
before touching a device."""
import os
import re

import pytest

from paper_2609_03922_amd import spdba

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="spdba.h"):
    src = open(os.path.join(ROOT, "include", name)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spdba_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = spdba.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(spdba.EXPORTS)
    pnames = header_functions("spdba_proposer.h")
    for n in pnames:
        assert hasattr(lib, n), n
    assert set(pnames) == set(spdba.PROPOSER_EXPORTS)


def test_status_strings():
    assert spdba.status_string(0) == "success"
    assert "invalid" in spdba.status_string(1)
    assert spdba.status_string(99) == "unknown status"


def _good(**kw):
    d = spdba.Desc(op="ch", dtype="f32", ndim=3, n=32, block=8, tau=1e-6, dx=1.0, dt=0.01,
                   params=(1.0, 1.0))
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("mutate,expect", [
    (lambda c: setattr(c, "ndim", 0), spdba.SPDBA_EINVAL),
    (lambda c: setattr(c, "ndim", 4), spdba.SPDBA_EINVAL),
    (lambda c: c.block.__setitem__(2, 5), spdba.SPDBA_EINVAL),      # does not divide
    (lambda c: c.dims.__setitem__(2, 48), spdba.SPDBA_EINVAL),      # not a power of two
    (lambda c: c.dims.__setitem__(1, 64), spdba.SPDBA_EINVAL),      # unequal extents
    (lambda c: setattr(c, "threshold", -1.0), spdba.SPDBA_EINVAL),
    (lambda c: setattr(c, "threshold", float("nan")), spdba.SPDBA_EINVAL),
    (lambda c: setattr(c, "dt", 0.0), spdba.SPDBA_EINVAL),
    (lambda c: setattr(c, "dx", -1.0), spdba.SPDBA_EINVAL),
    (lambda c: setattr(c, "reserved", 1), spdba.SPDBA_EINVAL),
    (lambda c: c.op_params.__setitem__(0, float("inf")), spdba.SPDBA_EINVAL),
    (lambda c: c.op_params.__setitem__(1, -1.0), spdba.SPDBA_EINVAL),   # negative kappa
    (lambda c: c.op_params.__setitem__(0, -0.5), spdba.SPDBA_EINVAL),   # negative mobility
    (lambda c: setattr(c, "op", 9), spdba.SPDBA_EUNSUPPORTED),
    (lambda c: setattr(c, "dtype", 7), spdba.SPDBA_EUNSUPPORTED),
    (lambda c: setattr(c, "flags", 1 << 20), spdba.SPDBA_EUNSUPPORTED),
    (lambda c: (c.block.__setitem__(2, 1)), spdba.SPDBA_EUNSUPPORTED),  # FP32 lane needs 2 values
    # consistency control parameters
    (lambda c: setattr(c, "reserved2", 3), spdba.SPDBA_EINVAL),
    (lambda c: setattr(c, "full_steps", -1), spdba.SPDBA_EINVAL),
    (lambda c: (setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_REFRESH),
                setattr(c, "refresh_period", 0)), spdba.SPDBA_EINVAL),
    (lambda c: (setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_DYN_THRESHOLD),
                setattr(c, "control_interval", 0), setattr(c, "target_ratio", 0.3)), spdba.SPDBA_EINVAL),
    (lambda c: (setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_DYN_THRESHOLD),
                setattr(c, "control_interval", 4), setattr(c, "target_ratio", 1.5)), spdba.SPDBA_EINVAL),
    (lambda c: (setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_DYN_THRESHOLD),
                setattr(c, "control_interval", 4), setattr(c, "target_ratio", 0.0)), spdba.SPDBA_EINVAL),
    (lambda c: (setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_DYN_THRESHOLD),
                setattr(c, "control_interval", 4), setattr(c, "target_ratio", 0.3),
                setattr(c, "deadband", 1.0)), spdba.SPDBA_EINVAL),
    (lambda c: setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_DENSE | spdba.SPDBA_FLAG_TRANSITION),
     spdba.SPDBA_EUNSUPPORTED),
    (lambda c: (setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_DENSE), setattr(c, "full_steps", 2)),
     spdba.SPDBA_EUNSUPPORTED),
    # the transition factors of a block must fit the LDS budget (here 1-D blocks of 8192)
    (lambda c: (setattr(c, "ndim", 1), [c.dims.__setitem__(a, 1) for a in (0, 1)],
                [c.block.__setitem__(a, 1) for a in (0, 1)], c.dims.__setitem__(2, 65536),
                c.block.__setitem__(2, 8192), setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_TRANSITION)),
     spdba.SPDBA_EUNSUPPORTED),
    # half-spectrum layout: real fields of two or three dimensions, x block edge
    # dividing nx/2 (at least 2 with transition states), LDS of the indicator
    (lambda c: (setattr(c, "op", spdba.OPS["nlse"]), setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_HALF_SPECTRUM)),
     spdba.SPDBA_EUNSUPPORTED),
    (lambda c: (setattr(c, "ndim", 1), [c.dims.__setitem__(a, 1) for a in (0, 1)],
                [c.block.__setitem__(a, 1) for a in (0, 1)], setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_HALF_SPECTRUM)),
     spdba.SPDBA_EUNSUPPORTED),
    (lambda c: (c.block.__setitem__(2, 32), setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_HALF_SPECTRUM)),
     spdba.SPDBA_EUNSUPPORTED),  # 32 does not divide 16
    (lambda c: (setattr(c, "dtype", spdba.SPDBA_F64), c.block.__setitem__(2, 1),
                setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_HALF_SPECTRUM | spdba.SPDBA_FLAG_TRANSITION)),
     spdba.SPDBA_EUNSUPPORTED),  # X_0 must hold the columns 0 and 1
    (lambda c: (setattr(c, "ndim", 2), c.dims.__setitem__(0, 1), c.block.__setitem__(0, 1),
                c.dims.__setitem__(1, 8192), c.dims.__setitem__(2, 8192), c.block.__setitem__(1, 2),
                c.block.__setitem__(2, 2), setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_HALF_SPECTRUM)),
     spdba.SPDBA_EUNSUPPORTED),  # 2049 blocks per block row
])
def test_invalid_descriptors_rejected_without_device(mutate, expect):
    c = _good().to_c()
    mutate(c)
    assert spdba.spdba_plan_create_status([c]) == expect


def test_mixed_batch_rejected():
    a = _good().to_c()
    b = _good(dtype="f64").to_c()
    assert spdba.spdba_plan_create_status([a, b]) == spdba.SPDBA_EUNSUPPORTED
    assert spdba.spdba_plan_create_status([]) == spdba.SPDBA_EINVAL


def test_null_arguments():
    lib = spdba.load()
    assert lib.spdba_plan_create(None, 1, None, None) == spdba.SPDBA_EINVAL
    assert lib.spdba_destroy(None) == spdba.SPDBA_OK
    assert lib.spdba_step(None, 1) == spdba.SPDBA_EINVAL
    assert lib.spdba_stats(None, 0, None) == spdba.SPDBA_EINVAL


def _xpfc(**kw):
    d = spdba.Desc(op="xpfc", dtype="f32", ndim=2, n=64, block=16, tau=1e-4, dx=0.7854, dt=0.01,
                   params=(1.0, 0.02, 0.1, 1.0, 1.0, 1.0, 1.0), state_indicator=True)
    for k, v in kw.items():
        setattr(d, k, v)
    return d.to_c()


@pytest.mark.parametrize("mutate,expect", [
    (lambda c: c.op_params.__setitem__(2, 0.0), spdba.SPDBA_EINVAL),      # peak width alpha
    (lambda c: c.op_params.__setitem__(5, 0.0), spdba.SPDBA_EINVAL),      # rho beta
    (lambda c: c.op_params.__setitem__(6, -1.0), spdba.SPDBA_EINVAL),
    (lambda c: setattr(c, "flags", c.flags & ~spdba.SPDBA_FLAG_STATE_INDICATOR), spdba.SPDBA_EUNSUPPORTED),
    (lambda c: setattr(c, "flags", c.flags | spdba.SPDBA_FLAG_HALF_SPECTRUM), spdba.SPDBA_EUNSUPPORTED),
])
def test_xpfc_descriptors_rejected(mutate, expect):
    """XPFC needs a positive peak width and rho beta, the state-amplitude
    measure (or Regular mode), and the full layout."""
    c = _xpfc()
    mutate(c)
    assert spdba.spdba_plan_create_status([c]) == expect


def test_half_layout_refused_above_tested_sizes():
    """The half layout stays on grids of at most 2^18 points: timed 256^3
    runs of it ended in device faults whose cause is still open."""
    d = _good(half=True, state_indicator=True).to_c()
    d.dims[0] = d.dims[1] = d.dims[2] = 128
    assert spdba.spdba_plan_create_status([d]) == spdba.SPDBA_EUNSUPPORTED


def test_half_layout_accepts_consistency_control():
    """Transition states (with the conjugate neighbour remap) and the
    threshold controller on the half layout: the descriptor passes the
    library's checks (the host-only audit runs them without a device)."""
    d = spdba.Desc(op="ch", dtype="f32", ndim=3, n=32, block=8, tau=1e-3, dx=1.0, dt=0.01, params=(1.0, 1.0),
                   half=True, transition=True, refresh=10, full_steps=2, target_ratio=0.2, control_interval=4,
                   deadband=0.05)
    st, msg = spdba.plan_audit([d])
    assert st == spdba.SPDBA_OK, msg
