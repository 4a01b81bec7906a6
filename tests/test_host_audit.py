"""Host-only layout audit (spdba_plan_audit): no GPU.

The audit builds a plan's instance table, grid groups and buffer regions the
way plan creation does and checks every transform's input and output span
(lengths, strides, distances, batch) and every device-to-device copy against
the region it runs on.  These cases cover the half-spectrum layout at the
256^3 size whose timed runs ended in device faults (plan creation refuses it;
the audit does not), its batches of unequal grids and FP64 pitches, and the
full layout of every operator.  A planted error -- a descriptor the layout
must reject -- shows that the audit reports rather than passes silently.
"""
import pytest

from paper_2609_03922_amd import spdba as S

CH = (1.0, 1.0)
GS = (0.16, 0.08, 0.035, 0.060)
XPFC = (1.0, 0.02, 0.1, 1.0, 1.0, 1.0, 1.0)


def D(op, dtype, ndim, n, block, **kw):
    params = {"ch": CH, "gs": GS, "nlse": (-21.7, 1.3, 0.0), "xpfc": XPFC}[op]
    return S.Desc(op=op, dtype=dtype, ndim=ndim, n=n, block=block, tau=1e-6, dx=1.0, dt=0.01, params=params, **kw)


CASES = {
    # the half layout at the sizes of its faulted timed runs
    "half-ch-f32-256^3-b8": [D("ch", "f32", 3, 256, 8, half=True, state_indicator=True)],
    "half-ch-f64-256^3-b8": [D("ch", "f64", 3, 256, 8, half=True)],
    "half-ch-f32-512^3-b8": [D("ch", "f32", 3, 512, 8, half=True)],
    "half-gs-f32-4096^2-b16": [D("gs", "f32", 2, 4096, 16, half=True)],
    # batches of unequal grids (groups in descending size, real slots packed per group)
    "half-gs-f32-batch": [D("gs", "f32", 2, n, 16, half=True) for n in (64, 256, 128, 256, 64)],
    "half-ch-f64-batch": [D("ch", "f64", 3, n, 4, half=True) for n in (16, 64, 32, 64)],
    # the full layout of each operator
    "full-ch-f32-512^3": [D("ch", "f32", 3, 512, 8)],
    "full-gs-f64-batch": [D("gs", "f64", 2, n, 16) for n in (128, 64, 128)],
    "full-nlse-f32-batch": [D("nlse", "f32", 1, 4096, 256) for _ in range(6)],
    "full-xpfc-f32-4096^2": [D("xpfc", "f32", 2, 4096, 16, state_indicator=True)],
}


@pytest.mark.parametrize("name", list(CASES))
def test_every_transform_and_copy_fits_its_region(name):
    st, msg = S.plan_audit(CASES[name])
    assert st == S.SPDBA_OK, (name, S.status_string(st), msg)
    assert msg == ""


def test_half_layout_above_the_cap_is_refused_by_plan_creation_but_audited():
    d = CASES["half-ch-f32-256^3-b8"]
    assert S.plan_audit(d)[0] == S.SPDBA_OK
    # the library's own descriptor check (no device) refuses the grid
    lib = S.load()
    arr = S.descs_array(d)
    import ctypes

    h = ctypes.c_void_p()
    assert lib.spdba_plan_create(arr, 1, None, ctypes.byref(h)) == S.SPDBA_EUNSUPPORTED


def test_audit_reports_invalid_descriptors():
    bad = D("ch", "f32", 3, 32, 8)
    bad.block = 64  # larger than the grid
    st, _ = S.plan_audit([bad])
    assert st == S.SPDBA_EINVAL
    st, _ = S.plan_audit([D("nlse", "f32", 2, 64, 8, half=True)])  # the half layout is for real fields
    assert st == S.SPDBA_EUNSUPPORTED
