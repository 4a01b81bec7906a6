"""The allocation-free entry point spdba_apply_noalloc against spdba_apply of
a plan, on the same seeded inputs: spectra, masks and FP64 k = 0 values equal
bit for bit, over consecutive calls of which the later ones are smaller (the
shared scratch array keeps the previous call's contents), in FP32 and FP64,
CH and GS, with the increment and the state measure and in Regular mode."""
import numpy as np
import pytest

from _parity import assert_bits_equal, draw_apply_inputs, k0path
from paper_2609_03922_amd import spdba as S

pytestmark = pytest.mark.gpu

PAR = {"ch": (1.0, 1.0), "gs": (0.16, 0.08, 0.035, 0.060)}


def D(op, dtype, ndim, n, block, tau, **kw):
    return S.Desc(op=op, dtype=dtype, ndim=ndim, n=n, block=block, tau=tau, dx=1.0,
                  dt=0.01 if op == "ch" else 1.0, params=PAR[op], **kw)


def _via_plan(d, q, r, k0, rk0):
    import torch

    plan = S.Plan([d])
    plan.set_spectrum(0, torch.from_numpy(q), k0=k0 if k0path(d) else None)
    plan.apply(torch.from_numpy(r), rk0 if k0path(d) else None)
    hat, k0g = plan.get_spectrum(0)
    out = (hat.cpu().numpy(), plan.active_mask(0), k0g.copy())
    plan.destroy()
    return out


def _noalloc(d, q, r, k0, rk0):
    import torch

    st = torch.from_numpy(q.copy()).cuda()
    rh = torch.from_numpy(r).cuda()
    mask = torch.full((d.n_blocks,), 7, dtype=torch.uint8, device="cuda")  # stale bytes
    k0t = rk0t = None
    if k0path(d):
        k0t = torch.zeros(2, dtype=torch.float64, device="cuda")
        k0t[: d.nspec] = torch.from_numpy(k0)
        rk0t = torch.zeros(2, dtype=torch.float64, device="cuda")
        rk0t[: d.nspec] = torch.from_numpy(rk0)
    torch.cuda.synchronize()
    s = S.spdba_apply_noalloc(d, st, rh, k0t, rk0t, mask)
    assert s == S.SPDBA_OK, S.status_string(s)
    torch.cuda.synchronize()
    k0o = k0t.cpu().numpy()[: d.nspec] if k0t is not None else np.zeros(d.nspec)
    return st.cpu().numpy(), mask.cpu().numpy(), k0o


SEQ = [  # consecutive calls, later ones smaller
    (D("ch", "f32", 3, 64, 8, 1e-3), 31),
    (D("ch", "f32", 3, 32, 8, 1e-3), 32),
    (D("gs", "f32", 2, 64, 16, 1e-2, state_indicator=True), 33),
    (D("ch", "f64", 2, 32, 8, 3e-2), 34),
    (D("ch", "f32", 2, 32, 8, 0.0, dense=True), 35),
]


def test_noalloc_equals_plan_apply_over_consecutive_calls():
    for d, seed in SEQ:
        q, r, k0, rk0 = draw_apply_inputs(d, seed, 0)
        if k0path(d):  # a plan keeps slot 0 of each species at zero (its value is k0)
            for s in range(d.nspec):
                q[s * d.n_modes] = 0
        want = _via_plan(d, q, r, k0, rk0)
        got = _noalloc(d, q, r, k0, rk0)
        tag = f"noalloc {d.op} {d.dtype} {d.ndim}-D n={d.n} seed {seed}"
        print(tag, "active", int(want[1].sum()), "of", d.n_blocks, flush=True)
        assert_bits_equal(got[1], want[1], tag + " mask")
        assert_bits_equal(got[0], want[0], tag + " coefficients")
        if k0path(d):
            assert_bits_equal(got[2], want[2], tag + " k0")
        if not d.dense:
            assert 0 < want[1].sum() < d.n_blocks


def test_noalloc_rejects_beyond_its_scratch():
    import torch

    d = D("ch", "f32", 3, 1024, 8, 1e-3)  # 2^21 blocks > 2^18
    t = torch.zeros(2, dtype=torch.complex64, device="cuda")
    assert S.spdba_apply_noalloc(d, t, t, None, None, t) == S.SPDBA_EUNSUPPORTED
    d = D("ch", "f32", 3, 32, 8, 1e-3, half=True)
    assert S.spdba_apply_noalloc(d, t, t, None, None, t) == S.SPDBA_EUNSUPPORTED
