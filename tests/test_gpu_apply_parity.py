"""Kernel-level parity through the C ABI: identical seeded spectra go into
spdba_apply and into the oracle; a_b, G, mask, ordered worklist, updated
coefficients and the FP64 k = 0 values must agree bit for bit."""
import numpy as np
import pytest

from _parity import (assert_bits_equal, draw_apply_inputs, k0path, oracle_apply)
from paper_2609_03922_amd import inputs
from paper_2609_03922_amd import spdba as S

pytestmark = pytest.mark.gpu

CH = (1.0, 1.0)
GS = (0.16, 0.08, 0.035, 0.060)
NL = (-21.7, 1.3, 0.0)


def D(op, dtype, ndim, n, block, tau, dx=1.0, dt=0.01, params=None, **kw):
    p = params or {"ch": CH, "gs": GS, "nlse": NL}[op]
    if op == "nlse" and dx == 1.0:
        dx, dt = 15.625, 0.8
    if op == "gs" and dt == 0.01:
        dt = 1.0
    return S.Desc(op=op, dtype=dtype, ndim=ndim, n=n, block=block, tau=tau, dx=dx, dt=dt, params=p, **kw)


def run_case(descs, seed, skip=None, floor=0.0, update_variant=None):
    import torch

    plan = S.Plan(descs)
    if update_variant is not None:
        plan.set_launch(3, update_variant)
    ins = [draw_apply_inputs(d, seed, i, floor=floor) for i, d in enumerate(descs)]
    for i, (d, (q, r, k0, rk0)) in enumerate(zip(descs, ins)):
        plan.set_spectrum(i, torch.from_numpy(q), k0=k0 if k0path(d) else None)
    rhs = None
    rk = None
    if descs[0].op != "nlse":
        rhs = torch.from_numpy(np.concatenate([r for (_, r, _, _) in ins]))
        if k0path(descs[0]):
            rk = np.concatenate([rk0 for (_, _, _, rk0) in ins])
    if skip is not None:
        plan.set_skip(torch.from_numpy(np.concatenate(skip)))
    plan.apply(rhs, rk)
    off = 0
    for i, (d, (q, r, k0, rk0)) in enumerate(zip(descs, ins)):
        sk = None if skip is None else skip[i]
        ref = oracle_apply(d, q, r, k0, rk0, skip=sk)
        ab, G = plan.indicator(i)
        mask = plan.active_mask(i)
        wl = plan.worklist(i)
        hat, k0g = plan.get_spectrum(i)
        tag = f"inst {i} {d.op}/{d.dtype} n={d.n} b={d.block} tau={d.tau}"
        assert_bits_equal(mask, ref["mask"], tag + " mask")
        assert_bits_equal(wl, ref["worklist"], tag + " worklist")
        if not d.dense:
            assert_bits_equal(ab, ref["a_b"], tag + " a_b")
            assert G == ref["G"], (tag, G, ref["G"])
        assert_bits_equal(hat.cpu().numpy(), ref["q"], tag + " coefficients")
        if k0path(d):
            assert_bits_equal(k0g, ref["k0"], tag + " k0")
    plan.destroy()
    return ins


CASES = [
    # (descs, seed)
    ([D("ch", "f64", 2, 64, 16, 1e-6)], 1),
    ([D("ch", "f64", 2, 128, 16, 1e-6)], 2),
    ([D("ch", "f64", 2, 64, 16, 0.0)], 3),
    ([D("ch", "f64", 2, 64, 8, 3e-2)], 4),
    ([D("ch", "f32", 3, 32, 8, 1e-6)], 5),
    ([D("ch", "f32", 3, 64, 8, 3e-3)], 6),
    ([D("ch", "f32", 2, 16, 4, 1e-2)], 7),     # strip narrower than a wave row
    ([D("ch", "f32", 1, 4096, 1024, 1e-3)], 8),  # block row wider than a wave row
    ([D("ch", "f32", 3, 32, 8, 1e-6, dense=True)], 9),
    ([D("ch", "f32", 3, 32, 8, 1e-3, pin_k0=False)], 10),
    ([D("gs", "f32", 2, n, 32, 1e-6) for n in (128, 64, 256, 64)], 11),
    ([D("gs", "f32", 2, n, 16, 1e-2) for n in (64, 32)], 12),
    ([D("gs", "f64", 2, 64, 16, 1e-4)], 13),
    ([D("nlse", "f32", 1, n, 1024, 1e-6) for n in (4096, 16384, 8192, 4096)], 14),
    ([D("nlse", "f32", 1, n, 64, 1e-3) for n in (2048, 1024)], 15),
    ([D("nlse", "f64", 1, 4096, 256, 1e-5)], 16),
    ([D("nlse", "f32", 1, 4096, 256, 1e-4, dense=True)], 17),
    ([D("ch", "f32", 2, 512, 256, 1e-3)], 18),    # 2-D blocks whose rows span two wave rows
    ([D("gs", "f32", 2, 512, 256, 1e-3), D("gs", "f32", 2, 1024, 256, 1e-3)], 19),
    ([D("ch", "f64", 3, 32, 8, 1e-6)], 23),     # three-dimensional FP64 (the equal-error truth's path)
    ([D("ch", "f64", 3, 64, 8, 3e-3)], 24),
    ([D("ch", "f64", 3, 32, 8, 0.0, dense=True)], 25),
]


@pytest.mark.parametrize("variant", [1, 0, 2, 3, 4],
                         ids=["strip_walk", "block_list", "block_list_x4", "wave_walk", "run_walk"])
@pytest.mark.parametrize("descs,seed", CASES, ids=[f"case{c[1]}" for c in CASES])
def test_apply_bit_exact(descs, seed, variant):
    print(f"apply parity case {seed} update variant {variant}: "
          f"{[(d.op, d.dtype, d.n, d.block, d.tau) for d in descs]}", flush=True)
    run_case(descs, seed, update_variant=variant)


def test_apply_skip_set_bit_exact():
    d = D("ch", "f32", 3, 32, 8, 1e-4)
    r = inputs.rng_for(77, 0)
    skip = (r.random(d.n_blocks) < 0.3).astype(np.uint8)
    run_case([d], 21, skip=[skip])


def test_apply_floor_all_active_and_nonfinite():
    import torch

    d = D("ch", "f32", 3, 32, 8, 1e-6)
    run_case([d], 22, floor=1e-3)
    plan = S.Plan([d])
    q, r, k0, rk0 = draw_apply_inputs(d, 23, 0)
    r[5] = np.nan
    plan.set_spectrum(0, torch.from_numpy(q), k0=k0)
    plan.apply(torch.from_numpy(r), rk0)
    with pytest.raises(S.SpdbaError) as e:
        plan.active_mask(0)
    assert e.value.status == S.SPDBA_ENONFINITE
    plan.destroy()


def _batch(cfg):
    from paper_2609_03922_amd import configs  # noqa: F401

    return [S.desc_from_config(cfg, n=n) for n in inputs.instance_sizes(cfg)]


def _full_cases():
    from paper_2609_03922_amd import configs as C

    return [
        ("ch3d_256_f32", lambda: [S.desc_from_config(C.CH3D_256_F32)], 31),
        ("ch2d_128_f64", lambda: [S.desc_from_config(C.CH2D_128_F64)], 32),
        ("nlse1d_batch48_f32", lambda: _batch(C.NLSE1D_BATCH48_F32), 33),
        ("gs2d_batch32_f32", lambda: _batch(C.GS2D_BATCH32_F32), 34),
        ("ch3d_512_f32", lambda: [S.desc_from_config(C.CH3D_512_F32_PROPOSER)], 35),
    ]


STATE_CASES = [
    ([D("ch", "f64", 2, 64, 16, 1e-3, state_indicator=True)], 41),
    ([D("ch", "f32", 3, 32, 8, 1e-2, state_indicator=True)], 42),
    ([D("ch", "f32", 3, 32, 8, 1e-2, state_indicator=True, pin_k0=False)], 43),
    ([D("gs", "f32", 2, n, 32, 1e-2, state_indicator=True) for n in (128, 64, 256)], 44),
    ([D("gs", "f64", 2, 64, 16, 1e-2, state_indicator=True)], 45),
    ([D("nlse", "f32", 1, n, 1024, 1e-2, state_indicator=True) for n in (4096, 16384)], 46),
    ([D("nlse", "f64", 1, 4096, 256, 1e-2, state_indicator=True)], 47),
    ([D("ch", "f32", 1, 4096, 1024, 1e-2, state_indicator=True)], 48),
]


@pytest.mark.parametrize("variant", [1, 0, 3, 4], ids=["strip_walk", "block_list", "wave_walk", "run_walk"])
@pytest.mark.parametrize("descs,seed", STATE_CASES, ids=[f"case{c[1]}" for c in STATE_CASES])
def test_apply_state_indicator_bit_exact(descs, seed, variant):
    print(f"state-indicator apply case {seed} variant {variant}", flush=True)
    run_case(descs, seed, update_variant=variant)


FULL = _full_cases()


@pytest.mark.parametrize("name,make,seed", FULL, ids=[f[0] for f in FULL])
def test_apply_bit_exact_full_size(name, make, seed):
    descs = make()
    print(f"full-size apply parity {name}: {len(descs)} instances, "
          f"{sum(d.n_modes for d in descs)} modes", flush=True)
    run_case(descs, seed)


def test_full_size_512_state_measure_in_the_timed_launch_configuration():
    """The 512^3 workload as the bench times it: the state measure, the launch
    shapes of the tuned cache (the wave walk), and two updates in a row, the
    second on the measure the first one kept; everything bit-exact against
    the oracle."""
    import torch

    from paper_2609_03922_amd import autotune
    from paper_2609_03922_amd import configs as C

    d = S.desc_from_config(C.CH3D_512_F32_PROPOSER, state_indicator=True)
    plan = S.Plan([d])
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    entry = autotune.apply_cached(plan, arch)
    print(f"512^3 state measure, cached launch {entry and entry['choice']}", flush=True)
    q, r, k0, rk0 = draw_apply_inputs(d, 36, 0)
    plan.set_spectrum(0, torch.from_numpy(q), k0=k0)
    for step in range(2):
        _, r, _, rk0 = draw_apply_inputs(d, 37 + step, 0)
        plan.apply(torch.from_numpy(r), rk0)
        ref = oracle_apply(d, q, r, k0, rk0)
        tag = f"512^3 update {step}"
        ab, G = plan.indicator(0)
        assert_bits_equal(plan.active_mask(0), ref["mask"], tag + " mask")
        assert_bits_equal(ab, ref["a_b"], tag + " a_b")
        assert G == ref["G"], tag
        hat, k0g = plan.get_spectrum(0)
        assert_bits_equal(hat.cpu().numpy(), ref["q"], tag + " coefficients")
        assert_bits_equal(k0g, ref["k0"], tag + " k0")
        assert 0 < ref["count"] < d.n_blocks, ref["count"]
        q, k0 = ref["q"].astype(q.dtype), ref["k0"]
    plan.destroy()
