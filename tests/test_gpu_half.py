"""Half-spectrum layout (Supplementary S1.2) on the GPU against the oracle.

Kernel level, through spdba_apply: a_b, G, mask, ordered list, coefficients
and FP64 k = 0 bit for bit, for CH and GS in both precisions, grids whose
stored rows are narrower than, equal to and wider than one wave row, blocks
wider than a wave row, a skip set, the state measure (kept by the update
kernel over sequences of updates) and Regular mode.  Step level: FP64
trajectories (masks per step bit-exact, field within 1e-10) through rocFFT's
real transforms, the FP32 error against the FP64 oracle, the field round trip,
graph replay, and the equality of the half and full layouts' dense runs.
"""
import numpy as np
import pytest

import oracle as O
from _parity import assert_bits_equal, draw_apply_inputs, k0path, oracle_apply, oracle_inst, rel_l2
from paper_2609_03922_amd import inputs
from paper_2609_03922_amd import spdba as S

pytestmark = pytest.mark.gpu

PAR = {"ch": (1.0, 1.0), "gs": (0.16, 0.08, 0.035, 0.060)}


def D(op, dtype, ndim, n, block, tau, **kw):
    dt = 0.01 if op == "ch" else 1.0
    kw.setdefault("half", True)
    return S.Desc(op=op, dtype=dtype, ndim=ndim, n=n, block=block, tau=tau, dx=1.0, dt=dt,
                  params=PAR[op], **kw)


def _load(plan, descs, ins):
    import torch

    for i, (d, (q, r, k0, rk0)) in enumerate(zip(descs, ins)):
        plan.set_spectrum(i, torch.from_numpy(q), k0=k0 if k0path(d) else None)


def _rhs(descs, ins):
    import torch

    rhs = torch.from_numpy(np.concatenate([x[1] for x in ins]))
    rk = np.concatenate([x[3] for x in ins]) if k0path(descs[0]) else None
    return rhs, rk


def _check(plan, i, d, ref, tag):
    assert_bits_equal(plan.active_mask(i), ref["mask"], tag + " mask")
    assert_bits_equal(plan.worklist(i), ref["worklist"], tag + " list")
    if not d.dense:
        ab, G = plan.indicator(i)
        assert_bits_equal(ab, ref["a_b"], tag + " a_b")
        assert G == ref["G"], (tag, G, ref["G"])
    hat, k0g = plan.get_spectrum(i)
    assert_bits_equal(hat.cpu().numpy(), ref["q"], tag + " coefficients")
    if k0path(d):
        assert_bits_equal(k0g, ref["k0"], tag + " k0")


APPLY = [
    ([D("ch", "f32", 3, 32, 8, 3e-2)], 101),                      # rows of 17: lanes idle past 16
    ([D("ch", "f32", 3, 64, 4, 3e-2)], 102),
    ([D("ch", "f64", 2, 128, 16, 3e-2)], 103),                    # rows of 65: one full wave row
    ([D("ch", "f32", 2, 256, 16, 3e-2)], 104),                    # two wave rows per stored row
    ([D("ch", "f64", 2, 512, 128, 3e-2)], 105),                   # blocks wider than a wave row
    ([D("ch", "f64", 2, 16, 1, 0.3)], 106),                       # one-column blocks
    ([D("ch", "f32", 3, 32, 8, 3e-2, pin_k0=False)], 107),
    ([D("gs", "f32", 2, n, 16, 1e-2) for n in (64, 32, 128)], 108),  # batch of unequal sizes
    ([D("gs", "f64", 2, 64, 8, 1e-2)], 109),
    ([D("ch", "f32", 3, 32, 8, 1e-2, state_indicator=True)], 110),
    ([D("gs", "f32", 2, n, 32, 1e-2, state_indicator=True) for n in (128, 64)], 111),
    ([D("ch", "f64", 2, 64, 16, 0.0, dense=True)], 112),
    ([D("gs", "f32", 2, n, 16, 0.0, dense=True) for n in (64, 128)], 113),
    ([D("ch", "f32", 3, 64, 8, 0.0, dense=True)], 114),
    ([D("ch", "f32", 2, 8, 2, 0.0, dense=True)], 119),             # row pitch beyond the grid
    ([D("gs", "f32", 3, 8, 2, 0.1)], 120),
]


@pytest.mark.parametrize("descs,seed", APPLY, ids=[f"case{c[1]}" for c in APPLY])
def test_half_apply_bit_exact(descs, seed):
    print(f"half-layout apply case {seed}: {[(d.op, d.dtype, d.n, d.block, d.dense) for d in descs]}",
          flush=True)
    plan = S.Plan(descs)
    ins = [draw_apply_inputs(d, seed, i, floor=1e-4) for i, d in enumerate(descs)]
    _load(plan, descs, ins)
    plan.apply(*_rhs(descs, ins))
    counts = []
    for i, (d, (q, r, k0, rk0)) in enumerate(zip(descs, ins)):
        ref = oracle_apply(d, q, r, k0, rk0)
        _check(plan, i, d, ref, f"case {seed} inst {i}")
        counts.append(ref["count"])
    if not descs[0].dense:
        assert any(0 < c < d.n_blocks for c, d in zip(counts, descs)), counts
    plan.destroy()


def test_half_apply_with_skip_set():
    import torch

    descs = [D("ch", "f32", 3, 32, 8, 1e-3), D("ch", "f32", 3, 32, 8, 1e-3)]
    ins = [draw_apply_inputs(d, 115, i, floor=1e-4) for i, d in enumerate(descs)]
    skip = [(inputs.rng_for(115, 7, i).random(d.n_blocks) < 0.3).astype(np.uint8) for i, d in enumerate(descs)]
    plan = S.Plan(descs)
    _load(plan, descs, ins)
    plan.set_skip(torch.from_numpy(np.concatenate(skip)))
    plan.apply(*_rhs(descs, ins))
    for i, (d, (q, r, k0, rk0)) in enumerate(zip(descs, ins)):
        _check(plan, i, d, oracle_apply(d, q, r, k0, rk0, skip=skip[i]), f"skip inst {i}")
    plan.destroy()


@pytest.mark.parametrize("descs,seed", [
    ([D("ch", "f32", 3, 32, 8, 1e-2, state_indicator=True)], 116),
    ([D("gs", "f32", 2, n, 16, 1e-2, state_indicator=True) for n in (64, 32)], 117),
    ([D("ch", "f64", 2, 64, 16, 3e-3, state_indicator=True)], 118),
], ids=["ch3d_f32", "gs2d_f32", "ch2d_f64"])
def test_half_state_measure_update_sequence(descs, seed):
    """The update kernel keeps the measure of what it stores: from the second
    update on no indicator pass runs; every update must still equal the
    oracle's, including after a reload that forces a full evaluation."""
    import torch

    plan = S.Plan(descs)
    ins = [draw_apply_inputs(d, seed, i, floor=1e-3) for i, d in enumerate(descs)]
    _load(plan, descs, ins)
    states = [[q, k0] for (q, r, k0, rk0) in ins]
    for step in range(5):
        if step == 3:
            for i, d in enumerate(descs):
                plan.set_spectrum(i, torch.from_numpy(states[i][0]), k0=states[i][1] if k0path(d) else None)
        rs = [draw_apply_inputs(d, seed + 100 + step, i, floor=1e-3) for i, d in enumerate(descs)]
        plan.apply(*_rhs(descs, rs))
        for i, d in enumerate(descs):
            q, k0 = states[i]
            ref = oracle_apply(d, q, rs[i][1], k0, rs[i][3])
            _check(plan, i, d, ref, f"update {step} inst {i}")
            states[i] = [ref["q"].astype(q.dtype), ref["k0"] if k0path(d) else k0]
    plan.destroy()


def _real_field(op, seed, n, ndim):
    shape = (n,) * ndim
    if op == "ch":
        return [inputs.uniform_field(seed, 0, shape, 0.0, 0.05)]
    u = np.ones(shape)
    v = np.zeros(shape)
    sl = tuple(slice(n // 4, n // 4 + n // 8) for _ in range(ndim))
    u[sl], v[sl] = 0.5, 0.25
    return [u, v + 0.01 * inputs.uniform_field(seed, 1, shape, 0.0, 1.0)]


@pytest.mark.parametrize("op,tau,steps", [("ch", 1e-3, 40), ("gs", 1e-3, 40), ("ch", 1e-6, 40)])
def test_half_f64_trajectory_masks_bit_exact(op, tau, steps):
    import torch

    n = 64
    d = D(op, "f64", 2, n, 8, tau)
    fields = _real_field(op, 1301, n, 2)
    ref = O.step(oracle_inst(d), np.concatenate([O.rfft(f).ravel() for f in fields]), steps, masks=True,
                 ab=True)
    plan = S.Plan([d])
    plan.set_field(0, torch.from_numpy(np.concatenate([f.ravel() for f in fields])))
    ties, seen = 0, set()
    for st in range(steps):
        plan.step(1)
        m = plan.active_mask(0)
        r = ref["masks"][st, 0]
        seen.add(int(m.sum()))
        if not np.array_equal(m, r):
            ab = ref["ab"][st, 0]
            thr = tau * tau * ab.max()
            bad = np.flatnonzero(m != r)
            near = np.abs(ab[bad] - thr) <= 1e-12 * thr
            assert near.all(), f"step {st}: mask mismatch at blocks {bad[~near][:8]}"
            ties += bad.size
    assert ties <= 2, ties
    got = plan.get_field(0).cpu().numpy()
    ns = d.nspec
    want = np.concatenate([O.irfft(ref["state"].reshape(ns, -1)[s], (n, n)).ravel() for s in range(ns)])
    err = rel_l2(got, want)
    print(f"half {op} f64 tau={tau}: rel-L2 {err:.3e}, ties {ties}, active counts {sorted(seen)[:6]}",
          flush=True)
    assert err <= 1e-10
    if op == "ch":
        assert min(seen) < d.n_blocks
    plan.destroy()


def test_half_ch3d_f32_error_and_mass():
    import torch

    n, steps = 64, 60
    d = D("ch", "f32", 3, n, 8, 1e-6, state_indicator=True)
    d64 = D("ch", "f64", 3, n, 8, 0.0, dense=True)
    c0 = inputs.uniform_field(1002, 1, (n, n, n), 0.1, 0.02)
    ref = O.step(oracle_inst(d64), O.rfft(c0).ravel(), steps)
    plan = S.Plan([d])
    plan.set_field(0, torch.from_numpy(c0.ravel().astype(np.float32)))
    mean0 = plan.stats(0)["mean"][0]
    plan.step(steps)
    s = plan.stats(0)
    assert s["mean"][0] == mean0
    got = plan.get_field(0).cpu().numpy().astype(np.float64)
    want = O.irfft(ref["state"], (n, n, n)).ravel()
    err = rel_l2(got - want.mean(), want - want.mean())
    print(f"half ch3d_64_f32 state measure: fluctuation rel-L2 vs FP64 dense {err:.3e}, "
          f"active {s['active_blocks']}/{d.n_blocks}", flush=True)
    assert err < 1e-4
    plan.destroy()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_half_field_round_trip_and_spectrum(dtype):
    import torch

    n = 32
    descs = [D("gs", dtype, 3, n, 8, 1e-3), D("gs", dtype, 3, n, 8, 1e-3)]
    fields = [np.concatenate([f.ravel() for f in _real_field("gs", 1400 + i, n, 3)]) for i in range(2)]
    rt = np.float64 if dtype == "f64" else np.float32
    plan = S.Plan(descs)
    for i in range(2):
        plan.set_field(i, torch.from_numpy(fields[i].astype(rt)))
    for i in range(2):
        got = plan.get_field(i).cpu().numpy().astype(np.float64)
        assert rel_l2(got, fields[i]) <= (1e-13 if dtype == "f64" else 2e-7)
        hat, k0 = plan.get_spectrum(i)
        hat = hat.cpu().numpy().reshape(2, -1).astype(np.complex128)
        for s in range(2):
            want = O.rfft(fields[i].astype(rt).astype(np.float64).reshape(2, n, n, n)[s]).ravel()
            if dtype == "f32":  # the k = 0 coefficient is held in FP64
                assert abs(k0[s] - want[0].real) <= 1e-12 * abs(want[0].real)
                want[0] = 0.0
            assert rel_l2(hat[s], want) <= (1e-13 if dtype == "f64" else 1e-6)
    plan.destroy()


def test_half_graph_replay_equals_eager():
    import torch

    c0 = inputs.uniform_field(1202, 0, (32, 32, 32), 0.1, 0.02).astype(np.float32)
    out = []
    for graph in (False, True):
        d = D("ch", "f32", 3, 32, 4, 1e-3, graph=graph, state_indicator=True)
        plan = S.Plan([d])
        runs = []
        for rep in range(2):
            plan.set_field(0, torch.from_numpy(c0.ravel()))
            plan.step(12)
            plan.synchronize()
            hat, k0 = plan.get_spectrum(0)
            ab, G = plan.indicator(0)
            runs.append((hat.cpu().numpy(), k0, plan.active_mask(0), ab, np.array([G])))
        for a, b in zip(*runs):
            assert_bits_equal(a, b, f"graph={graph}: run after reload")
        out.append(runs[0])
        plan.destroy()
    for a, b in zip(*out):
        assert_bits_equal(a, b, "graph replay vs eager")


@pytest.mark.parametrize("op", ["ch", "gs"])
def test_half_dense_matches_full_layout_dense(op):
    """Same physics: the dense half-layout run (r2c / c2r) and the dense
    full-layout run (c2c) give the same real field."""
    import torch

    n, steps = 64, 30
    fields = np.concatenate([f.ravel() for f in _real_field(op, 1500, n, 2)])
    got = []
    for half in (True, False):
        p = S.Plan([D(op, "f64", 2, n, 16, 0.0, dense=True, half=half)])
        p.set_field(0, torch.from_numpy(fields))
        p.step(steps)
        got.append(p.get_field(0).cpu().numpy())
        p.destroy()
    assert rel_l2(got[0], got[1]) <= 1e-12
