"""State-amplitude activity measure on the GPU against the oracle.

For CH and GS the update kernel keeps the measure of the blocks it stores, so
from the second update on the library evaluates no indicator pass; these
tests run sequences of updates and steps and require every update's a_b, G,
mask, list and coefficients to equal the oracle's bit for bit, also across
field loads (which force a full evaluation), graph replay, skip sets and
consistency control.
"""
import numpy as np
import pytest

import oracle as O
from _parity import assert_bits_equal, draw_apply_inputs, k0path, oracle_apply, oracle_inst
from paper_2609_03922_amd import inputs
from paper_2609_03922_amd import spdba as S

pytestmark = pytest.mark.gpu

PARAMS = {"ch": (1.0, 1.0), "gs": (0.16, 0.08, 0.035, 0.060), "nlse": (-21.7, 1.3, 0.0)}


def D(op, dtype, ndim, n, block, tau, **kw):
    dx, dt = {"ch": (1.0, 0.01), "gs": (1.0, 1.0), "nlse": (15.625, 0.8)}[op]
    return S.Desc(op=op, dtype=dtype, ndim=ndim, n=n, block=block, tau=tau, dx=dx, dt=dt,
                  params=PARAMS[op], state_indicator=True, **kw)


def check(plan, i, d, ref, tag):
    assert_bits_equal(plan.active_mask(i), ref["mask"], tag + " mask")
    assert_bits_equal(plan.worklist(i), ref["worklist"], tag + " list")
    ab, G = plan.indicator(i)
    assert_bits_equal(ab, ref["a_b"], tag + " a_b")
    assert G == ref["G"], (tag, G, ref["G"])
    hat, k0g = plan.get_spectrum(i)
    assert_bits_equal(hat.cpu().numpy(), ref["q"], tag + " coefficients")
    if k0path(d):
        assert_bits_equal(k0g, ref["k0"], tag + " k0")


def run_sequence(descs, seed, n_apply=4, variant=None, reload_at=None):
    """n_apply updates with fresh right-hand sides on the evolving state; the
    oracle follows the same sequence on its own state."""
    import torch

    plan = S.Plan(descs)
    if variant is not None:
        plan.set_launch(3, variant)
    ins = [draw_apply_inputs(d, seed, i, floor=1e-3) for i, d in enumerate(descs)]
    states = []
    for i, (d, (q, r, k0, rk0)) in enumerate(zip(descs, ins)):
        plan.set_spectrum(i, torch.from_numpy(q), k0=k0 if k0path(d) else None)
        states.append([q, k0])
    counts = []
    for step in range(n_apply):
        if reload_at is not None and step == reload_at:  # a load forces a full evaluation
            for i, d in enumerate(descs):
                plan.set_spectrum(i, torch.from_numpy(states[i][0]), k0=states[i][1] if k0path(d) else None)
        rs = [draw_apply_inputs(d, seed + 100 + step, i, floor=1e-3) for i, d in enumerate(descs)]
        rhs = rk = None
        if descs[0].op != "nlse":
            rhs = torch.from_numpy(np.concatenate([x[1] for x in rs]))
            if k0path(descs[0]):
                rk = np.concatenate([x[3] for x in rs])
        plan.apply(rhs, rk)
        for i, d in enumerate(descs):
            q, k0 = states[i]
            ref = oracle_apply(d, q, rs[i][1], k0, rs[i][3])
            check(plan, i, d, ref, f"update {step} inst {i} {d.op}/{d.dtype}")
            states[i] = [ref["q"].astype(q.dtype), ref["k0"] if k0path(d) else k0]
            counts.append(ref["count"])
    plan.destroy()
    return counts


SEQ = [
    ([D("ch", "f32", 3, 32, 8, 1e-2)], 61),
    ([D("ch", "f64", 2, 64, 16, 3e-3)], 62),
    ([D("ch", "f32", 3, 32, 4, 1e-2, pin_k0=False)], 63),
    ([D("gs", "f32", 2, n, 16, 1e-2) for n in (64, 32, 128)], 64),
    ([D("gs", "f64", 2, 64, 16, 1e-2)], 65),
    ([D("nlse", "f32", 1, 4096, 256, 1e-2)], 66),  # NLSE: a full pass every update
    ([D("ch", "f32", 3, 32, 4, 1e-2, transition=True)], 67),
]


@pytest.mark.parametrize("descs,seed", SEQ[:6], ids=[f"seq{c[1]}" for c in SEQ[:6]])
def test_state_measure_update_sequence_wave_walk(descs, seed):
    # one wave per list entry: the kept measure is a wave reduction
    print(f"state-measure sequence {seed}, wave walk", flush=True)
    run_sequence(descs, seed, variant=3)


@pytest.mark.parametrize("descs,seed", SEQ[:6], ids=[f"seq{c[1]}" for c in SEQ[:6]])
def test_state_measure_update_sequence_run_walk(descs, seed):
    # aligned runs of x-adjacent active blocks in bands of rows: the kept
    # measure is an atomic maximum over the bands of each block
    print(f"state-measure sequence {seed}, run walk", flush=True)
    run_sequence(descs, seed, variant=4)


@pytest.mark.parametrize("descs,seed", SEQ, ids=[f"seq{c[1]}" for c in SEQ])
def test_state_measure_update_sequence_bit_exact(descs, seed):
    print(f"state-measure sequence {seed}: {[(d.op, d.dtype, d.n, d.block) for d in descs]}", flush=True)
    counts = run_sequence(descs, seed)
    nb = sum(d.n_blocks for d in descs)
    assert any(0 < c < d.n_blocks for c, d in zip(counts, descs * len(counts)))


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_state_measure_sequence_other_variants_and_reload(variant):
    # the strip walk and the four-in-flight walk requested: the plan keeps the
    # measure through the block-list walk; the wave walk keeps it itself; a
    # reload in the middle forces a full evaluation
    run_sequence([D("ch", "f32", 3, 32, 8, 1e-2)], 68, n_apply=5, variant=variant, reload_at=3)


def test_state_measure_with_skip_set_falls_back_to_full_pass():
    import torch

    d = D("ch", "f32", 3, 32, 8, 1e-2)
    plan = S.Plan([d])
    q, r, k0, rk0 = draw_apply_inputs(d, 69, 0, floor=1e-3)
    plan.set_spectrum(0, torch.from_numpy(q), k0=k0)
    plan.apply(torch.from_numpy(r), rk0)
    ref = oracle_apply(d, q, r, k0, rk0)
    check(plan, 0, d, ref, "first")
    skip = (inputs.rng_for(69, 5).random(d.n_blocks) < 0.3).astype(np.uint8)
    plan.set_skip(torch.from_numpy(skip))
    q1, kk = ref["q"].astype(q.dtype), ref["k0"]
    plan.apply(torch.from_numpy(r), rk0)
    ref2 = oracle_apply(d, q1, r, kk, rk0, skip=skip)
    check(plan, 0, d, ref2, "with skip set")
    plan.set_skip(None)
    q2, kk2 = ref2["q"].astype(q.dtype), ref2["k0"]
    plan.apply(torch.from_numpy(r), rk0)
    ref3 = oracle_apply(d, q2, r, kk2, rk0)
    check(plan, 0, d, ref3, "after the skip set")
    plan.destroy()


def test_state_measure_fp64_trajectory_masks_bit_exact():
    import torch

    n, steps = 64, 40
    d = D("ch", "f64", 2, n, 8, 1e-3)
    c0 = inputs.uniform_field(1201, 0, (n, n), 0.0, 0.05)
    ref = O.step(oracle_inst(d), O.fft(c0, -1), steps, masks=True, ab=True)
    plan = S.Plan([d])
    plan.set_field(0, torch.from_numpy(c0.ravel()))
    seen = set()
    for st in range(steps):
        plan.step(1)
        m = plan.active_mask(0)
        assert_bits_equal(m, ref["masks"][st, 0], f"step {st} mask")
        seen.add(int(m.sum()))
    assert len(seen) > 3 and min(seen) < d.n_blocks
    plan.destroy()


def test_state_measure_graph_replay_matches_eager():
    import torch

    c0 = inputs.uniform_field(1202, 0, (32, 32, 32), 0.1, 0.02).astype(np.float32)
    out = []
    for graph in (False, True):
        d = D("ch", "f32", 3, 32, 4, 1e-3, graph=graph)
        plan = S.Plan([d])
        runs = []
        for rep in range(2):  # a field load in between forces one full evaluation
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
