"""Consistency control on the GPU (Supplementary S1.1, S1.3) against the oracle.

Kernel level (spdba_apply): block states 0/1/2, the ordered non-frozen list,
a_b, G, the tapered transition update and the FP64 k = 0 side path agree bit
for bit.  Inputs are damped block by block so that the active set is a chosen
random pattern; the tests check that every state occurs.

Step level (spdba_step, FP64): per-step states and the threshold trace of the
controller agree with the oracle's trajectory; graph replay and eager steps
agree bit for bit; a field load resets the schedule and the threshold.
"""
import numpy as np
import pytest

import oracle as O
from _parity import assert_bits_equal, draw_apply_inputs, k0path, oracle_apply, oracle_inst, rel_l2
from paper_2609_03922_amd import inputs
from paper_2609_03922_amd import spdba as S

pytestmark = pytest.mark.gpu

PARAMS = {"ch": (1.0, 1.0), "gs": (0.16, 0.08, 0.035, 0.060), "nlse": (-21.7, 1.3, 0.0)}


def D(op, dtype, ndim, n, block, tau, **kw):
    dx, dt = {"ch": (1.0, 0.01), "gs": (1.0, 1.0), "nlse": (15.625, 0.8)}[op]
    return S.Desc(op=op, dtype=dtype, ndim=ndim, n=n, block=block, tau=tau, dx=dx, dt=dt,
                  params=PARAMS[op], **kw)


def block_of_modes(d):
    """Block id of every mode (C order over the block grid), flattened."""
    dims, blk = d.dims3, d.block3
    nbk = [a // b for a, b in zip(dims, blk)]
    iz, iy, ix = np.meshgrid(*[np.arange(a) for a in dims], indexing="ij")
    return (((iz // blk[0]) * nbk[1] + iy // blk[1]) * nbk[2] + ix // blk[2]).ravel()


def patterned_inputs(d, seed, idx, keep, damp=1e-5):
    """Flat random spectra whose increments are scaled by `damp` in the blocks
    where keep is False (the increment of every operator is linear in the
    state and right-hand side jointly)."""
    q, r, k0, rk0 = draw_apply_inputs(d, seed, idx, width_frac=1e9, floor=0.0)
    scale = np.where(keep[block_of_modes(d)], 1.0, damp)
    sc = np.tile(scale, d.nspec)
    q = (q * sc).astype(q.dtype)
    r = (r * sc).astype(r.dtype)
    if not keep[0]:  # the FP64 k = 0 values are drawn on the scale of N
        k0 = k0 * (damp / d.n_modes)
        rk0 = rk0 * (damp / d.n_modes)
    return q, r, k0, rk0


def run_apply(descs, ins, full_now=0, applies=1, want_states=True):
    import torch

    plan = S.Plan(descs)
    for i, (d, (q, r, k0, rk0)) in enumerate(zip(descs, ins)):
        plan.set_spectrum(i, torch.from_numpy(q), k0=k0 if k0path(d) else None)
    rhs = rk = None
    if descs[0].op != "nlse":
        rhs = torch.from_numpy(np.concatenate([x[1] for x in ins]))
        if k0path(descs[0]):
            rk = np.concatenate([x[3] for x in ins])
    for _ in range(applies):
        plan.apply(rhs, rk)
    masks = []
    for i, (d, (q, r, k0, rk0)) in enumerate(zip(descs, ins)):
        ref = oracle_apply(d, q, r, k0, rk0, full_now=full_now)
        tag = f"inst {i} {d.op}/{d.dtype} n={d.n} b={d.block} tau={d.tau}"
        mask = plan.active_mask(i)
        assert_bits_equal(mask, ref["mask"], tag + " states")
        assert_bits_equal(plan.worklist(i), ref["worklist"], tag + " non-frozen list")
        ab, G = plan.indicator(i)
        assert_bits_equal(ab, ref["a_b"], tag + " a_b")
        assert G == ref["G"], (tag, G, ref["G"])
        hat, k0g = plan.get_spectrum(i)
        assert_bits_equal(hat.cpu().numpy(), ref["q"], tag + " coefficients")
        if k0path(d):
            assert_bits_equal(k0g, ref["k0"], tag + " k0")
        st = plan.stats(i)
        assert st["active_blocks"] == int((ref["mask"] == 1).sum())
        assert st["transition_blocks"] == int((ref["mask"] == 2).sum())
        masks.append(mask)
    plan.destroy()
    if want_states:
        allm = np.concatenate(masks)
        assert {0, 1, 2} <= set(np.unique(allm).tolist()), np.unique(allm)
    return masks


CASES = [
    # (desc, p_active, seed)
    (D("ch", "f64", 2, 64, 8, 1e-3, transition=True), 0.3, 1),
    (D("ch", "f32", 3, 32, 4, 1e-3, transition=True), 0.25, 2),
    (D("ch", "f32", 3, 32, 8, 1e-3, transition=True, pin_k0=False), 0.4, 3),
    (D("ch", "f32", 2, 32, 16, 1e-3, transition=True, pin_k0=False), 0.5, 4),   # two blocks per axis
    (D("gs", "f32", 2, 64, 16, 1e-3, transition=True), 0.1, 5),
    (D("gs", "f64", 2, 64, 8, 1e-3, transition=True), 0.3, 6),
    (D("nlse", "f32", 1, 4096, 256, 1e-3, transition=True), 0.3, 7),
    (D("nlse", "f64", 1, 4096, 64, 1e-3, transition=True), 0.3, 8),
    (D("nlse", "f32", 1, 16384, 1024, 1e-3, transition=True), 0.3, 9),  # block row over several chunks
]


@pytest.mark.parametrize("d,p,seed", CASES, ids=[f"case{c[2]}" for c in CASES])
def test_transition_apply_bit_exact(d, p, seed):
    print(f"transition apply case {seed}: {d.op}/{d.dtype} n={d.n} b={d.block}", flush=True)
    keep = inputs.rng_for(seed, 7).random(d.n_blocks) < p
    keep[1] = True  # at least one active block besides the pinned one
    if d.n_blocks == 4:  # 2 x 2 grid: one active corner, its diagonal frozen
        keep = np.array([False, True, False, False])
    run_apply([d], [patterned_inputs(d, seed, 0, keep)])


def test_transition_apply_batch_bit_exact():
    # instances of several sizes: blocks of different instances share
    # compaction chunks and waves
    descs = [D("gs", "f32", 2, n, 16, 1e-3, transition=True) for n in (64, 32, 128, 32, 16, 64)]
    ins = []
    for i, d in enumerate(descs):
        keep = inputs.rng_for(40 + i, 7).random(d.n_blocks) < 0.4
        ins.append(patterned_inputs(d, 40, i, keep))
    print(f"transition batch: {[d.n for d in descs]}", flush=True)
    run_apply(descs, ins)


@pytest.mark.parametrize("sigma0", [1, 0])
def test_transition_k0_side_path(sigma0):
    # GS FP32, block 0 unpinned and damped: it becomes a transition block and
    # its FP64 k = 0 values take the weighted increment with sigma(0) = 1 (no
    # frozen face) or 0 (a frozen low-x neighbour)
    d = D("gs", "f32", 2, 64, 16, 1e-3, transition=True, pin_k0=False)
    keep = np.ones(d.n_blocks, bool)
    keep[0] = False
    if sigma0 == 0:
        # block (0, 3) frozen: it and its face neighbours other than block 0
        for b in (3, 2, 7, 15):
            keep[b] = False
    masks = run_apply([d], [patterned_inputs(d, 50 + sigma0, 0, keep)], want_states=False)
    assert masks[0][0] == 2
    if sigma0 == 0:
        assert masks[0][3] == 0


def test_full_step_schedule_apply():
    # full_steps = 1: the first update activates every block; refresh 3: the
    # update of step 2 again (steps n with (n + 1) % 3 == 0)
    d = D("ch", "f32", 3, 32, 4, 1e-3, transition=True, full_steps=1, refresh=3)
    keep = inputs.rng_for(60, 7).random(d.n_blocks) < 0.3
    ins = [patterned_inputs(d, 60, 0, keep)]
    m = run_apply([d], ins, full_now=1, applies=1, want_states=False)
    assert (m[0] == 1).all()
    # state after one full update, then steps 1 (normal) and 2 (full)
    import torch

    q, r, k0, rk0 = ins[0]
    ref1 = oracle_apply(d, q, r, k0, rk0, full_now=1)
    ref2 = oracle_apply(d, ref1["q"].astype(q.dtype), r, ref1["k0"], rk0, full_now=0)
    ref3 = oracle_apply(d, ref2["q"].astype(q.dtype), r, ref2["k0"], rk0, full_now=1)
    plan = S.Plan([d])
    plan.set_spectrum(0, torch.from_numpy(q), k0=k0)
    for ref in (ref1, ref2, ref3):
        plan.apply(torch.from_numpy(r), rk0)
        assert_bits_equal(plan.active_mask(0), ref["mask"], "states")
        hat, k0g = plan.get_spectrum(0)
        assert_bits_equal(hat.cpu().numpy(), ref["q"], "coefficients")
        assert_bits_equal(k0g, ref["k0"], "k0")
    assert (ref2["mask"] == 2).any() and (ref3["mask"] == 1).all()
    assert plan.stats(0)["control_step"] == 3
    plan.destroy()


# ---------------------------------------------------------------------------
# step level: schedule and controller over trajectories (FP64)
# ---------------------------------------------------------------------------

def check_trajectory(d, field0, steps, oracle_state0):
    import torch

    per = 2 if d.op == "nlse" else 1
    ref = O.step(oracle_inst(d), oracle_state0, steps, masks=True, ab=True)
    plan = S.Plan([d])
    plan.set_field(0, torch.from_numpy(field0))
    st0 = plan.stats(0)
    assert st0["control_step"] == 0 and st0["tau"] == d.tau
    seen = set()
    for st in range(steps):
        plan.step(1)
        m = plan.active_mask(0)
        r = ref["masks"][st, per - 1]
        assert_bits_equal(m, r, f"step {st} states")
        seen |= set(np.unique(m).tolist())
        s = plan.stats(0)
        assert s["control_step"] == st + 1
        nf = int((ref["masks"][: st + 1] != 0).sum())
        assert s["nonfrozen_ratio_mean"] == nf / (d.n_blocks * per * (st + 1))
        if st + 1 < steps:
            assert s["tau"] == ref["tau"][st + 1], (st, s["tau"], ref["tau"][st + 1])
    taus = ref["tau"]
    print(f"{d.op} control trajectory: states seen {sorted(seen)}, tau {taus[0]:.3g} -> {taus[-1]:.3g}, "
          f"distinct tau {len(np.unique(taus))}", flush=True)
    plan.destroy()
    return ref, seen, taus


def test_ch_f64_control_trajectory():
    n, steps = 64, 48
    d = D("ch", "f64", 2, n, 8, 1e-4, transition=True, refresh=7, full_steps=2, target_ratio=0.35,
          control_interval=3, deadband=0.1)
    c0 = inputs.uniform_field(1101, 0, (n, n), 0.0, 0.05)
    ref, seen, taus = check_trajectory(d, c0.ravel(), steps, O.fft(c0, -1))
    assert seen == {0, 1, 2}
    assert len(np.unique(taus)) >= 3  # the controller moved the threshold


def test_nlse_f64_control_trajectory():
    n, steps = 4096, 24
    d = D("nlse", "f64", 1, n, 64, 1e-3, transition=True, target_ratio=0.5, control_interval=2,
          deadband=0.05, refresh=5)
    e0 = inputs.qam16_rrc_signal(1102, 0, n, dtype=np.complex128)
    ref, seen, taus = check_trajectory(d, e0, steps, e0)
    assert 2 in seen
    assert len(np.unique(taus)) >= 2


def test_control_graph_replay_matches_eager_and_reset():
    import torch

    kw = dict(transition=True, refresh=4, full_steps=1, target_ratio=0.3, control_interval=2,
              deadband=0.1)
    c0 = inputs.uniform_field(1103, 0, (32, 32, 32), 0.1, 0.02).astype(np.float32)
    out = []
    for graph in (False, True):
        d = D("ch", "f32", 3, 32, 4, 1e-4, graph=graph, **kw)
        plan = S.Plan([d])
        runs = []
        for rep in range(2):  # the second run starts after a field load (reset)
            plan.set_field(0, torch.from_numpy(c0.ravel()))
            s = plan.stats(0)
            assert s["control_step"] == 0 and s["tau"] == d.tau
            plan.step(15)
            plan.synchronize()
            hat, k0 = plan.get_spectrum(0)
            s = plan.stats(0)
            runs.append((hat.cpu().numpy(), k0, plan.active_mask(0), s["tau"], s["control_step"]))
        assert runs[0][4] == 15
        for a, b in zip(runs[0], runs[1]):
            assert_bits_equal(np.asarray(a), np.asarray(b), f"graph={graph}: run after reset")
        if graph:
            assert plan.stats(0)["graph_replay"] == 1
        out.append(runs[0])
        plan.destroy()
    for a, b in zip(out[0], out[1]):
        assert_bits_equal(np.asarray(a), np.asarray(b), "graph replay vs eager")


def test_control_off_matches_plain_plan():
    # with every control parameter at rest the control path reproduces the
    # plain threshold rule bit for bit (it walks the block list)
    import torch

    c0 = inputs.uniform_field(1104, 0, (32, 32, 32), 0.1, 0.02).astype(np.float32)
    res = []
    for kw in (dict(), dict(full_steps=0, refresh=1000000, control_interval=0)):
        d = D("ch", "f32", 3, 32, 4, 1e-4, **kw)
        plan = S.Plan([d])
        plan.set_field(0, torch.from_numpy(c0.ravel()))
        plan.step(10)
        hat, k0 = plan.get_spectrum(0)
        res.append((hat.cpu().numpy(), k0, plan.active_mask(0)))
        plan.destroy()
    for a, b in zip(*res):
        assert_bits_equal(a, b, "control path vs plain path")
