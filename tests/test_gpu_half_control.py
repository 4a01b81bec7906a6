"""Consistency control on the half-spectrum layout (Supplementary S1.1 with
the conjugate neighbour remap of S1.2) on the GPU against the oracle.

The stored half keeps the columns 0 .. nx/2; a neighbour that lies in the
omitted half is replaced by its conjugate counterpart (the blocks of the
same end column at the mirrored rows), so blocks at kx = 0 and next to
nx/2 take transition states from blocks they touch only through q(-k) =
q*(k).  Kernel level (spdba_apply): states 0/1/2, the ordered non-frozen
list, a_b, G, the weighted transition update and the FP64 k = 0 path agree
bit for bit; step level (FP64): per-step states and the controller's
threshold trace agree with the oracle's trajectory; graph replay equals
eager steps.
"""
import numpy as np
import pytest

import oracle as O
from _parity import assert_bits_equal, draw_apply_inputs, k0path, oracle_apply, oracle_inst
from paper_2609_03922_amd import inputs
from paper_2609_03922_amd import spdba as S

pytestmark = pytest.mark.gpu

PARAMS = {"ch": (1.0, 1.0), "gs": (0.16, 0.08, 0.035, 0.060)}


def D(op, dtype, ndim, n, block, tau, **kw):
    dt = {"ch": 0.01, "gs": 1.0}[op]
    return S.Desc(op=op, dtype=dtype, ndim=ndim, n=n, block=block, tau=tau, dx=1.0, dt=dt,
                  params=PARAMS[op], half=True, transition=True, **kw)


def half_block_of_modes(d):
    """Stored block of every stored mode: the columns below nx/2 in C order
    over (z, y, x) blocks, then one block per (z, y) block row for nx/2."""
    nz, ny, nx = d.dims3
    bz, by, bx = d.block3
    nbxm, nbm = nx // (2 * bx), (nz // bz) * (ny // by) * (nx // (2 * bx))
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx // 2 + 1), indexing="ij")
    row = (iz // bz) * (ny // by) + iy // by
    return np.where(ix == nx // 2, nbm + row, row * nbxm + ix // bx).ravel()


def patterned(d, seed, keep, damp=1e-5):
    """Flat random spectra, damped in the blocks where keep is False."""
    q, r, k0, rk0 = draw_apply_inputs(d, seed, 0, width_frac=1e9, floor=0.0)
    sc = np.tile(np.where(keep[half_block_of_modes(d)], 1.0, damp), d.nspec)
    q = (q * sc).astype(q.dtype)
    r = (r * sc).astype(r.dtype)
    if not keep[0]:
        k0 = k0 * (damp / d.n_modes)
        rk0 = rk0 * (damp / d.n_modes)
    return q, r, k0, rk0


def check_apply(d, ins, want_states=True):
    import torch

    q, r, k0, rk0 = ins
    plan = S.Plan([d])
    plan.set_spectrum(0, torch.from_numpy(q), k0=k0 if k0path(d) else None)
    plan.apply(torch.from_numpy(r), rk0 if k0path(d) else None)
    ref = oracle_apply(d, q, r, k0, rk0)
    tag = f"half {d.op}/{d.dtype} n={d.n} b={d.block}"
    mask = plan.active_mask(0)
    assert_bits_equal(mask, ref["mask"], tag + " states")
    assert_bits_equal(plan.worklist(0), ref["worklist"], tag + " non-frozen list")
    ab, G = plan.indicator(0)
    assert_bits_equal(ab, ref["a_b"], tag + " a_b")
    assert G == ref["G"], (tag, G, ref["G"])
    hat, k0g = plan.get_spectrum(0)
    assert_bits_equal(hat.cpu().numpy(), ref["q"], tag + " coefficients")
    if k0path(d):
        assert_bits_equal(k0g, ref["k0"], tag + " k0")
    st = plan.stats(0)
    assert st["transition_blocks"] == int((ref["mask"] == 2).sum())
    plan.destroy()
    if want_states:
        assert {0, 1, 2} <= set(np.unique(mask).tolist()), np.unique(mask)
    return ref


CASES = [
    # (desc, p_active, seed)
    (D("ch", "f64", 2, 64, 8, 1e-3), 0.25, 1),
    (D("ch", "f32", 3, 32, 4, 1e-3), 0.2, 2),
    (D("ch", "f32", 2, 64, 8, 1e-3, pin_k0=False), 0.3, 3),
    (D("gs", "f32", 2, 64, 8, 1e-3), 0.2, 4),
    (D("gs", "f64", 2, 32, 4, 1e-3), 0.3, 5),
    (D("ch", "f32", 3, 32, 8, 1e-3, state_indicator=True), 0.02, 6),
    (D("ch", "f64", 2, 64, 2, 1e-3), 0.2, 7),   # blocks of two columns: X_0 is columns 0 and 1
    # the largest grids the half layout takes (2^18 points)
    (D("ch", "f32", 2, 512, 16, 1e-3), 0.08, 8),
    (D("gs", "f32", 3, 64, 8, 1e-3), 0.05, 9),
    (D("ch", "f64", 3, 64, 4, 1e-3, state_indicator=True), 0.01, 10),
]


@pytest.mark.parametrize("d,p,seed", CASES, ids=[f"case{c[2]}" for c in CASES])
def test_half_transition_apply_bit_exact(d, p, seed):
    print(f"half transition apply case {seed}: {d.op}/{d.dtype} {d.ndim}-D n={d.n} b={d.block}", flush=True)
    keep = inputs.rng_for(seed, 7).random(d.n_blocks) < p
    keep[1] = True
    check_apply(d, patterned(d, seed, keep))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_half_conjugate_neighbours_on_the_gpu(dtype):
    """One active block at kx = 0 and one in the column nx/2: the transition
    blocks include their conjugate counterparts at the mirrored rows, as the
    oracle derives them."""
    d = D("ch", dtype, 2, 64, 8, 1e-3, pin_k0=False)
    nby, nbxm = 64 // 8, 32 // 8
    keep = np.zeros(d.n_blocks, bool)
    keep[2 * nbxm + 0] = True          # (by 2, X_0)
    keep[nby * nbxm + 5] = True        # (by 5, X_N)
    ref = check_apply(d, patterned(d, 70 + (dtype == "f32"), keep), want_states=False)
    mirror = {(6 * nbxm + 0), (5 * nbxm + 0)}     # rows of block 2 mirror into blocks 6 and 5
    beyond = {(3 * nbxm + nbxm - 1), (2 * nbxm + nbxm - 1)}  # rows of block 5 mirror into 3 and 2, in X_{nbxm-1}
    for b in mirror | beyond:
        assert ref["mask"][b] == 2, b


def test_half_state_measure_sequence_with_transitions():
    """The kept state measure with transition blocks on the half layout: each
    update's states, a_b, G and coefficients against the oracle fed the GPU's
    state."""
    import torch

    d = D("ch", "f32", 3, 32, 4, 1e-2, state_indicator=True)
    q, r, k0, rk0 = draw_apply_inputs(d, 71, 0, floor=1e-3)
    plan = S.Plan([d])
    plan.set_spectrum(0, torch.from_numpy(q), k0=k0)
    seen = set()
    for step in range(4):
        _, r, _, rk0 = draw_apply_inputs(d, 72 + step, 0, floor=1e-3)
        plan.apply(torch.from_numpy(r), rk0)
        ref = oracle_apply(d, q, r, k0, rk0)
        tag = f"update {step}"
        assert_bits_equal(plan.active_mask(0), ref["mask"], tag + " states")
        ab, G = plan.indicator(0)
        assert_bits_equal(ab, ref["a_b"], tag + " a_b")
        assert G == ref["G"], tag
        hat, k0g = plan.get_spectrum(0)
        assert_bits_equal(hat.cpu().numpy(), ref["q"], tag + " coefficients")
        assert_bits_equal(k0g, ref["k0"], tag + " k0")
        seen |= set(np.unique(ref["mask"]).tolist())
        q, k0 = ref["q"].astype(q.dtype), ref["k0"]
    assert 2 in seen
    plan.destroy()


@pytest.mark.parametrize("ndim,steps", [(2, 48), (3, 30)])
def test_half_f64_control_trajectory(ndim, steps):
    """FP64 steps with transitions, refresh, an initial full window and the
    threshold controller: every step's states and the threshold trace equal
    the oracle's, the field within 1e-10 (64^2, and 64^3 at the layout's
    largest size)."""
    import torch

    n = 64
    d = D("ch", "f64", ndim, n, 8, 1e-4, refresh=7, full_steps=2, target_ratio=0.35, control_interval=3,
          deadband=0.1)
    shape = (n,) * ndim
    c0 = inputs.uniform_field(1111, 0, shape, 0.0, 0.05)
    ref = O.step(oracle_inst(d), O.rfft(c0), steps, masks=True, ab=True)
    plan = S.Plan([d])
    plan.set_field(0, torch.from_numpy(c0.ravel()))
    seen = set()
    for st in range(steps):
        plan.step(1)
        m = plan.active_mask(0)
        assert_bits_equal(m, ref["masks"][st, 0], f"step {st} states")
        seen |= set(np.unique(m).tolist())
        s = plan.stats(0)
        if st + 1 < steps:
            assert s["tau"] == ref["tau"][st + 1], (st, s["tau"], ref["tau"][st + 1])
    got = plan.get_field(0).cpu().numpy()
    want = O.irfft(ref["state"].reshape(*shape[:-1], n // 2 + 1), shape).ravel()
    err = np.linalg.norm(got - want) / np.linalg.norm(want - want.mean())
    print(f"half control trajectory {ndim}-D: states {sorted(seen)}, tau {ref['tau'][0]:.3g} -> {ref['tau'][-1]:.3g}, "
          f"rel-L2 {err:.3e}", flush=True)
    assert seen == {0, 1, 2}
    assert len(np.unique(ref["tau"])) >= 3
    assert err <= 1e-10
    plan.destroy()


def test_half_control_graph_replay_matches_eager():
    import torch

    kw = dict(refresh=4, full_steps=1, target_ratio=0.3, control_interval=2, deadband=0.1)
    c0 = inputs.uniform_field(1112, 0, (32, 32, 32), 0.1, 0.02).astype(np.float32)
    out = []
    for graph in (False, True):
        d = D("ch", "f32", 3, 32, 4, 1e-4, graph=graph, **kw)
        plan = S.Plan([d])
        plan.set_field(0, torch.from_numpy(c0.ravel()))
        plan.step(15)
        plan.synchronize()
        hat, k0 = plan.get_spectrum(0)
        s = plan.stats(0)
        out.append((hat.cpu().numpy(), k0, plan.active_mask(0), np.array([s["tau"]]), np.array([s["control_step"]])))
        plan.destroy()
    for a, b in zip(*out):
        assert_bits_equal(a, b, "graph replay vs eager")
