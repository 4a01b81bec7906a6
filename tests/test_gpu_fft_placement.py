"""The placement of the step's forward transform (launch knob 5): out of place
into the right-hand-side buffer, or in place in the transform buffer, which
the update then reads.  rocFFT runs different kernels for the two, so the
fields differ at FP32 rounding; everything else is the same path.

Checked on the GPU: FP32 CH (3-D) and GS (2-D, a batch of two grids)
trajectories with the in-place forward against the FP64 oracle within the
FP32 bounds of the other trajectory tests; the update stage (spdba_apply,
which fills the buffer the update reads) bit-exact against the oracle in both
placements; graph replay equal to eager steps in place; switching the
placement between steps; and the refusal where the placement does not apply
(NLSE, XPFC, the half-spectrum layout).
"""
import numpy as np
import pytest

import oracle as O
from _parity import assert_bits_equal, draw_apply_inputs, k0path, oracle_apply, oracle_inst, rel_l2
from paper_2609_03922_amd import configs, inputs
from paper_2609_03922_amd import spdba as S

pytestmark = pytest.mark.gpu


def ch_desc(dtype, ndim, n, block, tau, **kw):
    return S.Desc(op="ch", dtype=dtype, ndim=ndim, n=n, block=block, tau=tau, dx=1.0, dt=0.01,
                  params=(1.0, 1.0), **kw)


def gs_desc(dtype, n, **kw):
    return S.Desc(op="gs", dtype=dtype, ndim=2, n=n, block=16, tau=1e-6, dx=1.0, dt=1.0,
                  params=configs.GS2D_BATCH32_F32["params"], **kw)


def field_of(d, spec):
    shape = d.dims3[3 - d.ndim:]
    return O.fft(np.asarray(spec).reshape(shape), +1).real.ravel()


@pytest.mark.parametrize("measure", ["increment", "state"])
def test_ch3d_f32_in_place_forward_trajectory(measure):
    import torch

    n, steps = 64, 100
    kw = dict(state_indicator=True) if measure == "state" else {}
    d = ch_desc("f32", 3, n, 8, 1e-6, **kw)
    c0 = inputs.uniform_field(1002, 1, (n, n, n), 0.1, 0.02)
    ref = O.step(oracle_inst(ch_desc("f64", 3, n, 8, 1e-6, **kw)), O.fft(c0, -1), steps)["state"]
    plan = S.Plan([d])
    plan.set_launch(5, 1)
    plan.set_field(0, torch.from_numpy(c0.ravel().astype(np.float32)))
    mean0 = plan.stats(0)["mean"][0]
    plan.step(steps)
    assert plan.stats(0)["mean"][0] == mean0
    got = plan.get_field(0).cpu().numpy().astype(np.float64)
    want = field_of(d, ref)
    err = rel_l2(got - want.mean(), want - want.mean())
    print(f"ch3d_64_f32 {measure}, forward in place: fluctuation rel-L2 vs FP64 oracle {err:.3e}", flush=True)
    assert err < 1e-4
    plan.destroy()


def test_gs_f32_batch_in_place_forward_trajectory():
    import torch

    sizes, steps = (64, 128), 200
    plan = S.Plan([gs_desc("f32", n) for n in sizes])
    plan.set_launch(5, 1)
    fields = []
    for i, n in enumerate(sizes):
        u, v = inputs.gs_patch_field(1004, i, n, dtype=np.float64)
        fields.append((u, v))
        plan.set_field(i, torch.from_numpy(np.concatenate([u.ravel(), v.ravel()]).astype(np.float32)))
    plan.step(steps)
    for i, n in enumerate(sizes):
        u, v = fields[i]
        d64 = gs_desc("f64", n)
        st = np.concatenate([O.fft(u, -1).ravel(), O.fft(v, -1).ravel()])
        ref = O.step(oracle_inst(d64), st, steps)["state"]
        N = n * n
        want = np.concatenate([field_of(d64, ref[:N]), field_of(d64, ref[N:])])
        got = plan.get_field(i).cpu().numpy().astype(np.float64)
        err = rel_l2(got, want)
        print(f"gs n={n}, forward in place: rel-L2 vs FP64 oracle after {steps} steps {err:.3e}", flush=True)
        assert err < 1e-3
    plan.destroy()


@pytest.mark.parametrize("placement", [0, 1])
@pytest.mark.parametrize("d", [ch_desc("f32", 3, 32, 8, 1e-3), ch_desc("f64", 2, 64, 16, 1e-3),
                               gs_desc("f32", 64), ch_desc("f32", 3, 32, 8, 1e-2, state_indicator=True)],
                         ids=["ch3d-f32", "ch2d-f64", "gs-f32", "ch3d-f32-state"])
def test_apply_bit_exact_in_both_placements(d, placement):
    """spdba_apply writes the caller's right-hand side where the update reads
    it in either placement."""
    import torch

    q, r, k0, rk0 = draw_apply_inputs(d, 91, 0)
    plan = S.Plan([d])
    plan.set_launch(5, placement)
    plan.set_spectrum(0, torch.from_numpy(q), k0=k0 if k0path(d) else None)
    for step in range(2):
        _, r, _, rk0 = draw_apply_inputs(d, 92 + step, 0)
        plan.apply(torch.from_numpy(r), rk0 if k0path(d) else None)
        ref = oracle_apply(d, q, r, k0, rk0)
        tag = f"{d.op}/{d.dtype} placement {placement} update {step}"
        assert_bits_equal(plan.active_mask(0), ref["mask"], tag + " mask")
        hat, k0g = plan.get_spectrum(0)
        assert_bits_equal(hat.cpu().numpy(), ref["q"], tag + " coefficients")
        if k0path(d):
            assert_bits_equal(k0g, ref["k0"], tag + " k0")
        q, k0 = ref["q"].astype(q.dtype), ref["k0"]
    plan.destroy()


def test_in_place_graph_replay_equals_eager_and_switching():
    import torch

    f = inputs.uniform_field(1002, 7, (32, 32, 32), 0.1, 0.02, dtype=np.float32).ravel()
    eager, graph = S.Plan([ch_desc("f32", 3, 32, 8, 1e-5)]), S.Plan([ch_desc("f32", 3, 32, 8, 1e-5, graph=True)])
    for p in (eager, graph):
        p.set_launch(5, 1)
        p.set_field(0, torch.from_numpy(f))
    for rep in range(4):
        eager.step(3)
        graph.step(3)
        torch.cuda.synchronize()
        a, ka = eager.get_spectrum(0)
        b, kb = graph.get_spectrum(0)
        assert_bits_equal(a.cpu().numpy(), b.cpu().numpy(), f"in-place replay {rep}")
        assert_bits_equal(ka, kb, f"in-place replay {rep} k0")
    # back to out of place mid-run (the captured graph is dropped and recaptured)
    graph.set_launch(5, 0)
    eager.set_launch(5, 0)
    for rep in range(2):
        eager.step(2)
        graph.step(2)
        torch.cuda.synchronize()
        assert_bits_equal(eager.get_spectrum(0)[0].cpu().numpy(), graph.get_spectrum(0)[0].cpu().numpy(),
                          f"switched replay {rep}")
    assert graph.stats(0)["graph_replay"] == 1
    # the placement changes only the transform's rounding
    ref = S.Plan([ch_desc("f32", 3, 32, 8, 1e-5)])
    ref.set_field(0, torch.from_numpy(f))
    ref.step(16)
    x = eager.get_field(0).cpu().numpy().astype(np.float64)
    y = ref.get_field(0).cpu().numpy().astype(np.float64)
    err = rel_l2(x - y.mean(), y - y.mean())
    print(f"in place then out of place vs out of place throughout: {err:.3e}", flush=True)
    assert err < 1e-5
    for p in (eager, graph, ref):
        p.destroy()


def test_placement_refused_where_it_does_not_apply():
    cfg = configs.NLSE1D_BATCH48_F32
    cases = [S.Desc(op="nlse", dtype="f32", ndim=1, n=4096, block=256, tau=1e-6, dx=cfg["dx"], dt=cfg["dt"],
                    params=cfg["params"]),
             ch_desc("f32", 2, 64, 8, 1e-3, half=True),
             S.Desc(op="xpfc", dtype="f32", ndim=2, n=64, block=8, tau=1e-3, dx=0.5, dt=0.5,
                    params=configs.XPFC2D_4096_F32["params"], state_indicator=True)]
    for d in cases:
        plan = S.Plan([d])
        plan.set_launch(5, 0)
        with pytest.raises(S.SpdbaError) as e:
            plan.set_launch(5, 1)
        assert e.value.status == S.SPDBA_EUNSUPPORTED, (d.op, e.value)
        with pytest.raises(S.SpdbaError):
            plan.set_launch(5, 2)
        plan.destroy()
