"""GPU checks of the proposer kernels through the C ABI against the CPU
reference (oracle/mlp.py): bf16 shadow bits, MFMA forward and backward passes,
loss, optimiser, training, block features, labels, skip sets and the miss
counter."""
import numpy as np
import pytest

import oracle as O
from _parity import draw_apply_inputs, k0path, oracle_apply
from oracle import mlp
from paper_2609_03922_amd import spdba as S

pytestmark = pytest.mark.gpu


def T(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=dtype) if dtype is not None else t.cuda()


def _x(seed, n):
    r = np.random.default_rng(seed)
    return r.uniform(-1, 1, (n, 8)).astype(np.float32)


def _shadow(w32):
    import torch

    w = T(w32)
    wb = torch.empty(mlp.NPARAM, dtype=torch.int16, device="cuda")
    S.spdba_mlp_to_bf16(w, wb)
    torch.cuda.synchronize()
    assert np.array_equal(wb.cpu().numpy().view(np.uint16), mlp.bf16_bits(w32))
    return w, wb


def _forward(x32, wb):
    import torch

    n = x32.shape[0]
    x = T(x32)
    prob = torch.empty(n, device="cuda")
    logit = torch.empty(n, device="cuda")
    h1 = torch.empty(n, 64, device="cuda")
    h2 = torch.empty(n, 64, device="cuda")
    S.spdba_mlp_forward(x, wb, prob, logit, h1, h2)
    torch.cuda.synchronize()
    return x, prob, logit, h1, h2


@pytest.mark.parametrize("n", [16, 1037, 20000])
def test_mlp_forward_matches_bf16_reference(n):
    w32 = mlp.init_params(11)
    w32[mlp.OB1:mlp.OW2] = 0.1
    w32[mlp.OB2:mlp.OW3] = -0.05
    w32[mlp.OB3] = 0.2
    _, wb = _shadow(w32)
    x32 = _x(n, n)
    x, prob, logit, h1, h2 = _forward(x32, wb)
    ref = mlp.forward_bf16(x32, w32)
    z = logit.cpu().numpy()
    err = np.abs(z - ref["logit"])
    scale = max(1.0, np.abs(ref["logit"]).max())
    print(f"n={n}: logit error max {err.max():.3e}, 99.9% quantile {np.quantile(err, 0.999):.3e}",
          flush=True)
    # FP32 accumulation order differs from the hardware's, so an activation that
    # sits on a bf16 rounding boundary can round the other way (one bf16 ulp,
    # 2^-8 relative) before the next layer: rare, bounded flips
    assert np.allclose(h1.cpu().numpy(), ref["h1"], rtol=1e-5, atol=1e-5)
    assert np.mean(np.abs(h2.cpu().numpy() - ref["h2"]) <= 1e-4 * (1 + np.abs(ref["h2"]))) > 0.999
    assert np.quantile(err, 0.999) <= 1e-4 * scale
    assert err.max() <= 8e-3 * scale


def test_mlp_backward_bce_adam_match_reference():
    import torch

    n = 5000
    w32 = mlp.init_params(12)
    w32[mlp.OB1:mlp.OW2] = 0.05
    w32[mlp.OB2:mlp.OW3] = 0.05
    w, wb = _shadow(w32)
    x32 = _x(3, n)
    y32 = (np.random.default_rng(4).random(n) < 0.3).astype(np.float32)
    x, prob, logit, h1, h2 = _forward(x32, wb)
    dlogit = torch.empty(n, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    scr = torch.empty(S.spdba_mlp_backward_scratch(n), dtype=torch.uint8, device="cuda")
    S.spdba_mlp_bce(logit, T(y32), 3.0, dlogit, loss, scr)
    torch.cuda.synchronize()
    ref_loss, ref_d = mlp.bce(logit.cpu().numpy(), y32, 3.0)
    assert abs(loss.item() - ref_loss) <= 1e-6 * abs(ref_loss)
    assert np.allclose(dlogit.cpu().numpy(), ref_d, rtol=1e-5, atol=1e-9)
    grad = torch.empty(mlp.NPARAM, device="cuda")
    S.spdba_mlp_backward(x, h1, h2, dlogit, w, grad, scr)
    torch.cuda.synchronize()
    fw = dict(h1=h1.cpu().numpy(), h2=h2.cpu().numpy())
    ref_g = mlp.backward_bf16(x32, w32, fw, dlogit.cpu().numpy())
    g = grad.cpu().numpy()
    for name, a, b in (("W1", mlp.OW1, mlp.OB1), ("b1", mlp.OB1, mlp.OW2), ("W2", mlp.OW2, mlp.OB2),
                       ("b2", mlp.OB2, mlp.OW3), ("W3", mlp.OW3, mlp.OB3), ("b3", mlp.OB3, mlp.NPARAM)):
        err = np.linalg.norm(g[a:b] - ref_g[a:b]) / max(np.linalg.norm(ref_g[a:b]), 1e-30)
        print(f"grad {name}: rel-L2 {err:.2e}", flush=True)
        assert err <= 1e-3, name
    # the bf16 gradients track the FP64 definition to bf16 precision
    g64 = mlp.backward64(x32, w32.astype(np.float64), mlp.forward64(x32, w32), dlogit.cpu().numpy())
    assert np.linalg.norm(g - g64) <= 0.05 * np.linalg.norm(g64)
    # Adam step
    m = torch.zeros(mlp.NPARAM, device="cuda")
    v = torch.zeros(mlp.NPARAM, device="cuda")
    S.spdba_mlp_adam(w, m, v, grad, wb, 1e-3, 1)
    torch.cuda.synchronize()
    ref_w, _, _ = mlp.adam(w32.astype(np.float64), 0, 0, g.astype(np.float64), 1, 1e-3)
    assert np.allclose(w.cpu().numpy(), ref_w, rtol=1e-6, atol=1e-7)
    assert np.array_equal(wb.cpu().numpy().view(np.uint16), mlp.bf16_bits(w.cpu().numpy()))


def test_training_on_device_reduces_loss():
    import torch

    n = 8192
    r = np.random.default_rng(8)
    x32 = r.uniform(-1, 1, (n, 8)).astype(np.float32)
    y32 = ((x32[:, 0] + 0.5 * x32[:, 1] - 0.3 * x32[:, 4]) > 0.2).astype(np.float32)
    w, wb = _shadow(mlp.init_params(9))
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    x, yt = T(x32), T(y32)
    prob = torch.empty(n, device="cuda")
    logit = torch.empty(n, device="cuda")
    h1 = torch.empty(n, 64, device="cuda")
    h2 = torch.empty(n, 64, device="cuda")
    dl = torch.empty(n, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(mlp.NPARAM, device="cuda")
    scr = torch.empty(S.spdba_mlp_backward_scratch(n), dtype=torch.uint8, device="cuda")
    losses = []
    for t in range(1, 301):
        S.spdba_mlp_forward(x, wb, prob, logit, h1, h2)
        S.spdba_mlp_bce(logit, yt, 1.0, dl, loss, scr)
        S.spdba_mlp_backward(x, h1, h2, dl, w, grad, scr)
        S.spdba_mlp_adam(w, m, v, grad, wb, 3e-3, t)
        if t % 50 == 1 or t == 300:
            losses.append(loss.item())
    acc = np.mean((prob.cpu().numpy() > 0.5) == (y32 > 0.5))
    print(f"training losses {['%.4f' % l for l in losses]}, accuracy {acc:.4f}", flush=True)
    assert losses[-1] < 0.3 * losses[0]
    assert acc > 0.95


def test_features_labels_skip_miss_match_reference():
    import torch

    d = S.Desc(op="ch", dtype="f32", ndim=3, n=32, block=8, tau=1e-4, dx=1.0, dt=0.01, params=(1.0, 1.0))
    q, r, k0, rk0 = draw_apply_inputs(d, 51, 0)
    plan = S.Plan([d])
    nb = d.n_blocks
    eb = torch.zeros(nb, dtype=torch.float64, device="cuda")
    plan.set_block_energy(eb)
    plan.set_spectrum(0, torch.from_numpy(q), k0=k0)
    plan.apply(torch.from_numpy(r), rk0)
    ab_addr, mask_addr, g_addr, nbt = plan.device_views()
    assert nbt == nb
    x = torch.empty(nb, 8, device="cuda")
    scr = torch.empty(4096, dtype=torch.uint8, device="cuda")
    S.spdba_proposer_features(plan, [ab_addr] * 3, [g_addr] * 3, mask_addr, eb, 0.3, x, scr,
                              stream=plan.stream)
    plan.synchronize()
    # reference: the oracle's own indicator on the same seeded spectra
    ref = oracle_apply(d, q, r, k0, rk0)
    qq = q.astype(np.complex128).reshape(32, 32, 32)
    e = (np.abs(qq) ** 2)
    e[0, 0, 0] = k0[0] ** 2  # the k = 0 coefficient lives in FP64
    e_b = e.reshape(4, 8, 4, 8, 4, 8).sum(axis=(1, 3, 5)).ravel()
    assert np.allclose(eb.cpu().numpy(), e_b, rtol=1e-12, atol=0)
    fref = mlp.block_features(d.dims3, d.block3, [ref["a_b"]] * 3, [ref["G"]] * 3, ref["mask"], e_b, 0.3)
    f = x.cpu().numpy()
    assert np.allclose(f, fref, rtol=1e-5, atol=1e-6), np.abs(f - fref).max(axis=0)
    # labels, skip sets and the miss counter
    masks = np.stack([ref["mask"], np.roll(ref["mask"], 3), np.zeros(nb, np.uint8)])
    y = torch.empty(nb, device="cuda")
    S.spdba_proposer_labels(T(masks), y)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), mlp.labels(masks))
    p = np.random.default_rng(3).random(nb).astype(np.float32)
    sk = torch.empty(nb, dtype=torch.uint8, device="cuda")
    nsk = torch.zeros(1, dtype=torch.int32, device="cuda")
    S.spdba_proposer_skip(T(p), 0.4, sk, count=nsk)
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    S.spdba_proposer_miss(sk, T(ref["mask"]), nb, cnt)
    torch.cuda.synchronize()
    assert np.array_equal(sk.cpu().numpy(), (p < 0.4).astype(np.uint8))
    assert nsk.item() == int(np.sum(p < 0.4))
    assert cnt.item() == int(np.sum((p < 0.4) & (ref["mask"] > 0)))
    # a set gate (a miss count) clears the whole set and counts nothing
    S.spdba_proposer_skip(T(p), 0.4, sk, gate=cnt if cnt.item() else torch.ones_like(cnt), count=nsk)
    torch.cuda.synchronize()
    assert int(sk.sum().item()) == 0 and nsk.item() == int(np.sum(p < 0.4))
    plan.destroy()
