"""Pins of the proposer's CPU reference: backprop against central finite
differences (FP64), bf16 rounding against torch's converter, Adam's first step
in closed form, and block features on hand-checkable inputs."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, n):
    r = np.random.default_rng(seed)
    x = r.uniform(-1, 1, (n, 8))
    y = (r.random(n) < 0.3).astype(np.float64)
    return x, y


def test_backprop_matches_finite_differences():
    x, y = _data(1, 40)
    w = mlp.init_params(3).astype(np.float64)
    w[mlp.OB1:mlp.OW2] = 0.05  # keep ReLUs away from their kinks
    w[mlp.OB2:mlp.OW3] = 0.05
    pw = 4.0
    fw = mlp.forward64(x, w)
    loss, d = mlp.bce(fw["logit"], y, pw)
    g = mlp.backward64(x, w, fw, d)
    r = np.random.default_rng(5)
    idx = np.concatenate([r.choice(mlp.NPARAM, 60, replace=False), [mlp.OB3, mlp.OW3, mlp.OB1]])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.bce(mlp.forward64(x, wp)["logit"], y, pw)[0] -
              mlp.bce(mlp.forward64(x, wm)["logit"], y, pw)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    import torch

    r = np.random.default_rng(2)
    v = np.concatenate([r.standard_normal(10000).astype(np.float32) * 10.0 ** r.integers(-8, 8, 10000),
                        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -1 - 2 ** -8, 0.0, 65504.0], np.float32)])
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16(v), want)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert mlp.bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert mlp.bf16(np.float32(1 + 3 * 2 ** -9)) == np.float32(1 + 2 ** -7)


def test_bf16_emulation_close_to_fp64():
    x, y = _data(4, 300)
    w = mlp.init_params(6)
    a = mlp.forward64(x, w)["logit"]
    b = mlp.forward_bf16(x, w)["logit"]
    assert np.max(np.abs(a - b)) < 0.05 * np.max(np.abs(a)) + 0.05
    fw64 = mlp.forward64(x, w)
    _, d = mlp.bce(fw64["logit"], y, 3.0)
    g64 = mlp.backward64(x, w, fw64, d)
    g16 = mlp.backward_bf16(x, w, mlp.forward_bf16(x, w), d.astype(np.float32))
    assert np.linalg.norm(g16 - g64) < 0.05 * np.linalg.norm(g64)


def test_adam_first_step_closed_form():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.02, 0.0])
    w1, m, v = mlp.adam(w, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    # first step: m_hat = g, v_hat = g^2, so the update is lr * g / (|g| + eps)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8))


def test_block_features_hand_cases():
    dims, block = (1, 8, 8), (1, 4, 4)
    ab = np.array([4.0, 1.0, 0.0, 0.04])
    mask = np.array([1, 0, 0, 1])
    eb = np.array([2.0, 1.0, 1.0, 0.0])
    f = mlp.block_features(dims, block, [ab, ab, ab], [4.0, 4.0, 4.0], mask, eb, 0.25)
    # log10(a/G): 0 -> 1.0; log10(1/4) -> 1 - 0.60206/40; zero -> 0; 0.01 -> 1 - 2/40
    assert np.allclose(f[:, 0], [1.0, 1 - np.log10(4) / 40, 0.0, 1 - 2 / 40])
    # 2x2 periodic block grid: each block's 4 face neighbours are the 2 others,
    # each counted twice (wrap); block 0's neighbours are blocks 1, 1, 2, 2
    assert np.allclose(f[:, 4] * 6, [0, 4, 4, 0])
    assert np.all(f[:, 5] == 0.25)
    # E_b * nb / E_tot: 2 * 4 / 4 = 2 -> log10 2 / 40
    assert np.isclose(f[0, 6], np.log10(2.0) / 40)
    assert f[3, 6] == -1.0
    assert np.array_equal(f[:, 7], mask)
    # one block covering the grid: mean |k| over all modes / (n/2)
    g = mlp.block_features((1, 1, 16), (1, 1, 16), [np.ones(1)] * 3, [1.0] * 3, np.ones(1), np.ones(1), 0.0)
    m = np.where(np.arange(16) < 8, np.arange(16), np.arange(16) - 16)
    assert np.isclose(g[0, 3], np.mean(np.abs(m)) / 8)
    assert np.array_equal(mlp.labels([[0, 1, 0], [0, 0, 1]]), [0, 1, 1])


def test_bce_closed_forms():
    """Weighted BCE on logits: at z = 0 every sample costs ln 2, the positive
    weight multiplying the positives only; far from zero the loss is |z| on the
    wrong side (times the weight for positives) and vanishes on the right side.
    A loss with the weight on the wrong class, or with a sign slip in the
    softplus arguments, fails these values."""
    ln2 = np.log(2.0)
    pw = 5.0
    y = np.array([1.0, 1.0, 0.0, 0.0, 0.0])
    loss, d = mlp.bce(np.zeros(5), y, pw)
    assert np.isclose(loss, (2 * pw * ln2 + 3 * ln2) / 5, rtol=0, atol=1e-15)
    # gradient at z = 0: sigmoid(0) = 1/2, so pw (p - 1) = -pw/2 for positives, +1/2 for negatives
    assert np.allclose(d, np.array([-pw / 2, -pw / 2, 0.5, 0.5, 0.5]) / 5, rtol=0, atol=1e-16)
    big = 40.0
    # all positives: right side costs pw * log(1 + e^-40), wrong side pw * (40 + log(1 + e^-40))
    l_right, _ = mlp.bce(np.array([big]), np.array([1.0]), pw)
    l_wrong, d_wrong = mlp.bce(np.array([-big]), np.array([1.0]), pw)
    assert np.isclose(l_right, pw * np.log1p(np.exp(-big)), rtol=1e-12)
    assert np.isclose(l_wrong, pw * (big + np.log1p(np.exp(-big))), rtol=1e-14)
    assert np.isclose(d_wrong[0], -pw * (1 - 1 / (1 + np.exp(big))), rtol=1e-14)
    # all negatives: no weight
    l_wrong0, d_wrong0 = mlp.bce(np.array([big]), np.array([0.0]), pw)
    assert np.isclose(l_wrong0, big + np.log1p(np.exp(-big)), rtol=1e-14)
    assert np.isclose(d_wrong0[0], 1 / (1 + np.exp(-big)), rtol=1e-14)
    assert np.isclose(mlp.bce(np.array([-big]), np.array([0.0]), pw)[0], np.log1p(np.exp(-big)), rtol=1e-12)


def _hand_net():
    """x = (1, 1, 0, ...): h1_0 = 1 + 2^-9 (FP32-exact, a bf16 tie that rounds
    to 1), h1_1 = 1; h2_0 = bf16(h1_0) + 2^-9 bf16(h1_1); logit = 512 h2_0.
    Every weight is a power of two (bf16-exact)."""
    W1 = np.zeros((8, 64))
    W2 = np.zeros((64, 64))
    W3 = np.zeros(64)
    W1[0, 0] = 1.0
    W1[1, 0] = 2.0 ** -9
    W1[0, 1] = 1.0
    W2[0, 0] = 1.0
    W2[1, 0] = 2.0 ** -9
    W2[1, 1] = 1.0
    W3[0] = 512.0
    w = mlp.pack(W1, np.zeros(64), W2, np.zeros(64), W3, 0.0, np.float32)
    x = np.zeros((1, 8), np.float32)
    x[0, :2] = 1.0
    return x, w


def test_bf16_rounding_points_of_the_forward():
    """The emulation rounds each layer's input to bf16 before its product.
    With both hidden roundings the logit is 512 exactly; dropping the h1
    rounding gives 512 (1 + 2^-8) = 514, dropping the h2 rounding gives
    512 (1 + 2^-9) = 513, and FP64 without rounding gives 514."""
    x, w = _hand_net()
    assert mlp.forward_bf16(x, w)["logit"][0] == 512.0
    assert mlp.forward64(x, w)["logit"][0] == 514.0
    # the layer values themselves: h1 keeps FP32 (the rounding is at the next input)
    fw = mlp.forward_bf16(x, w)
    assert fw["h1"][0, 0] == np.float32(1 + 2 ** -9) and fw["h2"][0, 0] == np.float32(1 + 2 ** -9)


def test_bf16_rounding_points_of_the_backward():
    """dW3 = bf16(h2)^T bf16(dlogit): with h2_0 = 1 + 2^-9 (rounds to 1) and
    dlogit = 1 + 2^-9 (rounds to 1) the emulated gradient entry is exactly 1,
    where FP64 gives (1 + 2^-9)^2.  dW1 = bf16(x)^T bf16(dh1) with dh1_0 =
    bf16(dh2) W2^T: dh2_0 = W3_0 dlogit = 512 + 1 = 513 rounds to 512 in bf16,
    so dh1_1 = 512 * 2^-9 = 1 (FP64: 513 * 2^-9)."""
    x, w = _hand_net()
    fw = mlp.forward_bf16(x, w)
    dl = np.array([1 + 2 ** -9], np.float32)
    g = mlp.backward_bf16(x, w, fw, dl)
    assert g[mlp.OW3 + 0] == 1.0
    W1g = g[mlp.OW1:mlp.OB1].reshape(8, 64)
    assert W1g[0, 1] == 1.0 and W1g[1, 1] == 1.0
    g64 = mlp.backward64(x, w, mlp.forward64(x, w), dl.astype(np.float64))
    assert g64[mlp.OW3 + 0] == (1 + 2 ** -8) * (1 + 2 ** -9)
    assert g64[mlp.OW1:mlp.OB1].reshape(8, 64)[1, 1] == 513 * 2.0 ** -9
