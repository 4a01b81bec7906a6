"""Learned activation proposer: training data from plain sp-DBA runs, on-device
training with the library's bf16-MFMA kernels, and the windowed run with exact
audits and fallback.

Window protocol (K steps per window, the last `audit` of them audits):
  * steps 0 .. K-audit-1 of window w+1 freeze the proposed skip set S without
    evaluating the indicator on it (spdba_set_skip);
  * the audit steps evaluate every block exactly; their a_b, G, mask and block
    energies feed the features of the next proposal;
  * a miss (a block of S found active at an audit step) makes the next window
    run the plain rule; the first window always runs the plain rule.
Labels for training: a block is positive if it is active at any step of the
next window under the plain rule.

Every step of the method runs in libspdba.so; this module only sequences calls
and moves device buffers.
"""
from __future__ import annotations

import numpy as np

from . import spdba as S

NPARAM = 4801
OW1, OB1, OW2, OB2, OW3, OB3 = 0, 512, 576, 4672, 4736, 4800


class Proposer:
    """MLP parameters (FP32 master, bf16 shadow) and Adam moments on the GPU."""

    def __init__(self, seed: int = 0, weights=None):
        import torch

        self.torch = torch
        if weights is None:
            r = np.random.default_rng([seed, 11])
            w = np.zeros(NPARAM, np.float32)
            w[OW1:OB1] = r.standard_normal(512) * np.sqrt(2.0 / 8)
            w[OW2:OB2] = r.standard_normal(4096) * np.sqrt(2.0 / 64)
            w[OW3:OB3] = r.standard_normal(64) * np.sqrt(1.0 / 64)
            weights = w
        self.w = torch.from_numpy(np.asarray(weights, np.float32).copy()).cuda()
        self.wb = torch.empty(NPARAM, dtype=torch.int16, device="cuda")
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.t = 0
        self.threshold = 0.5
        S.spdba_mlp_to_bf16(self.w, self.wb)

    def predict(self, x, prob=None, stream=None):
        if prob is None:
            prob = self.torch.empty(x.shape[0], device="cuda")
        S.spdba_mlp_forward(x, self.wb, prob, stream=stream)
        return prob

    def train(self, X, Y, epochs=4, batch=16384, lr=2e-3, pos_weight=4.0, seed=0):
        """Minibatch Adam on (X [n, 8] FP32, Y [n] FP32) resident on the GPU."""
        torch = self.torch
        n = X.shape[0]
        bsz = min(batch, n)
        logit = torch.empty(bsz, device="cuda")
        h1 = torch.empty(bsz, 64, device="cuda")
        h2 = torch.empty(bsz, 64, device="cuda")
        dl = torch.empty(bsz, device="cuda")
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        grad = torch.empty(NPARAM, device="cuda")
        scr = torch.empty(S.spdba_mlp_backward_scratch(bsz), dtype=torch.uint8, device="cuda")
        gen = torch.Generator(device="cuda")
        gen.manual_seed(int(seed))
        losses = []
        for _ in range(epochs):
            perm = torch.randperm(n, device="cuda", generator=gen)
            tot, cnt = 0.0, 0
            for s0 in range(0, n - bsz + 1, bsz):
                idx = perm[s0:s0 + bsz]
                xb = X.index_select(0, idx).contiguous()
                yb = Y.index_select(0, idx).contiguous()
                S.spdba_mlp_forward(xb, self.wb, None, logit, h1, h2)
                S.spdba_mlp_bce(logit, yb, pos_weight, dl, loss, scr)
                S.spdba_mlp_backward(xb, h1, h2, dl, self.w, grad, scr)
                self.t += 1
                S.spdba_mlp_adam(self.w, self.m, self.v, grad, self.wb, lr, self.t)
                tot += loss.item()
                cnt += 1
            losses.append(tot / max(cnt, 1))
        return losses

    def choose_threshold(self, X, Y, recall=1.0):
        """Largest threshold whose recall of positive labels is >= `recall`
        (recall 1: just below the lowest score of any positive)."""
        p = self.predict(X).cpu().numpy()
        y = Y.cpu().numpy() > 0.5
        pos = np.sort(p[y])
        if pos.size == 0:
            self.threshold = 0.5
            return self.threshold
        k = int(np.floor((1.0 - recall) * pos.size))
        self.threshold = float(np.nextafter(pos[k], -np.inf)) if k < pos.size else 0.0
        return self.threshold

    def state(self):
        return dict(weights=self.w.cpu().numpy(), threshold=self.threshold)


class WindowRunner:
    """Steps a bound plan with the window protocol (or the plain rule when
    `proposer` is None), keeping the audit snapshots on the device."""

    def __init__(self, plan: S.Plan, proposer: Proposer | None, K: int = 10, audit: int = 3,
                 total_steps: int = 500, log_masks: bool = False):
        import torch

        self.torch = torch
        self.plan, self.prop = plan, proposer
        self.K, self.audit, self.total = K, audit, total_steps
        self.nb = plan.total_blocks()
        n_inst = len(plan.descs)
        dev = "cuda"
        self.ab = torch.zeros(3, self.nb, dtype=torch.float64, device=dev)
        self.G = torch.zeros(3, n_inst, dtype=torch.float64, device=dev)
        self.eb = torch.zeros(self.nb, dtype=torch.float64, device=dev)
        self.x = torch.empty(self.nb, 8, device=dev)
        self.prob = torch.empty(self.nb, device=dev)
        self.skip = torch.zeros(self.nb, dtype=torch.uint8, device=dev)
        self.miss = torch.zeros(1, dtype=torch.int32, device=dev)
        self.fscr = torch.empty(max(4096, 520 * n_inst), dtype=torch.uint8, device=dev)
        self.ab_addr, self.mask_addr, self.g_addr, _ = plan.device_views()
        self.step_no = 0
        self.proposing = False  # a skip set is armed for the current window
        self.log_masks = log_masks
        self.win_masks = torch.zeros(K, self.nb, dtype=torch.uint8, device=dev)
        self.windows = []  # (features of window w) for training
        self.history = dict(windows=0, misses=0, fallbacks=0, skipped_block_steps=0, steps=0)
        self._skip_count = 0

    def _snapshot(self, slot):
        _copy_from_addr(self.ab[slot], self.ab_addr, self.nb * 8, self.plan.stream)
        _copy_from_addr(self.G[slot], self.g_addr, self.G.shape[1] * 8, self.plan.stream)

    def step(self, n: int = 1):
        torch = self.torch
        for _ in range(n):
            pos = self.step_no % self.K
            audit = pos >= self.K - self.audit
            if audit:
                self.plan.set_skip(None)
                self.plan.set_block_energy(self.eb)
            elif self.proposing:
                self.plan.set_skip(self.skip)
                self.plan.set_block_energy(None)
            else:
                self.plan.set_skip(None)
                self.plan.set_block_energy(None)
            self.plan.step(1)
            self.history["steps"] += 1
            if self.proposing and not audit:
                self.history["skipped_block_steps"] += int(self._skip_count)
            if self.log_masks:
                _copy_from_addr(self.win_masks[pos], self.mask_addr, self.nb, self.plan.stream)
            if audit:
                # newest snapshot first: slot 0 is the last audit step
                self._snapshot(self.K - 1 - pos)
                if self.proposing:
                    S.spdba_proposer_miss(self.skip, self.mask_addr, self.nb, self.miss, stream=self.plan.stream)
            self.step_no += 1
            if pos == self.K - 1:
                self._end_window()

    def _end_window(self):
        torch = self.torch
        self.history["windows"] += 1
        missed = False
        if self.proposing:
            self.plan.synchronize()
            missed = int(self.miss.item()) > 0
            self.miss.zero_()
            if missed:
                self.history["misses"] += 1
        frac = self.step_no / float(self.total)
        S.spdba_proposer_features(self.plan, [self.ab[0], self.ab[1], self.ab[2]],
                                  [self.G[0], self.G[1], self.G[2]], self.mask_addr, self.eb, frac,
                                  self.x, self.fscr, stream=self.plan.stream)
        if self.log_masks:
            self.windows.append((self.x.clone(), self.win_masks.clone()))
        if self.prop is None or missed:
            if missed:
                self.history["fallbacks"] += 1
            self.proposing = False
            return
        self.plan.synchronize()
        self.prop.predict(self.x, self.prob)
        S.spdba_proposer_skip(self.prob, self.prop.threshold, self.skip)
        torch.cuda.synchronize()
        self._skip_count = int(self.skip.sum().item())
        self.proposing = True

    def dataset(self):
        """(X, Y) pairs: features at the end of window w, labels = union of
        the masks of window w+1."""
        torch = self.torch
        X, Y = [], []
        for w in range(len(self.windows) - 1):
            X.append(self.windows[w][0])
            y = torch.empty(self.nb, device="cuda")
            S.spdba_proposer_labels(self.windows[w + 1][1], y)
            Y.append(y)
        torch.cuda.synchronize()
        return torch.cat(X), torch.cat(Y)


def _copy_from_addr(dst, src_addr: int, nbytes: int, stream):
    """Device-to-device copy from a raw library address into a torch tensor,
    ordered on the plan's stream."""
    import ctypes

    hip = _hip()
    rc = hip.hipMemcpyAsync(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_addr),
                            ctypes.c_size_t(nbytes), 3, ctypes.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({rc})")


_HIP = None


def _hip():
    global _HIP
    if _HIP is None:
        import ctypes

        import torch  # noqa: F401  (the runtime is already loaded by torch)

        _HIP = ctypes.CDLL("libamdhip64.so.7")
        _HIP.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int, ctypes.c_void_p]
        _HIP.hipMemcpyAsync.restype = ctypes.c_int
    return _HIP
