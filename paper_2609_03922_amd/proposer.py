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

    def choose_threshold_windows(self, X, Y, nb: int, max_miss_windows: float = 0.2):
        """Threshold from a simulation of the window protocol on held-out
        windows (X, Y: consecutive windows of nb blocks each).  A threshold t
        proposes the set p < t for the next window; a window whose set holds a
        positive block is a miss and the window after it runs the plain rule.
        Returns the t that maximises the skipped share over all windows, among
        those whose miss windows are at most `max_miss_windows` of the total
        (t = 0, nothing skipped, always qualifies)."""
        p = self.predict(X).cpu().numpy().reshape(-1, nb)
        y = Y.cpu().numpy().reshape(-1, nb) > 0.5
        W = p.shape[0]
        pos = np.sort(p[y])
        # candidates: just below each of the lowest positive scores, then a
        # coarse ladder above them
        cand = [0.0] + [float(np.nextafter(v, -np.inf)) for v in pos[:256]]
        cand += [float(v) for v in np.quantile(pos, np.linspace(0.001, 0.2, 60))]
        best, best_gain, table = 0.0, 0.0, []
        for t in sorted(set(cand)):
            skip = p < t
            share = skip.mean(axis=1)
            miss = (skip & y).any(axis=1)
            plain_next = np.concatenate([[False], miss[:-1]])  # fallback windows
            gain = float(np.where(plain_next, 0.0, share).mean())
            frac = float(miss.mean())
            table.append((t, gain, frac))
            if frac <= max_miss_windows and gain > best_gain:
                best, best_gain = t, gain
        self.threshold = best
        self.threshold_table = table
        return best

    def state(self):
        return dict(weights=self.w.cpu().numpy(), threshold=self.threshold)


class WindowRunner:
    """Steps a bound plan with the window protocol (or the plain rule when
    `proposer` is None), keeping the audit snapshots on the device.

    Nothing in a window waits for the host: the miss count of the audits gates
    the next skip set on the device (spdba_proposer_skip), and the per-window
    miss and skip counts are kept in device arrays that `history` reads once."""

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
        cap = total_steps // K + 2
        self.miss_hist = torch.zeros(cap, dtype=torch.int32, device=dev)  # misses found in window w
        self.skip_hist = torch.zeros(cap, dtype=torch.int32, device=dev)  # blocks skipped in window w
        self.fscr = torch.empty(max(4096, 520 * n_inst), dtype=torch.uint8, device=dev)
        self.ab_addr, self.mask_addr, self.g_addr, _ = plan.device_views()
        self.step_no = 0
        self.window = 0
        self.proposing = False  # a (possibly empty) skip set is armed for the current window
        self.log_masks = log_masks
        self.win_masks = torch.zeros(K, self.nb, dtype=torch.uint8, device=dev)
        self.windows = []  # (features of window w) for training

    def _grow(self):
        torch = self.torch
        if self.window + 1 >= self.miss_hist.numel():
            z = torch.zeros_like(self.miss_hist)
            self.miss_hist = torch.cat([self.miss_hist, z])
            self.skip_hist = torch.cat([self.skip_hist, z.clone()])

    def _snapshot(self, slot):
        _copy_from_addr(self.ab[slot], self.ab_addr, self.nb * 8, self.plan.stream)
        _copy_from_addr(self.G[slot], self.g_addr, self.G.shape[1] * 8, self.plan.stream)

    def step(self, n: int = 1):
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
        st = self.plan.stream
        self._grow()
        frac = self.step_no / float(self.total)
        S.spdba_proposer_features(self.plan, [self.ab[0], self.ab[1], self.ab[2]],
                                  [self.G[0], self.G[1], self.G[2]], self.mask_addr, self.eb, frac,
                                  self.x, self.fscr, stream=st)
        if self.log_masks:
            with torch.cuda.stream(st):
                self.windows.append((self.x.clone(), self.win_masks.clone()))
        if self.prop is not None:
            self.prop.predict(self.x, self.prob, stream=st)
            # a miss in this window's audits leaves the next window's set empty
            S.spdba_proposer_skip(self.prob, self.prop.threshold, self.skip, gate=self.miss,
                                  count=self.skip_hist[self.window + 1:self.window + 2], stream=st)
            self.proposing = True
        with torch.cuda.stream(st):
            self.miss_hist[self.window:self.window + 1].copy_(self.miss)
            self.miss.zero_()
        self.window += 1

    @property
    def history(self):
        """Window counts (one device read): windows, windows whose audits found
        a proposed-skip block active (each makes the next window plain),
        skipped block-steps (skip set size times the window's proposal steps)."""
        self.plan.synchronize()
        m = self.miss_hist[:self.window].cpu().numpy()
        sk = self.skip_hist[:self.window + 1].cpu().numpy().astype(np.int64)
        # the set armed at the end of window w acts in window w + 1, on its
        # non-audit steps that have run
        steps_in = [min(self.K - self.audit, max(0, self.step_no - w * self.K)) for w in range(len(sk))]
        misses = int((m > 0).sum())
        return dict(windows=self.window, misses=misses, fallbacks=misses,
                    skipped_block_steps=int(sum(int(a) * b for a, b in zip(sk, steps_in))), steps=self.step_no)

    def dataset(self):
        """(X, Y) pairs: features at the end of window w, labels = union of
        the masks of window w+1."""
        torch = self.torch
        X, Y = [], []
        for w in range(len(self.windows) - 1):
            X.append(self.windows[w][0])
            y = torch.empty(self.nb, device="cuda")
            S.spdba_proposer_labels(self.windows[w + 1][1], y, stream=self.plan.stream)
            Y.append(y)
        self.plan.synchronize()
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
