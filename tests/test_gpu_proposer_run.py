"""End-to-end learned proposer on a small 3-D Cahn-Hilliard grid: train on
masks logged from plain runs, choose the threshold on a held-out seed, then
run an unseen seed with the window protocol over a 500-step horizon.  The
proposer must save more than 8 % of the block-steps' indicator evaluations
while its field stays as close to the dense update as plain sp-DBA's."""
import numpy as np
import pytest

from paper_2609_03922_amd import inputs
from paper_2609_03922_amd import proposer as P
from paper_2609_03922_amd import spdba as S

pytestmark = pytest.mark.gpu

N, B, STEPS, K = 64, 8, 500, 10


def _desc(**kw):
    return S.Desc(op="ch", dtype="f32", ndim=3, n=N, block=B, tau=1e-6, dx=1.0, dt=0.01,
                  params=(1.0, 1.0), **kw)


def _plan(seed, **kw):
    import torch

    p = S.Plan([_desc(**kw)])
    f = inputs.uniform_field(seed, 0, (N, N, N), 0.1, 0.02, dtype=np.float32)
    p.set_field(0, torch.from_numpy(f.ravel()))
    return p


def _log(seed):
    plan = _plan(seed)
    run = P.WindowRunner(plan, None, K=K, total_steps=STEPS, log_masks=True)
    run.step(STEPS)
    X, Y = run.dataset()
    plan.destroy()
    return X, Y


def test_proposer_trains_and_skips_with_bounded_error():
    import torch

    Xs, Ys = zip(*[_log(s) for s in (2001, 2002)])
    X, Y = torch.cat(Xs), torch.cat(Ys)
    prop = P.Proposer(seed=1)
    losses = prop.train(X, Y, epochs=40, batch=2048, lr=3e-3, pos_weight=4.0)
    Xh, Yh = _log(2003)
    thr = prop.choose_threshold(Xh, Yh, recall=1.0)
    p = prop.predict(Xh).cpu().numpy()
    y = Yh.cpu().numpy() > 0.5
    recall = np.mean(p[y] >= thr)
    skip_share = np.mean(p < thr)
    print(f"losses {losses[0]:.4f} -> {losses[-1]:.4f}; held-out positives {y.mean():.3f}, "
          f"threshold {thr:.4f}, recall {recall:.4f}, proposed skip share {skip_share:.3f}", flush=True)
    assert losses[-1] < losses[0]
    assert recall == 1.0
    # the protocol-simulating threshold: the chosen entry respects the cap on
    # miss windows and is the best gain among those that do
    nb = (N // B) ** 3
    thr_w = prop.choose_threshold_windows(Xh, Yh, nb, max_miss_windows=0.2)
    tab = prop.threshold_table
    chosen = [r for r in tab if r[0] == thr_w][0]
    ok = [r for r in tab if r[2] <= 0.2]
    print(f"window-simulation threshold {thr_w:.4f}: held-out skip share {chosen[1]:.3f}, "
          f"miss windows {chosen[2]:.3f}", flush=True)
    assert chosen[2] <= 0.2 and chosen[1] >= max(r[1] for r in ok) - 1e-12
    prop.threshold = thr

    # unseen seed: plain, proposer, dense
    fields = {}
    hist = None
    for mode in ("plain", "proposer", "dense"):
        plan = _plan(1005, dense=(mode == "dense"))
        run = P.WindowRunner(plan, prop if mode == "proposer" else None, K=K, total_steps=STEPS)
        run.step(STEPS)
        fields[mode] = plan.get_field(0).double().cpu().numpy()
        if mode == "proposer":
            hist = dict(run.history)
        plan.destroy()
    mean = fields["dense"].mean()
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b - mean)
    e_plain = rel(fields["plain"], fields["dense"])
    e_prop = rel(fields["proposer"], fields["dense"])
    e_pp = rel(fields["proposer"], fields["plain"])
    skipped = hist["skipped_block_steps"] / (hist["steps"] * (N // B) ** 3)
    print(f"proposer run: {hist}; skipped block-steps {skipped:.3f}; rel-L2 plain-vs-dense {e_plain:.2e}, "
          f"proposer-vs-dense {e_prop:.2e}, proposer-vs-plain {e_pp:.2e}", flush=True)
    # the gain over the plain rule: the indicator evaluations of the skipped
    # block-steps are saved.  At 64^3 and tau = 1e-6 about two thirds of the
    # blocks turn active within a 10-step window (held-out positives 0.65),
    # and the audit steps evaluate every block, so at most about 0.35 x 7/10
    # of the block-steps can be skipped; with the recall-1 threshold the
    # proposer skips more than 8 % of all block-steps (0.102 measured), while
    # its field stays as close to the dense update as the plain rule's
    # (within a factor 1.5 of that error, plus FP32 round-off)
    print(f"indicator block evaluations saved vs plain: {skipped:.3f}", flush=True)
    assert skipped >= 0.08
    assert hist["misses"] <= hist["windows"] // 2
    assert e_prop <= 1.5 * e_plain + 1e-7 and e_pp < 1e-4
