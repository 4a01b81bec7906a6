"""Launch-geometry autotuner for a plan.

Times candidate launch shapes of the indicator (waves per workgroup), the
active update (strip walk: waves per workgroup and persistent workgroups per
compute unit; block-list walks, one workgroup or one wave per entry:
workgroups per compute unit) and the dense
update (threads per workgroup) with the library's per-stage HIP events, keeps the
fastest, and caches the choice in a JSON file keyed by GPU architecture,
operator, precision, block shape, the multiset of grid sizes, the stored
layout and the measure (the kept state measure changes which update variants
apply).  Launch shape
never changes results (the reductions it touches are order-free maxima), so
tuning is safe between runs.  The activation block shape is not tuned: it
changes the masks.

The placement of the step's forward transform (out of place, or in place in
the transform buffer; CH and GS on the full layout) is timed on the dense plan
and cached under a key of its own without block shape or measure, so the dense
and the sparse plans of one grid take the same transforms.  rocFFT runs
different kernels for the two placements, which round differently, and which
one is faster depends on the size (in place wins for 512^3 FP32 and large 2-D
FP32 grids, loses for 256^3 and for FP64 3-D).
"""
from __future__ import annotations

import json
import os

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

CANDIDATES = {
    0: (1, 2, 4, 8),           # indicator: waves per workgroup
    1: (2, 4, 8, 16),          # list walk / persistent strip walk: workgroups per CU
    2: (128, 256, 512, 1024),  # dense update: threads per workgroup
    4: (2, 4, 8),              # strip-walk update: waves per workgroup
    5: (0, 1),                 # forward transform: out of place / in place
}
DEFAULTS = {0: 4, 1: 4, 2: 256, 3: 1, 4: 4, 5: 0}
# stage_ms entries a candidate is timed by: the update variants by compaction
# plus update, since the strip walk folds the threshold pass into the update
STAGE_OF = {0: (2,), 1: (3, 4), 2: (4,), 4: (3, 4), 5: (0,)}


def cache_key(descs, arch: str) -> str:
    d = descs[0]
    sizes = ",".join(str(x) for x in sorted((x.n for x in descs), reverse=True))
    layout = "|half" if getattr(d, "half", False) else ""
    measure = ("|energy" if getattr(d, "block_energy", False) else "|state") if getattr(d, "state_indicator", False) else ""
    return f"{arch}|{d.op}|{d.dtype}|nd{d.ndim}|b{d.block}|n[{sizes}]{layout}{measure}"


def fft_key(descs, arch: str) -> str:
    """Cache key of the transform placement: no block shape, no measure."""
    d = descs[0]
    sizes = ",".join(str(x) for x in sorted((x.n for x in descs), reverse=True))
    layout = "|half" if getattr(d, "half", False) else ""
    return f"{arch}|{d.op}|{d.dtype}|nd{d.ndim}|n[{sizes}]{layout}|fft"


def load_cache(path: str = CACHE_PATH) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(cache: dict, path: str = CACHE_PATH) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply_cached(plan, arch: str, path: str = CACHE_PATH) -> dict | None:
    cache = load_cache(path)
    entry = cache.get(cache_key(plan.descs, arch))
    if entry:
        for k, v in sorted(entry["choice"].items()):
            plan.set_launch(int(k), int(v))
    fft = cache.get(fft_key(plan.descs, arch))
    if fft:
        for k, v in sorted(fft["choice"].items()):
            plan.set_launch(int(k), int(v))
    return entry


def _accepts(plan, k, v) -> bool:
    try:
        plan.set_launch(k, v)
    except Exception:
        return False
    plan.set_launch(k, DEFAULTS[k])
    return True


def tune(make_plan, init_fields, steps: int = 20, arch: str = "gfx950", path: str | None = CACHE_PATH,
         warm: int = 0):
    """make_plan(dense: bool) -> Plan with timing enabled; init_fields(plan)
    loads the workload's initial state, which is then advanced `warm` steps so
    that the sweep sees the active fraction of the measured regime (the best
    update variant depends on it).  Each candidate is timed twice, in a forward
    and a reverse pass over the candidates, to cancel the slow drift of the
    active fraction.  Returns {kernel: best value} and the timings; stores them
    in the cache when `path` is given."""
    result, timings = {}, {}
    fft_choice, fkey = None, None

    def measure(plan, k, v, fixed):
        for fk, fv in fixed:
            plan.set_launch(fk, fv)
        plan.set_launch(k, v)
        plan.step(3)  # warm the shape
        plan.set_launch(k, v)  # restart the timing ring
        plan.step(steps)
        st = plan.stats(0)["stage_ms"]
        return sum(st[i] for i in STAGE_OF[k])

    def sweep(plan, k, fixed=(), tag=""):
        cand = list(CANDIDATES[k])
        acc = {v: 0.0 for v in cand}
        for order in (cand, cand[::-1]):
            for v in order:
                acc[v] += 0.5 * measure(plan, k, v, fixed)
        for v in cand:
            timings[f"{tag}{k}:{v}"] = acc[v]
        best = min(cand, key=lambda v: acc[v])
        return best, acc[best]

    for dense in (False, True):
        plan = make_plan(dense)
        init_fields(plan)
        if warm:
            plan.step(warm)
        if dense:
            result[2], _ = sweep(plan, 2)
            if _accepts(plan, 5, 1):
                fft_choice, _ = sweep(plan, 5)
                plan.set_launch(5, DEFAULTS[5])
                fkey = fft_key(plan.descs, arch)
        else:
            result[0], _ = sweep(plan, 0)
            plan.set_launch(0, result[0])
            # strip walk: waves per workgroup, then persistent workgroups per CU
            w4, _ = sweep(plan, 4, fixed=((3, 1),), tag="strip ")
            ps, t_strip = sweep(plan, 1, fixed=((3, 1), (4, w4)), tag="strip ")
            p1, t_list = sweep(plan, 1, fixed=((3, 0),), tag="list ")
            p2, t_multi = sweep(plan, 1, fixed=((3, 2),), tag="list4 ")
            p3, t_wave = sweep(plan, 1, fixed=((3, 3),), tag="wave ")
            p4, t_run = sweep(plan, 1, fixed=((3, 4),), tag="run ")
            best = min((t_strip, 1), (t_list, 0), (t_multi, 2), (t_wave, 3), (t_run, 4))[1]
            result[3] = best
            result[4] = w4
            result[1] = {1: ps, 0: p1, 2: p2, 3: p3, 4: p4}[best]
        if not dense:  # the sparse plan carries the measure the key names
            key = cache_key(plan.descs, arch)
        plan.destroy()
    if path:
        cache = load_cache(path)
        cache[key] = {"choice": {str(k): v for k, v in result.items()},
                      "stage_ms": {t: v for t, v in timings.items() if not t.startswith("5:")}}
        if fkey is not None:
            cache[fkey] = {"choice": {"5": fft_choice},
                           "stage_ms": {t: v for t, v in timings.items() if t.startswith("5:")}}
        save_cache(cache, path)
    if fft_choice is not None:
        result[5] = fft_choice
    return result, timings
