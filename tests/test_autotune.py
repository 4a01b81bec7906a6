"""Host logic of the launch autotuner, on the CPU with a stand-in plan: the
cache key names the measure and the layout (the kept state measure changes
which update variants apply), the key of a tuning comes from the sparse plan,
and the fastest update variant and its grid are the ones kept."""
from paper_2609_03922_amd import autotune as A
from paper_2609_03922_amd import spdba as S


def _desc(**kw):
    return S.Desc(op="ch", dtype="f32", ndim=3, n=64, block=8, tau=1e-6, dx=1.0, dt=0.01, params=(1.0, 1.0), **kw)


def test_cache_key_names_measure_and_layout():
    keys = {A.cache_key([_desc(**kw)], "gfx950") for kw in
            ({}, {"state_indicator": True}, {"state_indicator": True, "block_energy": True}, {"half": True})}
    assert len(keys) == 4
    assert A.cache_key([_desc(state_indicator=True)], "gfx950").endswith("|state")
    assert A.cache_key([_desc()], "gfx950") == "gfx950|ch|f32|nd3|b8|n[64]"


class FakePlan:
    """Stage times from a table: update stages (3, 4) by (variant, per-CU), the
    indicator (2) by its waves, the dense update (4) by its threads."""

    def __init__(self, descs, dense):
        self.descs, self.dense, self.launch = descs, dense, {}

    def set_launch(self, k, v):
        self.launch[k] = v

    def step(self, n):
        pass

    def stats(self, i):
        st = [0.0] * 5
        st[0] = 2.0 - 0.5 * self.launch.get(5, 0)  # transforms: in place faster here
        if self.dense:
            st[4] = 1.0 / self.launch.get(2, 256)
        else:
            st[2] = 1.0 + self.launch.get(0, 4)
            v, g = self.launch.get(3, 1), self.launch.get(1, 4)
            st[3] = 0.1
            st[4] = {0: 5.0, 1: 6.0, 2: 5.5, 3: 4.0, 4: 4.5}[v] + abs(g - (8 if v == 3 else 4)) * 0.1
        return {"stage_ms": st}

    def destroy(self):
        pass


def test_tune_keys_the_sparse_plan_and_keeps_the_fastest_variant(tmp_path):
    sparse = [_desc(state_indicator=True)]
    path = str(tmp_path / "cache.json")
    res, timings = A.tune(lambda dense: FakePlan([_desc()] if dense else sparse, dense), lambda p: None,
                          steps=1, path=path)
    assert res[3] == 3 and res[1] == 8 and res[0] == 1 and res[2] == 1024
    assert "wave 1:8" in timings and "list4 1:4" in timings and "run 1:4" in timings
    cache = A.load_cache(path)
    assert sorted(cache) == sorted([A.cache_key(sparse, "gfx950"), A.fft_key(sparse, "gfx950")])
    assert cache[A.cache_key(sparse, "gfx950")]["choice"]["3"] == 3
    # the transform placement: timed on the dense plan, cached without block shape or measure
    assert res[5] == 1 and cache[A.fft_key(sparse, "gfx950")]["choice"] == {"5": 1}
    assert "5" not in cache[A.cache_key(sparse, "gfx950")]["choice"]
    assert A.fft_key([_desc()], "gfx950") == A.fft_key(sparse, "gfx950") == "gfx950|ch|f32|nd3|n[64]|fft"
    # both plans of the grid take it
    for descs in (sparse, [_desc()]):
        p = FakePlan(descs, False)
        A.apply_cached(p, "gfx950", path=path)
        assert p.launch[5] == 1


def test_tune_skips_the_placement_a_plan_refuses(tmp_path):
    class NoInPlace(FakePlan):
        def set_launch(self, k, v):
            if k == 5 and v:
                raise RuntimeError("EUNSUPPORTED")
            super().set_launch(k, v)

    sparse = [_desc(state_indicator=True)]
    path = str(tmp_path / "cache.json")
    res, _ = A.tune(lambda dense: NoInPlace([_desc()] if dense else sparse, dense), lambda p: None, steps=1,
                    path=path)
    assert 5 not in res
    assert list(A.load_cache(path)) == [A.cache_key(sparse, "gfx950")]


def test_bench_names_the_update_kernel_of_the_tuned_variant():
    """The roofline line names the kernel the plan launches for the tuned
    update variant: the kept state measure rules out the strip walk and the x4
    walk; the wave walk needs blocks of at least 64 lane slots."""
    import bench
    from paper_2609_03922_amd import configs as C

    cfg = C.CH3D_256_F32
    d = [S.desc_from_config(cfg)]
    name = bench.update_kernel_name
    assert name(cfg, d, "state", "full", {"3": 3}) == "k_update_wave"
    assert name(cfg, d, "state", "full", {"3": 1}) == "k_update"
    assert name(cfg, d, "state", "full", {"3": 2}) == "k_update"
    assert name(cfg, d, "increment", "full", {"3": 2}) == "k_update_multi"
    assert name(cfg, d, "increment", "full", None) == "k_update_strip"
    assert name(cfg, d, "state", "half", {"3": 3}) == "k_update_h"
    assert name(cfg, d, "state", "full", {"3": 4}) == "k_update_run"
    assert name(cfg, d, "increment", "full", {"3": 4}) == "k_update_run"
    assert name(cfg, d, "energy", "full", {"3": 4}) == "k_update"      # block energy: no band sums
    small = [S.Desc(op="ch", dtype="f32", ndim=2, n=16, block=4, tau=1e-2, dx=1.0, dt=0.01, params=(1.0, 1.0))]
    assert name(cfg, small, "increment", "full", {"3": 3}) == "k_update"   # 8 slots: below a wave
    assert name(cfg, small, "increment", "full", {"3": 4}) == "k_update"   # run walk: 256 or 512 slots
