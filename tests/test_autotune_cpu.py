"""Launch-tuning table of the C ABI and the autotuner's cache logic (no GPU).

The timings here come from a stand-in timer; the GPU tests run the tuned
variants against the oracle."""
import ctypes
import json
from types import SimpleNamespace

import pytest

torch = pytest.importorskip("torch")

from paper_2103_08253_amd import _lib as L
from paper_2103_08253_amd import autotune as A


@pytest.fixture(autouse=True)
def clean_table():
    A.reset_tuning()
    yield
    A.reset_tuning()


def test_tuning_table_validation():
    lib = L.lib()
    # every depth that runs has its default variant among the variants
    for K in range(1, 9):
        lanes, waves = A.get_tuning(K)
        assert lanes in A.lane_variants(K)
        assert waves == 8
        assert all(64 % v == 0 and v <= 2 ** K for v in A.lane_variants(K))
    assert A.lane_variants(8) == [64]
    # depth 9: one variant, each point split over the 128 lanes of two waves
    assert A.lane_variants(9) == [128] and A.get_tuning(9) == (128, 8)
    assert lib.dmn_gp_set_tuning(9, ctypes.byref(L.DmnGpTuning(64, 4))) == L.DMN_EUNSUPPORTED
    # depth 10 is not compiled for the update (the call returns DMN_EUNSUPPORTED)
    assert A.lane_variants(10) == []
    assert A.lane_variants(5) == [16, 8]
    assert lib.dmn_gp_lane_variants(0, None, 0) == 0
    assert lib.dmn_gp_lane_variants(11, None, 0) == 0
    t = L.DmnGpTuning(8, 4)
    assert lib.dmn_gp_set_tuning(5, ctypes.byref(t)) == L.DMN_OK
    assert A.get_tuning(5) == (8, 4)
    assert lib.dmn_gp_set_tuning(5, ctypes.byref(L.DmnGpTuning(4, 4))) == L.DMN_EUNSUPPORTED
    assert lib.dmn_gp_set_tuning(5, ctypes.byref(L.DmnGpTuning(8, 65))) == L.DMN_EINVAL
    assert lib.dmn_gp_set_tuning(5, ctypes.byref(L.DmnGpTuning(-1, 4))) == L.DMN_EINVAL
    assert lib.dmn_gp_set_tuning(0, None) == L.DMN_EINVAL
    assert lib.dmn_gp_get_tuning(5, None) == L.DMN_EINVAL
    assert A.get_tuning(5) == (8, 4)  # rejected calls leave the table alone
    assert lib.dmn_gp_set_tuning(5, None) == L.DMN_OK
    assert A.get_tuning(5) == (16, 8)


def fake_groups(spec=((5, 3000), (8, 60000), (5, 1000))):
    return [SimpleNamespace(w=torch.zeros(2 ** K), E=torch.zeros(P, 6)) for K, P in spec]


def fake_timer(calls):
    def timer(groups, fiber, matrix, reps, newton):
        K = int(round(torch.log2(torch.tensor(float(groups[0].w.numel()))).item()))
        lanes, waves = A.get_tuning(K)
        calls.append((K, lanes, waves, sum(g.E.shape[0] for g in groups)))
        best = {5: (8, 4), 8: (64, 16)}[K]
        return 1.0 + abs(lanes - best[0]) + abs(waves - best[1]) / 100.0
    return timer


def test_autotuner_picks_fastest_and_caches(tmp_path):
    """Groups of one depth: every lane variant x wave count, timed on the
    depth's groups together; the cache sets the winner in a later process."""
    path = str(tmp_path / "tune.json")
    calls = []
    got = A.tune_gauss_points(fake_groups(((5, 3000), (5, 1000))), {}, {}, cache_path=path,
                              timer=fake_timer(calls), tag="dev")
    assert got[5]["lanes_per_point"] == 8 and got[5]["waves_per_cu"] == 4
    assert not got[5]["cached"]
    assert sorted({c[:3] for c in calls}) == sorted(
        (5, l, w) for l in A.lane_variants(5) for w in A.WAVES_PER_CU)
    assert {c[3] for c in calls} == {4000}
    assert A.get_tuning(5) == (8, 4)
    data = json.load(open(path))
    assert data[A.cache_key("dev", 5, 4000)]["lanes_per_point"] == 8
    got = A.tune_gauss_points(fake_groups(((8, 60000),)), {}, {}, cache_path=path,
                              timer=fake_timer(calls), tag="dev")
    assert got[8]["lanes_per_point"] == 64 and got[8]["waves_per_cu"] == 16
    # a second process start: the table is reset, the cache sets it without timing
    A.reset_tuning()
    calls.clear()
    got = A.tune_gauss_points(fake_groups(((5, 3000), (5, 1000))), {}, {}, cache_path=path,
                              timer=fake_timer(calls), tag="dev")
    assert calls == [] and got[5]["cached"] and A.get_tuning(5) == (8, 4)
    # another device tag misses the cache
    A.tune_gauss_points(fake_groups(((5, 4000),)), {}, {}, cache_path=path,
                        timer=fake_timer(calls), tag="other")
    assert calls
    assert len(json.load(open(path))) == 3


def test_autotuner_mixed_depths_tunes_the_mixed_launch(tmp_path):
    """Fixed-normal groups of several depths run in one mixed-depth launch:
    its wave count is timed on all groups of depths >= 2 together (lane splits
    are fixed there); a depth-1 group is tuned on its own."""
    path = str(tmp_path / "tune.json")
    calls = []

    def timer(groups, fiber, matrix, reps, newton):
        depths = sorted({int(round(torch.log2(torch.tensor(float(g.w.numel()))).item()))
                         for g in groups})
        waves = {A.get_tuning(K)[1] for K in depths}
        calls.append((tuple(depths), tuple(sorted(waves)), sum(g.E.shape[0] for g in groups)))
        return 1.0 + abs(min(waves) - 8) / 10.0 if depths != [1] else 1.0

    got = A.tune_gauss_points(fake_groups(((5, 3000), (9, 500), (8, 6000), (1, 70))), {}, {},
                              cache_path=path, timer=timer, tag="dev")
    assert sorted(got) == [1, 5, 8, 9]
    mixed = [c for c in calls if c[0] != (1,)]
    assert [c[1] for c in mixed] == [(w,) for w in A.WAVES_PER_CU]  # one wave count for all
    assert all(c[0] == (5, 8, 9) and c[2] == 9500 for c in mixed)
    for K in (5, 8, 9):
        assert got[K]["launch"] == "mixed" and got[K]["waves_per_cu"] == 8
        assert A.get_tuning(K)[1] == 8
    assert A.get_tuning(9)[0] == 128 and A.get_tuning(5)[0] == A.lane_variants(5)[0]
    assert "launch" not in got[1]
    data = json.load(open(path))
    assert data[A.mixed_cache_key("dev", [5, 8, 9], 9500)]["waves_per_cu"] == 8
    A.reset_tuning()
    calls.clear()
    again = A.tune_gauss_points(fake_groups(((5, 3000), (9, 500), (8, 6000), (1, 70))), {}, {},
                                cache_path=path, timer=timer, tag="dev")
    assert calls == [] and all(v["cached"] for v in again.values())
    assert A.get_tuning(8)[1] == 8


def test_cache_key_buckets_point_counts():
    assert A.cache_key("d", 8, 65536) == A.cache_key("d", 8, 70000) == "d|K8|P65536"
    assert A.cache_key("d", 8, 65536) != A.cache_key("d", 8, 131072)
    assert A.cache_key("d", 8, 0) == "d|K8|P1"


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert A.load_cache(str(path)) == {}
