"""Every compiled lane variant of the Gauss-point kernel against the oracle,
the persistent loop with few waves, and the autotuner on a mixed batch.

Tuning changes only which lanes hold which laminates and how many persistent
waves run, never the per-point arithmetic, so every variant meets the same
1e-10 bar against the FP64 oracle and agrees with the default variant."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synthetic as S
from test_gpu_parity import compare_paths, gpu_path, say

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(autouse=True)
def default_table():
    from paper_2103_08253_amd import autotune as A
    A.reset_tuning()
    yield
    A.reset_tuning()


@pytest.mark.parametrize("K", [2, 3, 4, 5, 6, 7, 8])
def test_lane_variants_match_oracle(K):
    from paper_2103_08253_amd import autotune as A
    dev()
    rs = S.streams(100 + K)
    net = S.random_dmn(rs["dmn"], K, 0.25)
    E = S.ramp_with_noise(rs, 37, 4, 0.02, 1e-3)
    for lanes in A.lane_variants(K):
        for waves in (0, 1):
            say(f"case: depth {K}, {lanes} lanes per point, waves per CU {waves or 'default'}")
            A.set_tuning(K, lanes, waves)
            gpu = gpu_path(net, E)
            compare_paths(net, E, range(37), gpu)


def test_persistent_loop_many_batches_per_wave():
    """One wave per CU over 6,000 depth-5 points: each wave takes several
    batches from the work counter; results equal the default launch."""
    from paper_2103_08253_amd import autotune as A
    say("case: depth 5, 6000 points, 8 lanes per point, 1 wave per CU vs default")
    dev()
    rs = S.streams(205)
    net = S.random_dmn(rs["dmn"], 5, 0.3)
    E = S.ramp_with_noise(rs, 6000, 3, 0.02, 1e-3)
    ref = gpu_path(net, E)
    A.set_tuning(5, 8, 1)
    got = gpu_path(net, E)
    for r, g in zip(ref, got):
        assert np.array_equal(r["status"], g["status"]) and np.array_equal(r["iters"], g["iters"])
        for k in ("sigma", "C", "z", "a"):
            scale = np.abs(r[k]).max()
            assert np.abs(r[k] - g[k]).max() <= 1e-12 * scale, k


def test_autotuner_on_mixed_batch(tmp_path):
    """Tune a 16-DMN mixed-depth batch, then check the tuned launch against the
    default one and the cache file."""
    import json
    from paper_2103_08253_amd import PointGroup, autotune as A, dmn_update_gauss_points
    say("case: autotune 16 mixed-depth groups, 4096 points")
    d = dev()
    wl = S.config2(n_points=4096, n_steps=2)
    groups = []
    for m, net in enumerate(wl.nets):
        sel = np.nonzero(wl.dmn_id == m)[0]
        groups.append(PointGroup.allocate(torch.tensor(net.w, device=d),
                                          torch.tensor(net.normals, device=d),
                                          torch.tensor(wl.E[1, sel], device=d)))
    dmn_update_gauss_points(groups, S.FIBER, S.MATRIX)
    ref = [(g.sigma.clone(), g.tangent.clone(), g.z_out.clone(), g.iters.clone()) for g in groups]
    path = str(tmp_path / "tune.json")
    chosen = A.tune_gauss_points(groups, S.FIBER, S.MATRIX, cache_path=path, reps=1,
                                 waves=(4, 8))
    say("  chosen: " + ", ".join(f"K{k}: {v['lanes_per_point']} lanes, {v['waves_per_cu']} "
                                 f"waves/CU, {v['ms']:.3f} ms" for k, v in sorted(chosen.items())))
    assert sorted(chosen) == [5, 6, 7, 8, 9]
    for K, v in chosen.items():
        assert A.get_tuning(K) == (v["lanes_per_point"], v["waves_per_cu"])
        assert v["launch"] == "mixed"
    assert len({v["waves_per_cu"] for v in chosen.values()}) == 1
    assert len(json.load(open(path))) == 1  # one entry: the mixed launch
    for g in groups:
        g.sigma.fill_(np.nan)
    dmn_update_gauss_points(groups, S.FIBER, S.MATRIX)
    for g, (s, C, z, it) in zip(groups, ref):
        assert torch.equal(g.iters, it)
        for a, b in ((g.sigma, s), (g.tangent, C), (g.z_out, z)):
            assert (a - b).abs().max().item() <= 1e-12 * b.abs().max().item()
    again = A.tune_gauss_points(groups, S.FIBER, S.MATRIX, cache_path=path)
    assert all(v["cached"] for v in again.values())
