"""Host-side logic of the parameter predictor pipeline (no GPU): instance
sampling ranges, the label grid, standardisation and the evaluation summary."""
import numpy as np

from paper_1803_02156_amd import predictor as PR


def test_sampled_instances_cover_the_stated_ranges():
    rng = np.random.default_rng(0)
    insts = [PR.sample_instance(rng, 16, 48, k) for k in range(400)]
    dims = np.array([i.dims for i in insts])
    assert dims.min() >= 16 and dims.max() <= 48
    assert len({i.dims for i in insts}) > 300                 # random aspect ratios
    for key, lo, hi in (("m", 0.5, 2.5), ("W", 0.0, 3.0), ("half_width", 0.01, 0.1)):
        v = np.array([getattr(i, key) for i in insts])
        assert v.min() >= lo and v.max() <= hi and v.max() - v.min() > 0.8 * (hi - lo)


def test_grid_is_clamped_and_contains_the_heuristic():
    g = PR.grid(400, 64)
    assert (400, 64) in g and (800, 96) in g and (1600, 64) in g and (3200, 96) in g and len(g) == 8
    g = PR.grid(30, 512)
    assert all(50 <= a <= 20000 and b <= 512 for a, b in g) and (50, 512) in g and (240, 512) in g


def test_standardise_round_trip():
    lab = np.array([[100, 32], [400, 64], [1600, 96]], dtype=float)
    z, mean, std = PR.standardise(lab)
    assert np.allclose(z.mean(axis=0), 0.0) and np.allclose(z.std(axis=0), 1.0)
    assert np.allclose(np.exp(z * std + mean), lab)


def test_work_units_and_summary():
    assert PR.work_units(10, 130, 100, 32, 2) == 2 * (100 * 32 * 13 * 10 + PR.C_ORTH * 10 * 32 * 32)
    ev = [dict(heuristic=dict(failed=False, iters=3, seconds=2.0, work=10.0),
               mlp=dict(failed=False, iters=2, seconds=1.0, work=5.0)),
          dict(heuristic=dict(failed=True, iters=12, seconds=9.0, work=50.0),
               mlp=dict(failed=False, iters=3, seconds=1.5, work=6.0))]
    s = PR.summarise(ev)
    assert s["heuristic"]["failures"] == 1 and s["mlp"]["failures"] == 0
    assert s["work_ratio_mlp_over_heuristic"]["mean"] == 0.5
    assert s["mlp"]["mean_iters"] == 2.5
