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
    g = PR.grid(400, 64, 20.0)
    assert set(g) == {(a, b) for a in (200, 400, 800, 1600) for b in (32, 64, 96)}
    g = PR.grid(400, 64, 30.0)           # 1.2 n_hat = 36 > 32: no smaller subspace
    assert set(g) == {(a, b) for a in (200, 400, 800, 1600) for b in (64, 96)}
    g = PR.grid(30, 512, 200.0)
    assert all(50 <= a <= 20000 and b <= 512 for a, b in g) and (50, 512) in g and (120, 480) in g
    assert len(g) == 2 * 3


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


def test_targets_invert_through_choose_params():
    """A label, turned into the network's targets and standardised, comes back
    out of the parameter rule (oracle reading) as the same (n_p, n_s)."""
    import oracle as O
    rows = []
    for n_p, n_s, a, b, cnt in ((800, 96, -0.02, 0.03, 37.0), (1600, 64, -0.011, 0.009, 20.5),
                                (400, 128, -0.05, 0.05, 0.4)):
        f = np.zeros(258, dtype=np.float32)
        f[256], f[257] = a, b
        rows.append(dict(features=f.tolist(), label=(n_p, n_s), count_est=cnt))
    T = PR.targets(rows)
    f32 = lambda v: float(np.float32(v))  # noqa: E731  features are stored as FP32
    assert np.allclose(T[:, 0], [800 * (f32(0.03) - f32(-0.02)) / 2, 1600 * (f32(0.009) - f32(-0.011)) / 2,
                                 400 * (f32(0.05) - f32(-0.05)) / 2])
    assert np.allclose(T[:, 1], [96 / 74.0, 64 / 41.0, 128 / 32.0])
    z, mean, std = PR.standardise(T)
    for r, zz in zip(rows, z):
        a, b = r["features"][256], r["features"][257]
        assert O.choose_params(a, b, r["count_est"], 32, mlp_out=zz, t_mean=mean, t_std=std) == tuple(r["label"])
    assert PR.kappa_from_corpus(rows) == np.median(T[:, 0])


def test_adaptive_search_stops():
    # doubling while nothing converged, up to the cap
    assert PR.next_adaptive_np(100, [0], 800) == 200
    assert PR.next_adaptive_np(400, [0, 0, 0], 800) == 800
    assert PR.next_adaptive_np(800, [0, 0, 0, 0], 800) is None
    # pairs found but not converged: keep doubling while the count grows
    assert PR.next_adaptive_np(200, [0, 12], 1600) == 400
    assert PR.next_adaptive_np(400, [0, 12, 20], 1600) == 800
    # a doubling that found no more pairs ends the search
    assert PR.next_adaptive_np(800, [0, 20, 20], 1600) is None


def test_target_range_is_the_span_of_the_log_targets():
    T = np.array([[10.0, 1.0], [20.0, 2.5], [5.0, 1.2]])
    lo, hi = PR.target_range(T)
    assert np.allclose(lo, np.log([5.0, 1.0])) and np.allclose(hi, np.log([20.0, 2.5]))
