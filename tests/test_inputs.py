"""The seeded synthetic-input generator: determinism, structure, value ranges."""
import numpy as np
import pytest

import sdnn_inputs as gen


def test_pattern_is_deterministic_distinct_sorted():
    a, _ = gen.layer_pattern(7, 3, 256)
    b, _ = gen.layer_pattern(7, 3, 256)
    c, _ = gen.layer_pattern(7, 4, 256)
    assert a.dtype == np.int32 and a.shape == (256, 32)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert (np.diff(a, axis=1) > 0).all()          # strictly ascending => distinct
    assert a.min() >= 0 and a.max() < 256


def test_pattern_small_n_forces_redraws():
    idx, _ = gen.layer_pattern(1, 0, 40)            # 32 of 40: duplicates almost surely drawn first
    assert (np.diff(idx, axis=1) > 0).all()


def test_weight_kinds():
    cfg = gen.CONFIGS["C5"]
    _, w, b = gen.make_layer(cfg.with_(n_neurons=512), 0)
    assert w.dtype == np.float32 and w.min() >= 0.03 and w.max() <= 0.09
    assert (b == np.float32(-0.3)).all()
    _, w, _ = gen.make_layer(gen.CONFIGS["C1"], 0)
    assert (w == np.float32(1 / 16)).all()
    _, w, _ = gen.make_layer(gen.CONFIGS["G5"].with_(n_neurons=2048), 0)
    assert abs(float(w.std()) - 0.25) < 0.01 and abs(float(w.mean())) < 0.01


def test_inputs_binary_density_and_ranges():
    cfg = gen.CONFIGS["C1"]
    x = gen.make_inputs(cfg)
    assert x.dtype == np.float32 and x.shape == (1000, 1024)
    assert set(np.unique(x)) <= {0.0, 1.0}
    assert abs(float(x.mean()) - 0.2) < 0.003
    # any row range is reproducible on its own
    assert np.array_equal(gen.make_inputs(cfg, 123, 456, chunk=50), x[123:456])


def test_row_density_companion():
    cfg = gen.CONFIGS["S2"].with_(rows=400, n_neurons=1024)
    x = gen.make_inputs(cfg)
    d = x.mean(axis=1)
    assert d.min() > 0.05 and d.max() < 0.56 and d.std() > 0.08


@pytest.mark.parametrize("name", ["C3", "C4"])
def test_batches_cover_rows_within_bounds(name):
    cfg = gen.CONFIGS[name]
    off = gen.make_batches(cfg)
    sizes = np.diff(off)
    assert off[0] == 0 and off[-1] == cfg.rows and len(sizes) == cfg.n_batches
    assert sizes.min() >= cfg.batch_lo and sizes.max() <= cfg.batch_hi
    assert np.array_equal(off, gen.make_batches(cfg))


def test_teacher_perturbation():
    cfg = gen.CONFIGS["C5"]
    w = np.full((4096, 32), 0.06, np.float32)
    t = gen.teacher_weights(cfg, w, 3)
    d = t.astype(np.float64) - w
    assert abs(float(d.std()) - 0.005) < 2e-4 and t.dtype == np.float32
