"""Host-side pieces of the warm-start driver (no GPU)."""
import numpy as np
import pytest

from paper_2503_13802_amd import warmstart


def test_cosine_schedule_end_points_and_monotone():
    lr = [warmstart.learning_rate(j, 100, 1e-3, 1e-5) for j in range(100)]
    assert lr[0] == pytest.approx(1e-3) and lr[-1] == pytest.approx(1e-5)
    assert all(a >= b for a, b in zip(lr, lr[1:]))
    assert lr[49] == pytest.approx(0.5 * (1e-3 + 1e-5), rel=2e-2)
    assert warmstart.learning_rate(7, 100, 2e-3) == 2e-3


def test_crop_origin_in_range_and_deterministic():
    for seed in range(50):
        o = warmstart.crop_origin(seed, (128, 128, 96), (64, 64, 64))
        assert all(0 <= a <= n - 64 for a, n in zip(o, (128, 128, 96)))
        assert o == warmstart.crop_origin(seed, (128, 128, 96), (64, 64, 64))
    assert warmstart.crop_origin(3, (64, 64, 64), (64, 64, 64)) == [0, 0, 0]


def test_snr_draw_range():
    v = np.array([warmstart.sample_snr2(s) for s in range(500)])
    assert v.min() >= 20.0 and v.max() < 40.0
    assert abs(v.mean() - 30.0) < 1.0
