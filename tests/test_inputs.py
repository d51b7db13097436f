"""Seeded input generators: determinism and the bounding-box phantom shortcut."""
import math

import numpy as np
import pytest

import inputs


@pytest.mark.parametrize("n,e,seed", [(64, 10, 0), (96, 7, 11), (256, 30, 4000), (512, 20, 1000)])
def test_bounding_box_phantom_equals_full_grid(n, e, seed):
    assert np.array_equal(inputs.ellipse_phantom(n, e, seed),
                          inputs._ellipse_phantom_full_grid(n, e, seed))


def test_ellipse_parameters_within_ranges():
    p = inputs.ellipse_params(500, inputs.rng(1))
    r = np.hypot(p[:, 0], p[:, 1])
    assert np.all(r <= 0.8) and np.all((0.05 <= p[:, 2]) & (p[:, 2] <= 0.4))
    assert np.all((0.05 <= p[:, 3]) & (p[:, 3] <= 0.4))
    assert np.all((0.0 <= p[:, 4]) & (p[:, 4] < math.pi))
    assert np.all((0.1 <= p[:, 5]) & (p[:, 5] <= 1.0))


def test_single_disk_area():
    """One ellipse of known area: pixel count x h^2 approaches pi a b."""
    n = 512
    img = inputs.ellipse_phantom(n, 1, 7)
    cx, cy, a, b, rot, val = inputs.ellipse_params(1, inputs.rng(7))[0]
    area = (img > 0).sum() * (2.0 / n) ** 2
    assert abs(area - math.pi * a * b) < 4 * 2.0 * math.pi * max(a, b) * (2.0 / n)
    assert np.allclose(img[img > 0], val)


def test_workload_mixes_are_seeded():
    assert inputs.batch_mix(16) == inputs.batch_mix(16)
    mix = inputs.batch_mix(256)
    assert {r.side for r in mix} <= {128, 256, 512, 1024}
    assert {r.n_angles for r in mix} <= {90, 180, 360, 720}
    assert all(r.n_bins == math.ceil(r.side * math.sqrt(2.0)) for r in mix)
    s = inputs.serving_mix(400, 20.0)
    assert all(b.arrival_s > a.arrival_s for a, b in zip(s, s[1:]))
    assert all(r.side // 2 <= r.n_angles <= (3 * r.side) // 2 for r in s)
    assert {r.tol for r in s} <= {1e-2, 1e-3}
    # mean inter-arrival close to 1/rate
    assert abs(s[-1].arrival_s / len(s) - 1 / 20.0) < 0.2 / 20.0


def test_uniform_noise_is_seeded_and_in_open_interval():
    a = inputs.uniform_noise(100000, 12)
    assert np.array_equal(a, inputs.uniform_noise(100000, 12))
    assert not np.array_equal(a, inputs.uniform_noise(100000, 13))
    assert a.min() > -1.0 and a.max() < 1.0
    assert abs(a.mean()) < 0.01 and abs(a.var() - 1.0 / 3.0) < 0.01
