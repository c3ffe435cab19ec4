"""The seeded input generators are deterministic and have the stated shape."""
import numpy as np

from paper_1907_10526_amd import phantoms, workloads


def test_phantoms_are_deterministic():
    a = workloads.phantom(workloads.SMALL)
    b = workloads.phantom(workloads.SMALL)
    assert a.dtype == np.float32 and a.shape == (64, 64)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, workloads.phantom(workloads.SMALL, seed=99))
    y = phantoms.uniform((3, 4), 11)
    assert np.array_equal(y, phantoms.uniform((3, 4), 11))
    assert y.min() >= -1 and y.max() <= 1


def test_ellipse_parameters_follow_recipe():
    p = phantoms.ellipse_params(512, 2000, 2, (32.0, 160.0))
    r = np.hypot(p[:, 0], p[:, 1])
    assert r.max() <= 256.0
    assert p[:, 2].min() >= 32 and p[:, 3].max() <= 160
    assert p[:, 4].min() >= 0 and p[:, 4].max() < np.pi
    assert p[:, 5].min() >= -0.5 and p[:, 5].max() <= 1.0


def test_disk_area_weighted():
    d = phantoms.disk(64, 24.0)
    assert abs(float(d.sum()) - np.pi * 24.0 ** 2) < 1.0
    assert d[32, 32] == 1.0 and d[0, 0] == 0.0


def test_poisson_sinogram():
    clean = np.full((4, 5), 0.5)
    y = phantoms.poisson_log_sinogram(clean, 1e5, 33)
    assert np.array_equal(y, phantoms.poisson_log_sinogram(clean, 1e5, 33))
    assert abs(float(y.mean()) - 0.5) < 0.02
