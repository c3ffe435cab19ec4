"""The Python binding's shape checks, on the host: a tensor of the wrong
shape never reaches the C ABI (whose plain pointers carry no sizes)."""
import pytest
import torch


@pytest.fixture(scope="module")
def geom():
    from paper_1907_10526_amd import fanproj
    g = fanproj.Geometry.__new__(fanproj.Geometry)   # shape logic only, no device
    g.nx, g.ny, g.n_views, g.n_det = 5, 4, 3, 7
    g.handle = None
    return g


def test_batch_shapes(geom):
    assert geom._batch(torch.zeros(4, 5), (4, 5), "image") == 1
    assert geom._batch(torch.zeros(6, 4, 5), (4, 5), "image") == 6
    for bad in [(4, 6), (5, 4), (2, 3, 4, 5), (5,)]:
        with pytest.raises(ValueError):
            geom._batch(torch.zeros(bad), (4, 5), "image")


def test_output_shapes(geom):
    img = torch.zeros(6, 4, 5)
    out = geom._output(None, img, 6, (3, 7), torch.float32, "out")
    assert tuple(out.shape) == (6, 3, 7)
    assert geom._output(torch.zeros(6, 3, 7), img, 6, (3, 7), torch.float32, "out").shape == (6, 3, 7)
    single = torch.zeros(4, 5)
    assert geom._output(torch.zeros(3, 7), single, 1, (3, 7), torch.float32, "out").shape == (3, 7)
    for bad in [(5, 3, 7), (6, 3, 8), (3, 7)]:
        with pytest.raises(ValueError):
            geom._output(torch.zeros(bad), img, 6, (3, 7), torch.float32, "out")
