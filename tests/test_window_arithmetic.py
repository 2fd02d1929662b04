"""CPU checks of the exactness claims behind the stream kernels' LDS window
test, in the two precisions the kernels use (IEEE arithmetic is the same on
the host).  The kernels classify a nodal cell coordinate x = (k + L) / dk
against a window [r0, r0 + W) of the histogram grid by x - r0, without the
floor, and take the window cell by truncating x - r0.  That is the same as
floor(x) - r0 in [0, W) and its value, because for x >= r0 >= 0 (r0 an
integer) the difference is exact, and for x < r0 it is negative."""
import numpy as np
import pytest


def _window_by_offset(x, r0, w, dtype):
    d = (x - dtype(r0)).astype(dtype)              # one rounded subtraction
    inside = (d >= 0) & (d < dtype(w))
    return inside, np.trunc(d)


def _window_by_floor(x, r0, w, dtype):
    f = np.floor(x) - dtype(r0)
    inside = (f >= 0) & (f < dtype(w))
    return inside, f


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_offset_test_equals_floor_test(dtype):
    rng = np.random.default_rng(11)
    nk = 256
    for w in (2, 58, 80, 120, 256):
        r0 = (nk - w) // 2
        # coordinates spread over the grid and beyond it, dense near every
        # integer (the cell edges), including the edges themselves
        edges = np.arange(-4, nk + 4, dtype=np.float64)
        near = edges[:, None] + np.array([-1e-9, -1e-12, 0.0, 1e-12, 1e-9])[None, :]
        x = np.concatenate([rng.uniform(-10, nk + 10, 200_000), near.ravel(),
                            np.nextafter(edges, -np.inf), np.nextafter(edges, np.inf)])
        x = x.astype(dtype)
        a_in, a_cell = _window_by_offset(x, r0, w, dtype)
        b_in, b_cell = _window_by_floor(x, r0, w, dtype)
        assert np.array_equal(a_in, b_in), (w, dtype)
        assert np.array_equal(a_cell[a_in], b_cell[b_in]), (w, dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_offset_is_exact_past_the_origin(dtype):
    rng = np.random.default_rng(12)
    r0 = np.arange(0, 200, 7)
    x = rng.uniform(0, 300, 100_000).astype(dtype)
    for r in r0:
        sel = x >= dtype(r)
        d = (x[sel] - dtype(r)).astype(dtype)
        # exact: adding r back recovers x, and the wide difference agrees
        assert np.array_equal((d.astype(np.float64) + r), x[sel].astype(np.float64))


def test_nan_and_huge_fall_outside():
    for dtype in (np.float64, np.float32):
        x = np.array([np.nan, np.inf, -np.inf, 1e30, -1e30], dtype=dtype)
        inside, _ = _window_by_offset(x, 88, 80, dtype)
        assert not inside.any()
