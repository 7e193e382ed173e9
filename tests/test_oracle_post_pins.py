"""Pins of the oracle's polar-image epilogue (Sec. III-B "Polar Image",
Sec. III-C "Noise"): the dB map and 8-bit quantisation against closed forms,
the range blur against scipy's Gaussian filter, the uniform noise against
numpy's Philox, and the gradient noise against its defining properties
(zero at lattice points, gradient there equal to the lattice vector, C1 across
cell borders, bounded range)."""
import math

import numpy as np
import pytest
from scipy import ndimage

from test_oracle_pins import numpy_philox

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

GRADS = [(1, 1), (-1, 1), (1, -1), (-1, -1), (1, 0), (-1, 0), (0, 1), (0, -1)]


def energy(out, floor=-100.0, top=255):
    """Energy after blur and noise, recovered in float64 from the unrounded
    pixel value (the float32 dB output carries only ~5e-7 relative)."""
    pre = out[2]
    L = pre * (0.0 - floor) / top + floor
    return np.where(np.isfinite(pre), 10.0 ** (L / 10.0), 0.0)


def test_db_and_pixel_closed_forms(orc):
    vals = np.array([[1.0, 0.1, 1e-5, 1e-10, 0.0, 2.0, 1e-12, 0.5]], np.float32)
    db, u8, pre = orc.postprocess(vals, dict(db_floor=-100.0, max_value=255))
    assert db[0, 0] == 0.0
    assert db[0, 1] == pytest.approx(-10.0, abs=1e-5)
    assert db[0, 2] == pytest.approx(-50.0, abs=1e-5)
    assert db[0, 3] == pytest.approx(-100.0, abs=1e-5)
    assert db[0, 4] == -np.inf
    assert db[0, 5] == pytest.approx(10 * math.log10(2.0), abs=1e-6)
    assert db[0, 7] == pytest.approx(10 * math.log10(0.5), abs=1e-6)
    # 255 at 0 dB, 0 at the floor and below, linear in dB between, cut at 0 dB
    # (float32(0.1) lies just above 0.1 and float32(1e-5) just below 1e-5, so
    # the two half-way pixels round to opposite sides)
    assert list(u8[0]) == [255, 230, 127, 0, 0, 255, 0, round(255 * (1 - 10 * math.log10(2) / 100))]
    assert 229.5 < pre[0, 1] < 229.5 + 1e-6 and 127.5 - 1e-5 < pre[0, 2] < 127.5


def test_db_against_numpy_log10(orc):
    rng = np.random.default_rng(5)
    img = (10.0 ** rng.uniform(-14, 0.5, (7, 300))).astype(np.float32)
    img[rng.random(img.shape) < 0.1] = 0.0
    for floor, top in ((-100.0, 255), (-60.0, 200), (-30.0, 1)):
        db, u8, pre = orc.postprocess(img, dict(db_floor=floor, max_value=top))
        want = np.where(img > 0, 10.0 * np.log10(img.astype(np.float64)), -np.inf)
        assert np.array_equal(db, want.astype(np.float32))
        scaled = top * (want - floor) / (0.0 - floor)
        assert np.allclose(pre[img > 0], scaled[img > 0], rtol=1e-13, atol=1e-12)
        q = np.clip(np.floor(scaled + 0.5), 0, top)
        assert np.array_equal(u8, np.where(img > 0, q, 0).astype(np.uint8))


@pytest.mark.parametrize("sigma", [0.5, 1.0, 1.5, 2.0, 4.0, 7.5])
def test_blur_matches_scipy_gaussian_filter(orc, sigma):
    rng = np.random.default_rng(int(sigma * 10))
    img = rng.random((5, 257)).astype(np.float32) * (rng.random((5, 257)) < 0.2)
    img[2, 0] = 1.0
    img[3, 256] = 1.0
    out = orc.postprocess(img, dict(blur_sigma_bins=sigma))
    # scipy's radius int(truncate * sigma + 0.5) equals ceil(3 sigma) for these sigmas
    ref = ndimage.gaussian_filter1d(img.astype(np.float64), sigma, axis=1, mode="constant", cval=0.0,
                                    truncate=3.0)
    ref[ref < 1e-300] = 0.0
    assert np.allclose(energy(out), ref, rtol=1e-11, atol=1e-300)


def test_blur_conserves_energy_and_keeps_identity(orc):
    img = np.zeros((3, 200), np.float32)
    img[0, 100] = 1.0
    img[1, 50] = 0.25
    img[1, 120] = 0.5
    e = energy(orc.postprocess(img, dict(blur_sigma_bins=3.0)))
    assert e[0].sum() == pytest.approx(1.0, rel=1e-12)
    assert e[1].sum() == pytest.approx(0.75, rel=1e-12)
    assert np.argmax(e[0]) == 100 and e[0, 100 - 9] > 0 and e[0, 100 - 10] == 0 and e[0, 110] == 0
    assert np.allclose(e[0, 100 - 9:100], e[0, 101:110][::-1], rtol=1e-12)
    assert np.array_equal(energy(orc.postprocess(img, dict(blur_sigma_bins=0.0))).astype(np.float32), img)


def test_uniform_noise_from_numpy_philox(orc):
    seed, scan, amp = 0xABCDEF, 3, 2.0 ** -10  # amplitudes exact in float32
    img = np.zeros((6, 40), np.float32)
    out = orc.postprocess(img, dict(uniform_amp=amp, seed=seed, scan_id=scan, blur_sigma_bins=2.0))
    for k in range(6):
        for b in range(0, 40, 3):
            x = numpy_philox((seed, scan), (k, b // 4, 1, 0))[b % 4]
            want = amp * (x >> 11) * 2.0 ** -53
            # the noise is added after the blur: a zero image stays a noise floor
            assert energy(out)[k, b] == pytest.approx(want, rel=1e-12)
    out2 = orc.postprocess(img, dict(uniform_amp=amp, seed=seed, scan_id=scan + 1))
    assert not np.array_equal(out[2], out2[2])
    big = np.zeros((64, 512), np.float32)
    e = energy(orc.postprocess(big, dict(uniform_amp=1.0, seed=1)))
    assert e.max() < 1.0 and e.min() >= 0.0
    assert abs(e.mean() - 0.5) < 0.005 and abs(e.var() - 1 / 12) < 0.003


def _grad(key, i, j):
    return GRADS[numpy_philox(key, (i % 2**64, j % 2**64, 2, 0))[0] >> 61]


def test_perlin_zero_at_lattice_and_gradient_there(orc):
    seed, scan = 77, 1
    h = 1e-6
    for i in range(-3, 6):
        for j in range(0, 9, 2):
            assert orc.perlin(seed, scan, i, j) == 0.0
            gx = (orc.perlin(seed, scan, i + h, j) - orc.perlin(seed, scan, i - h, j)) / (2 * h)
            gy = (orc.perlin(seed, scan, i, j + h) - orc.perlin(seed, scan, i, j - h)) / (2 * h)
            want = _grad((seed, scan), i, j)
            assert gx == pytest.approx(want[0], abs=1e-6) and gy == pytest.approx(want[1], abs=1e-6)


def test_perlin_cell_centre_and_edges(orc):
    seed, scan = 9, 0
    key = (seed, scan)
    for i, j in ((0, 0), (4, 7), (-2, 3)):
        g = [_grad(key, i + a, j + b) for a, b in ((0, 0), (1, 0), (0, 1), (1, 1))]
        off = [(0.5, 0.5), (-0.5, 0.5), (0.5, -0.5), (-0.5, -0.5)]
        # the fade is 1/2 at the centre: the mean of the four corner terms
        want = sum(gg[0] * o[0] + gg[1] * o[1] for gg, o in zip(g, off)) / 4
        assert orc.perlin(seed, scan, i + 0.5, j + 0.5) == pytest.approx(want, abs=1e-15)
        # on the edge y = j the noise depends on the two lower corners only
        t = 0.3
        f = t ** 3 * (t * (6 * t - 15) + 10)
        want = g[0][0] * t + f * (g[1][0] * (t - 1) - g[0][0] * t)
        assert orc.perlin(seed, scan, i + t, j) == pytest.approx(want, abs=1e-15)


def test_perlin_range_and_smoothness(orc):
    rng = np.random.default_rng(3)
    pts = rng.uniform(-20, 20, (4000, 2))
    v = np.array([orc.perlin(5, 2, x, y) for x, y in pts])
    assert v.min() >= -1.0 and v.max() <= 1.0 and abs(v.mean()) < 0.05 and v.std() > 0.1
    # first derivative continuous across a cell border
    h = 1e-5
    for x in (1.0, -3.0, 7.0):
        for y in (0.3, 2.7):
            left = (orc.perlin(5, 2, x, y) - orc.perlin(5, 2, x - h, y)) / h
            right = (orc.perlin(5, 2, x + h, y) - orc.perlin(5, 2, x, y)) / h
            assert left == pytest.approx(right, abs=1e-4)


def test_perlin_image_noise(orc):
    img = np.zeros((40, 300), np.float32)
    post = dict(perlin_amp=2.0 ** -7, perlin_cell_az=8.0, perlin_cell_bins=32.0, seed=11, scan_id=4)
    e = energy(orc.postprocess(img, post))
    for k, b in ((0, 0), (8, 64), (16, 96), (5, 13), (39, 299)):
        n = orc.perlin(11, 4, k / 8.0, b / 32.0)
        assert e[k, b] == pytest.approx(2.0 ** -7 * (0.5 + 0.5 * n), rel=1e-12)
    assert np.allclose(e[::8, ::32], 2.0 ** -8, rtol=1e-12)
