"""Pins of the SSIM oracle (oracle/ssim.py): scipy's correlation with the same
window, identities, constant-image closed form, finite differences."""
import numpy as np
from scipy import ndimage

from oracle import ssim as Q


def rand_img(seed, shape=(3, 13, 17)):
    return np.random.default_rng(seed).uniform(0, 1, size=shape)


def test_window_is_normalised_separable_gaussian():
    w = Q.window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    g = w.sum(axis=1)
    np.testing.assert_allclose(w, np.outer(g, g), rtol=1e-14)
    np.testing.assert_allclose(g[5 + 1] / g[5], np.exp(-1 / (2 * 1.5 ** 2)), rtol=1e-14)


def test_window_sums_match_scipy_correlate():
    x = rand_img(0)
    w = Q.window()
    ref = np.stack([ndimage.correlate(x[c], w, mode="constant", cval=0.0) for c in range(3)])
    np.testing.assert_allclose(Q._window_sums(x, w), ref, rtol=1e-12, atol=1e-14)


def test_ssim_map_matches_scipy_formulation():
    x, y = rand_img(1), rand_img(2)
    w = Q.window()
    f = lambda a: np.stack([ndimage.correlate(a[c], w, mode="constant", cval=0.0) for c in range(3)])
    mx, my = f(x), f(y)
    vx, vy, cxy = f(x * x) - mx ** 2, f(y * y) - my ** 2, f(x * y) - mx * my
    S = (2 * mx * my + Q.C1) * (2 * cxy + Q.C2) / ((mx ** 2 + my ** 2 + Q.C1) * (vx + vy + Q.C2))
    np.testing.assert_allclose(Q.ssim_terms(x, y)["S"], S, rtol=1e-11)


def test_identical_images_give_one():
    x = rand_img(3)
    assert abs(Q.ssim(x, x) - 1.0) < 1e-14
    loss, g = Q.dssim_grad(x, x)
    assert abs(loss) < 1e-14 and np.abs(g).max() < 1e-12


def test_constant_images_closed_form():
    a, b = 0.3, 0.7
    x, y = np.full((1, 30, 30), a), np.full((1, 30, 30), b)
    S = Q.ssim_terms(x, y)["S"]
    inner = S[0, 5:25, 5:25]  # windows inside the image: no variance
    np.testing.assert_allclose(inner, (2 * a * b + Q.C1) / (a * a + b * b + Q.C1), rtol=1e-12)


def test_gradient_by_finite_differences():
    x, y = rand_img(4, (2, 9, 12)), rand_img(5, (2, 9, 12))
    _, g = Q.dssim_grad(x, y)
    h = 1e-6
    rng = np.random.default_rng(6)
    for _ in range(30):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = ((1 - Q.ssim(xp, y)) - (1 - Q.ssim(xm, y))) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(fd)), (idx, fd, g[idx])


def test_photometric_combines_terms():
    x, y = rand_img(7), rand_img(8)
    l0, g0 = Q.photometric(x, y, 0.0)
    np.testing.assert_allclose(l0, np.abs(x - y).mean(), rtol=1e-14)
    np.testing.assert_allclose(g0, np.sign(x - y) / x.size, rtol=1e-14)
    l1, g1 = Q.photometric(x, y, 1.0)
    d, gd = Q.dssim_grad(x, y)
    np.testing.assert_allclose(l1, d, rtol=1e-14)
    np.testing.assert_allclose(g1, gd, rtol=1e-14)
