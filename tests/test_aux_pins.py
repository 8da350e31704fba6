"""Pins of the oracle's loss masks and auxiliary outputs (Sec. 4: the 360Roam
evaluation leaves the images' bottom rows out of the loss; depth and alpha
images come from the same blend as the colour).

* A row crop (render only the top rows) is the restriction of the full render
  and of its backward.
* The depth image D = sum d_i alpha_i T_i: closed forms for one and two
  Gaussians on a pixel, equality with the colour channel of a scene whose
  colours are set to the depths, the brute-force renderer, and finite
  differences of <G_D, D> + <G_A, 1 - T_final>.
* The masked photometric loss: a mask of ones, scale invariance, the L1 of
  cropped images, finite differences.
CPU only.
"""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from oracle import ssim as Q
from paper_2404_03202_amd import scenes

Y00 = 0.5 / np.sqrt(np.pi)


def _single(means, scales=0.02, opac=0.9, dc=(0.3, 0.4, 0.5), sh_degree=0):
    means = np.atleast_2d(np.asarray(means, dtype=np.float64))
    n = means.shape[0]
    sh = np.zeros((n, 16, 3))
    sh[:, 0, :] = np.broadcast_to(np.asarray(dc, dtype=np.float64), (n, 3))
    return dict(means=means, scales=np.full((n, 3), scales, np.float64), quats=np.tile([1.0, 0, 0, 0], (n, 1)),
                opacities=np.broadcast_to(np.asarray(opac, np.float64), (n,)).copy(), sh=sh, sh_degree=sh_degree)


CAMS = {
    "erp": lambda rows=0: dict(scenes.camera(96, 48, scenes.rot_y(0.5).T, [0.1, 0.0, -0.2]), rows=rows),
    "pinhole": lambda rows=0: dict(scenes.pinhole_camera(88, 60, 90.0, scenes.rot_y(0.5).T, [0.1, 0.0, -0.2]),
                                   rows=rows),
}


# ----------------------------------------------------------------- row crop
@pytest.mark.parametrize("model", sorted(CAMS))
@pytest.mark.parametrize("rows", [1, 16, 37])
def test_row_crop_is_restriction(model, rows):
    """Rendering the top rows only gives exactly those rows of the full
    render (the mapping still uses the full height), and the backward of a
    cotangent on the crop equals the full backward of that cotangent padded
    with zeros."""
    g = scenes.shell_scene(110, 400, r0=1.0, r1=5.0, scale_lo=0.02, scale_hi=0.4)
    full = O.Scene(g, CAMS[model]())
    crop = O.Scene(g, CAMS[model](rows))
    assert crop.out_height == rows and crop.tiles_y == (rows + 15) // 16
    rf, rc = O.render(full, alt=False), O.render(crop, alt=False)
    # (n_contrib is a position in the tile's list, whose content differs)
    for k in ("image", "final_T", "n_blended", "depth"):
        np.testing.assert_array_equal(rc[k], rf[k][..., :rows, :], err_msg=k)
    rng = np.random.default_rng(rows)
    G = rng.normal(size=(3, rows, full.width))
    Gf = np.zeros((3, full.height, full.width))
    Gf[:, :rows] = G
    bc, bf = O.backward(crop, G, with_abs=False), O.backward(full, Gf, with_abs=False)
    for k in ("means", "scales", "quats", "opacities", "sh", "screen"):
        np.testing.assert_allclose(bc[k], bf[k], rtol=1e-12, atol=1e-15, err_msg=k)


# ------------------------------------------------------------- depth image
@pytest.mark.parametrize("model", sorted(CAMS))
def test_depth_closed_forms(model):
    """A Gaussian centred on a pixel contributes alpha = o there: D = d o,
    A = o.  Two on the same pixel, d1 < d2: D = d1 o1 + d2 o2 (1 - o1),
    A = 1 - (1 - o1)(1 - o2); d is t_r (ERP) or t_z (pinhole)."""
    cam = CAMS[model]()
    sc0 = O.Scene(_single([0.0, 0.0, 1.0]), cam)
    x, y = 40, 20
    # a point on pixel (x, y)'s centre ray, from the oracle's own inverse map
    if model == "erp":
        lon = np.pi * (2.0 * (x + 0.5) / sc0.width - 1.0)
        lat = 0.5 * np.pi * (2.0 * (y + 0.5) / sc0.height - 1.0)
        d_cam = np.array([np.cos(lat) * np.sin(lon), np.sin(lat), np.cos(lat) * np.cos(lon)])
    else:
        d_cam = np.array([(x + 0.5 - cam["cx"]) / cam["fx"], (y + 0.5 - cam["cy"]) / cam["fy"], 1.0])
    R, c = np.asarray(cam["R"]), -np.asarray(cam["R"]).T @ np.asarray(cam["t"])
    near, far = c + R.T @ (2.0 * d_cam), c + R.T @ (3.5 * d_cam)
    depth = (lambda p: np.linalg.norm(R @ p + cam["t"])) if model == "erp" else (lambda p: (R @ p + cam["t"])[2])
    o1, o2 = 0.6, 0.7
    r1 = O.render(O.Scene(_single(near, opac=o1), cam), alt=False)
    assert r1["depth"][y, x] == pytest.approx(depth(near) * o1, rel=1e-12)
    assert r1["alpha"][y, x] == pytest.approx(o1, rel=1e-12)
    g2 = _single(np.stack([far, near]), opac=[o2, o1])
    r2 = O.render(O.Scene(g2, cam), alt=False)
    assert r2["depth"][y, x] == pytest.approx(depth(near) * o1 + depth(far) * o2 * (1 - o1), rel=1e-12)
    assert r2["alpha"][y, x] == pytest.approx(1 - (1 - o1) * (1 - o2), rel=1e-12)


@pytest.mark.parametrize("model", sorted(CAMS))
def test_depth_is_colour_channel_with_depth_as_colour(model):
    """The depth image equals the colour image of the same scene whose
    (view-independent, degree-0) colours are set to the Gaussians' depths,
    with a black background."""
    g = scenes.shell_scene(111, 500, r0=1.0, r1=5.0, scale_lo=0.02, scale_hi=0.4)
    cam = CAMS[model]()
    sc = O.Scene(g, cam)
    d = O.project(sc)[:, O.REC_FIELDS["depth"]]
    sh = np.zeros((sc.n, 16, 3))
    sh[:, 0, :] = ((d - 0.5) / Y00)[:, None]
    sc_d = sc.with_params(sh=sh, sh_degree=0)
    r, rd = O.render(sc, alt=False), O.render(sc_d, alt=False)
    np.testing.assert_allclose(r["depth"], rd["image"][0], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(r["final_T"], rd["final_T"])


@pytest.mark.parametrize("model", sorted(CAMS))
def test_depth_brute_force(model):
    g = scenes.shell_scene(112, 300, r0=1.0, r1=5.0, scale_lo=0.02, scale_hi=0.4)
    sc = O.Scene(g, CAMS[model](rows=29))
    r = O.render(sc, alt=False)
    _, _, _, D = brute.render(sc, records=O.project(sc), with_depth=True)
    np.testing.assert_allclose(r["depth"], D, rtol=0, atol=1e-12)
    _, _, _, D2 = brute.render(sc, with_depth=True)
    np.testing.assert_allclose(r["depth"], D2, rtol=0, atol=1e-5)


def _richardson(f, h):
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


_ATTR = dict(means="means", scales="scales", quats="quats", opacities="opac")


@pytest.mark.parametrize("model", sorted(CAMS))
@pytest.mark.parametrize("name,width", [("means", 3), ("scales", 3), ("quats", 4), ("opacities", 1)])
def test_depth_alpha_gradients_match_finite_differences(model, name, width):
    """The backward of <G_D, depth> + <G_A, alpha> (alpha = 1 - T_final) and
    a colour cotangent against central differences."""
    g = scenes.shell_scene(113, 60, r0=1.0, r1=3.5, scale_lo=0.05, scale_hi=0.4)
    sc = O.Scene(g, CAMS[model](rows=40))
    rng = np.random.default_rng(114 + width)
    H, W = sc.out_height, sc.width
    G, GD, GA = rng.normal(size=(3, H, W)), rng.normal(size=(H, W)), rng.normal(size=(H, W))
    b = O.backward(sc, G, with_abs=False, dL_ddepth=GD, dL_dalpha=GA)
    base = getattr(sc, _ATTR[name])
    zero = np.zeros((3, H, W))
    mask = np.ones(sc.tiles_x * sc.tiles_y, np.uint8)
    visible = np.nonzero(O.project(sc)[:, 0] > 0)[0]

    def objective(s):
        r = O.render(s, alt=False)
        return float((r["image"] * G).sum() + (r["depth"] * GD).sum() + (r["alpha"] * GA).sum())

    checked = 0
    for _ in range(60):
        i, k = visible[rng.integers(len(visible))], rng.integers(width)

        def at(d):
            a = base.copy()
            a.reshape(sc.n, -1)[i, k] += d
            return sc.with_params(**{name: a})

        h = 1e-4
        if len({O.l1_tiles(at(d), zero, mask)[1] for d in (h, -h, h / 2, -h / 2)}) != 1:
            continue
        fd = _richardson(lambda d: objective(at(d)), h)
        an = b[name].reshape(sc.n, -1)[i, k]
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (model, name, i, k, an, fd)
        checked += 1
        if checked == 6:
            break
    assert checked == 6


# ------------------------------------------------------------ masked loss
def _images(seed, shape=(3, 24, 40)):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, size=shape)
    return x, np.clip(x + rng.normal(0, 0.1, size=shape), 0, 1)


@pytest.mark.parametrize("lam", [0.0, 0.2, 1.0])
def test_mask_of_ones_and_scale_invariance(lam):
    x, y = _images(120)
    L, g = Q.photometric(x, y, lam)
    Lm, gm = Q.photometric(x, y, lam, mask=np.ones(x.shape[1:]))
    assert Lm == pytest.approx(L, rel=1e-14)
    np.testing.assert_allclose(gm, g, rtol=1e-12, atol=1e-18)
    m = (np.random.default_rng(121).uniform(size=x.shape[1:]) > 0.3).astype(np.float64)
    L1_, g1_ = Q.photometric(x, y, lam, mask=m)
    L2_, g2_ = Q.photometric(x, y, lam, mask=3.0 * m)
    assert L2_ == pytest.approx(L1_, rel=1e-13)
    np.testing.assert_allclose(g2_, g1_, rtol=1e-12, atol=1e-18)


def test_masked_l1_is_l1_of_the_cropped_images():
    """With lambda = 0 and a mask of the top rows, the loss is the L1 of the
    images cropped to those rows, and the gradient vanishes below."""
    x, y = _images(122)
    m = np.zeros(x.shape[1:])
    m[:17] = 1.0
    L, g = Q.photometric(x, y, 0.0, mask=m)
    Lc, gc = Q.photometric(x[:, :17], y[:, :17], 0.0)
    assert L == pytest.approx(Lc, rel=1e-14)
    np.testing.assert_allclose(g[:, :17], gc, rtol=1e-14)
    assert np.all(g[:, 17:] == 0.0)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_masked_gradient_matches_finite_differences(lam):
    x, y = _images(123, shape=(2, 20, 26))
    m = np.random.default_rng(124).uniform(size=x.shape[1:]) * (np.arange(20)[:, None] < 15)
    L, g = Q.photometric(x, y, lam, mask=m)
    rng = np.random.default_rng(125)
    for _ in range(12):
        c, i, j = rng.integers(2), rng.integers(20), rng.integers(26)
        if abs(x[c, i, j] - y[c, i, j]) < 1e-3:
            continue
        h = 1e-6

        def f(d):
            xx = x.copy()
            xx[c, i, j] += d
            return Q.photometric(xx, y, lam, mask=m)[0]

        fd = (f(h) - f(-h)) / (2 * h)
        assert fd == pytest.approx(g[c, i, j], rel=1e-5, abs=1e-10)
