"""Parity of the loss masks and auxiliary outputs on the HIP path with the
FP64 oracle: row crops (forward and backward), the depth image, the
backward of depth and alpha cotangents, the masked photometric loss, and
batches with depth images and crops bit-identical to single renders.

Same seeded inputs on both sides; comparison rules in ``parity.py``."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import ssim as Q
from paper_2404_03202_amd import omnigs as B
from paper_2404_03202_amd import scenes

import parity
from test_gpu_parity import compare_backward, compare_forward, flagged_gaussians, np_, to_dev

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

CAMS = {
    "erp_rows": lambda: dict(scenes.camera(256, 128, scenes.rot_y(0.7).T, [0.1, -0.1, 0.2]), rows=113),
    "pinhole_rows": lambda: dict(scenes.pinhole_camera(150, 100, 80.0, scenes.rot_y(-0.9).T, [0.0, 0.2, -0.2]),
                                 rows=71),
    "erp_full": lambda: scenes.camera(128, 64, scenes.rot_y(0.2).T),
}


@pytest.mark.parametrize("case", ["erp_rows", "pinhole_rows"])
def test_row_crop_forward_and_backward(case):
    g = scenes.shell_scene(130, 8000)
    cam = CAMS[case]()
    r, orc, rep = compare_forward(g, cam, settings=dict(bg=(0.1, 0.3, 0.2)), what=case)
    assert r.image.shape == (3, cam["rows"], cam["width"])
    rep_b = compare_backward(g, cam, scenes.perturbed(131, g), settings=dict(bg=(0.1, 0.2, 0.3)))
    print(case, rep, rep_b)


def test_row_crop_equals_top_rows_of_full_render():
    g = scenes.shell_scene(132, 8000)
    full = scenes.camera(256, 128, scenes.rot_y(0.7).T, [0.1, -0.1, 0.2])
    crop = dict(full, rows=77)
    gd = to_dev(g)
    a = B.omnigs_forward(gd, full, with_depth=True)
    b = B.omnigs_forward(gd, crop, with_depth=True)
    torch.cuda.synchronize()
    # tiles 0..4 are whole in both, the crop's last tile row is partial
    assert torch.equal(b.image, a.image[:, :77]) and torch.equal(b.final_T, a.final_T[:77])
    assert torch.equal(b.depth, a.depth[:77])


@pytest.mark.parametrize("case", ["erp_full", "pinhole_rows"])
def test_depth_image(case):
    g = scenes.shell_scene(133, 6000)
    cam = CAMS[case]()
    sc = O.Scene(g, cam)
    orc = O.render(sc)
    r = B.omnigs_forward(to_dev(g), cam, with_depth=True)
    torch.cuda.synchronize()
    sel = orc["n_flags"] == 0
    d = np_(r.depth).astype(np.float64)
    scale = max(1.0, float(np.abs(orc["depth"]).max()))
    err = np.abs(d - orc["depth"])[sel]
    assert err.max() <= 1e-4 * scale, err.max()
    np.testing.assert_allclose(1.0 - np_(r.final_T)[sel], orc["alpha"][sel], atol=1e-4)


@pytest.mark.parametrize("case", ["erp_full", "pinhole_rows"])
def test_depth_and_alpha_backward(case):
    """Gradients of <G, image> + <G_D, depth> + <G_A, alpha> against the
    oracle (cotangents zeroed at pixels with a near-tie decision)."""
    g = scenes.shell_scene(134, 3000, r0=1.0, r1=5.0, scale_lo=0.02, scale_hi=0.4)
    cam = CAMS[case]()
    sc = O.Scene(g, cam, dict(bg=(0.1, 0.2, 0.3)))
    orc = O.render(sc)
    rng = np.random.default_rng(135)
    H, W = sc.out_height, sc.width
    keep = (orc["n_grad_flags"] == 0)
    G = rng.normal(size=(3, H, W)) * keep / (H * W)
    GD = rng.normal(size=(H, W)) * keep / (H * W)
    GA = rng.normal(size=(H, W)) * keep / (H * W)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    ob = O.backward(sc, f32(G), dL_ddepth=f32(GD), dL_dalpha=f32(GA))
    gd = to_dev(g)
    fwd = B.omnigs_forward(gd, cam, dict(bg=(0.1, 0.2, 0.3)))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)
    grads = B.omnigs_backward(gd, cam, dict(bg=(0.1, 0.2, 0.3)), fwd, t(G), dL_ddepth=t(GD), dL_dalpha=t(GA))
    torch.cuda.synchronize()
    gg = {k: np_(v) for k, v in grads.items()}
    rep = parity.check_grads(gg, ob, ["means", "scales", "quats", "opacities", "sh", "screen"],
                             skip_rows=flagged_gaussians(sc))
    print(case, rep)
    # only the depth cotangent: the colour path contributes nothing
    grads0 = B.omnigs_backward(gd, cam, dict(bg=(0.1, 0.2, 0.3)), fwd, t(np.zeros_like(G)), dL_ddepth=t(GD))
    ob0 = O.backward(sc, np.zeros_like(G), dL_ddepth=f32(GD))
    torch.cuda.synchronize()
    parity.check_grads({k: np_(v) for k, v in grads0.items()}, ob0, ["means", "opacities"],
                       skip_rows=flagged_gaussians(sc))


@pytest.mark.parametrize("lam", [0.0, 0.2, 1.0])
@pytest.mark.parametrize("shape", [(3, 64, 128), (2, 50, 250)])
def test_masked_photometric_loss(lam, shape):
    rng = np.random.default_rng([shape[2], int(lam * 10)])
    x = rng.uniform(0, 1, size=shape)
    y = np.clip(x + rng.normal(0, 0.1, size=shape), 0, 1)
    m = rng.uniform(0, 1, size=shape[1:]) * (np.arange(shape[1])[:, None] < shape[1] - 9)  # bottom rows out
    x32, y32, m32 = (a.astype(np.float32).astype(np.float64) for a in (x, y, m))
    ol, og = Q.photometric(x32, y32, lam, mask=m32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)
    loss, g = B.omnigs_photometric_loss(t(x), t(y), lam, mask=t(m))
    torch.cuda.synchronize()
    assert abs(float(loss.item()) - ol) <= 2e-6 * max(1.0, abs(ol)), (float(loss.item()), ol)
    gg = np_(g).astype(np.float64)
    scale = 1.0 / (shape[0] * m32.sum())
    sel = np.abs(x32 - y32) > 1e-6
    err = np.abs(gg - og)[sel]
    assert err.max() <= 2e-4 * scale, err.max() / scale
    assert np.all(gg[:, shape[1] - 9:] == 0.0) if lam == 0.0 else True


def test_mask_of_ones_matches_unmasked():
    rng = np.random.default_rng(136)
    x = torch.from_numpy(rng.uniform(0, 1, size=(3, 40, 96)).astype(np.float32)).to(DEV)
    y = torch.from_numpy(rng.uniform(0, 1, size=(3, 40, 96)).astype(np.float32)).to(DEV)
    l0, g0 = B.omnigs_photometric_loss(x, y, 0.2)
    l1, g1 = B.omnigs_photometric_loss(x, y, 0.2, mask=torch.ones(40, 96, device=DEV))
    torch.cuda.synchronize()
    assert torch.equal(l0, l1) and torch.equal(g0, g1)


def test_batch_with_depth_and_crops_is_bit_identical():
    g = scenes.shell_scene(137, 20000)
    cams = [dict(scenes.camera(256, 128, scenes.rot_y(0.4).T), rows=100),
            scenes.pinhole_camera(150, 100, 80.0, scenes.rot_y(0.4).T),
            dict(scenes.pinhole_camera(96, 96, 60.0, scenes.rot_y(-2.0).T), rows=50),
            scenes.camera(128, 64, scenes.rot_y(1.0).T, [0.0, 0.3, 0.0])]
    gd = to_dev(g)
    batch = B.omnigs_forward_batch(gd, cams, None, with_depth=True)
    torch.cuda.synchronize()
    for k, cam in enumerate(cams):
        one = B.omnigs_forward(gd, cam, None, with_depth=True)
        torch.cuda.synchronize()
        out = batch.outs[k]
        assert out["image"].shape[1] == B.image_rows(cam)
        for key in ("image", "final_T", "n_contrib", "depth"):
            assert torch.equal(out[key], getattr(one, key)), (k, key)
