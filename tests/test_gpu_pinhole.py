"""Parity of the pinhole camera (Eq. 2) on the HIP path with the FP64 oracle:
forward images, transmittance, contributor counts and tile lists, backward
gradients, a width that is not a multiple of 16, Gaussians behind the camera
and off-screen, and batches that mix pinhole and ERP cameras.

Same seeded inputs on both sides; comparison rules in ``parity.py``."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2404_03202_amd import omnigs as B
from paper_2404_03202_amd import scenes

import parity
from test_gpu_parity import compare_backward, compare_forward, gpu_forward, np_, to_dev

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


CASES = {
    # 10 x 8 tiles, a 90 degree crop from inside the shell
    "crop_160x120": lambda: (scenes.shell_scene(100, 20000),
                             scenes.pinhole_camera(160, 120, 90.0, scenes.rot_y(0.6).T, [0.2, -0.1, 0.3])),
    # ragged last tile column and row, off-centre principal point, fy != fx
    "ragged_150x100": lambda: (scenes.shell_scene(101, 8000),
                               scenes.pinhole_camera(150, 100, 80.0, scenes.rot_y(-1.2).T, [0.0, 0.2, -0.2], fy=70.0,
                                                     cx=71.3, cy=55.9)),
    # close, large Gaussians: many behind the camera, centres far off-screen
    "near_and_offscreen": lambda: (scenes.shell_scene(102, 3000, r0=0.3, r1=2.0, scale_lo=0.05, scale_hi=0.6),
                                   scenes.pinhole_camera(96, 80, 110.0, scenes.rot_y(2.0).T)),
    # a wide field of view on the room layout, 48 x 32 tiles
    "room_768x512": lambda: (scenes.room_scene(103, 60000),
                             scenes.pinhole_camera(768, 512, 100.0, (scenes.rot_y(0.3) @ scenes.rot_x(0.2)).T,
                                                   [0.1, 0.0, 0.2])),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_pinhole_forward(case):
    g, cam = CASES[case]()
    r, orc, rep = compare_forward(g, cam, settings=dict(bg=(0.1, 0.3, 0.2)), what=case)
    print(case, rep)
    assert rep["M"] > 0


def test_pinhole_offscreen_centres_are_rendered():
    """Gaussians whose centre projects outside the image still blend into
    the pixels their footprint reaches (no seam wrap of their offsets)."""
    g, cam = CASES["near_and_offscreen"]()
    rec = O.project(O.Scene(g, cam))
    vis = rec[:, 0] > 0
    off = vis & ((rec[:, 7] < 0) | (rec[:, 7] > cam["width"]) | (rec[:, 8] < 0) | (rec[:, 8] > cam["height"]))
    assert off.sum() > 20
    r = gpu_forward(g, cam)
    # the Gaussians with an off-screen centre appear in the GPU tile lists
    _, gid, _ = (np_(x) for x in r.instance_lists())
    assert np.isin(np.nonzero(off)[0], gid).sum() > 20


def test_pinhole_depth_order_is_t_z():
    g, cam = CASES["crop_160x120"]()
    rec = O.project(O.Scene(g, cam))
    r = gpu_forward(g, cam)
    vis = rec[:, 0] > 0
    ids = np.arange(len(vis))
    expect = np.concatenate([ids[vis][np.lexsort((ids[vis], rec[vis, O.REC_FIELDS["depth"]].astype(np.float32)))],
                             ids[~vis]])
    np.testing.assert_array_equal(np_(r.depth_order()), expect)


@pytest.mark.parametrize("case", ["crop_160x120", "ragged_150x100"])
def test_pinhole_backward(case):
    g, cam = CASES[case]()
    rep = compare_backward(g, cam, scenes.perturbed(104, g), settings=dict(bg=(0.1, 0.2, 0.3)))
    print(case, rep)


def test_batch_mixing_pinhole_and_erp_is_bit_identical():
    """One batch of ERP and pinhole cameras (ragged widths included): every
    output equals the same camera rendered alone, bit for bit."""
    g = scenes.shell_scene(105, 30000)
    cams = [scenes.camera(256, 128, scenes.rot_y(0.4).T, [0.1, 0.0, 0.0]),
            scenes.pinhole_camera(150, 100, 80.0, scenes.rot_y(0.4).T, [0.1, 0.0, 0.0]),
            scenes.pinhole_camera(64, 64, 60.0, scenes.rot_y(-2.0).T),
            scenes.camera(128, 72, scenes.rot_y(1.0).T, [0.0, 0.3, 0.0]),
            scenes.pinhole_camera(333, 211, 120.0, (scenes.rot_y(2.5) @ scenes.rot_x(-0.3)).T, [0.2, 0.2, 0.2])]
    gd = to_dev(g)
    batch = B.omnigs_forward_batch(gd, cams, None, with_blended=True)
    torch.cuda.synchronize()
    for k, cam in enumerate(cams):
        one = B.omnigs_forward(gd, cam, None, with_blended=True)
        torch.cuda.synchronize()
        out = batch.outs[k]
        assert torch.equal(out["image"], one.image), k
        assert torch.equal(out["final_T"], one.final_T), k
        assert torch.equal(out["n_contrib"], one.n_contrib), k
    # and one pinhole output against the oracle
    orc = O.render(O.Scene(g, cams[1]))
    parity.check_image(np_(batch.outs[1]["image"]), orc, what="batched pinhole")
