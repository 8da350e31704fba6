"""omnigs_forward with caller capacities (no read-back): the same outputs,
instance lists and backward as the call that reads the counts back, the
device counts, overflow flagged for every capacity below the counts, and the
oracle's image from a capacity-mode render.

Same seeded inputs on both sides; comparison rules in ``parity.py``."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2404_03202_amd import omnigs as B
from paper_2404_03202_amd import scenes

import parity
from test_gpu_parity import np_, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "erp_seam": lambda: (scenes.shell_scene(140, 20000), scenes.camera(256, 128, scenes.rot_y(2.9).T, [0.1, 0.0, 0.1])),
    "pinhole_rows": lambda: (scenes.shell_scene(141, 12000),
                             dict(scenes.pinhole_camera(150, 100, 80.0, scenes.rot_y(-0.9).T, [0.0, 0.2, -0.2]),
                                  rows=71)),
}


def _same_forward(a, b, what):
    for key in ("image", "final_T", "n_contrib", "n_blended"):
        assert torch.equal(getattr(a, key), getattr(b, key)), (what, key)
    for x, y in zip(a.instance_lists(), b.instance_lists()):
        assert torch.equal(x, y), what


@pytest.mark.parametrize("case", sorted(CASES))
def test_capacity_forward_equals_read_back(case):
    g, cam = CASES[case]()
    gd = to_dev(g)
    ref = B.omnigs_forward(gd, cam, with_blended=True)
    torch.cuda.synchronize()
    M, S = ref.n_instances, ref.n_entries
    assert M > 1000 and 0 < S <= M
    assert ref.counts() == (S, M)
    for cap in ((M, S), (M, 0), (2 * M + 7, S + 5)):
        r = B.omnigs_forward(gd, cam, with_blended=True, capacity=cap)
        torch.cuda.synchronize()
        assert r.n_instances == -1 and r.n_entries == -1
        assert int(r.overflow.item()) == 0, cap
        assert r.counts() == (S, M)
        _same_forward(r, ref, f"{case} {cap}")


@pytest.mark.parametrize("case", sorted(CASES))
def test_capacity_backward_matches(case):
    g, cam = CASES[case]()
    gd = to_dev(g)
    rng = np.random.default_rng(142)
    H, W = B.image_rows(cam), cam["width"]
    G = torch.from_numpy((rng.normal(size=(3, H, W)) / (H * W)).astype(np.float32)).to("cuda:0")
    ref = B.omnigs_forward(gd, cam)
    gref = B.omnigs_backward(gd, cam, None, ref, G)
    r = B.omnigs_forward(gd, cam, capacity=(ref.n_instances + 31, ref.n_entries + 3))
    gcap = B.omnigs_backward(gd, cam, None, r, G)
    torch.cuda.synchronize()
    assert int(r.overflow.item()) == 0
    for k in gref:
        # float atomics add in a different order from run to run
        a, b = gref[k].double(), gcap[k].double()
        scale = float(a.abs().max()) + 1e-30
        assert float((a - b).abs().max()) <= 1e-5 * scale, k


def test_capacity_overflow_is_flagged():
    g, cam = CASES["erp_seam"]()
    gd = to_dev(g)
    ref = B.omnigs_forward(gd, cam)
    torch.cuda.synchronize()
    M, S = ref.n_instances, ref.n_entries
    for cap in ((M - 1, S), (M, S - 1), (M // 3, 0), (1, 1)):
        r = B.omnigs_forward(gd, cam, capacity=cap)
        torch.cuda.synchronize()
        assert int(r.overflow.item()) == 1, cap
        assert r.counts() == (S, M), cap  # the counts stay exact
    # the next call is unaffected
    again = B.omnigs_forward(gd, cam, capacity=(M, S))
    torch.cuda.synchronize()
    assert int(again.overflow.item()) == 0
    assert torch.equal(again.image, ref.image)


def test_capacity_render_against_oracle():
    g, cam = CASES["pinhole_rows"]()
    r = B.omnigs_forward(to_dev(g), cam, capacity=(400000, 0))
    torch.cuda.synchronize()
    assert int(r.overflow.item()) == 0
    orc = O.render(O.Scene(g, cam))
    parity.check_image(np_(r.image), orc, what="capacity mode")


def test_capacity_empty_scene():
    empty = to_dev(dict(means=np.zeros((0, 3)), scales=np.zeros((0, 3)), quats=np.zeros((0, 4)),
                        opacities=np.zeros(0), sh=np.zeros((0, 16, 3)), sh_degree=3))
    cam = scenes.camera(64, 32)
    r = B.omnigs_forward(empty, cam, dict(bg=(0.25, 0.5, 0.75)), capacity=(100, 10))
    torch.cuda.synchronize()
    assert int(r.overflow.item()) == 0 and r.counts() == (0, 0)
    expect = np.broadcast_to(np.array((0.25, 0.5, 0.75), np.float32)[:, None, None], (3, 32, 64))
    np.testing.assert_array_equal(np_(r.image), expect)
