"""The tile binning's two sources of an entry's covered tiles agree: the
covers carried in the upper bits of the block-entry sort keys (the default)
and the covers recomputed from the Gaussians' tile rectangles (taken when a
call has more 8x8-tile blocks than the keys' id bits hold, forced here with
omnigs_set_cover_key_blocks).  The same switch moves the split of the block
lists into chunks from one workgroup to three kernels (chunk counts, their
scan, chunk owners).  Tile lists, ranges and images must be equal bit for
bit; the default path's lists are checked against the oracle's in
test_gpu_parity.py and test_gpu_fullsize.py."""
import numpy as np
import pytest
import torch

from paper_2404_03202_amd import omnigs as B
from paper_2404_03202_amd import scenes

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

CASES = {
    "config1": lambda: scenes.config1()[:2],
    # rectangles wrapping across the seam: two column intervals per cover
    "seam_straddlers": lambda: (scenes.room_scene(51, 4000, seam_fraction=0.5), scenes.camera(256, 128)),
    # 512 blocks: the block sort takes two passes and finds the ranges from
    # adjacent keys, which carry the covers above the id bits
    "two_pass_block_sort": lambda: (scenes.shell_scene(57, 20000), scenes.camera(4096, 2048)),
}


def render(g, cam):
    d = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(DEV)
         for k, v in g.items() if k != "sh_degree"}
    d["sh_degree"] = g["sh_degree"]
    r = B.omnigs_forward(d, cam, None)
    torch.cuda.synchronize()
    out = [r.image, r.final_T, r.n_contrib, *r.instance_lists()]
    return [x.detach().cpu().numpy() for x in out], r.n_instances


@pytest.mark.parametrize("case", sorted(CASES))
def test_cover_sources_agree(case):
    g, cam = CASES[case]()
    try:
        a, ma = render(g, cam)
        B.omnigs_set_cover_key_blocks(1)  # every call here has more than one block
        b, mb = render(g, cam)
    finally:
        B.omnigs_set_cover_key_blocks(0)
    assert ma == mb > 0
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
