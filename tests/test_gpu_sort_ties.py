"""Exact depth ties through the HIP path: the depth order breaks them by
Gaussian id (Sec. 3.3 orders by t_r; equal keys keep the id order), through
every pass of the radix sort and its lookback, and the tile lists match the
oracle's.

Same seeded inputs on both sides; comparison rules in ``parity.py``."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2404_03202_amd import omnigs as B
from paper_2404_03202_amd import scenes

import parity
from test_gpu_parity import flagged_gaussians, gpu_forward, np_

pytestmark = pytest.mark.gpu


def _expected_order(sc):
    rec = O.project(sc)
    vis = rec[:, 0] > 0
    ids = np.arange(len(vis))
    key = rec[vis, O.REC_FIELDS["depth"]].astype(np.float32)
    return np.concatenate([ids[vis][np.lexsort((ids[vis], key))], ids[~vis]])


def test_duplicated_scene_ties_break_by_id():
    """Every Gaussian twice (ids i and i + n): each depth key occurs in pairs
    of bit-identical values."""
    g = scenes.shell_scene(150, 6000)
    g2 = {k: (np.concatenate([v, v]) if k != "sh_degree" else v) for k, v in g.items()}
    cam = scenes.camera(256, 128, scenes.rot_y(0.8).T, [0.1, 0.05, -0.1])
    sc = O.Scene(g2, cam)
    r = gpu_forward(g2, cam)
    np.testing.assert_array_equal(np_(r.depth_order()), _expected_order(sc))
    # (the images are not compared: a pixel under two identical Gaussians is
    # a near-tie of the blend order by construction)
    t, gid, tr = O.tile_lists(sc)
    it, ig, _ = (np_(x) for x in r.instance_lists())
    rep = parity.check_tile_lists(it, ig, t, gid, tr, flagged_gaussians(sc))
    assert rep["M"] > 1000, rep


def test_all_keys_equal():
    """Thousands of Gaussians at one mean: one depth key for all, so every
    radix pass sees a single digit (the lookback sums one digit's counts) and
    the order is the id order."""
    rng = np.random.default_rng(151)
    n = 3000
    g = scenes.shell_scene(151, n, scale_lo=0.05, scale_hi=0.2)
    g["means"][:] = np.array([0.4, 0.1, -0.2])
    g["opacities"] = rng.uniform(0.01, 0.05, size=n)  # keep the walks long before T_min
    cam = scenes.camera(256, 128, np.eye(3), [0.0, 0.0, 0.0])
    sc = O.Scene(g, cam)
    r = gpu_forward(g, cam)
    np.testing.assert_array_equal(np_(r.depth_order()), _expected_order(sc))
    t, gid, tr = O.tile_lists(sc)
    it, ig, _ = (np_(x) for x in r.instance_lists())
    rep = parity.check_tile_lists(it, ig, t, gid, tr, flagged_gaussians(sc))
    assert rep["M"] > 2 * n, rep
