"""Saving and loading the resident serving scene (CPU): a round trip keeps
every parameter bit for bit, nothing is pickled, and inconsistent arrays are
refused."""
import numpy as np
import pytest
import torch

from paper_2404_03202_amd import scenes, serve


def test_scene_round_trip(tmp_path):
    g = scenes.room_scene(7, 2000)
    path = str(tmp_path / "scene.npz")
    serve.save_scene(path, g)
    back = serve.load_scene(path, "cpu")
    assert back["sh_degree"] == g["sh_degree"]
    for k in serve.SCENE_KEYS:
        np.testing.assert_array_equal(back[k].numpy(), np.asarray(g[k], np.float32))
        assert back[k].dtype == torch.float32 and back[k].is_contiguous()
    # the file holds plain arrays only
    with np.load(path, allow_pickle=False) as f:
        assert sorted(f.files) == sorted(list(serve.SCENE_KEYS) + ["sh_degree"])


def test_scene_shape_checks(tmp_path):
    g = scenes.shell_scene(8, 100)
    bad = dict(g, quats=g["quats"][:, :3])
    path = str(tmp_path / "bad.npz")
    serve.save_scene(path, bad)
    with pytest.raises(ValueError, match="quats"):
        serve.load_scene(path, "cpu")
    bad = dict(g, sh=g["sh"][:, :4], sh_degree=3)
    serve.save_scene(path, bad)
    with pytest.raises(ValueError, match="sh"):
        serve.load_scene(path, "cpu")
