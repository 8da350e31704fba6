"""Pins of the optimisation oracle (oracle/optim.py) against independent
references: torch's Adam, finite differences, closed forms and hand-built
densification cases."""
import numpy as np
import pytest
import torch

from oracle import optim as Q


def rand_raw(n=7, K=16, seed=0):
    rng = np.random.default_rng(seed)
    return dict(means=rng.normal(size=(n, 3)), log_scales=rng.normal(-3, 0.5, size=(n, 3)),
                quats=rng.normal(size=(n, 4)), logits=rng.normal(size=n), sh=rng.normal(size=(n, K, 3)), sh_degree=3)


def test_adam_matches_torch_adam():
    raw = rand_raw()
    lrs = Q.default_lrs(extent=2.5)
    groups = Q._split_groups(raw)
    tp = {k: torch.tensor(np.array(v), dtype=torch.float64, requires_grad=True) for k, v in groups.items()}
    opt = torch.optim.Adam([{"params": [tp[k]], "lr": lrs[k]} for k in Q.GROUPS], betas=(0.9, 0.999), eps=1e-15)
    mom = Q.zero_moments(raw)
    rng = np.random.default_rng(1)
    cur = raw
    for step in range(1, 5):
        g = dict(means=rng.normal(size=(7, 3)), log_scales=rng.normal(size=(7, 3)), quats=rng.normal(size=(7, 4)),
                 logits=rng.normal(size=7), sh=rng.normal(size=(7, 16, 3)))
        gg = Q._split_groups(g)
        for k in Q.GROUPS:
            tp[k].grad = torch.tensor(gg[k])
        opt.step()
        cur, mom = Q.adam_step(cur, g, mom, step, lrs)
        mine = Q._split_groups(cur)
        for k in Q.GROUPS:
            np.testing.assert_allclose(mine[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15, err_msg=k)


def test_raw_gradient_chain_by_finite_differences():
    raw = rand_raw(5, 4)
    rng = np.random.default_rng(2)
    ws, wo = rng.normal(size=(5, 3)), rng.normal(size=5)

    def f(r):
        a = Q.activate(r)
        return float((ws * a["scales"]).sum() + (wo * a["opacities"]).sum())
    g = Q.raw_grads(raw, dict(means=0, scales=ws, quats=0, opacities=wo, sh=0))
    h = 1e-6
    for key, shape in (("log_scales", (5, 3)), ("logits", (5,))):
        fd = np.zeros(shape)
        for idx in np.ndindex(shape):
            rp = dict(raw, **{key: raw[key].copy()}); rp[key][idx] += h
            rm = dict(raw, **{key: raw[key].copy()}); rm[key][idx] -= h
            fd[idx] = (f(rp) - f(rm)) / (2 * h)
        np.testing.assert_allclose(g[key], fd, rtol=1e-7, atol=1e-9)


def test_position_schedule_endpoints():
    assert Q.position_lr(0, 3.0) == pytest.approx(3.0 * 1.6e-4, rel=1e-12)
    assert Q.position_lr(30000, 3.0) == pytest.approx(3.0 * 1.6e-6, rel=1e-12)
    assert Q.position_lr(15000, 1.0) == pytest.approx(np.sqrt(1.6e-4 * 1.6e-6), rel=1e-12)
    assert Q.position_lr(99999, 1.0) == pytest.approx(1.6e-6, rel=1e-12)


def test_stats_accumulate_only_visible():
    st = Q.zero_stats(3)
    st = Q.update_stats(st, np.array([[3.0, 4.0], [1.0, 0.0], [0.0, 2.0]]), np.array([1, 0, 1]), np.array([5., 9., 1.]))
    st = Q.update_stats(st, np.array([[0.0, 1.0], [1.0, 1.0], [6.0, 8.0]]), np.array([1, 1, 0]), np.array([2., 3., 7.]))
    np.testing.assert_allclose(st["accum"], [6.0, np.sqrt(2.0), 2.0])
    np.testing.assert_allclose(st["denom"], [2, 1, 1])
    np.testing.assert_allclose(st["max_radius"], [5.0, 3.0, 1.0])


def hand_case():
    """Six Gaussians: 0 below the threshold; 1 clone (small); 2 split (large);
    3 would clone but is pruned for low opacity (with its clone); 4 pruned as
    big on screen; 5 split whose children (scale 2 / 1.6 = 1.25 > 0.1 * 10)
    are pruned as big in the world when the screen rule is on."""
    extent = 10.0
    raw = dict(means=np.arange(18, dtype=np.float64).reshape(6, 3),
               log_scales=np.log(np.array([[0.05] * 3, [0.05, 0.02, 0.01], [0.5, 0.2, 0.1], [0.05] * 3, [0.05] * 3,
                                           [2.0, 2.0, 2.0]])),
               quats=np.tile([1.0, 0.0, 0.0, 0.0], (6, 1)), logits=np.array([0.0, 1.0, 2.0, -6.0, 0.5, 0.3]),
               sh=np.arange(6 * 4 * 3, dtype=np.float64).reshape(6, 4, 3), sh_degree=1)
    stats = dict(accum=np.array([0.0001, 0.003, 0.004, 0.01, 0.0, 0.01]), denom=np.array([1.0, 2.0, 2.0, 1.0, 0.0, 1.0]),
                 max_radius=np.array([3.0, 3.0, 3.0, 3.0, 25.0, 3.0]))
    return raw, stats, extent


def test_densify_hand_case():
    raw, stats, extent = hand_case()
    mom = Q.zero_moments(raw)
    mom = {k: (m + 1.0, v + 2.0) for k, (m, v) in mom.items()}  # recognisable moments
    noise = np.zeros((6, 2, 3))
    noise[2, 0] = [1.0, 0.0, 0.0]
    noise[2, 1] = [0.0, -2.0, 0.5]
    # g = accum / denom = [1e-4, 1.5e-3, 2e-3, 1e-2, 0, 1e-2] against tau = 1e-3;
    # percent_dense * extent = 0.2 separates clones (max scale 0.05) from splits
    out, om, st, counts = Q.densify_and_prune(raw, mom, stats, noise, tau=1e-3, percent_dense=0.02, extent=extent,
                                              min_opacity=0.005, max_screen=20.0, big_fraction=0.1)
    assert {k: v for k, v in counts.items() if k != "flagged"} == dict(kept=2, clones=1, children=2, split=2, cloned=2)
    assert not any(f.any() for f in counts["flagged"].values())
    n_out = out["means"].shape[0]
    assert n_out == 5
    # originals 0 and 1, the clone of 1, the two children of 2
    np.testing.assert_array_equal(out["means"][0], raw["means"][0])
    np.testing.assert_array_equal(out["means"][1], raw["means"][1])
    np.testing.assert_array_equal(out["means"][2], raw["means"][1])
    np.testing.assert_array_equal(out["sh"][2], raw["sh"][1])
    np.testing.assert_array_equal(out["logits"], [0.0, 1.0, 1.0, 2.0, 2.0])
    # children of 2: m + R (S * z), R = I, S = (0.5, 0.2, 0.1)
    np.testing.assert_allclose(out["means"][3], raw["means"][2] + [0.5, 0.0, 0.0], rtol=1e-12)
    np.testing.assert_allclose(out["means"][4], raw["means"][2] + [0.0, -0.4, 0.05], rtol=1e-12)
    np.testing.assert_allclose(np.exp(out["log_scales"][3]), np.array([0.5, 0.2, 0.1]) / 1.6, rtol=1e-6)
    # moments kept for originals, zero for new Gaussians; statistics reset
    for k in Q.GROUPS:
        assert (om[k][0][:2] == 1.0).all() and (om[k][1][:2] == 2.0).all()
        assert (om[k][0][2:] == 0.0).all() and (om[k][1][2:] == 0.0).all()
    assert (st["accum"] == 0).all() and (st["denom"] == 0).all() and st["accum"].shape == (n_out,)


def test_densify_without_screen_rule_keeps_big_gaussians():
    raw, stats, extent = hand_case()
    out, _, _, counts = Q.densify_and_prune(raw, Q.zero_moments(raw), stats, np.zeros((6, 2, 3)), tau=1e-3,
                                            percent_dense=0.02, extent=extent, min_opacity=0.005, max_screen=None)
    # 4 survives (no screen rule), 5's children survive (no world rule)
    assert {k: v for k, v in counts.items() if k != "flagged"} == dict(kept=3, clones=1, children=4, split=2, cloned=2)


def test_split_children_rotate_with_the_gaussian():
    raw = dict(means=np.zeros((1, 3)), log_scales=np.log([[0.3, 0.1, 0.1]]),
               quats=np.array([[np.cos(np.pi / 4), 0.0, 0.0, np.sin(np.pi / 4)]]),  # 90 degrees about z
               logits=np.array([3.0]), sh=np.zeros((1, 1, 3)), sh_degree=0)
    stats = dict(accum=np.array([1.0]), denom=np.array([1.0]), max_radius=np.array([1.0]))
    noise = np.array([[[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]])
    out, _, _, counts = Q.densify_and_prune(raw, Q.zero_moments(raw), stats, noise, tau=0.5, percent_dense=0.1,
                                            extent=1.0, min_opacity=0.005, max_screen=None)
    assert counts["children"] == 2 and out["means"].shape == (2, 3)
    np.testing.assert_allclose(out["means"][0], [0.0, 0.3, 0.0], atol=1e-12)  # x axis -> y axis
    np.testing.assert_allclose(out["means"][1], [0.0, 0.0, 0.1], atol=1e-12)


def test_decisions_in_fp64_flag_near_thresholds():
    """Decisions are the FP64 comparisons of Alg. 1's rules; a mean gradient
    at tau (1 + 1e-7), an opacity at min_opacity (1 - 1e-7) and a largest
    scale at percent_dense * extent (1 - 1e-7) are flagged, and inverting a
    flagged comparison flips exactly that decision.  Values 1e-3 away from
    their thresholds are not flagged."""
    tau, pd, extent, min_o = 1e-3, 0.01, 2.0, 0.005
    n = 4
    accum = np.array([tau * (1 + 1e-7) * 3, tau * 1.5 * 2, tau * 1.5, tau * 0.999 * 5])
    denom = np.array([3.0, 2.0, 1.0, 5.0])
    ls = np.full((n, 3), np.log(0.5 * pd * extent))
    ls[2, 1] = np.log(pd * extent * (1 - 1e-7))
    o = np.array([0.5, min_o * (1 - 1e-7), 0.5, min_o * 1.001])
    raw = dict(means=np.zeros((n, 3)), log_scales=ls, quats=np.tile([1.0, 0, 0, 0], (n, 1)),
               logits=np.log(o / (1 - o)), sh=np.zeros((n, 1, 3)), sh_degree=0)
    stats = dict(accum=accum, denom=denom, max_radius=np.zeros(n))
    d = Q.decisions(raw, stats, tau, pd, extent, min_o, None)
    np.testing.assert_array_equal(d["flags"]["hot"], [True, False, False, False])
    np.testing.assert_array_equal(d["flags"]["low"], [False, True, False, False])
    np.testing.assert_array_equal(d["flags"]["small"], [False, False, True, False])
    # FP64: 0 hot (clone), 1 hot and pruned, 2 hot and small (clone), 3 cold
    np.testing.assert_array_equal(d["clone"], [True, True, True, False])
    np.testing.assert_array_equal(d["keep_orig"], [True, False, True, True])
    inv = Q.decisions(raw, stats, tau, pd, extent, min_o, None,
                      invert=dict(hot=[True, False, False, False], low=[False, True, False, False],
                                  small=[False, False, True, False]))
    np.testing.assert_array_equal(inv["clone"], [False, True, False, False])
    np.testing.assert_array_equal(inv["split"], [False, False, True, False])
    np.testing.assert_array_equal(inv["keep_orig"], [True, True, False, True])


def test_reset_opacity():
    raw = rand_raw(4, 1)
    raw["logits"] = np.array([-8.0, -4.0, 0.0, 3.0])
    mom = Q.zero_moments(raw)
    mom["logits"] = (np.ones(4), np.ones(4))
    out, om = Q.reset_opacity(raw, mom, 0.01)
    np.testing.assert_allclose(Q.sigmoid(out["logits"]), [Q.sigmoid(-8.0), 0.01, 0.01, 0.01], rtol=1e-12)
    assert (om["logits"][0] == 0).all() and (om["logits"][1] == 0).all()
