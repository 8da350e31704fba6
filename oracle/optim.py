"""FP64 oracle of the optimisation loop around the rasterizer (Alg. 1):
the optimizer step, the densification statistics, densification (clone,
split), pruning and the opacity reset.

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg use this module; the library never does.

The paper leaves the optimizer and the densification rules to 3DGS (Kerbl et
al. 2023) and its supplement (absent), with one change: the densification
gradient is dL/ds, the gradient w.r.t. the uniform ERP screen coordinate s of
Eq. 4 (Sec. 4, Alg. 1).  The readings taken here (3DGS's published method and
defaults):

* parameters are optimised raw: means m, log-scales (S = exp), raw
  quaternions (normalised in the rasterizer), opacity logits (o = sigmoid)
  and SH coefficients; the rasterizer's gradients w.r.t. the activated S and
  o are chained through exp and sigmoid;
* Adam (beta1 0.9, beta2 0.999, eps 1e-15) with bias correction, one
  learning rate per group: means (times the scene extent), SH degree-0,
  SH higher degrees, opacity logits, log-scales, quaternions;
* statistics: for every Gaussian visible in the view (covering a tile),
  accum += ||dL/ds||_2 and denom += 1; max_radius = max(max_radius, screen
  radius in pixels);
* densify (every interval, up to an iteration limit), decided in FP64 with
  the comparisons near their thresholds flagged: g = accum / denom
  (0 where denom = 0); clone if g >= tau and max(S) <= percent_dense *
  extent: an identical copy; split if g >= tau and max(S) > percent_dense *
  extent: two children at m + R(q) (S * z_k) for standard normal z_k (given
  as input), log-scales lowered by log(1.6), other parameters copied, the
  parent removed;
* prune after densifying: o < min_opacity, or (when enabled) max_radius >
  max_screen or max(S) > big_fraction * extent; new Gaussians have
  max_radius 0;
* output order: surviving originals in order, then surviving clones in
  order, then surviving first children, then surviving second children; new
  Gaussians start with zero Adam moments and zero statistics; all statistics
  are reset after densification;
* opacity reset: o <- min(o, reset_value) (logit space), the opacity Adam
  moments zeroed.
"""
from __future__ import annotations

import numpy as np

GROUPS = ("means", "sh_dc", "sh_rest", "logits", "log_scales", "quats")


def default_lrs(extent: float = 1.0) -> dict:
    """3DGS's learning rates (the position rate at its initial value)."""
    return dict(means=1.6e-4 * extent, sh_dc=2.5e-3, sh_rest=2.5e-3 / 20.0, logits=0.05, log_scales=5e-3, quats=1e-3)


def position_lr(step: int, extent: float, lr_init=1.6e-4, lr_final=1.6e-6, max_steps=30000) -> float:
    """Exponential interpolation of the position rate from lr_init to
    lr_final over max_steps (3DGS's schedule, without delay)."""
    t = min(max(step / max_steps, 0.0), 1.0)
    return extent * float(np.exp(np.log(lr_init) * (1 - t) + np.log(lr_final) * t))


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def activate(raw: dict) -> dict:
    """Rasterizer inputs from raw parameters."""
    return dict(means=raw["means"], scales=np.exp(raw["log_scales"]), quats=raw["quats"],
                opacities=sigmoid(raw["logits"]), sh=raw["sh"], sh_degree=raw["sh_degree"])


def raw_grads(raw: dict, grads: dict) -> dict:
    """Gradients w.r.t. the raw parameters from those w.r.t. the activated
    scales and opacities (d exp(x)/dx = exp(x); d sigmoid/dx = o (1 - o))."""
    o = sigmoid(raw["logits"])
    return dict(means=grads["means"], log_scales=grads["scales"] * np.exp(raw["log_scales"]), quats=grads["quats"],
                logits=grads["opacities"] * o * (1.0 - o), sh=grads["sh"])


def _split_groups(raw):
    return dict(means=raw["means"], sh_dc=raw["sh"][:, :1], sh_rest=raw["sh"][:, 1:], logits=raw["logits"],
                log_scales=raw["log_scales"], quats=raw["quats"])


def adam_step(raw: dict, grads_raw: dict, moments: dict, step: int, lrs: dict, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (step counts from 1).  moments: {group: (m, v)} arrays
    shaped like the group.  Returns (new raw, new moments)."""
    p = _split_groups(raw)
    g = _split_groups(dict(grads_raw, sh=grads_raw["sh"]))
    new_p, new_m = {}, {}
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    for k in GROUPS:
        m, v = moments[k]
        m = beta1 * m + (1.0 - beta1) * g[k]
        v = beta2 * v + (1.0 - beta2) * g[k] * g[k]
        denom = np.sqrt(v) / np.sqrt(bc2) + eps
        new_p[k] = p[k] - (lrs[k] / bc1) * m / denom
        new_m[k] = (m, v)
    out = dict(raw, means=new_p["means"], logits=new_p["logits"], log_scales=new_p["log_scales"],
               quats=new_p["quats"], sh=np.concatenate([new_p["sh_dc"], new_p["sh_rest"]], axis=1))
    return out, new_m


def zero_moments(raw: dict) -> dict:
    p = _split_groups(raw)
    return {k: (np.zeros_like(p[k]), np.zeros_like(p[k])) for k in GROUPS}


def update_stats(stats: dict, dscreen, visible, radii) -> dict:
    """accum += ||dL/ds|| and denom += 1 where visible; max_radius."""
    vis = np.asarray(visible, bool)
    n = np.linalg.norm(np.asarray(dscreen, np.float64), axis=1)
    return dict(accum=stats["accum"] + np.where(vis, n, 0.0), denom=stats["denom"] + vis.astype(np.float64),
                max_radius=np.where(vis, np.maximum(stats["max_radius"], radii), stats["max_radius"]))


def zero_stats(n: int) -> dict:
    return dict(accum=np.zeros(n), denom=np.zeros(n), max_radius=np.zeros(n))


def quat_to_rot(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


# Relative margin around each densification threshold within which a
# comparison is flagged: float32 inputs, a float32 mean of the statistic and
# thresholds rounded to float32 (or compared in log / logit space) move a
# comparison by a few 1e-7 relative at most.
DECISION_MARGIN = 1e-5

COMPARISONS = ("hot", "small", "low", "big_radius", "big_world", "child_big_world")


def decisions(raw: dict, stats: dict, tau: float, percent_dense: float, extent: float, min_opacity: float,
              max_screen: float | None, big_fraction: float = 0.1, shrink: float = 1.6, invert=None):
    """Clone / split / keep decisions, taken in FP64 on the given inputs:

    * hot: g = accum / denom (0 where denom = 0) >= tau;
    * small: max S <= percent_dense * extent (clone if hot, else split);
    * low: o < min_opacity (pruned);
    * big_radius: max_radius > max_screen; big_world: max S > big_fraction *
      extent; child_big_world: the same for the children's S / shrink (only
      when the screen rule is on; clones and children have radius 0).

    Each comparison whose value lies within a relative DECISION_MARGIN of its
    threshold is flagged (``flags[name]``, bool [n]): an implementation in
    float32 may take it either way.  ``invert`` (dict name -> bool [n], may be
    None) takes the listed comparisons the other way, so that a test can
    enumerate the results those flags allow."""
    n = raw["means"].shape[0]
    accum = np.asarray(stats["accum"], np.float64)
    denom = np.asarray(stats["denom"], np.float64)
    g = np.where(denom > 0, accum / np.where(denom > 0, denom, 1.0), 0.0)
    smax = np.exp(np.asarray(raw["log_scales"], np.float64)).max(axis=1) if n else np.zeros(0)
    o = sigmoid(np.asarray(raw["logits"], np.float64))
    radius = np.asarray(stats["max_radius"], np.float64)
    screen_on = max_screen is not None
    big_s = big_fraction * extent
    cmp = dict(hot=(g, tau, g >= tau), small=(smax, percent_dense * extent, smax <= percent_dense * extent),
               low=(o, min_opacity, o < min_opacity),
               big_radius=(radius, max_screen if screen_on else 1.0,
                           radius > max_screen if screen_on else np.zeros(n, bool)),
               big_world=(smax, big_s, smax > big_s if screen_on else np.zeros(n, bool)),
               child_big_world=(smax / shrink, big_s, smax / shrink > big_s if screen_on else np.zeros(n, bool)))
    flags, take = {}, {}
    for name, (v, thr, dec) in cmp.items():
        active = screen_on or name not in ("big_radius", "big_world", "child_big_world")
        flags[name] = (np.abs(v / thr - 1.0) < DECISION_MARGIN) & active if n else np.zeros(0, bool)
        inv = np.zeros(n, bool) if invert is None or name not in invert else np.asarray(invert[name], bool)
        take[name] = dec ^ inv
    hot, small, low = take["hot"], take["small"], take["low"]
    clone = hot & small
    split = hot & ~small
    keep_orig = ~split & ~low & ~(take["big_radius"] | take["big_world"])
    keep_clone = clone & ~low & ~take["big_world"]
    keep_child = split & ~low & ~take["child_big_world"]
    return dict(clone=clone, split=split, keep_orig=keep_orig, keep_clone=keep_clone, keep_child=keep_child,
                flags=flags, log_shrink=float(np.log(shrink)))


def densify_and_prune(raw: dict, moments: dict, stats: dict, noise, tau: float, percent_dense: float, extent: float,
                      min_opacity: float, max_screen: float | None, big_fraction: float = 0.1, shrink: float = 1.6,
                      invert=None):
    """Clone / split by the averaged dL/ds, then prune (see the module
    docstring for the order).  noise: [n, 2, 3] standard normals (only the
    rows of split Gaussians are used).  invert: as for ``decisions``.
    Returns (raw, moments, stats, counts); counts["flagged"] holds the
    flagged comparisons (``decisions``)."""
    n = raw["means"].shape[0]
    d = decisions(raw, stats, tau, percent_dense, extent, min_opacity, max_screen, big_fraction, shrink, invert)
    keep_orig, keep_clone, keep_child = d["keep_orig"], d["keep_clone"], d["keep_child"]
    clone, split = d["clone"], d["split"]
    scales = np.exp(np.asarray(raw["log_scales"], np.float64))
    child_log = np.asarray(raw["log_scales"], np.float64) - d["log_shrink"]
    R = quat_to_rot(raw["quats"]) if n else np.zeros((0, 3, 3))
    z = np.asarray(noise, np.float64).reshape(n, 2, 3)
    kids = [np.asarray(raw["means"], np.float64) + np.einsum("nij,nj->ni", R, scales * z[:, k]) for k in range(2)]

    def take(d, idx):
        return {k: v[idx] for k, v in d.items()}

    parts_raw, parts_mom = [], []
    per = dict(means=raw["means"], log_scales=raw["log_scales"], quats=raw["quats"], logits=raw["logits"], sh=raw["sh"])
    for sel, means, logs, fresh in ((keep_orig, raw["means"], raw["log_scales"], False),
                                    (keep_clone, raw["means"], raw["log_scales"], True),
                                    (keep_child, kids[0], child_log, True),
                                    (keep_child, kids[1], child_log, True)):
        idx = np.nonzero(sel)[0]
        r = take(per, idx)
        r["means"], r["log_scales"] = means[idx], logs[idx]
        parts_raw.append(r)
        mom = {}
        for k in GROUPS:
            m, v = moments[k]
            mom[k] = (np.zeros_like(m[idx]), np.zeros_like(v[idx])) if fresh else (m[idx], v[idx])
        parts_mom.append(mom)
    out = {k: np.concatenate([p[k] for p in parts_raw], axis=0) for k in per}
    out["sh_degree"] = raw["sh_degree"]
    mom = {k: (np.concatenate([p[k][0] for p in parts_mom]), np.concatenate([p[k][1] for p in parts_mom]))
           for k in GROUPS}
    counts = dict(kept=int(keep_orig.sum()), clones=int(keep_clone.sum()), children=2 * int(keep_child.sum()),
                  split=int(split.sum()), cloned=int(clone.sum()), flagged=d["flags"])
    return out, mom, zero_stats(out["means"].shape[0]), counts


def reset_opacity(raw: dict, moments: dict, value: float = 0.01):
    """o <- min(o, value) in logit space; opacity moments zeroed."""
    lo = np.log(value / (1.0 - value))
    out = dict(raw, logits=np.minimum(raw["logits"], lo))
    mom = dict(moments)
    m, v = moments["logits"]
    mom["logits"] = (np.zeros_like(m), np.zeros_like(v))
    return out, mom
