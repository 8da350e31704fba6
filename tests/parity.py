"""Comparison rules between the HIP path and the FP64 oracle.

* Images: max-abs <= 1e-4 per channel.  Pixels where the oracle met one
  near-threshold decision (alpha vs alpha_min, T vs T_min, a depth near-tie)
  pass if they match either branch; pixels with two or more are excluded and
  counted (their fraction is bounded).
* Tile lists: bit-exact, except that instances of one tile whose t_r agree to
  within the float32 resolution of the depth key may appear in any order.
* Gradients: |g - g_o| <= 1e-3 max(|g_o|, 1e-2 A), where A is the oracle's sum
  of |per-pixel contributions| to that entry, each weighted by 1 + the pixel's
  optical depth ln(1 / T_final) (float32 sums of terms of both signs are
  judged against that scale; a float32 alpha is accurate to ~1e-6 relative,
  and the transmittance products carry that error through every instance of
  the pixel), and per-group relative L2 <= 1e-3.
"""
import numpy as np

IMAGE_TOL = 1e-4
GRAD_REL = 1e-3
GRAD_FLOOR = 1e-2


def check_image(gpu_image, orc, tol=IMAGE_TOL, max_excluded=1e-3, what="image"):
    g = np.asarray(gpu_image, dtype=np.float64)
    o = orc["image"]
    nf = orc["n_flags"]
    err = np.abs(g - o).max(axis=0)
    err_alt = np.abs(g - orc["alt"]).max(axis=0) if orc.get("alt") is not None else err
    ok = ((nf == 0) & (err <= tol)) | ((nf == 1) & (np.minimum(err, err_alt) <= tol)) | (nf >= 2)
    excluded = float((nf >= 2).mean())
    if not ok.all():
        ys, xs = np.nonzero(~ok)
        k = np.argmax(err[~ok])
        raise AssertionError(
            f"{what}: {(~ok).sum()} pixels off by > {tol}; worst {err[ys[k], xs[k]]:.3e} at (x={xs[k]}, y={ys[k]}) "
            f"gpu={g[:, ys[k], xs[k]]} oracle={o[:, ys[k], xs[k]]} flags={nf[ys[k], xs[k]]}")
    assert excluded <= max_excluded, f"{what}: {excluded:.2e} of pixels excluded (two or more near-ties)"
    return dict(max_err=float(err[nf == 0].max()) if (nf == 0).any() else 0.0, excluded=excluded)


def check_transmittance(gpu_T, gpu_nc, orc, tol=IMAGE_TOL):
    nf = orc["n_flags"]
    sel = nf == 0
    dT = np.abs(np.asarray(gpu_T, np.float64) - orc["final_T"])[sel]
    assert dT.max(initial=0) <= tol, f"final T off by {dT.max():.3e}"
    bad = (np.asarray(gpu_nc) != orc["n_contrib"]) & sel
    assert not bad.any(), f"n_contrib differs at {bad.sum()} unflagged pixels"


def depth_groups(tile, tr, rel=2.0 ** -22):
    """Label runs of one tile's list whose consecutive t_r differ by less than
    ``rel`` (the float32 depth key cannot order them)."""
    new = np.ones(len(tile), bool)
    if len(tile) > 1:
        same_tile = tile[1:] == tile[:-1]
        close = np.abs(tr[1:] / tr[:-1] - 1.0) < rel
        new[1:] = ~(same_tile & close)
    return np.cumsum(new)


def check_tile_lists(gpu_tile, gpu_gid, orc_tile, orc_gid, orc_tr, flagged_gids=()):
    gt = np.asarray(gpu_tile, np.int64)
    gg = np.asarray(gpu_gid, np.int64)
    ot = np.asarray(orc_tile, np.int64)
    og = np.asarray(orc_gid, np.int64)
    if len(flagged_gids):
        fl = np.zeros(max(gg.max(initial=0), og.max(initial=0)) + 1, bool)
        fl[np.asarray(flagged_gids, np.int64)] = True
        keep_g = ~fl[gg]
        keep_o = ~fl[og]
        gt, gg = gt[keep_g], gg[keep_g]
        ot, og, orc_tr = ot[keep_o], og[keep_o], np.asarray(orc_tr)[keep_o]
    assert len(gt) == len(ot), f"instance count {len(gt)} vs oracle {len(ot)}"
    np.testing.assert_array_equal(gt, ot, err_msg="tile ids of the sorted instances")
    grp = depth_groups(ot, np.asarray(orc_tr, np.float64))
    ig = np.lexsort((gg, grp))
    io = np.lexsort((og, grp))
    np.testing.assert_array_equal(gg[ig], og[io], err_msg="Gaussian order inside tiles")
    exact = (gg == og).mean() if len(gg) else 1.0
    return dict(M=len(gt), exact_positions=float(exact))


def check_grads(gpu, orc, names, skip_rows=None, rel=GRAD_REL, floor=GRAD_FLOOR):
    report = {}
    for k in names:
        g = np.asarray(gpu[k], np.float64).reshape(len(orc[k]), -1)
        o = orc[k].reshape(len(orc[k]), -1)
        A = orc["abs_" + k].reshape(len(orc[k]), -1)
        keep = np.ones(len(o), bool)
        if skip_rows is not None:
            keep[np.asarray(skip_rows, np.int64)] = False
        g, o, A = g[keep], o[keep], A[keep]
        tol = rel * np.maximum(np.abs(o), floor * A)
        bad = np.abs(g - o) > tol
        if bad.any():
            i, j = np.argwhere(bad)[np.argmax((np.abs(g - o) - tol)[bad])]
            raise AssertionError(f"grad {k}: {bad.sum()} entries off; worst row {i} col {j}: gpu {g[i, j]:.6e} "
                                 f"oracle {o[i, j]:.6e} A {A[i, j]:.3e}")
        nrm = np.linalg.norm(o)
        rl2 = np.linalg.norm(g - o) / nrm if nrm > 0 else np.linalg.norm(g)
        assert rl2 <= rel, f"grad {k}: relative L2 {rl2:.3e}"
        report[k] = float(rl2)
    return report
