"""Comparison rules between the HIP path and the FP64 oracle.

* Images: max-abs <= 1e-4 per channel.  A pixel where the oracle met
  near-threshold decisions (alpha vs alpha_min, T vs T_min, the order of two
  depths the float32 key cannot tell apart) passes if its image, final T,
  contributor count and blended count all match one of the results those
  decisions allow (the oracle enumerates them: ``O.branches``).  Only pixels
  with more than ``O.MAX_BRANCHES`` such results are excluded, and their
  fraction is bounded by 1e-4.
* Tile lists: bit-exact, except that instances of one tile whose t_r agree to
  within the float32 resolution of the depth key may appear in any order.
* Gradients: |g - g_o| <= 1e-3 max(|g_o|, 1e-2 A), where A is the oracle's sum
  of |per-pixel contributions| to that entry (float32 sums of terms of both
  signs are judged against that scale), and per-group relative L2 <= 1e-3.
"""
import numpy as np

IMAGE_TOL = 1e-4
GRAD_REL = 1e-3
GRAD_FLOOR = 1e-2
MAX_EXCLUDED = 1e-4


def check_image(gpu_image, orc, tol=IMAGE_TOL, max_excluded=MAX_EXCLUDED, what="image", gpu_T=None, gpu_nc=None,
                gpu_nb=None, pixels=None):
    """Compare the GPU image (and, when given, final T, contributor and
    blended counts) with the oracle render ``orc`` (``O.render``, with its
    branches) at every pixel, or at ``pixels`` = (ys, xs)."""
    H, W = orc["final_T"].shape
    flat = np.arange(H * W) if pixels is None else np.asarray(pixels[0]) * W + np.asarray(pixels[1])
    gi = np.asarray(gpu_image, np.float64).reshape(3, -1)[:, flat]
    oi = orc["image"].reshape(3, -1)[:, flat]
    nf = orc["n_flags"].reshape(-1)[flat]
    err = np.abs(gi - oi).max(axis=0)
    extra = []  # (gpu values, oracle key, exact?)
    if gpu_T is not None:
        extra.append((np.asarray(gpu_T, np.float64).reshape(-1)[flat], "final_T", False))
    if gpu_nc is not None:
        extra.append((np.asarray(gpu_nc).reshape(-1)[flat], "n_contrib", True))
    if gpu_nb is not None:
        extra.append((np.asarray(gpu_nb).reshape(-1)[flat], "n_blended", True))
    ok = err <= tol
    for gv, key, exact in extra:
        ov = orc[key].reshape(-1)[flat]
        ok &= (gv == ov) if exact else (np.abs(gv - ov) <= tol)
    ok &= nf == 0
    excluded = np.zeros(len(flat), bool)
    fl = np.nonzero(nf > 0)[0]
    if len(fl):
        br = orc.get("branches")
        assert br is not None, f"{what}: the oracle render has no branches (render with alt=True)"
        rows = np.searchsorted(br["pixels"], flat[fl])
        assert (br["pixels"][rows] == flat[fl]).all()
        cnt = br["count"][rows]
        B = br["image"].shape[1]
        valid = np.arange(B)[None, :] < cnt[:, None]
        match = valid & (np.abs(br["image"][rows] - gi[:, fl].T[:, None, :]).max(axis=-1) <= tol)
        for gv, key, exact in extra:
            bv = br[key][rows]
            match &= (bv == gv[fl][:, None]) if exact else (np.abs(bv - gv[fl][:, None]) <= tol)
        ok[fl] = match.any(axis=1)
        excluded[fl] = cnt < 0
        ok |= excluded
    frac = float(excluded.mean()) if len(flat) else 0.0
    if not ok.all():
        bad = np.nonzero(~ok)[0]
        k = bad[np.argmax(err[bad])]
        y, x = divmod(int(flat[k]), W)
        raise AssertionError(
            f"{what}: {len(bad)} pixels off by > {tol} (image, T or counts); worst image error {err[k]:.3e} at "
            f"(x={x}, y={y}) gpu={gi[:, k]} oracle={oi[:, k]} flags={nf[k]}")
    assert frac <= max_excluded, f"{what}: {frac:.2e} of pixels excluded (more than the enumerated branches)"
    return dict(max_err=float(err[nf == 0].max()) if (nf == 0).any() else 0.0, excluded=frac,
                flagged=float((nf > 0).mean()) if len(flat) else 0.0)


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
            ratio = float((np.abs(g - o)[bad] / tol[bad]).max())
            raise AssertionError(f"grad {k}: {bad.sum()} entries off (worst at {ratio:.2f}x the bound); worst row {i} "
                                 f"col {j}: gpu {g[i, j]:.6e} oracle {o[i, j]:.6e} A {A[i, j]:.3e}")
        nrm = np.linalg.norm(o)
        rl2 = np.linalg.norm(g - o) / nrm if nrm > 0 else np.linalg.norm(g)
        assert rl2 <= rel, f"grad {k}: relative L2 {rl2:.3e}"
        report[k] = float(rl2)
        # largest |g - g_o| as a fraction of its bound (zero bounds: exact)
        pos = tol > 0
        report[k + "_worst_of_bound"] = float((np.abs(g - o)[pos] / tol[pos]).max(initial=0.0))
    return report
