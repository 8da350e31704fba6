"""Brute-force per-pixel ERP renderer in numpy (FP64), for tiny scenes.

TEST INFRASTRUCTURE ONLY.  A second, independent statement of the forward
pass, used to pin the tiled C oracle:

* no tiles and no radius of influence: every pixel visits every Gaussian in
  (depth, index) order (Eq. 6 and the depth criterion of Sec. 3.3: t_r for
  the ERP camera, t_z for the pinhole camera of Eq. 2);
* the Jacobian of Eq. 10 is taken by central finite differences of the
  projection (Eqs. 3-5, or Eq. 2 at the guarded direction) instead of closed
  forms;
* the rotation comes from scipy's quaternion conversion, the inverse 2D
  covariance from ``numpy.linalg.inv``;
* the SH basis comes from scipy's complex spherical harmonics
  (real form: sqrt2 Re / sqrt2 Im of Y_l^|m|, which carry the Condon-Shortley
  phase).

With ``records`` given (the C oracle's own projection), only the blending is
re-done, and the result must equal the tiled oracle exactly: the radius of
influence is the box of the alpha = alpha_min iso-ellipse, so tiling never
drops a contribution.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

try:  # scipy >= 1.15
    from scipy.special import sph_harm_y as _sph_y

    def _sph(m, l, polar, azim):
        return _sph_y(l, m, polar, azim)
except ImportError:  # pragma: no cover
    from scipy.special import sph_harm as _sph_old

    def _sph(m, l, polar, azim):
        return _sph_old(m, l, azim, polar)


def erp_project(t, W, H):
    """Eq. 3-5: camera-space point -> ERP pixel coordinates (x, y)."""
    lon = np.arctan2(t[..., 0], t[..., 2])
    lon = np.where(lon >= np.pi, -np.pi, lon)
    tr = np.linalg.norm(t, axis=-1)
    lat = np.arcsin(t[..., 1] / tr)
    return np.stack([(lon / np.pi + 1.0) * W / 2.0, (2.0 * lat / np.pi + 1.0) * H / 2.0], axis=-1)


def pinhole_project(t, fx, fy, cx, cy):
    """Eq. 2: camera-space point -> pinhole pixel coordinates (x, y)."""
    return np.stack([fx * t[..., 0] / t[..., 2] + cx, fy * t[..., 1] / t[..., 2] + cy], axis=-1)


def pinhole_guard(t, W, H, fx, fy, cx, cy):
    """The point at which the pinhole Jacobian is taken: t with its direction
    t_x / t_z, t_y / t_z clamped to 1.3 times the image's angular half-extent
    around the image's middle (3DGS's guard), at the same t_z."""
    lo_x, hi_x = (0.0 - cx) / fx, (W - cx) / fx
    lo_y, hi_y = (0.0 - cy) / fy, (H - cy) / fy
    mx, hx = 0.5 * (lo_x + hi_x), 0.65 * (hi_x - lo_x)
    my, hy = 0.5 * (lo_y + hi_y), 0.65 * (hi_y - lo_y)
    a = np.clip(t[0] / t[2], mx - hx, mx + hx)
    b = np.clip(t[1] / t[2], my - hy, my + hy)
    return np.array([a * t[2], b * t[2], t[2]])


def fd_jacobian(t, W, H, rel=1e-6, proj=None):
    """Central-difference Jacobian d p / d t (2x3) of Eq. 3-5 (or of the
    projection ``proj``)."""
    proj = proj or (lambda u: erp_project(u, W, H))
    J = np.zeros((2, 3))
    h = rel * np.linalg.norm(t)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (proj(t + e) - proj(t - e)) / (2.0 * h)
    return J


def real_sh(degree, d):
    """Real SH basis (index l*l + l + m) at unit direction d, via scipy."""
    x, y, z = d
    polar = np.arccos(np.clip(z, -1.0, 1.0))
    azim = np.arctan2(y, x)
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = _sph(abs(m), l, polar, azim)
            if m == 0:
                out.append(Y.real)
            elif m > 0:
                out.append(np.sqrt(2.0) * Y.real)
            else:
                out.append(np.sqrt(2.0) * Y.imag)
    return np.array(out, dtype=np.float64)


def project_independent(scene):
    """Per-Gaussian (visible, depth ("tr"), px, py, Q00, Q01, Q11, rgb)
    computed without the C oracle.  Returns a dict of arrays."""
    st = scene.settings
    n, W, H = scene.n, scene.width, scene.height
    out = dict(visible=np.zeros(n, bool), tr=np.zeros(n), px=np.zeros(n), py=np.zeros(n), Q=np.zeros((n, 3)),
               rgb=np.zeros((n, 3)))
    cam_centre = -scene.R.T @ scene.t
    pinhole = getattr(scene, "model", 0) == 1
    for i in range(n):
        t = scene.R @ scene.means[i] + scene.t
        tr = np.linalg.norm(t)
        rho = np.hypot(t[0], t[2])
        o = scene.opac[i]
        if pinhole:
            if t[2] <= st["near_plane"] or o <= st["alpha_min"]:
                continue
            proj = lambda u: pinhole_project(u, *scene.intrinsics)
            p = proj(t)
            J = fd_jacobian(pinhole_guard(t, W, H, *scene.intrinsics), W, H, proj=proj)
            depth = t[2]
        else:
            if tr <= st["near_plane"] or o <= st["alpha_min"] or rho <= 1e-6 * tr:
                continue
            p = erp_project(t, W, H)
            J = fd_jacobian(t, W, H)
            depth = tr
        q = scene.quats[i]
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sig = Rq @ np.diag(scene.scales[i] ** 2) @ Rq.T
        M = J @ scene.R
        cov = M @ Sig @ M.T + st["dilation"] * np.eye(2)
        if np.linalg.det(cov) <= 0:
            continue
        Q = np.linalg.inv(cov)
        d = scene.means[i] - cam_centre
        d = d / np.linalg.norm(d)
        Y = real_sh(scene.sh_degree, d)
        K = (scene.sh_degree + 1) ** 2
        rgb = np.maximum(Y @ scene.sh[i, :K, :] + 0.5, 0.0)
        out["visible"][i] = True
        out["tr"][i] = depth
        out["px"][i], out["py"][i] = p
        out["Q"][i] = (Q[0, 0], Q[0, 1], Q[1, 1])
        out["rgb"][i] = rgb
    return out


def render(scene, records=None, with_depth=False):
    """Per-pixel front-to-back blend over all Gaussians (no tiles).

    ``records``: the C oracle's projection records (exact tiling check) or
    None (independent projection).  Returns (image [3,H,W], final_T [H,W],
    n_blended [H,W]) and, with ``with_depth``, the depth image
    sum_i depth_i alpha_i T_i [H,W]; H is the rendered rows.
    """
    st = scene.settings
    W, H = scene.width, getattr(scene, "out_height", scene.height)
    if records is not None:
        vis = records[:, 0] > 0.5
        proj = dict(visible=vis, tr=records[:, 4], px=records[:, 7], py=records[:, 8], Q=records[:, 18:21],
                    rgb=records[:, 33:36])
    else:
        proj = project_independent(scene)
    ids = np.nonzero(proj["visible"])[0]
    order = ids[np.lexsort((ids, proj["tr"][ids]))]
    ys, xs = np.mgrid[0:H, 0:W]
    xc = xs.astype(np.float64) + 0.5
    yc = ys.astype(np.float64) + 0.5
    T = np.ones((H, W))
    C = np.zeros((3, H, W))
    active = np.ones((H, W), bool)
    nb = np.zeros((H, W), dtype=np.int64)
    D = np.zeros((H, W))
    wrap = getattr(scene, "model", 0) != 1  # the ERP seam; the pinhole image does not wrap
    for i in order:
        dx = xc - proj["px"][i]
        if wrap:
            dx = np.where(dx >= 0.5 * W, dx - W, dx)
            dx = np.where(dx < -0.5 * W, dx + W, dx)
        dy = yc - proj["py"][i]
        q00, q01, q11 = proj["Q"][i]
        power = -0.5 * (q00 * dx * dx + 2.0 * q01 * dx * dy + q11 * dy * dy)
        a = np.minimum(scene.opac[i] * np.exp(power), st["alpha_max"])
        take = active & (a >= st["alpha_min"])
        Tn = T * (1.0 - a)
        stop = take & (Tn < st["T_min"])
        active &= ~stop
        take &= ~stop
        for ch in range(3):
            C[ch] = np.where(take, C[ch] + proj["rgb"][i, ch] * a * T, C[ch])
        D = np.where(take, D + proj["tr"][i] * a * T, D)
        T = np.where(take, Tn, T)
        nb += take
    bg = np.asarray(st["bg"], dtype=np.float64)
    if with_depth:
        return C + T[None] * bg[:, None, None], T, nb, D
    return C + T[None] * bg[:, None, None], T, nb
