"""FP64 oracle of the SSIM term of the photometric loss (Eq. 17):
L = (1 - lambda) L1 + lambda (1 - SSIM).

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg use this module; the library never does.

The paper names D-SSIM and the weight lambda (its value is in the absent
supplement); the readings (3DGS's form of the term):

* SSIM per channel with an 11 x 11 Gaussian window (sigma 1.5, normalised to
  sum 1) over the zero-padded image (a window reaching past the border sees
  zeros there, in x as in y: the seam is not wrapped);
* mu_x = sum w x, mu_y = sum w y, s_xx = sum w x^2 - mu_x^2, s_yy likewise,
  s_xy = sum w x y - mu_x mu_y, with C1 = 0.01^2, C2 = 0.03^2:
  S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2));
* SSIM = mean of S over channels and pixels; the term is 1 - SSIM.

A loss mask m [H, W] (Sec. 4: the 360Roam evaluation leaves the images'
bottom rows out of the loss) weights both terms per pixel: L1 =
sum m |x - y| / (C sum m), SSIM = sum m S / (C sum m), with the windows still
taken over the whole (zero-padded) images.
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    """Separable Gaussian window w[a, b] = g[a] g[b], sum 1."""
    k = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-k * k / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def _window_sums(img, w):
    """out[c, i, j] = sum_{a,b} w[a, b] img[c, i + a - r, j + b - r], zero
    outside the image (r = half the window)."""
    img = np.asarray(img, np.float64)
    r = w.shape[0] // 2
    C, H, W = img.shape
    pad = np.zeros((C, H + 2 * r, W + 2 * r))
    pad[:, r:r + H, r:r + W] = img
    out = np.zeros((C, H, W))
    for a in range(w.shape[0]):
        for b in range(w.shape[1]):
            out += w[a, b] * pad[:, a:a + H, b:b + W]
    return out


def ssim_terms(x, y, w=None):
    """Per-pixel statistics and the SSIM map S [C, H, W]."""
    w = window() if w is None else w
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = _window_sums(x, w), _window_sums(y, w)
    sxx = _window_sums(x * x, w) - mx * mx
    syy = _window_sums(y * y, w) - my * my
    sxy = _window_sums(x * y, w) - mx * my
    num1, num2 = 2 * mx * my + C1, 2 * sxy + C2
    den1, den2 = mx * mx + my * my + C1, sxx + syy + C2
    S = num1 * num2 / (den1 * den2)
    return dict(mx=mx, my=my, sxx=sxx, syy=syy, sxy=sxy, num1=num1, num2=num2, den1=den1, den2=den2, S=S)


def ssim(x, y, w=None) -> float:
    return float(ssim_terms(x, y, w)["S"].mean())


def dssim_grad(x, y, w=None, mask=None):
    """(1 - SSIM, d(1 - SSIM)/dx).  For a window centred at q, S(q) depends
    on x through mu_x(q), s_xx(q), s_xy(q); x_p enters them with weight
    w(p - q): d mu_x(q)/dx_p = w, d s_xx(q)/dx_p = 2 w (x_p - mu_x(q)),
    d s_xy(q)/dx_p = w (y_p - mu_y(q)).  The gradient sums these over the
    windows that contain p.  With a mask, S(q) enters with weight m(q) and
    the mean is over C sum m."""
    w = window() if w is None else w
    t = ssim_terms(x, y, w)
    m = np.ones(t["S"].shape[1:]) if mask is None else np.asarray(mask, np.float64)
    N = t["S"].shape[0] * m.sum()
    # partials of S(q), weighted by the mask at q
    dS_dmx = ((2 * t["my"] * t["num2"]) / (t["den1"] * t["den2"]) - t["S"] * 2 * t["mx"] / t["den1"]) * m
    dS_dsxx = -t["S"] / t["den2"] * m
    dS_dsxy = 2 * t["num1"] / (t["den1"] * t["den2"]) * m
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    C, H, W = x.shape
    r = w.shape[0] // 2
    grad = np.zeros((C, H, W))
    # scatter each window's partials back onto its pixels (zero padding: only
    # pixels inside the image receive gradient)
    for a in range(w.shape[0]):
        for b in range(w.shape[1]):
            # window centred at q = p - (a - r, b - r) reaches p with weight w[a, b]
            wq = w[a, b]
            qi0, qi1 = max(0, r - a), min(H, H + r - a)   # rows of q whose p = q + a - r lies inside
            qj0, qj1 = max(0, r - b), min(W, W + r - b)
            pi0, pj0 = qi0 + a - r, qj0 + b - r
            sl_q = (slice(None), slice(qi0, qi1), slice(qj0, qj1))
            sl_p = (slice(None), slice(pi0, pi0 + qi1 - qi0), slice(pj0, pj0 + qj1 - qj0))
            xp, yp = x[sl_p], y[sl_p]
            grad[sl_p] += wq * (dS_dmx[sl_q] + dS_dsxx[sl_q] * 2 * (xp - t["mx"][sl_q])
                                + dS_dsxy[sl_q] * (yp - t["my"][sl_q]))
    return 1.0 - float((t["S"] * m).sum() / N), -grad / N


def photometric(x, y, lam: float, w=None, mask=None):
    """(L, dL/dx) for L = (1 - lam) L1 + lam (1 - SSIM), each the mean over
    channels and pixels, weighted by ``mask`` [H, W] when given."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    m = np.ones(x.shape[1:]) if mask is None else np.asarray(mask, np.float64)
    n = x.shape[0] * m.sum()
    l1 = float((np.abs(x - y) * m).sum() / n)
    g1 = np.sign(x - y) * m / n
    d, gd = dssim_grad(x, y, w, mask)
    return (1 - lam) * l1 + lam * d, (1 - lam) * g1 + lam * gd
