"""Brute-force NumPy/SciPy versions of each step, for tiny inputs only.

They pin the C oracle: every function here is built from a different route
than the oracle's plain loops (library least squares, scipy.ndimage
interpolation and filters, sorting), so a slip in either shows up as a
mismatch. FP64 throughout.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def pyr_down(img):
    """Binomial [1 4 6 4 1]/16 blur in each axis (replicate border), even samples."""
    k = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0
    b = ndimage.correlate1d(np.asarray(img, np.float64), k, axis=0, mode="nearest")
    b = ndimage.correlate1d(b, k, axis=1, mode="nearest")
    return b[::2, ::2]


def poly_expand(img, poly_n=5, sigma=1.1):
    """Per-pixel weighted least squares by numpy's lstsq on the padded image.

    Returns (5, h, w): rx, ry, rxx, ryy, rxy of f ~ c + rx x + ry y + rxx x^2
    + ryy y^2 + rxy x y around each pixel (x = column offset, y = row offset).
    """
    n = poly_n // 2
    img = np.asarray(img, np.float64)
    h, w = img.shape
    pad = np.pad(img, n, mode="edge")
    t = np.arange(-n, n + 1, dtype=np.float64)
    yy, xx = np.meshgrid(t, t, indexing="ij")
    wgt = np.exp(-(xx ** 2) / (2 * sigma ** 2)) * np.exp(-(yy ** 2) / (2 * sigma ** 2))
    B = np.stack([np.ones_like(xx), xx, yy, xx * xx, yy * yy, xx * yy], axis=-1).reshape(-1, 6)
    sw = np.sqrt(wgt).reshape(-1)
    # all windows as columns: (side^2, h*w)
    side = 2 * n + 1
    win = np.empty((side * side, h * w))
    for u in range(side):
        for v in range(side):
            win[u * side + v] = pad[u:u + h, v:v + w].reshape(-1)
    coef, *_ = np.linalg.lstsq(B * sw[:, None], win * sw[:, None], rcond=None)
    coef = coef.reshape(6, h, w)
    return np.stack([coef[1], coef[2], coef[3], coef[4], coef[5]])


def sample(plane, x, y):
    """Bilinear sample with the point clamped into the image (scipy, mode nearest)."""
    h, w = plane.shape
    xc = np.clip(x, 0, w - 1)
    yc = np.clip(y, 0, h - 1)
    return ndimage.map_coordinates(plane, [yc.ravel(), xc.ravel()], order=1, mode="nearest").reshape(np.shape(x))


def upsample(coarse, h, w):
    ii, jj = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    return np.stack([2 * sample(coarse[..., 0], jj / 2, ii / 2), 2 * sample(coarse[..., 1], jj / 2, ii / 2)], -1)


def update_terms(r1, r2, flow):
    _, h, w = r1.shape
    ii, jj = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    xs, ys = jj + flow[..., 0], ii + flow[..., 1]
    s = np.stack([sample(r2[k], xs, ys) for k in range(5)])
    # A as (h, w, 2, 2), b as (h, w, 2)
    def amat(r):
        return np.stack([np.stack([r[2], r[4] / 2], -1), np.stack([r[4] / 2, r[3]], -1)], -2)
    A = 0.5 * (amat(r1) + amat(s))
    b1 = np.stack([r1[0], r1[1]], -1)
    b2 = np.stack([s[0], s[1]], -1)
    db = -0.5 * (b2 - b1) + np.einsum("hwij,hwj->hwi", A, flow)
    G = np.einsum("hwki,hwkj->hwij", A, A)
    hv = np.einsum("hwki,hwk->hwi", A, db)
    return np.stack([G[..., 0, 0], G[..., 0, 1], G[..., 1, 1], hv[..., 0], hv[..., 1]])


def box_sum(planes, winsize):
    planes = np.asarray(planes, np.float64)
    out = np.empty_like(planes)
    for k in range(planes.shape[0]):
        out[k] = ndimage.uniform_filter(planes[k], size=winsize, mode="nearest") * (winsize * winsize)
    return out


def solve(gh, eps):
    """Per-pixel numpy solve where det >= eps tr^2; regularised formula elsewhere."""
    g11, g12, g22, h1, h2 = gh
    tr = g11 + g22
    det = g11 * g22 - g12 * g12
    out = np.zeros(g11.shape + (2,))
    well = (tr != 0) & (det >= eps * tr * tr)
    if well.any():
        G = np.stack([np.stack([g11, g12], -1), np.stack([g12, g22], -1)], -2)[well]
        hv = np.stack([h1, h2], -1)[well]
        out[well] = np.linalg.solve(G, hv[..., None])[..., 0]
    ill = (tr != 0) & ~well
    if ill.any():
        den = eps * tr[ill] ** 2
        out[ill, 0] = (g22[ill] * h1[ill] - g12[ill] * h2[ill]) / den
        out[ill, 1] = (g11[ill] * h2[ill] - g12[ill] * h1[ill]) / den
    return out


def flow(prev, next, levels=3, winsize=15, iterations=3, poly_n=5, poly_sigma=1.1, eps=1e-3, init=None):
    p = [np.asarray(prev, np.float64)]
    q = [np.asarray(next, np.float64)]
    for _ in range(1, levels):
        p.append(pyr_down(p[-1]))
        q.append(pyr_down(q[-1]))
    d = None
    for l in range(levels - 1, -1, -1):
        h, w = p[l].shape
        r1 = poly_expand(p[l], poly_n, poly_sigma)
        r2 = poly_expand(q[l], poly_n, poly_sigma)
        if d is None:
            d = np.zeros((h, w, 2))
            if init is not None:
                s = 2 ** l
                H, W = init.shape[:2]
                ii = np.minimum(np.arange(h) * s, H - 1)
                jj = np.minimum(np.arange(w) * s, W - 1)
                d = init[ii][:, jj] / s
        else:
            d = upsample(d, h, w)
        for _ in range(iterations):
            gh = box_sum(update_terms(r1, r2, d), winsize)
            d = solve(gh, eps)
    return d


def threshold_top(flow, q):
    m2 = flow[..., 0] ** 2 + flow[..., 1] ** 2
    k = int(np.floor(q * m2.size))
    t = np.sort(m2.ravel())[::-1][k]
    return (m2 > t).astype(np.uint8), t


def structuring_element(r, shape):
    u = np.arange(-r, r + 1)
    if shape == 0:
        return np.ones((2 * r + 1, 2 * r + 1), bool)
    return (u[:, None] ** 2 + u[None, :] ** 2) <= r * r


def dilate(pre, r, shape=0):
    if r == 0:
        return pre.astype(np.uint8).copy()
    return ndimage.binary_dilation(pre.astype(bool), structure=structuring_element(r, shape),
                                   border_value=0).astype(np.uint8)
