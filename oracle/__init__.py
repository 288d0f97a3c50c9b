"""FP64 CPU oracle of the FlowRoI flow -> RoI-mask hot path.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's CPU
baseline leg import this package. The product library never loads it, and it
shares no code with the HIP path: the computation lives in
``flowroi_oracle.c`` (plain C, double precision), compiled with gcc into
``oracle/_build/libflowroi_oracle.so``; this module only marshals numpy
arrays into it.

Readings of the paper (FlowRoI, Method section; the estimator is Farneback's
two-frame polynomial-expansion method, whose constants the paper leaves
open) are stated in the C file's header. Defaults below are the frozen
constants both implementations use: 3 pyramid levels, 5x5 expansion with
sigma 1.1, 15x15 box window, 3 iterations per level, eps 1e-3, square
dilation of radius 2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flowroi_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libflowroi_oracle.so")
_lock = threading.Lock()
_lib = None

DEFAULTS = dict(levels=3, winsize=15, iterations=3, poly_n=5, poly_sigma=1.1, eps=1e-3,
                thresh_mode=0, thresh=1.0, dilate_radius=2, se_shape=0)

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force=False):
    """Compile the oracle with gcc (OpenMP over rows). Returns the .so path."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            i, d, sz = ctypes.c_int, ctypes.c_double, ctypes.c_size_t
            lib.orc_pyr_down.argtypes = [_dp, i, i, _dp]
            lib.orc_poly_expand.argtypes = [_dp, i, i, i, d, _dp]
            lib.orc_poly_expand.restype = i
            lib.orc_bilinear.argtypes = [_dp, i, i, d, d]
            lib.orc_bilinear.restype = d
            lib.orc_flow_upsample.argtypes = [_dp, i, i, _dp, i, i]
            lib.orc_update_terms.argtypes = [_dp, _dp, _dp, i, i, _dp]
            lib.orc_box_sum.argtypes = [_dp, i, i, i, i, _dp]
            lib.orc_solve.argtypes = [_dp, i, i, d, _dp]
            lib.orc_flow.argtypes = [_dp, _dp, i, i, i, i, i, i, d, d, _dp, _dp]
            lib.orc_flow.restype = i
            lib.orc_threshold_abs.argtypes = [_dp, sz, d, _u8p]
            lib.orc_threshold_top.argtypes = [_dp, sz, d, _u8p, _dp]
            lib.orc_threshold_top.restype = i
            lib.orc_dilate.argtypes = [_u8p, i, i, i, i, _u8p]
            lib.orc_dilate.restype = i
            lib.orc_roi_mask.argtypes = [_dp, _dp, i, i, i, i, i, i, d, d, _dp, i, d, i, i, _dp, _u8p, _dp]
            lib.orc_roi_mask.restype = i
            lib.orc_num_threads.restype = i
            lib.orc_median.argtypes = [_dp, i, i, i, _dp]
            lib.orc_bilateral.argtypes = [_dp, i, i, i, d, d, _dp]
            lib.orc_denoise.argtypes = [_dp, i, i, i, i, d, d, _dp]
            lib.orc_denoise.restype = i
            lib.orc_saliency.argtypes = [_dp, i, i, d, _dp]
            lib.orc_open_close.argtypes = [_u8p, i, i, i, _u8p]
            lib.orc_cc_filter.argtypes = [_u8p, i, i, i, _u8p]
            _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def _check(rc):
    if rc != 0:
        raise ValueError("oracle returned status %d" % rc)


def num_threads():
    return _load().orc_num_threads()


def pyr_down(img):
    img = _f64(img)
    h, w = img.shape
    out = np.empty(((h + 1) // 2, (w + 1) // 2))
    _load().orc_pyr_down(_ptr(img), h, w, _ptr(out))
    return out


def poly_expand(img, poly_n=5, poly_sigma=1.1):
    """(5, h, w): rx, ry, rxx, ryy, rxy of the local quadratic fit."""
    img = _f64(img)
    h, w = img.shape
    out = np.empty((5, h, w))
    _check(_load().orc_poly_expand(_ptr(img), h, w, poly_n // 2, float(poly_sigma), _ptr(out)))
    return out


def bilinear(plane, x, y):
    plane = _f64(plane)
    h, w = plane.shape
    return _load().orc_bilinear(_ptr(plane), h, w, float(x), float(y))


def flow_upsample(coarse, h, w):
    coarse = _f64(coarse)
    hc, wc, _ = coarse.shape
    out = np.empty((h, w, 2))
    _load().orc_flow_upsample(_ptr(coarse), hc, wc, _ptr(out), h, w)
    return out


def update_terms(r1, r2, flow):
    """(5, h, w): G11, G12, G22, h1, h2 per pixel for prior flow (h, w, 2)."""
    r1, r2, flow = _f64(r1), _f64(r2), _f64(flow)
    _, h, w = r1.shape
    out = np.empty((5, h, w))
    _load().orc_update_terms(_ptr(r1), _ptr(r2), _ptr(flow), h, w, _ptr(out))
    return out


def box_sum(planes, winsize):
    planes = _f64(planes)
    k, h, w = planes.shape
    out = np.empty_like(planes)
    _load().orc_box_sum(_ptr(planes), k, h, w, int(winsize), _ptr(out))
    return out


def solve(gh, eps=DEFAULTS["eps"]):
    gh = _f64(gh)
    _, h, w = gh.shape
    out = np.empty((h, w, 2))
    _load().orc_solve(_ptr(gh), h, w, float(eps), _ptr(out))
    return out


def flow(prev, next, levels=3, winsize=15, iterations=3, poly_n=5, poly_sigma=1.1, eps=1e-3, init=None):
    """Dense flow prev -> next, (h, w, 2) as (dx, dy) per pixel."""
    p, q = _f64(prev), _f64(next)
    h, w = p.shape
    out = np.empty((h, w, 2))
    ip = None
    if init is not None:
        init = _f64(init)
        ip = _ptr(init)
    _check(_load().orc_flow(_ptr(p), _ptr(q), h, w, levels, winsize, iterations, poly_n,
                            float(poly_sigma), float(eps), ip, _ptr(out)))
    return out


def threshold_abs(flow, tau):
    flow = _f64(flow)
    n = flow.size // 2
    pre = np.empty(flow.shape[:-1], dtype=np.uint8)
    _load().orc_threshold_abs(_ptr(flow), n, float(tau), _ptr(pre, _u8p))
    return pre


def threshold_top(flow, q):
    """Returns (pre-mask, tau^2)."""
    flow = _f64(flow)
    n = flow.size // 2
    pre = np.empty(flow.shape[:-1], dtype=np.uint8)
    t2 = ctypes.c_double(0.0)
    _check(_load().orc_threshold_top(_ptr(flow), n, float(q), _ptr(pre, _u8p), ctypes.byref(t2)))
    return pre, t2.value


def dilate(pre, radius=2, shape=0):
    pre = np.ascontiguousarray(pre, dtype=np.uint8)
    h, w = pre.shape
    out = np.empty_like(pre)
    _check(_load().orc_dilate(_ptr(pre, _u8p), h, w, int(radius), int(shape), _ptr(out, _u8p)))
    return out


def median(img, radius=1):
    img = _f64(img)
    h, w = img.shape
    out = np.empty_like(img)
    _load().orc_median(_ptr(img), h, w, int(radius), _ptr(out))
    return out


def bilateral(img, radius=2, sigma_space=1.5, sigma_range=20.0):
    img = _f64(img)
    h, w = img.shape
    out = np.empty_like(img)
    _load().orc_bilateral(_ptr(img), h, w, int(radius), float(sigma_space), float(sigma_range), _ptr(out))
    return out


def denoise(img, median_radius=1, bilateral_radius=2, sigma_space=1.5, sigma_range=20.0):
    """Median then bilateral filter (FlowRoI's two-step denoising)."""
    img = _f64(img)
    h, w = img.shape
    out = np.empty_like(img)
    _check(_load().orc_denoise(_ptr(img), h, w, int(median_radius), int(bilateral_radius), float(sigma_space),
                               float(sigma_range), _ptr(out)))
    return out


def saliency(flow, weight=0.7):
    """Normalised motion saliency of a flow field (h, w, 2) -> (h, w)."""
    flow = _f64(flow)
    h, w = flow.shape[:2]
    out = np.empty((h, w))
    _load().orc_saliency(_ptr(flow), h, w, float(weight), _ptr(out))
    return out


def open_close(pre, radius=1):
    pre = np.ascontiguousarray(pre, dtype=np.uint8)
    h, w = pre.shape
    out = np.empty_like(pre)
    _load().orc_open_close(_ptr(pre, _u8p), h, w, int(radius), _ptr(out, _u8p))
    return out


def cc_filter(mask, min_area):
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    h, w = mask.shape
    out = np.empty_like(mask)
    _load().orc_cc_filter(_ptr(mask, _u8p), h, w, int(min_area), _ptr(out, _u8p))
    return out


def saliency_mask(flow, thresh_mode=1, thresh=0.2, weight=0.7, morph_radius=1, min_area=32, dilate_radius=2,
                  se_shape=0):
    """The paper's RoI rule on a flow field: saliency -> threshold (top
    fraction or absolute on the normalised saliency) -> opening + closing ->
    small-component removal -> dilation. Returns (mask, saliency, tau)."""
    s = saliency(flow, weight)
    if thresh_mode == 1:
        k = int(np.floor(float(thresh) * s.size))
        tau = np.sort(s.ravel())[::-1][k]
    else:
        tau = float(thresh)
    pre = (s > tau).astype(np.uint8)
    m = cc_filter(open_close(pre, morph_radius), min_area)
    return dilate(m, dilate_radius, se_shape), s, tau


# ---------------------------------------------------------------- stabilisation

PHASE_MAX = 2048


def phase_size(h, w):
    """Side P of the square window the translation is estimated on: the
    largest power of two <= min(h, w, 2048); 0 when the frame is thinner
    than 2 pixels."""
    m = min(h, w, PHASE_MAX)
    if m < 2:
        return 0
    return 1 << (int(m).bit_length() - 1)


def hann(n):
    """Symmetric Hann window of n points: 0.5 (1 - cos(2 pi i / (n - 1)))."""
    i = np.arange(n, dtype=np.float64)
    return 0.5 * (1.0 - np.cos(2.0 * np.pi * i / (n - 1)))


def phase_correlation(prev, next):
    """Phase-correlation surface of two frames (FlowRoI, Method, optical
    flow extraction: frames are registered to their predecessor by phase
    correlation). Both frames are cut to the centred P x P window and
    multiplied by the separable Hann window; with A, B their 2-D DFTs,
    r = IDFT(B conj(A) / |B conj(A)|) (0 where the product is 0). If next
    is prev moved by s (next(x) = prev(x - s)), then B = A e^{-2 pi i k s / P},
    the normalised product is that phase ramp alone and r peaks at s
    modulo P.
    Returns (r, P, y0, x0) with (y0, x0) the window's corner."""
    a, b = _f64(prev), _f64(next)
    h, w = a.shape
    P = phase_size(h, w)
    y0, x0 = (h - P) // 2, (w - P) // 2
    win = np.outer(hann(P), hann(P))
    A = np.fft.fft2(a[y0:y0 + P, x0:x0 + P] * win)
    B = np.fft.fft2(b[y0:y0 + P, x0:x0 + P] * win)
    X = B * np.conj(A)
    mag = np.abs(X)
    R = np.where(mag > 0, X / np.where(mag > 0, mag, 1.0), 0.0)
    return np.fft.ifft2(R).real, P, y0, x0


def phase_shift(prev, next):
    """Integer translation (sy, sx) of next relative to prev: the position of
    the largest value of the phase-correlation surface (the first in row-major
    order on ties), indices at or above P/2 read as negative. Returns
    (sy, sx, peak value); (0, 0, 0.0) for frames thinner than 2 pixels."""
    h, w = np.shape(prev)
    if phase_size(h, w) == 0:
        return 0, 0, 0.0
    r, P, _, _ = phase_correlation(prev, next)
    k = int(np.argmax(r))
    py, px = divmod(k, P)
    sy = py - P if py >= P // 2 else py
    sx = px - P if px >= P // 2 else px
    return sy, sx, float(r.flat[k])


def align(next, sy, sx):
    """next moved back by (sy, sx): out(y, x) = next(y + sy, x + sx), the
    coordinates clamped into the frame (replicated edges)."""
    q = _f64(next)
    h, w = q.shape
    ys = np.clip(np.arange(h) + sy, 0, h - 1)
    xs = np.clip(np.arange(w) + sx, 0, w - 1)
    return q[np.ix_(ys, xs)]


def roi_mask(prev, next, levels=3, winsize=15, iterations=3, poly_n=5, poly_sigma=1.1, eps=1e-3,
             thresh_mode=0, thresh=1.0, dilate_radius=2, se_shape=0, init=None, denoise_params=None,
             stabilize=False):
    """Whole path: returns (flow (h, w, 2), mask (h, w) uint8 0/1, tau^2).
    denoise_params (dict of denoise()'s keywords) applies the denoising
    pre-stage to both frames first; stabilize then registers next to prev
    (phase_shift, align) before the flow, in the paper's order."""
    p, q = _f64(prev), _f64(next)
    if denoise_params is not None:
        p, q = denoise(p, **denoise_params), denoise(q, **denoise_params)
    if stabilize:
        sy, sx, _ = phase_shift(p, q)
        q = align(q, sy, sx)
    h, w = p.shape
    fl = np.empty((h, w, 2))
    mask = np.empty((h, w), dtype=np.uint8)
    t2 = ctypes.c_double(0.0)
    ip = None
    if init is not None:
        init = _f64(init)
        ip = _ptr(init)
    _check(_load().orc_roi_mask(_ptr(p), _ptr(q), h, w, levels, winsize, iterations, poly_n,
                                float(poly_sigma), float(eps), ip, int(thresh_mode), float(thresh),
                                int(dilate_radius), int(se_shape), _ptr(fl), _ptr(mask, _u8p),
                                ctypes.byref(t2)))
    return fl, mask, t2.value


def ensemble(masks, adjacent):
    """Adjacent-frame ensemble (FlowRoI, Region of Interest extraction; the
    adjacent factor of Table 1): the output for frame t is the union of the
    frame's own mask and those of the previous `adjacent` frames."""
    out = []
    for t in range(len(masks)):
        m = np.zeros_like(masks[t], dtype=np.uint8)
        for k in range(max(0, t - adjacent), t + 1):
            m |= masks[k].astype(np.uint8)
        out.append(m)
    return out
