"""Seeded synthetic moving-cell frames.

This module only draws inputs. It holds none of the flow / threshold /
dilation arithmetic, so both the HIP path and the FP64 oracle can be fed from
it without sharing any of the method's code.

The paper's data (ComplexEye videos of migrating neutrophils, Experimental
setup section) is not available. These frames stand in for it: a flat
background with additive Gaussian noise, plus Gaussian-blob "cells" that move
between frames. The recipes:

* ``pair_512_u8(seed)``: one 512x512 uint8 pair. Background 128, noise
  sigma 3 (drawn independently per frame), 20 blobs with sigma ~ U[4, 8] px
  and amplitude ~ U[40, 80], centres ~ U[3 sigma, 512 - 3 sigma]^2, each blob
  displaced by a vector drawn uniformly from the disc |d| <= 3 px. Rounded
  and clipped to [0, 255].
* ``sequence_u16(h, w, n_frames, n_blobs, seed)``: 12-bit frames stored as
  uint16. Background 1200, noise sigma 25, blob sigma ~ U[5, 10] px, amplitude
  ~ U[375, 750] (the same amplitude / background ratio as the uint8 recipe).
  90 % of the blobs random-walk with step N(0, 1.5^2 I) per frame, 10 % stay
  put. Clipped to [0, 4095].
* ``lens_streams(...)``: the 16-stream mix of frame sizes
  {1024^2, 1536^2, 2048^2, 2448(W) x 2048(H)}, round-robin, with
  200 * area / 2048^2 blobs per stream and seeds 200 + stream index.

* ``flow_field(h, w, seed)``: a synthetic flow field for the mask stage
  alone: a smooth background drift (two ``smooth_texture`` fields with sigma
  8 px scaled to std 0.3 px) plus n_cells discs of radius ~ U[6, 20] px
  moving with velocity drawn from the disc |v| <= 4 px, float32.
* ``binary_pattern(h, w, kind, seed)``: uint8 0/1 patterns for the
  morphology and component stages ("noise": i.i.d. with density 0.5;
  "blobs": smoothed noise above its 70 % quantile; "snake": one 1-px wide
  path winding over the whole frame; "full"; "empty"; "dot": one pixel).

* ``drifting_frames(h, w, drifts, seed)``: frames under global translational
  drift, for the stabilisation stage. One canvas (background 1200, a
  ``smooth_texture`` field of sigma 2 px and std 150, 200 * area / 2048^2
  Gaussian-blob cells as in ``sequence_u16``) is cut at offsets that move by
  the integer drifts, so frame t is frame t-1 moved by drifts[t-1]
  (next(x) = prev(x - s)); independent Gaussian noise (sigma 25) per frame;
  uint16, clipped to [0, 4095].

All randomness comes from numpy's PCG64 generator seeded explicitly.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "render_frame",
    "pair_512_u8",
    "sequence_u16",
    "lens_stream_sizes",
    "lens_streams",
    "smooth_texture",
    "flow_field",
    "binary_pattern",
    "drifting_frames",
]

# Blobs are rendered inside +-5 sigma; the Gaussian tail beyond is < 4e-6 of
# the amplitude (below 0.003 grey levels for the largest amplitude used).
_BLOB_EXTENT = 5.0


def render_frame(h, w, background, noise_sigma, centres, sigmas, amps, rng):
    """Float64 frame: background + iid N(0, noise_sigma^2) + Gaussian blobs.

    ``centres`` is an (n, 2) array of (row, col) blob centres in pixels.
    """
    img = background + noise_sigma * rng.standard_normal((h, w))
    for (cy, cx), s, a in zip(centres, sigmas, amps):
        r = _BLOB_EXTENT * s
        y0, y1 = max(int(np.floor(cy - r)), 0), min(int(np.ceil(cy + r)) + 1, h)
        x0, x1 = max(int(np.floor(cx - r)), 0), min(int(np.ceil(cx + r)) + 1, w)
        if y0 >= y1 or x0 >= x1:
            continue
        yy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy
        xx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx
        img[y0:y1, x0:x1] += a * np.exp(-(yy * yy + xx * xx) / (2.0 * s * s))
    return img


def _quantise(img, vmax, dtype):
    return np.clip(np.rint(img), 0, vmax).astype(dtype)


def pair_512_u8(seed, size=512, n_blobs=20, max_disp=3.0):
    """One uint8 frame pair; returns (prev, next, displacements (n, 2) as (dy, dx))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sig = rng.uniform(4.0, 8.0, n_blobs)
    amp = rng.uniform(40.0, 80.0, n_blobs)
    cy = rng.uniform(3.0 * sig, size - 3.0 * sig)
    cx = rng.uniform(3.0 * sig, size - 3.0 * sig)
    rad = max_disp * np.sqrt(rng.uniform(0.0, 1.0, n_blobs))
    ang = 2.0 * np.pi * rng.uniform(0.0, 1.0, n_blobs)
    disp = np.stack([rad * np.sin(ang), rad * np.cos(ang)], axis=1)
    c0 = np.stack([cy, cx], axis=1)
    f0 = render_frame(size, size, 128.0, 3.0, c0, sig, amp, rng)
    f1 = render_frame(size, size, 128.0, 3.0, c0 + disp, sig, amp, rng)
    return _quantise(f0, 255, np.uint8), _quantise(f1, 255, np.uint8), disp


def sequence_u16(h, w, n_frames, n_blobs, seed, static_frac=0.1, step_sigma=1.5,
                 background=1200.0, noise_sigma=25.0, sig_range=(5.0, 10.0),
                 amp_range=(375.0, 750.0)):
    """A (n_frames, h, w) uint16 sequence of 12-bit frames with random-walk blobs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sig = rng.uniform(sig_range[0], sig_range[1], n_blobs)
    amp = rng.uniform(amp_range[0], amp_range[1], n_blobs)
    cy = rng.uniform(3.0 * sig, h - 3.0 * sig)
    cx = rng.uniform(3.0 * sig, w - 3.0 * sig)
    moving = rng.uniform(0.0, 1.0, n_blobs) >= static_frac
    pos = np.stack([cy, cx], axis=1)
    out = np.empty((n_frames, h, w), dtype=np.uint16)
    for t in range(n_frames):
        if t > 0:
            step = step_sigma * rng.standard_normal((n_blobs, 2))
            pos = pos + step * moving[:, None]
        out[t] = _quantise(render_frame(h, w, background, noise_sigma, pos, sig, amp, rng),
                           4095, np.uint16)
    return out


def lens_stream_sizes(n_streams=16):
    """(h, w) of each stream: round-robin over the four lens frame sizes."""
    sizes = [(1024, 1024), (1536, 1536), (2048, 2048), (2048, 2448)]
    return [sizes[i % 4] for i in range(n_streams)]


def lens_streams(n_streams=16, n_frames=2, seed0=200):
    """List of per-stream uint16 sequences with uneven frame sizes."""
    out = []
    for i, (h, w) in enumerate(lens_stream_sizes(n_streams)):
        nb = max(1, int(round(200.0 * h * w / (2048.0 * 2048.0))))
        out.append(sequence_u16(h, w, n_frames, nb, seed0 + i))
    return out


def smooth_texture(h, w, seed, sigma=2.0, amplitude=100.0, pad=16):
    """Float64 random texture low-passed by a Gaussian of ``sigma`` px.

    Returned with ``pad`` extra pixels on every side so that callers can cut
    integer-shifted windows out of one underlying field.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W = h + 2 * pad, w + 2 * pad
    noise = rng.standard_normal((H, W))
    r = int(np.ceil(4 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-t * t / (2 * sigma * sigma))
    k /= k.sum()
    # circular separable smoothing; the wrap keeps the field stationary
    f = np.zeros_like(noise)
    for i, kv in zip(range(-r, r + 1), k):
        f += kv * np.roll(noise, i, axis=0)
    g = np.zeros_like(f)
    for i, kv in zip(range(-r, r + 1), k):
        g += kv * np.roll(f, i, axis=1)
    g *= amplitude / g.std()
    return g


def flow_field(h, w, seed, n_cells=None, max_speed=4.0):
    """Synthetic (h, w, 2) float32 flow: smooth drift plus moving discs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n_cells is None:
        n_cells = max(1, h * w // 8000)
    f = np.zeros((h, w, 2))
    for c in range(2):
        f[..., c] = 0.1 * smooth_texture(h, w, seed * 7 + c, sigma=8.0, amplitude=3.0, pad=0)
    yy, xx = np.mgrid[0:h, 0:w]
    for _ in range(n_cells):
        r = rng.uniform(6, 20)
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        ang, mag = rng.uniform(0, 2 * np.pi), max_speed * np.sqrt(rng.uniform())
        inside = (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
        f[inside, 0] = mag * np.cos(ang)
        f[inside, 1] = mag * np.sin(ang)
    return f.astype(np.float32)


def binary_pattern(h, w, kind, seed=0):
    """uint8 0/1 test patterns (see the module docstring)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "noise":
        return (rng.uniform(size=(h, w)) < 0.5).astype(np.uint8)
    if kind == "blobs":
        t = smooth_texture(h, w, seed, sigma=3.0, pad=0)
        return (t > np.quantile(t, 0.7)).astype(np.uint8)
    if kind == "snake":
        m = np.zeros((h, w), np.uint8)
        for y in range(0, h, 4):
            m[y, :] = 1
            x = w - 1 if (y // 4) % 2 == 0 else 0
            m[y:y + 4, x] = 1
        return m
    if kind == "full":
        return np.ones((h, w), np.uint8)
    if kind == "empty":
        return np.zeros((h, w), np.uint8)
    if kind == "dot":
        m = np.zeros((h, w), np.uint8)
        m[h // 2, w // 2] = 1
        return m
    raise ValueError(kind)


def drifting_frames(h, w, drifts, seed, noise_sigma=25.0):
    """len(drifts) + 1 uint16 frames; frame t+1 is frame t moved by drifts[t]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cum = [(0, 0)]
    for dy, dx in drifts:
        cum.append((cum[-1][0] + int(dy), cum[-1][1] + int(dx)))
    pad_y = max(abs(c[0]) for c in cum) + 1
    pad_x = max(abs(c[1]) for c in cum) + 1
    H, W = h + 2 * pad_y, w + 2 * pad_x
    canvas = 1200.0 + smooth_texture(H, W, seed + 1, sigma=2.0, amplitude=150.0, pad=0)
    n_blobs = max(1, int(200 * H * W / 2048 ** 2))
    sig = rng.uniform(5, 10, n_blobs)
    cen = np.stack([rng.uniform(0, H, n_blobs), rng.uniform(0, W, n_blobs)], 1)
    amp = rng.uniform(375, 750, n_blobs)
    canvas = canvas + render_frame(H, W, 0.0, 0.0, cen, sig, amp, rng)
    out = []
    for cy, cx in cum:
        # frame(x) = canvas(x - c + pad): moving the cut by -c moves the content by +c
        f = canvas[pad_y - cy:pad_y - cy + h, pad_x - cx:pad_x - cx + w]
        f = f + rng.normal(0.0, noise_sigma, (h, w))
        out.append(np.clip(np.rint(f), 0, 4095).astype(np.uint16))
    return np.stack(out)
