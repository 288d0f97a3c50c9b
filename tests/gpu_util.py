"""Helpers shared by the GPU tests: device selection and the mask band rule."""
import numpy as np
import pytest
import torch

import bruteforce as bf

# FP32 flow tolerance against the FP64 oracle (pixels).
DELTA = 1e-3


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def band_mask(m_ref, tau_ref, width):
    """Pixels whose reference magnitude lies within `width` of the threshold."""
    return np.abs(m_ref - tau_ref) <= width


def check_mask(mask_gpu, flow_ref, tau2_ref, radius, shape, width):
    """GPU and oracle masks must agree wherever the structuring element placed
    at the pixel touches no band pixel. Returns (#checked, #band pixels)."""
    from oracle import dilate
    m_ref = np.hypot(flow_ref[..., 0], flow_ref[..., 1])
    tau = np.sqrt(tau2_ref)
    band = band_mask(m_ref, tau, width).astype(np.uint8)
    free = bf.dilate(band, radius, shape) == 0
    pre = (m_ref * m_ref > tau2_ref).astype(np.uint8)
    mask_ref = dilate(pre, radius, shape)
    bad = (mask_gpu != mask_ref) & free
    assert not bad.any(), "mask differs outside the threshold band at %d pixels, e.g. %s" % (
        bad.sum(), np.argwhere(bad)[:5].tolist())
    return int(free.sum()), int(band.sum())


# ---------------------------------------------------------------- the saliency rule

def oracle_chain(pre, p):
    """Opening/closing, small-component removal and dilation of a pre-mask,
    with the oracle, under the mask-stage fields of roi params p."""
    import oracle
    m = oracle.cc_filter(oracle.open_close(pre, p.morph_radius), p.min_area)
    return oracle.dilate(m, p.dilate_radius, p.se_shape)


def oracle_tau(s, p):
    if p.thresh_mode == 1:
        k = int(np.floor(float(np.float32(p.thresh)) * s.size))
        return np.sort(s.ravel())[::-1][k]
    return float(np.float32(p.thresh))


def check_sandwich(mask, s_ref, p, delta):
    """oracle(s > tau + delta) <= mask <= oracle(s > tau - delta): every step
    after the threshold is increasing in its input set. Returns the number
    of pixels where the two bounds differ."""
    tau = oracle_tau(s_ref, p)
    lo = oracle_chain((s_ref > tau + delta).astype(np.uint8), p)
    hi = oracle_chain((s_ref > tau - delta).astype(np.uint8), p)
    assert not (lo & (1 - mask)).any(), "GPU mask misses %d pixels of the lower bound" % (lo & (1 - mask)).sum()
    assert not (mask & (1 - hi)).any(), "GPU mask exceeds the upper bound at %d pixels" % (mask & (1 - hi)).sum()
    return int((hi != lo).sum())


def saliency_delta(flow_ref, flow_err, weight):
    """Bound on |s_gpu - s_oracle| implied by a flow error of flow_err per
    component (plus FP32 rounding): |dM| <= e, |dG| <= sqrt(2) e with
    e = sqrt(2) flow_err; each normalised term moves by at most twice its
    numerator's change over its (lowered) maximum."""
    e = np.sqrt(2.0) * flow_err
    M = np.hypot(flow_ref[..., 0], flow_ref[..., 1])
    P = np.pad(M, 1, mode="edge")
    G = np.hypot(0.5 * (P[1:-1, 2:] - P[1:-1, :-2]), 0.5 * (P[2:, 1:-1] - P[:-2, 1:-1]))
    da = 2 * e / (M.max() - e)
    db = 2 * np.sqrt(2) * e / (G.max() - np.sqrt(2) * e)
    eta = weight * da + (1 - weight) * db
    S = weight * M / M.max() + (1 - weight) * G / G.max()
    return 2 * eta / (S.max() - eta) + 1e-5
