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
