"""The saliency rule (Method, Region of Interest extraction) on the GPU,
against the FP64 oracle.

* Integer stages bit-exact: flows whose magnitude is a 0/1 pattern make the
  saliency decision unambiguous (magnitude-1 pixels have normalised saliency
  >= 0.7, the others <= 0.3 / 0.7), so opening, closing, component removal
  and dilation must reproduce the oracle's mask exactly.
* Saliency values: the normalised saliency of a given flow within a bound
  of FP32 rounding.
* Masks through the whole stage, and through the whole path, by the
  sandwich rule: every operation after the threshold (opening, closing,
  small-component removal, dilation) is increasing in its input set, so the
  GPU mask must contain the oracle's mask for the threshold raised by the
  saliency tolerance and lie inside the one for the threshold lowered by it.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DELTA, check_sandwich, device, saliency_delta, to_dev
from paper_2511_14419_amd import synth

pytestmark = pytest.mark.gpu


def F():
    from paper_2511_14419_amd import flowroi
    return flowroi


def params(**kw):
    fl = F()
    base = dict(rule=fl.ROI_RULE_SALIENCY, thresh_mode=1, thresh=0.2)
    base.update(kw)
    return fl.default_params(**base)


def gpu_stage(flow, **kw):
    fl = F()
    dev = device()
    m, s, ws = fl.mask_from_flow(to_dev(flow.astype(np.float32), dev), params(**kw), want_saliency=True)
    torch.cuda.synchronize()
    return m.cpu().numpy(), s.cpu().numpy().astype(np.float64)


# ---------------------------------------------------------------- integer stages, bit-exact

EXACT = [
    ((97, 203), "noise", 1, 1, 0, 0),
    ((97, 203), "noise", 0, 2, 1, 0),
    ((256, 320), "blobs", 1, 32, 2, 0),
    ((256, 320), "blobs", 2, 200, 3, 1),
    ((130, 1000), "snake", 0, 5000, 0, 0),
    ((130, 1000), "snake", 1, 50, 2, 1),
    ((64, 64), "full", 1, 4096, 2, 0),
    ((64, 64), "full", 1, 4097, 2, 0),
    ((300, 129), "empty", 1, 32, 2, 0),
    ((33, 35), "dot", 0, 1, 3, 1),
    ((33, 35), "dot", 0, 2, 3, 1),
    ((1, 1), "dot", 1, 1, 1, 0),
    ((1, 77), "noise", 1, 3, 1, 0),
    ((1030, 777), "blobs", 1, 64, 2, 0),
]


@pytest.mark.parametrize("shape,kind,morph,min_area,dil,se", EXACT)
def test_integer_stages_bit_exact(shape, kind, morph, min_area, dil, se):
    h, w = shape
    pat = synth.binary_pattern(h, w, kind, seed=h + w)
    flow = np.zeros((h, w, 2), np.float32)
    flow[..., 0] = pat
    mask, sal = gpu_stage(flow, thresh_mode=0, thresh=0.55, morph_radius=morph, min_area=min_area,
                          dilate_radius=dil, se_shape=se)
    ref, s_ref, _ = oracle.saliency_mask(flow.astype(np.float64), 0, float(np.float32(0.55)), 0.7, morph, min_area,
                                         dil, se)
    assert np.array_equal((s_ref > 0.55), pat.astype(bool))  # the decision is the pattern
    assert np.array_equal(mask, ref), "mask differs at %d pixels" % (mask != ref).sum()
    assert np.abs(sal - s_ref).max() <= 1e-6


# ---------------------------------------------------------------- saliency values and stage masks

@pytest.mark.parametrize("shape,seed,mode,thresh,weight", [
    ((256, 320), 1, 1, 0.2, 0.7),
    ((256, 320), 2, 1, 0.05, 0.7),
    ((200, 333), 3, 0, 0.5, 0.7),
    ((129, 515), 4, 1, 0.3, 1.0),
    ((129, 515), 5, 1, 0.3, 0.0),
])
def test_stage_on_given_flow(shape, seed, mode, thresh, weight):
    h, w = shape
    flow = synth.flow_field(h, w, seed)
    kw = dict(thresh_mode=mode, thresh=thresh, sal_weight=weight)
    mask, sal = gpu_stage(flow, **kw)
    s_ref = oracle.saliency(flow.astype(np.float64), float(np.float32(weight)))
    err = np.abs(sal - s_ref).max()
    assert err <= 2e-5, err
    band = check_sandwich(mask, s_ref, params(**kw), 2 * err + 1e-7)
    print("saliency max err %.3g, sandwich gap %d px" % (err, band))


def test_stage_matches_roi_mask():
    """A flow from roi_mask through the stage alone gives roi_mask's mask."""
    fl = F()
    dev = device()
    seq = synth.sequence_u16(300, 260, 2, 12, 5)
    for kw in (dict(), dict(thresh_mode=0, thresh=0.4, min_area=0), dict(morph_radius=0, min_area=100)):
        p = params(**kw)
        flow, mask, _ = fl.roi_mask(to_dev(seq[0], dev), to_dev(seq[1], dev), p)
        m2, _, _ = fl.mask_from_flow(flow, p)
        torch.cuda.synchronize()
        assert torch.equal(mask, m2)


# ---------------------------------------------------------------- whole path

@pytest.mark.parametrize("seed", [0, 1])
def test_whole_path_512_u8(seed):
    fl = F()
    dev = device()
    f0, f1, _ = synth.pair_512_u8(seed)
    p = params()
    flow, mask, _ = fl.roi_mask(to_dev(f0, dev), to_dev(f1, dev), p)
    torch.cuda.synchronize()
    flow = flow.cpu().numpy().astype(np.float64)
    mask = mask.cpu().numpy()
    ref_flow = oracle.flow(f0.astype(np.float64), f1.astype(np.float64))
    ferr = np.abs(flow - ref_flow).max()
    assert ferr <= DELTA
    s_ref = oracle.saliency(ref_flow, float(np.float32(0.7)))
    d = saliency_delta(ref_flow, ferr, 0.7)
    gap = check_sandwich(mask, s_ref, p, 2 * d)
    print("flow err %.3g, saliency delta %.3g, sandwich gap %d px, mask %.3f" % (ferr, d, gap, mask.mean()))
    assert mask.any() and not mask.all()


def test_streams_and_batched_with_saliency_rule():
    fl = F()
    dev = device()
    p = params()
    seq = synth.sequence_u16(180, 240, 4, 12, 81)
    frames = [to_dev(f, dev) for f in seq]
    st = fl.Stream(180, 240, fl.ROI_U16, p)
    flow = torch.empty((180, 240, 2), device=dev)
    mask = torch.empty((180, 240), dtype=torch.uint8, device=dev)
    assert st.push(frames[0], flow, mask) == fl.ROI_PRIMED
    for t in range(1, 4):
        assert st.push(frames[t], flow, mask) == fl.ROI_OK
        f, m, _ = fl.roi_mask(frames[t - 1], frames[t], p)
        torch.cuda.synchronize()
        assert torch.equal(f, flow) and torch.equal(m, mask), t
    st.close()
    prevs, nexts = frames[:3], frames[1:]
    flows = [torch.empty((180, 240, 2), device=dev) for _ in range(3)]
    masks = [torch.empty((180, 240), dtype=torch.uint8, device=dev) for _ in range(3)]
    pairs = fl.make_pairs(prevs, nexts, flows, masks)
    ws = fl.alloc_workspace(fl.batched_workspace_size(pairs, fl.ROI_U16, p), dev)
    for _ in range(2):
        fl.roi_mask_batched(pairs, fl.ROI_U16, p, ws)
        torch.cuda.synchronize()
        for i in range(3):
            f, m, _ = fl.roi_mask(prevs[i], nexts[i], p)
            torch.cuda.synchronize()
            assert torch.equal(f, flows[i]) and torch.equal(m, masks[i]), i
