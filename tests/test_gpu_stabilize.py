"""Stabilisation (phase-correlation registration, Method: optical flow
extraction) on the GPU against the FP64 oracle.

* The correlation surface within a bound of FP32 FFT rounding; the integer
  translation (an argmax) equal to the oracle's wherever the oracle's peak
  clears its runner-up by more than twice that bound (the decision is
  unique there), and equal to the drift the synthetic frames were built with.
* The registered frame equal to the oracle's (a copy with clamped
  coordinates: bit-exact).
* The whole path with ROI_STABILIZE (alone and after denoising): the shift
  equal to the oracle's, the flow within 1e-3 px, the mask by the band rule.
* Streams register each frame to its registered predecessor; batched pairs
  equal single calls.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DELTA, check_mask, device, to_dev
from paper_2511_14419_amd import synth

pytestmark = pytest.mark.gpu

SURF_TOL = 2e-5


def F():
    from paper_2511_14419_amd import flowroi
    return flowroi


def margin(r):
    """Largest value minus the runner-up of a correlation surface."""
    v = np.sort(r.ravel())
    return v[-1] - v[-2]


@pytest.mark.parametrize("shape,drift,dtype", [
    ((300, 340), (4, -6), "u16"),
    ((256, 256), (-9, 3), "u16"),
    ((333, 257), (0, 0), "u16"),
    ((200, 520), (1, 1), "u8"),
    ((160, 200), (-2, 5), "f32"),
    ((1030, 1100), (7, -11), "u16"),
])
def test_phase_correlation_surface_shift_and_alignment(shape, drift, dtype):
    fl = F()
    dev = device()
    h, w = shape
    fr = synth.drifting_frames(h, w, [drift], 50 + h)
    if dtype == "u8":
        fr = (fr // 16).astype(np.uint8)
    elif dtype == "f32":
        fr = fr.astype(np.float32)
    sy, sx, peak, surf, al = fl.phase_correlation(to_dev(fr[0], dev), to_dev(fr[1], dev))
    torch.cuda.synchronize()
    r_ref, P, _, _ = oracle.phase_correlation(fr[0], fr[1])
    assert surf.shape == (P, P)
    err = np.abs(surf.cpu().numpy() - r_ref).max()
    assert err <= SURF_TOL, err
    ry, rx, rpk = oracle.phase_shift(fr[0], fr[1])
    assert margin(r_ref) > 2 * SURF_TOL
    assert (sy, sx) == (ry, rx) == tuple(drift)
    assert abs(peak - rpk) <= SURF_TOL
    np.testing.assert_array_equal(al.cpu().numpy(), oracle.align(fr[1].astype(np.float64), sy, sx))


def test_degenerate_sizes():
    fl = F()
    dev = device()
    for h, w in [(1, 50), (3, 3), (2, 9), (40, 1)]:
        a = np.arange(h * w, dtype=np.float32).reshape(h, w)
        b = np.roll(a, 1, axis=1)
        sy, sx, _, surf, al = fl.phase_correlation(to_dev(a, dev), to_dev(b, dev))
        torch.cuda.synchronize()
        ry, rx, _ = oracle.phase_shift(a, b)
        P = oracle.phase_size(h, w)
        if P == 0:
            assert surf is None and (sy, sx) == (0, 0) == (ry, rx)
            np.testing.assert_array_equal(al.cpu().numpy(), b)
        else:
            r_ref, _, _, _ = oracle.phase_correlation(a, b)
            assert np.abs(surf.cpu().numpy() - r_ref).max() <= SURF_TOL
            if margin(r_ref) > 2 * SURF_TOL:
                assert (sy, sx) == (ry, rx)


def test_identical_frames_zero_shift_unit_peak():
    fl = F()
    dev = device()
    fr = synth.drifting_frames(256, 300, [(0, 0)], 3)
    sy, sx, peak, _, al = fl.phase_correlation(to_dev(fr[0], dev), to_dev(fr[0], dev))
    torch.cuda.synchronize()
    assert (sy, sx) == (0, 0) and abs(peak - 1.0) < 1e-4
    np.testing.assert_array_equal(al.cpu().numpy(), fr[0].astype(np.float32))


@pytest.mark.parametrize("denoise", [False, True])
def test_whole_path_with_stabilisation(denoise):
    fl = F()
    dev = device()
    fr = synth.drifting_frames(384, 448, [(5, -7)], 77)
    kw = dict(flags=fl.ROI_STABILIZE, thresh=0.5)
    dn = None
    if denoise:
        kw.update(denoise=1, sigma_range=60.0)
        dn = dict(median_radius=1, bilateral_radius=2, sigma_space=1.5, sigma_range=60.0)
    p = fl.default_params(**kw)
    flow, mask, ws = fl.roi_mask(to_dev(fr[0], dev), to_dev(fr[1], dev), p)
    sy, sx, _ = fl.read_shift(ws)
    tau2 = fl.read_tau2(ws)
    torch.cuda.synchronize()
    ref_flow, _, ref_t2 = oracle.roi_mask(fr[0], fr[1], thresh=float(np.float32(0.5)), denoise_params=dn,
                                          stabilize=True)
    a, b = fr[0].astype(np.float64), fr[1].astype(np.float64)
    if denoise:
        a, b = oracle.denoise(a, **dn), oracle.denoise(b, **dn)
    assert (sy, sx) == oracle.phase_shift(a, b)[:2] == (5, -7)
    err = np.abs(flow.cpu().numpy() - ref_flow).max()
    assert err <= DELTA, err
    check_mask(mask.cpu().numpy(), ref_flow, ref_t2, 2, 0, DELTA)
    assert abs(tau2 - ref_t2) < 1e-6
    # the drift is gone from the flow: the median residual is far below a pixel
    assert np.abs(np.median(ref_flow[40:-40, 40:-40], axis=(0, 1))).max() < 0.25


def test_stream_registers_to_registered_predecessor():
    fl = F()
    dev = device()
    drifts = [(3, -2), (-4, 5), (0, 1)]
    fr = synth.drifting_frames(256, 320, drifts, 91)
    p = fl.default_params(flags=fl.ROI_STABILIZE)
    st = fl.Stream(256, 320, fl.ROI_U16, p)
    flow = torch.empty((256, 320, 2), device=dev)
    mask = torch.empty((256, 320), dtype=torch.uint8, device=dev)
    assert st.push(to_dev(fr[0], dev), flow, mask) == fl.ROI_PRIMED
    assert st.read_shift()[:2] == (0, 0)
    reg = fr[0].astype(np.float64)
    for t in range(1, len(fr)):
        assert st.push(to_dev(fr[t], dev), flow, mask) == fl.ROI_OK
        sy, sx, _ = st.read_shift()
        ry, rx, _ = oracle.phase_shift(reg, fr[t])
        # each raw frame sits at the cumulative drift from the registered chain
        assert (sy, sx) == (ry, rx) == tuple(np.sum(drifts[:t], axis=0))
        nreg = oracle.align(fr[t].astype(np.float64), ry, rx)
        ref = oracle.flow(reg, nreg)
        err = np.abs(flow.cpu().numpy() - ref).max()
        assert err <= DELTA, (t, err)
        reg = nreg
    st.close()


def test_batched_with_stabilisation_equals_single_calls():
    fl = F()
    dev = device()
    p = fl.default_params(flags=fl.ROI_STABILIZE)
    seqs = [synth.drifting_frames(h, w, [d], 120 + i) for i, ((h, w), d) in
            enumerate([((200, 260), (2, 3)), ((150, 150), (-5, 0)), ((260, 130), (1, -4))])]
    prevs = [to_dev(s[0], dev) for s in seqs]
    nexts = [to_dev(s[1], dev) for s in seqs]
    flows = [torch.empty((s.shape[1], s.shape[2], 2), device=dev) for s in seqs]
    masks = [torch.empty((s.shape[1], s.shape[2]), dtype=torch.uint8, device=dev) for s in seqs]
    pairs = fl.make_pairs(prevs, nexts, flows, masks)
    ws = fl.alloc_workspace(fl.batched_workspace_size(pairs, fl.ROI_U16, p), dev)
    fl.roi_mask_batched(pairs, fl.ROI_U16, p, ws)
    torch.cuda.synchronize()
    for i in range(3):
        f, m, w1 = fl.roi_mask(prevs[i], nexts[i], p)
        torch.cuda.synchronize()
        assert torch.equal(f, flows[i]) and torch.equal(m, masks[i])
        assert fl.read_shift(ws, i) == fl.read_shift(w1, 0)
