"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, and validates requests exactly as
documented (nothing reaches the device on these paths)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flowroi.h")


@pytest.fixture(scope="module")
def F():
    from paper_2511_14419_amd import build, flowroi
    if build.stale():
        build.build()
    return flowroi


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(roi_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(F):
    L = F.lib()
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert sorted(F.EXPORTED) == names


def test_defaults(F):
    p = F.default_params()
    assert (p.levels, p.winsize, p.iterations, p.poly_n) == (3, 15, 3, 5)
    assert abs(p.poly_sigma - 1.1) < 1e-6 and abs(p.eps - 1e-3) < 1e-9
    assert (p.thresh_mode, p.thresh, p.dilate_radius, p.se_shape, p.flags) == (0, 1.0, 2, 0, 0)
    assert (p.denoise, p.median_radius, p.bilateral_radius) == (0, 1, 2)
    assert abs(p.sigma_space - 1.5) < 1e-6 and abs(p.sigma_range - 20.0) < 1e-6
    assert (p.adjacent, p.rule, p.morph_radius, p.min_area) == (0, F.ROI_RULE_MAGNITUDE, 1, 32)
    assert abs(p.sal_weight - 0.7) < 1e-6


@pytest.mark.parametrize("kw,h,w,dtype,expect", [
    ({}, 512, 512, 0, 0),
    ({}, 0, 512, 1, 0),
    ({}, -1, 5, 0, -1),
    ({}, 8, 8, 3, -1),
    ({"levels": 0}, 64, 64, 0, -1),
    ({"levels": 11}, 64, 64, 0, -1),
    ({"winsize": 14}, 64, 64, 0, -1),
    ({"winsize": 17}, 64, 64, 0, -4),
    ({"iterations": 0}, 64, 64, 0, -1),
    ({"poly_n": 6}, 64, 64, 0, -1),
    ({"poly_n": 9}, 64, 64, 0, -1),
    ({"poly_sigma": 0.0}, 64, 64, 0, -1),
    ({"eps": 0.0}, 64, 64, 0, -1),
    ({"thresh": -0.5}, 64, 64, 0, -1),
    ({"thresh_mode": 1, "thresh": 0.0}, 64, 64, 0, -1),
    ({"thresh_mode": 1, "thresh": 1.0}, 64, 64, 0, -1),
    ({"thresh_mode": 1, "thresh": 0.2}, 64, 64, 0, 0),
    ({"thresh_mode": 2}, 64, 64, 0, -1),
    ({"dilate_radius": -1}, 64, 64, 0, -1),
    ({"dilate_radius": 33}, 64, 64, 0, -4),
    ({"se_shape": 2}, 64, 64, 0, -1),
    ({"flags": 8}, 64, 64, 0, -1),
    ({"flags": 3}, 64, 64, 2, 0),
    ({}, 40000, 64, 0, -4),
    ({"denoise": 1}, 64, 64, 0, 0),
    ({"denoise": 2}, 64, 64, 0, -1),
    ({"denoise": 1, "median_radius": 3}, 64, 64, 0, -4),
    ({"denoise": 1, "bilateral_radius": 4}, 64, 64, 0, -4),
    ({"denoise": 1, "sigma_range": 0.0}, 64, 64, 0, -1),
    ({"denoise": 1, "bilateral_radius": 0, "sigma_range": 0.0}, 64, 64, 0, 0),
    ({"denoise": 0, "median_radius": 9}, 64, 64, 0, 0),
    ({"adjacent": 2}, 64, 64, 0, 0),
    ({"adjacent": -1}, 64, 64, 0, -1),
    ({"adjacent": 9}, 64, 64, 0, -4),
    ({"rule": 1}, 64, 64, 0, 0),
    ({"rule": 2}, 64, 64, 0, -1),
    ({"rule": 1, "thresh_mode": 1, "thresh": 0.2}, 64, 64, 0, 0),
    ({"rule": 1, "sal_weight": 1.5}, 64, 64, 0, -1),
    ({"rule": 1, "sal_weight": float("nan")}, 64, 64, 0, -1),
    ({"rule": 1, "morph_radius": -1}, 64, 64, 0, -1),
    ({"rule": 1, "morph_radius": 3}, 64, 64, 0, -4),
    ({"rule": 1, "min_area": -2}, 64, 64, 0, -1),
    ({"rule": 0, "morph_radius": 7, "min_area": -2}, 64, 64, 0, 0),
    ({"flags": 4}, 64, 64, 1, 0),
    ({"flags": 7}, 64, 64, 1, 0),
    ({"flags": 12}, 64, 64, 1, -1),
])
def test_validate(F, kw, h, w, dtype, expect):
    assert F.validate(h, w, dtype, F.default_params(**kw)) == expect


def test_workspace_size(F):
    p = F.default_params()
    a = F.lib().roi_workspace_size(512, 512, 0, ctypes.byref(p))
    b = F.lib().roi_workspace_size(2048, 2048, 1, ctypes.byref(p))
    assert 0 < a < b
    half = F.default_params(flags=F.ROI_FP16_STORAGE)
    assert F.lib().roi_workspace_size(2048, 2048, 1, ctypes.byref(half)) < b
    assert F.lib().roi_workspace_size(64, 64, 0, ctypes.byref(F.default_params(levels=0))) == 0


def test_roi_mask_rejects_before_launch(F):
    L = F.lib()
    p = F.default_params()
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    # null frame
    assert L.roi_mask(None, fake, 64, 64, 64, 0, ctypes.byref(p), fake, fake, ws, 1 << 30, None) == F.ROI_EINVAL
    # pitch < w
    assert L.roi_mask(fake, fake, 64, 64, 63, 0, ctypes.byref(p), fake, fake, ws, 1 << 30, None) == F.ROI_EINVAL
    # misaligned workspace
    assert L.roi_mask(fake, fake, 64, 64, 64, 0, ctypes.byref(p), fake, fake, ctypes.c_void_p(0x100010),
                      1 << 30, None) == F.ROI_EINVAL
    # workspace too small
    need = L.roi_workspace_size(64, 64, 0, ctypes.byref(p))
    assert L.roi_mask(fake, fake, 64, 64, 64, 0, ctypes.byref(p), fake, fake, ws, need - 1, None) == F.ROI_ENOMEM
    # bad params
    bad = F.default_params(winsize=4)
    assert L.roi_mask(fake, fake, 64, 64, 64, 0, ctypes.byref(bad), fake, fake, ws, 1 << 30, None) == F.ROI_EINVAL
    # empty frame: no-op
    assert L.roi_mask(None, None, 0, 64, 64, 0, ctypes.byref(p), None, None, None, 0, None) == F.ROI_OK


def test_mask_from_flow_rejects_before_launch(F):
    L = F.lib()
    p = F.default_params(rule=F.ROI_RULE_SALIENCY)
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    need = L.roi_flow_mask_workspace_size(64, 64, ctypes.byref(p))
    assert need > L.roi_flow_mask_workspace_size(0, 64, ctypes.byref(p)) > 0
    assert L.roi_flow_mask_workspace_size(64, 64, ctypes.byref(F.default_params(rule=5))) == 0
    assert L.roi_mask_from_flow(None, 64, 64, ctypes.byref(p), fake, None, ws, need, None) == F.ROI_EINVAL
    assert L.roi_mask_from_flow(fake, 64, 64, ctypes.byref(p), None, None, ws, need, None) == F.ROI_EINVAL
    assert L.roi_mask_from_flow(fake, 64, 64, ctypes.byref(p), fake, None, ctypes.c_void_p(0x100040), need,
                                None) == F.ROI_EINVAL
    assert L.roi_mask_from_flow(fake, 64, 64, ctypes.byref(p), fake, None, ws, need - 1, None) == F.ROI_ENOMEM
    bad = F.default_params(rule=1, morph_radius=3)
    assert L.roi_mask_from_flow(fake, 64, 64, ctypes.byref(bad), fake, None, ws, 1 << 30, None) == F.ROI_EUNSUPPORTED
    assert L.roi_mask_from_flow(None, 0, 64, ctypes.byref(p), None, None, None, 0, None) == F.ROI_OK


def test_phase_sizes_and_rejections(F):
    L = F.lib()
    assert [F.phase_size(h, w) for h, w in [(2048, 2448), (1536, 1536), (5, 300), (1, 300), (3000, 3000), (2, 2)]] \
        == [2048, 1024, 4, 0, 2048, 2]
    p = F.default_params()
    s = F.default_params(flags=F.ROI_STABILIZE)
    assert L.roi_workspace_size(512, 512, 1, ctypes.byref(s)) > L.roi_workspace_size(512, 512, 1, ctypes.byref(p))
    need = L.roi_phase_workspace_size(256, 300)
    assert need > L.roi_phase_workspace_size(0, 300) > 0
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    assert L.roi_phase_correlation(None, fake, 256, 300, 300, 1, None, None, ws, need, None) == F.ROI_EINVAL
    assert L.roi_phase_correlation(fake, fake, 256, 300, 299, 1, None, None, ws, need, None) == F.ROI_EINVAL
    assert L.roi_phase_correlation(fake, fake, 256, 300, 300, 5, None, None, ws, need, None) == F.ROI_EINVAL
    assert L.roi_phase_correlation(fake, fake, 256, 300, 300, 1, None, None, ws, need - 1, None) == F.ROI_ENOMEM
    assert L.roi_phase_correlation(None, None, 0, 300, 300, 1, None, None, None, 0, None) == F.ROI_OK
    i = ctypes.c_int32()
    assert L.roi_read_shift(None, 0, ctypes.byref(i), ctypes.byref(i), None, None) == F.ROI_EINVAL
    assert L.roi_read_shift(ws, 256, ctypes.byref(i), ctypes.byref(i), None, None) == F.ROI_EINVAL
    assert L.roi_stream_read_shift(None, ctypes.byref(i), ctypes.byref(i), None, None) == F.ROI_EINVAL


def test_batched_and_stream_reject_before_launch(F):
    L = F.lib()
    p = F.default_params()
    arr = (F.RoiPair * 1)()
    arr[0] = F.RoiPair(0, 0x1000, 0x1000, 0x1000, 64, 64, 64)
    assert L.roi_mask_batched(1, arr, 0, ctypes.byref(p), ctypes.c_void_p(0x100000), 1 << 30, None) == F.ROI_EINVAL
    assert L.roi_mask_batched(0, arr, 0, ctypes.byref(p), ctypes.c_void_p(0x100000), 1 << 30, None) == F.ROI_EINVAL
    assert L.roi_batched_workspace_size(257, arr, 0, ctypes.byref(p)) == 0
    ctx = ctypes.c_void_p()
    assert L.roi_stream_create(64, 64, 0, ctypes.byref(F.default_params(poly_n=4)), ctypes.byref(ctx)) == F.ROI_EINVAL
    assert L.roi_stream_create(0, 64, 0, ctypes.byref(p), ctypes.byref(ctx)) == F.ROI_EINVAL
    assert L.roi_stream_push(None, None, 64, None, None, None) == F.ROI_EINVAL
    assert L.roi_stream_state_bytes(2048, 2048, 1, ctypes.byref(p)) > 0


def test_strip_override_validation(F):
    L = F.lib()
    assert L.roi_set_strip(5) == F.ROI_EINVAL
    assert L.roi_set_strip(-8) == F.ROI_EINVAL
    assert L.roi_set_strip(0) == F.ROI_OK
    assert L.roi_tuned_strip(123, 456, 15, 0) == 0


def test_status_strings(F):
    for s in (0, 1, -1, -2, -3, -4):
        assert F.status_str(s)
    assert F.status_str(99) == "unknown status"


def test_server_config_rejected_before_any_device_work(F):
    L = F.lib()
    srv = ctypes.c_void_p()
    bad = F.server_config(64, 64, F.ROI_U8, max_streams=0)
    assert L.roi_server_create(ctypes.byref(bad), ctypes.byref(srv)) == F.ROI_EINVAL
    bad = F.server_config(64, 64, F.ROI_U8, max_inflight=9)
    assert L.roi_server_create(ctypes.byref(bad), ctypes.byref(srv)) == F.ROI_EINVAL
    bad = F.server_config(64, 64, F.ROI_U8, params=F.default_params(winsize=2))
    assert L.roi_server_create(ctypes.byref(bad), ctypes.byref(srv)) == F.ROI_EINVAL
    good = F.server_config(2048, 2048, F.ROI_U16)
    per = L.roi_server_stream_bytes(ctypes.byref(good))
    assert per > L.roi_stream_state_bytes(2048, 2048, 1, ctypes.byref(good.params))
    assert L.roi_server_poll(None, None, 4) == 0
    assert L.roi_server_submit(None, 0, None, 64, None, None, 0) == F.ROI_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    """No fallback: with the library absent every entry raises."""
    import subprocess
    import sys
    code = ("import paper_2511_14419_amd.flowroi as fl\n"
            "fl._LIB_PATH = %r\n"
            "fl._lib = None\n"
            "try:\n"
            "    fl.default_params()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    print('no error')\n" % str(tmp_path / "libflowroi.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("raised:") and "not built" in r.stdout


def test_product_package_never_loads_the_oracle():
    """The oracle is test infrastructure: nothing in the package imports,
    links or loads it (only tests, the smoke check and the benchmark's CPU
    baseline may)."""
    pkg = os.path.join(ROOT, "paper_2511_14419_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".h", ".hip", ".cpp", ".c")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "flowroi_oracle" not in text and "liboracle" not in text, f
