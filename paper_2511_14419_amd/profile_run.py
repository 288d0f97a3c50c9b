"""Workload driver for hardware-counter runs (rocprofv3 --pmc ...).

Runs a plain device-to-device copy of a known size (the calibration of the
FETCH_SIZE / WRITE_SIZE counters) and then a few plain per-pair calls on
2048x2048 uint16 frames with a fixed strip height, so every dispatch of the
iteration kernel has a known algorithmic byte count.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o run -- \
        python -m paper_2511_14419_amd.profile_run
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write -o run -- \
        python -m paper_2511_14419_amd.profile_run

then ``python -m paper_2511_14419_amd.profiling traffic OUT/fetch OUT/write``.

``--strip S`` forces every iteration launch to strips of S rows (the
hardware-counter passes of ``profiling counters`` use it; 0 = the size
heuristic).

``--mode`` selects the path: ``plain`` (default parameters), ``saliency``
(the saliency rule: top 20 % of saliency, 3x3 opening and closing,
components of at least 32 px), ``stabilize`` (phase-correlation
stabilisation on), ``denoise`` (denoising pre-stage on, sigma_range 60) or
``batched`` (the 16 lens streams of uneven sizes, one roi_mask_batched
launch per step, ``--pairs`` steps after one warm-up launch that captures
the graph).
"""
import argparse

COPY_BYTES = 256 << 20


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=3)
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--fp16", action="store_true")
    ap.add_argument("--mode", choices=["plain", "saliency", "stabilize", "denoise", "batched"], default="plain")
    ap.add_argument("--strip", type=int, default=0)
    args = ap.parse_args()

    import torch

    from . import flowroi as fl
    from . import synth

    dev = torch.device("cuda:0")
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    if args.mode == "batched":
        seqs = synth.lens_streams(16, 2)
        prevs = [torch.from_numpy(q[0]).to(dev) for q in seqs]
        nexts = [torch.from_numpy(q[1]).to(dev) for q in seqs]
        flows = [torch.empty((x.shape[0], x.shape[1], 2), device=dev) for x in prevs]
        masks = [torch.empty(x.shape, dtype=torch.uint8, device=dev) for x in prevs]
        p = fl.default_params()
        pairs = fl.make_pairs(prevs, nexts, flows, masks)
        ws = fl.alloc_workspace(fl.batched_workspace_size(pairs, fl.ROI_U16, p), dev)
        for _ in range(args.pairs + 1):
            fl.roi_mask_batched(pairs, fl.ROI_U16, p, ws)
        torch.cuda.synchronize()
        print("profile_run: %d batched launches of 16 lens-stream pairs done" % (args.pairs + 1), flush=True)
        return
    n = args.size
    seq = synth.sequence_u16(n, n, args.pairs + 1, max(1, 200 * n * n // (2048 * 2048)), 100)
    frames = [torch.from_numpy(s).to(dev) for s in seq]
    fl.autotune(0)
    if args.strip:
        fl.set_strip(args.strip)
    kw = {"plain": {}, "saliency": dict(rule=fl.ROI_RULE_SALIENCY, thresh_mode=1, thresh=0.2),
          "stabilize": dict(flags=fl.ROI_STABILIZE), "denoise": dict(denoise=1, sigma_range=60.0)}[args.mode]
    if args.fp16:
        kw["flags"] = kw.get("flags", 0) | fl.ROI_FP16_STORAGE
    p = fl.default_params(**kw)
    flow = torch.empty((n, n, 2), device=dev)
    mask = torch.empty((n, n), dtype=torch.uint8, device=dev)
    ws = fl.alloc_workspace(fl.workspace_size(n, n, fl.ROI_U16, p), dev)
    for i in range(args.pairs):
        fl.roi_mask(frames[i], frames[i + 1], p, flow=flow, mask=mask, ws=ws)
    torch.cuda.synchronize()
    print("profile_run: %d pairs %dx%d (%s) done" % (args.pairs, n, n, args.mode), flush=True)


if __name__ == "__main__":
    main()
