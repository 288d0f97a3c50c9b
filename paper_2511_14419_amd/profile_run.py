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
"""
import argparse

COPY_BYTES = 256 << 20


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=3)
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--fp16", action="store_true")
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
    n = args.size
    seq = synth.sequence_u16(n, n, args.pairs + 1, max(1, 200 * n * n // (2048 * 2048)), 100)
    frames = [torch.from_numpy(s).to(dev) for s in seq]
    fl.autotune(0)
    p = fl.default_params(flags=fl.ROI_FP16_STORAGE if args.fp16 else 0)
    flow = torch.empty((n, n, 2), device=dev)
    mask = torch.empty((n, n), dtype=torch.uint8, device=dev)
    ws = fl.alloc_workspace(fl.workspace_size(n, n, fl.ROI_U16, p), dev)
    for i in range(args.pairs):
        fl.roi_mask(frames[i], frames[i + 1], p, flow=flow, mask=mask, ws=ws)
    torch.cuda.synchronize()
    print("profile_run: %d pairs %dx%d done" % (args.pairs, n, n), flush=True)


if __name__ == "__main__":
    main()
