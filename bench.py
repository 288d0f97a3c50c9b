#!/usr/bin/env python3
"""Throughput of the flow -> RoI-mask hot path on one MI355X.

Workload (headline): the plain per-pair path over one stream of 64
consecutive 2048x2048 uint16 frames (12-bit moving-cell synthetic frames:
background 1200, noise sigma 25, 200 Gaussian-blob cells, sigma 5-10 px,
90 % on random walks with step sigma 1.5 px; seed 100), one roi_mask call
per consecutive pair with the default parameters (3 levels, 15x15 window,
3 iterations, poly_n 5 / sigma 1.1, |d| > 1 px, 5x5 square dilation).
A step is one pass over the 63 pairs; `value` is pairs (= output frames)
per second with every frame already resident in HBM.

Beside it the JSON line carries the plain path with the other stages
switched on (denoising, the saliency rule, a top-fraction threshold,
stabilisation), the mask stage alone per rule, the streaming path (previous
frame's expansion kept resident; with the adjacent-frame ensemble), the
batched path (16 lens streams of uneven sizes in one graph launch, FP32 and
FP16 storage, beside the same 16 pairs through one roi_mask call each), the
serving sweep, per-pair latency percentiles, the roofline
of the dominant kernel (the iteration kernel, timed with HIP events on its
own stream inside the timed region) and the FP64 oracle timed on the host
over consecutive 2048x2048 pairs (about 10 s of host work).

Progress goes to stderr; stdout gets exactly one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

H = W = 2048
N_FRAMES = 64
HBM_PEAK_GBS = 8000.0
TIMING_EVERY = 8  # timed-region calls bracketed by the kernel-time events: every 8th


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=N_FRAMES)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline path only")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-streams", type=int, default=64)
    ap.add_argument("--serve-rates", type=str, default="8,256,1024,1536,2048,2560,3072,3584")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (the frame streams "
              "are independent; see the sharding notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2511_14419_amd import flowroi as fl
    from paper_2511_14419_amd import synth

    dev = torch.device("cuda:0")
    fl.lib()  # fail loudly if the HIP library is missing
    log("generating %d frames %dx%d u16" % (args.frames, H, W))
    t = time.time()
    seq = synth.sequence_u16(H, W, args.frames, 200, 100)
    log("  %.1f s" % (time.time() - t))
    frames = [torch.from_numpy(seq[i]).to(dev) for i in range(args.frames)]
    npairs = args.frames - 1
    p = fl.default_params()
    flows = [torch.empty((H, W, 2), dtype=torch.float32, device=dev) for _ in range(npairs)]
    masks = [torch.empty((H, W), dtype=torch.uint8, device=dev) for _ in range(npairs)]
    ws = fl.alloc_workspace(fl.workspace_size(H, W, fl.ROI_U16, p), dev)

    def step():
        for i in range(npairs):
            fl.roi_mask(frames[i], frames[i + 1], p, flow=flows[i], mask=masks[i], ws=ws)

    log("warmup %d steps" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log("timed %d steps x %d pairs" % (args.steps, npairs))
    # iteration-kernel time inside the timed region: one pair of HIP events
    # around the 9 back-to-back iteration launches of every 8th call (each
    # record idles the GPU for a few us; the event pool is filled before the
    # clock starts)
    fl.timing_enable(True, per_call=True, every=TIMING_EVERY)
    fl.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fl.timing_enable(False)
    k_ms, k_n, k_px, k_bytes = fl.timing_read()
    # per-level breakdown: one more step, outside the timed region, with
    # events around every launch
    fl.timing_reset()
    fl.timing_enable(True)
    step()
    torch.cuda.synchronize()
    fl.timing_enable(False)
    recs = fl.timing_records()
    fl.timing_reset()
    per_level = {}
    for ms_, px_, b_ in recs:
        e = per_level.setdefault(px_, [0.0, 0.0, 0])
        e[0] += ms_
        e[1] += b_
        e[2] += 1
    elapsed = t1 - t0
    value = npairs * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    from paper_2511_14419_amd import profiling
    tr = profiling.load_traffic(os.path.join(ROOT, "profiles", "k_iter_traffic_plain_2048_u16.txt"))
    log("plain: %.1f pairs/s, %.2f ms/step; iteration kernel %.1f GB/s over %d launches"
        % (value, ms_per_step, achieved, k_n))

    # per-pair latency (GPU time between events around each call)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(npairs)]
    for i in range(npairs):
        evs[i][0].record()
        fl.roi_mask(frames[i], frames[i + 1], p, flow=flows[i], mask=masks[i], ws=ws)
        evs[i][1].record()
    torch.cuda.synchronize()
    lat = [a.elapsed_time(b) for a, b in evs]

    out = {
        "metric": "frames/s flow->RoI mask (2048x2048 u16), plain per-pair path",
        "value": round(value, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "plain per-pair path: 1 stream x %d frames 2048x2048 u16 (12-bit moving-cell "
                        "frames), one roi_mask call per consecutive pair" % args.frames,
            "pairs_per_step": npairs, "h": H, "w": W, "input": "u16",
            "params": p.as_dict(),
        },
        "latency_ms": {"p50": round(percentile(lat, 50), 4), "p99": round(percentile(lat, 99), 4)},
        "roofline": {
            "kernel": "k_iter (warp + update + 15x15 window + 2x2 solve)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": tr["hbm_bytes_per_launch"] if tr else None,
            "traffic_over_algorithmic": tr["hbm_over_algorithmic"] if tr else None,
            "launches": k_n,
            "avg_launch_us": round(1e3 * k_ms / max(k_n, 1), 3),
            "bytes_per_launch": round(k_bytes / max(k_n, 1)),
            "per_level": [{"pixels": px_, "launches": e[2], "avg_launch_us": round(1e3 * e[0] / e[2], 2),
                           "achieved_gbs": round(e[1] / (e[0] * 1e-3) / 1e9, 1),
                           "frac": round(e[1] / (e[0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
                          for px_, e in sorted(per_level.items(), reverse=True)],
        },
    }

    if not args.no_extras:
        out["plain_denoise"] = bench_plain_variant(fl, frames, flows, masks, dev, args,
                                                   fl.default_params(denoise=1, sigma_range=60.0), "denoise on")
        out["plain_saliency_rule"] = bench_plain_variant(
            fl, frames, flows, masks, dev, args, fl.default_params(rule=fl.ROI_RULE_SALIENCY, thresh_mode=1, thresh=0.2),
            "saliency rule: top 20 % of saliency (weight 0.7), 3x3 opening+closing, components >= 32 px")
        out["plain_top_fraction"] = bench_plain_variant(fl, frames, flows, masks, dev, args,
                                                        fl.default_params(thresh_mode=1, thresh=0.2),
                                                        "magnitude rule, top 20 % of |d|")
        out["plain_stabilized"] = bench_plain_variant(fl, frames, flows, masks, dev, args,
                                                      fl.default_params(flags=fl.ROI_STABILIZE),
                                                      "stabilisation on (phase correlation over 2048x2048)")
        out["mask_stage_us"] = bench_mask_stage(fl, flows[0], args)
        out["streaming"] = bench_streaming(fl, frames, p, dev, args)
        out["streaming_adjacent2"] = bench_streaming(fl, frames, fl.default_params(adjacent=2), dev, args)
        out["batched"] = bench_batched(fl, dev, args, fp16=False)
        out["batched_fp16"] = bench_batched(fl, dev, args, fp16=True)
        if not args.no_serving:
            del flows, masks
            torch.cuda.empty_cache()
            out["serving"] = bench_serving(fl, dev, args)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(seq)
    print(json.dumps(out), flush=True)


def bench_plain_variant(fl, frames, flows, masks, dev, args, p, name):
    """The plain per-pair path with other parameters, over the same 63 pairs."""
    import torch
    npairs = len(frames) - 1
    ws = fl.alloc_workspace(fl.workspace_size(H, W, fl.ROI_U16, p), dev)
    for i in range(npairs):
        fl.roi_mask(frames[i], frames[i + 1], p, flow=flows[i], mask=masks[i], ws=ws)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        for i in range(npairs):
            fl.roi_mask(frames[i], frames[i + 1], p, flow=flows[i], mask=masks[i], ws=ws)
    torch.cuda.synchronize()
    r = {"frames_per_s": round(npairs * reps / (time.perf_counter() - t0), 2), "params": name}
    log("plain (%s): %.1f frames/s" % (name, r["frames_per_s"]))
    return r


def bench_mask_stage(fl, flow, args):
    """GPU time of the mask stage alone (roi_mask_from_flow) on one 2048x2048
    flow field, per rule, microseconds per call."""
    import torch
    rules = {
        "magnitude_abs_1px": fl.default_params(),
        "magnitude_top20": fl.default_params(thresh_mode=1, thresh=0.2),
        "saliency_top20_cc32": fl.default_params(rule=fl.ROI_RULE_SALIENCY, thresh_mode=1, thresh=0.2),
        "saliency_top20_no_cc": fl.default_params(rule=fl.ROI_RULE_SALIENCY, thresh_mode=1, thresh=0.2, min_area=0),
    }
    out = {}
    for name, p in rules.items():
        m, _, ws = fl.mask_from_flow(flow, p)
        torch.cuda.synchronize()
        n = 20 * max(1, args.steps // 5)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fl.mask_from_flow(flow, p, ws=ws, mask=m)
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(1e3 * e0.elapsed_time(e1) / n, 2)
    log("mask stage alone (us): %s" % out)
    return out


def bench_streaming(fl, frames, p, dev, args):
    import torch
    npairs = len(frames) - 1
    s = fl.Stream(H, W, fl.ROI_U16, p)
    flow = torch.empty((H, W, 2), dtype=torch.float32, device=dev)
    mask = torch.empty((H, W), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        s.reset()
        for f in frames:
            s.push(f, flow, mask)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    for _ in range(args.steps):
        s.reset()
        for f in frames:
            if s.push(f, flow, mask) == fl.ROI_OK:
                n += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    r = {"frames_per_s": round(n / dt, 2), "pairs": n}
    log("streaming: %.1f frames/s" % r["frames_per_s"])
    return r


def bench_batched(fl, dev, args, fp16):
    import torch

    from paper_2511_14419_amd import synth
    seqs = synth.lens_streams(16, 2)
    prevs = [torch.from_numpy(s[0]).to(dev) for s in seqs]
    nexts = [torch.from_numpy(s[1]).to(dev) for s in seqs]
    flows = [torch.empty((x.shape[0], x.shape[1], 2), dtype=torch.float32, device=dev) for x in prevs]
    masks = [torch.empty(x.shape, dtype=torch.uint8, device=dev) for x in prevs]
    p = fl.default_params(flags=fl.ROI_FP16_STORAGE if fp16 else 0)
    pairs = fl.make_pairs(prevs, nexts, flows, masks)
    ws = fl.alloc_workspace(fl.batched_workspace_size(pairs, fl.ROI_U16, p), dev)
    for _ in range(max(args.warmup, 1)):
        fl.roi_mask_batched(pairs, fl.ROI_U16, p, ws)
    torch.cuda.synchronize()
    reps = max(args.steps, 5)
    t0 = time.perf_counter()
    for _ in range(reps):
        fl.roi_mask_batched(pairs, fl.ROI_U16, p, ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    px = sum(x.numel() for x in prevs)
    # the same pairs through the plain per-pair path, one roi_mask call each
    wss = [fl.alloc_workspace(fl.workspace_size(x.shape[0], x.shape[1], fl.ROI_U16, p), dev) for x in prevs]

    def one_by_one():
        for i in range(len(prevs)):
            fl.roi_mask(prevs[i], nexts[i], p, flow=flows[i], mask=masks[i], ws=wss[i])
    one_by_one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one_by_one()
    torch.cuda.synchronize()
    dts = (time.perf_counter() - t0) / reps
    del wss
    fl.roi_mask_batched(pairs, fl.ROI_U16, p, ws)  # leave the batched results in flows / masks
    torch.cuda.synchronize()
    r = {"pairs": len(prevs), "ms_per_launch": round(dt * 1e3, 3), "mpx_per_s": round(px / dt / 1e6, 1),
         "frames_2048_equiv_per_s": round(px / dt / (H * W), 2), "storage": "f16" if fp16 else "f32",
         "same_pairs_per_pair_calls": {"ms": round(dts * 1e3, 3), "frames_2048_equiv_per_s": round(px / dts / (H * W), 2)},
         "speedup_vs_per_pair_calls": round(dts / dt, 3)}
    if fp16 and not args.no_cpu_baseline:
        r["error_vs_oracle"] = fp16_error(seqs, flows, masks)
    log("batched %s: %s" % (r["storage"], r))
    return r


def fp16_error(seqs, flows, masks, delta=1e-3):
    """Flow error of the FP16-storage results against the FP64 oracle over
    every pixel of every pair, and the fraction of mask pixels that differ
    where the structuring element touches no threshold-band pixel."""
    import numpy as np

    import oracle
    emax, esum, n, flips, checked = 0.0, 0.0, 0, 0, 0
    for q, f, m in zip(seqs, flows, masks):
        ref_flow, ref_mask, t2 = oracle.roi_mask(q[0].astype(np.float64), q[1].astype(np.float64))
        g = f.cpu().numpy().astype(np.float64)
        e = np.abs(g - ref_flow)
        emax = max(emax, float(e.max()))
        esum += float(e.sum())
        n += e.size
        band = (np.abs(np.hypot(ref_flow[..., 0], ref_flow[..., 1]) - np.sqrt(t2)) <= delta).astype(np.uint8)
        free = oracle.dilate(band, 2, 0) == 0
        flips += int(((m.cpu().numpy() != ref_mask) & free).sum())
        checked += int(free.sum())
    return {"max_dflow_px": round(emax, 5), "mean_dflow_px": round(esum / n, 6),
            "mask_flip_rate_outside_band": round(flips / max(checked, 1), 6)}


def bench_serving(fl, dev, args):
    """64 lens streams (384-well mode) of 2048x2048 u16 frames arriving as a
    Poisson process at each aggregate rate; latency is arrival in host
    memory -> mask ready on the device."""
    import numpy as np
    import torch

    from paper_2511_14419_amd import synth
    ns = args.serve_streams
    nseq, nfr = 8, 4
    seqs = [synth.sequence_u16(H, W, nfr, 200, 500 + i) for i in range(nseq)]
    host = [[torch.from_numpy(q[t]).pin_memory() for t in range(nfr)] for q in seqs]
    cfg = fl.server_config(H, W, fl.ROI_U16, hbm_budget=96 << 30, max_streams=ns, max_batch=ns, max_inflight=2,
                           queue_depth=16)
    srv = fl.Server(cfg)
    ids = []
    for _ in range(ns):
        sid = srv.open_stream()
        if sid is None:
            break
        ids.append(sid)
    outs = [[(torch.empty((H, W, 2), device=dev), torch.empty((H, W), dtype=torch.uint8, device=dev))
             for _ in range(2)] for _ in ids]
    cyc = [0] * len(ids)
    nsub = [0] * len(ids)

    def next_frame(k):
        # palindromic cycle 0 1 2 3 2 1 0 1 ...
        c = cyc[k] % (2 * nfr - 2)
        cyc[k] += 1
        return host[k % nseq][c if c < nfr else 2 * nfr - 2 - c]

    for k, sid in enumerate(ids):  # prime every stream with its first frame
        srv.submit(sid, next_frame(k), outs[k][0][0], outs[k][0][1])
    srv.drain()
    srv.poll(1 << 16)
    rng = np.random.default_rng(7)
    points = []
    for rate in [float(r) for r in args.serve_rates.split(",")]:
        n = int(min(max(rate * 2.0, 64), 4000))
        gaps = rng.exponential(1.0 / rate, n)
        who = rng.integers(0, len(ids), n)
        t0 = fl.steady_now() + 0.01
        t_next = t0
        dropped = 0
        for g, k in zip(gaps, who):
            t_next += g
            while fl.steady_now() < t_next:
                pass
            slot = outs[k][nsub[k] % 2]
            if srv.submit(ids[k], next_frame(k), slot[0], slot[1], tag=int(k)):
                nsub[k] += 1
            else:
                dropped += 1
        srv.drain()
        res = [r for r in srv.poll(1 << 16) if r["status"] == fl.ROI_OK]
        lat = np.array([r["t_done"] - r["t_arrival"] for r in res]) * 1e3
        span = max(r["t_done"] for r in res) - min(r["t_arrival"] for r in res)
        pt = {"rate_fps": rate, "frames": len(res), "dropped": dropped, "frames_per_s": round(len(res) / span, 1),
              "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
              "mean_batch": round(float(np.mean([r["batch"] for r in res])), 2)}
        points.append(pt)
        log("serving: %s" % pt)
        if pt["p99_ms"] > 200 or dropped > n // 10:
            break
    srv.close()
    best = max(points, key=lambda q: q["frames_per_s"])
    return {"streams": len(ids), "stream_bytes": fl.Server.stream_bytes(cfg), "points": points,
            "max_frames_per_s": best["frames_per_s"]}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(seq, budget_s=10.0):
    """The FP64 oracle over consecutive pairs of the same sequence until about
    budget_s seconds of host work have run (at least one pair)."""
    import numpy as np

    import oracle
    log("cpu baseline: FP64 oracle on consecutive 2048x2048 pairs, ~%.0f s" % budget_s)
    n = 0
    t0 = time.perf_counter()
    while n + 1 < len(seq) and (n == 0 or time.perf_counter() - t0 < budget_s):
        oracle.roi_mask(seq[n].astype(np.float64), seq[n + 1].astype(np.float64))
        n += 1
    dt = time.perf_counter() - t0
    r = {"value": round(n / dt, 4), "unit": "frames/s", "cores": oracle.num_threads(), "kind": "oracle",
         "sample": "pairs 0->1 ... %d->%d of the 2048x2048 u16 sequence (%d pairs), full path, %.1f s on %s"
                   % (n - 1, n, n, dt, cpu_model())}
    log("  %s" % r)
    return r


if __name__ == "__main__":
    main()
