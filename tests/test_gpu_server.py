"""Serving loop on the GPU: continuous batching must not change any result.

Each stream's frames go through the server twice: once with that stream
alone, once mixed with the other streams under a random arrival order with
random gaps (so steps of different compositions form and overlap). Every
flow and mask must be bitwise equal, and equal to the plain per-pair call.
Admission by HBM budget and the queue limit are checked too.
"""
import random
import time

import numpy as np
import pytest
import torch

from gpu_util import device, to_dev
from paper_2511_14419_amd import synth

pytestmark = pytest.mark.gpu

H, W, NF = 96, 128, 5


def F():
    from paper_2511_14419_amd import flowroi
    return flowroi


def make_streams(n):
    return [synth.sequence_u16(H, W, NF, 6, 300 + i) for i in range(n)]


def outputs(dev, n):
    return ([[torch.full((H, W, 2), float("nan"), device=dev) for _ in range(NF)] for _ in range(n)],
            [[torch.full((H, W), 9, dtype=torch.uint8, device=dev) for _ in range(NF)] for _ in range(n)])


def run(srv, order, seqs, ids, flows, masks, jitter, seed):
    rng = random.Random(seed)
    for si, t in order:
        while not srv.submit(ids[si], seqs[si][t], flows[si][t], masks[si][t], tag=si * 100 + t):
            time.sleep(0.0005)  # queue full: retry
        if jitter:
            time.sleep(rng.uniform(0, 0.002))
    srv.drain()
    return srv.poll(4096)


def test_results_same_alone_and_in_the_mix():
    dev = device()
    fl = F()
    seqs = make_streams(4)
    cfg = fl.server_config(H, W, fl.ROI_U16, max_streams=4, max_batch=4, max_inflight=2, queue_depth=3)
    # alone: one server per stream, frames in order
    alone_f, alone_m = outputs(dev, 4)
    for si in range(4):
        srv = fl.Server(cfg)
        sid = srv.open_stream()
        res = run(srv, [(0, t) for t in range(NF)], [seqs[si]], [sid], [alone_f[si]], [alone_m[si]], False, 0)
        assert [r["status"] for r in res] == [fl.ROI_PRIMED] + [fl.ROI_OK] * (NF - 1)
        srv.close()
    torch.cuda.synchronize()
    # mixed: all streams, interleaved, random gaps, two different orders
    for seed in (1, 2):
        srv = fl.Server(cfg)
        ids = [srv.open_stream() for _ in range(4)]
        mix_f, mix_m = outputs(dev, 4)
        order, nxt = [], [0] * 4
        rng = random.Random(seed)
        while len(order) < 4 * NF:
            si = rng.randrange(4)
            if nxt[si] < NF:
                order.append((si, nxt[si]))
                nxt[si] += 1
        res = run(srv, order, seqs, ids, mix_f, mix_m, True, seed)
        assert len(res) == 4 * NF and all(r["status"] >= 0 for r in res)
        assert max(r["batch"] for r in res) >= 1
        for r in res:
            assert r["t_done"] >= r["t_arrival"]
        torch.cuda.synchronize()
        for si in range(4):
            for t in range(1, NF):
                assert torch.equal(alone_f[si][t], mix_f[si][t]), (seed, si, t)
                assert torch.equal(alone_m[si][t], mix_m[si][t]), (seed, si, t)
        srv.close()
    # and equal to the plain per-pair path
    p = fl.default_params()
    for si in range(4):
        for t in range(1, NF):
            f, m, _ = fl.roi_mask(to_dev(seqs[si][t - 1], dev), to_dev(seqs[si][t], dev), p)
            torch.cuda.synchronize()
            assert torch.equal(f, alone_f[si][t]) and torch.equal(m, alone_m[si][t])


def test_admission_by_hbm_budget():
    device()
    fl = F()
    cfg = fl.server_config(H, W, fl.ROI_U16, max_streams=8)
    per = fl.Server.stream_bytes(cfg)
    cfg.hbm_budget = 2 * per + per // 2
    srv = fl.Server(cfg)
    a, b = srv.open_stream(), srv.open_stream()
    assert a is not None and b is not None
    assert srv.open_stream() is None  # a third stream would exceed the budget
    srv.close_stream(a)
    c = srv.open_stream()
    assert c is not None
    srv.close()


def test_queue_limit_and_bad_ids():
    dev = device()
    fl = F()
    cfg = fl.server_config(H, W, fl.ROI_U16, max_streams=2, queue_depth=1, max_inflight=1)
    srv = fl.Server(cfg)
    sid = srv.open_stream()
    seq = make_streams(1)[0]
    flow = torch.empty((H, W, 2), device=dev)
    mask = torch.empty((H, W), dtype=torch.uint8, device=dev)
    with pytest.raises(fl.RoiError):
        srv.submit(sid + 1, seq[0], flow, mask)
    accepted = sum(srv.submit(sid, seq[t % NF], flow, mask, tag=t) for t in range(20))
    assert 1 <= accepted <= 20
    srv.drain()
    assert len(srv.poll()) == accepted
    srv.close()
