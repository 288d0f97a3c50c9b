"""Summaries of rocprofv3 output for the iteration kernel.

``traffic`` turns two counter runs of ``profile_run`` (FETCH_SIZE, then
WRITE_SIZE, each in KiB per dispatch) into HBM bytes per launch of the
iteration kernel. Each counter is scaled by what it reads for the plain
256 MiB device copy at the start of the run (read and written bytes are
known), so the numbers are in bytes whatever the counter's own unit or
sampling. The result is compared with the algorithmic bytes of the same
launches (expansion planes of both frames + prior flow + flow out + |d|^2).

``stats`` renders a ``--kernel-trace --stats`` kernel_stats.csv as a table.

``counters`` reads the four counter passes of COUNTER_PASSES (one
``rocprofv3 --pmc`` run each over ``profile_run``) and prints, per iteration
launch of the last pair, the busy fractions of the vector ALUs, the texture
address (TA) and data (TD) units and the L1 cache, the cache hit rates and
the instruction counts per wave.
"""
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(PKG, "csrc", "kernels.h")]
COPY_BYTES = 256 << 20


# The iteration kernel's source: the section of kernels.h from its own
# header line to the next section's (packed-plane loaders and buffer
# descriptors it uses sit above it and are hashed too).
ITER_SECTION = ("// ---------------------------------------------------------------- displacement update",
                "// ---------------------------------------------------------------- top-q select")


def kernel_source_sha():
    """SHA-256 of the source the iteration kernel is built from: kernels.h
    up to the end of its section (everything after it is other kernels)."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            text = fh.read().decode()
        end = text.find(ITER_SECTION[1])
        h.update((text if end < 0 else text[:end]).encode())
    return h.hexdigest()


def _dispatches(run_dir):
    path = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not path:
        raise FileNotFoundError("no counter_collection.csv under %s" % run_dir)
    out = {}
    for r in csv.DictReader(open(path[0])):
        d = out.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"], "grid": int(r["Grid_Size"])})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [out[k] for k in sorted(out)]


def _iter_algorithmic(levels, n, ts, mask_bytes=1):
    """Algorithmic bytes of the iteration launches of one pair, in launch order.
    The last launch also writes the mask stage's input: 1 B/px (the pre-mask
    of an absolute threshold, the plain path's default) or 4 B/px (|d|^2)."""
    out = []
    for l in range(levels - 1, -1, -1):
        px = (n >> l) ** 2
        for it in range(3):
            b = px * 2 * 5 * ts + px * 8
            if it > 0:
                b += px * 8
            elif l < levels - 1:
                b += (px // 4) * 8
            if l == 0 and it == 2:
                b += px * mask_bytes
            out.append((l, b))
    return out


def traffic(fetch_dir, write_dir, n=2048, levels=3, ts=4):
    fd, wd = _dispatches(fetch_dir), _dispatches(write_dir)
    cf = [d["FETCH_SIZE"] for d in fd if "copyBuffer" in d["name"]]
    cw = [d["WRITE_SIZE"] for d in wd if "copyBuffer" in d["name"]]
    f_factor = COPY_BYTES / (sum(cf) / len(cf) * 1024.0)
    w_factor = COPY_BYTES / (sum(cw) / len(cw) * 1024.0)
    fi = [d for d in fd if "k_iter" in d["name"]]
    wi = [d for d in wd if "k_iter" in d["name"]]
    alg = _iter_algorithmic(levels, n, ts)
    per = len(alg)
    if len(fi) != len(wi) or len(fi) % per:
        raise ValueError("unexpected number of iteration dispatches: %d / %d" % (len(fi), len(wi)))
    rows = []
    for i, (f, w) in enumerate(zip(fi, wi)):
        lvl, ab = alg[i % per]
        hb = f["FETCH_SIZE"] * 1024.0 * f_factor + w["WRITE_SIZE"] * 1024.0 * w_factor
        rows.append({"level": lvl, "hbm_bytes": hb, "algorithmic_bytes": ab})
    tot_h = sum(r["hbm_bytes"] for r in rows)
    tot_a = sum(r["algorithmic_bytes"] for r in rows)
    by_level = {}
    for r in rows:
        e = by_level.setdefault(r["level"], [0.0, 0.0, 0])
        e[0] += r["hbm_bytes"]
        e[1] += r["algorithmic_bytes"]
        e[2] += 1
    return {
        "kernel": "k_iter",
        "workload": "plain per-pair path, %dx%d u16, %d levels, 3 iterations, 15x15 window" % (n, n, levels),
        "kernel_source_sha256": kernel_source_sha(),
        "fetch_factor": round(f_factor, 4),
        "write_factor": round(w_factor, 4),
        "launches": len(rows),
        "hbm_bytes_per_launch": round(tot_h / len(rows)),
        "algorithmic_bytes_per_launch": round(tot_a / len(rows)),
        "hbm_over_algorithmic": round(tot_h / tot_a, 4),
        "per_level": {str(k): {"hbm_bytes_per_launch": round(v[0] / v[2]),
                               "algorithmic_bytes_per_launch": round(v[1] / v[2]),
                               "ratio": round(v[0] / v[1], 4)} for k, v in sorted(by_level.items())},
    }


def stats(stats_csv):
    rows = list(csv.DictReader(open(stats_csv)))
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows:
        out.append("| %s | %s | %.2f | %.2f | %s |" % (r["Name"].replace("|", "/"), r["Calls"],
                                                     int(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
                                                     r["Percentage"]))
    return "\n".join(out)


# Counter passes (each within one run's hardware limits: <= 8 SQ, <= 4 TCC,
# <= 4 TCP, <= 2 TA, <= 2 TD counters).
COUNTER_PASSES = [
    "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_LDS SQ_INSTS_SALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY",
    "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_VMEM SQ_ACTIVE_INST_LDS SQ_INST_CYCLES_VMEM_RD SQ_LDS_BANK_CONFLICT "
    "SQ_WAIT_INST_LDS SQ_ACTIVE_INST_ANY SQ_THREAD_CYCLES_VALU",
    "TA_TA_BUSY_sum TA_ADDR_STALLED_BY_TC_CYCLES_sum TD_TD_BUSY_sum TD_TC_STALL_sum TCP_TCC_READ_REQ_sum "
    "TCP_TOTAL_CACHE_ACCESSES_sum TCP_PENDING_STALL_CYCLES_sum TCP_TCR_TCP_STALL_CYCLES_sum GRBM_GUI_ACTIVE",
    "TCC_HIT_sum TCC_MISS_sum TCP_TCC_READ_REQ_LATENCY_sum TCP_TCP_LATENCY_sum TCP_TCP_TA_DATA_STALL_CYCLES_sum "
    "TCP_TOTAL_READ_sum",
]
N_CU, N_XCD, N_SIMD, CLOCK_GHZ = 256, 8, 1024, 2.4


def counters(pass_dirs, per_pair=9):
    """Unit utilisation of the last pair's iteration launches from the four
    counter passes. GRBM_GUI_ACTIVE counts cycles on each of the 8 XCDs;
    TA/TD/TCP sums run over the 256 CUs; a wave64 FP32 VALU instruction
    occupies a SIMD for 4 cycles."""
    runs = [[d for d in _dispatches(p) if "k_iter" in d["name"]] for p in pass_dirs]
    n = min(len(r) for r in runs)
    out = []
    for i in range(n - per_pair, n):
        c = {}
        for r in runs:
            c.update({k: v for k, v in r[i].items() if k not in ("name", "grid")})
        cyc = c["GRBM_GUI_ACTIVE"] / N_XCD
        acc = c["TCP_TOTAL_CACHE_ACCESSES_sum"]
        out.append({
            "launch": i % per_pair, "grid": runs[0][i]["grid"], "kernel": runs[0][i]["name"].split("(")[0],
            "us": round(cyc / (CLOCK_GHZ * 1e3), 1),
            "valu_busy": round(4 * c["SQ_INSTS_VALU"] / N_SIMD / cyc, 3),
            "ta_busy": round(c["TA_TA_BUSY_sum"] / N_CU / cyc, 3),
            "td_busy": round(c["TD_TD_BUSY_sum"] / N_CU / cyc, 3),
            "td_stalled_on_l1": round(c["TD_TC_STALL_sum"] / N_CU / cyc, 3),
            "l1_pending_stall": round(c["TCP_PENDING_STALL_CYCLES_sum"] / N_CU / cyc, 3),
            "l1_hit": round(1 - c["TCP_TCC_READ_REQ_sum"] / acc, 3),
            "l2_hit": round(c["TCC_HIT_sum"] / (c["TCC_HIT_sum"] + c["TCC_MISS_sum"]), 3),
            "l2_latency_cycles": round(c["TCP_TCC_READ_REQ_LATENCY_sum"] / c["TCP_TCC_READ_REQ_sum"]),
            "l1_to_l2_MB": round(c["TCP_TCC_READ_REQ_sum"] * 128 / 1e6),
            "lds_bank_conflict": round(c["SQ_LDS_BANK_CONFLICT"] / N_CU / cyc, 3),
            "valu_per_wave": round(c["SQ_INSTS_VALU"] / c["SQ_WAVES"]),
            "vmem_per_wave": round(c["SQ_INSTS_VMEM_RD"] / c["SQ_WAVES"]),
            "lds_per_wave": round(c["SQ_INSTS_LDS"] / c["SQ_WAVES"]),
        })
    return out


def load_traffic(path):
    """Measured HBM bytes per iteration launch, or None when the summary is
    missing or the kernel sources changed since the counters were taken."""
    try:
        with open(path) as fh:
            text = fh.read()
        data = json.loads(text[text.index("{"):text.rindex("}") + 1])
    except (OSError, ValueError):
        return None
    if data.get("kernel_source_sha256") != kernel_source_sha():
        return None
    return data


if __name__ == "__main__":
    if sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3]), indent=1))
    elif sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    elif sys.argv[1] == "counters":
        for row in counters(sys.argv[2:]):
            print(json.dumps(row))
