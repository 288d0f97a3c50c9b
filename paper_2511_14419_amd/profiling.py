"""Summaries of rocprofv3 output for the iteration kernel.

``traffic`` turns two counter runs of ``profile_run`` (FETCH_SIZE, then
WRITE_SIZE, each in KiB per dispatch) into HBM bytes per launch of the
iteration kernel. Each counter is scaled by what it reads for the plain
256 MiB device copy at the start of the run (read and written bytes are
known), so the numbers are in bytes whatever the counter's own unit or
sampling. The result is compared with the algorithmic bytes of the same
launches (expansion planes of both frames + prior flow + flow out + |d|^2).

``stats`` renders a ``--kernel-trace --stats`` kernel_stats.csv as a table.
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


def kernel_source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
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
