"""Summarise rocprofv3 runs of bench.py into the text files under profiles/.

Usage (after the three runs listed in profiles/README.md):
    python rocprof_summary.py <trace_dir> <fetch_dir> <write_dir> <workload> <prec> <command...>

Writes profiles/<kernel>_<workload>_<prec>.md (average duration per kernel
from the kernel trace, without each kernel's first (warm-up) dispatch, and HBM bytes from FETCH_SIZE / WRITE_SIZE scaled by
the 1 GiB calibration copy) and profiles/traffic.json (bytes per launch per
kernel with the sha256 of the source file the kernel was built from, and the
hash of every library source).
"""
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNELS = {  # bench.py name -> (unused, source file the kernel is built from)
    "legendre_inverse_gemm": ((), "k_gemm.hip"),
    "legendre_direct_gemm": ((), "k_gemm.hip"),
    "ring_fft_c2r": ((), "k_fft.hip"),
    "ring_fft_r2c": ((), "k_fft.hip"),
}
COPY_BYTES = 1 << 30


def classify(name):
    if "k_spec_absmax" in name:
        # the split-half form's per-field maxima, launched with the inverse GEMM
        return "legendre_inverse_gemm"
    if "k_leg_mfma" in name or "k_leg_split" in name:
        # the inverse-shaped instantiation has template argument INV = true
        # (5th of k_leg_mfma<T, BM, BN, BK, INV, NW> and of
        # k_leg_split<F16, BM, BN, BK, INV>)
        args = re.search(r"<([^<>]*)>", name)
        if args:
            parts = [x.strip() for x in args.group(1).split(",")]
            inv = len(parts) > 4 and parts[4] == "true"
        else:
            inv = name.endswith("Lb1EEEvNS0_8GemmArgsE") or "Lb1ELi8E" in name or "Lb1ELi4E" in name
        return "legendre_inverse_gemm" if inv else "legendre_direct_gemm"
    if "k_fft_c2r" in name:
        return "ring_fft_c2r"
    if "k_fft_r2c" in name or "k_zero_u32" in name:
        return "ring_fft_r2c"
    if "copy" in name.lower() or "elementwise" in name.lower():
        return "copy"
    return None


def one(pattern):
    files = glob.glob(pattern, recursive=True)
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[0]


def main():
    trace, fetch, write, workload, prec = sys.argv[1:6]
    command = " ".join(sys.argv[6:])
    # per kernel, dispatch durations from the kernel trace in launch order; the
    # first dispatch of each kernel is the bench's untimed warm-up call and is
    # left out.  A stage may be more than one kernel (a GEMM's main and
    # column-tail launches, one each per stage call): its time per call is the
    # sum of its kernels' averages.
    rows = list(csv.DictReader(open(one(os.path.join(trace, "**", "*kernel_trace.csv")))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    per_name = {}
    for r in rows:
        k = classify(r["Kernel_Name"])
        if k and k != "copy":
            d_ms = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
            per_name.setdefault(k, {}).setdefault(r["Kernel_Name"], []).append(d_ms)
    dur = {}
    for k, by_name in per_name.items():
        ms = sum(statistics.mean(v[1:] if len(v) > 1 else v) for v in by_name.values())
        calls = max(max(len(v) - 1, 1) for v in by_name.values())
        dur[k] = (ms, calls, list(by_name))

    def counter(d, cname):
        """Per stage: the sum over its kernels of each kernel's mean per dispatch."""
        rows = list(csv.DictReader(open(one(os.path.join(d, "**", "*counter_collection.csv")))))
        per = {}
        for r in rows:
            if r["Counter_Name"] != cname:
                continue
            k = classify(r["Kernel_Name"])
            if k == "copy" and float(r["Counter_Value"]) * 1024 < COPY_BYTES / 2:
                continue  # the fill kernels of the calibration tensors, not the copy
            if k:
                per.setdefault(k, {}).setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        out = {k: [sum(statistics.mean(v) for v in by_name.values())] for k, by_name in per.items() if k != "copy"}
        out["copy"] = [x for v in per.get("copy", {}).values() for x in v]  # calibration: largest single copy
        return out

    fr, wr = counter(fetch, "FETCH_SIZE"), counter(write, "WRITE_SIZE")
    f_scale = COPY_BYTES / (max(fr["copy"]) * 1024)
    w_scale = COPY_BYTES / (max(wr["copy"]) * 1024)
    sys.path.insert(0, ROOT)
    from paper_1908_06097_amd.build import build_id
    out = {"workload": workload, "prec": prec, "command": command, "library_build_id": build_id(),
           "copy_calibration": {"fetch_scale": f_scale, "write_scale": w_scale}, "kernels": {}}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    for k, (_, src) in KERNELS.items():
        if k not in dur:
            continue
        fb = statistics.mean(fr.get(k, [0])) * 1024 * f_scale
        wb = statistics.mean(wr.get(k, [0])) * 1024 * w_scale
        sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1908_06097_amd", "csrc", src), "rb").read()).hexdigest()
        out["kernels"][k] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                             "avg_ms": dur[k][0], "calls": dur[k][1], "source": src, "source_sha256": sha}
        tag = workload.lower().replace(" ", "_")
        with open(os.path.join(ROOT, "profiles", f"{k}_{tag}_{prec}.md"), "w") as fh:
            fh.write(f"# {k} — {workload}, {prec}\n\n")
            fh.write("Kernels: " + ", ".join(f"`{n}`" for n in dur[k][2]) + "\n\n")
            fh.write(f"* rocprofv3 kernel trace: {dur[k][1]} timed stage calls (warm-up call left out), average "
                     f"{dur[k][0]:.3f} ms per call{' (sum of its kernels)' if len(dur[k][2]) > 1 else ''}\n")
            fh.write(f"* FETCH_SIZE per launch: {fb / 1e9:.3f} GB (raw x {f_scale:.3f}, scale from a 1 GiB copy)\n")
            fh.write(f"* WRITE_SIZE per launch: {wb / 1e9:.3f} GB (raw x {w_scale:.3f})\n")
            fh.write(f"* HBM traffic per launch: {(fb + wb) / 1e9:.3f} GB -> {(fb + wb) / (dur[k][0] * 1e-3) / 1e9:.0f} GB/s\n\n")
            fh.write("Commands (run from the repository root on the GPU box):\n\n```\n")
            fh.write(f"{command}\n```\n")
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
