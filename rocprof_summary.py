"""Summarise rocprofv3 runs of bench.py into the text files under profiles/.

Usage (after the four runs listed in profiles/README.md):
    python rocprof_summary.py --trace DIR --fetch DIR --write DIR [--sq DIR]
                              --workload "TCo1279 O1280" --prec fp32 -- <command...>

Writes profiles/<kernel>_<workload>_<prec>.md for each of the four bench
stages: the average duration per stage call from the kernel trace (each
kernel's first, warm-up dispatch left out), the HBM bytes from FETCH_SIZE /
WRITE_SIZE scaled by the 1 GiB calibration copy, and, with --sq, the shader
counters of the stage (matrix-core busy fraction, VALU and LDS instructions
per CU-cycle, LDS bank-conflict cycles, the clock the kernels ran at).  The
record of (workload, prec) in profiles/traffic.json is replaced: bytes per
launch per stage with the sha256 of the stage's source file and the hash of
every library source.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNELS = {  # bench.py name -> source file the stage's kernels are built from
    "legendre_inverse_gemm": "k_gemm.hip",
    "legendre_direct_gemm": "k_gemm.hip",
    "ring_fft_c2r": "k_fft.hip",
    "ring_fft_r2c": "k_fft.hip",
}
COPY_BYTES = 1 << 30
N_CU, N_SIMD, N_XCD = 256, 1024, 8
SQ_COUNTERS = ["SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_LDS",
               "SQ_LDS_BANK_CONFLICT", "SQ_WAVES", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"]


def classify(name):
    if "k_probe" in name:
        return None  # the bench's peak probes, not a transform stage
    if "k_spec_absmax" in name or "k_clear_u32" in name:
        # the split-half form's per-field maxima (cleared, then taken), launched
        # with the inverse GEMM
        return "legendre_inverse_gemm"
    if "k_uv_spec" in name:
        # the wind step, launched with the inverse GEMM it feeds
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


def stage_durations(trace):
    """Per stage: (ms per stage call, calls, kernel names).  The first dispatch
    of each kernel is the bench's untimed warm-up call; a stage of several
    kernels (a GEMM's main and column-tail launches) sums their averages."""
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
    return dur


def counters(d, names):
    """Per stage and counter: the sum over the stage's kernels of each kernel's
    mean per dispatch; 'copy': every value of the calibration copy."""
    rows = list(csv.DictReader(open(one(os.path.join(d, "**", "*counter_collection.csv")))))
    per = {}
    for r in rows:
        c = r["Counter_Name"]
        if c not in names:
            continue
        k = classify(r["Kernel_Name"])
        if k == "copy" and c in ("FETCH_SIZE", "WRITE_SIZE") and float(r["Counter_Value"]) * 1024 < COPY_BYTES / 2:
            continue  # the fill kernels of the calibration tensors, not the copy
        if k:
            per.setdefault((k, c), {}).setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    out = {}
    for (k, c), by_name in per.items():
        if k == "copy":
            out[(k, c)] = [x for v in by_name.values() for x in v]
        else:
            out[(k, c)] = sum(statistics.mean(v) for v in by_name.values())
    return out


def sq_metrics(sq, k):
    """Rates per cycle from one stage's SQ counters.  GRBM_GUI_ACTIVE counts the
    busy cycles of each XCD's graphics engine, summed over the 8 XCDs."""
    g = {c: sq.get((k, c)) for c in SQ_COUNTERS}
    if not g["GRBM_GUI_ACTIVE"]:
        return None
    cyc = g["GRBM_GUI_ACTIVE"] / N_XCD
    out = {"cycles": cyc,
           "mfma_busy_per_simd": (g["SQ_VALU_MFMA_BUSY_CYCLES"] or 0) / (cyc * N_SIMD),
           "valu_insts_per_cu_cycle": (g["SQ_INSTS_VALU"] or 0) / (cyc * N_CU),
           "lds_insts_per_cu_cycle": (g["SQ_INSTS_LDS"] or 0) / (cyc * N_CU),
           "lds_bank_conflict_cycles_per_cu_cycle": (g["SQ_LDS_BANK_CONFLICT"] or 0) / (cyc * N_CU),
           "mfma_insts": g["SQ_INSTS_MFMA"], "valu_insts": g["SQ_INSTS_VALU"], "waves": g["SQ_WAVES"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--sq")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--prec", required=True)
    ap.add_argument("command", nargs=argparse.REMAINDER)
    a = ap.parse_args()
    command = " ".join(x for x in a.command if x != "--")
    dur = stage_durations(a.trace)
    fr = counters(a.fetch, {"FETCH_SIZE"})
    wr = counters(a.write, {"WRITE_SIZE"})
    sq = counters(a.sq, set(SQ_COUNTERS)) if a.sq else {}
    f_scale = COPY_BYTES / (max(fr[("copy", "FETCH_SIZE")]) * 1024)
    w_scale = COPY_BYTES / (max(wr[("copy", "WRITE_SIZE")]) * 1024)
    sys.path.insert(0, ROOT)
    from paper_1908_06097_amd.build import build_id
    rec = {"workload": a.workload, "prec": a.prec, "command": command, "library_build_id": build_id(),
           "copy_calibration": {"fetch_scale": f_scale, "write_scale": w_scale}, "kernels": {}}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    tag = a.workload.lower().replace(" ", "_")
    for k, src in KERNELS.items():
        if k not in dur:
            continue
        ms, calls, names = dur[k]
        fb = fr.get((k, "FETCH_SIZE"), 0.0) * 1024 * f_scale
        wb = wr.get((k, "WRITE_SIZE"), 0.0) * 1024 * w_scale
        sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1908_06097_amd", "csrc", src), "rb").read()).hexdigest()
        rec["kernels"][k] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                             "avg_ms": ms, "calls": calls, "source": src, "source_sha256": sha}
        m = sq_metrics(sq, k) if sq else None
        if m:
            rec["kernels"][k]["sq"] = m
        with open(os.path.join(ROOT, "profiles", f"{k}_{tag}_{a.prec}.md"), "w") as fh:
            fh.write(f"# {k} — {a.workload}, {a.prec}\n\n")
            fh.write("Kernels: " + ", ".join(f"`{n}`" for n in names) + "\n\n")
            fh.write(f"* rocprofv3 kernel trace: {calls} timed stage calls (warm-up call left out), average "
                     f"{ms:.3f} ms per call{' (sum of its kernels)' if len(names) > 1 else ''}\n")
            fh.write(f"* FETCH_SIZE per launch: {fb / 1e9:.3f} GB (raw x {f_scale:.3f}, scale from a 1 GiB copy)\n")
            fh.write(f"* WRITE_SIZE per launch: {wb / 1e9:.3f} GB (raw x {w_scale:.3f})\n")
            fh.write(f"* HBM traffic per launch: {(fb + wb) / 1e9:.3f} GB -> {(fb + wb) / (ms * 1e-3) / 1e9:.0f} GB/s\n")
            if m:
                clk = m["cycles"] / (ms * 1e-3) / 1e9
                fh.write(f"* shader counters per stage call ({m['cycles']:.3g} cycles per XCD, {clk:.2f} GHz "
                         f"over the traced duration): matrix cores busy {m['mfma_busy_per_simd']:.3f} of SIMD "
                         f"cycles; {m['valu_insts_per_cu_cycle']:.3f} VALU and {m['lds_insts_per_cu_cycle']:.3f} "
                         f"LDS instructions per CU-cycle; LDS bank conflicts "
                         f"{m['lds_bank_conflict_cycles_per_cu_cycle']:.3f} cycles per CU-cycle; "
                         f"{m['mfma_insts']:.4g} MFMA and {m['valu_insts']:.4g} VALU instructions\n")
            fh.write("\nCommands (run from the repository root on an MI355X):\n\n```\n")
            fh.write(f"{command}\n```\n")
    path = os.path.join(ROOT, "profiles", "traffic.json")
    recs = []
    if os.path.exists(path):
        old = json.load(open(path))
        recs = old if isinstance(old, list) else [old]
    recs = [r for r in recs if (r.get("workload"), r.get("prec")) != (a.workload, a.prec)] + [rec]
    with open(path, "w") as fh:
        json.dump(recs, fh, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
