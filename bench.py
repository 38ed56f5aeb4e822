"""Benchmark: inverse + direct spherical-harmonic transform throughput on one MI355X.

A step is one pass of the whole hot path over one batch: the inverse
transform (Legendre GEMM + ring c2r FFT) of every field, then the direct
transform (ring r2c FFT + Legendre GEMM) of the resulting grids.  Inputs are
resident in HBM before the timed region.  The default workload is TCo1279 on
O1280 with 411 fields and FP32 Legendre GEMMs; the same step is also timed in
FP64-plain and split-BF16 forms and reported beside it.

Prints one JSON line (see the design doc for every field's definition).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "fp64_TF": 78.6,
    "fp32_TF": 157.3,
    "bf16_TF": 2500.0,
}
KERNELS = ["legendre_inverse_gemm", "legendre_direct_gemm", "ring_fft_c2r", "ring_fft_r2c"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tco1279_o1280")
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--forms", default="fp64,bf16x3",
                    help="extra precision forms timed beside the headline (comma list, or none)")
    ap.add_argument("--form-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fields", type=int, default=0,
                    help="fields the oracle baseline transforms (0: as many as take about 15 s, "
                         "at most the workload's field count)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the fixed default tile shapes instead of the plan-time autotuner")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy, the reference kernel that "
                         "scales rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes")
    return ap.parse_args()


def kernel_bytes(plan, prec):
    """Algorithmic HBM bytes per launch of each kernel (roofline)."""
    info = plan.info
    F = info.nfld
    cplx = 16 if prec == "fp64" else 8
    real = 8 if prec == "fp64" else 4
    tab_el = {"fp64": 8, "fp32": 4, "bf16x3": 4}[prec]  # bf16 hi + lo
    nspec, npts, nfour = info.nspec, info.npts, info.nfour
    tables = tab_entries(plan) * tab_el
    four = F * nfour * cplx
    return {
        "legendre_inverse_gemm": tables + F * nspec * cplx + four,
        "legendre_direct_gemm": tables + four + F * nspec * cplx,
        "ring_fft_c2r": four + F * npts * real,
        "ring_fft_r2c": F * npts * real + four,
    }


def tab_entries(plan):
    """P̄ entries the method needs: sum over northern rings j and m <= M_j of (N - m + 1)."""
    N = plan.trunc
    nlon = plan.ring_lengths()[: plan.nlat // 2]
    tot = 0
    for n in nlon:
        M = min(N, (int(n) - 1) // 2)
        tot += (M + 1) * (N + 1) - M * (M + 1) // 2
    return tot


def run_form(torch, shtx, wl, prec, steps, warmup, spec_host, autotune):
    plan = shtx.Plan(wl.trunc, wl.grid, wl.nlat, wl.nfld, prec, nlon_full=wl.nlon_full, timing=True,
                     autotune=autotune)
    spec = spec_host.to(plan.complex_dtype).cuda()
    grid = torch.empty((wl.nfld, plan.npts), dtype=plan.real_dtype, device="cuda")
    out = torch.empty_like(spec)
    for _ in range(warmup):
        plan.inv(spec, out=grid)
        plan.dir(grid, out=out)
    torch.cuda.synchronize()
    plan.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.inv(spec, out=grid)
        plan.dir(grid, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, cnt = plan.timing_read()
    kern = {k: (float(ms[i]) / max(int(cnt[i]), 1)) for i, k in enumerate(KERNELS)}
    res = {
        "plan": plan, "seconds": dt, "ms_per_step": 1e3 * dt / steps,
        "fields_per_s": wl.nfld * steps / dt, "kernel_ms": kern,
        "grid": grid, "spec_out": out,
        "legendre_flops": float(plan.info.legendre_flops),
    }
    return res


def tiles_of(plan):
    i = plan.info
    return {"inverse_gemm": list(i.inv_tile), "direct_gemm": list(i.dir_tile), "fft_cap": int(i.fft_cap),
            "chosen_by": ["default", "autotuner", "tune cache"][int(i.tuned)]}


def roofline_for(res, prec):
    plan = res["plan"]
    nbytes = kernel_bytes(plan, prec)
    flops = res["legendre_flops"]
    peak_tf = {"fp64": PEAK["fp64_TF"], "fp32": PEAK["fp32_TF"], "bf16x3": PEAK["bf16_TF"]}[prec]
    out = {}
    for k, t in res["kernel_ms"].items():
        if k.startswith("legendre"):
            ach = flops / (t * 1e-3) / 1e12
            out[k] = {"bound": "mfma", "achieved": ach, "peak": peak_tf, "unit": "TFLOP/s",
                      "frac": ach / peak_tf, "ms": t, "hbm_GBps": nbytes[k] / (t * 1e-3) / 1e9,
                      "algorithmic_bytes": nbytes[k], "algorithmic_flops": flops}
        else:
            ach = nbytes[k] / (t * 1e-3) / 1e9
            out[k] = {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_GBps"], "unit": "GB/s",
                      "frac": ach / PEAK["hbm_GBps"], "ms": t, "algorithmic_bytes": nbytes[k]}
    return out


def traffic_for(kernel, workload, prec):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by
    a copy kernel of known size) from the committed counter summary, only if
    no library source (kernels, headers, planning code) has changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if rec.get("workload") != workload or rec.get("prec") != prec:
            return None
        from paper_1908_06097_amd.build import build_id
        if rec.get("library_build_id") != build_id():
            return None
        k = rec["kernels"][kernel]
        src = open(os.path.join(ROOT, "paper_1908_06097_amd", "csrc", k["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != k["source_sha256"]:
            return None
        return k["bytes_per_launch"]
    except Exception:
        return None


def cpu_baseline(wl, nfields, spec_np, target_s=15.0):
    """The oracle (inverse then direct) on a bounded sample of the workload's
    fields: `nfields` of them, or, if 0, one field and then as many more as
    bring the sample to about `target_s` seconds."""
    import numpy as np
    import oracle
    nlon = wl.ring_lengths()
    t0 = time.perf_counter()
    n = max(nfields, 1)
    g = oracle.inv(wl.trunc, nlon, spec_np[:n])
    b = oracle.dir(wl.trunc, nlon, g)
    dt = time.perf_counter() - t0
    if nfields == 0:
        more = min(wl.nfld, max(1, int(round(target_s / max(dt, 1e-6))))) - 1
        if more > 0:
            t1 = time.perf_counter()
            g2 = oracle.inv(wl.trunc, nlon, spec_np[1:1 + more])
            b2 = oracle.dir(wl.trunc, nlon, g2)
            dt += time.perf_counter() - t1
            g, b = np.concatenate([g, g2]), np.concatenate([b, b2])
            n += more
    return {"value": n / dt, "unit": "fields/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"inv+dir of {n} of the {wl.nfld} fields of {wl.name} (per-field cost is identical)",
            "seconds": dt}, g, b, n


def errors_vs_oracle(torch, res, g_ref, b_ref, wl, nfields):
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from metrics import grid_errors, spec_errors
    import oracle
    _, w = oracle.gauss(wl.nlat)
    g = res["grid"][:nfields].double().cpu().numpy()
    b = res["spec_out"][:nfields].cpu().numpy().astype(np.complex128)
    gm, gr = grid_errors(g, g_ref, wl.ring_lengths(), w)
    sm, sr = spec_errors(b, b_ref, wl.trunc)
    return {"fields": nfields, "inv_grid_e_max": float(gm.max()), "inv_grid_e_rms": float(gr.max()),
            "dir_spec_e_max": float(sm.max()), "dir_spec_e_rms": float(sr.max())}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "see DESIGN.md for how the transform would shard", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1908_06097_amd as shtx
    import synth_inputs as si

    wl = si.WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] {wl.name}: generating {wl.nfld} seeded fields", file=sys.stderr, flush=True)
    spec_np = si.spectral_fields(wl.trunc, wl.key, range(wl.nfld))
    spec_host = torch.from_numpy(spec_np)

    print(f"[bench] headline form {args.prec}", file=sys.stderr, flush=True)
    res = run_form(torch, shtx, wl, args.prec, args.steps, args.warmup, spec_host, not args.no_autotune)
    roof = roofline_for(res, args.prec)
    dom = max(roof, key=lambda k: roof[k]["ms"])
    d = roof[dom]
    roofline = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
                "frac": d["frac"], "traffic": traffic_for(dom, wl.name, args.prec), "kernel": dom}
    line = {
        "metric": "inv+dir SH transform fields/s",
        "value": res["fields_per_s"],
        "unit": "fields/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[args.prec],
        "data": "synthetic",
        "config": {"workload": wl.name, "trunc": wl.trunc, "grid": f"O{wl.nlat // 2}" if wl.grid == "octahedral"
                   else f"full {wl.nlat}x{wl.nlon_full}", "nlat": wl.nlat, "fields": wl.nfld,
                   "legendre_form": args.prec, "fft_dtype": "f64" if args.prec == "fp64" else "f32",
                   "tiles": tiles_of(res["plan"])},
        "legendre_tflops": res["legendre_flops"] * 2 / (
            (res["kernel_ms"]["legendre_inverse_gemm"] + res["kernel_ms"]["legendre_direct_gemm"]) * 1e-3) / 1e12,
        "roofline": roofline,
        "kernels": roof,
        "plan_seconds": float(res["plan"].info.plan_seconds),
    }
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline: oracle on {args.cpu_fields or 'about 15 s of'} field(s)", file=sys.stderr,
              flush=True)
        cb, g_ref, b_ref, n_ref = cpu_baseline(wl, args.cpu_fields, spec_np)
        line["cpu_baseline"] = cb
        line["error_vs_oracle"] = errors_vs_oracle(torch, res, g_ref, b_ref, wl, n_ref)
    res["plan"].close()
    del res
    torch.cuda.empty_cache()

    forms = {}
    for prec in [p for p in args.forms.split(",") if p and p != "none" and p != args.prec]:
        print(f"[bench] form {prec}", file=sys.stderr, flush=True)
        r = run_form(torch, shtx, wl, prec, args.form_steps, 1, spec_host, not args.no_autotune)
        rf = roofline_for(r, prec)
        forms[prec] = {"fields_per_s": r["fields_per_s"], "ms_per_step": r["ms_per_step"],
                       "kernel_ms": r["kernel_ms"], "tiles": tiles_of(r["plan"]),
                       "legendre_frac": {k: rf[k]["frac"] for k in rf if k.startswith("legendre")}}
        if not args.no_cpu_baseline:
            forms[prec]["error_vs_oracle"] = errors_vs_oracle(torch, r, g_ref, b_ref, wl, n_ref)
        r["plan"].close()
        del r
        torch.cuda.empty_cache()
    if forms:
        line["forms"] = forms
        if "fp64" in forms:
            line["vs_fp64_plain_same_gpu"] = line["value"] / forms["fp64"]["fields_per_s"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
