"""Benchmark: inverse + direct spherical-harmonic transform throughput on one MI355X.

A step is one pass of the whole hot path over one batch: the inverse
transform (Legendre GEMM + ring c2r FFT) of every field, then the direct
transform (ring r2c FFT + Legendre GEMM) of the resulting grids.  Inputs are
resident in HBM before the timed region.  The default workload is TCo1279 on
O1280 with 411 fields and FP32 Legendre GEMMs; the same step is also timed in
the FP64-plain and split-precision forms and reported beside it.

Each form is measured in two passes over one plan:
  1. the product path: each transform replayed as its captured hipGraph on a
     non-default stream, HIP events around every step; `value` is fields per
     second at the median step time (the minimum and the wall-clock rate are
     reported too);
  2. the kernel breakdown: the same steps launched eagerly with the library's
     per-kernel HIP events on the launch stream; these average durations give
     the roofline figures.
The forward + adjoint pair (inverse transform, then the adjoint of the
inverse applied to its grids) is timed the same way as pass 1.

Prints one JSON line; main() below assembles its keys.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "fp64_TF": 78.6,
    "fp32_TF": 157.3,
    "bf16_TF": 2500.0,
    "fp16_TF": 2500.0,
}
PEAK_TF = {"fp64": PEAK["fp64_TF"], "fp32": PEAK["fp32_TF"], "bf16x3": PEAK["bf16_TF"], "fp16x3": PEAK["fp16_TF"]}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "fp16x3": "fp16x3"}
KERNELS = ["legendre_inverse_gemm", "legendre_direct_gemm", "ring_fft_c2r", "ring_fft_r2c"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tco1279_o1280")
    ap.add_argument("--prec", default="fp32", choices=sorted(PEAK_TF))
    ap.add_argument("--forms", default="fp64,bf16x3,fp16x3",
                    help="extra precision forms timed beside the headline (comma list, or none)")
    ap.add_argument("--form-steps", type=int, default=5)
    ap.add_argument("--kernel-steps", type=int, default=5,
                    help="eager steps with per-kernel events (the roofline figures)")
    ap.add_argument("--no-pair", action="store_true", help="skip the inverse + adjoint-of-inverse pair")
    ap.add_argument("--no-energy", action="store_true", help="skip the amd-smi energy window")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the peak probes (matrix-core and vector-ALU loops, HBM copy and read)")
    ap.add_argument("--no-single-core", action="store_true",
                    help="skip the one-thread oracle run of one field")
    ap.add_argument("--cpu-fields", type=int, default=0,
                    help="fields the oracle baseline transforms (0: as many as take about 15 s, "
                         "at most the workload's field count)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the fixed default tile shapes instead of the plan-time autotuner")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy, the reference kernel that "
                         "scales rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes")
    return ap.parse_args()


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_bytes(plan, prec):
    """Algorithmic HBM bytes per launch of each kernel: the P̄ entries the method
    needs, the spectral array and the Fourier array, each once (GEMMs); the
    Fourier array and the grid, each once (FFTs)."""
    info = plan.info
    F = info.nfld
    cplx = 16 if prec == "fp64" else 8
    real = 8 if prec == "fp64" else 4
    tab_el = {"fp64": 8, "fp32": 4, "bf16x3": 4, "fp16x3": 4}[prec]  # split forms: hi + lo halves
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


def graph_steps(torch, stream, steps, warmup, fn):
    """Run `fn` (one step of graph launches on `stream`) warmup + steps times;
    HIP events around each timed step.  Returns per-step ms and the wall time."""
    for _ in range(warmup):
        fn()
    stream.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    return [a.elapsed_time(b) for a, b in ev], wall


def energy_window(torch, stream, step, step_ms, busy_s=4.0, idle_s=2.5):
    """Mean GPU power over repeated steps (graph replay) lasting about
    `busy_s` seconds and over `idle_s` idle seconds just before, through
    amd-smi; energy per step = mean busy power x median step time."""
    from energy_meter import EnergyMeter
    meter = EnergyMeter()
    if not meter.available:
        return {"error": meter.error}
    stream.synchronize()
    meter.start()
    time.sleep(idle_s)
    idle = meter.stop()
    n = max(10, int(busy_s / max(step_ms * 1e-3, 1e-6)) + 1)
    meter.start()
    for _ in range(n):
        step()
    stream.synchronize()
    busy = meter.stop()
    if busy is None or idle is None:
        return {"error": meter.error}
    w = busy["counter_mean_W"]
    return {"steps": n, "wall_s": busy["wall_s"], "mean_W": w,
            "J_per_step": w * step_ms * 1e-3 if w else None,
            "counter_updates": busy["counter_updates"], "counter_span_s": busy["counter_span_s"],
            "sampled_mean_W": busy["sampled_mean_W"],
            "sampled_J_per_step": busy["sampled_mean_W"] * step_ms * 1e-3 if busy["sampled_mean_W"] else None,
            "samples": busy["samples"], "idle_W": idle["counter_mean_W"], "idle_sampled_W": idle["sampled_mean_W"],
            "method": "amd-smi energy accumulator: energy between its updates inside the window over their "
                      "timestamps (about one update per second); socket power polled every 10 ms and "
                      "integrated by the trapezoid rule beside it; J per step = mean power x median step time"}


def run_form(torch, shtx, wl, prec, steps, warmup, kernel_steps, spec_host, autotune, pair, energy=False):
    stream = torch.cuda.Stream()  # graph replay needs a non-default stream
    with torch.cuda.stream(stream):
        plan = shtx.Plan(wl.trunc, wl.grid, wl.nlat, wl.nfld, prec, nlon_full=wl.nlon_full, graph=True,
                         timing=True, autotune=autotune)
        spec = spec_host.to(plan.complex_dtype).to("cuda", non_blocking=False)
        grid = torch.empty((wl.nfld, plan.npts), dtype=plan.real_dtype, device="cuda")
        out = torch.empty_like(spec)
        adj = torch.empty_like(spec)
        stream.synchronize()

        def step():
            plan.inv(spec, out=grid)
            plan.dir(grid, out=out)

        # 1. product path: graph replay, events around each step
        plan.timing_enable(False)
        ms, wall = graph_steps(torch, stream, steps, warmup, step)
        res = {
            "plan": plan, "grid": grid, "spec_out": out, "legendre_flops": float(plan.info.legendre_flops),
            "step_ms": ms, "ms_median": statistics.median(ms), "ms_min": min(ms), "wall_s": wall,
            "fields_per_s": wl.nfld / (statistics.median(ms) * 1e-3),
        }
        if pair:
            def pair_step():
                plan.inv(spec, out=grid)
                plan.inv_adj(grid, out=adj)
            pms, pwall = graph_steps(torch, stream, steps, 1, pair_step)
            res["pair"] = {"ms_median": statistics.median(pms), "ms_min": min(pms),
                           "fields_per_s": wl.nfld / (statistics.median(pms) * 1e-3),
                           "wall_fields_per_s": wl.nfld * steps / pwall}
            res["adj_out"] = adj
        if energy:
            res["energy"] = energy_window(torch, stream, step, res["ms_median"])
        # 2. kernel breakdown: eager launches with per-kernel events
        plan.timing_enable(True)
        step()
        stream.synchronize()
        plan.timing_reset()
        for _ in range(kernel_steps):
            step()
        stream.synchronize()
        kms, cnt = plan.timing_read()
        res["kernel_ms"] = {k: (float(kms[i]) / max(int(cnt[i]), 1)) for i, k in enumerate(KERNELS)}
        plan.timing_enable(False)
        # the outputs the error check reads come from the graph path
        step()
        if pair:
            plan.inv_adj(grid, out=adj)
        stream.synchronize()
    return res


def tiles_of(plan):
    i = plan.info
    return {"inverse_gemm": list(i.inv_tile), "direct_gemm": list(i.dir_tile), "fft_cap": int(i.fft_cap),
            "chosen_by": ["default", "autotuner", "tune cache"][int(i.tuned)]}


def roofline_for(res, prec):
    plan = res["plan"]
    nbytes = kernel_bytes(plan, prec)
    flops = res["legendre_flops"]
    peak_tf = PEAK_TF[prec]
    out = {}
    for k, t in res["kernel_ms"].items():
        if k.startswith("legendre"):
            ach = flops / (t * 1e-3) / 1e12
            out[k] = {"bound": "mfma", "achieved": ach, "peak": peak_tf, "unit": "TFLOP/s",
                      "frac": ach / peak_tf, "ms": t, "hbm_GBps": nbytes[k] / (t * 1e-3) / 1e9,
                      "hbm_frac": nbytes[k] / (t * 1e-3) / 1e9 / PEAK["hbm_GBps"],
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
        recs = json.load(open(path))
        if isinstance(recs, dict):
            recs = [recs]
        from paper_1908_06097_amd.build import build_id
        for rec in recs:
            if rec.get("workload") != workload or rec.get("prec") != prec:
                continue
            if rec.get("library_build_id") != build_id():
                return None
            k = rec["kernels"][kernel]
            src = open(os.path.join(ROOT, "paper_1908_06097_amd", "csrc", k["source"]), "rb").read()
            if hashlib.sha256(src).hexdigest() != k["source_sha256"]:
                return None
            return k["bytes_per_launch"]
    except Exception:
        return None
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, nfields, spec_np, single_core, target_s=15.0):
    """The oracle (inverse then direct) on a bounded sample of the workload's
    fields on every host thread: `nfields` of them, or, if 0, one field and
    then as many more as bring the sample to about `target_s` seconds; then,
    unless disabled, one field on one thread."""
    import numpy as np
    import oracle
    nlon = wl.ring_lengths()
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    n = max(nfields, 1)
    g = oracle.inv(wl.trunc, nlon, spec_np[:n], nthreads=cores)
    b = oracle.dir(wl.trunc, nlon, g, nthreads=cores)
    dt = time.perf_counter() - t0
    if nfields == 0:
        more = min(wl.nfld, max(1, int(round(target_s / max(dt, 1e-6))))) - 1
        if more > 0:
            t1 = time.perf_counter()
            g2 = oracle.inv(wl.trunc, nlon, spec_np[1:1 + more], nthreads=cores)
            b2 = oracle.dir(wl.trunc, nlon, g2, nthreads=cores)
            dt += time.perf_counter() - t1
            g, b = np.concatenate([g, g2]), np.concatenate([b, b2])
            n += more
    out = {"value": n / dt, "unit": "fields/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"inv+dir of {n} of the {wl.nfld} fields of {wl.name} on {cores} threads "
                     f"(per-field cost is identical)",
           "seconds": dt}
    if single_core:
        say("cpu baseline: one field on one thread")
        t1 = time.perf_counter()
        g1 = oracle.inv(wl.trunc, nlon, spec_np[:1], nthreads=1)
        oracle.dir(wl.trunc, nlon, g1, nthreads=1)
        s1 = time.perf_counter() - t1
        out["single_core"] = {"value": 1.0 / s1, "unit": "fields/s", "seconds": s1,
                              "sample": f"inv+dir of field 0 of {wl.name} on 1 thread"}
    return out, g, b, n, cores


def errors_vs_oracle(res, g_ref, b_ref, wl, nfields):
    import numpy as np
    from error_metrics import grid_errors, spec_errors
    import oracle
    _, w = oracle.gauss(wl.nlat)
    g = res["grid"][:nfields].double().cpu().numpy()
    b = res["spec_out"][:nfields].cpu().numpy().astype(np.complex128)
    gm, gr = grid_errors(g, g_ref, wl.ring_lengths(), w)
    sm, sr = spec_errors(b, b_ref, wl.trunc)
    return {"fields": nfields, "inv_grid_e_max": float(gm.max()), "inv_grid_e_rms": float(gr.max()),
            "dir_spec_e_max": float(sm.max()), "dir_spec_e_rms": float(sr.max())}


def pair_errors(res, c_ref, wl, nfields):
    """inv_adj(inv(a)) on the sampled fields against the oracle's."""
    import numpy as np
    from error_metrics import spec_errors
    c = res["adj_out"][:nfields].cpu().numpy().astype(np.complex128)
    sm, sr = spec_errors(c, c_ref, wl.trunc)
    return {"fields": nfields, "inv_adj_spec_e_max": float(sm.max()), "inv_adj_spec_e_rms": float(sr.max())}


def form_summary(res, prec, wl):
    rf = roofline_for(res, prec)
    return {"fields_per_s": res["fields_per_s"], "ms_median": res["ms_median"], "ms_min": res["ms_min"],
            "wall_fields_per_s": wl.nfld * len(res["step_ms"]) / res["wall_s"],
            "kernel_ms": res["kernel_ms"], "tiles": tiles_of(res["plan"]),
            "legendre_frac": {k: rf[k]["frac"] for k in rf if k.startswith("legendre")},
            "fft_hbm_frac": {k: rf[k]["frac"] for k in rf if k.startswith("ring")}}


# the probe whose measured rate stands beside each form's published MFMA peak
PEAK_PROBE = {"fp64": "mfma_f64_TF", "fp32": "mfma_f32_TF", "bf16x3": "mfma_bf16_TF", "fp16x3": "mfma_f16_TF"}


def measure_peaks(torch, shtx):
    """Rates this GPU sustains (shtx_probe_peak): matrix-core loops per
    precision, the non-packed FP32 vector-ALU rate, and a 1 GiB HBM copy and
    read; the published peaks stay the roofline denominators."""
    out = {}
    for kind in ("mfma_f64", "mfma_f32", "mfma_bf16", "mfma_f16", "valu_f32"):
        out[kind + "_TF"] = shtx.probe_peak(kind)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    dst = torch.empty_like(src)
    out["hbm_copy_GB_s"] = shtx.probe_peak("hbm_copy", src, dst)
    out["hbm_read_GB_s"] = shtx.probe_peak("hbm_read", src)
    del src, dst
    torch.cuda.empty_cache()
    out["method"] = ("one warm-up and three timed launches each (HIP events): 8 independent MFMA chains per wave "
                     "on register operands; 8 FP32 FMA chains per lane; 16-byte grid-stride copy (read + write "
                     "counted) and read of 1 GiB")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: one GPU only (asked for --gpus {args.gpus}); fields are independent, so "
              "P GPUs would each transform F/P of them with their own copy of the tables", file=sys.stderr)
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
    say(f"{wl.name}: generating {wl.nfld} seeded fields")
    spec_np = si.spectral_fields(wl.trunc, wl.key, range(wl.nfld))
    spec_host = torch.from_numpy(spec_np)
    pair = not args.no_pair

    say(f"headline form {args.prec}")
    res = run_form(torch, shtx, wl, args.prec, args.steps, args.warmup, args.kernel_steps, spec_host,
                   not args.no_autotune, pair, energy=not args.no_energy)
    say(f"  {res['fields_per_s']:.1f} fields/s (median {res['ms_median']:.3f} ms, min {res['ms_min']:.3f} ms)")
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
        "ms_per_step": res["ms_median"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": wl.name, "trunc": wl.trunc, "grid": f"O{wl.nlat // 2}" if wl.grid == "octahedral"
                   else f"full {wl.nlat}x{wl.nlon_full}", "nlat": wl.nlat, "fields": wl.nfld,
                   "legendre_form": args.prec, "fft_dtype": "f64" if args.prec == "fp64" else "f32",
                   "tiles": tiles_of(res["plan"])},
        "timing": {"path": "hipGraph replay, one inverse and one direct graph per step, non-default stream",
                   "ms_median": res["ms_median"], "ms_min": res["ms_min"],
                   "wall_fields_per_s": wl.nfld * args.steps / res["wall_s"],
                   "kernel_breakdown": f"{args.kernel_steps} eager steps, library HIP events per kernel"},
        "legendre_tflops": res["legendre_flops"] * 2 / (
            (res["kernel_ms"]["legendre_inverse_gemm"] + res["kernel_ms"]["legendre_direct_gemm"]) * 1e-3) / 1e12,
        "roofline": roofline,
        "kernels": roof,
        "plan_seconds": float(res["plan"].info.plan_seconds),
    }
    if pair:
        line["pair_fwd_adj"] = dict(res["pair"], what="inv_trans then inv_trans_adj of its grids (graph replay)")
    if "energy" in res:
        en = dict(res["energy"])
        if en.get("J_per_step"):
            en["J_per_field_pair"] = en["J_per_step"] / wl.nfld
            en["fields_per_J"] = wl.nfld / en["J_per_step"]
        line["energy"] = en
    if not args.no_cpu_baseline:
        say(f"cpu baseline: oracle on {args.cpu_fields or 'about 15 s of'} field(s)")
        cb, g_ref, b_ref, n_ref, cores = cpu_baseline(wl, args.cpu_fields, spec_np, not args.no_single_core)
        line["cpu_baseline"] = cb
        line["error_vs_oracle"] = errors_vs_oracle(res, g_ref, b_ref, wl, n_ref)
        if pair:
            import oracle
            c_ref = oracle.inv_adj(wl.trunc, wl.ring_lengths(), g_ref, nthreads=cores)
            line["pair_fwd_adj"]["error_vs_oracle"] = pair_errors(res, c_ref, wl, n_ref)
    res["plan"].close()
    del res
    torch.cuda.empty_cache()

    forms = {}
    for prec in [p for p in args.forms.split(",") if p and p != "none" and p != args.prec]:
        say(f"form {prec}")
        r = run_form(torch, shtx, wl, prec, args.form_steps, 1, max(2, args.kernel_steps // 2), spec_host,
                     not args.no_autotune, False)
        forms[prec] = form_summary(r, prec, wl)
        say(f"  {r['fields_per_s']:.1f} fields/s")
        if not args.no_cpu_baseline:
            forms[prec]["error_vs_oracle"] = errors_vs_oracle(r, g_ref, b_ref, wl, n_ref)
        r["plan"].close()
        del r
        torch.cuda.empty_cache()
    if forms:
        line["forms"] = forms
        if "fp64" in forms:
            line["vs_fp64_plain_same_gpu"] = line["value"] / forms["fp64"]["fields_per_s"]
    if not args.no_peaks:
        say("peak probes")
        peaks = measure_peaks(torch, shtx)
        line["peaks_measured"] = peaks
        key = {"TFLOP/s": PEAK_PROBE[args.prec], "GB/s": "hbm_copy_GB_s"}[roofline["unit"]]
        if peaks.get(key):
            line["roofline_vs_measured"] = {"peak": peaks[key], "probe": key,
                                            "frac": roofline["achieved"] / peaks[key]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
