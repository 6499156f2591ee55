"""Benchmark: output pixels/s of the FFT convolution hot path on one MI355X.

One step = one lp_convolve of the whole map (rows forward transform, column
transform x kernel spectrum x inverse, rows inverse transform with crop) with
the map already resident in HBM.  Default workload: the continental map,
16384x16384 FP32 city-cluster radiance (6000 blobs, 20% background), 2001x2001
kernel d^-2.5 exp(-d/80 km) cut at 500 km (0.5 km pitch), padded to
18432x18432, run three times on the same map: plain FP32 transforms (`value`,
`ms_per_step`) and the two split-precision matrix-core forms (BF16 x3 and
FP16 hi+lo operands, FP32 accumulation) beside it.

Each form: W warm-up steps, then exactly K steps between two HIP events with
nothing else recorded inside (`ms_per_step`); then, separately, K steps with
an event pair each (`median_ms`) and K steps with per-stage events (the stage
times and the roofline entry of the dominant kernel, the column stage).  The
FP64 CPU oracle is timed on a bounded pixel sample on the host cores (all
threads, and one), and its values on that sample are compared with every
form's output.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# rocprofv3 --pmc summaries of the column stage, per workload: one block per
# column variant (kernel name, FETCH_SIZE / WRITE_SIZE KiB per dispatch, VALU
# wave-instructions), with the kernel-source hash they were taken on
PMC_FILES = {"country": os.path.join(ROOT, "profiles", "pmc_cols_conv_country4096.txt"),
             "continental": os.path.join(ROOT, "profiles", "pmc_cols_conv_continental16384.txt"),
             "paper": os.path.join(ROOT, "profiles", "pmc_cols_conv_paper11920x11804.txt")}
KERNEL_SOURCES = ["paper_1907_02891_amd/csrc/lp_kernels.hip", "paper_1907_02891_amd/csrc/fft_lds.h",
                  "paper_1907_02891_amd/csrc/fft_reg.h", "paper_1907_02891_amd/csrc/lp_internal.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workloads():
    from paper_1907_02891_amd import synth
    return {
        "country": (synth.COUNTRY, synth.country_inputs),
        "small": (synth.SMALL, synth.small_inputs),
        "adjoint": (synth.ADJOINT, lambda: synth.adjoint_inputs()[:2]),
        "continental": (synth.CONTINENTAL, synth.continental_inputs),
        "large": (synth.LARGE, synth.large_inputs),
        "paper": (synth.PAPER, synth.paper_inputs),
    }


def model_bytes_four_step(ny, nx, py, px, form):
    """As model_bytes, for a plan whose padded columns take the four-step
    column stage: the outer forward reads the ny stored rows and writes a
    Py-long scratch column, the middle reads and writes it and reads the
    spectrum (all Py rows: 4 B real or 8 B complex), the outer inverse reads
    it and writes the ny rows back."""
    h = px // 2 + 1
    kh = (4 if form == 1 else 8) * py * h
    cols = 8 * h * (2 * ny + 4 * py) + kh
    path = 4 * ny * nx + 4 * ny * nx + 2 * 8 * ny * h + cols
    return path, cols, kh


def model_bytes(ny, nx, py, px, form):
    """Algorithmic HBM bytes: whole path (three passes) and the column stage.

    Whole path: read R, write S (4 B/px each), write+read the intermediate
    after the row pass and after the column pass (2 x 2 x 8 B per stored
    complex, ny x (Px/2+1)), read the stored spectrum once.
    Column stage: read and write the intermediate, read the spectrum."""
    h = px // 2 + 1
    kh = 4 * (py // 2 + 1) * h if form == 1 else 8 * py * h
    inter = 8 * ny * h
    path = 4 * ny * nx + 4 * ny * nx + 4 * inter + kh
    cols = 2 * inter + kh
    return path, cols, kh


def read_pmc(src_hash, workload, config_name, col_variant):
    """(HBM bytes, VALU wave-instructions) per column-stage dispatch from the
    committed rocprofv3 --pmc summary of this workload, if it was taken on
    the current kernel sources, the same configuration and the column
    variant this run chose (else None for each)."""
    path = PMC_FILES.get(workload)
    if path is None or col_variant is None or not os.path.exists(path):
        return None, None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != src_hash or vals.get("workload") != config_name:
        return None, None
    pre = f"variant {col_variant} "
    try:
        f = float(vals[pre + "fetch_kib_per_dispatch"]) * float(vals.get("fetch_scale", 1.0))
        w = float(vals[pre + "write_kib_per_dispatch"]) * float(vals.get("write_scale", 1.0))
    except (KeyError, ValueError):
        return None, None
    valu = vals.get(pre + "valu_wave_instructions_per_dispatch")
    return (f + w) * 1024.0, (float(valu) if valu else None)


def host_cpu():
    """The host's core count and CPU model (lscpu), for the CPU baseline."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info["lscpu " + k.strip()] = v.strip()
    except (OSError, ValueError):
        pass
    return info


def cpu_leg(oracle_at, n_total, gpu_at, budget_s, unit, what, one_core_s=None):
    """The CPU baseline: the FP64 oracle as it stands, timed on the host cores
    on a uniformly drawn sample of output units sized to about budget_s of
    work; its values on that sample are also compared with the GPU result at
    the same units (relative L2 and max error over max |value|).
    oracle_at(idx) -> FP64 values at flat unit indices; gpu_at(idx) -> the
    GPU's values there, or a dict of such functions (one per arithmetic form,
    all checked on the same sample).  one_core_s: also time the oracle on one
    thread over a sample sized to about that many seconds."""
    import oracle
    rng = np.random.default_rng(99)
    n = 16
    for _ in range(2):  # the first round also starts the thread pool
        t0 = time.perf_counter()
        oracle_at(np.sort(rng.choice(n_total, min(n, n_total), replace=False)))
        dt = time.perf_counter() - t0
        n = int(max(16, min(n_total, n * min(budget_s, 2.0) / max(dt, 1e-6))))
    n = int(max(16, min(n_total, n * budget_s / 2.0)))
    idx = np.sort(rng.choice(n_total, n, replace=False))
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    ref = oracle_at(idx)
    dt = time.perf_counter() - t0
    rate = n / dt

    def parity(fn):
        got = fn(idx)
        return {"units": int(n), "rel_l2": oracle.rel_l2(got, ref), "max_err_frac": oracle.max_err_frac(got, ref)}

    out = {"value": rate, "unit": unit, "cores": threads, "kind": "oracle",
           "sample": f"{n} uniformly drawn {what}, {dt:.1f} s on {threads} threads"}
    if isinstance(gpu_at, dict):
        out["parity"] = {k: parity(f) for k, f in gpu_at.items()}
    else:
        out["parity"] = parity(gpu_at)
    if one_core_s:
        n1 = int(max(4, min(n, rate / threads * one_core_s)))
        idx1 = idx[:n1]
        oracle.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            oracle_at(idx1)
            dt1 = time.perf_counter() - t0
        finally:
            oracle.set_num_threads(threads)
        out["one_core"] = {"value": n1 / dt1, "unit": unit, "cores": 1,
                           "sample": f"the first {n1} units of the same sample, {dt1:.1f} s"}
    out["host"] = host_cpu()
    return out


def cpu_baseline(R, K, budget_s, gpu_at, one_core_s=None):
    """The oracle's direct FP64 sum of the same map on sampled output pixels."""
    import oracle
    Rd = R.astype(np.float64)
    return cpu_leg(lambda idx: oracle.conv_same_pixels(Rd, K, idx), R.size, gpu_at,
                   budget_s, "output pixels/s",
                   f"output pixels of the same map, FP64 direct sum over the {K.shape[0]}x{K.shape[1]} kernel",
                   one_core_s)


PRECISIONS = {"fp32": (0, "f32", "FP32 FFT convolution"),
              "fp16x2": (1, "f16x2 split, f32 accumulate",
                         "FFT convolution, radix-16 passes on MFMA with FP16 hi+lo operands"),
              "bf16x3": (2, "bf16x3 split, f32 accumulate",
                         "FFT convolution, radix-16 passes on MFMA with BF16 x3 operands")}
# the headline metric: the plain FP32 form beside the split-BF16 matrix-core form
METRIC = "output pixels/s per MI355X (FP32 vs split-BF16 MFMA FFT) at rel-L2 <=1e-5"


def timed_steps(fn, stream, steps):
    """Wall time of exactly `steps` calls on `stream` between two HIP events,
    synchronised on both sides; nothing else is recorded inside."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def per_step_ms(fn, stream, steps):
    """Each of `steps` calls between its own pair of events (a separate pass
    after the timed one): the per-step times, for the median."""
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for k in range(steps):
        fn()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    return [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]


def kernels_label(lp, plan):
    """Which stages run specialised (register-resident) kernels: the split
    forms have them for the rows of some lengths only (radix-16 pass on the
    matrix cores); their column stage is generic."""
    if plan.kernels != lp.KERNELS_SPECIALISED:
        return "generic"
    rows = plan.variant_count(lp.STAGE_ROWS) > 0
    cols = plan.variant_count(lp.STAGE_COLUMNS) > 0 or (plan.column_split[0] > 1 and plan.precision == 0)
    if rows and cols:
        return "specialised"
    return "specialised rows, generic columns" if rows else "specialised columns, generic rows"


def bench_form(lp, torch, wl, K, x, args, precision, pad, stream, dev):
    """One arithmetic form on one plan: set-up (plan, spectrum, autotuner),
    warm-up, the timed steps, then the per-step and per-stage passes.
    Returns the plan's figures and its output."""
    ny, nx = x.shape
    mode, dtype, what = PRECISIONS[precision]
    t0 = time.perf_counter()
    plan = lp.Plan(ny, nx, *K.shape, pitch_km=wl.pitch_km, padding=pad)
    plan.set_precision(mode)
    if args.kernels == "generic":
        plan.set_kernels(lp.KERNELS_GENERIC)
    plan.bind(device=dev, stream=stream)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan.set_kernel(K)
    t_spec = time.perf_counter() - t0
    y = torch.empty_like(x)
    t0 = time.perf_counter()
    tuning = None
    if args.variants:
        for st, k in zip((lp.STAGE_ROWS, lp.STAGE_COLUMNS, lp.STAGE_ROWS_INVERSE), args.variants.split(",")):
            if plan.variant_count(st) > 0:
                plan.set_variant(st, int(k))
    elif not args.no_tune and plan.kernels == lp.KERNELS_SPECIALISED:
        from paper_1907_02891_amd import tune
        tuning = tune.autotune(plan, x, y, use_cache=False)
    t_tune = time.perf_counter() - t0

    def step():
        plan.convolve(x, out=y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ms_total = timed_steps(step, stream, args.steps)
    wall = time.perf_counter() - w0
    ms_step = ms_total / args.steps
    steps_ms = per_step_ms(step, stream, max(args.steps, 20))
    # per-stage HIP events on every call of a separate pass
    plan.timing(True, every=1)
    timed_steps(step, stream, max(args.steps, 20))
    stage_ms, calls = plan.stage_ms()
    plan.timing(False)
    stage_avg = [v / max(calls, 1) for v in stage_ms]

    variants = {}
    if plan.kernels == lp.KERNELS_SPECIALISED:
        for name, st in (("rows", lp.STAGE_ROWS), ("columns", lp.STAGE_COLUMNS), ("rows_inverse", lp.STAGE_ROWS_INVERSE)):
            if plan.variant_count(st) > 0:
                t = (tuning or {}).get("rows" if st != lp.STAGE_COLUMNS else "columns", {})
                tried = {lp.STAGE_ROWS: t.get("forward_ms", t.get("all", [])), lp.STAGE_COLUMNS: t.get("all", []),
                         lp.STAGE_ROWS_INVERSE: t.get("inverse_ms", [])}[st]
                variants[name] = {"chosen": plan.variant(st), "info": plan.variant_info(st, plan.variant(st)),
                                  "tried_ms": [round(v, 5) for v in tried]}
    py, px = plan.padding
    res = {"precision": precision, "dtype": dtype, "what": what,
           "value": ny * nx / (ms_step * 1e-3), "ms_per_step": round(ms_step, 5),
           "median_ms": round(float(np.median(steps_ms)), 5),
           "stage_ms": [round(v, 5) for v in stage_avg], "stage_calls": calls,
           "padding": [py, px], "form": plan.form, "shape": plan.shape,
           "kernels": kernels_label(lp, plan),
           "four_step": plan.column_split[0] > 1, "column_split": plan.column_split,
           "col_variant": plan.variant(lp.STAGE_COLUMNS) if plan.kernels == lp.KERNELS_SPECIALISED and
           plan.variant_count(lp.STAGE_COLUMNS) > 0 else None,
           "variants": variants, "wall_s": round(wall, 4),
           "setup_s": {"plan_bind": round(t_plan, 3), "kernel_spectrum": round(t_spec, 3),
                       "autotune": round(t_tune, 3)}}
    del plan
    return res, y


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="continental",
                    choices=["country", "small", "adjoint", "continental", "large", "slab", "batched", "classes", "reproject",
                             "bands", "paper"])
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work (all threads)")
    ap.add_argument("--cpu-one-core", type=float, default=4.0, help="seconds of oracle work on one thread")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (variant 0 of each stage)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for PMC byte calibration)")
    ap.add_argument("--precision", default="all", choices=list(PRECISIONS) + ["all"],
                    help="transform arithmetic: FP32 vector ALU, radix-16 passes on the matrix cores with "
                         "FP16 hi+lo / BF16 x3 split operands, or all three on the same map (FP32 is `value`)")
    ap.add_argument("--kernels", default="auto", choices=["auto", "generic"],
                    help="generic: LDS-staged kernels only (no specialised register kernels)")
    ap.add_argument("--padding", default="config", choices=["config", "window"],
                    help="config: the workload's padded size; window: the smallest size that still "
                         "gives the exact input-sized window (n + floor(k/2) per axis)")
    ap.add_argument("--branches", type=int, default=None,
                    help="batched workload: parallel class branches of the captured graph (1 to 4; "
                         "default: the autotuner's choice)")
    ap.add_argument("--pad", default=None,
                    help="PY,PX: explicit padded sizes (>= n + floor(k/2), 5-smooth, PX even) instead of --padding")
    ap.add_argument("--variants", default=None,
                    help="ROWS,COLUMNS[,ROWS_INVERSE]: run these specialised variants instead of autotuning")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_02891_amd import lp

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "classes":
        return bench_classes(args)
    if args.workload == "reproject":
        return bench_reproject(args)
    if args.workload == "bands":
        return bench_bands(args)
    if args.workload == "slab":
        return bench_slab(args)
    wl, make_inputs = workloads()[args.workload]
    t0 = time.perf_counter()
    R, K = make_inputs()
    t_gen = time.perf_counter() - t0
    ny, nx = R.shape
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    pad = (wl.py, wl.px) if args.padding == "config" else lp.window_padding(ny, nx, *K.shape)
    if args.pad:
        pad = tuple(int(v) for v in args.pad.split(","))
    forms = ["fp32", "bf16x3", "fp16x2"] if args.precision == "all" else [args.precision]

    x = torch.from_numpy(R).to(dev)
    results, samples = {}, {}
    for prec in forms:
        res, y = bench_form(lp, torch, wl, K, x, args, prec, pad, stream, dev)
        results[prec] = res
        samples[prec] = y.cpu().numpy().ravel()
        del y
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    head = results[forms[0]]

    py, px = head["padding"]
    path_b, cols_b, kh_b = (model_bytes_four_step if head["four_step"] else model_bytes)(ny, nx, py, px, head["form"])
    src_hash = kernel_source_hash()
    config_name = wl.name if args.padding == "config" and not args.pad else f"{wl.name}-p{pad[0]}x{pad[1]}"
    traffic, valu = read_pmc(src_hash, args.workload, config_name, head["col_variant"])
    if forms[0] != "fp32":
        traffic, valu = None, None
    cols_s = head["stage_ms"][1] * 1e-3
    achieved = cols_b / cols_s / 1e9
    col_kernel = "k_cols_conv (generic)"
    if head["kernels"] == "specialised" and "columns" in head["variants"]:
        ci = head["variants"]["columns"]["info"]
        col_kernel = "%s<%d, radices %s>" % ("k_cols_half" if ci["half_exchange"] else "k_cols_reg", ci["length"],
                                              "x".join(str(r) for r in ci["radices"]))
    if head["four_step"]:
        col_kernel = "k_long_fwd + k_long_mid + k_long_inv (four-step, P1 x P2 = %d x %d)" % head["column_split"]
        traffic, valu = None, None
    roofline = {"bound": "hbm", "kernel": col_kernel, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes": cols_b, "avg_ms": round(head["stage_ms"][1], 5),
                "avg_ms_source": "HIP events around the column stage on every call of a pass of "
                                 f"{head['stage_calls']} steps after the timed ones, on the plan's stream"}
    if valu is not None:
        # VALU issue (no packed FP32): a wave64 instruction takes its SIMD 4
        # cycles; 256 CUs x 4 SIMDs at 2.4 GHz
        issue_peak = 256 * 4 * 2.4e9 / 4.0  # wave-instructions per second
        rate = valu / cols_s
        roofline["valu_issue"] = {"wave_instructions": valu, "achieved_per_s": rate,
                                  "peak_per_s": issue_peak, "frac": round(rate / issue_peak, 4)}

    def form_entry(r):
        return {"value": r["value"], "unit": "output pixels/s", "ms_per_step": r["ms_per_step"],
                "median_ms": r["median_ms"], "dtype": r["dtype"], "kernels": r["kernels"],
                "stage_ms": r["stage_ms"],
                "model_frac": round(path_b / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "setup_s": r["setup_s"], "variants": r["variants"]}

    metric = METRIC if args.precision == "all" else f"output pixels/s per MI355X ({head['what']}) at rel-L2 <=1e-5"
    out = {
        "metric": metric,
        "value": head["value"],
        "unit": "output pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": head["dtype"], "data": "synthetic",
        "config": {"workload": config_name,
                   "ny": ny, "nx": nx, "ky": K.shape[0], "kx": K.shape[1],
                   "padding": [py, px], "pitch_km": wl.pitch_km,
                   "spectrum_form": {1: "real-quadrant", 2: "complex"}[head["form"]],
                   "cols_per_group": head["shape"][0], "rows_per_group": head["shape"][1],
                   "precision": forms[0], "kernels": head["kernels"]},
        "roofline": roofline,
        "median_ms": head["median_ms"],
        "path": {"stage_ms": head["stage_ms"],
                 "stage_names": ["rows forward", "columns", "rows inverse"],
                 "stage_calls": head["stage_calls"],
                 "model_bytes": path_b,
                 "model_GBs": round(path_b / (head["ms_per_step"] * 1e-3) / 1e9, 1),
                 "model_frac": round(path_b / (head["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "wall_s": head["wall_s"]},
        "setup_s": dict(inputs=round(t_gen, 2), **head["setup_s"]),
        "variants": head["variants"],
        "kernel_source": src_hash,
    }
    for prec in forms[1:]:
        out["split_" + prec] = form_entry(results[prec])
        out["split_" + prec]["vs_fp32"] = round(results[prec]["value"] / head["value"], 4)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * a.numel() * 4

    if not args.no_cpu:
        gpu_at = {p: (lambda idx, h=samples[p]: h[idx]) for p in forms}
        out["cpu_baseline"] = cpu_baseline(R, K, args.cpu_budget, gpu_at if len(forms) > 1 else gpu_at[forms[0]],
                                           args.cpu_one_core)
        out["cpu_baseline"]["gpu_over_cpu"] = round(out["value"] / out["cpu_baseline"]["value"], 1)
    out["paper_context"] = {"px_per_s": 3.28e6, "hardware": "Matlab R2011a, Intel Core i7 2.40 GHz",
                            "workload": "11920x11804 map, ZSB kernel, incl. file output"}
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """64 tiles x 3 bands with 4 kernels: one lp_convolve_batched per step
    (HIP graph replay); value = output pixels of all maps per second."""
    import torch
    from paper_1907_02891_amd import lp, synth

    t0 = time.perf_counter()
    tiles, psf_ids, psfs = synth.batched_inputs()
    shapes, ids, maps = [], [], []
    for t, bands in enumerate(tiles):
        for band in bands:
            shapes.append(band.shape)
            ids.append(int(psf_ids[t]))
            maps.append(band)
    t_gen = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    xs = [torch.from_numpy(m).to(dev) for m in maps]
    ys = [torch.empty_like(x) for x in xs]
    t0 = time.perf_counter()
    tune_report = None
    if args.no_tune:
        b = lp.Batch(shapes, ids, [p.shape for p in psfs]).bind(device=dev, stream=stream)
        b.set_kernels(psfs)
    else:
        from paper_1907_02891_amd import tune
        b, tune_report = tune.autotune_batch(shapes, ids, psfs, xs)
    if args.branches is not None:
        b.set_graph_branches(args.branches)
    t_setup = time.perf_counter() - t0
    for _ in range(args.warmup):
        b.convolve(xs, ys)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        b.convolve(xs, ys)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    npx = sum(a * c for a, c in shapes)
    out = {
        "metric": "output pixels/s per MI355X (FP32 FFT convolution) at rel-L2 <= 1e-5",
        "value": npx / (ms_step * 1e-3), "unit": "output pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched-64tiles-3bands-4psf1201", "maps": len(maps), "output_px": npx,
                   "graph_branches": args.branches if args.branches is not None else next(
                       (r["graph_branches"] for r in (tune_report or []) if "graph_branches" in r), 2),
                   "classes": [g["padding"] for g in b.groups]},
        "setup_s": {"inputs": round(t_gen, 2), "batch_spectra_and_autotune": round(t_setup, 3)},
        "autotune": [{"classes": r["classes"], "ms": round(r["ms"], 4)} if "classes" in r else r
                     for r in (tune_report or [])],
    }
    if not args.no_cpu:
        import oracle
        # units: output pixels of all maps, numbered map by map
        offs = np.cumsum([0] + [m.size for m in maps])
        yh = [o.cpu().numpy().ravel() for o in ys]
        md = [m.astype(np.float64) for m in maps]

        def split(idx):
            t = np.searchsorted(offs, idx, side="right") - 1
            return [(k, idx[t == k] - offs[k]) for k in np.unique(t)]

        def oracle_at(idx):
            return np.concatenate([oracle.conv_same_pixels(md[k], psfs[ids[k]], j) for k, j in split(idx)])

        def gpu_at(idx):
            return np.concatenate([yh[k][j] for k, j in split(idx)])

        out["cpu_baseline"] = cpu_leg(oracle_at, int(offs[-1]), gpu_at, args.cpu_budget, "output pixels/s",
                                      "output pixels over all maps, FP64 direct sums with each map's kernel")
    print(json.dumps(out), flush=True)


def bench_classes(args):
    """Three source classes (Eq. 4) over a 4096^2 grid, 1201^2 kernels, P =
    5400: one lp_convolve_classes per step (three forward row transforms, one
    column stage that sums the three products, one inverse row transform);
    value = output pixels of the summed map per second.  Also timed: the same
    sum as three separate convolutions plus two additions."""
    import torch
    from paper_1907_02891_amd import lp, synth, tune

    wl = synth.CLASSES
    t0 = time.perf_counter()
    maps, Ks = synth.classes_inputs()
    t_gen = time.perf_counter() - t0
    T = len(maps)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    xs = [torch.from_numpy(m).to(dev) for m in maps]
    y = torch.empty_like(xs[0])
    t0 = time.perf_counter()
    plan = lp.Plan(wl.ny, wl.nx, wl.ky, wl.kx, pitch_km=wl.pitch_km, padding=(wl.py, wl.px))
    plan.set_classes(T)
    plan.bind(device=dev, stream=stream)
    plan.set_kernels_classes(Ks)
    # separate single-class plans: the baseline this path replaces
    singles = [lp.make_plan(K, wl.ny, wl.nx, padding=(wl.py, wl.px), device=dev) for K in Ks]
    ys = [torch.empty_like(y) for _ in range(T)]
    if not args.no_tune:
        tune.autotune(plan, xs, y, use_cache=False)
        tune.autotune(singles[0], xs[0], ys[0], use_cache=False)
        for p in singles[1:]:
            for st in (lp.STAGE_ROWS, lp.STAGE_COLUMNS):
                if p.variant_count(st) > 0:
                    p.set_variant(st, singles[0].variant(st))
    t_setup = time.perf_counter() - t0

    def run_sum():
        plan.convolve_classes(xs, out=y)

    def run_separate():
        for p, x, o in zip(singles, xs, ys):
            p.convolve(x, out=o)
        torch.add(ys[0], ys[1], out=y)
        for o in ys[2:]:
            y.add_(o)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms_sep = timed(run_separate)
    ms_step = timed(run_sum)
    # per-stage events on every call of a separate pass
    plan.timing(True, every=1)
    timed_steps(run_sum, stream, max(args.steps, 20))
    stage_ms, calls = plan.stage_ms()
    plan.timing(False)
    stage_avg = [s / max(calls, 1) for s in stage_ms]
    ny, nx, py, px = wl.ny, wl.nx, wl.py, wl.px
    h = px // 2 + 1
    kh = 4 * (py // 2 + 1) * h if plan.form == 1 else 8 * py * h
    inter = 8 * ny * h
    cols_b = T * (inter + kh) + inter
    path_b = T * (4 * ny * nx + inter) + cols_b + inter + 4 * ny * nx
    achieved = cols_b / (stage_avg[1] * 1e-3) / 1e9
    out = {
        "metric": "output pixels/s per MI355X (FP32 FFT convolution, 3 source classes summed) at rel-L2 <= 1e-5",
        "value": ny * nx / (ms_step * 1e-3), "unit": "output pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "classes": T, "ny": ny, "nx": nx, "ky": wl.ky, "kx": wl.kx,
                   "padding": [py, px], "spectrum_form": {1: "real-quadrant", 2: "complex"}[plan.form]},
        "roofline": {"bound": "hbm", "kernel": "k_cols_reg (class sum)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "algorithmic_bytes": cols_b, "avg_ms": round(stage_avg[1], 5)},
        "path": {"stage_ms": [round(s, 5) for s in stage_avg],
                 "stage_names": ["rows forward (all classes)", "columns (class sum)", "rows inverse"],
                 "stage_calls": calls,
                 "model_bytes": path_b,
                 "model_frac": round(path_b / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "separate_convolutions_ms": round(ms_sep, 5),
        "speedup_vs_separate": round(ms_sep / ms_step, 3),
        "setup_s": {"inputs": round(t_gen, 2), "plans_spectra_autotune": round(t_setup, 3)},
        "variants": {"rows": plan.variant(lp.STAGE_ROWS), "columns": plan.variant(lp.STAGE_COLUMNS),
                     "separate": [singles[0].variant(lp.STAGE_ROWS), singles[0].variant(lp.STAGE_COLUMNS)]},
    }
    if not args.no_cpu:
        import oracle
        yh = y.cpu().numpy().ravel()
        md = [m.astype(np.float64) for m in maps]
        out["cpu_baseline"] = cpu_leg(lambda idx: oracle.conv_same_classes_pixels(md, Ks, idx), ny * nx,
                                      lambda idx: yh[idx], args.cpu_budget, "output pixels/s",
                                      "pixels of the summed map, FP64 direct sums over the three classes")
    print(json.dumps(out), flush=True)


def _timed(fn, stream, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_reproject(args):
    """Nearest-neighbour reprojection (Sec. 2.4) of a 15 arc-second
    longitude-latitude map onto the paper's projected grid: 11920 x 11804
    pixels of 404.4 m, transverse Mercator about -3 degrees (UTM zone 30),
    centred at 40 N; the source covers the whole target (17-64 N, 52 W-46 E:
    11280 x 23520 pixels).  One step = one lp_reproject_nn; value = projected
    pixels per second."""
    import torch
    from paper_1907_02891_amd import lp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    step = 1.0 / 240.0
    sg = lp.LatLonGrid(11280, 23520, 64.0 - step / 2, -52.0 + step / 2, step, step)
    ny, nx, pitch = 11920, 11804, 0.4044
    dg = lp.TMGrid(ny, nx, -(nx - 1) / 2 * pitch, 4430.0 + (ny - 1) / 2 * pitch, pitch, -3.0, 0.9996, 6367.0)
    rng = np.random.default_rng(1006)
    t0 = time.perf_counter()
    src = torch.from_numpy(rng.random((sg.rows, sg.cols), dtype=np.float32)).to(dev)
    t_gen = time.perf_counter() - t0
    out = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    ms = _timed(lambda: lp.reproject_nn(src, sg, dg, out=out, stream=stream), stream, args.steps, args.warmup)
    algo = 8 * ny * nx  # one gathered 4-byte read and one 4-byte write per projected pixel
    res = {
        "metric": "projected pixels/s per MI355X (nearest-neighbour transverse Mercator reprojection)",
        "value": ny * nx / (ms * 1e-3), "unit": "projected pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64 index, f32 data",
        "data": "synthetic",
        "config": {"workload": "reproject-15arcsec-to-11920x11804-utm30-404m", "source": [sg.rows, sg.cols],
                   "target": [ny, nx], "pitch_km": pitch},
        "roofline": {"bound": "hbm", "kernel": "k_reproject_nn", "achieved": round(algo / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes": algo},
        "setup_s": {"inputs": round(t_gen, 2)},
    }
    if not args.no_cpu:
        from oracle import latlon as olat
        # units: projected rows; the oracle's gather is vectorised per row
        got = out.cpu().numpy()
        h = src.cpu().numpy().astype(np.float64)
        stats = {"mismatches": 0, "rounding_ties": 0}

        def oracle_at(rows):
            vals = []
            for i in rows:
                ref, rowf, colf = olat.reproject_nn(h, sg.lat_first_deg, sg.lon_first_deg, step, step, 1, nx,
                                                    dg.x_first_km, dg.y_first_km - i * pitch, pitch, -3.0,
                                                    0.9996, 6367.0)
                tie = ((np.abs(np.abs(rowf - np.floor(rowf)) - 0.5) < 1e-9)
                       | (np.abs(np.abs(colf - np.floor(colf)) - 0.5) < 1e-9))
                stats["rounding_ties"] += int(tie.sum())
                stats["mismatches"] += int((got[i][~tie[0]] != ref[0][~tie[0]].astype(np.float32)).sum())
                vals.append(ref[0])
            return np.concatenate(vals)

        res["cpu_baseline"] = cpu_leg(oracle_at, ny, lambda rows: got[rows].ravel().astype(np.float64),
                                      args.cpu_budget, "projected rows/s",
                                      f"projected rows of {nx} pixels, FP64 numpy gather")
        res["cpu_baseline"]["parity"].update(stats)
        res["cpu_baseline"]["value_px_per_s"] = res["cpu_baseline"]["value"] * nx
    print(json.dumps(res), flush=True)


def bench_bands(args):
    """Latitude-band convolution in the native longitude-latitude grid
    (Sec. 4): a 2400 x 2400 map at 30 arc-seconds (60-40 N), 8 bands of 300
    rows, each with the d^-2.5 exp(-d/80 km) kernel sampled for its centre
    latitude and cut at 300 km (649 x 1007 pixels at the widest); one batched
    call per step (slabs with halos, band rows written in place)."""
    import torch
    from paper_1907_02891_amd import latlon, lp, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    ny = nx = 2400
    step = 1.0 / 120.0
    lat_first = 60.0 - step / 2
    edges = list(range(0, ny + 1, 300))
    rng = np.random.default_rng(1007)
    L = synth.radiance_map(ny, nx, 150, 0.05, (2.0, 20.0), rng)
    half_y = int(300.0 / (latlon.EARTH_RADIUS_KM * step * np.pi / 180.0))
    lat_min_centre = min(latlon.band_centres(edges, lat_first, step))
    half_x = int(300.0 / (latlon.EARTH_RADIUS_KM * np.cos(np.radians(lat_min_centre)) * step * np.pi / 180.0))

    def radial(d):
        dd = np.maximum(d, 0.5 * latlon.EARTH_RADIUS_KM * step * np.pi / 180.0)
        return np.where(d <= 300.0, dd ** -2.5 * np.exp(-dd / 80.0), 0.0)

    Ks = [latlon.band_kernel(radial, c, step, step, half_y, half_x) for c in latlon.band_centres(edges, lat_first, step)]
    t0 = time.perf_counter()
    bands = latlon.LatitudeBands(ny, nx, edges, Ks, device=dev, stream=stream)
    t_setup = time.perf_counter() - t0
    x = torch.from_numpy(L).to(dev)
    y = torch.empty_like(x)
    ms = _timed(lambda: bands.convolve(x, out=y), stream, args.steps, args.warmup)
    res = {
        "metric": "output pixels/s per MI355X (latitude-band FFT convolution on the longitude-latitude grid)",
        "value": ny * nx / (ms * 1e-3), "unit": "output pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "bands-2400x2400-30arcsec-8bands", "kernel": [2 * half_y + 1, 2 * half_x + 1],
                   "bands": len(edges) - 1, "padding_classes": [g["padding"] for g in bands.batch.groups]},
        "setup_s": {"band_kernels_plans_spectra": round(t_setup, 3)},
    }
    if not args.no_cpu:
        from oracle import latlon as olat
        yh = y.cpu().numpy().ravel()
        Ld = L.astype(np.float64)
        res["cpu_baseline"] = cpu_leg(lambda idx: olat.conv_latitude_bands_pixels(Ld, edges, Ks, idx), ny * nx,
                                      lambda idx: yh[idx], args.cpu_budget, "output pixels/s",
                                      "output pixels, FP64 direct sums with each row's band kernel")
    print(json.dumps(res), flush=True)


def bench_slab(args):
    """One GPU's share of the continental map (16384 x 16384, 2001 x 2001
    kernel) under an 8-way split by overlap-save row slabs: output rows
    [r0, r0 + 2048) from input rows [r0 - 1000, r0 + 3048) (a 4048-row slab
    with whole halos), so the kept rows need only 4048 padded rows: class
    4320 x 18432.  Whole-job rate of 8 such GPUs = 8 x this value (weak
    scaling, no communication when every GPU holds its input rows)."""
    import torch
    from paper_1907_02891_amd import lp, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    R, K = synth.continental_inputs()
    n, k = R.shape[1], K.shape[0]
    cy = (k - 1) // 2
    r0, rows = 3 * 2048, 2048
    slab = np.ascontiguousarray(R[r0 - cy:r0 + rows + cy])
    del R
    t0 = time.perf_counter()
    b = lp.Batch([slab.shape], [0], [K.shape], pitch_km=synth.CONTINENTAL.pitch_km)
    b.set_output_rows(0, cy, rows)
    b.bind(device=dev, stream=stream)
    b.set_kernels([K])
    t_setup = time.perf_counter() - t0
    x = torch.from_numpy(slab).to(dev)
    y = torch.empty((rows, n), dtype=torch.float32, device=dev)
    ms = _timed(lambda: b.convolve([x], [y]), stream, args.steps, args.warmup)
    py, px = b.groups[0]["padding"]
    h = px // 2 + 1
    path_b = 4 * slab.size + 4 * rows * n + 4 * 8 * slab.shape[0] * h + 4 * (py // 2 + 1) * h
    res = {
        "metric": "output pixels/s per MI355X (one GPU's overlap-save slab of the continental map)",
        "value": rows * n / (ms * 1e-3), "unit": "output pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "slab-4048x16384-keep2048-psf2001 (continental, 8-way row split)",
                   "slab_rows": slab.shape[0], "kept_rows": [cy, cy + rows], "padding": [py, px]},
        "roofline": {"bound": "hbm", "kernel": "whole step (three passes)", "achieved": round(path_b / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(path_b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "algorithmic_bytes": path_b},
        "eight_gpu_projection": {"value": 8 * rows * n / (ms * 1e-3), "ms_per_step": round(ms, 5),
                                 "assumes": "input rows resident on every GPU, no halo exchange"},
        "setup_s": {"batch_bind_spectrum": round(t_setup, 3)},
    }
    if not args.no_cpu:
        yh = y.cpu().numpy().ravel()
        Sd = slab.astype(np.float64)
        # flat index into the kept rows -> the slab's "same" output at row cy + i
        res["cpu_baseline"] = cpu_leg(lambda idx: oracle_slab(Sd, K, idx, cy, n), rows * n,
                                      lambda idx: yh[idx], args.cpu_budget, "output pixels/s",
                                      "kept output pixels, FP64 direct sums over the 2001 x 2001 kernel")
    print(json.dumps(res), flush=True)


def oracle_slab(S, K, idx, cy, n):
    import oracle
    return oracle.conv_same_pixels(S, K, np.asarray(idx, np.int64) + cy * n)


if __name__ == "__main__":
    main()
