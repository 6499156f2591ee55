"""Benchmark: output pixels/s of the FFT convolution hot path on one MI355X.

One step = one lp_convolve of the whole map (rows forward transform, column
transform x kernel spectrum x inverse, rows inverse transform with crop) with
the map already resident in HBM.  Default workload: 4096x4096 FP32 city-cluster
radiance map, 1201x1201 kernel d^-2.5 exp(-d/80 km) cut at 300 km (0.5 km
pitch), padded to 5400x5400.

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (the column stage, timed with HIP events on the stream it runs on) and
the FP64 CPU oracle timed on a bounded pixel sample on the host cores.
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
             "continental": os.path.join(ROOT, "profiles", "pmc_cols_conv_continental16384.txt")}
KERNEL_SOURCES = ["paper_1907_02891_amd/csrc/lp_kernels.hip", "paper_1907_02891_amd/csrc/fft_lds.h",
                  "paper_1907_02891_amd/csrc/fft_reg.h", "paper_1907_02891_amd/csrc/lp_internal.h"]


def stage_every(steps):
    """Interval between timed steps that carry the per-stage HIP events.  The
    four events of a recorded call add about 11 us to it (7% of the 4096^2
    step), so recording them on every timed step would inflate the step
    time; about 8 sampled steps inside the timed region give the stage
    averages."""
    return max(1, steps // 8)


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


def cpu_leg(oracle_at, n_total, gpu_at, budget_s, unit, what):
    """The CPU baseline: the FP64 oracle as it stands, timed on the host cores
    on a uniformly drawn sample of output units sized to about budget_s of
    work; its values on that sample are also compared with the GPU result at
    the same units (relative L2 and max error over max |value|).
    oracle_at(idx) -> FP64 values at flat unit indices; gpu_at(idx) -> the
    GPU's values there."""
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
    t0 = time.perf_counter()
    ref = oracle_at(idx)
    dt = time.perf_counter() - t0
    got = gpu_at(idx)
    return {"value": n / dt, "unit": unit, "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n} uniformly drawn {what}, {dt:.1f} s",
            "parity": {"units": int(n), "rel_l2": oracle.rel_l2(got, ref),
                       "max_err_frac": oracle.max_err_frac(got, ref)}}


def cpu_baseline(R, K, budget_s, y):
    """The oracle's direct FP64 sum of the same map on sampled output pixels."""
    import oracle
    Rd = R.astype(np.float64)
    yh = y.cpu().numpy().ravel()
    return cpu_leg(lambda idx: oracle.conv_same_pixels(Rd, K, idx), R.size, lambda idx: yh[idx],
                   budget_s, "output pixels/s",
                   f"output pixels of the same map, FP64 direct sum over the {K.shape[0]}x{K.shape[1]} kernel")


PRECISIONS = {"fp32": (0, "f32", "FP32 FFT convolution"),
              "fp16x2": (1, "f16x2 split, f32 accumulate",
                         "FFT convolution, radix-16 passes on MFMA with FP16 hi+lo operands"),
              "bf16x3": (2, "bf16x3 split, f32 accumulate",
                         "FFT convolution, radix-16 passes on MFMA with BF16 x3 operands")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="country",
                    choices=["country", "small", "adjoint", "continental", "large", "slab", "batched", "classes", "reproject",
                             "bands"])
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (variant 0 of each stage)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for PMC byte calibration)")
    ap.add_argument("--precision", default="fp32", choices=list(PRECISIONS),
                    help="transform arithmetic: FP32 vector ALU, or radix-16 passes on the "
                         "matrix cores with FP16 hi+lo / BF16 x3 split operands")
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

    t0 = time.perf_counter()
    pad = (wl.py, wl.px) if args.padding == "config" else lp.window_padding(ny, nx, *K.shape)
    if args.pad:
        pad = tuple(int(v) for v in args.pad.split(","))
    plan = lp.Plan(ny, nx, *K.shape, pitch_km=wl.pitch_km, padding=pad)
    mode, dtype, what = PRECISIONS[args.precision]
    plan.set_precision(mode)
    if args.kernels == "generic":
        plan.set_kernels(lp.KERNELS_GENERIC)
    plan.bind(device=dev, stream=stream)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan.set_kernel(K)
    t_spec = time.perf_counter() - t0

    x = torch.from_numpy(R).to(dev)
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
    for _ in range(args.warmup):
        plan.convolve(x, out=y)
    torch.cuda.synchronize()

    plan.timing(True, every=stage_every(args.steps))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.convolve(x, out=y)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = ev0.elapsed_time(ev1)
    stage_ms, calls = plan.stage_ms()
    plan.timing(False)
    ms_step = ms_total / args.steps
    stage_avg = [s / max(calls, 1) for s in stage_ms]

    py, px = plan.padding
    four_step = plan.column_split[0] > 1
    path_b, cols_b, kh_b = (model_bytes_four_step if four_step else model_bytes)(ny, nx, py, px, plan.form)
    src_hash = kernel_source_hash()
    col_variant = plan.variant(lp.STAGE_COLUMNS) if plan.kernels == lp.KERNELS_SPECIALISED and \
        plan.variant_count(lp.STAGE_COLUMNS) > 0 else None
    config_name = wl.name if args.padding == "config" and not args.pad else f"{wl.name}-p{pad[0]}x{pad[1]}"
    traffic, valu = read_pmc(src_hash, args.workload, config_name, col_variant)
    if args.precision != "fp32":
        traffic, valu = None, None
    cols_s = stage_avg[1] * 1e-3
    achieved = cols_b / cols_s / 1e9
    col_kernel = "k_cols_reg" if plan.kernels == lp.KERNELS_SPECIALISED else "k_cols_conv"
    if four_step:
        col_kernel = "k_long_fwd + k_long_mid + k_long_inv (four-step, P1 x P2 = %d x %d)" % plan.column_split
        traffic, valu = None, None
    roofline = {"bound": "hbm", "kernel": col_kernel, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes": cols_b, "avg_ms": round(stage_avg[1], 5)}
    if valu is not None:
        # the unit that binds this kernel: VALU issue (no packed FP32): a wave64
        # instruction takes its SIMD 4 cycles; 256 CUs x 4 SIMDs at 2.4 GHz
        issue_peak = 256 * 4 * 2.4e9 / 4.0  # wave-instructions per second
        rate = valu / cols_s
        roofline["valu_issue"] = {"wave_instructions": valu, "achieved_per_s": rate,
                                  "peak_per_s": issue_peak, "frac": round(rate / issue_peak, 4)}

    variants = {}
    if plan.kernels == lp.KERNELS_SPECIALISED:
        for name, st in (("rows", lp.STAGE_ROWS), ("columns", lp.STAGE_COLUMNS), ("rows_inverse", lp.STAGE_ROWS_INVERSE)):
            if plan.variant_count(st) > 0:
                t = (tuning or {}).get("rows" if st != lp.STAGE_COLUMNS else "columns", {})
                tried = {lp.STAGE_ROWS: t.get("forward_ms", t.get("all", [])), lp.STAGE_COLUMNS: t.get("all", []),
                         lp.STAGE_ROWS_INVERSE: t.get("inverse_ms", [])}[st]
                variants[name] = {"chosen": plan.variant(st), "info": plan.variant_info(st, plan.variant(st)),
                                  "tried_ms": [round(x, 5) for x in tried]}
    out = {
        "metric": f"output pixels/s per MI355X ({what}) at rel-L2 <= 1e-5",
        "value": ny * nx / (ms_step * 1e-3),
        "unit": "output pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": config_name,
                   "ny": ny, "nx": nx, "ky": K.shape[0], "kx": K.shape[1],
                   "padding": [py, px], "pitch_km": wl.pitch_km,
                   "spectrum_form": {1: "real-quadrant", 2: "complex"}[plan.form],
                   "cols_per_group": plan.shape[0], "rows_per_group": plan.shape[1],
                   "precision": args.precision,
                   "kernels": "specialised" if plan.kernels == lp.KERNELS_SPECIALISED else "generic"},
        "roofline": roofline,
        "path": {"stage_ms": [round(s, 5) for s in stage_avg],
                 "stage_names": ["rows forward", "columns", "rows inverse"],
                 "stage_sampled_steps": calls,
                 "model_bytes": path_b,
                 "model_GBs": round(path_b / (ms_step * 1e-3) / 1e9, 1),
                 "model_frac": round(path_b / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "wall_s": round(wall, 4)},
        "setup_s": {"inputs": round(t_gen, 2), "plan_bind": round(t_plan, 3),
                    "kernel_spectrum": round(t_spec, 3), "autotune": round(t_tune, 3)},
        "variants": variants,
        "kernel_source": src_hash,
    }

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * a.numel() * 4

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(R, K, args.cpu_budget, y)
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
    plan.timing(True, every=stage_every(args.steps))
    ms_step = timed(run_sum)
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
                 "stage_sampled_steps": calls,
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
