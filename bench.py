#!/usr/bin/env python3
"""Throughput of the least-misfit gridding / FFT / degridding path on one MI355X.

One step is one pass of the whole hot path over the workload's visibilities:
build the uv plan (coordinates -> tap cells and offsets in FP64, counting
sort by uv tile), make the dirty image (grid, inverse FFT, correct, crop) and
predict visibilities from that image (correct, pad, forward FFT, degrid).
The table (host LM optimisation, once per W/x0/size) is built before timing.

Default workload: 16,777,152 visibilities from a synthetic 64-antenna array
(2,016 baselines x 8,322 hour angles, 50-source sky) on a 4096^2 grid, W = 7,
x0 = 0.25, 300-entry table with cubic interpolation, FP32 data.

Prints ONE JSON line. Per-kernel times come from HIP events the library
records around its own launches on the launch stream (lmg_trace_*).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
METRIC = "visibilities/s gridded+degridded at W=7, 4096² grid (HBM GB/s % peak)"
HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_1906_07102_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(name: str, nvis: int, N: int, M: int, cs: int) -> float:
    """Bytes the method must move per launch of each kernel (counted per visibility / per grid cell).

    uv 16 B, visibility cs B, weight 4 B per visibility; grids and images
    counted once per read or write.
    """
    rs = cs // 2
    return {
        "plan_count": 16.0 * nvis,
        "plan_scan": 0.0,
        "plan_scatter": 16.0 * nvis,
        "grid_items": (16.0 + cs + 4.0) * nvis,
        "assemble": float(N) * N * cs,
        "degrid_items": (16.0 + cs) * nvis + float(N) * N * cs,
        "fft_rows_inverse": float(N) * N * cs + float(M) * N * cs,
        "fft_cols_inverse_correct_crop": float(M) * N * cs + float(M) * M * cs + 0 * rs,
        "fft_rows_forward_correct_pad": float(M) * M * cs + float(N) * M * cs,
        "fft_cols_forward": float(N) * M * cs + float(N) * N * cs,
    }.get(name, 0.0)


def load_traffic(kernel: str, nvis: int):
    """Counter-measured HBM bytes per launch from profiles/, if taken on the current kernel sources."""
    path = os.path.join(HERE, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash() or d.get("nvis") != nvis:
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


# Library trace names -> device kernel symbols (rocprofv3 names them by symbol).
TRACE_TO_SYMBOL = {
    "plan_count": "k_plan_count", "plan_colscan": "k_plan_colscan", "plan_scan": "k_plan_scan",
    "plan_scatter": "k_plan_scatter", "plan_place": "k_plan_place", "plan_sort_items": "k_plan_sort_items",
    "plan_compose": "k_plan_compose",
    "permute_in": "k_permute_in", "grid_items": "k_grid_items", "assemble": "k_assemble",
    "degrid_items": "k_degrid_items", "permute_out": "k_permute_out",
    "fft_pass": "k_fft_pass",            # the four passes of a step (summaries take the median)
}
CALIBRATION_SYMBOL = "MulFunctor"       # torch.mul(a, 1.0, out=b) over 2^28 floats: 1 GiB read + 1 GiB written
CALIBRATION_BYTES = float(1 << 30)


def _short_name(kernel_name: str) -> str:
    import re
    k = re.sub(r"\(.*", "", kernel_name)
    return k.replace("void lmg::dev::", "").replace("lmg::dev::", "").strip()


def summarize_trace(stats_csv: str, command: str) -> str:
    """Text summary of a rocprofv3 --kernel-trace --stats kernel_stats.csv."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# rocprofv3 kernel statistics", f"# command: {command}", "",
           f"{'kernel':58s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        out.append(f"{_short_name(r['Name'])[:58]:58s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                   f"{float(r['TotalDurationNs']) / 1e6:10.3f} {100 * float(r['TotalDurationNs']) / tot:6.2f}")
    return "\n".join(out) + "\n"


def _counter_per_dispatch(path: str, counter: str):
    """{short kernel name: [value per dispatch, ...]} for one counter of a --pmc counter_collection.csv."""
    import csv
    import collections
    per = collections.defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        per[r["Dispatch_Id"]] += float(r["Counter_Value"])
        names[r["Dispatch_Id"]] = r["Kernel_Name"]
    out = collections.defaultdict(list)
    for d, v in per.items():
        out[_short_name(names[d])].append(v)
    return out


def summarize_traffic(fetch_csv: str, write_csv: str, command: str, nvis: int):
    """HBM bytes per launch from FETCH_SIZE and WRITE_SIZE passes (KiB per dispatch), each scaled by what the
    same counter reads for a plain 1 GiB copy in the same run. Returns (text, json dict)."""
    fetch = _counter_per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _counter_per_dispatch(write_csv, "WRITE_SIZE")

    def calib(d):
        vals = [v for k, vs in d.items() if CALIBRATION_SYMBOL in k for v in vs if v * 1024 > CALIBRATION_BYTES / 2]
        if not vals:
            raise SystemExit("calibration copy not found in the counter run (bench.py --copy-calibration)")
        return CALIBRATION_BYTES / (float(np.median(vals)) * 1024.0)
    fr, wr = calib(fetch), calib(write)
    kernels = {}
    lines = [f"# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch)",
             f"# command (FETCH_SIZE pass): {command.replace('PMC', 'FETCH_SIZE')}",
             f"# command (WRITE_SIZE pass): {command.replace('PMC', 'WRITE_SIZE')}",
             f"# calibration: torch.mul(a, 1.0, out=b) over 1 GiB; bytes = counter KiB x 1024 x factor; "
             f"fetch factor {fr:.4f}, write factor {wr:.4f}",
             f"# nvis {nvis}", "",
             f"{'trace name':24s} {'kernel':44s} {'launches':>8s} {'fetch_MB':>10s} {'write_MB':>10s} {'B/vis':>8s}"]
    for trace, sym in TRACE_TO_SYMBOL.items():
        f = [v for k, vs in fetch.items() if k.startswith(sym + "<") or k == sym for v in vs]
        w = [v for k, vs in write.items() if k.startswith(sym + "<") or k == sym for v in vs]
        if not f or not w:
            continue
        fb = float(np.median(f)) * 1024.0 * fr
        wb = float(np.median(w)) * 1024.0 * wr
        kname = next(k for k in fetch if k.startswith(sym))
        kernels[trace] = {"kernel": kname, "fetch_bytes": round(fb), "write_bytes": round(wb),
                          "bytes_per_launch": round(fb + wb)}
        lines.append(f"{trace:24s} {kname[:44]:44s} {len(f):8d} {fb / 1e6:10.2f} {wb / 1e6:10.2f} "
                     f"{(fb + wb) / nvis:8.2f}")
    data = {"source_hash": kernel_source_hash(), "nvis": nvis, "fetch_factor": fr, "write_factor": wr,
            "kernels": kernels}
    return "\n".join(lines) + "\n", data


READ_SIZE_COUNTERS = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")


def summarize_read_sizes(csv_path: str, command: str, nvis: int) -> str:
    """Read bytes per launch from the L2 -> memory read requests counted by size (one --pmc pass with the four
    READ_SIZE_COUNTERS). FETCH_SIZE takes every request it cannot size as 64 bytes, so a kernel issuing
    128-byte requests reads as half its bytes (the copy's factor 2) and one issuing narrower requests is
    over-counted by that factor; sizing each request removes the calibration."""
    per = {c: _counter_per_dispatch(csv_path, c) for c in READ_SIZE_COUNTERS}
    n, n32, n64, n128 = (per[c] for c in READ_SIZE_COUNTERS)

    def sized(name):
        a, b, c, d = (np.array(x[name], dtype=float) for x in (n, n32, n64, n128))
        rest = np.maximum(a - b - c - d, 0.0)
        return 32 * b + 64 * c + 128 * d + 64 * rest, a, b, c, d

    lines = ["# HBM read bytes per launch from read requests counted by size (L2 -> memory)",
             f"# command: {command}",
             "# bytes = 32 x RDREQ_32B + 64 x RDREQ_64B + 128 x RDREQ_128B (+ 64 x any unsized request)", ""]
    cal = [k for k in n if CALIBRATION_SYMBOL in k]
    if cal:
        by, *_ = sized(cal[0])
        big = by[by > CALIBRATION_BYTES / 2]
        if len(big):
            lines.append(f"calibration copy (1 GiB read): {float(np.median(big)) / CALIBRATION_BYTES:.4f} GiB read")
    lines += [f"# nvis {nvis}", "",
              f"{'trace name':24s} {'kernel':44s} {'read_MB':>9s} {'B/vis':>7s} {'32B':>6s} {'64B':>6s} {'128B':>6s}"]
    for trace, sym in TRACE_TO_SYMBOL.items():
        names = [k for k in n if k.startswith(sym + "<") or k == sym]
        if not names:
            continue
        by, a, b, c, d = sized(names[0])
        i = int(np.argsort(by)[len(by) // 2])
        tot = max(a[i], 1.0)
        lines.append(f"{trace:24s} {names[0][:44]:44s} {by[i] / 1e6:9.2f} {by[i] / nvis:7.2f} "
                     f"{b[i] / tot:6.2f} {c[i] / tot:6.2f} {d[i] / tot:6.2f}")
    return "\n".join(lines) + "\n"


def summarize_counters(csv_paths, command: str) -> str:
    """Per-kernel medians (over dispatches) of every counter in one or more --pmc counter_collection.csv files,
    with each SQ wave-cycle counter also given as a fraction of SQ_WAVE_CYCLES."""
    import csv
    counters = []
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] not in counters:
                counters.append(r["Counter_Name"])
    per = {}
    for path in csv_paths:
        for c in counters:
            for k, vs in _counter_per_dispatch(path, c).items():
                if vs:
                    per.setdefault(k, {})[c] = float(np.median(vs))
    cyc = "SQ_WAVE_CYCLES"
    lines = ["# hardware counters per launch (median over dispatches)", f"# command: {command}", ""]
    for trace, sym in TRACE_TO_SYMBOL.items():
        names = [k for k in per if k.startswith(sym + "<") or k == sym]
        if not names:
            continue
        d = per[names[0]]
        lines.append(f"{trace} ({names[0]})")
        for c in counters:
            if c not in d:
                continue
            frac = ""
            if cyc in d and c != cyc and d[cyc] > 0 and ("WAIT" in c or "ACTIVE" in c or "BUSY" in c):
                frac = f"   ({d[c] / d[cyc]:.3f} of {cyc})"
            lines.append(f"  {c:28s} {d[c]:16.0f}{frac}")
    return "\n".join(lines) + "\n"


def cpu_baseline(case, nvis_sample: int):
    """The FP64 oracle on a bounded sample of the same workload, scaled to visibilities/s of a whole step."""
    from oracle import imaging as im
    from oracle import lmtable as lt
    tab, h = lt.make_table(case.W, case.x0, case.table_size, case.degree)
    hp = lt.correction(h, case.W, case.x0, case.N)
    uv = case.uv[:nvis_sample]
    vis = case.vis[:nvis_sample].astype(np.complex128)
    t0 = time.perf_counter()
    G = im.grid(uv, vis, None, case.N, tab)
    t1 = time.perf_counter()
    img = im.dirty_from_grid(G, hp, case.x0)
    t2 = time.perf_counter()
    Gp = im.grid_from_image(img, hp, case.N, case.x0)
    t3 = time.perf_counter()
    im.degrid(uv, Gp, tab)
    t4 = time.perf_counter()
    per_vis = ((t1 - t0) + (t4 - t3)) / nvis_sample
    step = per_vis * len(case.uv) + (t2 - t1) + (t3 - t2)
    # The work the method avoids: the direct DFT dirty image (Eq. 3) as the oracle computes it (a chunked
    # complex GEMM, NumPy's BLAS on all host threads), timed on the 256 x 256 lattice of every 8th retained
    # pixel over the first 65,536 visibilities and scaled by visibilities x pixels to the whole image.
    M = im.crop_size(case.N, case.x0)
    lattice = np.arange(-M // 2, M // 2, max(1, M // 256))
    nd = min(65536, len(case.uv))
    t5 = time.perf_counter()
    im.dft_dirty_image(case.uv[:nd], case.vis[:nd], None, case.N, case.x0, lattice, lattice)
    t6 = time.perf_counter()
    dft_full = (t6 - t5) * (len(case.uv) / nd) * (M * M) / (len(lattice) ** 2)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": len(case.uv) / step,
        "unit": "visibilities/s",
        "cores": 1,
        "cpu_model": model,
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": (f"FP64 NumPy oracle: grid + degrid of the first {nvis_sample} visibilities "
                   f"({(t1 - t0) + (t4 - t3):.1f} s) and one inverse + one forward {case.N}^2 radix-2 FFT with "
                   f"correction ({(t2 - t1) + (t3 - t2):.1f} s), scaled to the full {len(case.uv)}-visibility step; "
                   f"NumPy on one thread"),
        "seconds": round(t4 - t0, 2),
        "dft_ground_truth": {
            "seconds_estimate_whole_image": round(dft_full, 1),
            "threads": os.cpu_count(),
            "sample": (f"oracle direct DFT (Eq. 3) of {len(lattice)}^2 pixels over {nd} visibilities in "
                       f"{t6 - t5:.1f} s, scaled to the {M}^2 image and {len(case.uv)} visibilities"),
        },
    }


def _timed(fn, reps, stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def measured_copy_gbps(reps=10) -> float:
    """Bandwidth of a plain device copy on this GPU: torch.mul(a, 1.0, out=b) over 1 GiB (1 GiB read and 1 GiB
    written per pass; the same kernel the byte counters are calibrated on), HIP events over `reps` passes."""
    import torch
    a = torch.ones(int(CALIBRATION_BYTES) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ms = _timed(lambda: torch.mul(a, 1.0, out=b), reps)
    del a, b
    return 2.0 * CALIBRATION_BYTES / (ms * 1e-3) / 1e9


def precision_study(lmg, case, uv, vis64, reps=5):
    """Dirty images of the workload for W = 3, 5, 7 in the three accumulation modes against the direct DFT on
    the 256 x 256 pixel lattice (every 8th pixel of the retained field) of tests/golden/dft_samples_16m_4096.npy; with the time of one dirty image +
    prediction (plan reused). The compensated FP32 mode goes through the autograd wrappers."""
    import torch
    dft = np.load(os.path.join(HERE, "tests", "golden", "dft_samples_16m_4096.npy"))
    pix = -1024 + 8 * np.arange(256)
    rows = []
    for W in (3, 5, 7):
        table = lmg.Table.create(W, case.x0, case.table_size, case.degree)
        for name, prec in (("f32", lmg.F32), ("kahan", lmg.F32_KAHAN), ("f64", lmg.F64)):
            plan = lmg.Plan(table, case.N, uv, prec)
            vis = vis64.to(torch.complex128) if prec == lmg.F64 else vis64
            if prec == lmg.F32_KAHAN:
                run = lambda: lmg.PredictVisibilities.apply(plan, lmg.MakeDirtyImage.apply(plan, vis))
            else:
                run = lambda: plan.predict_visibilities(plan.make_dirty_image(vis))
            img = plan.make_dirty_image(vis)
            sel = torch.as_tensor(pix + plan.M // 2, device=img.device)
            smp = img.index_select(0, sel).index_select(1, sel).to(torch.complex128).cpu().numpy()
            err = float(np.linalg.norm(smp - dft) / np.linalg.norm(dft))
            ms = _timed(run, reps)
            rows.append({"W": W, "mode": name, "rel_rms_vs_dft": err, "ms_dirty_plus_predict": round(ms, 4)})
            print(f"# precision W={W} {name}: err {err:.3e}, {ms:.3f} ms", file=sys.stderr, flush=True)
            del plan, img
    t = {(r["W"], r["mode"]): r for r in rows}
    return {
        "rows": rows,
        "speedup_kahan_over_f64_W7": round(t[(7, "f64")]["ms_dirty_plus_predict"] /
                                           t[(7, "kahan")]["ms_dirty_plus_predict"], 3),
        "note": "error = relative RMS against the FP64 direct DFT (Eq. 3) on the 256 x 256 lattice of every 8th "
                "pixel of the retained field; "
                "time = make_dirty_image + predict_visibilities with the plan reused; the compensated mode "
                "runs through the autograd wrappers",
    }


def direct_flops_per_visibility(W: int) -> float:
    """FP64 flops of the direct weights of one visibility (both axes): per axis 32 steps of the angle-sum
    recurrence (2 multiplies + 2 FMAs) and 2 W FMAs into the taps; one sincos per axis not counted."""
    return 2.0 * 32 * (2 + 2 * 2 + 2 * 2 * W)


def direct_study(lmg, case, uv, vis64, reps=5):
    """Direct calculation of the weights (lmg_table_create_direct): the workload's dirty image against the
    direct DFT in the three modes for W = 5 and 7, the time of one dirty image + prediction (plan reused),
    and the gridding kernel's FP64 rate (it is bound by the weights' arithmetic)."""
    import torch
    dft = np.load(os.path.join(HERE, "tests", "golden", "dft_samples_16m_4096.npy"))
    pix = -1024 + 8 * np.arange(256)
    nvis = uv.shape[0]
    rows = []
    for W in (5, 7):
        table = lmg.Table.create(W, case.x0, case.table_size, case.degree).direct_calculation()
        for name, prec in (("f32", lmg.F32), ("kahan", lmg.F32_KAHAN), ("f64", lmg.F64)):
            plan = lmg.Plan(table, case.N, uv, prec)
            vis = vis64.to(torch.complex128) if prec == lmg.F64 else vis64
            img = plan.make_dirty_image(vis)
            sel = torch.as_tensor(pix + plan.M // 2, device=img.device)
            smp = img.index_select(0, sel).index_select(1, sel).to(torch.complex128).cpu().numpy()
            err = float(np.linalg.norm(smp - dft) / np.linalg.norm(dft))
            ms = _timed(lambda: plan.predict_visibilities(plan.make_dirty_image(vis)), reps)
            lmg.trace_report()
            lmg.trace_enable(True)
            for _ in range(reps):
                plan.grid(vis)
            torch.cuda.synchronize()
            tr = lmg.trace_report()
            lmg.trace_enable(False)
            n, tot = tr["grid_items"]
            g_ms = tot / n
            tflops = direct_flops_per_visibility(W) * nvis / (g_ms * 1e-3) / 1e12
            rows.append({"W": W, "mode": name, "rel_rms_vs_dft": err, "ms_dirty_plus_predict": round(ms, 4),
                         "grid_items_ms": round(g_ms, 4), "weights_fp64_tflops": round(tflops, 2),
                         "fp64_peak_frac": round(tflops / 78.6, 3)})
            print(f"# direct W={W} {name}: err {err:.3e}, {ms:.3f} ms, grid {g_ms:.3f} ms, {tflops:.1f} TFLOP/s",
                  file=sys.stderr, flush=True)
            del plan, img
    return {"rows": rows,
            "note": "exact kernel evaluated per visibility (no table); error = relative RMS against the FP64 "
                    "direct DFT on the precision study's lattice; FP64 rate counts the weights' arithmetic only "
                    "(%d flops per visibility at W = 7), peak 78.6 TFLOP/s" % direct_flops_per_visibility(7)}


def interpolation_study(lmg, N, uv, vis, W=7, x0=0.25, sizes=(5, 9, 18, 36, 72, 144)):
    """App. F on the device: the table's own error in an FP64 dirty image, as the relative RMS distance from
    the direct-calculation image (same plan geometry, exact weights), for degrees 0..3 and M_s up to the
    largest FP64 table the kernels stage in LDS. The slope of log(error) against log(M_s) over the finer
    half should approach -(d + 1)."""
    import torch
    base = lmg.Table.create(W, x0, 300, 3)
    h, _ = base.export()
    ref_plan = lmg.Plan(base.direct_calculation(), N, uv, lmg.F64)
    ref = ref_plan.make_dirty_image(vis)
    nref = torch.linalg.vector_norm(ref).item()
    del ref_plan
    out = {}
    for d in (0, 1, 2, 3):
        errs = []
        for ms in sizes:
            plan = lmg.Plan(lmg.Table.from_h(W, x0, W * ms, d, h), N, uv, lmg.F64)
            img = plan.make_dirty_image(vis)
            errs.append(torch.linalg.vector_norm(img - ref).item() / nref)
            del plan, img
        lx, ly = np.log(np.asarray(sizes[len(sizes) // 2:], float)), np.log(np.asarray(errs[len(sizes) // 2:]))
        slope = float(np.polyfit(lx, ly, 1)[0])
        out[f"degree_{d}"] = {"Ms": list(sizes), "rel_rms_vs_direct": errs, "slope": round(slope, 3)}
        print(f"# interpolation d={d}: slope {slope:.2f}, errors {['%.2e' % e for e in errs]}", file=sys.stderr,
              flush=True)
    out["note"] = (f"W = {W}, x0 = {x0}, FP64; error = relative RMS distance of the dirty image from the "
                   "direct-calculation image (the table's contribution alone); slope fitted over the finer half")
    return out


def large_table_study(lmg, N, uv, vis, x0=0.25):
    """App. F's table rates beyond LDS on the device (coefficients read from a device copy): the table's own
    error in an FP64 dirty image of the workload, as the relative RMS distance from a reference image with a
    negligible table error. W = 7: nearest node and linear at M_s = 1e3 .. 1e6 against direct calculation.
    W = 14 (where direct calculation does not hold FP64 accuracy): linear at 1e3 .. 1e6 against a cubic table
    at M_s = 1e5, whose own error is far below (error ~ M_s^-4)."""
    import torch
    out = {}
    h7, _ = lmg.Table.create(7, x0, 300, 3).export()
    ref = lmg.Plan(lmg.Table.from_h(7, x0, 300, 3, h7).direct_calculation(), N, uv, lmg.F64).make_dirty_image(vis)
    nref = torch.linalg.vector_norm(ref).item()
    sizes = (1000, 10000, 100000, 1000000)
    for d in (0, 1):
        errs = []
        for ms in sizes:
            t = lmg.Table.from_h(7, x0, 7 * ms, d, h7)
            t.attach_device(lmg.F64)
            img = lmg.Plan(t, N, uv, lmg.F64).make_dirty_image(vis)
            errs.append(torch.linalg.vector_norm(img - ref).item() / nref)
            del t, img
            torch.cuda.synchronize()
        out[f"W7_degree_{d}"] = {"Ms": list(sizes), "rel_rms_vs_direct": errs}
        print(f"# large tables W=7 d={d}: {['%.2e' % e for e in errs]}", file=sys.stderr, flush=True)
    del ref
    h14, _ = lmg.Table.create(14, x0, 14 * 300, 3).export()
    t = lmg.Table.from_h(14, x0, 14 * 100000, 3, h14)
    t.attach_device(lmg.F64)
    ref = lmg.Plan(t, N, uv, lmg.F64).make_dirty_image(vis)
    nref = torch.linalg.vector_norm(ref).item()
    del t
    errs = []
    for ms in sizes:
        t = lmg.Table.from_h(14, x0, 14 * ms, 1, h14)
        t.attach_device(lmg.F64)
        img = lmg.Plan(t, N, uv, lmg.F64).make_dirty_image(vis)
        errs.append(torch.linalg.vector_norm(img - ref).item() / nref)
        del t, img
        torch.cuda.synchronize()
    out["W14_degree_1"] = {"Ms": list(sizes), "rel_rms_vs_cubic_1e5": errs}
    print(f"# large tables W=14 d=1: {['%.2e' % e for e in errs]}", file=sys.stderr, flush=True)
    out["note"] = ("FP64 dirty images of the workload; tables beyond the LDS budget read from device memory "
                   "(lmg_table_attach_device); error = relative RMS distance from the reference image")
    return out


def _dirty_from_grid(lmg, G, hpix, M):
    """Centred inverse FFT of one grid (library FFT), correction h(x) h(y) and crop to M x M (torch glue)."""
    import torch
    N = G.shape[0]
    F = lmg.fft2_centred(G.clone(), +1)
    sl = slice(N // 2 - M // 2, N // 2 + M // 2)
    h = torch.as_tensor(hpix[sl], device=G.device, dtype=torch.float64)
    return F[sl, sl].to(torch.complex128) * h[:, None] * h[None, :]


def equal_misfit_comparison(lmg, case, uv16, vis16, reps=3):
    """The batched, differentiable, compensated-FP32 form against the plain one-channel FP64 path, at equal
    misfit against the direct DFT.

    W = 5, 256 channels (1024^2, log-uniform counts): one batched compensated-FP32 plan through autograd
    (forward = degridding of 256 model grids, loss = sum |V_hat - V|^2, backward = gridding) against 256
    single-channel FP64 plans doing the same degrid + grid of the residual. At W = 5 both reach the method's
    own misfit (FP32 rounding is far below it), measured on four channels' dirty images against the direct-DFT
    samples of tests/golden/dft_multichannel.npz.
    W = 7, 16.8M visibilities on 4096^2 (the paper's single-precision level): prediction through autograd
    (forward = predict_visibilities of the image, backward = dirty image) in compensated FP32 against the same
    forward and backward in FP64. FP64 needs W = 7 to stay at or below the compensated form's misfit, so the
    pair is W = 7 against W = 7 (FP64 then has the smaller misfit: the comparison favours FP64)."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    out = {}
    # ---- W = 5, batched
    uv_np, off, _ = synth.multichannel_case()
    uv = torch.from_numpy(uv_np).to(dev)
    v32 = torch.from_numpy(synth.multichannel_vis(len(uv_np))).to(dev)
    v64 = v32.to(torch.complex128)
    N, W, M = 1024, 5, 512
    nch = len(off) - 1
    table = lmg.Table.create(W, 0.25, 300, 3)
    bplan = lmg.BatchPlan(table, N, uv, off, lmg.F32_KAHAN, tile=32)
    singles = [lmg.Plan(table, N, uv[int(off[c]):int(off[c + 1])].contiguous(), lmg.F64) for c in range(nch)]
    G32 = bplan.grid(v32)
    G64 = G32.to(torch.complex128)
    grad64 = torch.empty_like(G64)

    def batched():
        g = G32.detach().requires_grad_(True)
        vh = lmg.Degrid.apply(bplan, g)
        (vh - v32).abs().pow(2).sum().backward()
        return g.grad

    def fp64_separate():
        for c, p in enumerate(singles):
            a, b = int(off[c]), int(off[c + 1])
            vh = p.degrid(G64[c])
            p.grid(2 * (vh - v64[a:b]), out=grad64[c])

    ms_b = _timed(batched, reps)
    ms_s = _timed(fp64_separate, max(1, reps // 2))
    gold = np.load(os.path.join(HERE, "tests", "golden", "dft_multichannel.npz"))
    hpix = table.correction(N)
    sel = torch.as_tensor(-256 + 8 * np.arange(64) + M // 2, device=dev)
    mis_k, mis_64 = [], []
    for c in (0, 85, 170, 255):
        a, b = int(off[c]), int(off[c + 1])
        ref = gold[f"chan_{c}"]
        ik = _dirty_from_grid(lmg, G32[c], hpix, M)
        i64 = singles[c].make_dirty_image(v64[a:b])
        for img, dst in ((ik, mis_k), (i64, mis_64)):
            smp = img.index_select(0, sel).index_select(1, sel).to(torch.complex128).cpu().numpy()
            dst.append(float(np.linalg.norm(smp - ref) / np.linalg.norm(ref)))
    out["W5_batched_256_channels"] = {
        "nvis": int(off[-1]), "ms_batched_differentiable_kahan": round(ms_b, 4),
        "ms_256_single_channel_fp64": round(ms_s, 4), "speedup": round(ms_s / ms_b, 2),
        "dft_misfit_kahan_channels_0_85_170_255": mis_k, "dft_misfit_fp64_channels_0_85_170_255": mis_64,
    }
    print(f"# equal misfit W=5: batched kahan {ms_b:.2f} ms, 256 x fp64 {ms_s:.2f} ms; misfit {mis_k} vs {mis_64}",
          file=sys.stderr, flush=True)
    del bplan, singles, G32, G64, grad64
    torch.cuda.synchronize()
    # ---- W = 7, one channel of 16.8M visibilities
    t7 = lmg.Table.create(7, case.x0, case.table_size, case.degree)
    pk = lmg.Plan(t7, case.N, uv16, lmg.F32_KAHAN)
    p64 = lmg.Plan(t7, case.N, uv16, lmg.F64)
    v7 = vis16.to(torch.complex64)
    v7d = vis16.to(torch.complex128)
    img_k = pk.make_dirty_image(v7)
    img_64 = p64.make_dirty_image(v7d)
    model_k = img_k / float(len(case.uv))
    model_64 = model_k.to(torch.complex128)

    def diff_kahan():
        im_ = model_k.detach().requires_grad_(True)
        vh = lmg.PredictVisibilities.apply(pk, im_)
        (vh - v7).abs().pow(2).sum().backward()
        return im_.grad

    def fp64_plain():
        vh = p64.predict_visibilities(model_64)
        return p64.make_dirty_image(2 * (vh - v7d))

    ms_k7 = _timed(diff_kahan, reps)
    ms_64 = _timed(fp64_plain, reps)
    dft = np.load(os.path.join(HERE, "tests", "golden", "dft_samples_16m_4096.npy"))
    sel = torch.as_tensor(-1024 + 8 * np.arange(256) + pk.M // 2, device=dev)
    mis = []
    for img in (img_k, img_64):
        smp = img.index_select(0, sel).index_select(1, sel).to(torch.complex128).cpu().numpy()
        mis.append(float(np.linalg.norm(smp - dft) / np.linalg.norm(dft)))
    out["W7_single_precision_level"] = {
        "nvis": len(case.uv), "ms_differentiable_kahan": round(ms_k7, 4), "ms_fp64": round(ms_64, 4),
        "speedup": round(ms_64 / ms_k7, 3), "dft_misfit_kahan": mis[0], "dft_misfit_fp64": mis[1],
    }
    print(f"# equal misfit W=7: kahan {ms_k7:.3f} ms, fp64 {ms_64:.3f} ms; misfit {mis}", file=sys.stderr,
          flush=True)
    out["pairing"] = ("W = 5: both forms reach the method's own misfit (equal to 3 digits on four channels); "
                      "W = 7: FP64 needs the same W to stay at or below the compensated form's misfit, and "
                      "then has the smaller misfit (the comparison favours FP64)")
    return out


def multichannel_study(lmg, reps=5):
    """256 channels (log-uniform 1e4..2e5 visibilities), 1024^2 grids, W = 5, compensated FP32: gridding +
    degridding in one batched plan (autotuned tile) against 256 single-channel plans on one stream."""
    import torch
    import synth
    uv_np, off, _ = synth.multichannel_case()
    dev = torch.device("cuda:0")
    vis = torch.from_numpy(synth.multichannel_vis(len(uv_np))).to(dev)
    uv = torch.from_numpy(uv_np).to(dev)
    N, W = 1024, 5
    table = lmg.Table.create(W, 0.25, 300, 3)
    prec = lmg.F32_KAHAN
    plan, tune = lmg.autotune_batch(table, N, uv, off, vis, None, prec, tiles=(16, 32, 64))
    grids = plan.grid(vis)
    vout = plan.degrid(grids)
    ms_batched = _timed(lambda: (plan.grid(vis, out=grids), plan.degrid(grids, out=vout)), reps)
    singles = []
    for c in range(len(off) - 1):
        a, b = int(off[c]), int(off[c + 1])
        singles.append((lmg.Plan(table, N, uv[a:b].contiguous(), prec), vis[a:b].contiguous(), grids[c],
                        vout[a:b]))

    def separate():
        for p, v, g, o in singles:
            p.grid(v, out=g)
            p.degrid(g, out=o)
    ms_sep = _timed(separate, max(1, reps // 2))
    nvis = int(off[-1])
    return {
        "workload": "256 channels, 1024^2 grids, W=5, compensated FP32, log-uniform 1e4..2e5 visibilities",
        "nvis": nvis, "tile": plan.info()["tile"], "autotune_ms": {str(k): round(v, 4) for k, v in tune.items()},
        "ms_batched_grid_plus_degrid": round(ms_batched, 4), "ms_256_separate": round(ms_sep, 4),
        "speedup_batched": round(ms_sep / ms_batched, 3), "vis_per_s_batched": nvis / (ms_batched * 1e-3),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["f32", "kahan", "f64"], default="f32")
    ap.add_argument("--workload", choices=["array-16m-4096", "array-1m-2048"], default="array-16m-4096")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the precision study and the multichannel comparison")
    ap.add_argument("--only-studies", default="", help="comma-separated study names to run (default: all)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 19)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--summarize-trace", metavar="KERNEL_STATS_CSV",
                    help="print a text summary of a rocprofv3 --stats run and exit (no GPU use)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from FETCH_SIZE and WRITE_SIZE passes, print a summary, exit")
    ap.add_argument("--summarize-read-sizes", metavar="COUNTER_CSV",
                    help="print read bytes per launch from a pass with the sized read-request counters, exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="COUNTER_CSV",
                    help="print per-kernel medians of the counters of one or more --pmc passes, exit")
    ap.add_argument("--profile-command", default="", help="command line recorded in a summary")
    ap.add_argument("--nvis", type=int, default=16777152, help="visibilities of the profiled run (traffic summary)")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.profile_command), end="")
        return
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.profile_command), end="")
        return
    if args.summarize_read_sizes:
        print(summarize_read_sizes(args.summarize_read_sizes, args.profile_command, args.nvis), end="")
        return
    if args.summarize_traffic:
        text, data = summarize_traffic(*args.summarize_traffic, args.profile_command, args.nvis)
        with open(os.path.join(HERE, "profiles", "traffic.json"), "w") as f:
            json.dump(data, f, indent=1)
        print(text, end="")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(sharding over several GPUs is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    sys.path.insert(0, HERE)
    import paper_1906_07102_amd as lmg
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prec = {"f32": lmg.F32, "kahan": lmg.F32_KAHAN, "f64": lmg.F64}[args.precision]
    cdt = torch.complex128 if prec == lmg.F64 else torch.complex64
    cs = 16 if prec == lmg.F64 else 8
    t_in = time.perf_counter()
    case = synth.array_16m_case(with_vis=True, device="cuda") if args.workload == "array-16m-4096" \
        else synth.array_1m_case(with_vis=True, device="cuda")
    N, W, nvis = case.N, case.W, len(case.uv)
    M = int(round(2 * case.x0 * N))
    uv = torch.from_numpy(case.uv).to(dev)
    vis = torch.from_numpy(case.vis).to(dev, cdt)
    w = torch.ones(nvis, dtype=torch.float32, device=dev)
    t_inputs = time.perf_counter() - t_in
    t_tab = time.perf_counter()
    table = lmg.Table.create(W, case.x0, case.table_size, case.degree)
    t_tab = time.perf_counter() - t_tab
    print(f"# inputs {t_inputs:.1f}s, table {t_tab:.2f}s, nvis={nvis} N={N}", file=sys.stderr, flush=True)
    img = torch.empty((M, M), dtype=cdt, device=dev)
    vout = torch.empty(nvis, dtype=cdt, device=dev)

    def step():
        plan = lmg.Plan(table, N, uv, prec)
        plan.make_dirty_image(vis, w, out=img)
        plan.predict_visibilities(img, out=vout)
        return plan

    # After the warm-up, two steps record every kernel (HIP events on the launch stream) for the
    # per-kernel table; the kernel with the most time per launch is the one the roofline is quoted
    # for. In the timed steps only that kernel is recorded, so that its duration is measured over the
    # timed region with little tracing overhead.
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lmg.trace_report()                       # discard anything recorded so far
    lmg.trace_enable(True)
    lmg.trace_only(None)
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    trace = lmg.trace_report()
    dom = max(trace.items(), key=lambda kv: kv[1][1] / kv[1][0])[0]
    lmg.trace_only(dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_trace = lmg.trace_report()[dom]
    lmg.trace_only(None)
    lmg.trace_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    print(f"# step {ms:.3f} ms; plan {plan.info()}", file=sys.stderr, flush=True)

    # Steady state with the plan reused (uv fixed, as in iterative imaging).
    plan = lmg.Plan(table, N, uv, prec)
    for _ in range(2):
        plan.make_dirty_image(vis, w, out=img)
        plan.predict_visibilities(img, out=vout)
    torch.cuda.synchronize()
    r0 = time.perf_counter()
    for _ in range(args.steps):
        plan.make_dirty_image(vis, w, out=img)
        plan.predict_visibilities(img, out=vout)
    torch.cuda.synchronize()
    ms_reuse = (time.perf_counter() - r0) * 1e3 / args.steps

    # The unit of work the metric names: one visibility gridded (lmg_grid_planned, overwriting the 4096^2
    # grid) and degridded (lmg_degrid_planned) with the plan reused, data in caller order (two reorderings
    # per pair of calls); and the same pair on data kept in the plan's order (lmg_*_planned_ordered).
    gu = torch.empty((N, N), dtype=cdt, device=dev)
    vu = torch.empty(nvis, dtype=cdt, device=dev)
    vp = plan.to_plan_order(vis, w)
    vpo = torch.zeros_like(vp)
    ms_unit_caller = _timed(lambda: (plan.grid(vis, w, out=gu), plan.degrid(gu, out=vu)), args.steps)
    ms_unit_plan = _timed(lambda: (plan.grid_ordered(vp, out=gu), plan.degrid_ordered(gu, out=vpo)), args.steps)
    unit_bytes = (16.0 + cs + 4.0) * nvis + (16.0 + cs) * nvis + 2.0 * N * N * cs
    grid_degrid_unit = {
        "ms_caller_order": round(ms_unit_caller, 4), "vis_per_s_caller_order": nvis / (ms_unit_caller * 1e-3),
        "ms_plan_order": round(ms_unit_plan, 4), "vis_per_s_plan_order": nvis / (ms_unit_plan * 1e-3),
        "algorithmic_bytes_per_vis": round(unit_bytes / nvis, 2),
        "hbm_frac_caller_order": round(unit_bytes / (ms_unit_caller * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "hbm_frac_plan_order": round(unit_bytes / (ms_unit_plan * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "note": "lmg_grid_planned + lmg_degrid_planned on the 4096^2 grid, plan reused (HIP events, mean of "
                "--steps); plan order = data kept in the plan's order (lmg_to_plan_order once), no reordering",
    }
    print(f"# unit: caller order {ms_unit_caller:.3f} ms, plan order {ms_unit_plan:.3f} ms", file=sys.stderr,
          flush=True)
    del gu, vu, vp, vpo

    kernels = {}
    for name, (n, tot) in trace.items():
        avg = tot / n
        ab = algorithmic_bytes(name, nvis, N, M, cs)
        kernels[name] = {"launches": n, "avg_ms": round(avg, 5),
                         "algorithmic_GBps": round(ab / (avg * 1e-3) / 1e9, 1) if ab else None,
                         "traffic": load_traffic(name, nvis)}
    dom_avg_s = dom_trace[1] / dom_trace[0] * 1e-3
    kernels[dom]["avg_ms_timed_region"] = round(dom_avg_s * 1e3, 5)
    ab = algorithmic_bytes(dom, nvis, N, M, cs)
    achieved = ab / dom_avg_s / 1e9
    copy_gbps = measured_copy_gbps()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(dom, nvis), "kernel": dom,
                "copy_GBps": round(copy_gbps, 1), "frac_of_copy": round(achieved / copy_gbps, 4)}
    for order in ("caller_order", "plan_order"):
        grid_degrid_unit[f"copy_frac_{order}"] = round(
            unit_bytes / (grid_degrid_unit[f"ms_{order}"] * 1e-3) / 1e9 / copy_gbps, 4)
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    out = {
        "metric": METRIC,
        "value": nvis / (ms * 1e-3),
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "kahan": "f32", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": (f"{case.name}: 64-antenna Gaussian array, 2016 baselines x {nvis // 2016} hour angles, "
                         f"50-source sky; W={W}, x0={case.x0}, {case.table_size}-entry table, "
                         f"degree {case.degree}; step = uv plan + dirty image + prediction"),
            "nvis": nvis, "N": N, "W": W, "x0": case.x0, "table_size": case.table_size,
            "degree": case.degree, "precision": args.precision, "accumulation": args.precision,
        },
        "roofline": roofline,
        "kernels": kernels,
        "grid_degrid_unit": grid_degrid_unit,
        "value_plan_reused": nvis / (ms_reuse * 1e-3),
        "ms_per_step_plan_reused": round(ms_reuse, 4),
        "source_hash": kernel_source_hash(),
    }
    if not args.no_studies and args.workload == "array-16m-4096":
        for key, fn in (("precision_study", lambda: precision_study(lmg, case, uv, vis.to(torch.complex64))),
                        ("direct_weights", lambda: direct_study(lmg, case, uv, vis.to(torch.complex64))),
                        ("interpolation_study", lambda: interpolation_study(lmg, case.N, uv, vis.to(torch.complex128))),
                        ("large_table_study", lambda: large_table_study(lmg, case.N, uv, vis.to(torch.complex128))),
                        ("multichannel", lambda: multichannel_study(lmg)),
                        ("equal_misfit_comparison", lambda: equal_misfit_comparison(lmg, case, uv, vis))):
            if args.only_studies and key not in args.only_studies.split(","):
                continue
            try:
                out[key] = fn()
            except Exception as e:          # a study must not cost the main line
                out[key] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, min(args.cpu_sample, nvis))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
