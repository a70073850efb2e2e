"""Benchmark: solved right-hand sides per second at a 1e-12 true residual.

One step is one complete block solve D_W X = B (Sec. 3 of arXiv:0903.4936)
from X = 0 with the mixed-precision block BiCGGR (FP32 inner iteration, FP64
defect correction), on a synthetic quenched-like lattice already resident on
the GPU.  The default workload is the largest single-GPU one: the 32^3 x 64
lattice (links exp(i 0.3 H), seed 4), kappa = 0.135, c_SW = 1.6, with 64 Z2
noise sources (seed 41).  The library solves them as 8 column blocks of 8.

Printed (one JSON line): RHS/s of the timed steps; the FP32 Dslash kernel's
algorithmic bandwidth against the HBM roofline (HIP events around every
operator application inside the solve, on the solver's stream); the block
update kernels likewise; the same GPU's plain FP64 BiCGSTAB solving one
column at a time (on a sample of the columns); the 24^3 x 48 point-source
workload as an extra field; and the CPU oracle leg: the oracle timed on a
bounded sample, the critical hopping parameter of the link recipe, and the
oracle's FP64 true residual of the GPU solution over the whole lattice.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4_64]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s

WORKLOADS = {
    # name: dims (Lx,Ly,Lz,Lt), link eps, link seed, kappa, csw, L, sources
    "c1": dict(dims=(4, 4, 4, 4), eps=0.4, seed=1, kappa=0.125, csw=1.0, L=12, src="point"),
    "c2": dict(dims=(16, 16, 16, 32), eps=0.3, seed=2, kappa=0.136, csw=1.6, L=12, src="point"),
    "c3": dict(dims=(24, 24, 24, 48), eps=0.3, seed=3, kappa=0.135, csw=1.6, L=12, src="point"),
    "c4_24": dict(dims=(32, 32, 32, 64), eps=0.3, seed=4, kappa=0.135, csw=1.6, L=24, src="z2"),
    "c4_32": dict(dims=(32, 32, 32, 64), eps=0.3, seed=4, kappa=0.135, csw=1.6, L=32, src="z2"),
    "c4_64": dict(dims=(32, 32, 32, 64), eps=0.3, seed=4, kappa=0.135, csw=1.6, L=64, src="z2"),
}


def dslash_bytes_per_site(L: int, real_bytes: int, link_reals: int = 18) -> int:
    """Compulsory bytes of one operator application per site: 4 links (each
    shared by two sites, counted once), the 72 reals of the two clover
    blocks, one read and one write of the 12 complex spinor components of
    each of the L columns."""
    return (4 * link_reals + 72 + 48 * L) * real_bytes


def sources(w):
    import synthetic as S
    if w["src"] == "point":
        return S.point_sources(w["dims"])
    if w["src"] == "z2":
        return S.z2_sources(w["dims"], w["L"], 41)
    return S.gaussian_sources(w["dims"], w["L"], 51)


def cpu_baseline(w, block_iters, sample_dims=(12, 12, 12, 24), sample_iters: int = 5):
    """The oracle on the host, on a bounded sample of the workload: the same
    link recipe, kappa, c_SW and sources on a lattice of 12^3 x 24, running
    `sample_iters` iterations of the oracle's FP64 block BiCGGR on one block
    of the GPU's column-block width.  Every step of an iteration costs time
    proportional to the volume, so the per-iteration time is scaled by the
    volume ratio and by the iteration counts of the GPU's column blocks
    (`block_iters`: (width, iterations) per block) to give RHS/s at the full
    size.  Set-up of the site-local matrices and the solver's start (the
    first residual and its operator application) are excluded: the time per
    iteration is taken between the ends of the first and the last iteration."""
    import synthetic as S
    from oracle import dirac, solvers
    width = max(wb for wb, _ in block_iters)
    wd = dict(w, dims=sample_dims, L=width)
    U = S.gauge_links(sample_dims, w["eps"], w["seed"])
    A = dirac.as_matrix_operator(U, w["kappa"], w["csw"])
    N = 12 * S.volume(sample_dims)
    B = sources(wd).reshape(N, width)
    marks = []
    _, info = solvers.block_bicggr(A, B, 1e-30, sample_iters,
                                   callback=lambda k, st: marks.append((time.perf_counter(), time.process_time())))
    if len(marks) < 2:
        raise RuntimeError("the oracle sample stopped before two iterations")
    wall, cpu = marks[-1][0] - marks[0][0], marks[-1][1] - marks[0][1]
    iters = len(marks) - 1
    ratio = S.volume(w["dims"]) / S.volume(sample_dims)
    t_col_iter = wall / iters / width * ratio  # one column-iteration at full size
    t_solve = sum(wb * it for wb, it in block_iters) * t_col_iter
    return {
        "value": w["L"] / t_solve,
        "unit": "RHS/s",
        "cores": max(1, round(cpu / wall)),
        "kind": "oracle",
        "sample": (f"{iters} timed iterations (after a first one) of the oracle's FP64 block BiCGGR on one block of "
                   f"{width} columns, on a "
                   f"{'x'.join(map(str, sample_dims))} lattice with the workload's link recipe, kappa, c_SW and "
                   f"sources: {wall:.1f} s wall, {cpu:.1f} s CPU (cores = CPU / wall; host has {os.cpu_count()} "
                   f"logical CPUs, OMP_NUM_THREADS={os.environ.get('OMP_NUM_THREADS', 'unset')}); scaled by the "
                   f"volume ratio {ratio:g} and by the GPU's {sum(it for _, it in block_iters)} iterations over "
                   f"its {len(block_iters)} column blocks"),
    }


def oracle_leg_checks(w, U, X_host, B_np):
    """The oracle's view of the timed solve: the FP64 true residual
    max_i ||b_i - D x_i|| / ||b_i|| of the GPU's solution over the whole
    lattice, recomputed with the oracle's operator (plain-C version), and the
    critical hopping parameter of the link recipe from the oracle's
    eigenvalue probe on a 4^4 lattice with the same recipe and seed (a few
    seconds; the probe gives 0.1420 there and 0.1431 on 8^4, which takes
    minutes)."""
    import synthetic as S
    from oracle import native, spectrum
    t0 = time.perf_counter()
    M = native.local_matrix(U, w["kappa"], w["csw"])
    rel, _ = native.residual(U, w["kappa"], M, X_host, B_np)
    t1 = time.perf_counter()
    Uk = S.gauge_links((4, 4, 4, 4), w["eps"], w["seed"])
    kc = spectrum.kappa_critical(Uk, w["csw"])
    t2 = time.perf_counter()
    return ({"true_residual_max": float(rel.max()), "true_residual_min": float(rel.min()),
             "columns": int(rel.size), "sites": "whole lattice", "seconds": round(t1 - t0, 1)},
            {"value": round(kc, 5), "lattice": "4x4x4x4, same link recipe and seed", "kappa": w["kappa"],
             "bare_quark_mass": round(0.5 * (1.0 / w["kappa"] - 1.0 / kc), 5), "seconds": round(t2 - t1, 1)})


def g1_measure():
    """The differentiable-solve workload (16^3 x 32, kappa 0.134, c_SW 1.6, 12
    Gaussian sources, loss Re sum <eta_i, X_i>): forward mixed block solve,
    adjoint solve D^dagger Lam = eta, and the gradient kernels (kappa, c_SW,
    links), each timed with the device synchronised around it."""
    import torch
    import synthetic as S
    from paper_0903_4936_amd import Lattice
    dims, L = (16, 16, 16, 32), 12
    U = S.gauge_links(dims, 0.3, 5)
    lat = Lattice(U, 0.134, 1.6, device="cuda:0")
    B = torch.from_numpy(S.gaussian_sources(dims, L, 51)).to("cuda:0")
    eta = torch.from_numpy(S.gaussian_sources(dims, L, 52)).to("cuda:0")
    opts = dict(method="block_bicggr", prec="mixed", tol=1e-12)
    lat.block_solve(B, **opts)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, i_f = lat.block_solve(B, **opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Lam, i_a = lat.block_solve(eta, dagger=True, **opts)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = lat.gradients(X, Lam)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    return {"workload": "16x16x16x32, kappa 0.134, c_SW 1.6, 12 Gaussian sources, loss Re sum <eta_i, X_i>",
            "value": round(1.0 / (t3 - t0), 4), "unit": "gradient evaluations/s (forward + adjoint + gradients)",
            "forward_s": round(t1 - t0, 4), "adjoint_s": round(t2 - t1, 4), "gradients_ms": round(1e3 * (t3 - t2), 3),
            "forward_iterations": i_f["iterations"], "adjoint_iterations": i_a["iterations"],
            "adjoint_true_residual": i_a["true_residual_max"], "grad_kappa": g["kappa"], "grad_csw": g["csw"]}


def committed_traffic(kernel: str, workload: str):
    """HBM traffic per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from
    the committed profile summary, or None when the kernel's source has
    changed since the counters were taken or the workload differs."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "dslash_traffic.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("kernel") != kernel or rec.get("workload") != workload:
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return rec["traffic_bytes_per_launch"]


def copy_calibration(mib: int = 256, reps: int = 5):
    """A copy of known size: `mib` MiB read and `mib` MiB written per launch."""
    import torch
    n = mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": n * 4, "bytes_written_per_launch": n * 4,
                                           "launches": reps}}), flush=True)


def summarize_profile(trace_dir: str, pmc_dirs, regex: str, top: int = 16):
    """Markdown tables from rocprofv3 CSV output: per (kernel, grid) the
    dispatch count and the duration of the working dispatches (a launch
    queued after a block's stop returns at once; working = at least a
    quarter of the group's longest), then, for the kernels matching `regex`,
    the mean of every counter of the `--pmc` runs over working dispatches."""
    import csv
    import glob
    import re
    import statistics

    def rows(d, name):
        fs = sorted(glob.glob(os.path.join(d, "**", name), recursive=True))
        if not fs:
            raise SystemExit(f"no {name} under {d}")
        with open(fs[0]) as f:
            return list(csv.DictReader(f))

    def short(k):
        k = k.replace("(anonymous namespace)::", "").replace("void ", "")
        return k.split("(")[0] if "(" in k and not k.startswith("(") else k

    groups = {}
    for r in rows(trace_dir, "*kernel_trace.csv"):
        key = (short(r["Kernel_Name"]), int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in groups.values())
    print("| kernel | grid (threads) | dispatches | working | avg µs (working) | min µs | max µs | % of GPU time |")
    print("|---|---|---|---|---|---|---|---|")
    for (k, g), v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]:
        wk = [x for x in v if x >= 0.25 * max(v)]
        print(f"| `{k}` | {g} | {len(v)} | {len(wk)} | {statistics.mean(wk):.1f} | {min(wk):.1f} | {max(wk):.1f} "
              f"| {100 * sum(v) / total:.1f} |")
    pat = re.compile(regex)
    for d in pmc_dirs or []:
        agg = {}
        for r in rows(d, "*counter_collection.csv"):
            k = short(r["Kernel_Name"])
            if not pat.search(k):
                continue
            key = (k, int(r.get("Grid_Size") or r.get("Grid_Size_X") or 0))
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            agg.setdefault(key, {}).setdefault(r["Dispatch_Id"], {"dur": dur})[r["Counter_Name"]] = \
                float(r["Counter_Value"])
        print(f"\nCounters from `{os.path.relpath(d)}` (mean per working dispatch):\n")
        names = sorted({n for disp in agg.values() for rec in disp.values() for n in rec if n != "dur"})
        print("| kernel | grid | dispatches | " + " | ".join(names) + " |")
        print("|---|---|---|" + "---|" * len(names))
        for (k, g), disp in sorted(agg.items()):
            recs = list(disp.values())
            dmax = max(rc["dur"] for rc in recs)
            wk = [rc for rc in recs if rc["dur"] >= 0.25 * dmax]
            vals = [statistics.mean(rc[n] for rc in wk if n in rc) if any(n in rc for rc in wk) else float("nan")
                    for n in names]
            print(f"| `{k}` | {g} | {len(wk)} | " + " | ".join(f"{v:.6g}" for v in vals) + " |")


def traffic_record(kernel: str, workload: str, fetch_dir: str, write_dir: str, cal_fetch: str, cal_write: str,
                   grid: int = 0):
    """JSON record of one kernel's HBM traffic per launch: FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch, mean over working dispatches) scaled by what
    the same counters read for the 256 MiB copy of --copy-calibration."""
    import csv
    import glob
    import hashlib
    import statistics

    def counter(d, name, match):
        fs = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
        recs = []
        for r in csv.DictReader(open(fs[0])):
            if r["Counter_Name"] == name and match(r):
                recs.append(((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3, float(r["Counter_Value"])))
        dmax = max(d for d, _ in recs)
        wk = [(d, v) for d, v in recs if d >= 0.25 * dmax]
        return statistics.mean(v for _, v in wk), statistics.mean(d for d, _ in wk), len(wk)

    def is_kernel(r):
        return kernel in r["Kernel_Name"] and (not grid or int(r["Grid_Size"]) == grid)

    def is_copy(r):
        return "copy" in r["Kernel_Name"].lower()

    copy_kib = 256 * 1024
    cf, _, _ = counter(cal_fetch, "FETCH_SIZE", is_copy)
    cw, _, _ = counter(cal_write, "WRITE_SIZE", is_copy)
    f, dur, n = counter(fetch_dir, "FETCH_SIZE", is_kernel)
    wr, _, _ = counter(write_dir, "WRITE_SIZE", is_kernel)
    src = "paper_0903_4936_amd/csrc/dslash.hip" if "dslash" in kernel else "paper_0903_4936_amd/csrc/blas.hip"
    ff, wf = copy_kib / cf, copy_kib / cw
    rec = {"kernel": kernel, "workload": workload, "source": src,
           "source_sha256": hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest(),
           "fetch_size_kib": f, "write_size_kib": wr, "fetch_factor": ff, "write_factor": wf,
           "traffic_bytes_per_launch": (f * ff + wr * wf) * 1024, "avg_duration_us_under_counters": dur,
           "dispatches": n}
    print(json.dumps(rec, indent=1))


def copy_rate_gbs(mib: int = 1024, reps: int = 10) -> float:
    """Achievable HBM bandwidth on this GPU: a plain device-to-device copy of
    `mib` MiB, (read + written bytes) / time, median of `reps` event-timed
    launches."""
    import torch
    n = mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del x, y
    return 2 * n * 4 / float(np.median(ts)) / 1e9


def timed_solves(lat, B, X, opts, steps: int, warmup: int, tag: str):
    """`warmup` untimed and `steps` timed solves from X = 0; returns the
    solve infos and the wall time of the timed ones (device synchronised on
    both sides)."""
    import torch

    def step():
        X.zero_()
        return lat.block_solve(B, X, opts=opts)[1]

    print(f"[bench] {tag}: warmup {warmup}", file=sys.stderr, flush=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(steps):
        infos.append(step())
        print(f"[bench] {tag} step {k}: {infos[-1]['seconds']:.3f} s, iterations {infos[-1]['iterations']}, "
              f"true residual {infos[-1]['true_residual_max']:.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return infos, time.perf_counter() - t0


def kernel_figures(infos, V, L, fp32: bool, link_reals: int, method: str, ms_per_step: float):
    """Rooflines of the operator and the block update kernels of the
    full-width column blocks, from the HIP events the solver records around
    each launch (launches after a block's stop are not counted)."""
    Lw = infos[-1]["main_width"]
    widths = [Lw] * (L // Lw) + ([L % Lw] if L % Lw else [])
    calls = sum(i["dslash_calls_fp32_main"] if fp32 else i["dslash_calls"] for i in infos)
    ms = sum(i["dslash_ms_fp32_main"] if fp32 else i["dslash_ms"] for i in infos)
    bytes_per_launch = V * dslash_bytes_per_site(Lw, 4 if fp32 else 8, link_reals)
    avg_s = (ms / calls) * 1e-3 if calls else float("nan")
    achieved = bytes_per_launch / avg_s / 1e9
    # the solver's blocks are component-major: the folded-link record kernel,
    # or the staged kernel with two-row links
    if link_reals == 12:
        kname = "k_dslash_st<float, false, true, 0, true>"
    else:
        kname = f"k_dslash_sr<{'float' if fp32 else 'double'}, false, true>"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": kname + " (multi-RHS clover Wilson-Dirac operator)",
                "bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_s * 1e6, 2),
                "launches_timed": calls}
    upd = []
    if method == "block_bicggr":
        if fp32 and Lw == 8:
            # the lane-per-real kernels: the solution update rides in the U pass;
            # with gram_operator the Gram pass rides in the operator launch
            # W' = A T, whose algorithmic bytes are the operator's plus one
            # pass over R~ (T and W' are the operator's own input and output)
            names = ["U = (T - zeta W') m1 + (U - zeta Y) m2; X += T m3 + U m4",
                     "T = (T - zeta W') m3 - Y; Grams T^H T, R~^H T, R~^H Y",
                     "Grams of T, W' and R~ (the frame's Gram pass)"]
            passes = [7, 5, 3]
            if infos[-1].get("gram_operator"):
                names[2] = "W' = A T with the Grams T^H W', W'^H W', R~^H W' (operator launch)"
                passes[2] = None
        elif fp32 and Lw <= 16:
            names = ["U = (T - zeta W') m1 + (U - zeta Y) m2",
                     "X += T m1 + U m2; T = (T - zeta W') m3 - Y; Grams T^H T, R~^H T, R~^H Y",
                     "Grams of T, W' and R~ (the frame's Gram pass)"]
            passes = [5, 8, 3]
        else:
            names = ["U = (P - zeta V) alpha", "X += (zeta Q + U) xi; T = Q - zeta W - Y; Grams T^H T, R~^H T",
                     "Q = T tau^-1; W = W' tau^-1; P = Q + U gamma; V = W + Y gamma; Grams R~^H V, W^H Q, W^H W"]
            passes = [3, 8, 9]
        pass_b = 12 * V * Lw * (8 if fp32 else 16)
        for q in range(3):
            ms_q = sum(i["update_ms_main"][q] for i in infos)
            n_q = sum(i["update_calls_main"][q] for i in infos)
            if n_q:
                avg = ms_q / n_q * 1e-3
                nbytes = (V * dslash_bytes_per_site(Lw, 4, link_reals) + pass_b) if passes[q] is None \
                    else passes[q] * pass_b
                gbs = nbytes / avg / 1e9
                upd.append({"step": names[q], "block_passes": passes[q], "bytes_per_launch": nbytes,
                            "avg_launch_us": round(avg * 1e6, 1), "achieved": round(gbs, 1), "unit": "GB/s",
                            "frac": round(gbs / HBM_PEAK_GBS, 4), "launches_timed": n_q})
    # the whole solve against HBM: iterations x algorithmic bytes of one
    # iteration of the fused schedule (2 operator applications + 15 block
    # passes of N x (block width) complex values) at 8 TB/s, over the measured
    # time; with blocks of several widths, the bytes of one iteration are
    # averaged over the blocks (their iteration counts are close)
    it_total = sum(i["iterations"] for i in infos) / len(infos)
    rb = 4 if fp32 else 8
    iter_bytes = sum(2 * V * dslash_bytes_per_site(wb, rb, link_reals) + 15 * 12 * V * wb * 2 * rb
                     for wb in widths) / len(widths)
    solve_frac = it_total * iter_bytes / (HBM_PEAK_GBS * 1e9) / (ms_per_step * 1e-3)
    return widths, roofline, upd, round(solve_frac, 4), round(ms / len(infos), 2)


def schur_bytes_per_site(L: int, real_bytes: int) -> int:
    """Compulsory bytes of one even-odd Schur application, per site of the
    whole lattice: its two launches each touch every link once (4 x 18 reals
    per site) and the site-local blocks of half the sites (A^{-1} on the odd,
    A on the even sites: 36 reals per site); the compact blocks move five
    half-lattice spinor passes (read x_e, write and read A_oo^{-1} H_oe x_e,
    read x_e again for A_ee, write the result), each 24 L reals per site of
    one parity, i.e. 12 L reals per site of the whole lattice: 5 x 12 L."""
    return (2 * 4 * 18 + 2 * 36 + 5 * 12 * L) * real_bytes


def evenodd_figures(lat, B, X, L, V, steps: int, warmup: int, tag: str, ref_value: float):
    """The same solve with the even-odd split (opts.evenodd): RHS/s, and the
    Schur operator's algorithmic bandwidth from the events around its launches."""
    opts = lat.make_opts(method="block_bicggr", prec="mixed", tol=1e-12, profile=True, evenodd=True)
    infos, elapsed = timed_solves(lat, B, X, opts, steps, warmup, tag + " even-odd")
    value = L * steps / elapsed
    Lw = infos[-1]["main_width"]
    calls = sum(i["dslash_calls_fp32_main"] for i in infos)
    ms = sum(i["dslash_ms_fp32_main"] for i in infos)
    bpl = V * schur_bytes_per_site(Lw, 4)
    avg_s = (ms / calls) * 1e-3 if calls else float("nan")
    out = {"value": round(value, 4), "unit": "RHS/s", "steps": steps, "ms_per_step": round(1e3 * elapsed / steps, 2),
           "iterations": infos[-1]["iterations"], "true_residual_max": infos[-1]["true_residual_max"],
           "speedup_over_whole_lattice_solve": round(value / ref_value, 3),
           "schur_operator": {"achieved": round(bpl / avg_s / 1e9, 1), "unit": "GB/s",
                              "frac": round(bpl / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                              "bytes_per_application": bpl, "avg_application_us": round(avg_s * 1e6, 2),
                              "applications_timed": calls}}
    if infos[-1].get("gram_operator"):
        # W' = S T with the frame's Grams: the Schur operator's bytes and one
        # compact pass over R~ (12 L reals per site of the whole lattice)
        gcalls = sum(i["update_calls_main"][2] for i in infos)
        gms = sum(i["update_ms_main"][2] for i in infos)
        gb = V * (schur_bytes_per_site(Lw, 4) + 12 * Lw * 4)
        if gcalls:
            g_s = gms / gcalls * 1e-3
            out["schur_gram_launch"] = {"achieved": round(gb / g_s / 1e9, 1), "unit": "GB/s",
                                        "frac": round(gb / g_s / 1e9 / HBM_PEAK_GBS, 4), "bytes_per_launch": gb,
                                        "avg_launch_us": round(g_s * 1e6, 2), "launches_timed": gcalls}
    return out


def workload_text(w, method, prec):
    return (f"{'x'.join(map(str, w['dims']))} clover Wilson, links exp(i {w['eps']} H) seed {w['seed']}, "
            f"kappa {w['kappa']}, c_SW {w['csw']}, {w['L']} {w['src']} sources, {method} {prec}, true residual 1e-12")


def extra_workload(name: str, steps: int = 3):
    """A second workload measured the same way (3 timed solves after one
    warm-up), reported beside the headline."""
    import torch
    import synthetic as S
    from paper_0903_4936_amd import Lattice
    w = WORKLOADS[name]
    V = S.volume(w["dims"])
    U = S.gauge_links(w["dims"], w["eps"], w["seed"])
    lat = Lattice(U, w["kappa"], w["csw"], device="cuda:0")
    B = torch.from_numpy(sources(w)).to("cuda:0")
    X = torch.zeros_like(B)
    opts = lat.make_opts(method="block_bicggr", prec="mixed", tol=1e-12, profile=True)
    infos, elapsed = timed_solves(lat, B, X, opts, steps, 1, name)
    ms_per_step = 1e3 * elapsed / steps
    widths, roofline, upd, solve_frac, _ = kernel_figures(infos, V, w["L"], True, 18, "block_bicggr", ms_per_step)
    eo = evenodd_figures(lat, B, X, w["L"], V, steps, 1, name, w["L"] * steps / elapsed)
    return {"workload": workload_text(w, "block_bicggr", "mixed"), "value": round(w["L"] * steps / elapsed, 4),
            "evenodd": eo,
            "unit": "RHS/s", "steps": steps, "ms_per_step": round(ms_per_step, 2), "block_columns": widths,
            "iterations": infos[-1]["iterations"], "true_residual_max": infos[-1]["true_residual_max"],
            "roofline_dslash": {k: roofline[k] for k in ("achieved", "frac", "avg_launch_us", "launches_timed")},
            "update_kernels": [{k: u[k] for k in ("block_passes", "avg_launch_us", "frac")} for u in upd],
            "solve_roofline_frac": solve_frac}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4_64", choices=sorted(WORKLOADS))
    ap.add_argument("--method", default="block_bicggr")
    ap.add_argument("--prec", default="mixed")
    ap.add_argument("--compress", type=int, default=0)
    ap.add_argument("--max-block", type=int, default=0,
                    help="most columns per block solve (0: the library's choice: blocks of 8 for mixed "
                         "solves, of 16 above 16 columns for FP64)")
    ap.add_argument("--check-every", type=int, default=8,
                    help="iterations queued between the host's status reads (1: no launch is queued after a "
                         "block's stop, so every profiled dispatch does work)")
    ap.add_argument("--fp64-baseline-cols", type=int, default=8,
                    help="columns of the FP64 one-column BiCGSTAB baseline (a sample: each column is an "
                         "independent solve; 0 = all L)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (CPU timing, kappa_c, "
                                                                    "oracle residual of the GPU solution)")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    ap.add_argument("--no-g1", action="store_true", help="skip the differentiable-solve measurement")
    ap.add_argument("--no-extra", action="store_true", help="skip the 24^3 x 48 point-source workload")
    ap.add_argument("--no-evenodd", action="store_true", help="skip the even-odd preconditioned solve")
    ap.add_argument("--no-one-block", action="store_true",
                    help="skip the comparison solve of all L columns as one block (L <= 16 only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy five times (the reference kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    ap.add_argument("--summarize-profile", metavar="TRACE_DIR",
                    help="only print markdown tables of a rocprofv3 --kernel-trace output directory (and of the "
                         "--pmc directories), reading the CSV files")
    ap.add_argument("--pmc", nargs="*", default=[], metavar="DIR")
    ap.add_argument("--kernels", default="k_dslash|k_l8|k_s_", help="kernel-name pattern of the counter tables")
    ap.add_argument("--traffic-json", nargs=6, metavar=("KERNEL", "WORKLOAD", "FETCH_DIR", "WRITE_DIR",
                                                         "CAL_FETCH_DIR", "CAL_WRITE_DIR"),
                    help="only print the copy-calibrated HBM traffic record of one kernel from rocprofv3 "
                         "FETCH_SIZE / WRITE_SIZE runs")
    ap.add_argument("--grid", type=int, default=0, help="grid size (threads) of the --traffic-json dispatches")
    args = ap.parse_args()
    if args.traffic_json:
        traffic_record(*args.traffic_json, grid=args.grid)
        return
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.pmc, args.kernels)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synthetic as S
    from paper_0903_4936_amd import Lattice

    w = WORKLOADS[args.workload]
    dims, L = w["dims"], w["L"]
    V = S.volume(dims)
    U = S.gauge_links(dims, w["eps"], w["seed"])
    B_np = sources(w)
    dev = torch.device("cuda:0")
    lat = Lattice(U, w["kappa"], w["csw"], flags=args.compress, device="cuda:0")
    B = torch.from_numpy(B_np).to(dev)
    X = torch.zeros_like(B)
    opts = lat.make_opts(method=args.method, prec=args.prec, tol=1e-12, profile=True, max_block=args.max_block,
                         check_every=args.check_every)
    infos, elapsed = timed_solves(lat, B, X, opts, args.steps, args.warmup,
                                  f"workload {args.workload} dims={dims} L={L} {args.method}/{args.prec}")
    X_host = X.cpu().numpy() if not args.no_cpu_baseline else None

    # downstream use of the 12 point-source solutions: pion and rho two-point
    # functions, one pass over X (bkwd_meson_correlators), outside the timed region
    mesons = None
    if w["src"] == "point" and L == 12:
        lat.meson_correlators(X)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        ev0.record()
        for _ in range(reps):
            pion, rho = lat.meson_correlators(X)
        ev1.record()
        torch.cuda.synchronize()
        ms_c = ev0.elapsed_time(ev1) / reps
        p = pion.cpu().numpy()
        mesons = {"ms": round(ms_c, 3), "read_GBs": round(V * 144 * 16 / (ms_c * 1e-3) / 1e9, 1),
                  "pion_t0_t1_t2": [float(v) for v in p[:3]],
                  "pion_effective_mass_t1": float(np.log(p[1] / p[2])),
                  "rho_t1": float(rho[1].item())}
    ms_per_step = 1e3 * elapsed / args.steps
    value = L * args.steps / elapsed
    fp32 = args.prec == "mixed"
    link_reals = 12 if (args.compress and fp32) else 18
    widths, roofline, upd, solve_frac, dslash_ms = kernel_figures(infos, V, L, fp32, link_reals, args.method,
                                                                   ms_per_step)
    Lw = infos[-1]["main_width"]
    wl = f"{'x'.join(map(str, dims))} L={Lw} {'FP32' if fp32 else 'FP64'}"
    traffic = committed_traffic(roofline["kernel"].split(" (")[0], wl)
    roofline["traffic"] = round(traffic) if traffic is not None else None
    copy_gbs = copy_rate_gbs()
    roofline["copy_GBs"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 4)

    iters = infos[-1]["iterations"]
    out = {
        "metric": "solved RHS/s at 1e-12 true residual (block mixed vs plain FP64); Dslash GB/s",
        "value": round(value, 4),
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": workload_text(w, args.method, args.prec),
                   "lattice": list(dims), "L": L, "kappa": w["kappa"], "csw": w["csw"], "method": args.method,
                   "prec": args.prec, "compress12": bool(args.compress),
                   "block_columns": widths},
        "iterations": iters,
        "outer_cycles": infos[-1]["outer_cycles"],
        "matvecs": infos[-1]["matvecs"],
        "true_residual_max": infos[-1]["true_residual_max"],
        "roofline": roofline,
        "solve_roofline_frac": solve_frac,
        "update_kernels": upd,
        "dslash_ms_per_step": dslash_ms,
    }

    if not args.no_fp64_baseline:
        k = L if args.fp64_baseline_cols <= 0 else min(L, args.fp64_baseline_cols)
        print(f"[bench] FP64 BiCGSTAB one column at a time ({k} of {L} columns)", file=sys.stderr, flush=True)
        o64 = lat.make_opts(method="bicgstab", prec="fp64", tol=1e-12, profile=True, shadow=0)
        Bk = B[..., :k].contiguous()
        Xk = torch.zeros_like(Bk)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, i64 = lat.block_solve(Bk, Xk, opts=o64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        del Bk, Xk
        bps = V * dslash_bytes_per_site(1, 8)
        out["gpu_fp64_bicgstab"] = {
            "value": round(k / t64, 4), "unit": "RHS/s", "seconds": round(t64, 4), "columns_solved": k,
            "iterations_total": i64["iterations"], "true_residual_max": i64["true_residual_max"],
            "dslash_GBs": round(bps / (i64["dslash_ms"] / i64["dslash_calls"] * 1e-3) / 1e9, 1)
            if i64["dslash_calls"] else None,
            "speedup_of_block_mixed": round(value / (k / t64), 3),
        }
    if mesons is not None:
        out["meson_correlators"] = mesons
    if not args.no_evenodd and fp32 and args.method == "block_bicggr" and all(d % 2 == 0 for d in dims):
        # at most 5 timed solves: a comparison, not the headline
        out["evenodd"] = evenodd_figures(lat, B, X, L, V, min(args.steps, 5), 1, args.workload, value)
    if fp32 and args.method != "bicgstab" and Lw < L <= 16 and not args.no_one_block:
        # the same columns as one block of L, for comparison (not the value), in
        # its fastest measured form: the explicit QR frame
        o1 = lat.make_opts(method=args.method, prec=args.prec, tol=1e-12, max_block=L, qr_frame=1)
        X.zero_()
        lat.block_solve(B, X, opts=o1)
        X.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, i1 = lat.block_solve(B, X, opts=o1)
        torch.cuda.synchronize()
        t_one = time.perf_counter() - t1
        out["one_block_of_L"] = {"value": round(L / t_one, 4), "unit": "RHS/s", "qr_frame": 1,
                                 "iterations": i1["iterations"], "true_residual_max": i1["true_residual_max"]}
    del lat, B, X
    torch.cuda.empty_cache()
    if not args.no_extra and args.workload != "c3":
        out["c3_24x24x24x48_point"] = extra_workload("c3")
    if not args.no_g1:
        print("[bench] differentiable solve (16^3 x 32)", file=sys.stderr, flush=True)
        out["g1_gradients"] = g1_measure()
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle leg", file=sys.stderr, flush=True)
        # block widths and iteration counts of the GPU's column blocks (the
        # iterations of the blocks are not reported separately: equal split)
        nb = len(widths)
        block_iters = [(wb, iters / nb) for wb in widths]
        out["cpu_baseline"] = cpu_baseline(w, block_iters)
        chk, kc = oracle_leg_checks(w, U, X_host, B_np)
        out["oracle_check"] = chk
        out["kappa_c"] = kc
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
