"""Benchmark: solved right-hand sides per second at a 1e-12 true residual.

One step is one complete block solve D_W X = B (Sec. 3 of arXiv:0903.4936)
from X = 0 with the mixed-precision block BiCGGR (FP32 inner iteration, FP64
defect correction), on a synthetic quenched-like lattice already resident on
the GPU.  The default workload is the 24^3 x 48 lattice (links exp(i 0.3 H),
seed 3), kappa = 0.135, c_SW = 1.6, with the 12 point sources of Sec. 2.

Printed (one JSON line): RHS/s of the timed steps, the FP32 Dslash kernel's
algorithmic bandwidth against the HBM roofline (HIP events around every
operator application inside the solve), the same GPU's plain FP64 BiCGSTAB
solving one column at a time (the comparison the metric names), and the
CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]
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


def cpu_baseline(w, gpu_iters: int, sample_dims=(12, 12, 12, 24), sample_iters: int = 5):
    """The oracle on the host, on a bounded sample of the workload: the same
    link recipe, kappa, c_SW, L and sources on a lattice of 1/16 of the
    volume, running `sample_iters` iterations of the oracle's FP64 block
    BiCGGR.  Every step of an iteration costs time proportional to the
    volume, so the per-iteration time is scaled by the volume ratio and by the
    GPU solve's iteration count to give RHS/s at the full size (setup of the
    site-local matrices is excluded, as on the GPU side)."""
    import synthetic as S
    from oracle import dirac, solvers
    wd = dict(w, dims=sample_dims)
    U = S.gauge_links(sample_dims, w["eps"], w["seed"])
    A = dirac.as_matrix_operator(U, w["kappa"], w["csw"])
    N = 12 * S.volume(sample_dims)
    B = sources(wd).reshape(N, w["L"])
    c0, t0 = time.process_time(), time.perf_counter()
    _, info = solvers.block_bicggr(A, B, 1e-30, sample_iters)
    wall, cpu = time.perf_counter() - t0, time.process_time() - c0
    iters = max(1, info["iterations"])
    t_iter_full = wall / iters * (S.volume(w["dims"]) / S.volume(sample_dims))
    return {
        "value": w["L"] / (t_iter_full * gpu_iters),
        "unit": "RHS/s",
        "cores": max(1, round(cpu / wall)),
        "kind": "oracle",
        "sample": (f"{iters} iterations of the oracle's FP64 block BiCGGR, L={w['L']}, on a "
                   f"{'x'.join(map(str, sample_dims))} lattice with the workload's link recipe, kappa, c_SW and "
                   f"sources: {wall:.1f} s wall, {cpu:.1f} s CPU; scaled by the volume ratio "
                   f"{S.volume(w['dims']) // S.volume(sample_dims)} and by {gpu_iters} iterations (the GPU's solve "
                   f"of the {w['L']} columns as one block)"),
    }


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--method", default="block_bicggr")
    ap.add_argument("--prec", default="mixed")
    ap.add_argument("--compress", type=int, default=0)
    ap.add_argument("--max-block", type=int, default=0,
                    help="most columns per block solve (0: the library's choice: blocks of 8 for mixed "
                         "solves, of 16 above 16 columns for FP64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    ap.add_argument("--no-g1", action="store_true", help="skip the differentiable-solve measurement")
    ap.add_argument("--no-one-block", action="store_true",
                    help="skip the comparison solve of all L columns as one block")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy five times (the reference kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
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
    opts = lat.make_opts(method=args.method, prec=args.prec, tol=1e-12, profile=True, max_block=args.max_block)

    def step():
        X.zero_()
        return lat.block_solve(B, X, opts=opts)[1]

    print(f"[bench] workload {args.workload} dims={dims} L={L} {args.method}/{args.prec}: warmup {args.warmup}",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        infos.append(step())
        print(f"[bench] step {k}: {infos[-1]['seconds']:.3f} s, iterations {infos[-1]['iterations']}, "
              f"true residual {infos[-1]['true_residual_max']:.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

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

    # the library solves the L columns as blocks of main_width columns and one
    # with the rest; the kernel rooflines use the launches of the full blocks
    Lw = infos[-1]["main_width"]
    widths = [Lw] * (L // Lw) + ([L % Lw] if L % Lw else [])
    # dominant kernel: the operator application in the inner precision
    fp32 = args.prec == "mixed"
    calls = sum(i["dslash_calls_fp32_main"] if fp32 else i["dslash_calls"] for i in infos)
    ms = sum(i["dslash_ms_fp32_main"] if fp32 else i["dslash_ms"] for i in infos)
    link_reals = 12 if (args.compress and fp32) else 18
    bytes_per_launch = V * dslash_bytes_per_site(Lw, 4 if fp32 else 8, link_reals)
    avg_s = (ms / calls) * 1e-3 if calls else float("nan")
    achieved = bytes_per_launch / avg_s / 1e9
    kname = f"k_dslash_st<{'float' if fp32 else 'double'}, false, {'true' if link_reals == 12 else 'false'}, 0, true>"
    wl = f"{'x'.join(map(str, dims))} L={Lw} {'FP32' if fp32 else 'FP64'}"
    traffic = committed_traffic(kname, wl) if Lw >= 8 else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic) if traffic is not None else None,
                "kernel": kname + " (multi-RHS clover Wilson-Dirac operator)",
                "bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_s * 1e6, 2),
                "launches_timed": calls}
    # the three block update kernels of the QR-frame Block BiCGGR, against HBM:
    # algorithmic bytes = block passes x N x (block width) complex values
    upd = []
    if args.method == "block_bicggr":
        if fp32 and Lw <= 16:
            # the default frame of mixed solves: the fused QR frame (16 passes)
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
                gbs = passes[q] * pass_b / avg / 1e9
                upd.append({"step": names[q], "block_passes": passes[q], "avg_launch_us": round(avg * 1e6, 1),
                            "achieved": round(gbs, 1), "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                            "launches_timed": n_q})
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
        "config": {"workload": f"{'x'.join(map(str, dims))} clover Wilson, links exp(i {w['eps']} H) seed {w['seed']}, "
                               f"kappa {w['kappa']}, c_SW {w['csw']}, {L} {w['src']} sources, {args.method} "
                               f"{args.prec}, true residual 1e-12",
                   "lattice": list(dims), "L": L, "kappa": w["kappa"], "csw": w["csw"], "method": args.method,
                   "prec": args.prec, "compress12": bool(args.compress),
                   "block_columns": widths},
        "iterations": iters,
        "outer_cycles": infos[-1]["outer_cycles"],
        "matvecs": infos[-1]["matvecs"],
        "true_residual_max": infos[-1]["true_residual_max"],
        "roofline": roofline,
        "solve_roofline_frac": round(solve_frac, 4),
        "update_kernels": upd,
        "dslash_ms_per_step": round(ms / len(infos), 2),
    }

    if not args.no_fp64_baseline:
        print("[bench] FP64 BiCGSTAB one column at a time", file=sys.stderr, flush=True)
        o64 = lat.make_opts(method="bicgstab", prec="fp64", tol=1e-12, profile=True, shadow=0)
        X.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, i64 = lat.block_solve(B, X, opts=o64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        bps = V * dslash_bytes_per_site(1, 8)
        out["gpu_fp64_bicgstab"] = {
            "value": round(L / t64, 4), "unit": "RHS/s", "seconds": round(t64, 4),
            "iterations_total": i64["iterations"], "true_residual_max": i64["true_residual_max"],
            "dslash_GBs": round(bps / (i64["dslash_ms"] / i64["dslash_calls"] * 1e-3) / 1e9, 1)
            if i64["dslash_calls"] else None,
            "speedup_of_block_mixed": round(value / (L / t64), 3),
        }
    if mesons is not None:
        out["meson_correlators"] = mesons
    if fp32 and args.method != "bicgstab" and Lw < L <= 16 and not args.no_one_block:
        # the same columns as one block of L, for comparison (not the value), in
        # its fastest measured form: the explicit QR frame (the fused one needs
        # more iterations at 12 columns)
        o1 = lat.make_opts(method=args.method, prec=args.prec, tol=1e-12, max_block=L, qr_frame=1)
        X.zero_()
        lat.block_solve(B, X, opts=o1)
        X.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, i1 = lat.block_solve(B, X, opts=o1)
        torch.cuda.synchronize()
        t_one = time.perf_counter() - t1
        out["one_block_of_L"] = {"value": round(L / t_one, 4), "unit": "RHS/s", "qr_frame": 1, "iterations": i1["iterations"],
                                 "true_residual_max": i1["true_residual_max"]}
    if not args.no_g1 and args.workload == "c3":
        print("[bench] differentiable solve (16^3 x 32)", file=sys.stderr, flush=True)
        out["g1_gradients"] = g1_measure()
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        # the oracle iterates on one block of all L columns: scale by the
        # iteration count of that form of the solve
        out["cpu_baseline"] = cpu_baseline(w, out.get("one_block_of_L", {}).get("iterations", iters))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
