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


def cpu_baseline(w, U, gpu_iters_per_rhs: float):
    """The oracle on the host: one FP64 operator application with one column
    on the full lattice, extrapolated to two applications per iteration and
    the GPU's iteration count per right-hand side (vector updates and the
    oracle's own iteration count are not included: an optimistic bound)."""
    import synthetic as S
    from oracle import dirac
    local = dirac.local_matrix(U, w["kappa"], w["csw"])
    x = S.gaussian_sources(w["dims"], 1, 5)
    t0 = time.perf_counter()
    dirac.apply(U, w["kappa"], w["csw"], x, local=local)
    t_apply = time.perf_counter() - t0
    per_rhs = 2.0 * gpu_iters_per_rhs * t_apply
    return {
        "value": 1.0 / per_rhs,
        "unit": "RHS/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one oracle D_W application, 1 column, {'x'.join(map(str, w['dims']))} lattice: "
                   f"{t_apply:.2f} s on 1 thread of {os.cpu_count()} host cores; extrapolated to 2 applications "
                   f"x {gpu_iters_per_rhs:.0f} iterations per RHS"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--method", default="block_bicggr")
    ap.add_argument("--prec", default="mixed")
    ap.add_argument("--compress", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    args = ap.parse_args()
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
    opts = lat.make_opts(method=args.method, prec=args.prec, tol=1e-12, profile=True)

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
    ms_per_step = 1e3 * elapsed / args.steps
    value = L * args.steps / elapsed

    # dominant kernel: the operator application in the inner precision
    fp32 = args.prec == "mixed"
    calls = sum(i["dslash_calls_fp32"] if fp32 else i["dslash_calls"] for i in infos)
    ms = sum(i["dslash_ms_fp32"] if fp32 else i["dslash_ms"] for i in infos)
    link_reals = 12 if (args.compress and fp32) else 18
    bytes_per_launch = V * dslash_bytes_per_site(L, 4 if fp32 else 8, link_reals)
    avg_s = (ms / calls) * 1e-3 if calls else float("nan")
    achieved = bytes_per_launch / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_dslash<float> (FP32 multi-RHS clover Wilson)" if fp32 else "k_dslash<double>",
                "bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_s * 1e6, 2),
                "launches_timed": calls}

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
                   "prec": args.prec, "compress12": bool(args.compress)},
        "iterations": iters,
        "outer_cycles": infos[-1]["outer_cycles"],
        "matvecs": infos[-1]["matvecs"],
        "true_residual_max": infos[-1]["true_residual_max"],
        "roofline": roofline,
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
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, U, iters / 1.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
