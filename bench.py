"""Benchmark of the even-odd Wilson-clover inversion on one MI355X.

One step = the whole hot path on one synthetic gauge field and source:
  operator set-up (pack links to reconstruct-12, clover build, clover inverse
  in FP64 and in the inner precision), an FP64 even-odd BiCGStab solve to an
  FP64 true residual of 1e-10, and a mixed-precision solve (BF16 storage,
  FP32 arithmetic, FP64 reliable updates) of the same system to 1e-10.

Workload: 16^3 x 32 lattice, kappa 0.124, csw 1.0, links exp(i 0.2 H), Z2
source (seed 1000).  Inputs are generated on the host and copied to HBM
before the timed region.

Printed line (rank 0): metric/value = algorithmic bytes of the Krylov
iterations (byte model per iteration and precision, counted with the actual
iteration numbers) divided by the step's wall time; roofline = the dominant
hop kernel (H_oe with fused A_oo^-1) timed with HIP events on the library's
stream during the timed steps; cpu_baseline = the FP64 CPU oracle's full
operator on the same lattice.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# algorithmic bytes per even site (compulsory traffic of each kernel, inputs read once, outputs written once)
#   hop into odd sites with A_oo^-1 : 8 links + psi + A^-1 + out
#   per BiCGStab iteration          : 2 such hops, 2 hops into even sites with xpay, one dot operand,
#                                     s = r - a v (3 vectors), x/r update with dots (7), p update (4)
LINK_R12 = {"f64": 96, "f32": 48, "bf16": 24, "f16": 24}
SPINOR = {"f64": 192, "f32": 96, "bf16": 48, "f16": 48}
CLOVER = {"f64": 576, "f32": 288, "bf16": 144, "f16": 144}


def hop_a_bytes(prec):
    return 8 * LINK_R12[prec] + 2 * SPINOR[prec] + CLOVER[prec]


def hop_b_bytes(prec):
    return hop_a_bytes(prec) + SPINOR[prec]


def iter_bytes(prec):
    s = SPINOR[prec]
    xs = SPINOR["f64"] if prec == "f64" else SPINOR["f32"]  # x is kept in FP64 / FP32
    hops = 2 * hop_a_bytes(prec) + 2 * hop_b_bytes(prec) + s
    return hops + 3 * s + (2 * xs + 5 * s) + 4 * s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--inner", default="bf16", choices=["f32", "bf16", "f16"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--eager", action="store_true", help="launch the iteration kernels eagerly instead of "
                    "replaying captured hipGraphs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extra-lattice", default="24,24,24,64",
                    help="also time the hop kernel on this lattice (empty to skip)")
    ap.add_argument("--matpc-only", default="",
                    help="profiling mode: a 256 MiB device copy (counter calibration), then a few M_hat "
                         "applications in FP64 and BF16 on this lattice, e.g. 24,24,24,64; prints nothing else")
    return ap.parse_args()


def matpc_only(L):
    import numpy as np
    import torch

    import lattice_inputs as li
    import paper_2411_08461_amd as q

    src = torch.empty(32 * 2 ** 20, dtype=torch.float64, device="cuda")  # 256 MiB
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    Vh = int(np.prod(L)) // 2
    U = torch.from_numpy(li.random_gauge(L, 0.2, 0)).cuda()
    xe = torch.from_numpy(li.z2_source(L, 1000).reshape(-1, 4, 3)[:Vh].copy()).cuda()
    out = torch.empty_like(xe)
    ctx = q.Context(0)
    op = q.Operator(ctx, q.make_lattice(L), U, 0.125, 1.1, "bf16", 12)
    for prec in ("f64", "bf16"):
        for _ in range(3):
            q.qcdw_op_matpc(op, prec, xe, out)
    torch.cuda.synchronize()
    op.close()
    ctx.close()
    print(json.dumps({"matpc_only": list(L), "copy_bytes": 2 * src.numel() * 8}))


def main():
    args = parse()
    if args.matpc_only:
        matpc_only([int(v) for v in args.matpc_only.split(",")])
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the multi-GPU "
              "decomposition is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import lattice_inputs as li
    import paper_2411_08461_amd as q

    w = li.WORKLOADS["wc16x32"]
    L, kappa, csw = w["L"], w["kappa"], w["csw"]
    Vh = int(np.prod(L)) // 2
    U = li.random_gauge(L, w["eps"], w["seed"])
    b = li.z2_source(L, w["source_seed"])

    ctx = q.Context(0)
    lat = q.make_lattice(L)
    Ud = torch.from_numpy(U).cuda()
    bd = torch.from_numpy(b).cuda()
    x64 = torch.zeros_like(bd)
    xlo = torch.zeros_like(bd)
    torch.cuda.synchronize()

    p64 = q.make_params(tol=1e-10, maxiter=20000, inner="f64", use_graph=not args.eager)
    plo = q.make_params(tol=1e-10, maxiter=20000, inner=args.inner, delta=0.1 if args.inner != "f16" else 0.2,
                        use_graph=not args.eager)

    def step():
        op = q.Operator(ctx, lat, Ud, kappa, csw, args.inner, 12)
        x64.zero_()
        xlo.zero_()
        i64 = q.qcdw_invert(op, bd, x64, p64, raise_on_error=True)
        ilo = q.qcdw_invert(op, bd, xlo, plo, raise_on_error=True)
        op.close()
        return i64, ilo

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    total_bytes = sum(i64.iters * iter_bytes("f64") * Vh + ilo.iters * iter_bytes(args.inner) * Vh
                      for i64, ilo in infos)
    value = total_bytes / elapsed / 1e9

    # roofline of the dominant kernel, the FP64 hop into odd sites with fused A_oo^-1 (two launches
    # per iteration): the same solves again, launched eagerly, every hop dispatch timed by HIP events
    # that the dispatch itself records on the library's stream
    t64 = q.make_params(tol=1e-10, maxiter=20000, inner="f64", collect_timing=True)
    tlo = q.make_params(tol=1e-10, maxiter=20000, inner=args.inner, delta=plo.delta, collect_timing=True)
    op = q.Operator(ctx, lat, Ud, kappa, csw, args.inner, 12)
    timed = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        x64.zero_()
        xlo.zero_()
        timed.append((q.qcdw_invert(op, bd, x64, t64, raise_on_error=True),
                      q.qcdw_invert(op, bd, xlo, tlo, raise_on_error=True)))
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t1) / args.steps
    op.close()
    ms_a = sum(i64.hop_ms[0] for i64, _ in timed)
    n_a = sum(i64.n_hop[0] for i64, _ in timed)
    avg_a_ms = ms_a / max(n_a, 1)
    achieved = hop_a_bytes("f64") * Vh / (avg_a_ms * 1e-3) / 1e9
    ms_b = sum(i64.hop_ms[1] + i64.hop_ms[2] for i64, _ in timed)
    n_b = sum(i64.n_hop[1] + i64.n_hop[2] for i64, _ in timed)
    ms_alo = sum(ilo.hop_ms[0] for _, ilo in timed)
    n_alo = sum(ilo.n_hop[0] for _, ilo in timed)
    lo_gbs = hop_a_bytes(args.inner) * Vh / (ms_alo / max(n_alo, 1) * 1e-3) / 1e9

    i64, ilo = infos[-1]
    result = {
        "metric": "dslash GB/s (% HBM peak); time to 1e-10 residual, plain FP64 vs mixed/ML",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "wilson-clover even-odd BiCGStab 16^3x32, kappa 0.124, csw 1.0, eps 0.2, Z2 source",
                   "lattice": list(L), "kappa": kappa, "csw": csw, "tol": 1e-10, "inner": args.inner},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "hop_kernel<P64, r12, EPI_CLOV, RED_NONE>", "launches_timed": n_a,
                     "bytes_per_launch": hop_a_bytes("f64") * Vh, "avg_launch_us": round(avg_a_ms * 1e3, 2)},
        "solve": {
            "f64": {"iters": i64.iters, "true_res": i64.true_res, "time_ms": round(i64.time_ms, 3),
                    "reliable": i64.n_reliable},
            args.inner: {"iters": ilo.iters, "true_res": ilo.true_res, "time_ms": round(ilo.time_ms, 3),
                         "reliable": ilo.n_reliable},
            "speedup_mixed": round(i64.time_ms / ilo.time_ms, 3),
            "graph": not args.eager,
            "eager_instrumented_ms_per_step": round(eager_ms, 3),
        },
        "hop_gbs": {"f64_into_odd": round(achieved, 1),
                    "f64_into_even_xpay": round((hop_b_bytes("f64") + SPINOR["f64"] / 2) * Vh /
                                                (ms_b / max(n_b, 1) * 1e-3) / 1e9, 1),
                    f"{args.inner}_into_odd": round(lo_gbs, 1)},
    }

    result["stream_gbs"] = stream_probe(torch)
    if args.extra_lattice:
        result["hop_gbs_large"] = time_large_hop(q, li, np, torch, ctx, [int(v) for v in args.extra_lattice.split(",")])

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(li, np, L, U, b, kappa, csw, args.cpu_seconds)

    print(json.dumps(result))
    sys.stdout.flush()
    ctx.close()


def stream_probe(torch):
    """Context only: what plain torch copy / sum kernels reach on this GPU (1 GiB operands)."""
    a = torch.empty(128 * 2 ** 20, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 2 * a.numel() * 8),
                             ("read_sum", lambda: a.sum(), a.numel() * 8)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(10 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def time_large_hop(q, li, np, torch, ctx, L):
    """Hop-kernel bandwidth on a lattice whose working set exceeds the on-die caches.

    Uses FP64 and BF16 solves capped at a few iterations with event timing;
    reported beside the main line, not part of the step.
    """
    Vh = int(np.prod(L)) // 2
    U = li.random_gauge(L, 0.2, 0)
    b = li.z2_source(L, 1000)
    lat = q.make_lattice(L)
    Ud = torch.from_numpy(U).cuda()
    bd = torch.from_numpy(b).cuda()
    del U
    out = {"lattice": list(L)}
    op = q.Operator(ctx, lat, Ud, 0.125, 1.1, "bf16", 12)
    for prec in ("f64", "bf16"):
        x = torch.zeros_like(bd)
        prm = q.make_params(tol=1e-10, maxiter=24, inner=prec, collect_timing=True, check_every=8)
        info = q.qcdw_invert(op, bd, x, prm)
        ms = info.hop_ms[0] / max(info.n_hop[0], 1)
        gbs = hop_a_bytes(prec) * Vh / (ms * 1e-3) / 1e9
        out[prec] = {"gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_launch_us": round(ms * 1e3, 2)}
    op.close()
    return out


def cpu_baseline(li, np, L, U, b, kappa, csw, seconds):
    """The FP64 oracle's full operator M on the same lattice, on the host cores."""
    import oracle

    threads = oracle.num_threads()
    C = oracle.clover_build(L, U)
    V = int(np.prod(L))
    oracle.dirac(L, U, C, b, kappa, csw)  # warm-up
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.dirac(L, U, C, b, kappa, csw)
        n += 1
        if time.perf_counter() - t0 > seconds or n >= 500:
            break
    dt = (time.perf_counter() - t0) / n
    # same byte model as the GPU hop with clover and xpay, FP64 reconstruct-12, per site
    gbs = (hop_b_bytes("f64") - SPINOR["f64"]) * V / dt / 1e9
    return {"value": round(gbs, 2), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} full-lattice applications of M (16^3x32, FP64) in {n * dt:.1f} s, "
                      f"{dt * 1e3:.1f} ms each; bytes counted with the GPU hop byte model"}


if __name__ == "__main__":
    main()
