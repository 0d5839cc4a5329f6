"""Benchmark of the even-odd Wilson-clover inversion on one MI355X.

One step = the whole single-RHS hot path on one synthetic gauge field and source:
  operator set-up (pack links to reconstruct-12, clover build, clover inverse
  in FP64 and in the inner precision), an FP64 even-odd BiCGStab solve to an
  FP64 true residual of 1e-10, and a mixed-precision solve (BF16 storage,
  FP32 arithmetic, FP64 reliable updates) of the same system to 1e-10.

Workload: 24^3 x 64 lattice, kappa 0.125, csw 1.1, links exp(i 0.2 H) (seed 0),
point source (origin, spin 0, colour 0): the lattice on which the HBM claim is
quoted (its working set is several times the 256 MB memory-side cache).  Inputs
are generated on the host and copied to HBM before the timed region.

Printed line (rank 0): metric/value = algorithmic GB/s of the dslash, the FP64
hop into odd sites with fused A_oo^-1 (the dominant kernel, two launches per
iteration), i.e. its bytes per launch (1728 B per odd site, inputs read once
and the output written once) divided by its mean launch duration, timed with
HIP events that every dispatch records on the library's stream during the
timed steps; roofline = the same kernel against 8 TB/s; cpu_baseline = the
FP64 CPU oracle's full operator on the same lattice, plus its 1-core figure and
its FP64 solve at 16^3 x 32.

Beside the timed steps (not part of them) the line carries the other
workloads: "wc16x32_cache_resident" (the 16^3 x 32 Z2-source solves with
graphs, whose working set fits the memory-side cache), "propagator"
(24^3 x 64, 12 point sources solved together with the multi-RHS hop in BF16
against 12 separate FP64 and 12 separate BF16-mixed solves), "batch" (48
uneven problems in one persistent batched solve against a loop of single
solves, solves/s), "learned" (32^3 x 64 near the critical kappa: FGMRES(32)
with the trained gauge-covariant preconditioner against plain FP64 and mixed
BiCGStab), "aniso" (the paper's anisotropic example action on 16^3 x 32 with
antiperiodic time) and "multishift" (8 shifted normal-equation solves in one
Krylov space against separate solves).  ``--bisect-kappa`` finds the learned
section's kappa.  "solve_vs_oracle" states each solve's error against the
oracle.
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


def hop_a_bytes_multi(prec, nrhs):
    """One multi-RHS hop into odd sites with A_oo^-1: links and clover once, nrhs spinors in and out."""
    return 8 * LINK_R12[prec] + CLOVER[prec] + nrhs * 2 * SPINOR[prec]


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
    ap.add_argument("--extra-lattice", default="",
                    help="also time the hop kernel on this lattice (empty to skip)")
    ap.add_argument("--sections", default="propagator,batch,learned,aniso,multishift",
                    help="comma-separated extra workloads to run after the timed steps (empty: none)")
    ap.add_argument("--bisect-kappa", action="store_true",
                    help="find the 32^3x64 kappa at which FP64 BiCGStab first needs >= 2000 iterations, then exit")
    ap.add_argument("--matpc-only", default="",
                    help="profiling mode: a 256 MiB device copy (counter calibration), then a few M_hat "
                         "applications in FP64 and BF16 on this lattice, e.g. 24,24,24,64; prints nothing else")
    ap.add_argument("--net-only", default="",
                    help="profiling mode: a 256 MiB device copy, then three applications of the learned net "
                         "(12 hidden channels) in FP32 and in BF16 on this lattice, with its BF16 layers on "
                         "the vector units and then on the matrix cores; prints one JSON line")
    ap.add_argument("--mg-only", action="store_true",
                    help="profiling mode: the learned section's multigrid set-up and FGMRES solve at 32^3x64 "
                         "only; prints one JSON line")
    ap.add_argument("--forms", default="",
                    help="with --matpc-only: hop forms nt:cgroup[:fma] to run one after the other (each in a fresh "
                         "context whose tuning file fixes the form), e.g. 1:0,1:27,2:12")
    ap.add_argument("--mrhs-forms", default="",
                    help="with --matpc-only: instead of the single-RHS forms, M_hat on 12 BF16 right-hand sides "
                         "with each of these multi-RHS hop forms (values of qcdw_ctx_tuned's mrhs_hop keys), "
                         "e.g. 0,1024")
    return ap.parse_args()


def matpc_only(L, forms, mrhs_forms=()):
    import tempfile

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
    runs = []
    if mrhs_forms:
        xs = torch.from_numpy(np.stack([li.z2_source(L, 1000 + k).reshape(-1, 4, 3)[:Vh] for k in range(12)])).cuda()
        outs = torch.empty_like(xs)
        for v in mrhs_forms:
            path = os.path.join(tempfile.gettempdir(), f"qcdw_mrhs_form_{v}.txt")
            with open(path, "w") as fh:
                fh.write(f"mrhs_hop/p2/L{L[0]}x{L[1]}x{L[2]}x{L[3]}/n12 {v}\n")
            os.environ["QCDW_TUNE_CACHE"] = path
            ctx = q.Context(0)
            op = q.Operator(ctx, q.make_lattice(L), U, 0.125, 1.1, "bf16", 12)
            for _ in range(3):
                q.qcdw_op_matpc_multi(op, "bf16", xs, outs)
            torch.cuda.synchronize()
            runs.append({"mrhs_form": v})
            op.close()
            ctx.close()
        forms = []
    for f in forms or ([] if mrhs_forms else [None]):
        if f is not None:  # a fresh context reads the tuning file that fixes the form
            nt, cg, fma = (tuple(f) + (0,))[:3]
            path = os.path.join(tempfile.gettempdir(), f"qcdw_form_{nt}_{cg}_{fma}.txt")
            with open(path, "w") as fh:
                for p in range(4):
                    fh.write(f"hop_nt/p{p}/L{L[0]}x{L[1]}x{L[2]}x{L[3]} {nt + 16 * cg + 4096 * fma}\n")
            os.environ["QCDW_TUNE_CACHE"] = path
        ctx = q.Context(0)
        op = q.Operator(ctx, q.make_lattice(L), U, 0.125, 1.1, "bf16", 12)
        runs.append({"f64": q.qcdw_op_hop_form(op, "f64"), "bf16": q.qcdw_op_hop_form(op, "bf16")})
        for prec in ("f64", "bf16"):
            for _ in range(3):
                q.qcdw_op_matpc(op, prec, xe, out)
        torch.cuda.synchronize()
        op.close()
        ctx.close()
    print(json.dumps({"matpc_only": list(L), "copy_bytes": 2 * src.numel() * 8, "forms": runs}))


def net_only(L):
    import tempfile

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
    U = torch.from_numpy(li.random_gauge(L, 0.15, 0)).cuda()
    xe = torch.from_numpy(li.gaussian_source(L, 1000).reshape(-1, 4, 3)[:Vh].copy()).cuda()
    out = torch.empty_like(xe)
    runs = []
    for mfma in (0, 3):  # a fresh context reads the tuning file that fixes the layer kinds (3: both on MFMA)
        path = os.path.join(tempfile.gettempdir(), f"qcdw_net_mfma_{mfma}.txt")
        with open(path, "w") as fh:
            fh.write(f"net_mfma/h12/L{L[0]}x{L[1]}x{L[2]}x{L[3]} {mfma}\n")
        os.environ["QCDW_TUNE_CACHE"] = path
        ctx = q.Context(0)
        op = q.Operator(ctx, q.make_lattice(L), U, 0.12781, 1.0, "bf16", 12)
        net = q.Net(op, 12, seed=5, init_scale=0.01)
        ms = {}
        for prec in ("f32", "bf16"):
            q.qcdw_net_apply(net, prec, xe, out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                q.qcdw_net_apply(net, prec, xe, out)
            torch.cuda.synchronize()
            ms[prec] = round((time.perf_counter() - t0) / 3 * 1e3, 3)
        runs.append({"mfma": mfma, "apply_ms": ms})
        net.close()
        op.close()
        ctx.close()
    print(json.dumps({"net_only": list(L), "copy_bytes": 2 * src.numel() * 8, "runs": runs}))


# multigrid of the learned section at 32^3x64: 8^4 aggregates (a 4^3x8 coarse lattice), 12 near-null vectors
# from 120 BF16 relaxation iterations each, at most 40 coarse BiCGStab iterations, 4 smoothing steps, inside
# FGMRES(12)
MG_PARAMS = dict(block=(8, 8, 8, 8), nvec=12, setup_iters=120, coarse_iters=40, smooth_iters=4)
MG_RESTART = 12


def mg_only():
    import torch

    import lattice_inputs as li
    import paper_2411_08461_amd as q

    w = li.WORKLOADS["wc32x64"]
    L = w["L"]
    U = li.random_gauge(L, w["eps"], w["seed"])
    b = torch.from_numpy(li.gaussian_source(L, w["source_seed"])).cuda()
    ctx = q.Context(0)
    op = q.Operator(ctx, q.make_lattice(L), torch.from_numpy(U).cuda(), w["kappa"], w["csw"], "bf16", 12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mg = q.Multigrid(op, q.make_mg_params(**MG_PARAMS))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    x = torch.zeros_like(b)
    t0 = time.perf_counter()
    info = q.qcdw_invert_mg(op, mg, b, x, q.make_params(tol=1e-10, maxiter=4000, gmres_restart=MG_RESTART))
    torch.cuda.synchronize()
    print(json.dumps({"mg_only": list(L), "params": MG_PARAMS, "restart": MG_RESTART, "setup_ms": round(1e3 * t_setup, 1),
                      "status": info.status_name, "iters": info.iters, "true_res": info.true_res,
                      "time_ms": round(1e3 * (time.perf_counter() - t0), 1)}))
    mg.close()
    op.close()
    ctx.close()


def main():
    args = parse()
    if args.net_only:
        net_only([int(v) for v in args.net_only.split(",")])
        return
    if args.mg_only:
        mg_only()
        return
    if args.matpc_only:
        forms = [tuple(int(x) for x in f.split(":")) for f in args.forms.split(",") if f]
        mrhs = [int(v) for v in args.mrhs_forms.split(",") if v]
        matpc_only([int(v) for v in args.matpc_only.split(",")], forms, mrhs)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the multi-GPU "
              "decomposition is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import lattice_inputs as li
    import paper_2411_08461_amd as q

    if args.bisect_kappa:
        print(json.dumps(bisect_kappa(q, li, np, torch)))
        return
    sections = [v for v in args.sections.split(",") if v]
    for sec in sections:
        if sec not in SECTIONS:
            raise SystemExit(f"unknown section {sec}; choose from {', '.join(SECTIONS)}")

    # every host input is drawn before the GPU is initialised (the field generator forks workers);
    # a field that several sections use is drawn once
    w = li.WORKLOADS["wc24x64"]
    L, kappa, csw = w["L"], w["kappa"], w["csw"]
    Vh = int(np.prod(L)) // 2
    w16 = li.WORKLOADS["wc16x32"]
    jobs = {"main": [(tuple(L), w["eps"], w["seed"])], "cache16": [(tuple(w16["L"]), w16["eps"], w16["seed"])]}
    for sec in sections:
        jobs[sec] = [(tuple(j[0]), j[1], j[2]) for j in SECTIONS[sec][0](li)]
    uniq = list(dict.fromkeys(j for js in jobs.values() for j in js))
    t_gen = time.perf_counter()
    by_job = dict(zip(uniq, li.random_gauges(uniq)))
    t_gen = time.perf_counter() - t_gen
    host_fields = {name: [by_job[j] for j in js] for name, js in jobs.items()}
    del by_job
    U = host_fields["main"][0]
    b = li.point_source(L, 0, 0)

    ctx = q.Context(0)
    lat = q.make_lattice(L)
    Ud = torch.from_numpy(U).cuda()
    bd = torch.from_numpy(b).cuda()
    x64 = torch.zeros_like(bd)
    xlo = torch.zeros_like(bd)
    torch.cuda.synchronize()

    # every hop dispatch of the solves records HIP events on the library's stream (the solves then
    # launch eagerly; at this size a launch is ~0.2 ms of work, so the graphs' saving is negligible)
    delta = 0.1 if args.inner != "f16" else 0.2
    p64 = q.make_params(tol=1e-10, maxiter=20000, inner="f64", collect_timing=True)
    plo = q.make_params(tol=1e-10, maxiter=20000, inner=args.inner, delta=delta, collect_timing=True)

    def step():
        op = q.Operator(ctx, lat, Ud, kappa, csw, args.inner, 12)
        x64.zero_()
        xlo.zero_()
        i64 = q.qcdw_invert(op, bd, x64, p64, raise_on_error=True)
        ilo = q.qcdw_invert(op, bd, xlo, plo, raise_on_error=True)
        form = q.qcdw_op_hop_form(op, "f64")
        op.close()
        return i64, ilo, form

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    forms = {f for _, _, f in infos}
    form = infos[-1][2]
    ms_a = sum(i64.hop_ms[0] for i64, _, _ in infos)
    n_a = sum(i64.n_hop[0] for i64, _, _ in infos)
    avg_a_ms = ms_a / max(n_a, 1)
    achieved = hop_a_bytes("f64") * Vh / (avg_a_ms * 1e-3) / 1e9
    ms_b = sum(i64.hop_ms[1] + i64.hop_ms[2] for i64, _, _ in infos)
    n_b = sum(i64.n_hop[1] + i64.n_hop[2] for i64, _, _ in infos)
    ms_alo = sum(ilo.hop_ms[0] for _, ilo, _ in infos)
    n_alo = sum(ilo.n_hop[0] for _, ilo, _ in infos)
    lo_gbs = hop_a_bytes(args.inner) * Vh / (ms_alo / max(n_alo, 1) * 1e-3) / 1e9
    krylov_bytes = sum(i64.iters * iter_bytes("f64") * Vh + ilo.iters * iter_bytes(args.inner) * Vh
                       for i64, ilo, _ in infos)
    i64, ilo, _ = infos[-1]
    host_x = {"wc24x64": {"f64": x64.cpu().numpy(), args.inner: xlo.cpu().numpy()}}

    result = {
        "metric": "dslash GB/s (% HBM peak); time to 1e-10 residual, plain FP64 vs mixed/ML",
        "value": round(achieved, 1),
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
        "config": {"workload": "wilson-clover dslash (FP64 hop into odd sites with A_oo^-1) inside even-odd "
                               "BiCGStab, 24^3x64, kappa 0.125, csw 1.1, eps 0.2, point source",
                   "lattice": list(L), "kappa": kappa, "csw": csw, "tol": 1e-10, "inner": args.inner},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(form, L),
                     "kernel": hop_kernel_name(form), "form": {"nt": form[0], "cgroup": form[1], "fma": form[2]},
                     "forms_in_timed_steps": len(forms),
                     "launches_timed": n_a, "bytes_per_launch": hop_a_bytes("f64") * Vh,
                     "avg_launch_us": round(avg_a_ms * 1e3, 2)},
        "solve": {
            "f64": {"iters": i64.iters, "true_res": i64.true_res, "time_ms": round(i64.time_ms, 3),
                    "reliable": i64.n_reliable},
            args.inner: {"iters": ilo.iters, "true_res": ilo.true_res, "time_ms": round(ilo.time_ms, 3),
                         "reliable": ilo.n_reliable, "fallback": ilo.fallback},
            "speedup_mixed": round(i64.time_ms / ilo.time_ms, 3),
            "krylov_gbs_step": round(krylov_bytes / elapsed / 1e9, 1),
            "note": "solves launched eagerly with per-dispatch HIP events; step includes operator set-up",
        },
        "hop_gbs": {"f64_into_odd": round(achieved, 1),
                    "f64_into_even_xpay": round((hop_b_bytes("f64") + SPINOR["f64"] / 2) * Vh /
                                                (ms_b / max(n_b, 1) * 1e-3) / 1e9, 1),
                    f"{args.inner}_into_odd": round(lo_gbs, 1)},
    }
    del Ud, bd, x64, xlo
    torch.cuda.empty_cache()

    result["stream_gbs"] = stream_probe(torch)
    cres, host_x["wc16x32"] = cache_resident(q, li, np, torch, ctx, host_fields["cache16"][0], args)
    result["wc16x32_cache_resident"] = cres
    if args.extra_lattice:
        result["hop_gbs_large"] = time_large_hop(q, li, np, torch, ctx, [int(v) for v in args.extra_lattice.split(",")])

    for sec in sections:
        result[sec] = SECTIONS[sec][1](q, li, np, torch, ctx, host_fields.pop(sec), args)
        host_fields[sec] = None
    result["input_generation_s"] = round(t_gen, 1)
    torch.cuda.synchronize()
    ctx.close()

    if not args.no_cpu_baseline:
        result["cpu_baseline"], result["solve_vs_oracle"] = cpu_baseline(
            li, np, (L, U, b, kappa, csw), (w16, host_fields["cache16"][0]), host_x, args.cpu_seconds)

    print(json.dumps(result))
    sys.stdout.flush()


def cache_resident(q, li, np, torch, ctx, U, args):
    """The 16^3x32 Z2-source system (kappa 0.124, csw 1.0): FP64 and mixed solves launched through the
    captured hipGraphs, and the FP64 hop rate from an instrumented solve.  The hop's working set
    (~113 MB) fits the 256 MB memory-side cache, so these are not HBM figures."""
    w = li.WORKLOADS["wc16x32"]
    L, kappa, csw = w["L"], w["kappa"], w["csw"]
    Vh = int(np.prod(L)) // 2
    lat = q.make_lattice(L)
    bd = torch.from_numpy(li.z2_source(L, w["source_seed"])).cuda()
    op = q.Operator(ctx, lat, torch.from_numpy(U).cuda(), kappa, csw, args.inner, 12)
    delta = 0.1 if args.inner != "f16" else 0.2
    out = {"workload": "16^3x32, kappa 0.124, csw 1.0, eps 0.2, Z2 source (cache-resident: not an HBM figure)"}
    xs = {}
    for prec in ("f64", args.inner):
        prm = q.make_params(tol=1e-10, maxiter=20000, inner=prec, delta=delta, use_graph=not args.eager)
        x = torch.zeros_like(bd)
        q.qcdw_invert(op, bd, x, prm)  # warm-up: graph capture
        ts = []
        for _ in range(3):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = q.qcdw_invert(op, bd, x, prm, raise_on_error=True)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t = sorted(ts)[1]
        out[prec] = {"iters": info.iters, "true_res": info.true_res, "time_ms": round(1e3 * t, 3),
                     "krylov_gbs": round(info.iters * iter_bytes(prec) * Vh / t / 1e9, 1)}
        xs[prec] = x.cpu().numpy()
    out["speedup_mixed"] = round(out["f64"]["time_ms"] / out[args.inner]["time_ms"], 3)
    x = torch.zeros_like(bd)
    info = q.qcdw_invert(op, bd, x, q.make_params(tol=1e-10, maxiter=20000, inner="f64", collect_timing=True))
    us = 1e3 * info.hop_ms[0] / max(info.n_hop[0], 1)
    out["hop_f64"] = {"gbs": round(hop_a_bytes("f64") * Vh / us / 1e3, 1), "avg_launch_us": round(us, 2),
                      "form": q.qcdw_op_hop_form(op, "f64")}
    op.close()
    del bd, x
    torch.cuda.empty_cache()
    return out, xs


def hop_kernel_name(form):
    nt, cg, fma = form
    f = "true" if fma else "false"
    if nt == 1:
        name = f"hop_kernel<P64, r12, EPI_CLOV, RED_NONE, {f}>"
    else:
        name = f"hop_tkernel<P64, r12, EPI_CLOV, RED_NONE, {nt}, {f}>"
    return name + (f" (slice groups of {cg} c-tiles)" if cg else "")


KERNEL_SOURCES = ("paper_2411_08461_amd/csrc/hop.hip", "paper_2411_08461_amd/csrc/hop_common.h",
                  "paper_2411_08461_amd/csrc/dev.h", "paper_2411_08461_amd/csrc/internal.h")
TRAFFIC_FILES = {(16, 16, 16, 32): os.path.join(ROOT, "profiles", "hop_wc16x32_traffic.md"),
                 (24, 24, 24, 64): os.path.join(ROOT, "profiles", "hop_wc24x64_traffic.md")}


def kernel_sources_sha256():
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(form, L):
    """HBM bytes per launch of the dominant kernel from the committed FETCH_SIZE / WRITE_SIZE
    profile of this lattice: the record taken from the current kernel sources with the same hop
    form, if there is one; otherwise None."""
    path = TRAFFIC_FILES.get(tuple(L))
    if path is None:
        return None
    try:
        with open(path) as f:
            recs = [json.loads(ln[len("traffic-json: "):]) for ln in f if ln.startswith("traffic-json: ")]
    except (OSError, ValueError):
        return None
    sha = kernel_sources_sha256()
    for rec in recs:
        if rec.get("sources_sha256") == sha and [rec.get("nt"), rec.get("cgroup"), rec.get("fma")] == list(form):
            return int(rec["read_bytes"] + rec["write_bytes"])
    return None


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


def _solve_summary(infos):
    return {"iters_max": max(i.iters for i in infos), "iters_sum": sum(i.iters for i in infos),
            "max_true_res": max(i.true_res for i in infos),
            "all_ok": all(i.status == 0 for i in infos)}


def propagator_jobs(li):
    w = li.WORKLOADS["wc24x64"]
    return [(w["L"], w["eps"], w["seed"])]


def propagator(q, li, np, torch, ctx, fields, args):
    """12 point sources (all spins and colours) at 24^3x64: one lockstep multi-RHS solve with BF16
    storage against 12 separate FP64 solves; both to an FP64 true residual of 1e-10."""
    w = li.WORKLOADS["wc24x64"]
    L, kappa, csw = w["L"], w["kappa"], w["csw"]
    Vh = int(np.prod(L)) // 2
    Ud = torch.from_numpy(fields[0]).cuda()
    bs = torch.zeros((12,) + li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    for s in range(4):
        for c in range(3):
            bs[3 * s + c][0, 0, 0, 0, 0, s, c] = 1.0
    op = q.Operator(ctx, q.make_lattice(L), Ud, kappa, csw, "bf16", 12)
    del Ud
    torch.cuda.empty_cache()
    x = torch.zeros_like(bs)
    pm = q.make_params(tol=1e-10, maxiter=20000, inner="bf16", delta=0.1)
    q.qcdw_invert_multi(op, bs, x, pm)  # warm-up: autotuner choice and graph capture
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    multi = q.qcdw_invert_multi(op, bs, x, pm)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - t0
    p64 = q.make_params(tol=1e-10, maxiter=20000, inner="f64")
    x64 = torch.zeros_like(bs)
    q.qcdw_invert(op, bs[0], x64[0], p64)  # warm-up
    x64.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sep = [q.qcdw_invert(op, bs[k], x64[k], p64) for k in range(12)]
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t0
    diff = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
    # 12 separate BF16-mixed solves: what the lockstep multi-RHS solve saves over the same precision
    plo = q.make_params(tol=1e-10, maxiter=20000, inner="bf16", delta=0.1)
    xlo = torch.zeros_like(bs)
    q.qcdw_invert(op, bs[0], xlo[0], plo)  # warm-up
    xlo.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sep_lo = [q.qcdw_invert(op, bs[k], xlo[k], plo) for k in range(12)]
    torch.cuda.synchronize()
    t_sep_lo = time.perf_counter() - t0
    del xlo
    # the contraction after the solves: pion two-point function of the propagator (reads the 12 fields once)
    lat = q.make_lattice(L)
    corr = torch.empty(L[3], dtype=torch.complex128, device="cuda")
    q.qcdw_meson_2pt(ctx, lat, x, 15, 15, (0, 0, 0), corr)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        q.qcdw_meson_2pt(ctx, lat, x, 15, 15, (0, 0, 0), corr)
    torch.cuda.synchronize()
    t_con = (time.perf_counter() - t0) / 5
    pion = corr.cpu().numpy()
    # the same trace through the two-propagator (three-point) kernel with a copy as the backward leg: it
    # reads twice the bytes and must give the pion bit for bit (same per-site arithmetic and order)
    x2 = x.clone()
    corr2 = torch.empty_like(corr)
    q.qcdw_meson_contract(ctx, lat, x, x2, 15, 15, (0, 0, 0), corr2)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        q.qcdw_meson_contract(ctx, lat, x, x2, 15, 15, (0, 0, 0), corr2)
    torch.cuda.synchronize()
    t_con2 = (time.perf_counter() - t0) / 5
    same2 = bool(np.array_equal(corr2.cpu().numpy(), pion))
    del x2
    # hop bandwidth of the multi-RHS kernel: a capped solve with every hop dispatch timed
    pt = q.make_params(tol=1e-10, maxiter=16, inner="bf16", collect_timing=True, check_every=8)
    xt = torch.zeros_like(bs)
    ti = q.qcdw_invert_multi(op, bs, xt, pt)[0]
    ms = ti.hop_ms[0] / max(ti.n_hop[0], 1)
    gbs = hop_a_bytes_multi("bf16", 12) * Vh / (ms * 1e-3) / 1e9
    form = q.qcdw_ctx_tuned(ctx, f"mrhs_hop/p{q.QCDW_BF16}/L{L[0]}x{L[1]}x{L[2]}x{L[3]}/n12")
    op.close()
    del bs, x, x64, xt
    torch.cuda.empty_cache()
    return {"workload": "24^3x64, kappa 0.125, csw 1.1, eps 0.2, 12 point sources",
            "multi_bf16": dict(_solve_summary(multi), time_ms=round(1e3 * t_multi, 1)),
            "separate_f64": dict(_solve_summary(sep), time_ms=round(1e3 * t_sep, 1)),
            "separate_bf16": dict(_solve_summary(sep_lo), time_ms=round(1e3 * t_sep_lo, 1)),
            "speedup": round(t_sep / t_multi, 3), "speedup_vs_separate_bf16": round(t_sep_lo / t_multi, 3),
            "rel_diff_multi_vs_f64": diff,
            "multi_hop": {"gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                          "avg_launch_us": round(ms * 1e3, 1), "bytes_per_site_12rhs": hop_a_bytes_multi("bf16", 12),
                          "form": form, "matrix_cores": bool(form is not None and form & 1024)},
            "pion_2pt": {"call_ms": round(1e3 * t_con, 3),
                         "gbs_incl_call": round(12 * 192 * 2 * Vh / t_con / 1e9, 1),
                         "c_t0": float(pion[0].real), "c_t_mid": float(pion[L[3] // 2].real),
                         "positive": bool((pion.real > 0).all())},
            "two_propagator_contract": {"call_ms": round(1e3 * t_con2, 3),
                                        "gbs_incl_call": round(2 * 12 * 192 * 2 * Vh / t_con2 / 1e9, 1),
                                        "equals_pion": same2}}


def batch_jobs(li):
    return [(p["L"], p["eps"], p["seed"]) for p in li.batch48()]


def batch(q, li, np, torch, ctx, fields, args):
    """48 uneven problems: one persistent batched solve against a loop of single solves (solves/s)."""
    specs = li.batch48()
    ops, bs = [], []
    for p, U in zip(specs, fields):
        ops.append(q.Operator(ctx, q.make_lattice(p["L"]), torch.from_numpy(U).cuda(), p["kappa"], p["csw"],
                              "bf16", 12))
        bs.append(torch.from_numpy(li.gaussian_source(p["L"], p["source_seed"])).cuda())
    xs = [torch.zeros_like(t) for t in bs]
    bt = q.Batch(ctx, ops)
    out = {"workload": "48 problems: 16 each of 8^3x16, 12^3x24, 16^3x32; kappa in [0.115, 0.124], eps 0.25"}
    for prec in ("f64", "bf16"):
        prm = q.make_params(tol=1e-10, maxiter=20000, inner=prec, delta=0.1)
        q.qcdw_invert_batch(bt, bs, xs, prm)  # warm-up: autotuner and graph capture
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = q.qcdw_invert_batch(bt, bs, xs, prm)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        for x in xs:
            x.zero_()
        q.qcdw_invert(ops[0], bs[0], xs[0], prm)
        xs[0].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        single = [q.qcdw_invert(op, bb, xx, prm) for op, bb, xx in zip(ops, bs, xs)]
        torch.cuda.synchronize()
        t_s = time.perf_counter() - t0
        out[prec] = {"batched": dict(_solve_summary(infos), time_ms=round(1e3 * t_b, 1),
                                     solves_per_s=round(48 / t_b, 1)),
                     "sequential": dict(_solve_summary(single), time_ms=round(1e3 * t_s, 1),
                                        solves_per_s=round(48 / t_s, 1)),
                     "speedup": round(t_s / t_b, 3)}
    bt.close()
    for op in ops:
        op.close()
    del bs, xs
    torch.cuda.empty_cache()
    return out


LEARNED_TRAIN_SEEDS = range(1, 9)
LEARNED_STRIDE = 20  # training pairs: errors of BiCGStab iterates restarted every 20 iterations


def learned_jobs(li):
    w = li.WORKLOADS["wc32x64"]
    if w["kappa"] is None:
        return []
    return [(w["L"], w["eps"], s) for s in [w["seed"], *LEARNED_TRAIN_SEEDS]]


def learned(q, li, np, torch, ctx, fields, args):
    """32^3x64 near the critical kappa: train the gauge-covariant net on 8 other fields of the ensemble
    (32 solver-generated pairs each: the errors of BiCGStab iterates against an FP64 solution of a Gaussian
    source of that field, 256 in all), then FGMRES(32)+net against plain FP64 and mixed BiCGStab
    and FGMRES(32) without the net, all to an FP64 true residual of 1e-10 from the Gaussian source."""
    w = li.WORKLOADS["wc32x64"]
    if w["kappa"] is None:
        return {"skipped": "kappa not set; run bench.py --bisect-kappa"}
    L, kappa, csw = w["L"], w["kappa"], w["csw"]
    lat = q.make_lattice(L)
    out = {"workload": f"32^3x64, kappa {kappa} (bisected), csw 1.0, eps 0.15, Gaussian source"}
    # training on fields 1..8
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net, losses, prev = None, [], None
    for k, U in zip(LEARNED_TRAIN_SEEDS, fields[1:]):
        op = q.Operator(ctx, lat, torch.from_numpy(U).cuda(), kappa, csw, "bf16", 12)
        if net is None:
            net = q.Net(op, 12, seed=5, init_scale=0.01)
        else:
            q.qcdw_net_bind(net, op)
        if prev is not None:
            prev.close()
        prev = op
        src = torch.from_numpy(li.gaussian_source(L, w["source_seed"] + k)).cuda()
        r, e = q.qcdw_make_training_pairs(op, src, 32, LEARNED_STRIDE)
        h = q.qcdw_net_train(net, r, e, steps=60, batch=4, lr=2e-3, seed=k)
        losses.append((float(np.mean(h[:4])), float(np.mean(h[-4:]))))
        del r, e, src
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    op = q.Operator(ctx, lat, torch.from_numpy(fields[0]).cuda(), kappa, csw, "bf16", 12)
    q.qcdw_net_bind(net, op)
    prev.close()
    torch.cuda.empty_cache()
    b = torch.from_numpy(li.gaussian_source(L, w["source_seed"])).cuda()
    # hop bandwidth on this lattice (the largest of the workloads): a capped solve, every hop timed
    Vh = int(np.prod(L)) // 2
    out["hop_gbs"] = {"lattice": list(L)}
    for prec in ("f64", "bf16"):
        xt = torch.zeros_like(b)
        ti = q.qcdw_invert(op, b, xt, q.make_params(tol=1e-10, maxiter=24, inner=prec, collect_timing=True,
                                                    check_every=8))
        ms = ti.hop_ms[0] / max(ti.n_hop[0], 1)
        gbs = hop_a_bytes(prec) * Vh / (ms * 1e-3) / 1e9
        out["hop_gbs"][prec] = {"gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                "avg_launch_us": round(ms * 1e3, 1), "form": q.qcdw_op_hop_form(op, prec)}
    del xt
    out["training"] = {"fields": len(losses), "pairs": 32 * len(losses), "steps": 60 * len(losses),
                       "pairs_from": f"BiCGStab iterates restarted every {LEARNED_STRIDE} iterations",
                       "time_s": round(t_train, 2), "loss_first_field": [round(v, 4) for v in losses[0]],
                       "loss_last_field": [round(v, 4) for v in losses[-1]]}
    runs = {
        "bicgstab_f64": lambda x: q.qcdw_invert(op, b, x, q.make_params(tol=1e-10, maxiter=40000, inner="f64")),
        "bicgstab_bf16": lambda x: q.qcdw_invert(op, b, x, q.make_params(tol=1e-10, maxiter=40000, inner="bf16")),
        "fgmres32_net": lambda x: q.qcdw_invert_fgmres(op, net, b, x, q.make_params(tol=1e-10, maxiter=12000,
                                                                                      inner="bf16")),
        "fgmres32_plain": lambda x: q.qcdw_invert_fgmres(op, None, b, x, q.make_params(tol=1e-10, maxiter=12000,
                                                                                         inner="bf16")),
    }
    for name, fn in runs.items():
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = fn(x)
        torch.cuda.synchronize()
        out[name] = {"status": info.status_name, "iters": info.iters, "true_res": info.true_res,
                     "time_ms": round(1e3 * (time.perf_counter() - t0), 1)}
        if name.startswith("fgmres"):
            out[name].update(fallback=info.fallback, fallback_iters=info.fallback_iters, cycles=info.n_restarts)
        print(f"[learned] {name}: {out[name]}", file=sys.stderr, flush=True)
    out["speedup_net_vs_f64"] = round(out["bicgstab_f64"]["time_ms"] / out["fgmres32_net"]["time_ms"], 3)
    # the paper's accelerator for clover solves: two-level aggregation multigrid (MG_PARAMS: aggregates,
    # near-null vectors relaxed by BF16 iterations), set up on this operator, then FGMRES(32) with it
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mg = q.Multigrid(op, q.make_mg_params(**MG_PARAMS))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = q.qcdw_invert_mg(op, mg, b, x, q.make_params(tol=1e-10, maxiter=4000, gmres_restart=MG_RESTART))
    torch.cuda.synchronize()
    out["fgmres_mg"] = {"status": info.status_name, "iters": info.iters, "true_res": info.true_res,
                          "time_ms": round(1e3 * (time.perf_counter() - t0), 1), "setup_ms": round(1e3 * t_setup, 1),
                          "fallback": info.fallback, "params": MG_PARAMS, "restart": MG_RESTART}
    print(f"[learned] fgmres_mg: {out['fgmres_mg']}", file=sys.stderr, flush=True)
    out["speedup_mg_vs_f64"] = round(out["bicgstab_f64"]["time_ms"] / out["fgmres_mg"]["time_ms"], 3)
    out["speedup_mg_with_setup_vs_f64"] = round(out["bicgstab_f64"]["time_ms"] /
                                                (out["fgmres_mg"]["time_ms"] + out["fgmres_mg"]["setup_ms"]), 3)
    mg.close()
    del x
    net.close()
    op.close()
    del b
    torch.cuda.empty_cache()
    return out


ANISO_ACTION = {"xi_0": 2.464, "nu": 0.95, "m_0": 0.3, "csw_t": 0.91, "csw_r": 1.07}  # the paper's example


def aniso_jobs(li):
    return [((16, 16, 16, 32), 0.2, 7)]


def aniso(q, li, np, torch, ctx, fields, args):
    """The anisotropic clover action of the paper's example (Sec. III.B) on 16^3x32 with antiperiodic t:
    FP64 and BF16-mixed solves (graphs on, timed), and the FP64 hop bandwidth from an instrumented solve."""
    a = ANISO_ACTION
    L = (16, 16, 16, 32)
    Vh = int(np.prod(L)) // 2
    kappa = 1.0 / (2.0 * (a["m_0"] + 1.0 + 3.0 * a["nu"] / a["xi_0"]))
    op = q.Operator(ctx, q.make_lattice(L, -1), torch.from_numpy(fields[0]).cuda(), kappa, 0.0, "bf16", 12,
                    aniso=(a["xi_0"], a["nu"], a["csw_t"], a["csw_r"]))
    b = torch.from_numpy(li.gaussian_source(L, 1007)).cuda()
    x = torch.zeros_like(b)
    out = {"workload": "16^3x32, antiperiodic t, xi_0 2.464, nu 0.95, m_0 0.3, csw_t 0.91, csw_r 1.07, eps 0.2, "
                       "Gaussian source", "kappa": round(kappa, 6)}
    for prec in ("f64", "bf16"):
        prm = q.make_params(tol=1e-10, maxiter=20000, inner=prec, delta=0.1)
        q.qcdw_invert(op, b, x, prm)  # warm-up: graph capture
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = q.qcdw_invert(op, b, x, prm)
        torch.cuda.synchronize()
        out[prec] = dict(_solve_summary([info]), time_ms=round(1e3 * (time.perf_counter() - t0), 3))
        x.zero_()
    info = q.qcdw_invert(op, b, x, q.make_params(tol=1e-10, maxiter=20000, inner="f64", collect_timing=True))
    us = 1e3 * info.hop_ms[0] / max(info.n_hop[0], 1)
    out["hop_f64"] = {"gbs": round(hop_a_bytes("f64") * Vh / us / 1e3, 1), "avg_launch_us": round(us, 2),
                      "form": q.qcdw_op_hop_form(op, "f64")}
    op.close()
    return out


def multishift_jobs(li):
    w = li.WORKLOADS["wc16x32"]
    return [(w["L"], w["eps"], w["seed"])]


def multishift(q, li, np, torch, ctx, fields, args):
    """Multi-shift CG on the normal even-odd operator (RHMC's rational-approximation solves) at 16^3x32:
    8 shifts spread over four decades, FP64, one Krylov space against 8 separate single-shift solves."""
    w = li.WORKLOADS["wc16x32"]
    L = w["L"]
    Vh = int(np.prod(L)) // 2
    op = q.Operator(ctx, q.make_lattice(L), torch.from_numpy(fields[0]).cuda(), w["kappa"], w["csw"])
    b = torch.from_numpy(li.gaussian_source(L, 1009).reshape(-1, 4, 3)[:Vh].copy()).cuda()
    shifts = [1e-4 * 4 ** k for k in range(8)]
    xs = [torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda") for _ in shifts]
    q.qcdw_invert_multishift(op, b, xs, shifts)  # warm-up
    torch.cuda.synchronize()
    reps = 3  # mean over a few calls of each
    t0 = time.perf_counter()
    for _ in range(reps):
        it, res = q.qcdw_invert_multishift(op, b, xs, shifts)
    torch.cuda.synchronize()
    t_ms = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        its1 = [q.qcdw_invert_multishift(op, b, [xs[k]], [shifts[k]])[0] for k in range(len(shifts))]
    torch.cuda.synchronize()
    t_sep = (time.perf_counter() - t0) / reps
    op.close()
    return {"workload": "16^3x32, kappa 0.124, csw 1.0, eps 0.2, Gaussian even-site source, shifts 1e-4 * 4^k, k < 8",
            "multishift": {"iters": it, "max_res": max(res), "time_ms": round(1e3 * t_ms, 2)},
            "separate": {"iters_sum": sum(its1), "time_ms": round(1e3 * t_sep, 2)},
            "speedup": round(t_sep / t_ms, 3), "calls_averaged": reps}


SECTIONS = {"propagator": (propagator_jobs, propagator), "batch": (batch_jobs, batch),
            "learned": (learned_jobs, learned), "aniso": (aniso_jobs, aniso),
            "multishift": (multishift_jobs, multishift)}


def bisect_kappa(q, li, np, torch):
    """Smallest kappa on a 1e-5 grid in [0.120, 0.135] at which FP64 even-odd BiCGStab on the 32^3x64
    field (eps 0.15, seed 0, Gaussian source seed 1000) does not converge to 1e-10 within 2000
    iterations (counting divergence and breakdown as 'too far'); then the converged iteration count
    there with maxiter 20000."""
    w = li.WORKLOADS["wc32x64"]
    L, csw = w["L"], w["csw"]
    U = li.random_gauge(L, w["eps"], w["seed"])
    b = torch.from_numpy(li.gaussian_source(L, w["source_seed"])).cuda()
    Ud = torch.from_numpy(U).cuda()
    del U
    ctx = q.Context(0)
    lat = q.make_lattice(L)
    lo, hi = 12000, 13500  # kappa in units of 1e-5
    trail = []

    def run(kap, maxiter):
        op = q.Operator(ctx, lat, Ud, kap * 1e-5, csw, "bf16", 12)
        x = torch.zeros_like(b)
        info = q.qcdw_invert(op, b, x, q.make_params(tol=1e-10, maxiter=maxiter, inner="f64"))
        op.close()
        trail.append((kap * 1e-5, info.status_name, info.iters))
        print(f"[bisect] kappa {kap * 1e-5:.5f}: {info.status_name} after {info.iters}", file=sys.stderr, flush=True)
        return info

    while hi - lo > 1:
        mid = (lo + hi) // 2
        info = run(mid, 2000)
        if info.status == 0 and info.iters < 2000:
            lo = mid
        else:
            hi = mid
    final = run(hi, 20000)
    ctx.close()
    return {"kappa": hi * 1e-5, "status": final.status_name, "iters": final.iters, "true_res": final.true_res,
            "trail": trail}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(li, np, main, small, host_x, seconds):
    """The FP64 oracle on the host cores: (1) its full operator M on the benchmark's 24^3x64 lattice, all
    threads (the line's value, in the GPU hop's byte model), and on one core; (2) its FP64 BiCGStab solve
    of the 16^3x32 Z2-source system to 1e-10 (full lattice, no even-odd).  Also returns each GPU solve's
    error against the oracle: the oracle's true residual of the 24^3x64 solutions, and the distance of
    the 16^3x32 solutions from the oracle's own solution."""
    import oracle

    L, U, b, kappa, csw = main
    threads = oracle.num_threads()
    V = int(np.prod(L))
    t0 = time.perf_counter()
    C = oracle.clover_build(L, U)
    t_clover = time.perf_counter() - t0
    oracle.dirac(L, U, C, b, kappa, csw)  # warm-up
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.dirac(L, U, C, b, kappa, csw)
        n += 1
        if time.perf_counter() - t0 > seconds or n >= 500:
            break
    dt = (time.perf_counter() - t0) / n
    # same byte model as the GPU hop with clover, FP64 reconstruct-12, per site of the full lattice
    gbs = hop_a_bytes("f64") * V / dt / 1e9
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.dirac(L, U, C, b, kappa, csw)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    vs = {"wc24x64": {}}
    bn = np.linalg.norm(b)
    for prec, x in host_x["wc24x64"].items():
        vs["wc24x64"][prec] = {"oracle_true_res": float(np.linalg.norm(b - oracle.dirac(L, U, C, x, kappa, csw)) / bn)}
    del C
    w16, U16 = small
    L16 = w16["L"]
    b16 = li.z2_source(L16, w16["source_seed"])
    C16 = oracle.clover_build(L16, U16)
    t0 = time.perf_counter()
    sol = oracle.bicgstab(L16, U16, C16, b16, w16["kappa"], w16["csw"], tol=1e-10, maxiter=20000)
    t_solve = time.perf_counter() - t0
    xo = sol.x
    vs["wc16x32"] = {"oracle": {"status": sol.status, "iters": sol.iters}}
    for prec, x in host_x["wc16x32"].items():
        vs["wc16x32"][prec] = {
            "rel_err_vs_oracle_x": float(np.linalg.norm(x - xo) / np.linalg.norm(xo)),
            "oracle_true_res": float(np.linalg.norm(b16 - oracle.dirac(L16, U16, C16, x, w16["kappa"], w16["csw"]))
                                     / np.linalg.norm(b16))}
    base = {"value": round(gbs, 2), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n} full-lattice applications of M (24^3x64, FP64, {threads} threads) in {n * dt:.1f} s, "
                      f"{dt * 1e3:.1f} ms each; bytes counted with the GPU hop byte model (1728 B per site)",
            "one_core": {"apply_ms": round(1e3 * dt1, 1), "gbs": round(hop_a_bytes("f64") * V / dt1 / 1e9, 2)},
            "clover_build_s": round(t_clover, 2),
            "solve_16x32_f64": {"time_s": round(t_solve, 2), "iters": sol.iters, "status": sol.status,
                                "note": "textbook BiCGStab on the full lattice (no even-odd), Z2 source, tol 1e-10"}}
    return base, vs


if __name__ == "__main__":
    main()
