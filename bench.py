#!/usr/bin/env python3
"""Benchmark of the BU-MBAR hot path on one MI355X.

Default (--workload all): every configuration of the metric in one run, the
K = 1000 ladder (c2) as the headline. One step = one full FP64 solve of the
ladder u_kn = beta_k E_n + lambda_k V_n (K = 1000, N = 2e6, u 16 GB stored,
BU-MBAR on (E, V) bins, Newton finisher, tolerance 1e-7 kT) with u resident
in HBM; value = K N / the average duration of its unbinned sweep kernel (the
sample-major single pass, HIP events on the library's stream over the timed
solves); roofline = that kernel against 8 TB/s (8 bytes per element). The
same line carries, under "configs": c2 in mixed precision from FP32 storage,
c1 (below), c4 (the Muller-Brown grid, energies in-kernel; its FP16-core
Hessian against the FP16 peak with the algorithmic K (K + 1) N flops), c4
with N_k = 500, and c3 (the 512-problem stream served at 0.8 x its measured
saturation rate, p50/p99, against the sequential FP64 solver); every result
with its error against the oracle's certified solution in tests/golden.

--workload double_well: one step = one full solve (binning, Algorithm 1
binned stage, unbinned Newton finisher, outputs) of the umbrella-sampling
workload: 1-D double well
U(x) = (x^2 - 1)^2, K = 100 harmonic windows (kappa = 50) on [-1.5, 1.5],
N_k = 10^4 Metropolis samples each (N = 10^6), u_kn 100 x 10^6 FP64, adaptive
binning, tolerance 1e-7 kT on the final step. Inputs are resident in HBM
before the timed region.

Reported value: unbinned sweep throughput, K*N elements per second, from the
average duration of the sweep kernel (HIP events on the library's stream)
over all unbinned sweeps of the timed solves. ms_per_step is the
time-to-solve. The roofline object is the same sweep kernel (HBM-bound:
8 bytes per element read once).

With --workload stream: the batched-serving workload, a seeded stream of 512
independent harmonic / double-well problems (K uniform in [4, 256], N_k
uniform in [100, 20000]) arriving as a Poisson process; each request carries
its coordinates and bias model, and u_kn is built on the device. The served
run (mixed precision, several problems resident at once, admission by device
footprint) is compared with the plain FP64 solver taking the same stream one
problem at a time. Value: solves/s of the served run; p50/p99 latency from
arrival to result; the largest |f - f_FP64| over all problems in kT.

With --workload ladder: the temperature/alchemical ladder, K = 1000 states,
N_k = 2000 (N = 2e6), u_kn = beta_k E_n + lambda_k V_n stored as a 16 GB FP64
matrix (built on the device from E, V); BU-MBAR solved in FP64 and in mixed
precision from an FP32 copy of u (FP32 sweeps, FP64 refinement).

With --workload mb2d: the 2-D umbrella grid on the Muller-Brown surface,
K = 40 x 40 = 1600 windows (kappa = 20), N_k = 5000 (N = 8e6), FP32 (x, y)
samples; u_kn is never stored: every sweep evaluates the harmonic biases
inside the kernel. Mixed-precision BU-MBAR: the windows form a product
grid, so the binned steps and the Newton sweeps run on the factored FP64
passes and the Newton Hessian on the FP16 matrix cores from the FP32 model.
value = K N / the FP64 sweep; roofline = that Hessian (the dominant kernel).

With --workload tladder: the shape of the paper's parallel-tempering
example, K = 50 temperatures geometric over a factor of two, N_k = 2e5
(N = 1e7), u_kn = beta_k E_n with unit-variance energies at 80% neighbour
overlap, stored as a 4 GB FP64 matrix built on the device. BU-MBAR (bins on
E, model representatives, Newton finisher) against plain SCI and plain
Newton (one SCI step, then Newton) on the same GPU, each to the tolerance.

With --workload scaling: the replica-count study of the paper's synthetic
section in reduced form (one seed, own solver variants): temperature ladders
of M = 10, 30, 100, 300 states with N_k = N0, N0/M and N0/M^2 samples per
state (N0 = 1e4, 3e6, 9e8: 1e4 per state at M = 300 in all three), each
solved by BU-MBAR and plain Newton, and by plain SCI up to M = 100.

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu]
       python bench.py --workload double_well [--copy-calibration]
       python bench.py --workload stream [--n-problems 512] [--rate 100]
       python bench.py --workload ladder|mb2d|tladder|scaling [--steps 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweep-reps", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload",
                    choices=["all", "double_well", "stream", "ladder", "mb2d", "tladder",
                             "scaling"],
                    default="all")
    ap.add_argument("--n-problems", type=int, default=512)
    ap.add_argument("--seeds", type=int, default=12, help="seeds per point of the scaling study")
    ap.add_argument("--rate", type=float, default=100.0, help="stream arrivals per second")
    ap.add_argument("--max-active", type=int, default=8)
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0)
    ap.add_argument("--skip-sequential", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--configs", default="c0,c2,c1,c4,c3",
                    help="default workload: the configurations to run (c2 always runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding "
              "of the sweep is described in the design notes and not implemented.", file=sys.stderr)
        sys.exit(2)
    stream = None
    if args.workload == "stream" or (args.workload == "all" and "c3" in args.configs):
        # host-side generation runs in worker processes before this process touches the GPU
        stream = generate_stream(args)

    import torch

    import paper_2609_03541_amd as bm
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs the GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "all":
        return run_all(args, bm, synth, stream)
    if args.workload == "stream":
        return run_stream(args, bm, stream)
    if args.workload == "ladder":
        return run_ladder(args, bm, synth)
    if args.workload == "mb2d":
        return run_mb2d(args, bm, synth)
    if args.workload == "tladder":
        return run_tladder(args, bm, synth)
    if args.workload == "scaling":
        return run_scaling(args, bm, synth)
    dev = torch.device("cuda:0")
    t = time.time()
    p = synth.double_well(K=100, Nk=10000, seed=1)
    K, N = p["K"], p["N"]
    log(f"workload generated in {time.time() - t:.1f}s: K={K} N={N}")
    u = torch.tensor(p["u"], device=dev)
    Nk = torch.tensor(p["Nk"], device=dev)
    xi = torch.tensor(p["xi"], device=dev)
    coef = torch.tensor(p["coef"], device=dev)
    torch.cuda.synchronize()
    ctx = bm.context()

    def one_solve(profile):
        return bm.solve(u, Nk, xi=xi, model=bm.MODEL_HARMONIC, coef=coef, tol=args.tol,
                        profile=int(profile), ctx=ctx)

    for i in range(args.warmup):
        f, info = one_solve(False)
        log(f"warmup {i}: phase1={info['phase1_iters']} phase2={info['phase2_iters']} "
            f"checks={info['n_checks']} newton={info['finisher_steps']}")
    if args.copy_calibration:
        _copy_calibration(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweep_ms, launches = 0.0, 0
    infos = []
    for i in range(args.steps):
        f, info = one_solve(True)
        sweep_ms += info["sweep_kernel_ms"]
        launches += info["sweep_kernel_launches"]
        infos.append(info)
        log(f"step {i}: status={info['status']} binning={info['time_binning_ms']:.1f}ms "
            f"binned={info['time_binned_ms']:.1f}ms final={info['time_final_ms']:.1f}ms "
            f"sweeps={info['unbinned_sweeps']} newton={info['finisher_steps']}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    avg_sweep_s = sweep_ms / max(1, launches) / 1e3
    elems = K * N
    value = elems / avg_sweep_s if launches else None

    # dedicated sweep loop on the library stream (same kernel, back to back)
    f0 = f.clone()
    s = ctx.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    bm.sweep(u, Nk, f0, ctx=ctx, with_stats=False)
    e0.record(s)
    for _ in range(args.sweep_reps):
        bm.sweep(u, Nk, f0, ctx=ctx, with_stats=False)
    e1.record(s)
    torch.cuda.synchronize()
    loop_s = e0.elapsed_time(e1) / 1e3 / args.sweep_reps

    # accuracy: the FP64 oracle's fixed-point residual and gradient at the GPU result
    import oracle
    f_host = f.cpu().numpy()
    fn = oracle.sci_step(p["u"], p["Nk"], f_host)
    residual = float(np.max(np.abs(fn - f_host)))

    cpu = None
    if not args.no_cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        reps, tc = 0, time.perf_counter()
        while True:
            oracle.sci_step(p["u"], p["Nk"], f_host)
            reps += 1
            if time.perf_counter() - tc > args.cpu_seconds or reps >= 50:
                break
        per = (time.perf_counter() - tc) / reps
        cpu = {"value": elems / per, "unit": "elem/s", "cores": threads, "kind": "oracle",
               "sample": f"{reps} FP64 oracle unbinned SCI sweeps over the full 100 x 1e6 "
                         f"u_kn ({per:.2f} s each)"}

    achieved = 8.0 * elems / avg_sweep_s / 1e9 if launches else None
    traffic = _counter_traffic("sweep_fast_double_well_K100_N1e6")
    out = {
        "metric": "sweep K*N elem/s + time-to-solve at 1e-6 kT; batched solves/s, p50/p99",
        "value": value,
        "unit": "elem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "double-well umbrella sampling, K=100 windows, N=1e6 "
                               "(N_k=1e4), u_kn 100x1e6 FP64, adaptive binning + Newton",
                   "K": K, "N": N, "tol_kT": args.tol},
        "time_to_solve_s": ms_per_step / 1e3,
        "sweep_kernel_us": avg_sweep_s * 1e6,
        "sweep_kernel_launches": launches,
        "sweep_loop_elem_s": elems / loop_s,
        "oracle_sci_residual_kT": residual,
        "grad_norm": infos[-1]["grad_norm"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


GOLDEN = os.path.join(ROOT, "tests", "golden")
METRIC = "sweep K*N elem/s + time-to-solve at 1e-6 kT; batched solves/s, p50/p99"


def _golden(name):
    """Golden f of a workload: the oracle's certified solution (tests/golden)."""
    try:
        with open(os.path.join(GOLDEN, name + ".json")) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return None


def _err(f, gold):
    if gold is None:
        return None
    f = f.detach().cpu().numpy() if hasattr(f, "detach") else np.asarray(f)
    return float(np.max(np.abs(f - np.asarray(gold["f"]))))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _side(args, steps=3):
    """Steps and warm-up for the non-headline configurations (bounded)."""
    a = argparse.Namespace(**vars(args))
    a.steps = max(1, min(args.steps, steps))
    a.warmup = 1
    return a


def _ladder_u(torch, p):
    """u_kn = beta_k E_n + lambda_k V_n on the device (the generator's arithmetic)."""
    E = torch.tensor(p["xi"][:, 0], device="cuda")
    V = torch.tensor(p["xi"][:, 1], device="cuda")
    beta = torch.tensor(p["beta"], device="cuda")
    lam = torch.tensor(p["lam"], device="cuda")
    return beta[:, None] * E[None, :] + lam[:, None] * V[None, :]


def run_all(args, bm, synth, stream):
    """Default run: every configuration of the metric on one GPU, c2 as the headline."""
    import torch

    import oracle
    ctx = bm.context()
    side = _side(args)
    cfg = {}
    t_all = time.time()

    # ---- c2: K = 1000 ladder, N = 2e6, u stored FP64 (16 GB); the headline ----
    p = synth.ladder_2d(K=1000, Nk=2000, seed=2, materialize=False)
    K, N = p["K"], p["N"]
    xi = torch.tensor(p["xi"], device="cuda")
    coef = torch.tensor(p["coef"], device="cuda")
    Nk = torch.tensor(p["Nk"], device="cuda")
    u = _ladder_u(torch, p)
    torch.cuda.synchronize()
    g2 = _golden("c2_ladder_K1000_N2e6")

    def c2(uu, prec):
        return lambda prof: bm.solve(uu, Nk, xi=xi, model=bm.MODEL_LINEAR, coef=coef,
                                     tol=args.tol, precision=prec, profile=int(prof), ctx=ctx)

    f64, inf64, ms64 = _timed_solves(bm, args, "c2 f64", c2(u, bm.PREC_FP64))
    cov_ms = _covariance_ms(bm, u, Nk, f64, ctx)
    sw64, nsw = _avg_sweep_s(inf64)
    elems = K * N
    value = elems / sw64
    achieved = 8.0 * elems / sw64 / 1e9
    up_ms, up_gbs = _upload_solve_ms(torch, u, c2(u, bm.PREC_FP64))
    cfg["c2_f64"] = dict(time_to_solve_s=ms64 / 1e3, sweep_us=sw64 * 1e6, sweep_launches=nsw,
                         error_vs_oracle_kT=_err(f64, g2), status=inf64[-1]["status"],
                         covariance_ms=cov_ms,
                         with_upload=dict(time_to_solve_s=up_ms / 1e3, upload_gb_s=up_gbs),
                         **_stages(inf64[-1]))
    # FP32 storage (8 GB, no FP64 copy anywhere): mixed precision, and FP64
    # arithmetic on the same storage (the oracle's problem is the FP64 one,
    # so the error against it includes the rounding of u to FP32)
    u32 = u.float()
    del u
    torch.cuda.empty_cache()
    fm, infm, msm = _timed_solves(bm, side, "c2 mixed fp32 storage", c2(u32, bm.PREC_MIXED))
    f32s, inf32s, ms32s = _timed_solves(bm, side, "c2 f64 on fp32 storage",
                                        c2(u32, bm.PREC_FP64))
    swm, _ = _avg_sweep_s(infm)
    cfg["c2_mixed_fp32_storage"] = dict(
        time_to_solve_s=msm / 1e3, sweep_us=swm * 1e6, mixed_steps=infm[-1]["mixed_steps"],
        error_vs_oracle_kT=_err(fm, g2),
        error_vs_fp64_on_same_storage_kT=float((fm - f32s).abs().max()),
        storage_rounding_error_kT=_err(f32s, g2), status=infm[-1]["status"],
        speedup_vs_f64=ms64 / msm)
    del u32
    torch.cuda.empty_cache()
    log(f"c2 done ({time.time() - t_all:.0f} s)")

    want = set(args.configs.split(","))
    # ---- c0: K = 8 harmonic wells, N = 8000, FP64: latency-bound ----
    if "c0" in want:
        cfg["c0_f64"] = _c0(bm, synth, ctx, args.tol)
        log(f"c0 done ({time.time() - t_all:.0f} s)")
    # ---- c1: K = 100 double-well umbrella windows, N = 1e6, FP64 ----
    if "c1" in want:
        cfg["c1_f64"] = _c1(bm, synth, side, ctx)
        log(f"c1 done ({time.time() - t_all:.0f} s)")
    # ---- c4: 40 x 40 Muller-Brown umbrella grid, N = 8e6, energies in-kernel ----
    if "c4" in want:
        cfg["c4_mixed"] = _c4(bm, synth, side, ctx, Nk_per=5000)
        cfg["c4r_mixed_Nk500"] = _c4(bm, synth, side, ctx, Nk_per=500,
                                     gold=_golden("c4r_mullerbrown_K1600_N8e5"), hessian=False)
        log(f"c4 done ({time.time() - t_all:.0f} s)")
    # ---- c3: 512-problem stream at 0.8 x the measured saturation rate ----
    if "c3" in want:
        cfg["c3_serving"] = _c3(bm, side, stream)
        log(f"c3 done ({time.time() - t_all:.0f} s)")
    # ---- the FP64 oracle on this host: per-sweep rate on a bounded sample ----
    cpu = None
    if not args.no_cpu:
        cpu = _cpu_baseline(oracle, synth, args)

    out = _base_line(args, value, "elem/s", ms64, "f64", {
        "workload": "temperature/alchemical ladder u_kn = beta_k E_n + lambda_k V_n, K=1000, "
                    "N=2e6 (N_k=2000), u_kn 1000x2e6 FP64 stored (16 GB), BU-MBAR on (E, V) "
                    "bins + Newton; value = its unbinned sweep (sample-major copy)",
        "K": K, "N": N, "tol_kT": args.tol})
    out.update({
        "time_to_solve_s": ms64 / 1e3,
        "error_vs_oracle_kT": cfg["c2_f64"]["error_vs_oracle_kT"],
        "sweep_kernel_us": sw64 * 1e6,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _counter_traffic("sweep_smaj_ladder_K1000_N2e6")},
        "configs": cfg,
        "cpu_baseline": cpu,
        "bench_wall_s": time.time() - t_all,
    })
    print(json.dumps(out), flush=True)


def _covariance_ms(bm, u, Nk, f, ctx, reps=3):
    """Wall time of bumbar_covariance at the solution (one warm-up call)."""
    import torch
    bm.covariance(u, Nk, f, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        bm.covariance(u, Nk, f, ctx=ctx)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def _c0(bm, synth, ctx, tol, reps=25):
    """K = 8 harmonic wells (N_k = 1000): time-to-solve in microseconds (median of
    the timed solves), BU-MBAR and plain Newton, errors against the oracle's
    golden f and the analytic free energies."""
    import torch
    p = synth.harmonic_1d(K=8, Nk=1000, seed=0)
    u = torch.tensor(p["u"], device="cuda")
    Nk = torch.tensor(p["Nk"], device="cuda")
    xi = torch.tensor(p["xi"], device="cuda")
    coef = torch.tensor(p["coef"], device="cuda")
    gold = _golden("c0_harmonic_K8_N8e3")
    out = {}
    for name, kw in (("bu_mbar", dict(xi=xi, model=bm.MODEL_HARMONIC, coef=coef)),
                     ("plain_newton", dict(binning=False))):
        times = []
        for i in range(reps + 5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f, info = bm.solve(u, Nk, tol=tol, ctx=ctx, **kw)
            torch.cuda.synchronize()
            if i >= 5:
                times.append(time.perf_counter() - t0)
        fa = f.cpu().numpy()
        stages = _stages(bm.solve(u, Nk, tol=tol, ctx=ctx, profile=1, **kw)[1])
        out[name] = dict(time_to_solve_us=1e6 * float(np.median(times)), status=info["status"],
                         **stages,
                         error_vs_oracle_kT=_err(f, gold),
                         error_vs_analytic_kT=(float(np.max(np.abs(fa - np.asarray(gold["analytic"]))))
                                               if gold else None))
    return out


def _c1(bm, synth, args, ctx):
    import torch
    p1 = synth.double_well(K=100, Nk=10000, seed=1)
    u1 = torch.tensor(p1["u"], device="cuda")
    Nk1 = torch.tensor(p1["Nk"], device="cuda")
    xi1 = torch.tensor(p1["xi"], device="cuda")
    coef1 = torch.tensor(p1["coef"], device="cuda")
    f1, inf1, ms1 = _timed_solves(
        bm, args, "c1 f64",
        lambda prof: bm.solve(u1, Nk1, xi=xi1, model=bm.MODEL_HARMONIC, coef=coef1, tol=args.tol,
                              profile=int(prof), ctx=ctx))
    sw1, _ = _avg_sweep_s(inf1)
    cov_ms = _covariance_ms(bm, u1, Nk1, f1, ctx)
    up_ms, up_gbs = _upload_solve_ms(
        torch, u1, lambda prof: bm.solve(u1, Nk1, xi=xi1, model=bm.MODEL_HARMONIC, coef=coef1,
                                         tol=args.tol, profile=int(prof), ctx=ctx))
    a1 = 8.0 * p1["K"] * p1["N"] / sw1 / 1e9
    res = dict(time_to_solve_s=ms1 / 1e3, sweep_us=sw1 * 1e6,
               sweep_elem_s=p1["K"] * p1["N"] / sw1, roofline_frac=a1 / HBM_PEAK_GBS,
               traffic=_counter_traffic("sweep_fast_double_well_K100_N1e6"),
               error_vs_oracle_kT=_err(f1, _golden("c1_double_well_K100_N1e6")),
               status=inf1[-1]["status"], covariance_ms=cov_ms,
               with_upload=dict(time_to_solve_s=up_ms / 1e3, upload_gb_s=up_gbs),
               **_stages(inf1[-1]))
    del u1
    torch.cuda.empty_cache()
    return res


def _c4(bm, synth, args, ctx, Nk_per, gold=None, hessian=True):
    import torch
    t = time.time()
    p = synth.muller_brown_grid(G=40, Nk=Nk_per, seed=4)
    K, N = p["K"], p["N"]
    xi = torch.tensor(p["xi"], device="cuda")
    coef = torch.tensor(p["coef"], device="cuda")
    Nk = torch.tensor(p["Nk"], device="cuda")
    log(f"muller-brown grid N_k={Nk_per} generated in {time.time() - t:.1f}s")
    f, infos, ms = _timed_solves(
        bm, args, f"c4 N_k={Nk_per} mixed",
        lambda prof: bm.solve(None, Nk, xi=xi, model=bm.MODEL_HARMONIC, coef=coef, tol=args.tol,
                              precision=bm.PREC_MIXED, profile=int(prof), ctx=ctx))
    fn, lD, S, st = bm.sweep_model(xi, coef, bm.MODEL_HARMONIC, Nk, f, precision=bm.PREC_FP64,
                                   ctx=ctx)
    res = dict(time_to_solve_s=ms / 1e3, K=K, N=N, status=infos[-1]["status"],
               fp64_sci_residual_kT=st["max_df"], grad_norm=st["grad_norm"],
               grid_sweeps=infos[-1]["grid_sweeps"], **_stages(infos[-1]))
    # one unbinned model sweep of each kind at the solution: the FP32 model
    # (two passes, one hardware exp2 per element each: bound by the
    # transcendental rate, 256 CUs x 16 per clock x 2.4 GHz = 9.83e12/s) and
    # the solve's FP64 sweep (the factored product-grid passes on this grid)
    sw = {}
    for name, prec in (("fp32_model", bm.PREC_MIXED), ("fp64", bm.PREC_FP64)):
        bm.sweep_model(xi, coef, bm.MODEL_HARMONIC, Nk, f, precision=prec, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            bm.sweep_model(xi, coef, bm.MODEL_HARMONIC, Nk, f, precision=prec, ctx=ctx)
        torch.cuda.synchronize()
        sw[name] = (time.perf_counter() - t0) / 3
    res["sweeps"] = dict(
        fp32_model_ms=1e3 * sw["fp32_model"], fp64_ms=1e3 * sw["fp64"],
        fp32_elem_s=K * N / sw["fp32_model"],
        fp32_exp_roofline_frac=2.0 * K * N / sw["fp32_model"] / 9.83e12)
    if gold is not None:
        res["error_vs_oracle_kT"] = _err(f, gold)
        f64, _, ms64 = _timed_solves(
            bm, args, f"c4 N_k={Nk_per} f64",
            lambda prof: bm.solve(None, Nk, xi=xi, model=bm.MODEL_HARMONIC, coef=coef,
                                  tol=args.tol, profile=int(prof), ctx=ctx))
        res["f64_time_to_solve_s"] = ms64 / 1e3
        res["f64_error_vs_oracle_kT"] = _err(f64, gold)
    if hessian:
        # the FP16-core Hessian of the mixed stage, timed on the context's stream;
        # algorithmic flops K (K + 1) N (the symmetric product, no padding)
        bm.hessian_model(xi, coef, bm.MODEL_HARMONIC, Nk, f, lD, S, precision=bm.PREC_MIXED,
                         ctx=ctx)
        h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        h0.record(ctx.stream)
        for _ in range(2):
            bm.hessian_model(xi, coef, bm.MODEL_HARMONIC, Nk, f, lD, S,
                             precision=bm.PREC_MIXED, ctx=ctx)
        h1.record(ctx.stream)
        torch.cuda.synchronize()
        th = h0.elapsed_time(h1) / 2e3
        flops = K * (K + 1) * N
        res["hessian"] = dict(seconds=th, algorithmic_flops=flops, tflop_s=flops / th / 1e12,
                              peak_tflop_s=2500.0, frac=flops / th / 1e12 / 2500.0,
                              dtype="fp16 inputs, fp32 accumulation")
    del xi, coef, Nk
    torch.cuda.empty_cache()
    return res


def _served(bm, probs, n, rate_seed, max_active, budget, opts, gold, fuse=False):
    """Saturation (closed loop), then Poisson arrivals at 0.8x that rate.

    fuse: a caller-driven server that fuses the small binned batches of its
    problems into one launch per tick."""
    drive = dict(caller_driven=fuse, fuse=fuse)
    _, wall_sat, _ = _serve(bm, probs, [0.0] * n, max_active, budget, opts, **drive)
    sat = n / wall_sat
    rate = 0.8 * sat
    g = np.random.Generator(np.random.PCG64(rate_seed))
    arrivals = list(np.cumsum(g.exponential(1.0 / rate, size=n)))
    log(f"  saturation {sat:.1f} solves/s; served run at {rate:.1f}/s")
    res, wall, cnt = _serve(bm, probs, arrivals, max_active, budget, opts, **drive)
    lat = np.array([info["latency_ms"] for _, info in res])
    err_gold = None
    if gold is not None:
        err_gold = max(float(np.max(np.abs(res[it["index"]][0] - np.asarray(it["f"]))))
                       for it in gold["problems"] if it["index"] < n)
    out = dict(solves_per_s=n / wall, p50_ms=float(np.percentile(lat, 50)),
               p99_ms=float(np.percentile(lat, 99)), rate_per_s=rate,
               saturation_solves_per_s=sat, max_active=max_active,
               hbm_budget_gb=budget / 2**30,
               failed=int(sum(1 for _, i in res if i["status"] not in (0, -4))),
               peak_active=cnt["peak_active"], peak_arena_gb=cnt["peak_bytes"] / 2**30,
               memory_bound_admissions=cnt["mem_waits"],
               error_vs_oracle_subset64_kT=err_gold)
    if fuse:
        out.update(fused_launches=cnt["fused_launches"], fused_batches=cnt["fused_items"])
    return out, res


def _c3(bm, args, stream):
    _, probs = stream
    n = len(probs)
    mixed = dict(tol=args.tol, precision=bm.PREC_MIXED)
    gold = _golden("c3_stream_subset64")
    _serve(bm, probs[:2], [0.0, 0.0], 2, 8 << 30, mixed)  # warm-up
    # the stream's recipe: u materialised on the device in FP32 (K N 4 bytes
    # resident per problem, counted by admission) and solved in mixed
    # precision; a 32 GB arena with 16 slots, so that admission is bound by
    # memory whenever several large problems are resident
    log("c3 materialised FP32 u, 16 slots, 32 GB arena")
    mat, res = _served(bm, probs, n, 33, 16, 32 << 30, dict(mixed, materialize=True), gold)
    # the same, driven by progress() ticks with the small binned batches of
    # all resident problems fused into one graph-replayed launch per tick
    log("c3 materialised FP32 u, 16 slots, 32 GB arena, fused launches")
    fused, res_f = _served(bm, probs, n, 33, 16, 32 << 30, dict(mixed, materialize=True), gold,
                           fuse=True)
    fused["max_abs_diff_vs_unfused_kT"] = max(float(np.max(np.abs(a[0] - b[0])))
                                              for a, b in zip(res, res_f))
    # the same requests with the energies evaluated inside the kernels (no
    # stored u): the faster mode, in the arena of --hbm-budget-gb
    log("c3 energies in the kernels, %d slots" % args.max_active)
    otf, res_otf = _served(bm, probs, n, 34, args.max_active, int(args.hbm_budget_gb * 2**30),
                           mixed, gold)
    log("c3 sequential FP64 run")
    res64, wall64, _ = _serve(bm, probs, [0.0] * n, 1, int(args.hbm_budget_gb * 2**30),
                              dict(tol=args.tol, precision=bm.PREC_FP64))
    lat64 = np.array([info["latency_ms"] for _, info in res64])
    out = dict(mat)
    out.update(
        n_problems=n, precision="mixed", storage="u materialised on the device, FP32",
        fused=fused, energies_in_kernel=otf,
        sequential_fp64=dict(solves_per_s=n / wall64, p50_ms=float(np.percentile(lat64, 50)),
                             p99_ms=float(np.percentile(lat64, 99))),
        max_abs_diff_vs_sequential_fp64_kT=max(float(np.max(np.abs(a[0] - b[0])))
                                               for a, b in zip(res_otf, res64)))
    return out


def _cpu_baseline(oracle, synth, args):
    """The FP64 oracle on this host: sweep rate on a bounded slice of c2, c1 in full."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    p = synth.ladder_2d(K=1000, Nk=100, seed=2, materialize=False)  # the c2 ladder, 1e5 samples
    E, V = p["xi"][:, 0], p["xi"][:, 1]
    u = np.empty((p["K"], p["N"]))
    for k in range(p["K"]):
        u[k] = p["beta"][k] * E + p["lam"][k] * V
    f = np.zeros(p["K"])
    reps, tc = 0, time.perf_counter()
    while True:
        oracle.sci_step(u, p["Nk"], f)
        reps += 1
        if time.perf_counter() - tc > args.cpu_seconds or reps >= 20:
            break
    per = (time.perf_counter() - tc) / reps
    rate = u.size / per
    tts = {}
    for name, key in (("c1", "c1_double_well_K100_N1e6"), ("c2", "c2_ladder_K1000_N2e6"),
                      ("c4r", "c4r_mullerbrown_K1600_N8e5")):
        gd = _golden(key)
        if gd is not None:
            c = gd["certificate"]
            tts[name] = {"seconds": c.get("oracle_seconds"), "threads": gd.get("threads"),
                         "how": "measured once, Algorithm 1 + Newton polish to the "
                                "certificate, on the host that wrote tests/golden"}
    return {"value": rate, "unit": "elem/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} FP64 oracle unbinned SCI sweeps over a 1000 x 1e5 slice of the "
                      f"c2 ladder ({per:.2f} s each; the full 1000 x 2e6 sweep would take "
                      f"{per * 20:.1f} s)",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "per_sweep_s_full_c2_extrapolated": per * 20,
            "time_to_solve": tts}


def _copy_calibration(torch):
    """A plain device copy of known size (1 GiB read + 1 GiB written): the
    reference kernel that scales the HBM byte counters."""
    xc = torch.empty(2**27, dtype=torch.float64, device="cuda")
    yc = torch.empty_like(xc)
    yc.copy_(xc)
    torch.cuda.synchronize()
    del xc, yc
    log("copy calibration: 1 GiB device copy done")


def _counter_traffic(name):
    """HBM bytes per launch of a kernel from its committed counter summary.

    The summary (profiles/<name>_traffic.json) records FETCH_SIZE and
    WRITE_SIZE per dispatch scaled by a plain copy kernel, and the hash of the
    kernel source it was taken with; a changed source gives None.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", name + "_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        src = os.path.join(ROOT, rec["source"])
        with open(src, "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if digest != rec.get("source_sha256"):
        return None
    return rec.get("bytes_per_launch")


def _timed_solves(bm, args, label, solve):
    """Warm-up and timed solves; returns (last f, infos, ms per solve)."""
    import torch
    for i in range(args.warmup):
        f, info = solve(False)
        log(f"{label} warmup {i}: status={info['status']} p1={info['phase1_iters']} "
            f"p2={info['phase2_iters']} newton={info['finisher_steps']} "
            f"mixed={info['mixed_steps']} hess={info['hessians']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        f, info = solve(True)
        infos.append(info)
        log(f"{label} step {i}: status={info['status']} binning={info['time_binning_ms']:.1f}ms "
            f"binned={info['time_binned_ms']:.1f}ms final={info['time_final_ms']:.1f}ms "
            f"sweeps={info['unbinned_sweeps']} newton={info['finisher_steps']} "
            f"hess={info['hessians']} sweep_ms={info['sweep_kernel_ms']:.2f}")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    return f, infos, ms


def _avg_sweep_s(infos):
    ms = sum(i["sweep_kernel_ms"] for i in infos)
    n = sum(i["sweep_kernel_launches"] for i in infos)
    return ms / max(1, n) / 1e3, n


def _stages(info):
    """Stage times of a timed solve, and the binned stage per binned SCI step
    (phase 1 and phase 2 of Algorithm 1, one sweep and its finaliser each)."""
    steps = info["phase1_iters"] + info["phase2_iters"]
    return dict(stages_ms=dict(binning=info["time_binning_ms"], binned=info["time_binned_ms"],
                               finisher=info["time_final_ms"]),
                binned_steps=dict(phase1=info["phase1_iters"], phase2=info["phase2_iters"],
                                  us_per_step=1e3 * info["time_binned_ms"] / max(1, steps)))


def _upload_solve_ms(torch, u, solve, reps=2):
    """Time-to-solve with u first copied from pinned host memory (PCIe included).

    The copy is synchronous, so it ends before the solve starts on the
    library's stream; returns (ms per upload + solve, upload GB/s)."""
    host = torch.empty(u.shape, dtype=u.dtype, pin_memory=True)
    host.copy_(u)
    solve(False)
    torch.cuda.synchronize()
    tot, up = 0.0, 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        u.copy_(host)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        solve(False)
        torch.cuda.synchronize()
        tot += time.perf_counter() - t0
        up += t1 - t0
    del host
    return 1e3 * tot / reps, u.numel() * u.element_size() * reps / up / 1e9


def _library_version():
    from paper_2609_03541_amd import _capi
    return _capi.load().bumbar_version().decode()


def _base_line(args, value, unit, ms, dtype, config):
    return {
        "metric": "sweep K*N elem/s + time-to-solve at 1e-6 kT; batched solves/s, p50/p99",
        "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic", "config": config, "library": _library_version(),
    }


def run_ladder(args, bm, synth):
    import torch
    t = time.time()
    p = synth.ladder_2d(K=1000, Nk=2000, seed=2, materialize=False)
    K, N = p["K"], p["N"]
    xi = torch.tensor(p["xi"], device="cuda")
    coef = torch.tensor(p["coef"], device="cuda")
    u = _ladder_u(torch, p)  # stored K x N FP64 (16 GB)
    u32 = u.float()          # FP32 storage for the mixed-precision solve (8 GB)
    Nk = torch.tensor(p["Nk"], device="cuda")
    torch.cuda.synchronize()
    log(f"ladder generated in {time.time() - t:.1f}s: K={K} N={N}, u {u.numel() * 8 / 1e9:.1f} GB")
    if args.copy_calibration:
        _copy_calibration(torch)
    ctx = bm.context()
    res = {}
    for name, prec, uu in (("f64", bm.PREC_FP64, u), ("mixed", bm.PREC_MIXED, u32)):
        f, infos, ms = _timed_solves(
            bm, args, name,
            lambda prof, prec=prec, uu=uu: bm.solve(uu, Nk, xi=xi, model=bm.MODEL_LINEAR,
                                                    coef=coef, tol=args.tol, precision=prec,
                                                    profile=int(prof), ctx=ctx))
        sw, n = _avg_sweep_s(infos)
        res[name] = dict(f=f.cpu().numpy(), ms=ms, sweep_s=sw, launches=n, info=infos[-1])
    diff = float(np.max(np.abs(res["mixed"]["f"] - res["f64"]["f"])))
    # single-sweep rates of the two stored-matrix sweeps at the solution
    f0 = torch.tensor(res["f64"]["f"], device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    bm.sweep(u, Nk, f0, ctx=ctx, with_stats=False)
    e0.record(ctx.stream)
    for _ in range(5):
        bm.sweep(u, Nk, f0, ctx=ctx, with_stats=False)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    f64_sweep_s = e0.elapsed_time(e1) / 5e3
    elems = K * N
    achieved = 8.0 * elems / f64_sweep_s / 1e9
    out = _base_line(args, elems / f64_sweep_s, "elem/s", res["f64"]["ms"], "f64", {
        "workload": "ladder u_kn = beta_k E_n + lambda_k V_n, K=1000, N=2e6 (N_k=2000), "
                    "u_kn 1000x2e6 FP64 stored (mixed: FP32 storage), BU-MBAR on (E, V) bins + "
                    "Newton",
        "K": K, "N": N, "tol_kT": args.tol})
    out.update({
        "time_to_solve_s": {"f64": res["f64"]["ms"] / 1e3, "mixed": res["mixed"]["ms"] / 1e3},
        "sweep_kernel_us_in_solve": {k: v["sweep_s"] * 1e6 for k, v in res.items()},
        "max_abs_diff_mixed_vs_f64_kT": diff,
        "grad_norm": res["f64"]["info"]["grad_norm"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": None,
    })
    print(json.dumps(out), flush=True)


def run_tladder(args, bm, synth):
    import torch
    t = time.time()
    p = synth.temperature_ladder(K=50, Nk=200000, seed=3, materialize=False)
    K, N = p["K"], p["N"]
    xi = torch.tensor(p["xi"], device="cuda")
    coef = torch.tensor(p["coef"], device="cuda")
    u = bm.model_energies(xi, coef, bm.MODEL_LINEAR, K)  # stored K x N FP64 (4 GB)
    Nk = torch.tensor(p["Nk"], device="cuda")
    torch.cuda.synchronize()
    log(f"temperature ladder generated in {time.time() - t:.1f}s: K={K} N={N}, "
        f"u {u.numel() * 8 / 1e9:.1f} GB")
    ctx = bm.context()
    variants = {
        "bumbar": dict(xi=xi, model=bm.MODEL_LINEAR, coef=coef),
        "newton": dict(binning=False, finisher=bm.FINISH_NEWTON, sci_switch=1e300),
        "sci": dict(binning=False, finisher=bm.FINISH_SCI, max_iter=200000),
    }
    res = {}
    for name, kw in variants.items():
        f, infos, ms = _timed_solves(
            bm, args, name,
            lambda prof, kw=kw: bm.solve(u, Nk, tol=args.tol, profile=int(prof), ctx=ctx, **kw))
        sw, n = _avg_sweep_s(infos)
        res[name] = dict(f=f.cpu().numpy(), ms=ms, sweep_s=sw, launches=n, info=infos[-1])
    ref = res["bumbar"]["f"]
    sw = res["bumbar"]["sweep_s"]
    elems = K * N
    achieved = 8.0 * elems / sw / 1e9
    out = _base_line(args, elems / sw, "elem/s", res["bumbar"]["ms"], "f64", {
        "workload": "temperature ladder u_kn = beta_k E_n, K=50 (beta geometric over 2x), "
                    "N=1e7 (N_k=2e5), 80% neighbour overlap, u_kn 50x1e7 FP64 stored; "
                    "BU-MBAR on E bins + Newton vs plain SCI vs plain Newton",
        "K": K, "N": N, "tol_kT": args.tol})
    out.update({
        "time_to_solve_s": {k: v["ms"] / 1e3 for k, v in res.items()},
        "status": {k: v["info"]["status"] for k, v in res.items()},
        "iterations": {k: {"binned": v["info"]["phase1_iters"] + v["info"]["phase2_iters"],
                           "finisher": v["info"]["finisher_steps"],
                           "unbinned_sweeps": v["info"]["unbinned_sweeps"]}
                       for k, v in res.items()},
        "max_abs_diff_vs_bumbar_kT": {k: float(np.max(np.abs(v["f"] - ref)))
                                      for k, v in res.items() if k != "bumbar"},
        "sweep_kernel_us": sw * 1e6,
        "grad_norm": res["bumbar"]["info"]["grad_norm"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": None,
    })
    print(json.dumps(out), flush=True)


# The replica-count study of Section 4 (Fig. 3): scenario name, N0, power p
# with N_k = N0 / M^p; seeds 9000 + 100 M + 10 scenario + s (the same recipe
# tests/golden/make_golden.py gives the oracle).
FIG3 = (("i", 1e4, 0), ("ii", 3e6, 1), ("iii", 9e8, 2))


def run_scaling(args, bm, synth):
    import torch
    ctx = bm.context()
    gold = _golden("fig3_replicas_full_small")
    gmap = {}
    if gold is not None:
        gmap = {(it["scenario"], it["M"], it["seed"]): np.asarray(it["f"])
                for it in gold["problems"]}
    table = []
    top = None
    for si, (sname, n0, pw) in enumerate(FIG3):
        for M in (10, 30, 100, 300):
            nk = int(round(n0 / M ** pw))
            times = {"bumbar": [], "newton": [], "sci": []}
            errs, diffs, sweeps = [], [], []
            for s in range(args.seeds):
                seed = 9000 + 100 * M + 10 * si + s
                p = synth.temperature_ladder(K=M, Nk=nk, seed=seed, materialize=False)
                K, N = p["K"], p["N"]
                xi = torch.tensor(p["xi"], device="cuda")
                coef = torch.tensor(p["coef"], device="cuda")
                u = bm.model_energies(xi, coef, bm.MODEL_LINEAR, K)
                Nk = torch.tensor(p["Nk"], device="cuda")
                torch.cuda.synchronize()
                variants = {
                    "bumbar": dict(xi=xi, model=bm.MODEL_LINEAR, coef=coef, profile=1),
                    "newton": dict(binning=False, finisher=bm.FINISH_NEWTON, sci_switch=1e300),
                }
                if s == 0 and M <= 100:
                    variants["sci"] = dict(binning=False, finisher=bm.FINISH_SCI, max_iter=20000)
                fs = {}
                for name, kw in variants.items():
                    if s == 0:  # untimed first solve of this shape
                        bm.solve(u, Nk, tol=args.tol, ctx=ctx, **kw)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    f, info = bm.solve(u, Nk, tol=args.tol, ctx=ctx, **kw)
                    torch.cuda.synchronize()
                    times[name].append((time.perf_counter() - t0) * 1e3)
                    fs[name] = f.cpu().numpy()
                    if name == "bumbar":
                        sw, _ = _avg_sweep_s([info])
                        sweeps.append(sw)
                diffs.append(float(np.max(np.abs(fs["newton"] - fs["bumbar"]))))
                g = gmap.get((sname, M, seed))
                if g is not None:
                    errs.append(max(float(np.max(np.abs(fs[v] - g))) for v in ("bumbar", "newton")))
                del u, xi, coef, Nk
            row = {"M": M, "scenario": sname, "N_k": nk, "N": M * nk, "seeds": args.seeds}
            for name, ts in times.items():
                if ts:
                    row[name + "_ms_mean"] = float(np.mean(ts))
                    row[name + "_ms_sd"] = float(np.std(ts, ddof=1)) if len(ts) > 1 else 0.0
                    row[name + "_seeds"] = len(ts)
            row["sweep_us_mean"] = float(np.mean(sweeps)) * 1e6
            row["max_abs_diff_newton_vs_bumbar_kT"] = max(diffs)
            row["max_err_vs_oracle_kT"] = max(errs) if errs else None
            row["oracle_checked_seeds"] = len(errs)
            table.append(row)
            log(json.dumps(row))
            if M == 300 and sname == "i":
                top = (M, M * nk, row)
            torch.cuda.empty_cache()
    K, N, row = top
    sw = row["sweep_us_mean"] / 1e6
    achieved = 8.0 * K * N / sw / 1e9
    out = _base_line(args, K * N / sw, "elem/s", row["bumbar_ms_mean"], "f64", {
        "workload": "replica-count study: temperature ladders M = 10, 30, 100, 300 at 80% "
                    "neighbour overlap, N_k = 1e4, 3e6/M, 9e8/M^2, "
                    f"{args.seeds} seeds each; BU-MBAR vs plain Newton vs plain SCI (seed 0); "
                    "value and roofline from M=300, N_k=1e4 (u 300x3e6 FP64)",
        "tol_kT": args.tol})
    out.update({
        "scaling_table": table,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": None,
    })
    print(json.dumps(out), flush=True)


def run_mb2d(args, bm, synth):
    import torch
    t = time.time()
    p = synth.muller_brown_grid(G=40, Nk=5000, seed=4)
    K, N = p["K"], p["N"]
    xi = torch.tensor(p["xi"], device="cuda")
    coef = torch.tensor(p["coef"], device="cuda")
    Nk = torch.tensor(p["Nk"], device="cuda")
    torch.cuda.synchronize()
    log(f"muller-brown grid generated in {time.time() - t:.1f}s: K={K} N={N}")
    if args.copy_calibration:
        _copy_calibration(torch)
    ctx = bm.context()
    f, infos, ms = _timed_solves(
        bm, args, "mixed",
        lambda prof: bm.solve(None, Nk, xi=xi, model=bm.MODEL_HARMONIC, coef=coef, tol=args.tol,
                              precision=bm.PREC_MIXED, profile=int(prof), ctx=ctx))
    # single model sweeps at the solution, FP32 and FP64
    rates = {}
    for name, prec in (("f32", bm.PREC_MIXED), ("f64", bm.PREC_FP64)):
        bm.sweep_model(xi, coef, bm.MODEL_HARMONIC, Nk, f, precision=prec, ctx=ctx)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            fn, lD, S, st = bm.sweep_model(xi, coef, bm.MODEL_HARMONIC, Nk, f, precision=prec,
                                           ctx=ctx)
        torch.cuda.synchronize()
        rates[name] = (time.perf_counter() - t0) / reps
        if name == "f64":
            residual = st["max_df"]
            gnorm = st["grad_norm"]
    elems = K * N
    # the dominant kernel of the solve: the FP16-core Hessian of the mixed
    # stage, algorithmic flops K (K + 1) N (the symmetric product, no
    # padding), timed on the context's stream
    bm.hessian_model(xi, coef, bm.MODEL_HARMONIC, Nk, f, lD, S, precision=bm.PREC_MIXED, ctx=ctx)
    torch.cuda.synchronize()
    h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 2
    h0.record()
    for _ in range(reps):
        bm.hessian_model(xi, coef, bm.MODEL_HARMONIC, Nk, f, lD, S, precision=bm.PREC_MIXED,
                         ctx=ctx)
    h1.record()
    torch.cuda.synchronize()
    t_hess = h0.elapsed_time(h1) / reps / 1e3
    hflops = K * (K + 1) * N
    hrate = hflops / t_hess / 1e12
    # the solve's sweeps on this grid are the factored FP64 passes
    out = _base_line(args, elems / rates["f64"], "elem/s", ms, "f32+f64", {
        "workload": "2-D umbrella grid on the Muller-Brown surface, K=1600 windows (kappa=20), "
                    "N=8e6 (N_k=5000) FP32 (x,y); u_kn evaluated in-kernel, mixed-precision "
                    "BU-MBAR", "K": K, "N": N, "tol_kT": args.tol})
    out.update({
        "time_to_solve_s": ms / 1e3,
        "sweep_s": rates,
        "fp64_sci_residual_kT": residual,
        "grad_norm": gnorm,
        "hessian_s": t_hess,
        "roofline": {"bound": "mfma", "achieved": hrate, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": hrate / 2500.0, "traffic": None},
        "cpu_baseline": None,
    })
    print(json.dumps(out), flush=True)


def _gen_problem(spec):
    import synth
    p = synth.materialize_problem(spec, materialize=False)
    return {k: p[k] for k in ("K", "N", "Nk", "xi", "coef", "model_type")}


def _serve(bm, probs, arrivals, max_active, budget, opts, caller_driven=False, fuse=False):
    """Submit the problems at their arrival times; returns (results, wall s, counters).

    caller_driven: the server has no worker threads; this loop ticks it
    (progress) between arrivals. fuse: fused small batches (caller-driven)."""
    srv = bm.Server(hbm_budget_bytes=budget, max_active=max_active, caller_driven=caller_driven,
                    fuse=fuse)
    try:
        t0 = time.perf_counter()
        tickets = []
        done = 0
        for p, ta in zip(probs, arrivals):
            while True:
                dt = t0 + ta - time.perf_counter()
                if dt <= 0:
                    break
                if caller_driven:
                    done += srv.progress()
                else:
                    time.sleep(dt)
            tickets.append(srv.submit(p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                                      **opts))
        res = []
        for i, t in enumerate(tickets):
            res.append(srv.result(t))
            if (i + 1) % 64 == 0:
                log(f"  {i + 1}/{len(tickets)} results")
        wall = time.perf_counter() - t0
        return res, wall, srv.counters()
    finally:
        srv.close()


def generate_stream(args):
    """Problems of the seeded 512-problem stream (the specs do not depend on the
    arrival rate) and Poisson arrival times at args.rate from a separate seed."""
    from concurrent.futures import ProcessPoolExecutor

    import synth
    stream = synth.serving_stream(n_problems=args.n_problems, seed=3)
    t = time.time()
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(workers) as ex:
        probs = list(ex.map(_gen_problem, [s for _, s in stream], chunksize=4))
    log(f"stream generated in {time.time() - t:.1f}s with {workers} processes")
    g = np.random.Generator(np.random.PCG64(33))
    arrivals = list(np.cumsum(g.exponential(1.0 / args.rate, size=len(probs))))
    return arrivals, probs


def run_stream(args, bm, stream):
    arrivals, probs = stream
    kn = np.array([p["K"] * p["N"] for p in probs], dtype=np.float64)
    log(f"{len(probs)} problems, mean K*N {kn.mean():.3g}, max {kn.max():.3g}")
    budget = int(args.hbm_budget_gb * 2**30)
    mixed = dict(tol=args.tol, precision=bm.PREC_MIXED)
    # warm-up: one small problem through a server (loads kernels, sizes caches)
    _serve(bm, probs[:2], [0.0, 0.0], 2, budget, mixed)
    log(f"served run: max_active={args.max_active}, mixed precision, rate {args.rate}/s")
    res, wall, cnt = _serve(bm, probs, arrivals, args.max_active, budget, mixed)
    lat = np.array([info["latency_ms"] for _, info in res])
    status = [info["status"] for _, info in res]
    out_seq = None
    err = None
    if not args.skip_sequential:
        log("sequential run: one problem at a time, FP64")
        res64, wall64, _ = _serve(bm, probs, arrivals, 1, budget,
                                  dict(tol=args.tol, precision=bm.PREC_FP64))
        lat64 = np.array([info["latency_ms"] for _, info in res64])
        err = max(float(np.max(np.abs(a[0] - b[0]))) for a, b in zip(res, res64))
        out_seq = {"solves_per_s": len(probs) / wall64, "p50_ms": float(np.percentile(lat64, 50)),
                   "p99_ms": float(np.percentile(lat64, 99)), "wall_s": wall64,
                   "precision": "f64", "max_active": 1}
    value = len(probs) / wall
    out = {
        "metric": "sweep K*N elem/s + time-to-solve at 1e-6 kT; batched solves/s, p50/p99",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"batched serving: {len(probs)} harmonic/double-well problems, "
                               "K in [4,256], N_k in [100,20000], Poisson arrivals, u_kn built "
                               "on the device from the bias model, mixed precision",
                   "n_problems": len(probs), "rate_per_s": args.rate,
                   "max_active": args.max_active, "hbm_budget_gb": args.hbm_budget_gb,
                   "mean_KN": float(kn.mean()), "tol_kT": args.tol},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "failed": int(sum(1 for s_ in status if s_ not in (0, -4))),
        "peak_active": cnt["peak_active"],
        "peak_arena_gb": cnt["peak_bytes"] / 2**30,
        "sequential_fp64": out_seq,
        "max_abs_diff_vs_fp64_kT": err,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
