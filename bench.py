"""Benchmark: imaginary-time steps of the SGS method on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config NAME] [--weight unit|printed]
                    [--no-cpu-baseline] [--gpus 1]

One step is the whole hot path (pair inverses, overlaps with phase, Wick
elements, amplitude solve, force, Euler step and purification) over every
pair of the R Gaussian states of the workload.  The default workload is the
largest single-GPU configuration: the two-channel Kondo model with two chains
of 150 sites (N = 602 modes, n = 1204 Majoranas) and R = 24 states.  The inputs
(Hamiltonian and seeded Haar-random covariance matrices) are resident in HBM
before the timed region.  The FP64 path is timed for the headline; the
FP32-force path is timed on the same steps after it, and both one-step results
are compared with the oracle's stored step where one exists
(tests/golden/<workload>_step.json).  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix peak

# HBM bytes per launch of the force products, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters on the workload (FETCH_SIZE scaled by 1.99992,
# WRITE_SIZE by 1.0: the factors a 1 GiB device copy reads back), in
# profiles/force_tck_L150_R24_fp64.md.  Only valid for the kernel and workload
# they were taken on; any other combination reports null.
FORCE_TRAFFIC_BYTES = {("tck_L150_R24_J0.3", "fp64", "k_force_big"): 6.6751e10}


def force_kernel(n: int, precision: str) -> str:
    """Name of the force-product kernel the library's built-in choice uses:
    128 x 128 tiles from n = 1000 in float64 (n = 600 in float32)."""
    return "k_force_big" if n >= (600 if precision == "fp32" else 1000) else "k_force"


def inverse_flops(n: int, P: int) -> float:
    """Algorithmic flops of the pair inverses: 2 n^3 per pair (Gauss-Jordan)."""
    return P * 2.0 * n ** 3


def pfaffian_flops(n: int, Q: int) -> float:
    """Algorithmic flops of the phase Pfaffians: n^3 / 3 complex multiply-adds
    (8 real flops each) per phase pair, (8/3) n^3."""
    return Q * 8.0 / 3.0 * n ** 3


def step_flops(n: int, R: int) -> float:
    """The step's dense work by the method's own operation counts: inverses,
    Pfaffians, the transition matrices (n^3 per pair, skew output), the phase
    matrices X_a (4 n^3 per state but the reference), the force products, and
    about three polar iterations (4 n^3 each) per state."""
    P = R * (R - 1) // 2
    Q = (R - 1) * (R - 2) // 2
    return (inverse_flops(n, P) + pfaffian_flops(n, Q) + P * 1.0 * n ** 3 + (R - 1) * 4.0 * n ** 3
            + force_flops(n, R) + R * 12.0 * n ** 3)


def dense_equiv_flops(n: int, R: int) -> float:
    """The fixed dense-equivalent accounting of the measurement plan: 14.7 n^3
    per pair-eval (a 2 n^3 factorization, a 2 n^3 real GEMM, an 8 n^3 complex
    GEMM and an (8/3) n^3 complex Pfaffian) plus 18 n^3 per state (the force
    sandwich, X_a and about three polar iterations), whatever the kernels
    actually do."""
    P = R * (R - 1) // 2
    return P * (2 + 2 + 8 + 8.0 / 3.0) * n ** 3 + R * 18.0 * n ** 3


def golden_step(config: str):
    """The oracle's stored one-step result for this workload, or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{config}_step.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def sample_err(gam_dev, gold) -> float:
    import numpy as np
    g = gam_dev.cpu().numpy()
    idx = np.array(gold["sample_idx"])
    return float(np.abs(g[idx[:, 0], idx[:, 1], idx[:, 2]] - np.array(gold["sample_val"])).max())


def cpu_info():
    """CPU model and BLAS library behind numpy (for the oracle's timing)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas, threads = "unknown", os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        info = [x for x in threadpool_info() if x.get("user_api") == "blas"]
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
            threads = max(int(x.get("num_threads", 1)) for x in info)
    except Exception:  # pragma: no cover
        pass
    return model, blas, threads


def force_flops(n: int, R: int) -> float:
    """Algorithmic flops of one force launch: for every ordered pair mu != b the
    real part of c1 (Delta F) Delta is two real n x n x n products, of which the
    skew output needs half (2 n^3); the diagonal term b = mu needs one product,
    half of it (n^3)."""
    return R * (R - 1) * 2.0 * n ** 3 + R * 1.0 * n ** 3


def _tune_arg(t):
    if t is None:
        return None
    if t.lstrip().startswith("["):
        return json.loads(t)
    return t


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="tck_L150_R24_J0.3")
    ap.add_argument("--weight", choices=["unit", "printed"], default="unit")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="fp32: the force's dense product on the FP32 matrix cores")
    ap.add_argument("--update", choices=["euler", "exp"], default="euler",
                    help="exp: the orthogonal exponential-map update instead of Euler + purification")
    ap.add_argument("--dtau", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="replay each step as one HIP graph launch (no per-stage times)")
    ap.add_argument("--tune", default=None,
                    help="tuning table: a JSON file written by paper_2105_01088_amd/autotune.py, or an "
                         "inline JSON list of rows")
    ap.add_argument("--grow", type=int, default=0, metavar="STEPS",
                    help="run the rank-growing protocol (Sec. III.C) on the workload: STEPS steps at "
                         "each rank from 1 to R, one rotated copy of the largest-amplitude state added "
                         "per rank; prints its own JSON line")
    ap.add_argument("--renyi", default=None, metavar="NA[,NA...]",
                    help="time the Renyi-2 entropy S_2 of the first NA Majoranas (impurity plus sites) "
                         "on the workload after the warmup steps, automatic method and block form; "
                         "prints its own JSON line")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (counter calibration) and exit")
    args = ap.parse_args(argv)

    if args.copy_probe > 0:
        import torch
        x = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 8}), flush=True)
        return 0

    if args.config.startswith("batched"):
        # up to 8 worker streams of three HIP streams each run concurrently
        # only on as many hardware queues (read when HIP starts)
        try:
            have = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
        except ValueError:
            have = 4
        if have < 28:
            os.environ["GPU_MAX_HW_QUEUES"] = "28"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the sharding of this path over several GPUs is not built.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import sgs_inputs as si
    from paper_2105_01088_amd import SGS, default_options

    if args.config.startswith("batched"):
        return bench_batched(args)
    if args.grow > 0:
        return bench_grow(args)
    if args.renyi:
        return bench_renyi(args)

    ham, gam, cfg = si.config_problem(args.config)
    n, R = ham.n, gam.shape[0]
    P = R * (R - 1) // 2
    dtau = float(args.dtau if args.dtau is not None else cfg["dtau"])
    weight = 1 if args.weight == "unit" else 0

    prec = 1 if args.precision == "fp32" else 0
    upd = 1 if args.update == "exp" else 0
    ctx = SGS([ham], [gam], options=default_options(weight=weight, precision=prec, update=upd,
                                                    tune=_tune_arg(args.tune), graph=int(args.graph)))
    stream = ctx.stream
    gold = golden_step(args.config) if (weight == 1 and upd == 0 and dtau == 0.05) else None
    # warmup (the first step is compared with the oracle's stored step)
    e_first = ctx.step(dtau, 1)
    step1_err = sample_err(ctx.gammas(0), gold) if gold is not None else None
    if args.warmup > 1:
        ctx.step(dtau, args.warmup - 1)
    torch.cuda.synchronize()
    st = ctx.status()
    if st != 0:
        raise SystemExit(f"device status {st} during warmup")

    # timed region: K steps, stage events on the library's stream
    ctx.set_timing(True)
    ctx.stage_times()  # clear
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.time()
    t0.record(stream)
    h0 = time.perf_counter()
    energies = ctx.step(dtau, args.steps)
    host_enqueue = time.perf_counter() - h0
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    ms_total = t0.elapsed_time(t1)
    stages = ctx.stage_times()
    ctx.set_timing(False)
    st = ctx.status()
    if st != 0:
        raise SystemExit(f"device status {st} in the timed region")

    # the standalone table evaluation (sgs_pair_eval: inverses, overlaps,
    # phases, Wick elements and the amplitude solve, no force or update)
    ctx.pair_eval()
    torch.cuda.synchronize()
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    for _ in range(args.steps):
        ctx.pair_eval()
    p1.record(stream)
    torch.cuda.synchronize()
    ms_pe = p0.elapsed_time(p1) / args.steps
    if ctx.status() != 0:
        raise SystemExit("device status error in sgs_pair_eval")

    # the variance of H (Eq. residual) of the current states: the tables are
    # current after sgs_pair_eval, so each call times the variance kernels only
    from paper_2105_01088_amd import SGS_OBS_VARIANCE
    vout = ctx.observables(SGS_OBS_VARIANCE, [0], [], 3)
    torch.cuda.synchronize()
    v0 = torch.cuda.Event(enable_timing=True)
    v1 = torch.cuda.Event(enable_timing=True)
    nvar = 5
    v0.record(stream)
    for _ in range(nvar):
        vout = ctx.observables(SGS_OBS_VARIANCE, [0], [], 3)
    v1.record(stream)
    torch.cuda.synchronize()
    ms_var = v0.elapsed_time(v1) / nvar
    var = vout.cpu().numpy()
    if ctx.status() != 0:
        raise SystemExit("device status error in the variance")

    ms_step = ms_total / args.steps
    value = P * args.steps / (ms_total / 1e3)
    f_ms, f_n = stages["force"]
    f_avg_ms = f_ms / max(1, f_n)
    achieved = force_flops(n, R) / (f_avg_ms / 1e3) / 1e12 if f_avg_ms > 0 else None
    peak = FP32_PEAK_TFLOPS if prec == 1 else FP64_PEAK_TFLOPS
    Q = (R - 1) * (R - 2) // 2
    stage_ms = {k: v[0] / max(1, args.steps) for k, v in stages.items()}

    def frac(flops, ms):
        if not ms > 0:
            return None
        tf = flops / (ms / 1e3) / 1e12
        return {"achieved": tf, "frac": tf / FP64_PEAK_TFLOPS, "flops": flops, "ms": ms}

    out = {
        "metric": "Gaussian-pair evals/s",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "us_per_step": ms_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": args.config,
            "model": cfg["model"], "L": cfg["L"], "N_modes": ham.N, "n_majoranas": n, "R": R,
            "pairs_per_step": P, "dtau": dtau, "seed": cfg["seed"],
            "weights": args.weight, "precision": args.precision, "update": args.update,
            "graph": bool(args.graph),
        },
        "roofline": {
            "bound": "mfma",
            "kernel": force_kernel(n, args.precision),
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak if achieved is not None else None,
            "traffic": (None if args.tune else
                        FORCE_TRAFFIC_BYTES.get((args.config, args.precision, force_kernel(n, args.precision)))),
            "force_avg_ms": f_avg_ms,
            "force_flops_per_launch": force_flops(n, R),
        },
        # FP64 matrix peak fractions by the method's own counts, per stage
        # (stage times are intervals on their streams; the inverse and the
        # Pfaffian chain run concurrently, so their sum exceeds the step)
        "stage_roofline": {
            "inverse": frac(inverse_flops(n, P), stage_ms["inverse"]),
            "pfaffian": frac(pfaffian_flops(n, Q), stage_ms["pfaffian"]),
            "step": frac(step_flops(n, R), ms_step),
            "step_dense_equivalent": frac(dense_equiv_flops(n, R), ms_step),
            "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS,
            "note": "step: the method's own operation counts (skew outputs halved); step_dense_equivalent: "
                    "14.7 n^3 per pair + 18 n^3 per state, the plan's fixed accounting",
        },
        "pair_eval": {"ms_per_call": ms_pe, "pair_evals_per_s": P / (ms_pe / 1e3)},
        "variance": {"ms_per_call": ms_var, "E": float(var[0]), "H2": float(var[1]), "delta_H2": float(var[2])},
        "stages_ms_per_step": stage_ms,
        "wall_s": wall,
        "host_enqueue_ms_per_step": host_enqueue * 1e3 / args.steps,
        "E_last": float(energies[-1].item()),
    }

    if gold is not None:
        out["step1_state_err_vs_oracle"] = step1_err
        out["E_step0_rel_err_vs_oracle"] = abs(float(e_first[0].item()) - gold["E"]) / abs(gold["E"])

    if prec == 0 and upd == 0:
        # the FP32-force path on the same steps from the same states (after
        # the FP64 timed region): its own time, its per-step energy difference
        # from the FP64 run, and its one-step error against the oracle
        ctx.close()
        ctx = None
        torch.cuda.empty_cache()
        ctx32 = SGS([ham], [gam], options=default_options(weight=weight, precision=1, tune=_tune_arg(args.tune)))
        e32_first = ctx32.step(dtau, 1)
        err32 = sample_err(ctx32.gammas(0), gold) if gold is not None else None
        if args.warmup > 1:
            ctx32.step(dtau, args.warmup - 1)
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(ctx32.stream)
        e32 = ctx32.step(dtau, args.steps)
        a1.record(ctx32.stream)
        torch.cuda.synchronize()
        ms32 = a0.elapsed_time(a1) / args.steps
        st32 = ctx32.status()
        e32 = e32.cpu().numpy()
        e64 = energies.cpu().numpy()
        out["fp32_force"] = {
            "ms_per_step": ms32, "pair_evals_per_s": P / (ms32 / 1e3), "status": st32,
            "speedup_vs_fp64": ms_step / ms32,
            "E_rel_diff_vs_fp64_max": float((np.abs(e32 - e64) / np.abs(e64)).max()),
            "step1_state_err_vs_oracle": err32,
            "note": "force products on the FP32 matrix cores; tables, eigen-solve and purification in FP64",
        }
        ctx32.close()

    if not args.no_cpu_baseline:
        # the oracle as it stands, on a bounded sample of the workload: one
        # step of the first Rs states (Rs (Rs - 1) / 2 pairs at the full n),
        # Rs chosen so that the sample is some 10-30 s of host work
        from oracle import sgs as osgs
        model, blas, cores = cpu_info()
        Rs = R if n <= 400 else min(R, 8)  # 28 pairs: about 14 s at n = 1204 on 16 cores
        Ps = Rs * (Rs - 1) // 2
        hp = ham.poly()
        c0 = time.time()
        ref = osgs.step(ham, gam[:Rs], dtau, mode=args.weight, hpoly=hp, update=args.update)
        c_dt = time.time() - c0
        out["cpu_baseline"] = {
            "value": Ps / c_dt,
            "unit": "pair-evals/s",
            "cores": cores,
            "kind": "oracle",
            "sample": f"1 oracle step of the first {Rs} of the {R} states of {args.config} "
                      f"({Ps} pairs at n={n}), from the same seeded states",
            "s_per_sample": c_dt,
            "cpu": model,
            "blas": blas,
        }
        if Rs == R:
            out["E_step0_rel_err_vs_oracle"] = abs(float(e_first[0].item()) - ref.E) / abs(ref.E)

    print(json.dumps(out), flush=True)
    if ctx is not None:
        ctx.close()
    return 0


def bench_batched(args):
    """The batched workload: 64 independent Anderson problems of uneven size
    (n = 84..1204, R in {4, 8, 16}) in one context, all stepped together.
    Timed four ways: one worker stream (problems one after another), one HIP
    graph launch per step, 4 and 6 worker streams; `value` is the fastest.
    28 hardware queues are requested (GPU_MAX_HW_QUEUES, raised to 28 if it is
    lower), so that the workers' streams do not share queues."""
    import torch

    import sgs_inputs as si
    from paper_2105_01088_amd import SGS, default_options

    count = int(args.config[len("batched"):] or 64)
    probs = si.batched_problems(0, count=count)
    hams = [h for h, _, _ in probs]
    gams = [g for _, g, _ in probs]
    pairs = sum(g.shape[0] * (g.shape[0] - 1) // 2 for g in gams)
    flops = sum(step_flops(h.n, g.shape[0]) for h, g in zip(hams, gams))
    dtau = float(args.dtau if args.dtau is not None else 0.05)
    weight = 1 if args.weight == "unit" else 0
    rates = {}
    ms = {}
    # (8 worker streams measured slower, and slowed the contexts created after
    # them in the same process: 1004 ms, then 1030 ms for 6 workers that had
    # taken 825 ms before)
    for streams, graph in ((1, 0), (4, 1), (4, 0), (6, 0)):
        key = (streams, graph)
        ctx = SGS(hams, gams, options=default_options(weight=weight, streams=streams, graph=graph))
        ctx.step(dtau, max(1, args.warmup))
        torch.cuda.synchronize()
        if ctx.status() != 0:
            raise SystemExit(f"device status {ctx.status()} during warmup")
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(ctx.stream)
        ctx.step(dtau, args.steps)
        t1.record(ctx.stream)
        torch.cuda.synchronize()
        if ctx.status() != 0:
            raise SystemExit(f"device status {ctx.status()} in the timed region")
        total = t0.elapsed_time(t1)
        ms[key] = total / args.steps
        rates[key] = pairs * args.steps / (total / 1e3)
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    names = {(1, 0): "1 worker stream", (4, 0): "4 worker streams", (6, 0): "6 worker streams",
             (4, 1): "one HIP graph launch per step (one worker stream inside)"}
    best = min(ms, key=ms.get)
    out = {
        "metric": "Gaussian-pair evals/s",
        "value": rates[best],
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms[best],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched{count}", "problems": count, "pairs_per_step": pairs,
                   "n_range": [min(h.n for h in hams), max(h.n for h in hams)], "dtau": dtau, "seed": 0,
                   "weights": args.weight, "precision": args.precision},
        "launch": names[best],
        "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
        "sequential": {"value": rates[(1, 0)], "ms_per_step": ms[(1, 0)], "streams": 1,
                       "speedup": rates[best] / rates[(1, 0)]},
        "all": {names[k]: {"value": rates[k], "ms_per_step": ms[k]} for k in ms},
        "roofline": {"bound": "mfma", "kernel": "whole step", "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS,
                     "achieved": flops / (ms[best] / 1e3) / 1e12,
                     "frac": flops / (ms[best] / 1e3) / 1e12 / FP64_PEAK_TFLOPS, "traffic": None,
                     "flops_per_step": flops,
                     "note": "the method's own operation counts summed over the problems (step_flops)"},
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_renyi(args) -> int:
    """S_2 (Eq. S2_SGS, App. B) of A = Majoranas 0..NA-1 on the workload's
    states after the warmup steps: milliseconds per evaluation (the call waits
    for its stream) with the automatic method and with the block form for
    every term, and the number of representative terms, about R^4 / 4."""
    import torch

    import sgs_inputs as si
    from paper_2105_01088_amd import SGS, SGS_REN_AUTO, SGS_REN_BLOCK, default_options

    ham, gam, cfg = si.config_problem(args.config)
    R = gam.shape[0]
    ctx = SGS([ham], [gam], options=default_options(weight=1 if args.weight == "unit" else 0))
    ctx.step(float(args.dtau if args.dtau is not None else 0.05), max(1, args.warmup))
    torch.cuda.synchronize()
    out = []
    for nA in (int(x) for x in args.renyi.split(",")):
        for method in ((SGS_REN_AUTO, SGS_REN_BLOCK) if nA > 32 else (SGS_REN_AUTO,)):
            v = ctx.renyi2(nA, method=method)  # buffers, tables
            reps = max(1, args.steps)
            t0 = time.perf_counter()
            for _ in range(reps):
                v = ctx.renyi2(nA, method=method)
            ms = (time.perf_counter() - t0) * 1e3 / reps
            out.append({"nA": nA, "method": "auto" if method == SGS_REN_AUTO else "block", "ms_per_eval": ms,
                        "S2": v})
            print(f"renyi2 nA={nA} {out[-1]['method']}: {ms:.2f} ms, S2 = {v:.12f}", file=sys.stderr, flush=True)
    status = ctx.status()
    ctx.close()
    terms = sum(1 for p in range(R * R) for q in range(p, R * R)
                if tuple(sorted(((p % R) * R + p // R, (q % R) * R + q // R))) >= (p, q))
    print(json.dumps({"metric": "Renyi-2 evaluations", "unit": "ms/eval", "higher_is_better": False,
                      "config": {"workload": args.config, "n_majoranas": ham.n, "R": R, "terms": terms,
                                 "warmup_steps": max(1, args.warmup)},
                      "status": status, "results": out}), flush=True)
    return 0 if status == 0 else 1


def bench_grow(args) -> int:
    """The rank-growing protocol on one workload: R - 1 rotations (|Q - 1|_F =
    0.3, seeded), STEPS steps per rank, from the workload's first state."""
    import numpy as np
    import torch

    import sgs_inputs as si
    from paper_2105_01088_amd import SGS, SGS_OBS_VARIANCE, default_options, grow

    ham, gam, cfg = si.config_problem(args.config)
    R = gam.shape[0]
    dtau = float(args.dtau if args.dtau is not None else cfg["dtau"])
    weight = 1 if args.weight == "unit" else 0
    rots = si.small_rotations(ham.n, R - 1, 0.3, seed=cfg["seed"])
    opts = default_options(weight=weight)
    torch.cuda.synchronize()
    t0 = time.time()
    g, e, ranks = grow(ham, gam[0], dtau, args.grow, rots, options=opts)
    torch.cuda.synchronize()
    wall = time.time() - t0
    e = e.cpu().numpy()
    ctx = SGS([ham], [g], options=opts)
    var = ctx.observables(SGS_OBS_VARIANCE, [0], [], 3).cpu().numpy()
    st = ctx.status()
    ctx.close()
    if st != 0:
        raise SystemExit(f"device status {st} in the protocol")
    steps = len(ranks)
    pairs = sum(r * (r - 1) // 2 for r in ranks)
    out = {
        "metric": "rank-growing protocol",
        "config": {"workload": args.config, "steps_per_rank": args.grow, "ranks": [1, R], "dtau": dtau,
                   "weights": args.weight, "rotation_norm": 0.3},
        "wall_s": wall,
        "steps": steps,
        "pair_evals": pairs,
        "pair_evals_per_s": pairs / wall,
        "E_per_rank_end": [float(e[(r + 1) * args.grow - 1]) for r in range(R)],
        "E_final": float(e[-1]),
        "variance_final": {"E": float(var[0]), "H2": float(var[1]), "delta_H2": float(var[2])},
        "note": "wall clock of the whole protocol, including one context set-up per rank",
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

