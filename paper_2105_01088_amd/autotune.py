"""Autotuner for the library's scheduling and blocking choices.

    python -m paper_2105_01088_amd.autotune [--out tuning.json] [--steps 3]
                                            [--config NAME ...]

For each workload (one per size bucket) it times imaginary-time steps on the
GPU while it varies one tuning field at a time over its candidates (coordinate
descent from the library's built-in choices: Gauss-Jordan super-panel width,
inverse order, Pfaffian super-panel depth, force term split and elementwise
placement, force tile edge, deferral of the Gauss-Jordan inner updates), keeps the fastest value of each field, and writes the rows as
JSON: {"rows": [{n_max, gj_super, ...}], "measured": {...}}.  The file is read
by paper_2105_01088_amd.default_options(tune=path) and bench.py --tune.
Every choice changes scheduling and blocking only; results agree with the
built-in choices to rounding (the parity tests cover every choice).
"""

from __future__ import annotations

import argparse
import json
import sys

CANDIDATES = {
    "gj_super": [64, 128, 256],
    "gj_first": [2, 1],
    "pf_super": [16, 24, 32],
    "force_split": [1, 2, 3],
    "force_elem": [1, 2],
    "force_tile": [64, 128],
    "gj_defer": [1, 2, 3],
}
DEFAULT_CONFIGS = ["anderson_L99_R16", "anderson_L199_R32_U1", "tck_L150_R24_J0.3"]


def time_steps(ham, gam, row, steps, warmup=1):
    """ms per step with the tuning row (unit weights, dtau = 0.05)."""
    import torch

    from . import SGS, default_options
    ctx = SGS([ham], [gam], options=default_options(weight=1, tune=[row]))
    ctx.step(0.05, warmup)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(ctx.stream)
    ctx.step(0.05, steps)
    t1.record(ctx.stream)
    torch.cuda.synchronize()
    st = ctx.status()
    ctx.close()
    if st != 0:
        raise RuntimeError(f"device status {st} with {row}")
    return t0.elapsed_time(t1) / steps


def tune_workload(name, steps, log=print):
    import sgs_inputs as si
    ham, gam, cfg = si.config_problem(name)
    n = ham.n
    best = {"n_max": n}
    best_ms = time_steps(ham, gam, best, steps)
    measured = {"built-in": best_ms}
    log(f"{name}: built-in {best_ms:.3f} ms/step")
    for field, values in CANDIDATES.items():
        for v in values:
            row = dict(best, **{field: v})
            ms = time_steps(ham, gam, row, steps)
            measured[f"{field}={v}"] = ms
            log(f"  {field}={v}: {ms:.3f} ms/step")
            if ms < best_ms * 0.995:  # keep a change only if it gains
                best, best_ms = row, ms
    log(f"  best {best} {best_ms:.3f} ms/step")
    return best, best_ms, measured


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="tuning.json")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--config", action="append", default=None)
    args = ap.parse_args(argv)
    configs = args.config or DEFAULT_CONFIGS
    rows, meas = [], {}
    for name in configs:
        best, ms, measured = tune_workload(name, args.steps)
        rows.append(best)
        meas[name] = {"best_ms_per_step": ms, "candidates_ms_per_step": measured}
    rows.sort(key=lambda r: r["n_max"])
    # each row covers the sizes up to the next bucket's workload
    for i in range(len(rows) - 1):
        rows[i]["n_max"] = (rows[i]["n_max"] + rows[i + 1]["n_max"]) // 2
    rows[-1]["n_max"] = 4096
    with open(args.out, "w") as f:
        json.dump({"rows": rows, "measured": meas}, f, indent=1)
    print(json.dumps({"rows": rows}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
