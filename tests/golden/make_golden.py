"""Write the stored expected values under tests/golden/ from the oracle only.

Run from the repository root:

    python tests/golden/make_golden.py small        # anderson_L7.json (seconds)
    python tests/golden/make_golden.py traj400      # anderson_L99_R16_traj500.json (hours)
    python tests/golden/make_golden.py step800      # anderson_L199_R32_U1_step.json (minutes)
    python tests/golden/make_golden.py step1204     # tck_L150_R24_J0.3_step.json (minutes)
    python tests/golden/make_golden.py cond800      # adds phase-matrix conditions (minutes)
    python tests/golden/make_golden.py cond1204
    python tests/golden/make_golden.py big          # big_steps.json: n = 1604, 2500, 4096 (minutes)

Each value records the oracle routine that produced it and the passage of
Boutin & Bauer (arXiv:2105.01088) it follows.  Inputs come from sgs_inputs
(seeded states and model Hamiltonians); every number is computed by oracle/.
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import sgs_inputs as si  # noqa: E402
from oracle import ed, sgs  # noqa: E402

HERE = os.path.join(ROOT, "tests", "golden")
STEP_CITE = "Eqs. (eigLambda), (EOM-Gamma3), (RKstep), (CM-normal-form)"


def small():
    out = {}
    # Anderson impurity, L = 7 bath sites per spin (N = 16 modes): even-sector ED
    # bound for the variational energies (Sec. III.C: energy descent; Sec. II.C).
    N, terms = si.anderson_terms(7, 1.0, 0.5)
    out["anderson_L7_U1_V0.5_ed_even"] = dict(
        value=ed.even_sector_ground_energy(N, terms),
        source="oracle.ed.even_sector_ground_energy", cite="Sec. IV model, even parity sector")
    # the seeded R = 4 trajectory (printed weights, dtau = 0.05): the first 10
    # step energies, and all 200 of the configured run
    ham, gam, cfg = si.config_problem("anderson_L7_R4")
    _, es = sgs.run(ham, gam, 0.05, 200)
    out["anderson_L7_R4_seed0_first10_E"] = dict(
        value=[float(x) for x in es[:10]], source="oracle.sgs.run", cite=STEP_CITE)
    out["anderson_L7_R4_seed0_200_E"] = dict(
        value=[float(x) for x in es], source="oracle.sgs.run (200 steps, printed weights)", cite=STEP_CITE)
    with open(os.path.join(HERE, "anderson_L7.json"), "w") as f:
        json.dump(out, f, indent=1)


def traj400(steps=500):
    """Energies of the 500-step benchmark trajectory (n = 400, R = 16, unit
    weights), with the final states' sampled entries."""
    ham, gam, cfg = si.config_problem("anderson_L99_R16")
    hp = ham.poly()
    es = []
    g = gam
    t0 = time.time()
    for k in range(steps):
        r = sgs.step(ham, g, 0.05, mode="unit", hpoly=hp)
        es.append(float(r.E))
        g = r.gammas
        print(f"step {k} E={r.E:.15f} t={time.time() - t0:.0f}s", flush=True)
    E_end, _, _ = sgs.energy(ham, g, hpoly=hp)
    out = dict(workload="anderson_L99_R16", weights="unit", dtau=0.05, steps=steps,
               source="oracle.sgs.step (unit weights), oracle.sgs.energy", cite=STEP_CITE,
               energies=es, E_end=float(E_end))
    out.update(_samples(g, seed=400))
    with open(os.path.join(HERE, "anderson_L99_R16_traj500.json"), "w") as f:
        json.dump(out, f)


def _samples(g, seed, count=4096):
    R, n, _ = g.shape
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, R, count), rng.integers(0, n, count), rng.integers(0, n, count)], axis=1)
    return dict(sample_idx=idx.tolist(), sample_val=[float(g[m, i, j]) for m, i, j in idx])


def one_step(name, seed):
    """Tables, energy and the new states (sampled entries, per-state norms of
    the change) of one step from the seeded states of a full-size workload."""
    ham, gam, cfg = si.config_problem(name)
    t0 = time.time()
    r = sgs.step(ham, gam, 0.05, mode="unit")
    print(f"{name}: one step in {time.time() - t0:.0f} s, E = {r.E}", flush=True)
    tab = r.tables
    out = dict(workload=name, weights="unit", dtau=0.05,
               source="oracle.sgs.step (unit weights)", cite=STEP_CITE,
               E=float(r.E), logabs=tab.logabs.tolist(), arg=tab.arg.tolist(),
               eps_re=tab.eps.real.tolist(), eps_im=tab.eps.imag.tolist(),
               dgamma_max=float(np.abs(r.dgamma).max()),
               change_norm=[float(np.linalg.norm(r.gammas[m] - gam[m])) for m in range(gam.shape[0])])
    out.update(_samples(r.gammas, seed=seed))
    out["phase_cond"] = phase_conditions(gam)
    with open(os.path.join(HERE, f"{name}_step.json"), "w") as f:
        json.dump(out, f)


BIG_CASES = [  # (L, R, eps, seed): n = 4 (L + 1) Majoranas
    (400, 3, 1.5, 61),    # n = 1604: panel shapes of 1536 < n <= 2048
    (624, 3, 1.5, 62),    # n = 2500: shapes above 2048
    (1023, 2, 1.5, 63),   # n = 4096, N = 2048: the largest problem the library takes
]


def big_steps():
    """One step (unit weights) at the largest sizes, from rotated near-copy
    states (overlaps of order one, so every amplitude is well defined): E,
    the tables and sampled entries of the new states."""
    out = {"source": "oracle.sgs.step (unit weights)", "cite": STEP_CITE, "cases": []}
    for L, R, eps, seed in BIG_CASES:
        ham = si.anderson(L, 1.0, 0.5)
        gam = si.near_copy_states(ham.N, R, eps, seed=seed)
        t0 = time.time()
        r = sgs.step(ham, gam, 0.05, mode="unit")
        tab = r.tables
        print(f"n = {ham.n}, R = {R}: one step in {time.time() - t0:.0f} s, E = {r.E}, "
              f"cond(G) = {np.linalg.cond(tab.G):.2e}", flush=True)
        case = dict(L=L, R=R, eps=eps, seed=seed, n=ham.n, E=float(r.E),
                    logabs=tab.logabs.tolist(), arg=tab.arg.tolist(),
                    eps_re=tab.eps.real.tolist(), eps_im=tab.eps.imag.tolist(),
                    dgamma_max=float(np.abs(r.dgamma).max()))
        case.update(_samples(r.gammas, seed=seed, count=2048))
        case["phase_cond"] = phase_conditions(gam)
        out["cases"].append(case)
    with open(os.path.join(HERE, "big_steps.json"), "w") as f:
        json.dump(out, f)


def phase_conditions(gam):
    """2-norm condition number of every matrix C_ab (1 <= a < b) whose Pfaffian
    gives the phase of G_ab (Schur-reduced triple product, Sec. II.B):
    [[a, b, cond], ...]; a phase computed by elimination is accurate to about
    n cond eps."""
    from oracle import gaussian as ga
    R = gam.shape[0]
    out = []
    for a in range(1, R):
        for b in range(a + 1, R):
            c = ga.schur_matrix(gam[0], gam[a], gam[b])
            out.append([a, b, float(np.linalg.cond(c))])
    return out


def add_phase_conditions(name):
    """Add phase_cond to an existing one-step golden (same states)."""
    path = os.path.join(HERE, f"{name}_step.json")
    with open(path) as f:
        out = json.load(f)
    ham, gam, cfg = si.config_problem(name)
    out["phase_cond"] = phase_conditions(gam)
    with open(path, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "small"
    if what == "small":
        small()
    elif what == "traj400":
        traj400()
    elif what == "step800":
        one_step("anderson_L199_R32_U1", seed=800)
    elif what == "step1204":
        one_step("tck_L150_R24_J0.3", seed=1204)
    elif what == "cond800":
        add_phase_conditions("anderson_L199_R32_U1")
    elif what == "cond1204":
        add_phase_conditions("tck_L150_R24_J0.3")
    elif what == "big":
        big_steps()
    else:
        raise SystemExit(f"unknown golden: {what}")
