"""Write the stored expected values under tests/golden/ from the oracle only.

Run from the repository root:  python tests/golden/make_golden.py
Each value records the oracle routine that produced it and the passage of
Boutin & Bauer (arXiv:2105.01088) it follows.
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import sgs_inputs as si  # noqa: E402
from oracle import ed, sgs  # noqa: E402


def main():
    out = {}
    # Anderson impurity, L = 7 bath sites per spin (N = 16 modes): even-sector ED
    # bound for the variational energies (Sec. III.C: energy descent; Sec. II.C).
    N, terms = si.anderson_terms(7, 1.0, 0.5)
    out["anderson_L7_U1_V0.5_ed_even"] = dict(
        value=ed.even_sector_ground_energy(N, terms),
        source="oracle.ed.even_sector_ground_energy", cite="Sec. IV model, even parity sector")
    # first 10 step energies of the seeded R = 4 trajectory (printed weights, dtau = 0.05)
    ham, gam, cfg = si.config_problem("anderson_L7_R4")
    _, es = sgs.run(ham, gam, 0.05, 10)
    out["anderson_L7_R4_seed0_first10_E"] = dict(
        value=[float(x) for x in es], source="oracle.sgs.run",
        cite="Eqs. (eigLambda), (EOM-Gamma3), (RKstep), (CM-normal-form)")
    with open(os.path.join(ROOT, "tests", "golden", "anderson_L7.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
