"""The benchmark workloads, as seeded synthetic inputs.

Each entry names a model Hamiltonian, its size, the rank R of the ansatz, the
number of imaginary-time steps and the step size.  The paper measures on model
Hamiltonians only (Secs. IV and V), so these synthetic inputs are the workloads
themselves, not stand-ins for a dataset.
"""

from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from .models import MajoranaHamiltonian, anderson, two_channel_kondo
from .states import random_states

CONFIGS: Dict[str, Dict[str, object]] = {
    # single-orbital Anderson impurity, N = 16 modes, n = 32 Majoranas
    "anderson_L7_R4": dict(model="anderson", L=7, U=1.0, V=0.5, R=4, steps=200, dtau=0.05, seed=0),
    # Anderson impurity, N = 200 modes, n = 400
    "anderson_L99_R16": dict(model="anderson", L=99, U=1.0, V=0.5, R=16, steps=500, dtau=0.05, seed=0),
    # precision path, N = 400 modes, n = 800 (U in {1, 2, 4})
    "anderson_L199_R32_U1": dict(model="anderson", L=199, U=1.0, V=0.4, R=32, steps=1000, dtau=0.05, seed=0),
    "anderson_L199_R32_U2": dict(model="anderson", L=199, U=2.0, V=0.4, R=32, steps=1000, dtau=0.05, seed=0),
    "anderson_L199_R32_U4": dict(model="anderson", L=199, U=4.0, V=0.4, R=32, steps=1000, dtau=0.05, seed=0),
    # two-channel Kondo, N = 602 modes, n = 1204 (J in {0.3, 0.5})
    "tck_L150_R24_J0.3": dict(model="tck", L=150, J=0.3, U=8.0, R=24, steps=1500, dtau=0.05, seed=0),
    "tck_L150_R24_J0.5": dict(model="tck", L=150, J=0.5, U=8.0, R=24, steps=1500, dtau=0.05, seed=0),
}


def config_problem(name_or_cfg, R: int | None = None,
                   seed: int | None = None) -> Tuple[MajoranaHamiltonian, np.ndarray, Dict[str, object]]:
    """Hamiltonian, initial states (R, n, n) and the config dict."""
    cfg = dict(CONFIGS[name_or_cfg]) if isinstance(name_or_cfg, str) else dict(name_or_cfg)
    if R is not None:
        cfg["R"] = R
    if seed is not None:
        cfg["seed"] = seed
    if cfg["model"] == "anderson":
        ham = anderson(int(cfg["L"]), float(cfg["U"]), float(cfg["V"]), float(cfg.get("t", 1.0)))
    elif cfg["model"] == "tck":
        ham = two_channel_kondo(int(cfg["L"]), float(cfg["J"]), float(cfg.get("U", 8.0)),
                                t=float(cfg.get("t", 1.0)))
    else:
        raise ValueError(cfg["model"])
    gam = random_states(ham.N, int(cfg["R"]), int(cfg["seed"]))
    return ham, gam, cfg


def batched_problems(seed: int = 0, count: int = 64,
                     L_range: Tuple[int, int] = (20, 300)) -> List[Tuple[MajoranaHamiltonian, np.ndarray, Dict[str, object]]]:
    """Independent Anderson problems of uneven size: L uniform in L_range
    (inclusive), U in [0.5, 4], V in [0.2, 0.8], t = 1, R in {4, 8, 16}.
    Parameters are drawn first, then each problem's states in order."""
    rng = np.random.default_rng(seed)
    params = []
    for _ in range(count):
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        U = float(rng.uniform(0.5, 4.0))
        V = float(rng.uniform(0.2, 0.8))
        R = int(rng.choice([4, 8, 16]))
        params.append(dict(model="anderson", L=L, U=U, V=V, R=R, dtau=0.05))
    out = []
    for p in params:
        ham = anderson(p["L"], p["U"], p["V"])
        gam = random_states(ham.N, p["R"], rng=rng)
        out.append((ham, gam, p))
    return out
