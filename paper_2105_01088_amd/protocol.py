"""Rank-growing protocol of Sec. III.C on the GPU.

Starting from one Gaussian state (the mean-field, GHF, solution is its
fixed point), run a number of imaginary-time steps, then add one state: a
random special orthogonal transformation Q, close to the identity, of the
current state with the largest amplitude |lambda_a|; repeat.  Adding the
states one at a time keeps the optimal amplitudes from vanishing (Sec.
III.C).  Every step and every new state run in the library (sgs_step,
sgs_energy, sgs_rotate); the rotations are inputs, drawn by the caller.
"""

from __future__ import annotations

from typing import Optional, Sequence

from ._lib import SGS, default_options, rotate_state


def grow(ham, gamma0, dtau: float, steps_per_rank: int, rotations: Sequence, options=None,
         device: str = "cuda:0"):
    """Run the protocol: steps_per_rank steps at rank 1, then one more state
    per rotation in `rotations` (n x n special orthogonal, host or device)
    and steps_per_rank steps at each new rank.

    Returns (states: device (R, n, n) tensor, energies: device tensor of the
    energy of the states entering every step, ranks: list of the rank of
    every step)."""
    import torch

    g = torch.as_tensor(gamma0, dtype=torch.float64).to(device)
    if g.dim() == 2:
        g = g[None]
    opts = options if options is not None else default_options()
    energies, ranks = [], []
    for r in range(len(rotations) + 1):
        ctx = SGS([ham], [g], options=opts, device=device)
        energies.append(ctx.step(dtau, steps_per_rank))
        ranks += [g.shape[0]] * steps_per_rank
        g = ctx.gammas(0).clone()
        if r < len(rotations):
            _, lam = ctx.energy()
            lam = lam.view(-1, 2)
            a = int(torch.argmax(lam[:, 0] ** 2 + lam[:, 1] ** 2).item())
            q = torch.as_tensor(rotations[r], dtype=torch.float64).to(device)
            g = torch.cat([g, rotate_state(q, g[a], ctx.stream)[None]])
        ctx.close()
    return g, torch.cat(energies), ranks
