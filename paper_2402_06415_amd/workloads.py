"""Seeded synthetic inputs of the benchmark and test workloads.

Recipes only: which lattice sides, temperatures, seeds and ids a workload
uses.  Nothing here computes any part of the Monte Carlo method; both the
HIP path and the CPU oracle take their inputs from these recipes.
"""
from __future__ import annotations

import numpy as np

BETA_C = 0.4406868  # critical coupling used by the single-lattice workloads


def batched_workload(count: int = 1024, seed: int = 11):
    """Many independent 2D lattices of uneven size on a grid of
    temperatures: sides drawn uniformly from {32, 64, 128, 256} (numpy's
    Philox generator keyed by `seed`), beta_k = 0.30 + 0.30 k / 63 for
    k = 0..63 and lattice j at beta_{j mod 64}.  Random starts use the same
    seed and lattice id j.  Returns (L, beta) as numpy arrays."""
    rng = np.random.Generator(np.random.Philox(seed))
    L = rng.choice(np.array([32, 64, 128, 256], dtype=np.int32), size=count)
    grid = 0.30 + 0.30 * np.arange(64, dtype=np.float64) / 63.0
    beta = grid[np.arange(count) % 64]
    return L.astype(np.int32), beta


# masked-convolution proposal network: (in, out, taps) of its four layers
_NN_LAYERS = ((1, 16, 4), (16, 16, 5), (16, 16, 5), (16, 1, 5))


def nn_initial_params(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Seeded float32 starting parameters of the 16-channel proposal network
    (flat, per layer W[out][in][tap] then b[out]): weights normal with
    variance scale^2 / fan-in, biases zero."""
    rng = np.random.Generator(np.random.Philox(seed))
    out = []
    for ci, co, nt in _NN_LAYERS:
        out.append(rng.normal(0.0, scale / np.sqrt(ci * nt), co * ci * nt))
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def learned_workload():
    """The learned-proposal study: L = 32 at beta in {0.40, 0.4406868, 0.48}
    (1024 chains per beta); training sets of 10^5 configurations drawn from
    the plain sampler; one whole-lattice proposal per 10 sweeps."""
    return {"L": 32, "betas": (0.40, 0.4406868, 0.48), "chains": 1024, "train_configs": 100_000,
            "sweeps_per_proposal": 10}
