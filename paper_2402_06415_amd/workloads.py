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


def ea_bonds(L: int, seed: int = 3) -> np.ndarray:
    """Couplings of the 3D Edwards-Anderson +-J glass: int8 [3, L, L, L]
    (axis d = x, y, z; index [d, z, y, x]), i.i.d. +1 / -1 with p = 1/2 from
    numpy's Philox generator keyed by `seed`."""
    rng = np.random.Generator(np.random.Philox(seed))
    return (2 * rng.integers(0, 2, size=(3, L, L, L), dtype=np.int8) - 1).astype(np.int8)


def ea_workload(replicas: int = 64, L: int = 128):
    """The spin-glass study: cubic L = 128, bonds from seed 3, 64 replicas
    at beta_k = 0.5 + 0.7 k / 63 (uniform in [0.5, 1.2]), replica exchange
    every 10 sweeps, 10^4 sweeps, random starts (seed 3, replica id r)."""
    beta = 0.5 + 0.7 * np.arange(replicas, dtype=np.float64) / max(replicas - 1, 1)
    return {"L": L, "beta": beta, "bond_seed": 3, "seed": 3, "every": 10, "sweeps": 10_000}
