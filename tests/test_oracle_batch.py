"""Pins of the oracle's batch functions (moments of a chain segment, and a
batch as independent per-lattice chains)."""
import numpy as np

import oracle
from paper_2402_06415_amd.workloads import batched_workload


def test_moments_beta_zero_closed_form_needs_128_bits():
    """At beta = 0 every site flips every half-sweep, so from the cold start
    of an L x L lattice E stays -2N and M alternates -N, +N, ...  With L = 256,
    N^4 = 2^64: the M^4 sum exceeds 64 bits after one sweep."""
    L, n = 256, 3
    N = L * L
    s = oracle.init(L, oracle.START_COLD_UP, 5)
    E, M = oracle.sweep(s, oracle.MODE_SITE, 5, 0, 0, n, 0.0, nthreads=4)
    m = oracle.moments(E, M)
    assert m["E"] == -2 * N and m["M"] == -N
    assert m["sum_E"] == -2 * N * n and m["sum_E2"] == 4 * N * N * n
    assert m["sum_absM"] == N * n and m["sum_M2"] == N * N * n
    assert m["sum_M4"] == n * 2 ** 64


def test_moments_of_split_segments_add_up():
    s = oracle.init(16, oracle.START_RANDOM, 3)
    E1, M1 = oracle.sweep(s, oracle.MODE_SITE, 3, 0, 0, 40, 0.44)
    E2, M2 = oracle.sweep(s, oracle.MODE_SITE, 3, 0, 40, 25, 0.44)
    a, b = oracle.moments(E1, M1), oracle.moments(E2, M2)
    ab = oracle.moments(np.concatenate([E1, E2]), np.concatenate([M1, M2]))
    for k in ("sum_E", "sum_E2", "sum_absM", "sum_M2", "sum_M4"):
        assert a[k] + b[k] == ab[k]
    assert ab["E"] == b["E"] and ab["M"] == b["M"]


def test_batch_is_independent_chains_with_consecutive_ids():
    """Lattice j of a batch is the chain of lattice id lattice_id0 + j; the
    order and company of the other lattices does not matter."""
    Ls, betas, seed = [8, 16, 24], [0.3, 0.44, 0.6], 11
    states = [oracle.init(L, oracle.START_RANDOM, seed, 7 + j) for j, L in enumerate(Ls)]
    got = oracle.batch_sweep(states, betas, seed, 7, 0, 12)
    alone = oracle.init(16, oracle.START_RANDOM, seed, 8)
    E, M = oracle.sweep(alone, oracle.MODE_SITE, seed, 8, 0, 12, 0.44)
    assert got[1] == oracle.moments(E, M)
    assert (states[1] == alone).all()
    # a batch of one (the third lattice alone, same id) gives the same chain
    third = oracle.init(24, oracle.START_RANDOM, seed, 9)
    assert oracle.batch_sweep([third], [0.6], seed, 9, 0, 12)[0] == got[2]
    assert (third == states[2]).all()


def test_batched_workload_recipe():
    L, beta = batched_workload()
    assert len(L) == 1024 and set(np.unique(L)) == {32, 64, 128, 256}
    assert beta[0] == 0.30 and abs(beta[63] - 0.60) < 1e-15 and beta[64] == beta[0]
    assert len(np.unique(beta)) == 64
    L2, beta2 = batched_workload()
    assert (L == L2).all() and (beta == beta2).all()
