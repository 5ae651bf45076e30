"""Pins of the oracle's Markov chain against exact results and invariants.

The chain must sample the Boltzmann distribution of H = -sum s_i s_j (Eq. (1)
of the paper restricted to theta in {0, pi}).  Statistical checks compare
time averages (binned error bars, first 10% discarded) with:
  - exact enumeration of the 4x4 torus (2^16 states),
  - Kaufman's finite-torus energy at L = 16 and L = 64,
  - Onsager's infinite-lattice energy deep in the disordered phase,
  - Yang's spontaneous magnetisation deep in the ordered phase.
Exact invariants: beta = 0 flips every spin every half-sweep; the chain is
odd under s -> -s for a fixed stream of draws; split sweeps equal one call;
the running E and M equal full recounts; threads do not change a bit.
"""
import numpy as np
import pytest

import exact
import oracle

BC = 0.4406868
SITE, PLANE = oracle.MODE_SITE, oracle.MODE_PLANE


def _series(L, mode, seed, beta, n, start=oracle.START_COLD_UP, nthreads=4):
    s = oracle.init(L, start, seed)
    E, M = oracle.sweep(s, mode, seed, 0, 0, n, beta, nthreads=nthreads)
    cut = n // 10
    N = L * L
    return E[cut:] / N, M[cut:] / N, s


def _close(x, want, nsig=4.5, nbins=32):
    mean, err = exact.binned_mean_error(x, nbins)
    assert abs(mean - want) < nsig * err + 1e-12, (mean, want, err)
    return mean, err


@pytest.mark.parametrize("beta", [0.3, BC, 0.6])
def test_4x4_matches_enumeration(beta):
    ex = exact.enumeration_moments(4, beta)
    e, m, _ = _series(4, SITE, 11, beta, 200_000)
    _close(e, ex["e"])
    _close(e * e, ex["e2"])
    _close(np.abs(m), ex["absm"])
    _close(m * m, ex["m2"])


def test_4x4_energy_histogram_matches_boltzmann():
    beta = BC
    E_all, _ = exact.enumerate_states(4)
    w = np.exp(-beta * (E_all - E_all.min()).astype(np.float64))
    levels = np.unique(E_all)
    pE = {int(E): float(w[E_all == E].sum() / w.sum()) for E in levels}
    e, _, _ = _series(4, SITE, 3, beta, 200_000)
    Es = np.rint(e * 16).astype(np.int64)
    for E, p in pE.items():
        if p < 1e-3:
            continue
        _close((Es == E).astype(np.float64), p)


def test_L16_critical_energy_matches_kaufman():
    # The parity workload: L = 16, beta = 0.4406868, cold start.
    want = exact.kaufman_energy(BC, 16)  # -1.45306490...
    e, _, _ = _series(16, SITE, 1, BC, 100_000)
    mean, err = _close(e, want)
    # the test separates the finite-L value from the infinite-L one
    assert abs(exact.onsager_energy(BC) - want) > 8 * err


def test_L64_plane_mode_critical_energy_matches_kaufman():
    want = exact.kaufman_energy(BC, 64)
    e, _, _ = _series(64, PLANE, 7, BC, 20_000, start=oracle.START_RANDOM)
    _close(e, want, nbins=20)


def test_L32_plane_mode_critical_energy_matches_kaufman():
    # L % 64 == 32: every draw group spans two rows
    want = exact.kaufman_energy(BC, 32)
    e, _, _ = _series(32, PLANE, 11, BC, 40_000, start=oracle.START_RANDOM)
    _close(e, want, nbins=20)


def test_L64_disordered_energy_matches_onsager():
    # xi(0.3) ~ 1.4 lattice spacings: the L = 64 torus is infinite to 1e-12
    want = exact.onsager_energy(0.3)
    e, _, _ = _series(64, PLANE, 5, 0.3, 4_000, start=oracle.START_RANDOM)
    _close(e, want)


@pytest.mark.parametrize("mode", [SITE, PLANE])
def test_L64_ordered_magnetisation_matches_yang(mode):
    want = exact.yang_magnetisation(0.6)  # 0.97360866...
    _, m, _ = _series(64, mode, 9, 0.6, 4_000)
    _close(np.abs(m), want)


@pytest.mark.parametrize("mode,L", [(SITE, 6), (SITE, 16), (PLANE, 64)])
def test_beta_zero_flips_every_spin(mode, L):
    s0 = oracle.init(L, oracle.START_RANDOM, 4)
    s = s0.copy()
    E0, M0 = oracle.measure(s0)
    E, M = oracle.sweep(s, mode, 4, 0, 0, 5, 0.0)
    # each half-sweep inverts one sublattice; a sweep inverts both
    assert (s == -s0).all()
    assert (E == E0).all()
    assert M.tolist() == [M0 * (-1) ** (j + 1) for j in range(5)]


@pytest.mark.parametrize("mode,L", [(SITE, 8), (SITE, 16), (PLANE, 64)])
def test_z2_symmetry_bit_exact(mode, L):
    s0 = oracle.init(L, oracle.START_RANDOM, 21)
    a, b = s0.copy(), (-s0).copy()
    Ea, Ma = oracle.sweep(a, mode, 21, 0, 0, 50, BC)
    Eb, Mb = oracle.sweep(b, mode, 21, 0, 0, 50, BC)
    assert (a == -b).all()
    assert (Ea == Eb).all() and (Ma == -Mb).all()


@pytest.mark.parametrize("mode,L", [(SITE, 16), (PLANE, 64)])
def test_split_sweeps_equal_one_call(mode, L):
    s0 = oracle.init(L, oracle.START_RANDOM, 3)
    a, b = s0.copy(), s0.copy()
    Ea, Ma = oracle.sweep(a, mode, 3, 0, 0, 30, BC)
    E1, M1 = oracle.sweep(b, mode, 3, 0, 0, 11, BC)
    E2, M2 = oracle.sweep(b, mode, 3, 0, 11, 19, BC)
    assert (a == b).all()
    assert (Ea == np.concatenate([E1, E2])).all()
    assert (Ma == np.concatenate([M1, M2])).all()


@pytest.mark.parametrize("mode,L", [(SITE, 10), (PLANE, 64)])
def test_running_observables_equal_recount(mode, L):
    s = oracle.init(L, oracle.START_RANDOM, 8)
    E, M = oracle.sweep(s.copy(), mode, 8, 0, 0, 40, BC)
    for j in range(40):
        oracle.sweep(s, mode, 8, 0, j, 1, BC, record=False)
        assert oracle.measure(s) == (E[j], M[j])


@pytest.mark.parametrize("mode,L", [(SITE, 64), (PLANE, 128)])
def test_threads_do_not_change_the_chain(mode, L):
    s0 = oracle.init(L, oracle.START_RANDOM, 13)
    a, b = s0.copy(), s0.copy()
    Ea, Ma = oracle.sweep(a, mode, 13, 0, 0, 20, BC, nthreads=1)
    Eb, Mb = oracle.sweep(b, mode, 13, 0, 0, 20, BC, nthreads=8)
    assert (a == b).all() and (Ea == Eb).all() and (Ma == Mb).all()


def test_lattice_id_and_seed_select_independent_streams():
    s0 = oracle.init(16, oracle.START_COLD_UP, 1)
    runs = []
    for seed, lid in ((1, 0), (2, 0), (1, 1)):
        s = s0.copy()
        oracle.sweep(s, SITE, seed, lid, 0, 20, BC)
        runs.append(s)
    assert (runs[0] != runs[1]).any() and (runs[0] != runs[2]).any()


@pytest.mark.parametrize("L,mode,t0,n", [(7, SITE, 0, 1), (2, SITE, 0, 1), (48, PLANE, 0, 1),
                                         (16, SITE, 0, -1), (16, SITE, 2 ** 31, 1),
                                         (16, SITE, 2 ** 31 - 1, 2)])
def test_sweep_rejects_bad_arguments(L, mode, t0, n):
    s = np.ones((L, L), dtype=np.int8)
    with pytest.raises(ValueError):
        oracle.sweep(s, mode, 1, 0, t0, n, BC)
