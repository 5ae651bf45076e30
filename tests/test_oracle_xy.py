"""Pins of the XY oracle (oracle/xy_oracle.c): its Ising restriction
against the Ising oracle, the direction of the energy change (annealing),
the infinite-temperature limit, exact sampling on the 2x2 torus against
the Bessel-function closed form of a four-spin XY ring, and the trial and
random-start counter maps (with their 53-bit uniforms) recomputed through
PyTorch's independent Philox engine."""
import math

import numpy as np
import pytest
from scipy.special import iv

import oracle

BETA_XY = 1.0 / 0.85  # the paper's T = 0.85


def test_ising_restriction_reproduces_the_ising_energy():
    """theta in {0, pi}: cos(theta_i - theta_j) = s_i s_j exactly."""
    rng = np.random.default_rng(1)
    for L in (4, 6, 16):
        s = rng.choice(np.array([-1, 1], np.int8), size=(L, L))
        theta = np.where(s > 0, 0.0, np.pi)
        assert oracle.xy_energy(theta) == oracle.measure(s)[0]


def test_ground_state_energy_and_annealing():
    L = 8
    assert oracle.xy_energy(np.full((L, L), 1.234)) == pytest.approx(-2 * L * L, abs=1e-12)
    th = oracle.xy_init(L, 1, 5, 0)
    E, _ = oracle.xy_sweep(th, 5, 0, 0, 400, 20.0)
    # the chain descends towards -2N at low temperature (a wrong sign of dE
    # would climb towards +2N)
    assert E[-1] < -1.8 * L * L
    assert E[-1] < E[0]


def test_infinite_temperature_accepts_everything():
    L = 6
    th = oracle.xy_init(L, 0, 3, 0)
    E, acc = oracle.xy_sweep(th, 3, 0, 0, 2000, 0.0)
    assert acc == 2000 * L * L
    assert abs(E.mean()) < 4 * np.sqrt(2 * L * L / 2 / len(E)) + 0.05


def _ring_mean_energy(beta):
    """2x2 torus = ring of 4 spins with doubled bonds (J = 2):
    Z = (2 pi)^4 sum_m I_m(K)^4, K = 2 beta; <E> = -dlnZ/dbeta."""
    K = 2.0 * beta
    m = np.arange(-60, 61)
    I = iv(m, K)
    dI = 0.5 * (iv(m - 1, K) + iv(m + 1, K))
    return -2.0 * (4 * I ** 3 * dI).sum() / (I ** 4).sum()


@pytest.mark.parametrize("beta", [0.5, BETA_XY])
def test_two_by_two_torus_samples_exactly(beta):
    th = oracle.xy_init(2, 1, 7, 0)
    n = 400000
    E, _ = oracle.xy_sweep(th, 7, 0, 0, n, beta)
    x = E[1000:]
    blocks = x[: len(x) // 50 * 50].reshape(50, -1).mean(axis=1)
    err = blocks.std(ddof=1) / np.sqrt(50)
    exact = _ring_mean_energy(beta)
    assert abs(blocks.mean() - exact) < 4 * err, (blocks.mean(), exact, err)


# ---------------------------------------------------------------------------
# Counter maps of the XY draws, recomputed through PyTorch's own Philox
# engine (conftest.py), with the 53-bit uniforms built here from the raw
# words: the top 53 bits of (hi << 32 | lo) scaled by 2^-53, the angle
# being that uniform times the double nearest 2 pi.

TWO_PI = 2.0 * math.pi


def _u53(hi, lo):
    return float(((int(hi) << 32) | int(lo)) >> 11) * 2.0 ** -53


def test_random_start_counter_layout(torch_philox):
    """theta_n = u53(out[0], out[1]) 2 pi of the block (n, lattice, 0, 9)."""
    L, seed, lid = 6, (9 << 32) | 5, 4
    th = oracle.xy_init(L, 1, seed, lid).reshape(-1)
    ref = torch_philox([[seed & 0xFFFFFFFF, seed >> 32, n, lid, 0, 9] for n in range(L * L)])
    want = np.array([_u53(o[0], o[1]) * TWO_PI for o in ref])
    assert (th == want).all()  # exact: one product of two doubles each
    assert (oracle.xy_init(L, 0, seed, lid) == 0.0).all()


@pytest.mark.parametrize("c,t", [(0, 0), (1, 3), (0, 1000)])
def test_trial_counter_layout(torch_philox, c, t):
    """The trial of site n in half-sweep 2t + c uses the block (n >> 1,
    lattice, 2t + c, 8): theta' = u53(out[0], out[1]) 2 pi, p = u53(out[2],
    out[3]); theta <- theta' iff p < exp(-beta dE) with dE = -sum over the
    right, left, down and up neighbours of cos(theta' - nb) - cos(theta - nb)
    (libm cos and exp, one rounding per operation, as in the oracle).  Sites
    of one colour do not neighbour each other, so every trial sees the
    state before the half-sweep."""
    L, seed, lid, beta = 6, (2 << 32) | 123, 7, 1.0 / 0.85
    th0 = oracle.xy_init(L, 1, 31, lid)
    want = th0.copy()
    moved = kept = 0
    sites = [(y, x) for y in range(L) for x in range(L) if (x + y) % 2 == c]
    ref = torch_philox([[seed & 0xFFFFFFFF, seed >> 32, (y * L + x) >> 1, lid, 2 * t + c, 8]
                        for y, x in sites])
    for (y, x), o in zip(sites, ref):
        th_new = _u53(o[0], o[1]) * TWO_PI
        p = _u53(o[2], o[3])
        th = float(th0[y, x])
        nbs = (th0[y, (x + 1) % L], th0[y, (x - 1) % L], th0[(y + 1) % L, x], th0[(y - 1) % L, x])
        d = 0.0
        for nb in nbs:
            d += math.cos(th_new - float(nb)) - math.cos(th - float(nb))
        if p < math.exp(-beta * -d):
            want[y, x] = th_new
            moved += 1
        else:
            kept += 1
    assert moved > 2 and kept > 2
    th = th0.copy()
    acc = oracle.xy_halfsweep(th, c, seed, lid, t, beta)
    assert acc == moved
    assert (th == want).all()
