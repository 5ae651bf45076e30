"""Pins of the XY oracle (oracle/xy_oracle.c): its Ising restriction
against the Ising oracle, the direction of the energy change (annealing),
the infinite-temperature limit, and exact sampling on the 2x2 torus against
the Bessel-function closed form of a four-spin XY ring."""
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
