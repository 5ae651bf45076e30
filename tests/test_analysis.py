"""Pins of the autocorrelation analysis against processes whose
integrated autocorrelation time is known in closed form."""
import numpy as np
import pytest

from paper_2402_06415_amd.analysis import autocorrelation, binned_mean, tau_int


def _ar1(rho, T, chains, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((T, chains))
    e = rng.normal(size=(T, chains)) * np.sqrt(1 - rho * rho)
    x[0] = rng.normal(size=chains)
    for t in range(1, T):
        x[t] = rho * x[t - 1] + e[t]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9, 0.98])
def test_tau_int_of_ar1(rho):
    """AR(1): rho(t) = rho^t, so tau = 1/2 + rho/(1-rho) = (1+rho)/(2(1-rho))."""
    x = _ar1(rho, 40000, 16, 3)
    tau, err, W = tau_int(x)
    exact = (1 + rho) / (2 * (1 - rho))
    assert abs(tau - exact) < max(4 * err, 0.02 * exact), (tau, err, exact)


def test_autocorrelation_of_ar1_decays_geometrically():
    x = _ar1(0.8, 50000, 8, 4)
    r = autocorrelation(x)
    assert abs(r[0] - 1) < 1e-12
    assert np.allclose(r[1:6], 0.8 ** np.arange(1, 6), atol=0.01)


def test_binned_mean_error_of_white_noise():
    x = np.random.default_rng(5).normal(2.0, 1.0, (64000, 4))
    m, e = binned_mean(x)
    assert abs(e - 1 / np.sqrt(x.size)) < 0.3 / np.sqrt(x.size)
    assert abs(m - 2.0) < 5 * e
