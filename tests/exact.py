"""Independent exact results for the 2D Ising model used to pin the oracle.

Nothing here calls the oracle or the HIP library.  Sources:
  - brute-force enumeration of all 2^(L*L) states of a small periodic lattice;
  - Kaufman (1949), partition function of the finite m x n torus, in the form
    Z = 1/2 (2 sinh 2K)^(mn/2) (Z1 + Z2 + Z3 + Z4) with
    cosh g_l = cosh 2K coth 2K - cos(l pi / n) (l >= 1), g_0 = 2K + ln tanh K
    (as written out by Beale, PRL 76, 78 (1996));
  - Onsager (1944), energy per site of the infinite lattice;
  - Yang (1952), spontaneous magnetisation (1 - sinh(2K)^-4)^(1/8).
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np
from scipy import special

BETA_C = float(mp.log(1 + mp.sqrt(2)) / 2)


# ----------------------------------------------------------------- enumeration
@functools.lru_cache(maxsize=4)
def enumerate_states(L: int):
    """All states of an L x L periodic lattice: (E[2^N], M[2^N]) as int64.

    Bit j of the state index is the spin at site j = y*L + x (1 -> -1)."""
    N = L * L
    assert N <= 20
    idx = np.arange(1 << N, dtype=np.int64)
    bits = ((idx[:, None] >> np.arange(N, dtype=np.int64)[None, :]) & 1).astype(np.int8)
    s = (1 - 2 * bits).reshape(-1, L, L)
    E = -(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    return E.astype(np.int64), M.astype(np.int64)


def enumeration_moments(L: int, beta: float):
    """Exact <e>, <e^2>, <|m|>, <m^2>, <m^4> per site by enumeration."""
    E, M = enumerate_states(L)
    N = L * L
    w = np.exp(-beta * (E - E.min()).astype(np.float64))
    Z = w.sum()
    e = E / N
    m = M / N
    return {
        "e": float((w * e).sum() / Z),
        "e2": float((w * e * e).sum() / Z),
        "absm": float((w * np.abs(m)).sum() / Z),
        "m2": float((w * m * m).sum() / Z),
        "m4": float((w * m ** 4).sum() / Z),
    }


def density_of_states(L: int):
    E, _ = enumerate_states(L)
    vals, counts = np.unique(E, return_counts=True)
    return dict(zip(vals.tolist(), counts.tolist()))


# -------------------------------------------------------------------- Kaufman
def kaufman_logZ(K, m: int, n: int):
    """ln Z of the m x n periodic Ising lattice at coupling K (mpmath)."""
    K = mp.mpf(K)
    c = mp.cosh(2 * K) / mp.tanh(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + mp.log(mp.tanh(K))
        return mp.acosh(c - mp.cos(mp.pi * l / n))

    z1 = z2 = z3 = z4 = mp.mpf(1)
    for k in range(n):
        g_odd = gamma(2 * k + 1)
        g_even = gamma(2 * k)
        z1 *= 2 * mp.cosh(m * g_odd / 2)
        z2 *= 2 * mp.sinh(m * g_odd / 2)
        z3 *= 2 * mp.cosh(m * g_even / 2)
        z4 *= 2 * mp.sinh(m * g_even / 2)
    pref = (2 * mp.sinh(2 * K)) ** (mp.mpf(m * n) / 2) / 2
    return mp.log(pref * (z1 + z2 + z3 + z4))


def kaufman_energy(beta: float, L: int, dps: int = 40) -> float:
    """Exact <H>/N on the L x L torus: -(1/N) d ln Z / dK."""
    with mp.workdps(dps):
        d = mp.diff(lambda k: kaufman_logZ(k, L, L), mp.mpf(beta))
        return float(-d / (L * L))


def kaufman_specific_heat(beta: float, L: int, dps: int = 40) -> float:
    """c = beta^2 N (<e^2> - <e>^2) = (beta^2/N) d^2 ln Z / dK^2."""
    with mp.workdps(dps):
        d2 = mp.diff(lambda k: kaufman_logZ(k, L, L), mp.mpf(beta), 2)
        return float(mp.mpf(beta) ** 2 * d2 / (L * L))


# -------------------------------------------------------------------- Onsager
def onsager_energy(beta: float) -> float:
    """Energy per site of the infinite square lattice (J = 1)."""
    t2 = np.tanh(2 * beta)
    kappa = 2 * np.sinh(2 * beta) / np.cosh(2 * beta) ** 2
    K1 = special.ellipk(kappa * kappa)  # scipy takes the parameter m = k^2
    return float(-(1 / t2) * (1 + (2 / np.pi) * (2 * t2 * t2 - 1) * K1))


# ----------------------------------------------------------------------- Yang
def yang_magnetisation(beta: float) -> float:
    if beta <= BETA_C:
        return 0.0
    return float((1 - np.sinh(2 * beta) ** -4) ** 0.125)


# -------------------------------------------------------- series statistics
def binned_mean_error(x: np.ndarray, nbins: int = 32):
    """Mean and its standard error from nbins contiguous bins (autocorrelated data)."""
    x = np.asarray(x, dtype=np.float64)
    nb = len(x) // nbins
    means = x[: nb * nbins].reshape(nbins, nb).mean(axis=1)
    return float(x.mean()), float(means.std(ddof=1) / np.sqrt(nbins))
