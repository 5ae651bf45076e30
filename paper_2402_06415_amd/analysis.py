"""Host-side analysis of Monte Carlo time series: integrated
autocorrelation times and binned errors (numpy).  Used to turn chain
throughput into independent samples per second."""
from __future__ import annotations

import numpy as np


def autocorrelation(x: np.ndarray) -> np.ndarray:
    """Normalised autocorrelation rho(t), t = 0..T-1, of series x [T] or of
    several chains x [T, chains] (averaged over chains), by FFT."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    T = x.shape[0]
    d = x - x.mean(axis=0)
    f = np.fft.rfft(d, n=2 * T, axis=0)
    acf = np.fft.irfft(f * np.conj(f), axis=0)[:T].mean(axis=1)
    acf /= np.arange(T, 0, -1)
    return acf / acf[0] if acf[0] > 0 else np.zeros(T)


def tau_int(x: np.ndarray, c: float = 6.0):
    """Integrated autocorrelation time tau = 1/2 + sum_{t>=1} rho(t) with
    Sokal's automatic window (the smallest W with W >= c tau(W)), and the
    Madras-Sokal error tau sqrt(2 (2W + 1) / T).  Returns (tau, error, W);
    the units are those of the series' time step."""
    rho = autocorrelation(x)
    T = len(rho)
    tau = 0.5
    W = 0
    for W in range(1, T):
        tau += rho[W]
        if W >= c * tau:
            break
    n = np.asarray(x).shape[0] * (np.asarray(x).shape[1] if np.asarray(x).ndim > 1 else 1)
    err = tau * np.sqrt(2.0 * (2 * W + 1) / n)
    return float(tau), float(err), int(W)


def binned_mean(x: np.ndarray, bins: int = 32):
    """Mean of x [T] or [T, chains] and its error from `bins` consecutive
    blocks of the time axis (chains averaged inside each block)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    T = (x.shape[0] // bins) * bins
    b = x[:T].reshape(bins, -1).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / np.sqrt(bins))
