"""Pins of the learned-proposal oracle (oracle/nn.py) against mathematics
that does not come from the oracle itself: finite differences, exact
normalisation of an autoregressive model, sampling frequencies, Adam's
closed-form first step, and exact detailed balance of the independent
Metropolis-Hastings kernel."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import nn


def _params(C, seed, scale=0.5):
    return np.random.default_rng(seed).normal(0.0, scale, nn.param_count(C))


def _all_states(L):
    N = L * L
    bits = np.array(list(itertools.product([1, -1], repeat=N)), dtype=np.int8)
    return bits.reshape(-1, L, L)


def test_param_count():
    # 1*16*4+16 + 2*(16*16*5+16) + 16*5+1
    assert nn.param_count(16) == 80 + 2 * 1296 + 81


def test_gradient_matches_central_differences():
    C, L = 3, 5
    p = _params(C, 1)
    s = np.random.default_rng(2).choice(np.array([-1, 1], np.int8), size=(4, L, L))
    loss, g = nn.loss_and_grad(p, s, C)
    h = 1e-6
    idx = np.random.default_rng(3).choice(len(p), 40, replace=False)
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (nn.loss_and_grad(p + e, s, C)[0] - nn.loss_and_grad(p - e, s, C)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])
    assert abs(loss + nn.logq(p, s, C).mean()) < 1e-12


def test_model_is_normalised_and_autoregressive():
    """sum over all 2^9 states of q(s) = 1 holds only if each logit depends
    on earlier sites alone (a wrong mask breaks it)."""
    C, L = 4, 3
    p = _params(C, 5, 0.8)
    S = _all_states(L)
    q = np.exp(nn.logq(p, S, C))
    assert abs(q.sum() - 1.0) < 1e-12
    # changing site i (and later sites) leaves the logits at sites <= i unchanged
    s = S[123:124].copy()
    z0, _ = nn.forward(p, s, C)
    for i in range(L * L):
        t = s.copy()
        t.reshape(-1)[i:] *= -1
        z1, _ = nn.forward(p, t, C)
        assert np.allclose(z1.reshape(-1)[:i + 1], z0.reshape(-1)[:i + 1], rtol=0, atol=1e-14)


def test_symmetrised_model_is_normalised_and_even():
    C, L = 4, 3
    p = _params(C, 6, 0.8)
    S = _all_states(L)
    lq = nn.logq_sym(p, S, C)
    assert abs(np.exp(lq).sum() - 1.0) < 1e-12
    assert np.allclose(lq, nn.logq_sym(p, -S, C), rtol=0, atol=1e-13)
    # (q(s) + q(-s)) / 2 from the plain model, term by term
    q = np.exp(nn.logq(p, S, C))
    assert np.allclose(np.exp(lq), 0.5 * (q + np.exp(nn.logq(p, -S, C))), rtol=1e-12)


def test_sampler_frequencies_match_q():
    C, L, B = 3, 2, 20000
    p = _params(C, 7, 0.7)
    r = np.random.default_rng(8).integers(0, 2 ** 32, size=(B, L * L), dtype=np.uint64)
    s, lq = nn.sample(p, r.astype(np.uint32), L, C)
    assert np.allclose(lq, nn.logq(p, s, C))
    S = _all_states(L)
    q = np.exp(nn.logq(p, S, C))
    codes = {tuple(x.ravel()): k for k, x in enumerate(S)}
    counts = np.bincount([codes[tuple(x.ravel())] for x in s], minlength=len(S))
    exp = q * B
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 45.0  # 15 degrees of freedom: p < 1e-4


def test_adam_first_step_is_lr_times_sign():
    g = np.array([0.3, -2.0, 1e-3, -5e-2])
    p0 = np.zeros(4)
    p1, m, v = nn.adam_step(p0, np.zeros(4), np.zeros(4), g, 1, 1e-2, 0.9, 0.999, 1e-12)
    assert np.allclose(p1, -1e-2 * np.sign(g), rtol=1e-9)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


@pytest.mark.parametrize("beta", [0.3, 0.4406868, 0.6])
def test_independent_mh_kernel_has_exact_detailed_balance(beta):
    """P(s -> s') = q(s') min(1, exp(log ratio)) for s' != s: with the
    oracle's log ratio, pi(s) P(s -> s') = pi(s') P(s' -> s) for every pair
    of the 2^4 states of a 2 x 2 periodic lattice, and pi is stationary."""
    C, L = 3, 2
    p = _params(C, 11, 0.6)
    S = _all_states(L)
    E = np.array([oracle.measure(x)[0] for x in S], dtype=np.float64)
    lq = nn.logq(p, S, C)
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    n = len(S)
    P = np.zeros((n, n))
    for a in range(n):
        for c in range(n):
            if a != c:
                P[a, c] = np.exp(lq[c]) * min(1.0, np.exp(nn.mh_log_ratio(beta, E[a], E[c], lq[a], lq[c])))
        P[a, a] = 1.0 - P[a].sum()
    flow = pi[:, None] * P
    assert np.allclose(flow, flow.T, rtol=0, atol=1e-15)
    assert np.allclose(pi @ P, pi, rtol=0, atol=1e-14)
