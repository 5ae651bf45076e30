"""Pins of the oracle's per-site rules against the paper's definitions.

- thresholds: the paper accepts iff p < P(dE) = exp(-beta dE) (Supplementary,
  "Detail of the MC calculation", step 3).  With p = r / 2^32 the smallest
  rejected r must be ceil(2^32 P); checked in 80-digit arithmetic.
- local field / measure: against brute-force enumeration of the 4x4 torus and
  its density of states, which Kaufman's closed form reproduces.
- half-sweep kernel: exact detailed balance on the 4x4 torus, built from the
  oracle's own neighbour sum and decision rule.
- draws: the counter layouts, recomputed through PyTorch's independent
  Philox engine, and their marginal uniformity.
"""
import functools

import mpmath as mp
import numpy as np
import pytest

import exact
import oracle

BETAS = [0.0, 1e-12, 0.1, 0.3, 0.4, 0.4406868, 0.48, 0.5, 0.6, 1.2, 3.0]


@pytest.mark.parametrize("beta", BETAS)
def test_thresholds_bracket_the_acceptance_probability(beta):
    T, always = oracle.thresholds(beta)
    assert always[:3].tolist() == [1, 1, 1]  # dE <= 0 always accepted
    with mp.workdps(80):
        for k in (3, 4):
            u = 2 * k - 4
            P = mp.e ** (-mp.mpf(beta) * 2 * u)
            if always[k]:
                # only when 2^32 P is within rounding of 2^32
                assert mp.ldexp(P, 32) > 2 ** 32 - 1
                continue
            t = int(T[k])
            # r = t - 1 accepted: (t-1)/2^32 < P ; r = t rejected: t/2^32 >= P
            assert mp.mpf(t - 1) / 2 ** 32 < P
            assert mp.mpf(t) / 2 ** 32 >= P
            # and the double-precision exp is far from a rounding tie
            frac = mp.ldexp(P, 32) - mp.floor(mp.ldexp(P, 32))
            assert min(frac, 1 - frac) > 1e-6 or frac == 0


def test_thresholds_depend_only_on_beta_times_dE():
    T3, _ = oracle.thresholds(0.3)
    T6, _ = oracle.thresholds(0.6)
    assert T3[4] == T6[3]  # dE = 8 at beta 0.3 equals dE = 4 at beta 0.6


@pytest.mark.parametrize("beta", [-0.1, float("nan"), float("inf")])
def test_thresholds_reject_invalid_beta(beta):
    with pytest.raises(ValueError):
        oracle.thresholds(beta)


def test_accept_rule_is_strict_less_than():
    T, a = oracle.thresholds(0.4406868)
    for u in (2, 4):
        k = (u + 4) // 2
        assert oracle.accept(u, int(T[k]) - 1, T, a)
        assert not oracle.accept(u, int(T[k]), T, a)
        assert oracle.accept(u, 0, T, a)
        assert not oracle.accept(u, 2 ** 32 - 1, T, a)
    for u in (-4, -2, 0):
        assert oracle.accept(u, 2 ** 32 - 1, T, a)


def test_measure_reproduces_4x4_density_of_states():
    # Enumerate through the oracle's measure and compare with the independent
    # numpy enumeration; the latter is itself pinned to Kaufman's Z below.
    L = 4
    want = exact.density_of_states(L)
    got = {}
    Ms = []
    for idx in range(1 << 16):
        bits = (idx >> np.arange(16)) & 1
        s = (1 - 2 * bits).astype(np.int8).reshape(L, L)
        E, M = oracle.measure(s)
        got[E] = got.get(E, 0) + 1
        Ms.append(M)
    assert got == want
    assert sorted(set(Ms)) == list(range(-16, 17, 2))


@pytest.mark.parametrize("beta", [0.1, 0.3, 0.4406868, 0.6])
def test_enumeration_matches_kaufman_closed_form(beta):
    g = exact.density_of_states(4)
    Z = sum(mp.mpf(c) * mp.e ** (-mp.mpf(beta) * E) for E, c in g.items())
    assert abs(float(mp.log(Z)) - float(exact.kaufman_logZ(beta, 4, 4))) < 1e-12


def test_local_u_matches_bond_energy_difference():
    # u = s_i h_i must equal half the energy change of flipping site i,
    # measured by two full recounts, at every site of random lattices,
    # including the periodic wrap.
    rng = np.random.default_rng(5)
    for L in (4, 6, 8):
        for _ in range(3):
            s = rng.choice(np.array([-1, 1], dtype=np.int8), size=(L, L))
            E0, _ = oracle.measure(s)
            for y in range(L):
                for x in range(L):
                    u = oracle.local_u(s, x, y)
                    s2 = s.copy()
                    s2[y, x] = -s2[y, x]
                    E1, _ = oracle.measure(s2)
                    assert E1 - E0 == 2 * u


def _flip_probabilities(beta):
    """Per-u acceptance probability implied by the oracle's decision rule,
    found by bisection on r (the rule is monotone in r)."""
    T, a = oracle.thresholds(beta)
    probs = {}
    for u in (-4, -2, 0, 2, 4):
        lo, hi = 0, 2 ** 32  # smallest rejected r lies in [lo, hi]
        if oracle.accept(u, 2 ** 32 - 1, T, a):
            probs[u] = mp.mpf(1)
            continue
        while lo < hi:
            mid = (lo + hi) // 2
            if oracle.accept(u, mid, T, a):
                lo = mid + 1
            else:
                hi = mid
        probs[u] = mp.mpf(lo) / 2 ** 32
    return probs


@functools.lru_cache(maxsize=1)
def _oracle_u_table_4x4():
    """u for every (state, site) of the 4x4 torus, through the oracle."""
    L, N = 4, 16
    U = np.zeros((1 << N, N), dtype=np.int64)
    for idx in range(1 << N):
        bits = (idx >> np.arange(N)) & 1
        s = (1 - 2 * bits).astype(np.int8).reshape(L, L)
        for j in range(N):
            U[idx, j] = oracle.local_u(s, j % L, j // L)
    return U


@pytest.mark.parametrize("beta", [0.3, 0.4406868, 0.6])
def test_halfsweep_detailed_balance_4x4(beta):
    """pi(x) K_c(x,y) = pi(y) K_c(y,x) for every pair on the 4x4 torus.

    K_c flips each colour-c site independently with the oracle's acceptance
    probability for its u (from oracle.local_u).  The full sweep K_0 K_1 is
    only stationary, so detailed balance is checked per half-sweep, and
    stationarity of the full sweep separately.  The 2^-32 quantisation of
    P bounds the relative defect by 2^-32 / min P."""
    L, N = 4, 16
    probs = _flip_probabilities(beta)
    pu = np.array([float(probs[u]) for u in (-4, -2, 0, 2, 4)])
    E, _ = exact.enumerate_states(L)
    logpi = -beta * (E - E.min()).astype(np.float64)
    logpi -= np.log(np.exp(logpi).sum())
    nstates = 1 << N
    U = _oracle_u_table_4x4()
    P = pu[(U + 4) // 2]  # flip probability per (state, site)
    # Each flipped site contributes a relative error <= 2^-32 / P(u) from the
    # quantisation; a move flips at most N/2 sites.
    p_min = float(min(probs[2], probs[4]))
    bound = (N // 2) * 2 ** -32 / p_min
    worst = 0.0
    pi_after = {}
    for c in (0, 1):
        sites = [j for j in range(N) if ((j % L) + (j // L)) % 2 == c]
        masks = []
        for F in range(1 << len(sites)):
            m = 0
            for b, j in enumerate(sites):
                if (F >> b) & 1:
                    m |= 1 << j
            masks.append(m)
        masks = np.array(masks, dtype=np.int64)
        Fbits = ((np.arange(1 << len(sites))[:, None] >> np.arange(len(sites))) & 1).astype(bool)
        Pc = P[:, sites]  # (states, 8)
        # log K(x -> x ^ F) for all x, F
        with np.errstate(divide="ignore"):
            lp = np.log(Pc)
            lq = np.log1p(-Pc)
        logK = np.where(Fbits[None, :, :], lp[:, None, :], lq[:, None, :]).sum(axis=2)
        x = np.arange(nstates)[:, None]
        y = x ^ masks[None, :]
        # reverse move index: the same mask F from y
        fwd = logpi[x] + logK
        rev = logpi[y] + logK[y, np.arange(len(masks))[None, :]]
        ok = np.isfinite(fwd) | np.isfinite(rev)
        d = np.abs(np.exp(fwd[ok]) - np.exp(rev[ok])) / np.maximum(np.exp(fwd[ok]), 1e-300)
        worst = max(worst, float(d.max()))
        # stationarity of this half-sweep: sum_x pi(x) K(x, y) = pi(y)
        flow = np.zeros(nstates)
        np.add.at(flow, y.ravel(), np.exp(fwd).ravel())
        pi_after[c] = flow
        rel = np.abs(flow - np.exp(logpi)) / np.exp(logpi)
        assert rel.max() < bound + 1e-12, (c, rel.max(), bound)
    assert worst < bound + 1e-12, (worst, bound)
    # a plausible mistake (e.g. exp(+beta dE) or a wrong neighbour) breaks
    # detailed balance by O(1), far above the quantisation bound
    assert bound < 1e-5


def test_init_cold_and_random():
    s = oracle.init(8, oracle.START_COLD_UP, 1)
    assert (s == 1).all()
    s = oracle.init(256, oracle.START_RANDOM, 7)
    assert set(np.unique(s).tolist()) == {-1, 1}
    N = s.size
    assert abs(s.mean()) < 5 / np.sqrt(N)
    # no nearest-neighbour correlation in either direction
    assert abs((s * np.roll(s, 1, 0)).mean()) < 5 / np.sqrt(N)
    assert abs((s * np.roll(s, 1, 1)).mean()) < 5 / np.sqrt(N)
    # a different seed or lattice id gives a different start
    assert (oracle.init(256, oracle.START_RANDOM, 8) != s).any()
    assert (oracle.init(256, oracle.START_RANDOM, 7, lattice_id=1) != s).any()
    with pytest.raises(ValueError):
        oracle.init(7, oracle.START_RANDOM, 1)


def test_init_counter_layout(torch_philox):
    L, seed, lid = 16, (5 << 32) | 9, 3
    s = oracle.init(L, oracle.START_RANDOM, seed, lid)
    rows = []
    for n in range(L * L):
        rows.append([seed & 0xFFFFFFFF, seed >> 32, n >> 2, lid, 0, 2])
    ref = torch_philox(rows)
    want = np.array([-1 if (int(ref[n][n & 3]) >> 31) else 1 for n in range(L * L)])
    assert (s.ravel() == want).all()


def test_site_mode_counter_layout(torch_philox):
    L, seed, lid, t, c = 12, 77, 2, 5, 1
    r = oracle.fill_uniforms(L, oracle.MODE_SITE, seed, lid, t, c)
    rows, where = [], []
    for y in range(L):
        for x in range(L):
            if (x + y) % 2 != c:
                assert r[y, x] == 0
                continue
            q = (y * L + x) >> 1
            rows.append([seed, 0, q >> 2, lid, 2 * t + c, 0])
            where.append((y, x, q & 3))
    ref = torch_philox(rows)
    for (y, x, j), out in zip(where, ref):
        assert int(r[y, x]) == int(out[j])


@pytest.mark.parametrize("L,c", [(64, 0), (32, 1), (96, 0)])
def test_plane_mode_counter_layout(torch_philox, L, c):
    # L = 32 and 96: a group of 32 compact indices spans two rows
    seed, lid, t = 12345, 0, 3
    r = oracle.fill_uniforms(L, oracle.MODE_PLANE, seed, lid, t, c)
    rng = np.random.default_rng(0)
    picks = [(int(y), int(x)) for y, x in zip(rng.integers(0, L, 40), rng.integers(0, L, 40))]
    for y, x in picks:
        if (x + y) % 2 != c:
            x = (x + 1) % L
        q = (y * L + x) >> 1
        g, lane = q >> 5, q & 31
        rows = [[seed, 0, g, lid, 2 * t + c, 1 | (b << 8)] for b in range(8)]
        ref = torch_philox(rows)
        planes = [int(ref[k >> 2][k & 3]) for k in range(32)]
        want = sum(((planes[k] >> lane) & 1) << (31 - k) for k in range(32))
        assert int(r[y, x]) == want


@pytest.mark.parametrize("mode", [oracle.MODE_SITE, oracle.MODE_PLANE])
def test_uniforms_are_uniform_and_decorrelated(mode):
    L = 128
    r = oracle.fill_uniforms(L, mode, 99, 0, 0, 0)
    mask = ((np.arange(L)[:, None] + np.arange(L)[None, :]) % 2) == 0
    v = r[mask].astype(np.float64) / 2 ** 32
    n = v.size
    # top-4-bit histogram
    hist = np.bincount((r[mask] >> 28).astype(np.int64), minlength=16)
    chi2 = ((hist - n / 16) ** 2 / (n / 16)).sum()
    assert chi2 < 50  # 15 dof, p ~ 1e-5
    assert abs(v.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    # lag-1 correlation along the colour's compact order and across sweeps
    w = v - 0.5
    assert abs((w[1:] * w[:-1]).mean() * 12) < 5 / np.sqrt(n)
    r2 = oracle.fill_uniforms(L, mode, 99, 0, 1, 0)
    v2 = r2[mask].astype(np.float64) / 2 ** 32 - 0.5
    assert abs((w * v2).mean() * 12) < 5 / np.sqrt(n)
    # within a PLANE group all 32 bit positions of r are balanced
    bits = ((r[mask][:, None] >> np.arange(32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(n))


def test_plane_mode_requires_L_multiple_of_32():
    for L in (48, 16):
        with pytest.raises(ValueError):
            oracle.fill_uniforms(L, oracle.MODE_PLANE, 1, 0, 0, 0)
