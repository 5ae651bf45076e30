"""Pins of the 3D spin-glass oracle (oracle/ea_oracle.c): thresholds
against 80-digit arithmetic and printed closed-form values, the energy
against an independent numpy formula, E(flip) - E = 2u, exact gauge
invariance of the whole chain, exact detailed balance of each half-sweep
on the 2^8 states of a 2x2x2 lattice, replica exchange sampling each
temperature's exact distribution, and every counter map (per-site draws,
plane draws, random start, exchange draws) recomputed through PyTorch's
independent Philox engine."""
import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2402_06415_amd.workloads import ea_bonds


def _energy_numpy(s, J):
    s = s.astype(np.int64)
    E = 0
    for d, ax in enumerate((2, 1, 0)):  # x, y, z are array axes 2, 1, 0
        E -= int((J[d].astype(np.int64) * s * np.roll(s, -1, axis=ax)).sum())
    return E


def test_thresholds_printed_values():
    assert oracle.ea_thresholds(0.5)[0].tolist() == [581260616, 78665071, 10646160]
    assert oracle.ea_thresholds(1.2)[0].tolist() == [35346495, 290893, 2394]


@pytest.mark.parametrize("beta", [0.0, 1e-12, 0.5, 0.7, 0.9, 1.2])
def test_thresholds_bracket_exp(beta):
    T, a = oracle.ea_thresholds(beta)
    with mp.workdps(80):
        for i, u in enumerate((2, 4, 6)):
            P = mp.e ** (-mp.mpf(beta) * 2 * u)
            if a[i]:
                assert mp.ldexp(P, 32) > 2 ** 32 - 1
                continue
            assert mp.mpf(int(T[i]) - 1) / 2 ** 32 < P <= mp.mpf(int(T[i])) / 2 ** 32


@pytest.mark.parametrize("blo,bhi,D", [(0.5, 0.5 + 0.7 / 63, 4), (0.5, 0.5 + 0.7 / 63, 400),
                                       (1.0, 1.2, 12), (0.5, 0.6, 2000), (0.5, 0.9, 100000)])
def test_swap_threshold_brackets_exp(blo, bhi, D):
    T, a = oracle.ea_swap_threshold(blo, bhi, D)
    with mp.workdps(80):
        P = mp.e ** (-(mp.mpf(bhi) - mp.mpf(blo)) * D)
        assert not a
        if T == 0:
            assert P < mp.mpf(2) ** -1070  # exp underflows in double
        else:
            assert mp.mpf(T - 1) / 2 ** 32 < P <= mp.mpf(T) / 2 ** 32
    assert oracle.ea_swap_threshold(blo, bhi, 0) == (0, True)
    assert oracle.ea_swap_threshold(blo, bhi, -8) == (0, True)


def test_energy_and_local_field():
    L = 6
    J = ea_bonds(L, 7)
    s = oracle.ea_init(L, 1, 9, 0)
    assert oracle.ea_energy(s, J) == _energy_numpy(s, J)
    assert oracle.ea_energy(np.ones((L, L, L), np.int8), np.ones((3, L, L, L), np.int8)) == -3 * L ** 3
    E0 = oracle.ea_energy(s, J)
    for n in range(L ** 3):
        t = s.copy()
        t.reshape(-1)[n] *= -1
        assert oracle.ea_energy(t, J) - E0 == 2 * oracle.ea_local_u(s, J, n)


def test_chain_is_gauge_invariant():
    """With tau_n = +-1, J'_d(n) = tau_n J_d(n) tau_{n+e_d} and s' = tau s have
    the same energies and local fields, so the same draws give the chain
    tau * chain, exchanges included, bit for bit."""
    L, R = 4, 3
    J = ea_bonds(L, 11)
    tau = oracle.ea_init(L, 1, 12, 5)
    Jg = np.empty_like(J)
    for d, ax in enumerate((2, 1, 0)):
        Jg[d] = tau * J[d] * np.roll(tau, -1, axis=ax)
    beta = np.array([0.5, 0.8, 1.1])
    a = np.stack([oracle.ea_init(L, 1, 3, r) for r in range(R)])
    b = a * tau[None]
    Ea = np.array([oracle.ea_energy(x, J) for x in a])
    Eb = np.array([oracle.ea_energy(x, Jg) for x in b])
    assert (Ea == Eb).all()
    pa, pb = np.arange(R, dtype=np.int32), np.arange(R, dtype=np.int32)
    ta = oracle.ea_run(a, J, beta, 3, 0, 60, 2, pa, Ea)
    tb = oracle.ea_run(b, Jg, beta, 3, 0, 60, 2, pb, Eb)
    assert (ta == tb).all() and (pa == pb).all()
    assert (b == a * tau[None]).all()
    assert sorted(pa.tolist()) == list(range(R))


def _all_states_3d():
    idx = np.arange(256)
    return (1 - 2 * ((idx[:, None] >> np.arange(8)) & 1)).astype(np.int8).reshape(256, 2, 2, 2)


@pytest.mark.parametrize("beta", [0.3, 0.9])
def test_halfsweep_detailed_balance_2x2x2(beta):
    """K_c flips each colour-c site independently with probability
    T(u)/2^32 (1 for u <= 0): pi K_c is reversible up to the 2^-32
    quantisation, for random couplings on the 2x2x2 torus."""
    J = ea_bonds(2, 21)
    S = _all_states_3d()
    E = np.array([oracle.ea_energy(x, J) for x in S], np.float64)
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    T, a = oracle.ea_thresholds(beta)
    code = {x.tobytes(): k for k, x in enumerate(S)}
    for c in (0, 1):
        sites = [n for n in range(8) if ((n & 1) + ((n >> 1) & 1) + (n >> 2)) % 2 == c]
        K = np.zeros((256, 256))
        for k, x in enumerate(S):
            p = []
            for n in sites:
                u = oracle.ea_local_u(x, J, n)
                p.append(1.0 if u <= 0 or a[u // 2 - 1] else float(T[u // 2 - 1]) / 2 ** 32)
            for F in range(1 << len(sites)):
                y = x.copy().reshape(-1)
                w = 1.0
                for b, n in enumerate(sites):
                    if (F >> b) & 1:
                        y[n] *= -1
                        w *= p[b]
                    else:
                        w *= 1 - p[b]
                K[k, code[y.reshape(2, 2, 2).tobytes()]] += w
        flow = pi[:, None] * K
        assert np.allclose(flow, flow.T, rtol=4 * 2.0 ** -32 / float(T[2]) * 2 ** 32, atol=1e-17)
        assert np.allclose(pi @ K, pi, atol=1e-12)


def test_replica_exchange_samples_each_temperature():
    """Three replicas on the 2x2x2 glass, exchange after every sweep: the
    energy seen at each temperature averages to the exact Boltzmann mean."""
    J = ea_bonds(2, 23)
    beta = np.array([0.3, 0.6, 0.9])
    S = _all_states_3d()
    E_all = np.array([oracle.ea_energy(x, J) for x in S], np.float64)
    exact = [float((E_all * np.exp(-b * E_all)).sum() / np.exp(-b * E_all).sum()) for b in beta]
    R = 3
    spins = np.stack([oracle.ea_init(2, 1, 31, r) for r in range(R)])
    E = np.array([oracle.ea_energy(x, J) for x in spins])
    perm = np.arange(R, dtype=np.int32)
    acc = np.zeros(R - 1, np.uint64)
    n = 30000
    hist = np.zeros((n, R))
    for t in range(n):
        oracle.ea_run(spins, J, beta, 31, t, 1, 1, perm, E, acc, trace=False)
        hist[t] = E[perm]
    assert (acc > 0).all()
    for k in range(R):
        x = hist[1000:, k]
        blocks = x[: len(x) // 50 * 50].reshape(50, -1).mean(axis=1)
        err = blocks.std(ddof=1) / np.sqrt(50)
        assert abs(blocks.mean() - exact[k]) < 4 * err + 1e-9, (k, blocks.mean(), exact[k], err)


PLANE = oracle.MODE_PLANE


@pytest.mark.parametrize("L,c,t", [(8, 0, 3), (16, 1, 0), (64, 0, 7)])
def test_plane_draw_counter_layout(torch_philox, L, c, t):
    """Plane draws of the spin glass: site q = n >> 1 of colour c takes bit
    q & 31 of the eight blocks (q >> 5, replica, 2t + c, 1 | b << 8) as its
    32-bit r, most significant plane first (checked against PyTorch's own
    Philox for sampled sites; at L = 8 and 16 a group spans several rows)."""
    seed, rid = 4242, 5
    r = oracle.ea_fill_plane(L, c, seed, rid, t)
    rng = np.random.default_rng(L)
    picks = rng.integers(0, L, size=(24, 3))
    for z, y, x in picks:
        if (x + y + z) % 2 != c:
            x = (x + 1) % L
        n = (int(z) * L + int(y)) * L + int(x)
        q = n >> 1
        g, lane = q >> 5, q & 31
        rows = [[seed, 0, g, rid, 2 * t + c, 1 | (b << 8)] for b in range(8)]
        ref = torch_philox(rows)
        planes = [int(ref[k >> 2][k & 3]) for k in range(32)]
        want = sum(((planes[k] >> lane) & 1) << (31 - k) for k in range(32))
        assert int(r[z, y, x]) == want
    other = ((np.arange(L)[:, None, None] + np.arange(L)[None, :, None] +
              np.arange(L)[None, None, :]) % 2) != c
    assert (r[other] == 0).all()


def test_plane_draws_are_uniform_and_decorrelated():
    L = 32
    r = oracle.ea_fill_plane(L, 0, 99, 0, 0)
    mask = ((np.arange(L)[:, None, None] + np.arange(L)[None, :, None] +
             np.arange(L)[None, None, :]) % 2) == 0
    v = r[mask].astype(np.float64) / 2 ** 32
    n = v.size
    hist = np.bincount((r[mask] >> 28).astype(np.int64), minlength=16)
    chi2 = ((hist - n / 16) ** 2 / (n / 16)).sum()
    assert chi2 < 50  # 15 dof
    assert abs(v.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    w = v - 0.5
    assert abs((w[1:] * w[:-1]).mean() * 12) < 5 / np.sqrt(n)
    v2 = oracle.ea_fill_plane(L, 0, 99, 0, 1)[mask].astype(np.float64) / 2 ** 32 - 0.5
    assert abs((w * v2).mean() * 12) < 5 / np.sqrt(n)
    bits = ((r[mask][:, None] >> np.arange(32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(n))


def test_plane_mode_replica_exchange_samples_each_temperature():
    """The plane-draw chain (one partial draw group per colour on the 2x2x2
    glass) with exchanges after every sweep: each temperature's mean energy
    is the exact Boltzmann mean."""
    J = ea_bonds(2, 23)
    beta = np.array([0.3, 0.6, 0.9])
    S = _all_states_3d()
    E_all = np.array([oracle.ea_energy(x, J) for x in S], np.float64)
    exact = [float((E_all * np.exp(-b * E_all)).sum() / np.exp(-b * E_all).sum()) for b in beta]
    R = 3
    spins = np.stack([oracle.ea_init(2, 1, 37, r) for r in range(R)])
    E = np.array([oracle.ea_energy(x, J) for x in spins])
    perm = np.arange(R, dtype=np.int32)
    acc = np.zeros(R - 1, np.uint64)
    n = 30000
    hist = np.zeros((n, R))
    for t in range(n):
        oracle.ea_run(spins, J, beta, 37, t, 1, 1, perm, E, acc, trace=False, mode=PLANE)
        hist[t] = E[perm]
    assert (acc > 0).all()
    for k in range(R):
        x = hist[1000:, k]
        blocks = x[: len(x) // 50 * 50].reshape(50, -1).mean(axis=1)
        err = blocks.std(ddof=1) / np.sqrt(50)
        assert abs(blocks.mean() - exact[k]) < 4 * err + 1e-9, (k, blocks.mean(), exact[k], err)
    assert (E == [oracle.ea_energy(x, J) for x in spins]).all()


def test_plane_and_site_modes_differ_but_share_everything_else():
    """Same start, same couplings: the two draw modes give different chains,
    and at beta = 0 (every site flips) identical ones."""
    J = ea_bonds(8, 5)
    a = np.stack([oracle.ea_init(8, 1, 3, r) for r in range(2)])
    b = a.copy()
    for beta, same in ((np.array([0.4, 0.8]), False), (np.array([0.0, 0.0]), True)):
        Ea = np.array([oracle.ea_energy(x, J) for x in a])
        Eb = Ea.copy()
        pa, pb = np.arange(2, dtype=np.int32), np.arange(2, dtype=np.int32)
        oracle.ea_run(a, J, beta, 3, 0, 4, 0, pa, Ea, trace=False)
        oracle.ea_run(b, J, beta, 3, 0, 4, 0, pb, Eb, trace=False, mode=PLANE)
        assert (a == b).all() == same
        b[:] = a


# ---------------------------------------------------------------------------
# Counter maps of the per-site draws, the random start and the exchange
# draws, recomputed through PyTorch's own Philox engine (conftest.py): the
# oracle's decisions must follow from those draws and from the pinned
# thresholds and local fields alone.

@pytest.mark.parametrize("L,c,t,rid", [(6, 0, 0, 0), (6, 1, 5, 3), (8, 0, 11, 62)])
def test_site_draw_counter_layout(torch_philox, L, c, t, rid):
    """Per-site draws: site n of colour c takes r = out[q & 3] of the block
    (q >> 2, replica, 2t + c, 0), q = n >> 1; it flips iff u <= 0 or
    r < T(u).  Sites of one colour do not neighbour each other, so every
    decision is taken on the state before the half-sweep."""
    seed = (7 << 32) | 4242
    beta = 0.15
    J = ea_bonds(L, 17)
    s0 = oracle.ea_init(L, 1, 19, rid)
    T, a = oracle.ea_thresholds(beta)
    sites = [n for n in range(L ** 3)
             if ((n % L) + (n // L) % L + n // (L * L)) % 2 == c]
    rows = [[seed & 0xFFFFFFFF, seed >> 32, (n >> 1) >> 2, rid, 2 * t + c, 0] for n in sites]
    ref = torch_philox(rows)
    want = s0.copy().reshape(-1)
    dE_want, drawn_flips, drawn_keeps = 0, 0, 0
    for n, out in zip(sites, ref):
        u = oracle.ea_local_u(s0, J, n)
        if u <= 0 or a[u // 2 - 1]:
            flip = True
        else:
            flip = int(out[(n >> 1) & 3]) < int(T[u // 2 - 1])
            drawn_flips += flip
            drawn_keeps += not flip
        if flip:
            want[n] = -want[n]
            dE_want += 2 * u
    assert drawn_flips > 3 and drawn_keeps > 3  # both outcomes hinge on the draws
    s = s0.copy()
    dE = oracle.ea_halfsweep(s, J, c, seed, rid, t, beta, mode=oracle.MODE_SITE)
    assert (s.reshape(-1) == want).all()
    assert dE == dE_want


def test_random_start_counter_layout(torch_philox):
    """Random start of replica r: s_n = -1 iff the top bit of out[n & 3] of
    the block (n >> 2, r, 0, 2) is set."""
    L, seed, rid = 6, (3 << 32) | 11, 9
    s = oracle.ea_init(L, 1, seed, rid).reshape(-1)
    ref = torch_philox([[seed & 0xFFFFFFFF, seed >> 32, n >> 2, rid, 0, 2] for n in range(L ** 3)])
    want = np.array([-1 if int(ref[n][n & 3]) >> 31 else 1 for n in range(L ** 3)])
    assert (s == want).all()
    assert (oracle.ea_init(L, 0, seed, rid) == 1).all()


@pytest.mark.parametrize("m", [0, 1, 6, 7])
def test_exchange_draw_counter_layout(torch_philox, m):
    """Exchange number m visits the pairs (k, k + 1), k = m & 1, m & 1 + 2,
    ...; with D = E(at k) - E(at k + 1) > 0 the swap takes r = out[0] of the
    block (k, m, 0, 5) and is accepted iff r < T(beta_k, beta_k+1, D)."""
    R, seed = 12, (5 << 32) | 77
    beta = 0.5 + 0.05 * np.arange(R)
    rng = np.random.default_rng(m)
    E = rng.integers(-400, -300, R).astype(np.int64)
    # energies decreasing along the ladder so that most pairs need a draw,
    # with steps giving acceptance probabilities between 0.1 and 0.8
    E = -300 - np.cumsum(rng.integers(1, 12, R) * 4).astype(np.int64)
    E[R // 2] = E[R // 2 + 1] - 8  # one pair with D < 0: swaps without a draw
    perm0 = rng.permutation(R).astype(np.int32)
    Erep = np.empty(R, np.int64)
    Erep[perm0] = E  # replica perm0[k] sits at temperature k with energy E[k]
    want = perm0.copy()
    drawn = {True: 0, False: 0}
    for k in range(m & 1, R - 1, 2):
        D = int(Erep[want[k]] - Erep[want[k + 1]])
        T, always = oracle.ea_swap_threshold(beta[k], beta[k + 1], D)
        if always:
            swap = True
        else:
            r = int(torch_philox([[seed & 0xFFFFFFFF, seed >> 32, k, m, 0, 5]])[0][0])
            swap = r < T
            drawn[swap] += 1
        if swap:
            want[k], want[k + 1] = want[k + 1], want[k]
    perm = perm0.copy()
    oracle.ea_exchange(Erep, perm, beta, m, seed)
    assert (perm == want).all()
    assert drawn[True] + drawn[False] >= 3
