"""GPU parity of the 3D spin glass with bit-plane draws (ISING_DRAWS_PLANE):
spins and couplings packed into colour bit planes, 32 sites per lane,
against the oracle's plane mode.  Integer work: the spins of every
replica, every replica's energy after every sweep, the temperature order
and the accepted swaps must be bit-exact; graph replay must continue the
run; and the full-size workload is checked on its first sweeps."""
import sys

import numpy as np
import pytest

import oracle
from paper_2402_06415_amd.workloads import ea_bonds, ea_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_06415_amd as lib  # noqa: E402

PLANE = oracle.MODE_PLANE


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib.load_library()
    yield
    torch.cuda.synchronize()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _compare(L, R, betas, seed, bond_seed, n_chunks, every, start="random", nthreads=16,
             check=None):
    say(f"ea plane L={L} R={R} every={every} chunks={n_chunks}")
    J = ea_bonds(L, bond_seed)
    g = lib.SpinGlass(J, betas, seed=seed, start=start, draws="plane")
    st = oracle.START_RANDOM if start == "random" else oracle.START_COLD_UP
    spins = np.stack([oracle.ea_init(L, st, seed, r) for r in range(R)])
    E = np.array([oracle.ea_energy(x, J) for x in spins])
    perm = np.arange(R, dtype=np.int32)
    acc = np.zeros(max(R - 1, 1), np.uint64)
    t = 0
    check = range(R) if check is None else check
    for n in n_chunks:
        tr = torch.empty((n, R), dtype=torch.int64, device="cuda")
        g.sweep(n, every, trace=tr)
        want = oracle.ea_run(spins, J, betas, seed, t, n, every, perm, E, acc, nthreads=nthreads,
                             mode=PLANE)
        t += n
        assert (_host(tr) == want).all(), f"energy trace differs in sweeps up to {t}"
        gt, gperm, gE, gacc = g.state()
        assert gt == t and (gperm == perm).all() and (gE == E).all()
        assert (gacc == acc[:R - 1]).all()
        for r in check:
            assert (_host(g.replica(r)) == spins[r]).all(), f"replica {r} after sweep {t}"
    assert (_host(g.measure()) == E).all()
    g.check()
    return g, acc


def test_plane_ladder_bit_exact():
    _, acc = _compare(64, 4, np.array([0.5, 0.7, 0.9, 1.1]), 5, 3, (5, 4), 3)


def test_plane_cold_start_odd_replicas_no_exchange():
    _compare(64, 3, np.array([0.3, 0.6, 0.9]), 9, 4, (4,), 0, start="cold")


def test_plane_two_words_per_row():
    # L = 128: two words per row, so the side word of a row edge comes from
    # the row's other word
    _compare(128, 2, np.array([0.4, 1.2]), 2, 5, (3,), 2)


def test_plane_graph_replay_continues_the_run():
    say("ea plane graph")
    L, R = 64, 4
    J = ea_bonds(L, 6)
    betas = np.array([0.5, 0.8, 1.0, 1.2])
    eager = lib.SpinGlass(J, betas, seed=7, draws="plane")
    cap = lib.SpinGlass(J, betas, seed=7, draws="plane")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        cap.sweep(10, 5)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cap.sweep(10, 5)
    torch.cuda.synchronize()
    eager.sweep(10, 5)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        eager.sweep(10, 5)
        a, b = cap.state(), eager.state()
        assert a[0] == b[0] == 20 + 10 * rep
        assert (a[1] == b[1]).all() and (a[2] == b[2]).all() and (a[3] == b[3]).all()
    for r in range(R):
        assert (_host(cap.replica(r)) == _host(eager.replica(r))).all()
    cap.check()


def test_plane_and_site_modes_agree_at_beta_zero():
    """At beta = 0 every site flips in every half-sweep whatever the draws:
    the two modes give the same spins."""
    say("ea plane vs site at beta 0")
    J = ea_bonds(64, 8)
    betas = np.array([0.0])
    a = lib.SpinGlass(J, betas, seed=4, draws="plane")
    b = lib.SpinGlass(J, betas, seed=4, draws="site")
    a.sweep(3, 0)
    b.sweep(3, 0)
    assert (_host(a.replica(0)) == _host(b.replica(0))).all()


def test_plane_spin_glass_workload_full_size_first_sweeps():
    """L = 128, 64 replicas on beta in [0.5, 1.2], bonds from seed 3,
    exchange every 10 sweeps, plane draws: the first 20 sweeps (two
    exchanges) bit-exact for every replica's energy and the order; four
    replicas' spins."""
    wl = ea_workload()
    L, betas, every = wl["L"], wl["beta"], wl["every"]
    R = len(betas)
    say("ea plane workload L=128 R=64, 20 sweeps")
    J = ea_bonds(L, wl["bond_seed"])
    g = lib.SpinGlass(J, betas, seed=wl["seed"], draws="plane")
    tr = torch.empty((20, R), dtype=torch.int64, device="cuda")
    g.sweep(20, every, trace=tr)
    spins = np.stack([oracle.ea_init(L, oracle.START_RANDOM, wl["seed"], r) for r in range(R)])
    E = np.array([oracle.ea_energy(x, J) for x in spins])
    perm = np.arange(R, dtype=np.int32)
    acc = np.zeros(R - 1, np.uint64)
    want = oracle.ea_run(spins, J, betas, wl["seed"], 0, 20, every, perm, E, acc, nthreads=16,
                         mode=PLANE)
    assert (_host(tr) == want).all()
    t, gperm, gE, gacc = g.state()
    assert t == 20 and (gperm == perm).all() and (gacc == acc).all()
    for r in (0, 21, 42, 63):
        assert (_host(g.replica(r)) == spins[r]).all(), f"replica {r}"
    g.check()


def test_plane_most_replicas():
    """1024 replicas, the most the ABI takes, at the smallest plane side
    (L = 64): energies, order and three replicas' spins after two sweeps."""
    _compare(64, 1024, np.linspace(0.2, 2.2, 1024), 31, 5, (2,), 1, check=(0, 511, 1023))


def test_plane_largest_side():
    """L = 512, the largest side (2^27 spins per replica), two replicas over
    two sweeps with an exchange after each."""
    _compare(512, 2, np.array([0.5, 1.0]), 37, 7, (2,), 1)
