"""GPU parity of the 3D spin glass with replica exchange against the
oracle (oracle/ea_oracle.c): spins of every replica, the energy of every
replica after every sweep, the temperature order and the accepted swaps,
bit for bit; graph replay; and the full-size workload on sampled sweeps."""
import sys

import numpy as np
import pytest

import oracle
from paper_2402_06415_amd.workloads import ea_bonds, ea_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_06415_amd as lib  # noqa: E402


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


def _compare(L, R, betas, seed, bond_seed, n_chunks, every, start="random", nthreads=8):
    say(f"ea L={L} R={R} every={every} chunks={n_chunks}")
    J = ea_bonds(L, bond_seed)
    g = lib.SpinGlass(J, betas, seed=seed, start=start)
    st = oracle.START_RANDOM if start == "random" else oracle.START_COLD_UP
    spins = np.stack([oracle.ea_init(L, st, seed, r) for r in range(R)])
    for r in range(R):
        assert (_host(g.replica(r)) == spins[r]).all(), f"start of replica {r}"
    E = np.array([oracle.ea_energy(x, J) for x in spins])
    perm = np.arange(R, dtype=np.int32)
    acc = np.zeros(max(R - 1, 1), np.uint64)
    t = 0
    for n in n_chunks:
        tr = torch.empty((n, R), dtype=torch.int64, device="cuda")
        g.sweep(n, every, trace=tr)
        want = oracle.ea_run(spins, J, betas, seed, t, n, every, perm, E, acc, nthreads=nthreads)
        t += n
        assert (_host(tr) == want).all(), f"energy trace differs in sweeps up to {t}"
        gt, gperm, gE, gacc = g.state()
        assert gt == t and (gperm == perm).all() and (gE == E).all()
        assert (gacc == acc[:R - 1]).all()
        for r in range(R):
            assert (_host(g.replica(r)) == spins[r]).all(), f"replica {r} after sweep {t}"
    assert (_host(g.measure()) == E).all()
    g.check()
    return g, acc


def test_small_ladder_bit_exact():
    _, acc = _compare(8, 4, np.array([0.5, 0.7, 0.9, 1.1]), 5, 3, (7, 5), 3)
    assert acc.sum() > 0


def test_odd_replica_count_and_cold_start():
    _compare(16, 5, np.array([0.2, 0.35, 0.5, 0.65, 0.8]), 9, 4, (6, 6), 2, start="cold")


def test_no_exchange_and_single_replica():
    _compare(8, 1, np.array([0.8]), 2, 5, (5,), 0)
    _compare(8, 3, np.array([0.3, 0.6, 0.9]), 2, 5, (4,), 0)


def test_graph_replay_continues_the_run():
    say("ea graph")
    L, R = 16, 4
    J = ea_bonds(L, 6)
    betas = np.array([0.5, 0.8, 1.0, 1.2])
    eager = lib.SpinGlass(J, betas, seed=7)
    cap = lib.SpinGlass(J, betas, seed=7)
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


def test_sweep_without_setup_is_a_device_error():
    say("ea no setup")
    L, R = 8, 2
    nb = lib.ising_ea_spins_bytes(L, R)
    raw_s, spins = lib.binding._aligned_buffer(nb, "cuda")
    raw_b, bonds = lib.binding._aligned_buffer(3 * L ** 3, "cuda")
    raw_w, ws = lib.binding._aligned_buffer(lib.ising_ea_workspace_bytes(L, R), "cuda")
    spins.fill_(1)
    c = lib.ising_ea(lib.binding.ABI_VERSION, L, R, 0, 1, spins.data_ptr(), bonds.data_ptr(), ws.data_ptr())
    lib.ising_ea_sweep(c, 3, 1)
    with pytest.raises(lib.IsingError) as e:
        lib.ising_ea_check_device_error(c)
    assert e.value.code == lib.binding.E_STATE
    assert (_host(spins) == 1).all()


def test_spin_glass_workload_full_size_first_sweeps():
    """L = 128, 64 replicas on beta in [0.5, 1.2], bonds from seed 3,
    exchange every 10 sweeps: the first 20 sweeps (two exchanges) bit-exact
    for every replica's energy and the order; four replicas' spins."""
    wl = ea_workload()
    L, betas, every = wl["L"], wl["beta"], wl["every"]
    R = len(betas)
    say("ea workload L=128 R=64, 20 sweeps")
    J = ea_bonds(L, wl["bond_seed"])
    g = lib.SpinGlass(J, betas, seed=wl["seed"])
    tr = torch.empty((20, R), dtype=torch.int64, device="cuda")
    g.sweep(20, every, trace=tr)
    spins = np.stack([oracle.ea_init(L, oracle.START_RANDOM, wl["seed"], r) for r in range(R)])
    E = np.array([oracle.ea_energy(x, J) for x in spins])
    perm = np.arange(R, dtype=np.int32)
    acc = np.zeros(R - 1, np.uint64)
    want = oracle.ea_run(spins, J, betas, wl["seed"], 0, 20, every, perm, E, acc, nthreads=16)
    assert (_host(tr) == want).all()
    t, gperm, gE, gacc = g.state()
    assert t == 20 and (gperm == perm).all() and (gacc == acc).all()
    for r in (0, 21, 42, 63):
        assert (_host(g.replica(r)) == spins[r]).all(), f"replica {r}"
    g.check()


def test_most_replicas():
    """1024 replicas, the most the ABI takes, on an 8^3 glass: every
    replica's energy trace, the temperature order and every spin, over two
    calls with an exchange every other sweep.  Adjacent betas are 0.002
    apart: the swap table of a pair holds 4096 entries, which needs a step
    of at least 32 ln 2 / 16384."""
    _compare(8, 1024, np.linspace(0.2, 2.2, 1024), 31, 5, (4, 3), 2, nthreads=16)


def test_largest_side():
    """L = 512, the largest side (2^27 spins per replica), two replicas over
    two sweeps with an exchange after each."""
    _compare(512, 2, np.array([0.5, 1.0]), 37, 7, (2,), 1, nthreads=16)
