"""GPU parity of the batch API: many INT8 lattices of uneven side, each at
its own beta, swept in one persistent launch, against the oracle run
lattice by lattice.  Integer work, so spins, E, M and every moment must be
bit-exact; the launch shape, graph capture and the autotuner must not
change the chain."""
import sys

import numpy as np
import pytest

import oracle
from paper_2402_06415_amd.workloads import batched_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_06415_amd as lib  # noqa: E402

MIXED_L = [8, 16, 24, 32, 40, 64, 128, 256, 8, 48, 96, 16]
MIXED_BETA = [0.0, 1e-12, 0.3, 0.4406868, 0.6, 3.0, 0.35, 0.5, 0.4406868, 0.42, 0.45, 1.0]
KEYS = ("E", "M", "sum_E", "sum_E2", "sum_absM", "sum_M2")


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


def _oracle_states(Ls, seed, lid0, start="random"):
    st = oracle.START_RANDOM if start == "random" else oracle.START_COLD_UP
    return [oracle.init(int(L), st, seed, lid0 + j) for j, L in enumerate(Ls)]


def _check_moments(mom, want, js=None):
    mom = _host(mom)
    for j, w in enumerate(want) if js is None else zip(js, want):
        row = mom[j]
        got = dict(zip(KEYS, (int(v) for v in row[:6])))
        mask = (1 << 64) - 1
        m4 = ((int(row[7]) & mask) << 64) | (int(row[6]) & mask)
        assert got == {k: w[k] for k in KEYS}, f"lattice {j}"
        assert m4 == w["sum_M4"], f"lattice {j} M^4"


def _check_spins(b, states, js=None):
    for j, s in enumerate(states) if js is None else zip(js, states):
        got = _host(b.lattice(j))
        if not (got == s).all():
            raise AssertionError(f"lattice {j} (L={b.L[j]}): {(got != s).sum()} sites differ")


def _run_mixed(threads=0, groups_per_cu=0, chunks=(7, 5), seed=21, lid0=3):
    say(f"mixed batch threads={threads} gpc={groups_per_cu} chunks={chunks}")
    b = lib.Batch(MIXED_L, MIXED_BETA, seed=seed, lattice_id0=lid0, start="random",
                  threads=threads, groups_per_cu=groups_per_cu)
    states = _oracle_states(MIXED_L, seed, lid0)
    _check_spins(b, states)
    t = 0
    for n in chunks:
        mom = b.sweep(n)
        want = oracle.batch_sweep(states, MIXED_BETA, seed, lid0, t, n, nthreads=8)
        t += n
        _check_moments(mom, want)
        _check_spins(b, states)
    E, M = b.measure()
    assert [tuple(x) for x in zip(_host(E), _host(M))] == [oracle.measure(s) for s in states]
    assert b.sweep_index == t
    b.check()
    return b


def test_mixed_batch_bit_exact():
    _run_mixed()


@pytest.mark.parametrize("threads,gpc", [(64, 1), (256, 3), (1024, 2)])
def test_launch_shape_does_not_change_the_chain(threads, gpc):
    _run_mixed(threads, gpc, chunks=(4, 3))


def test_cold_start_and_single_lattice_batch():
    say("cold single")
    b = lib.Batch([64], [0.4406868], seed=1, start="cold")
    s = oracle.init(64, oracle.START_COLD_UP, 1, 0)
    assert (_host(b.lattice(0)) == s).all()
    mom = b.sweep(30)
    _check_moments(mom, oracle.batch_sweep([s], [0.4406868], 1, 0, 0, 30))
    _check_spins(b, [s])


def test_batch_lattice_equals_single_lattice_api():
    """Lattice j of a batch is the INT8 chain of the single-lattice API with
    lattice id lattice_id0 + j."""
    say("batch vs single")
    b = lib.Batch([32, 64], [0.45, 0.45], seed=9, lattice_id0=5, start="random")
    b.sweep(20, moments=False)
    one = lib.Lattice(64, "int8", seed=9, lattice_id=6, start="random")
    one.sweep(0.45, 20, record=False)
    assert (_host(b.lattice(1)) == _host(one.to_int8())).all()


def test_beta_change_between_calls():
    say("set_beta")
    Ls, b0, b1 = [16, 32], [0.3, 0.5], [0.6, 0.2]
    b = lib.Batch(Ls, b0, seed=4, start="random")
    states = _oracle_states(Ls, 4, 0)
    b.sweep(6, moments=False)
    oracle.batch_sweep(states, b0, 4, 0, 0, 6)
    b.set_beta(b1)
    mom = b.sweep(5)
    _check_moments(mom, oracle.batch_sweep(states, b1, 4, 0, 6, 5))
    _check_spins(b, states)


def test_graph_capture_replays_continue_the_chain():
    """The sweep call captured once in a HIP graph: each replay advances the
    device sweep index, so three replays of 10 sweeps equal 30 eager sweeps;
    eager work and synchronisations run between the replays."""
    say("graph capture")
    Ls, betas = [32, 64, 16, 128], [0.4, 0.44, 0.5, 0.3]
    eager = lib.Batch(Ls, betas, seed=13, start="random")
    g_b = lib.Batch(Ls, betas, seed=13, start="random")
    mom = torch.zeros((4, 8), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        # warm-up on the side stream first, as torch requires before capture
        g_b.sweep(10, out=mom)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        g_b.sweep(10, out=mom)
    torch.cuda.synchronize()
    assert g_b.sweep_index == 10  # capture itself does not run the kernels
    eager.sweep(10, moments=False)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        want = eager.sweep(10)
        E, M = g_b.measure()          # eager work between replays
        assert (_host(mom) == _host(want)).all(), f"replay {rep}"
        assert (_host(E) == _host(want)[:, 0]).all()
        assert (_host(M) == _host(want)[:, 1]).all()
        assert g_b.sweep_index == eager.sweep_index == 20 + 10 * rep
    for j in range(4):
        assert (_host(g_b.lattice(j)) == _host(eager.lattice(j))).all()
    g_b.check()


def test_autotune_keeps_the_chain():
    say("autotune")
    Ls, betas = [256, 32, 64, 128, 32, 256, 64, 8], [0.44] * 8
    tuned = lib.Batch(Ls, betas, seed=17, start="random")
    plain = lib.Batch(Ls, betas, seed=17, start="random")
    tuned.sweep(3, moments=False)
    plain.sweep(3, moments=False)
    times = tuned.autotune(probe_sweeps=5)
    assert len(times) >= 4 and all(ms > 0 for _, _, ms in times)
    assert (tuned.c.threads, tuned.c.groups_per_cu) in [(t, g) for t, g, _ in times]
    assert tuned.sweep_index == 3  # the probes ran on a copy
    a, b = tuned.sweep(9), plain.sweep(9)
    assert (_host(a) == _host(b)).all()
    for j in range(len(Ls)):
        assert (_host(tuned.lattice(j)) == _host(plain.lattice(j))).all()
    assert tuned.rng_blocks() == plain.rng_blocks()


def test_sweep_without_setup_is_a_device_error_not_a_fault():
    """A workspace never set up: the prepare kernel flags it and no lattice
    is touched."""
    say("no setup")
    L = [16, 16]
    nb, _ = lib.ising_batch_spins_bytes(L)
    raw_s, spins = lib.binding._aligned_buffer(nb, "cuda")
    raw_w, ws = lib.binding._aligned_buffer(lib.ising_batch_workspace_bytes(2), "cuda")
    spins.fill_(1)
    c = lib.ising_batch(lib.binding.ABI_VERSION, 2, 1, 0, 16, 0, 0, 0, 0, nb, spins.data_ptr(), ws.data_ptr())
    lib.ising_batch_sweep(c, 5)
    with pytest.raises(lib.IsingError) as e:
        lib.ising_batch_check_device_error(c)
    assert e.value.code == lib.binding.E_STATE and "not set up" in lib.ising_last_error()
    assert (_host(spins) == 1).all()
    assert lib.ising_batch_sweep_index(c) == 0


def test_batched_workload_full_size_sampled():
    """The 1024-lattice workload (sides 32..256, 64 betas in [0.30, 0.60],
    seed 11, random starts) for 10^4 sweeps in one launch: eight lattices,
    two of each side, are checked bit for bit against the oracle over the
    whole run; every lattice's last E and M equal a recount."""
    L, beta = batched_workload()
    n, seed = 10_000, 11
    say("batched workload 1024 x 10^4")
    b = lib.Batch(L, beta, seed=seed, start="random")
    mom = b.sweep(n)
    E, M = b.measure()
    momh = _host(mom)
    assert (momh[:, 0] == _host(E)).all() and (momh[:, 1] == _host(M)).all()
    js = []
    for side in (32, 64, 128, 256):
        js += [int(j) for j in np.nonzero(L == side)[0][:2]]
    states, want = [], []
    for j in js:
        s = oracle.init(int(L[j]), oracle.START_RANDOM, seed, j)
        want.append(oracle.batch_sweep([s], [beta[j]], seed, j, 0, n, nthreads=16)[0])
        states.append(s)
    _check_moments(mom, want, js)
    _check_spins(b, states, js)
    assert b.sweep_index == n
    b.check()


@pytest.mark.parametrize("draws", ["site", "plane"])
def test_largest_batch_count_sampled(draws):
    """65536 lattices, the most a batch takes, of two alternating sides:
    five sampled lattices (both ends and the middle) bit for bit against the
    oracle, and every lattice's last E and M against a recount."""
    count, n, seed = 65536, 4, 23
    sides = (16, 32) if draws == "site" else (32, 64)
    L = np.array([sides[j & 1] for j in range(count)], np.int32)
    beta = np.array([0.30 + 0.3 * (j % 64) / 63 for j in range(count)])
    say(f"largest batch {count} draws={draws}")
    b = lib.Batch(L, beta, seed=seed, start="random", draws=draws)
    mom = b.sweep(n)
    E, M = b.measure()
    momh = _host(mom)
    assert (momh[:, 0] == _host(E)).all() and (momh[:, 1] == _host(M)).all()
    mode = oracle.MODE_SITE if draws == "site" else oracle.MODE_PLANE
    js = [0, 1, count // 2, count - 2, count - 1]
    states, want = [], []
    for j in js:
        s = oracle.init(int(L[j]), oracle.START_RANDOM, seed, j)
        want.append(oracle.batch_sweep([s], [beta[j]], seed, j, 0, n, mode=mode)[0])
        states.append(s)
    _check_moments(mom, want, js)
    _check_spins(b, states, js)
    assert b.sweep_index == n
    b.check()
