"""GPU parity of batches with bit-plane draws (ISING_DRAWS_PLANE): lattices
of side 32 or a multiple of 64, kept in LDS as colour bit planes and
updated 32 sites per lane, against the oracle's plane mode run lattice by
lattice.  Integer work: spins, E, M, every moment and every trace entry
must be bit-exact, and the launch shape, graph capture and the autotuner
must not change the chain."""
import sys

import numpy as np
import pytest

import oracle
from paper_2402_06415_amd.workloads import batched_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_06415_amd as lib  # noqa: E402

PLANE = oracle.MODE_PLANE
# every side the plane sweep handles, several of each, uneven order
MIXED_L = [32, 64, 128, 256, 192, 32, 64, 32, 128, 32, 64, 256]
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


def _states(Ls, seed, lid0, start="random"):
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
    say(f"plane batch threads={threads} gpc={groups_per_cu} chunks={chunks}")
    b = lib.Batch(MIXED_L, MIXED_BETA, seed=seed, lattice_id0=lid0, start="random",
                  threads=threads, groups_per_cu=groups_per_cu, draws="plane")
    states = _states(MIXED_L, seed, lid0)
    _check_spins(b, states)
    t = 0
    for n in chunks:
        mom = b.sweep(n)
        want = oracle.batch_sweep(states, MIXED_BETA, seed, lid0, t, n, nthreads=8, mode=PLANE)
        t += n
        _check_moments(mom, want)
        _check_spins(b, states)
    E, M = b.measure()
    assert [tuple(x) for x in zip(_host(E), _host(M))] == [oracle.measure(s) for s in states]
    assert b.sweep_index == t
    b.check()
    return b


def test_plane_batch_bit_exact():
    _run_mixed()


@pytest.mark.parametrize("threads,gpc", [(64, 1), (128, 2), (256, 3), (512, 2), (1024, 1)])
def test_launch_shape_does_not_change_the_chain(threads, gpc):
    # 64 threads: a 256-side lattice is 16 words per lane; 1024: 64 lattices
    # of side 32 share one workgroup
    _run_mixed(threads, gpc, chunks=(4, 3))


def test_trace_matches_the_oracle_series():
    say("plane trace")
    Ls, betas, seed, n = [32, 64, 256], [0.44, 0.3, 0.5], 5, 12
    b = lib.Batch(Ls, betas, seed=seed, lattice_id0=7, start="random", draws="plane")
    tr = torch.empty((n, 3, 2), dtype=torch.int64, device="cuda")
    b.sweep(n, moments=False, trace=tr)
    trh = _host(tr)
    for j, L in enumerate(Ls):
        s = oracle.init(L, oracle.START_RANDOM, seed, 7 + j)
        E, M = oracle.sweep(s, PLANE, seed, 7 + j, 0, n, betas[j])
        assert (trh[:, j, 0] == E).all() and (trh[:, j, 1] == M).all(), f"lattice {j}"


def test_plane_batch_lattice_equals_single_bit1_lattice():
    """Lattice j of a plane-draw batch is the BIT1 chain of the single-lattice
    API with lattice id lattice_id0 + j (same start, same plane draws)."""
    say("plane batch vs single BIT1")
    b = lib.Batch([64, 128], [0.45, 0.45], seed=9, lattice_id0=5, start="random", draws="plane")
    b.sweep(20, moments=False)
    one = lib.Lattice(128, "bit1", seed=9, lattice_id=6, start="random")
    one.sweep(0.45, 20, record=False)
    assert (_host(b.lattice(1)) == _host(one.to_int8())).all()


def test_graph_capture_replays_continue_the_chain():
    say("plane graph capture")
    Ls, betas = [32, 64, 32, 128], [0.4, 0.44, 0.5, 0.3]
    eager = lib.Batch(Ls, betas, seed=13, start="random", draws="plane")
    g_b = lib.Batch(Ls, betas, seed=13, start="random", draws="plane")
    mom = torch.zeros((4, 8), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        g_b.sweep(10, out=mom)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        g_b.sweep(10, out=mom)
    torch.cuda.synchronize()
    assert g_b.sweep_index == 10
    eager.sweep(10, moments=False)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        want = eager.sweep(10)
        E, M = g_b.measure()
        assert (_host(mom) == _host(want)).all(), f"replay {rep}"
        assert (_host(E) == _host(want)[:, 0]).all()
        assert (_host(M) == _host(want)[:, 1]).all()
        assert g_b.sweep_index == eager.sweep_index == 20 + 10 * rep
    for j in range(4):
        assert (_host(g_b.lattice(j)) == _host(eager.lattice(j))).all()
    g_b.check()


def test_autotune_keeps_the_chain():
    say("plane autotune")
    Ls, betas = [256, 32, 64, 128, 32, 256, 64, 32], [0.44] * 8
    tuned = lib.Batch(Ls, betas, seed=17, start="random", draws="plane")
    plain = lib.Batch(Ls, betas, seed=17, start="random", draws="plane")
    tuned.sweep(3, moments=False)
    plain.sweep(3, moments=False)
    times = tuned.autotune(probe_sweeps=5)
    assert len(times) >= 4 and all(ms > 0 for _, _, ms in times)
    assert tuned.sweep_index == 3
    a, b = tuned.sweep(9), plain.sweep(9)
    assert (_host(a) == _host(b)).all()
    for j in range(len(Ls)):
        assert (_host(tuned.lattice(j)) == _host(plain.lattice(j))).all()
    assert tuned.rng_blocks() == plain.rng_blocks()


def test_several_passes_per_workgroup():
    """20,000 lattices of side 32 on 64-thread workgroups, one per CU: each
    workgroup holds about 78 lattices, more than the 64 teams of one pass,
    so it sweeps them in two passes of one lane per lattice.  Lattices from
    both passes and from both ends of the snake are checked bit for bit."""
    say("plane batch, two passes per workgroup")
    cnt, n, seed = 20_000, 5, 29
    Ls = [32] * cnt
    betas = [0.30 + 0.30 * (k % 64) / 63 for k in range(cnt)]
    b = lib.Batch(Ls, betas, seed=seed, start="random", threads=64, groups_per_cu=1,
                  draws="plane")
    mom = b.sweep(n)
    G = min(cnt, torch.cuda.get_device_properties(0).multi_processor_count)
    # first and second pass of workgroup 0 and of the last workgroup
    js = sorted({0, 2 * G - 1, 64 * G, 64 * G + 2 * G - 1 if 64 * G + 2 * G - 1 < cnt else cnt - 1,
                 G - 1, G, cnt - 1, cnt // 2})
    want, states = [], []
    for j in js:
        s = oracle.init(32, oracle.START_RANDOM, seed, j)
        want.append(oracle.batch_sweep([s], [betas[j]], seed, j, 0, n, nthreads=4, mode=PLANE)[0])
        states.append(s)
    _check_moments(mom, want, js)
    _check_spins(b, states, js)
    b.check()


def test_draw_mode_must_match_setup():
    """A sweep whose draw mode differs from setup's is a device error and
    touches no lattice."""
    say("draw mode mismatch")
    b = lib.Batch([32, 64], [0.4, 0.4], seed=3, start="random", draws="site")
    before = [_host(b.lattice(j)).copy() for j in range(2)]
    b.c.draws = lib.binding.DRAWS_PLANE
    b.sweep(4, moments=False)
    with pytest.raises(lib.IsingError) as e:
        b.check()
    assert e.value.code == lib.binding.E_STATE and "draw mode" in lib.ising_last_error()
    for j in range(2):
        assert (_host(b.lattice(j)) == before[j]).all()
    assert b.sweep_index == 0


def test_batched_workload_full_size_sampled():
    """The 1024-lattice workload (sides 32..256, 64 betas in [0.30, 0.60],
    seed 11, random starts) with plane draws for 10^4 sweeps in one launch,
    in the launch shape the benchmark picks by default: eight lattices, two
    of each side, are checked bit for bit against the oracle over the whole
    run; every lattice's last E and M equal a recount."""
    L, beta = batched_workload()
    n, seed = 10_000, 11
    say("plane batched workload 1024 x 10^4")
    b = lib.Batch(L, beta, seed=seed, start="random", draws="plane")
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
        want.append(oracle.batch_sweep([s], [beta[j]], seed, j, 0, n, nthreads=16,
                                       mode=PLANE)[0])
        states.append(s)
    _check_moments(mom, want, js)
    _check_spins(b, states, js)
    assert b.sweep_index == n
    b.check()
