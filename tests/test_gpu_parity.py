"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer work, so the bar is bit-exact: the spin configuration (through
ising_to_int8) and the int64 E and M after every sweep must equal the
oracle's under the same Philox streams and thresholds.  Cases span the
parity workload (L = 16, int8, cold start, beta = 0.4406868, 10^4 sweeps,
E and M every sweep), ragged and tiny lattices, every kernel variant (the
resident single-workgroup, the persistent tile-resident, and the
one-launch-per-half-sweep kernels), beta edge cases, and the throughput
workload (L = 4096, one bit per spin, random start seed 7) at full size on
sampled sweeps.
"""
import sys

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_06415_amd as lib  # noqa: E402

BC = 0.4406868
SITE, PLANE = oracle.MODE_SITE, oracle.MODE_PLANE


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib.load_library()
    yield
    torch.cuda.synchronize()


def _mode(layout):
    return SITE if layout == "int8" else PLANE


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _gpu_lattice(L, layout, seed, start, flags=0, lattice_id=0):
    lat = lib.Lattice(L, layout, seed=seed, lattice_id=lattice_id, start=start, flags=flags)
    return lat


def _compare_stepwise(L, layout, seed, start, beta, n, flags=0, chunk=1, lattice_id=0,
                      record=True, tiles=None):
    """Sweep GPU and oracle side by side; compare spins, E, M after each call.

    record=False runs the sweeps without per-sweep observables (the kernel
    the benchmark times) and compares a recount instead."""
    say(f"L={L} layout={layout} seed={seed} start={start} beta={beta} n={n} flags={flags} "
        f"chunk={chunk} record={record} tiles={tiles}")
    g = _gpu_lattice(L, layout, seed, start, flags, lattice_id)
    s = oracle.init(L, oracle.START_COLD_UP if start == "cold" else oracle.START_RANDOM, seed,
                    lattice_id)
    assert (_host(g.to_int8()) == s).all(), "initial configuration differs"
    done = 0
    while done < n:
        k = min(chunk, n - done)
        E, M = g.sweep(beta, k, record=record, tiles=tiles)
        Eo, Mo = oracle.sweep(s, _mode(layout), seed, lattice_id, done, k, beta,
                              nthreads=oracle.max_threads())
        if record:
            Eg, Mg = _host(E), _host(M)
            assert (Eg == Eo).all() and (Mg == Mo).all(), f"E/M differ in sweeps {done}..{done + k}"
        else:
            assert tuple(_host(g.measure()).tolist()) == (Eo[-1], Mo[-1])
        got = _host(g.to_int8())
        if not (got == s).all():
            bad = np.argwhere(got != s)
            raise AssertionError(f"spins differ after sweep {done + k}: {len(bad)} sites, "
                                 f"first {bad[:5].tolist()}")
        done += k
    m = _host(g.measure())
    assert tuple(m.tolist()) == oracle.measure(s)
    assert g.sweep_index == n
    g.check()


def test_parity_workload_L16_int8_every_sweep():
    """L=16 int8, cold start, beta=0.4406868, Philox seed 1, 10^4 sweeps,
    E and M every sweep: whole traces and final spins bit-exact."""
    L, n, seed = 16, 10_000, 1
    say("parity workload L=16 n=10000")
    g = _gpu_lattice(L, "int8", seed, "cold")
    E, M = g.sweep(BC, n)
    s = oracle.init(L, oracle.START_COLD_UP, seed)
    Eo, Mo = oracle.sweep(s, SITE, seed, 0, 0, n, BC)
    assert (_host(E) == Eo).all()
    assert (_host(M) == Mo).all()
    assert (_host(g.to_int8()) == s).all()
    g.check()


def test_parity_workload_L16_spins_after_every_sweep():
    _compare_stepwise(16, "int8", 1, "cold", BC, 300)


@pytest.mark.parametrize("L", [4, 6, 10, 14, 64, 122])
def test_int8_resident_kernel(L):
    # up to L = 64, and sides up to 128 that are not multiples of 8
    _compare_stepwise(L, "int8", 3, "random", BC, 40, chunk=7)


@pytest.mark.parametrize("L", [4, 6, 16, 130, 256, 1024, 2056])
def test_int8_global_halfsweep_kernel(L):
    # L % 8 == 0 takes the span kernel (L = 2056: 257 spans per row), others
    # the per-site one
    _compare_stepwise(L, "int8", 5, "random", BC, 12, flags=lib.FLAG_GLOBAL_HALFSWEEP, chunk=5)


@pytest.mark.parametrize("record", [True, False])
@pytest.mark.parametrize("L", [72, 128, 136, 200, 256, 1024, 4096])
def test_int8_tile_kernel(L, record):
    """INT8 lattices above L = 64 with L % 8 == 0 run the persistent tile
    kernel (tiles of full rows as bytes in LDS, tagged halo hand-off of the
    edge rows' new bytes): one-row tiles from L = 72 (nine spans a row) to
    256, taller ones from L = 512 on."""
    _compare_stepwise(L, "int8", 11, "random", BC, 7 if L >= 4096 else 12, chunk=4,
                      record=record)


@pytest.mark.parametrize("L,rows,waves", [(1024, 4, 4), (1024, 2, 1), (1024, 16, 16),
                                          (256, 1, 1), (256, 8, 2), (4096, 8, 8)])
def test_int8_tile_shapes(L, rows, waves):
    """The INT8 tile kernel under tile shapes other than the library's."""
    _compare_stepwise(L, "int8", 12, "random", BC, 9, chunk=3, tiles=(rows, waves))


@pytest.mark.parametrize("beta", [0.0, 3.0])
def test_int8_tile_kernel_beta_edges(beta):
    _compare_stepwise(256, "int8", 13, "random", beta, 6, chunk=3)


@pytest.mark.parametrize("record", [True, False])
@pytest.mark.parametrize("L", [64, 128, 192, 320, 1024, 2048])
def test_bit1_tile_kernel(L, record):
    # record=True and record=False instantiate the tile kernel with and
    # without per-sweep observables
    _compare_stepwise(L, "bit1", 7, "random", BC, 12, chunk=5, record=record)


@pytest.mark.parametrize("L", [64, 192, 512])
def test_bit1_global_halfsweep_kernel(L):
    _compare_stepwise(L, "bit1", 9, "random", BC, 8, flags=lib.FLAG_GLOBAL_HALFSWEEP, chunk=3)


def test_bit1_global_kernel_several_words_per_thread():
    """L = 24576 does not fit the tile plan (the whole lattice must sit in
    LDS), so it runs one launch per half-sweep from global memory, where a
    thread takes nine words in a grid-stride loop."""
    _compare_stepwise(24576, "bit1", 5, "random", BC, 2, chunk=2)


@pytest.mark.parametrize("beta", [0.0, 1e-12, 0.3, 0.6, 3.0])
@pytest.mark.parametrize("layout,L", [("int8", 12), ("bit1", 128)])
def test_beta_edge_cases(layout, L, beta):
    _compare_stepwise(L, layout, 2, "random", beta, 6, chunk=3)


def test_seed_high_word_and_lattice_id():
    _compare_stepwise(16, "int8", (123 << 32) | 77, "random", BC, 5, lattice_id=9)
    _compare_stepwise(128, "bit1", (5 << 32) | 3, "random", BC, 5, lattice_id=4)


@pytest.mark.parametrize("layout,L", [("int8", 16), ("int8", 200), ("bit1", 256)])
def test_measure_and_roundtrip_on_random_states(layout, L):
    say(f"measure/roundtrip {layout} L={L}")
    rng = np.random.default_rng(L)
    g = _gpu_lattice(L, layout, 1, "cold")
    for _ in range(3):
        s = rng.choice(np.array([-1, 1], dtype=np.int8), size=(L, L))
        g.from_int8(torch.from_numpy(s))
        assert (_host(g.to_int8()) == s).all()
        assert tuple(_host(g.measure()).tolist()) == oracle.measure(s)


@pytest.mark.parametrize("layout,L", [("int8", 16), ("bit1", 128)])
def test_z2_and_split_invariance(layout, L):
    say(f"z2/split {layout} L={L}")
    a = _gpu_lattice(L, layout, 4, "random")
    s0 = _host(a.to_int8())
    b = _gpu_lattice(L, layout, 4, "cold")
    b.from_int8(torch.from_numpy(-s0))
    Ea, Ma = a.sweep(BC, 30)
    Eb1, Mb1 = b.sweep(BC, 13)
    Eb2, Mb2 = b.sweep(BC, 17)
    assert (_host(a.to_int8()) == -_host(b.to_int8())).all()
    assert (_host(Ea) == np.concatenate([_host(Eb1), _host(Eb2)])).all()
    assert (_host(Ma) == -np.concatenate([_host(Mb1), _host(Mb2)])).all()


def test_no_trace_equals_trace_run():
    for layout, L in (("int8", 16), ("bit1", 256)):
        say(f"record=False {layout} L={L}")
        a = _gpu_lattice(L, layout, 6, "random")
        b = _gpu_lattice(L, layout, 6, "random")
        a.sweep(BC, 9, record=False)
        b.sweep(BC, 9, record=True)
        assert (_host(a.to_int8()) == _host(b.to_int8())).all()


@pytest.mark.parametrize("record", [True, False])
def test_throughput_workload_L4096_bit1_first_sweeps(record):
    """L=4096, 1 bit/spin, random start seed 7, beta=0.4406868: the first
    sweeps bit-exact against the oracle at full size, in both tile kernels
    (record=False is the kernel the benchmark times)."""
    _compare_stepwise(4096, "bit1", 7, "random", BC, 6, chunk=2, record=record)


def test_bit1_tile_kernel_L8192_two_rows_per_wave():
    """L = 8192 puts four tiles of eight rows on each CU, four waves per
    tile: every wave updates two rows per half-sweep."""
    _compare_stepwise(8192, "bit1", 3, "random", BC, 3, chunk=2, record=True)


def test_bit1_tile_kernel_L16384_four_words_per_lane():
    """L = 16384: four tiles of sixteen rows per CU still fit LDS; a lane
    updates four words of each of its four rows per half-sweep."""
    _compare_stepwise(16384, "bit1", 4, "random", BC, 2, chunk=2, record=True)


def test_throughput_workload_L4096_sampled_over_1000_sweeps():
    """Full 10^3-sweep run: one call equals the split run, and sampled
    sweeps are checked one by one against the oracle from the GPU state."""
    L, seed, n = 4096, 7, 1000
    say("L=4096 1000 sweeps sampled")
    full = _gpu_lattice(L, "bit1", seed, "random")
    Ef, Mf = full.sweep(BC, n)
    bench = _gpu_lattice(L, "bit1", seed, "random")
    bench.sweep(BC, n, record=False)  # the configuration the benchmark times
    samples = [0, 1, 250, 777, 999]
    g = _gpu_lattice(L, "bit1", seed, "random")
    done = 0
    for t in samples:
        if t > done:
            g.sweep(BC, t - done, record=False)
            done = t
        before = _host(g.to_int8())
        E, M = g.sweep(BC, 1)
        done += 1
        s = before.copy()
        Eo, Mo = oracle.sweep(s, PLANE, seed, 0, t, 1, BC, nthreads=16)
        assert (_host(g.to_int8()) == s).all(), f"sweep {t}"
        assert _host(E)[0] == Eo[0] and _host(M)[0] == Mo[0]
        assert _host(Ef)[t] == Eo[0] and _host(Mf)[t] == Mo[0]
    if done < n:
        g.sweep(BC, n - done, record=False)
    assert (_host(g.to_int8()) == _host(full.to_int8())).all()
    assert (_host(bench.to_int8()) == _host(full.to_int8())).all()
    bench.check()
    assert tuple(_host(full.measure()).tolist()) == (int(_host(Ef)[-1]), int(_host(Mf)[-1]))
    full.check()
    g.check()


def test_throughput_workload_L4096_chained_50_sweeps():
    """L=4096, 1 bit/spin, random start seed 7, beta=0.4406868: 50
    consecutive sweeps of the kernel the benchmark times (no per-sweep
    observables), the spins compared with the oracle's after every one."""
    _compare_stepwise(4096, "bit1", 7, "random", BC, 50, chunk=1, record=False)


def test_throughput_workload_L4096_full_1000_sweeps_against_oracle():
    """The whole throughput workload in one call (10^3 sweeps): E and M
    after every sweep and the final spins equal the oracle's chain from the
    same start."""
    L, seed, n = 4096, 7, 1000
    say("L=4096 1000 sweeps, full chain against the oracle")
    g = _gpu_lattice(L, "bit1", seed, "random")
    E, M = g.sweep(BC, n)
    s = oracle.init(L, oracle.START_RANDOM, seed)
    Eo, Mo = oracle.sweep(s, PLANE, seed, 0, 0, n, BC, nthreads=oracle.max_threads())
    assert (_host(E) == Eo).all() and (_host(M) == Mo).all()
    assert (_host(g.to_int8()) == s).all()
    g.check()


# (rows per tile, waves per tile): the library's plan at L = 4096 on 256
# CUs is (4, 4); the others put one, two or four rows on a wave, one to
# sixteen waves on a tile, and 128 to 1024 tiles on the GPU.
TILE_SHAPES = [(4, 4), (4, 2), (4, 1), (8, 8), (8, 2), (16, 16), (16, 4), (32, 8)]


def test_tile_shapes_give_the_same_chain_L4096():
    """The throughput lattice under eight tile shapes: every shape gives the
    same E and M after every sweep and the same spins, equal to the
    oracle's chain."""
    L, seed, n = 4096, 7, 20
    s = oracle.init(L, oracle.START_RANDOM, seed)
    Eo, Mo = oracle.sweep(s, PLANE, seed, 0, 0, n, BC, nthreads=oracle.max_threads())
    for rows, waves in TILE_SHAPES:
        say(f"L=4096 tiles rows={rows} waves={waves} n={n}")
        g = _gpu_lattice(L, "bit1", seed, "random")
        E, M = g.sweep(BC, n, tiles=(rows, waves))
        assert (_host(E) == Eo).all() and (_host(M) == Mo).all(), (rows, waves)
        assert (_host(g.to_int8()) == s).all(), (rows, waves)
        g.check()


@pytest.mark.parametrize("rows,waves", [(2, 2), (4, 1), (8, 4)])
def test_tile_shapes_at_a_ragged_side(rows, waves):
    """L = 320 (five words per row) under shapes other than the library's."""
    _compare_stepwise(320, "bit1", 8, "random", BC, 9, chunk=4, tiles=(rows, waves))


def test_sweep_tiles_reports_shapes_the_device_cannot_hold():
    """A tile of 512 rows at L = 4096 needs 256 KiB of LDS: refused before
    any launch, the lattice untouched."""
    g = _gpu_lattice(4096, "bit1", 7, "random")
    before = _host(g.to_int8())
    with pytest.raises(lib.IsingError) as e:
        g.sweep(BC, 1, tiles=(512, 16))
    assert e.value.code == lib.binding.E_UNSUPPORTED
    assert g.sweep_index == 0
    assert (_host(g.to_int8()) == before).all()


@pytest.mark.parametrize("layout,L,flags", [("bit1", 256, 0), ("bit1", 4096, 0),
                                            ("int8", 64, 0), ("int8", 200, 0),
                                            ("bit1", 192, lib.FLAG_GLOBAL_HALFSWEEP)])
def test_checkpoint_and_resume(layout, L, flags):
    """Checkpoint = the spins in the canonical int8 form plus the sweep
    index.  Restored into a fresh lattice, the chain continues bit for bit
    as if it had never stopped: spins, and E and M after every sweep."""
    say(f"checkpoint {layout} L={L} flags={flags}")
    seed, n1, n2 = 13, 7, 11
    a = _gpu_lattice(L, layout, seed, "random", flags)
    Ea, Ma = a.sweep(BC, n1 + n2)
    b = _gpu_lattice(L, layout, seed, "random", flags)
    b.sweep(BC, n1, record=False)
    ckpt_spins, ckpt_t = b.to_int8().cpu(), b.sweep_index
    del b
    c = _gpu_lattice(L, layout, seed, "cold", flags)  # fresh lattice, other start
    c.from_int8(ckpt_spins)
    c.set_sweep_index(ckpt_t)
    Ec, Mc = c.sweep(BC, n2)
    assert (_host(Ec) == _host(Ea)[n1:]).all() and (_host(Mc) == _host(Ma)[n1:]).all()
    assert (_host(c.to_int8()) == _host(a.to_int8())).all()
    assert c.sweep_index == n1 + n2
    c.check()


def _expected_plane_blocks(s, beta, seed, lid, t0, n):
    """Philox blocks a bit-plane sweep must draw, counted from the oracle's
    chain: a word (32 sites of one colour) needs blocks until each of its
    sites with a draw is decided, i.e. ceil(d / 4) for the deepest site,
    d being the position (from the most significant bit, counted from 1)
    of the first bit where r and the site's threshold differ (32 if equal).
    The oracle's own sweep advances the state."""
    L = s.shape[0]
    T, a = oracle.thresholds(beta)
    yy, xx = np.indices((L, L))
    group = ((yy * L + xx) >> 1) >> 5
    total = 0
    for t in range(t0, t0 + n):
        for c in (0, 1):
            r = oracle.fill_uniforms(L, PLANE, seed, lid, t, c)
            h = (np.roll(s, 1, 0) + np.roll(s, -1, 0) + np.roll(s, 1, 1) +
                 np.roll(s, -1, 1)).astype(np.int64)
            u = s.astype(np.int64) * h
            k = (u + 4) // 2
            need = (((xx + yy) & 1) == c) & (u > 0) & (a[k] == 0)
            x = (r ^ T[k]).astype(np.uint64)
            depth = np.where(x == 0, 32,
                             32 - np.floor(np.log2(np.maximum(x, 1).astype(np.float64))))
            blocks = np.where(need, (depth.astype(np.int64) + 3) // 4, 0)
            per_group = np.zeros(group.max() + 1, np.int64)
            np.maximum.at(per_group, group.ravel(), blocks.ravel())
            total += int(per_group.sum())
            oracle.halfsweep(s, c, r, T, a)
    return total


@pytest.mark.parametrize("L,flags", [(256, 0), (4096, 0), (192, lib.FLAG_GLOBAL_HALFSWEEP)])
def test_rng_block_count_equals_count_from_the_oracle(L, flags):
    """ising_rng_blocks (the draw count behind the benchmark's ALU work)
    equals the blocks the oracle's chain needs, word by word; without the
    counting flag the kernels count nothing and give the same chain."""
    say(f"rng blocks L={L} flags={flags}")
    seed, n = 21, 3 if L > 1024 else 6
    g = _gpu_lattice(L, "bit1", seed, "random", flags | lib.FLAG_COUNT_DRAWS)
    g.sweep(BC, n, record=False)
    got = g.rng_blocks()
    plain = _gpu_lattice(L, "bit1", seed, "random", flags)
    plain.sweep(BC, n, record=False)
    assert plain.rng_blocks() == 0
    assert (_host(plain.to_int8()) == _host(g.to_int8())).all()
    s = oracle.init(L, oracle.START_RANDOM, seed)
    want = _expected_plane_blocks(s, BC, seed, 0, 0, n)
    assert got == want
    assert (_host(g.to_int8()) == s).all()
