"""GPU parity of the XY model against the float64 oracle (oracle/xy_oracle.c).

Both sides draw the same Philox trials and form the energy change in
double precision without fused multiply-adds: the oracle as the sum of
eight cosines of angle differences, the kernel through cached cos/sin of
every angle and the angle-difference identity (in LDS, one workgroup per
lattice or one per band of rows, or in global memory for many large
lattices).  The two agree to a few units in the last place, so the angles
must agree bit for bit: a decision could only differ where p lies that
close to the acceptance probability (probability ~1e-15 per trial).  The
energy trace is a recount at the start of each call plus the accepted
changes: within 1e-12 relative of 2 L^2 of the oracle's recount."""
import sys

import numpy as np
import pytest

import oracle

from test_oracle_xy import _ring_mean_energy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_06415_amd as lib  # noqa: E402

BETA_XY = 1.0 / 0.85


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


def _compare(L, count, beta, seed, chunks, lid0=0, start="random"):
    say(f"xy L={L} count={count} beta={beta} chunks={chunks}")
    g = lib.XYLattices(L, count, seed=seed, lattice_id0=lid0, start=start)
    st = oracle.START_RANDOM if start == "random" else oracle.START_COLD_UP
    th = [oracle.xy_init(L, st, seed, lid0 + j) for j in range(count)]
    assert (_host(g.theta) == np.stack(th)).all()
    t = 0
    accs = np.zeros(count, np.int64)
    for n in chunks:
        E = _host(g.sweep(beta, n))
        for j in range(count):
            Eo, a = oracle.xy_sweep(th[j], seed, lid0 + j, t, n, beta)
            accs[j] += a
            assert np.allclose(E[:, j], Eo, rtol=0, atol=1e-12 * 2 * L * L), (j, E[:, j], Eo)
        t += n
        got = _host(g.theta)
        for j in range(count):
            if not (got[j] == th[j]).all():
                raise AssertionError(f"lattice {j}: {(got[j] != th[j]).sum()} angles differ "
                                     f"after sweep {t}")
    gt, gacc = g.state()
    assert gt == t and (gacc == accs).all()
    assert np.allclose(_host(g.energy()), [oracle.xy_energy(x) for x in th], rtol=0,
                       atol=1e-12 * 2 * L * L)
    g.check()


@pytest.mark.parametrize("L", [2, 4, 6, 16, 32])
def test_xy_bit_exact_at_the_papers_temperature(L):
    _compare(L, 3, BETA_XY, 11, (5, 4), lid0=2)


@pytest.mark.parametrize("beta", [0.0, 0.3, 20.0])
def test_xy_beta_cases(beta):
    _compare(8, 2, beta, 5, (6,), start="cold" if beta == 20.0 else "random")


@pytest.mark.parametrize("L", [34, 64, 80, 82, 84])
def test_xy_band_tiled_form(L):
    """Two lattices (fewer than compute units) of 32 < L <= 128 take the
    band-tiled form: bands of rows resident for the whole call, the edge
    rows' cosines and sines handed over through tagged slots, refilled from
    the angles at each of the two calls.  L = 34 and 82 have only bands of
    two rows (L/2 prime)."""
    _compare(L, 2, BETA_XY, 13, (4, 3), lid0=1)


def test_xy_one_workgroup_form_above_l32():
    """As many lattices as compute units keep one workgroup per lattice up
    to L = 80 (angles, cosines and sines in LDS, 150 KiB at L = 80): three
    sampled lattices of 48 equal the oracle's bit for bit."""
    L, seed, lid0 = 48, 23, 3
    count = torch.cuda.get_device_properties(0).multi_processor_count
    say(f"xy one workgroup L={L} count={count}")
    g = lib.XYLattices(L, count, seed=seed, lattice_id0=lid0, start="random")
    picks = (0, count // 2, count - 1)
    th = {j: oracle.xy_init(L, oracle.START_RANDOM, seed, lid0 + j) for j in picks}
    t = 0
    for n in (3, 2):
        E = _host(g.sweep(BETA_XY, n))
        for j in picks:
            Eo, _ = oracle.xy_sweep(th[j], seed, lid0 + j, t, n, BETA_XY)
            assert np.allclose(E[:, j], Eo, rtol=0, atol=1e-12 * 2 * L * L), j
        t += n
        got = _host(g.theta[list(picks)])
        for k, j in enumerate(picks):
            assert (got[k] == th[j]).all(), f"lattice {j} after sweep {t}"
    g.check()


@pytest.mark.parametrize("L", [32, 96])
def test_xy_trace_does_not_change_the_chain(L):
    """Sweeping without an energy trace skips all energy work; the angles
    must equal the traced run's bit for bit, and the trace's last entry the
    recount (workgroup-resident form at L = 32, band-tiled form at L = 96)."""
    say(f"xy no trace L={L}")
    a = lib.XYLattices(L, 3, seed=17, start="random")
    b = lib.XYLattices(L, 3, seed=17, start="random")
    E = _host(a.sweep(BETA_XY, 7))
    assert b.sweep(BETA_XY, 7, trace=False) is None
    assert (_host(a.theta) == _host(b.theta)).all()
    assert np.allclose(E[-1], _host(b.energy()), rtol=0, atol=1e-12 * 2 * L * L)
    (ta, acc_a), (tb, acc_b) = a.state(), b.state()
    assert ta == tb == 7 and (acc_a == acc_b).all()
    a.check()
    b.check()


def test_xy_papers_largest_size():
    """L = 128 (the paper's largest), ten seeds as in its energy study."""
    _compare(128, 10, BETA_XY, 21, (10,))


def test_xy_sweep_before_init_is_a_device_error():
    say("xy no init")
    raw_t, th = lib.binding._aligned_buffer(4 * 4 * 8, "cuda")
    raw_w, ws = lib.binding._aligned_buffer(lib.ising_xy_workspace_bytes(4, 1), "cuda")
    th.fill_(0)
    c = lib.ising_xy(lib.binding.ABI_VERSION, 4, 1, 0, 1, th.data_ptr(), ws.data_ptr())
    lib.ising_xy_sweep(c, 1.0, 3)
    with pytest.raises(lib.IsingError):
        lib.ising_xy_check_device_error(c)
    assert (_host(th) == 0).all()


def test_xy_two_by_two_torus_on_the_gpu():
    """256 GPU chains on the 2x2 torus: <E> against the Bessel closed form."""
    say("xy 2x2 torus")
    g = lib.XYLattices(2, 256, seed=17)
    g.sweep(BETA_XY, 200, trace=False)
    E = _host(g.sweep(BETA_XY, 4000))
    blocks = E.reshape(40, -1).mean(axis=1)
    err = blocks.std(ddof=1) / np.sqrt(40)
    exact = _ring_mean_energy(BETA_XY)
    assert abs(blocks.mean() - exact) < 4 * err, (blocks.mean(), exact, err)


def test_xy_largest_batch_at_the_largest_side():
    """4096 lattices of L = 128, the most the ABI takes, in the global-memory
    form (1 GiB of cached cosines and sines): three sampled lattices equal
    the oracle's bit for bit over two calls, and every lattice's carried
    energy equals its recount."""
    L, count, seed, lid0 = 128, 4096, 29, 5
    say(f"xy largest batch L={L} count={count}")
    g = lib.XYLattices(L, count, seed=seed, lattice_id0=lid0, start="random")
    picks = (0, 2047, count - 1)
    th = {j: oracle.xy_init(L, oracle.START_RANDOM, seed, lid0 + j) for j in picks}
    t = 0
    for n in (2, 1):
        E = _host(g.sweep(BETA_XY, n))
        for j in picks:
            Eo, _ = oracle.xy_sweep(th[j], seed, lid0 + j, t, n, BETA_XY)
            assert np.allclose(E[:, j], Eo, rtol=0, atol=1e-12 * 2 * L * L), j
        t += n
        got = _host(g.theta[list(picks)])
        for k, j in enumerate(picks):
            assert (got[k] == th[j]).all(), f"lattice {j} after sweep {t}"
    assert np.allclose(E[-1], _host(g.energy()), rtol=0, atol=1e-12 * 2 * L * L)
    assert g.state()[0] == 3
    g.check()
