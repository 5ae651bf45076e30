"""End-to-end physics of the GPU path, independent of the oracle: long
chains on the GPU against exact results (Kaufman's finite-lattice energy
at the critical point, Onsager's infinite-lattice energy in the disordered
phase, Yang's spontaneous magnetisation in the ordered phase).  Errors are
from contiguous bins of the autocorrelated series; the bar is 4 standard
errors, and each test also checks that its error is small enough to
separate the exact value from a nearby wrong one."""
import sys

import numpy as np
import pytest

import exact

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_06415_amd as lib  # noqa: E402

BC = 0.4406868


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib.load_library()
    yield
    torch.cuda.synchronize()


def _series(L, layout, seed, beta, burn, n, start="random"):
    g = lib.Lattice(L, layout, seed=seed, start=start)
    g.sweep(beta, burn, record=False)
    E, M = g.sweep(beta, n)
    torch.cuda.synchronize()
    g.check()
    N = L * L
    return E.cpu().numpy() / N, M.cpu().numpy() / N


@pytest.mark.parametrize("layout,L", [("bit1", 64), ("int8", 32)])
def test_critical_energy_matches_kaufman(layout, L):
    say(f"{layout} L={L} beta_c 2e5 sweeps")
    e, _ = _series(L, layout, 13, BC, 2_000, 200_000)
    want = exact.kaufman_energy(BC, L)
    mean, err = exact.binned_mean_error(e, 40)
    assert abs(mean - want) < 4 * err, (mean, want, err)
    # precise enough to tell the finite lattice from the infinite one
    assert abs(exact.onsager_energy(BC) - want) > 4 * err


def test_disordered_energy_matches_onsager():
    say("bit1 L=256 beta=0.3")
    e, _ = _series(256, "bit1", 17, 0.3, 500, 20_000)
    mean, err = exact.binned_mean_error(e, 40)
    want = exact.onsager_energy(0.3)
    assert abs(mean - want) < 4 * err and err < 2e-4, (mean, want, err)


def test_ordered_magnetisation_matches_yang():
    # from the aligned start: a random start can leave the torus in a
    # long-lived striped state with |m| near 0
    say("bit1 L=256 beta=0.6")
    _, m = _series(256, "bit1", 19, 0.6, 2_000, 20_000, start="cold")
    mean, err = exact.binned_mean_error(np.abs(m), 40)
    want = exact.yang_magnetisation(0.6)
    assert abs(mean - want) < 4 * err and err < 2e-4, (mean, want, err)


def test_batch_of_independent_lattices_matches_onsager():
    """256 independent plane-draw lattices of side 64 at beta = 0.3: the
    per-lattice means of e over 4000 sweeps scatter as independent samples
    around Onsager's value."""
    say("plane batch 256 x L=64 beta=0.3")
    b = lib.Batch([64] * 256, [0.3] * 256, seed=23, start="random", draws="plane")
    b.sweep(500, moments=False)
    mom = b.sweep(4000).cpu().numpy()
    b.check()
    e = mom[:, 2].astype(np.float64) / 4000 / (64 * 64)  # sum_E per lattice
    mean, err = float(e.mean()), float(e.std(ddof=1) / np.sqrt(len(e)))
    want = exact.onsager_energy(0.3)
    assert abs(mean - want) < 4 * err and err < 2e-4, (mean, want, err)
