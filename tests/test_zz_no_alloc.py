"""ising_sweep_noalloc (the sweep whose workspace is the library's static
scratch array) against ising_sweep (the caller's workspace), through the
C ABI: the same spins and the same E and M after every sweep, on calls in a
row that reuse the scratch, the second with a smaller lattice; a BIT1
lattice above the scratch limit is refused before any launch."""
import sys

import numpy as np
import pytest

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


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _noalloc(b, n, E=0, M=0, status=0):
    """The no-alloc sweep with the lattice's workspace pointer removed (the
    call must not need it); restored afterwards for the other calls."""
    ws = b.c.workspace
    b.c.workspace = None
    try:
        lib.ising_sweep_noalloc(b.c, BC, n, E, M, status, _stream())
    finally:
        b.c.workspace = ws


def _run_pair(L, layout, seed, n):
    say(f"noalloc {layout} L={L} n={n}")
    a = lib.Lattice(L, layout, seed=seed, start="random")
    b = lib.Lattice(L, layout, seed=seed, start="random")
    Ea, Ma = a.sweep(BC, n)
    Eb = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    Mb = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    status = torch.full((1,), 0xDEAD, dtype=torch.int32, device="cuda")
    _noalloc(b, n, Eb.data_ptr(), Mb.data_ptr(), status.data_ptr())
    assert b.c.sweep_index == n
    assert int(_host(status)[0]) == 0
    assert (_host(Eb) == _host(Ea)).all() and (_host(Mb) == _host(Ma)).all()
    assert (_host(b.to_int8()) == _host(a.to_int8())).all()
    # no traces, continuing the chain from sweep n
    Ea2, Ma2 = a.sweep(BC, 3)
    _noalloc(b, 3)
    assert (_host(b.to_int8()) == _host(a.to_int8())).all()
    a.check()


def test_noalloc_equals_sweep_two_calls_second_smaller():
    """BIT1 L = 4096 (the tile kernel, the most scratch: 1024 tiles of
    halo slots), then BIT1 L = 256 on the same scratch."""
    _run_pair(4096, "bit1", 7, 12)
    _run_pair(256, "bit1", 3, 9)


@pytest.mark.parametrize("layout,L", [("bit1", 8192), ("int8", 200), ("int8", 16), ("bit1", 192)])
def test_noalloc_equals_sweep_other_paths(layout, L):
    """The largest BIT1 side the scratch takes, the INT8 global and resident
    kernels (only the scratch header), a ragged BIT1 side."""
    _run_pair(L, layout, 5, 4 if L >= 4096 else 10)


def test_noalloc_refuses_lattices_above_the_scratch_limit():
    g = lib.Lattice(16384, "bit1", seed=1, start="cold")
    before = bytes(g.c)
    with pytest.raises(lib.IsingError) as e:
        _noalloc(g, 1)
    assert e.value.code == lib.binding.E_UNSUPPORTED
    assert bytes(g.c) == before
