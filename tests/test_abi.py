"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-only logic (sizes, thresholds, argument validation) is right.
No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2402_06415_amd as lib
from paper_2402_06415_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc))
                   if f.endswith(".h"))
    return sorted(set(re.findall(r"ISING_API\s+[\w\s\*]*?\b(ising_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    declared = _declared_symbols()
    assert len(declared) >= 12
    so = ctypes.CDLL(binding.LIB_PATH)
    for name in declared:
        assert hasattr(so, name), name
    assert sorted(binding.EXPORTED) == declared


def test_abi_version():
    assert lib.ising_abi_version() == lib.ABI_VERSION


def test_struct_layout_matches_header():
    # int32 x4, uint64, uint32 x2, uint64, two pointers
    assert ctypes.sizeof(binding.ising_lattice) == 56
    assert binding.ising_lattice.spins.offset == 40
    assert binding.ising_lattice.sweep_index.offset == 32


@pytest.mark.parametrize("L,layout,want", [(16, 0, 256), (4096, 1, 2 ** 21), (6, 0, 36),
                                           (7, 0, 0), (2, 0, 0), (96, 1, 0), (128, 1, 2048),
                                           (65536, 1, 2 ** 29), (65538, 0, 0)])
def test_spins_bytes(L, layout, want):
    assert lib.ising_spins_bytes(2, L, layout) == want
    assert lib.ising_spins_bytes(3, L, layout) == 0


def test_workspace_bytes():
    for L, layout in ((16, 0), (4096, 1), (64, 1)):
        ws = lib.ising_workspace_bytes(2, L, layout)
        assert ws > 0 and ws % 256 == 0
    assert lib.ising_workspace_bytes(2, 4096, 1) >= 256 * 128 + 256 * 4 * 64 * 4


@pytest.mark.parametrize("beta", [0.0, 1e-12, 0.1, 0.3, 0.4, 0.4406868, 0.48, 0.6, 1.2, 5.0])
def test_thresholds_equal_oracle(beta):
    T, a = lib.ising_thresholds(beta)
    To, ao = oracle.thresholds(beta)
    assert (T == To).all() and (a == ao).all()


@pytest.mark.parametrize("beta", [-1e-9, float("nan"), float("inf"), -float("inf")])
def test_thresholds_reject(beta):
    with pytest.raises(lib.IsingError) as e:
        lib.ising_thresholds(beta)
    assert e.value.code == binding.E_INVALID
    assert "beta" in lib.ising_last_error()


def _lat(**kw):
    d = dict(abi_version=binding.ABI_VERSION, dim=2, L=16, layout=0, seed=1, lattice_id=0, flags=0,
             sweep_index=0, spins=0x1000, workspace=0x2000)
    d.update(kw)
    return binding.ising_lattice(**d)


@pytest.mark.parametrize("kw,code", [
    (dict(abi_version=1), binding.E_INVALID),
    (dict(dim=3), binding.E_UNSUPPORTED),
    (dict(L=7), binding.E_INVALID),
    (dict(L=2), binding.E_INVALID),
    (dict(layout=1, L=96), binding.E_INVALID),
    (dict(layout=5), binding.E_INVALID),
    (dict(flags=8), binding.E_INVALID),
    (dict(spins=0), binding.E_INVALID),
    (dict(spins=0x1001), binding.E_INVALID),
    (dict(workspace=0), binding.E_INVALID),
    (dict(workspace=0x2080), binding.E_INVALID),
    (dict(sweep_index=2 ** 31 + 1), binding.E_INVALID),
])
def test_invalid_lattices_are_rejected_before_any_launch(kw, code):
    lat = _lat(**kw)
    before = bytes(lat)
    for call in (lambda: lib.ising_init(lat, 0), lambda: lib.ising_sweep(lat, 0.4, 1),
                 lambda: lib.ising_measure(lat, 0x3000, 0x3008),
                 lambda: lib.ising_to_int8(lat, 0x4000),
                 lambda: lib.ising_from_int8(lat, 0x4000)):
        with pytest.raises(lib.IsingError) as e:
            call()
        assert e.value.code == code
        assert bytes(lat) == before  # the lattice description is untouched


@pytest.mark.parametrize("beta,n,t0", [(-0.1, 1, 0), (float("nan"), 1, 0), (0.4, -1, 0),
                                       (0.4, 2, 2 ** 31 - 1)])
def test_sweep_argument_errors(beta, n, t0):
    lat = _lat(sweep_index=t0)
    with pytest.raises(lib.IsingError) as e:
        lib.ising_sweep(lat, beta, n)
    assert e.value.code == binding.E_INVALID
    assert lat.sweep_index == t0


def test_bad_start_and_null_buffers():
    lat = _lat()
    with pytest.raises(lib.IsingError):
        lib.ising_init(lat, 7)
    with pytest.raises(lib.IsingError):
        lib.ising_to_int8(lat, 0)
    with pytest.raises(lib.IsingError):
        lib.ising_from_int8(lat, 0)


@pytest.mark.parametrize("kw,rows,waves", [
    (dict(L=12), 4, 4),                  # INT8 tiles need L % 8 == 0
    (dict(L=16), 5, 4),                  # rows must divide L
    (dict(layout=1, L=128), 3, 1),       # rows must divide L
    (dict(layout=1, L=128), 128, 4),     # one tile: at least two
    (dict(layout=1, L=4096), 2, 2),      # 2048 tiles: at most 1024
    (dict(layout=1, L=128), 8, 0),       # waves in 1..min(16, rows)
    (dict(layout=1, L=128), 8, 9),
    (dict(layout=1, L=128, abi_version=1), 8, 8),
])
def test_sweep_tiles_rejects_bad_shapes_before_any_launch(kw, rows, waves):
    lat = _lat(**kw)
    before = bytes(lat)
    with pytest.raises(lib.IsingError) as e:
        lib.ising_sweep_tiles(lat, 0.4, 1, rows, waves)
    assert e.value.code == binding.E_INVALID
    assert bytes(lat) == before


def test_sweep_of_zero_sweeps_launches_nothing():
    lat = _lat(sweep_index=5)
    lib.ising_sweep(lat, 0.4, 0)  # host-only early return, no device touched
    assert lat.sweep_index == 5


def test_product_path_does_not_import_oracle():
    import sys
    import subprocess

    code = ("import sys; import paper_2402_06415_amd as m; m.load_library(); "
            "assert not any(k == 'oracle' or k.startswith('oracle.') for k in sys.modules)")
    subprocess.check_call([sys.executable, "-c", code], cwd=ROOT)
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_2402_06415_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "ising_oracle" not in text, f


# ------------------------------------------------------------ batch API (host side only)
def test_batch_struct_layout_matches_header():
    assert ctypes.sizeof(binding.ising_batch) == 64
    assert binding.ising_batch.draws.offset == 32
    assert binding.ising_batch.spins_bytes.offset == 40
    assert binding.ising_batch.spins.offset == 48


def test_batch_spins_bytes_and_offsets():
    nb, off = lib.ising_batch_spins_bytes([32, 8, 256, 24])
    # each lattice starts on a 256-byte boundary
    assert list(off) == [0, 1024, 1280, 1280 + 65536]
    assert nb == 1280 + 65536 + 768
    for bad in ([6], [12], [264], [0], [8, 30]):
        assert lib.ising_batch_spins_bytes(bad)[0] == 0
    assert lib.ising_batch_workspace_bytes(0) == 0
    assert lib.ising_batch_workspace_bytes(65537) == 0
    ws = lib.ising_batch_workspace_bytes(1024)
    assert ws % 256 == 0 and ws >= 1280 + 4 * 1024 + 32 * 1024


def _batch(**kw):
    d = dict(abi_version=binding.ABI_VERSION, count=2, seed=1, lattice_id0=0, max_L=32, threads=0, groups_per_cu=0,
             spins_bytes=4096, spins=0x10000, workspace=0x20000)
    d.update(kw)
    return binding.ising_batch(**d)


@pytest.mark.parametrize("kw", [
    dict(abi_version=99), dict(count=0), dict(count=65537), dict(max_L=12), dict(max_L=264),
    dict(threads=100), dict(threads=2048), dict(groups_per_cu=17), dict(spins=0),
    dict(spins=0x10010), dict(workspace=0), dict(workspace=0x20004),
    dict(lattice_id0=2 ** 32 - 1), dict(draws=2), dict(draws=-1), dict(reserved=1),
])
def test_invalid_batches_are_rejected_before_any_launch(kw):
    b = _batch(**kw)
    before = bytes(b)
    for call in (lambda: lib.ising_batch_setup(b, [8, 8], [0.4, 0.4]),
                 lambda: lib.ising_batch_init(b, 1), lambda: lib.ising_batch_sweep(b, 3),
                 lambda: lib.ising_batch_measure(b, 0x3000, 0x3008)):
        with pytest.raises(lib.IsingError) as e:
            call()
        assert e.value.code == binding.E_INVALID
    assert bytes(b) == before


@pytest.mark.parametrize("L,beta,msg", [([8, 40], [0.4, 0.4], "max_L"),
                                        ([8, 12], [0.4, 0.4], "multiple of 8"),
                                        ([8, 8], [0.4, float("nan")], "beta"),
                                        ([8, 8], [-1.0, 0.4], "beta"),
                                        ([32, 32], [0.4, 0.4], "spins_bytes")])
def test_batch_setup_rejects_bad_lattices_before_copying(L, beta, msg):
    b = _batch(spins_bytes=1024 + 512)
    with pytest.raises(lib.IsingError) as e:
        lib.ising_batch_setup(b, L, beta)
    assert e.value.code == binding.E_INVALID
    assert msg in lib.ising_last_error()


@pytest.mark.parametrize("L", [[32, 48], [96, 16]])
def test_plane_draws_need_L_32_or_multiple_of_64(L):
    b = _batch(draws=binding.DRAWS_PLANE, max_L=96, spins_bytes=1 << 16)
    with pytest.raises(lib.IsingError) as e:
        lib.ising_batch_setup(b, L, [0.4, 0.4])
    assert e.value.code == binding.E_INVALID and "plane draws" in lib.ising_last_error()


def test_batch_sweep_argument_errors():
    b = _batch()
    for n in (-1, 2 ** 31 + 1):
        with pytest.raises(lib.IsingError) as e:
            lib.ising_batch_sweep(b, n)
        assert e.value.code == binding.E_INVALID
    lib.ising_batch_sweep(b, 0)  # host-only early return
    with pytest.raises(lib.IsingError):
        lib.ising_batch_init(b, 9)


def _ea(**kw):
    d = dict(abi_version=binding.ABI_VERSION, L=64, replicas=2, draws=0, seed=1, spins=0x10000,
             bonds=0x20000, workspace=0x30000)
    d.update(kw)
    return binding.ising_ea(**d)


def test_ea_struct_layout_matches_header():
    assert ctypes.sizeof(binding.ising_ea) == 48
    assert binding.ising_ea.draws.offset == 12 and binding.ising_ea.seed.offset == 16


@pytest.mark.parametrize("kw,msg", [(dict(draws=2), "draws"), (dict(draws=-1), "draws"),
                                    (dict(draws=1, L=32), "plane draws need L >= 64"),
                                    (dict(L=24), "power of two"),
                                    (dict(workspace=0x30004), "aligned")])
def test_invalid_spin_glasses_are_rejected_before_any_launch(kw, msg):
    e = _ea(**kw)
    before = bytes(e)
    with pytest.raises(lib.IsingError) as err:
        lib.ising_ea_setup(e, [0.4, 0.8])
    assert err.value.code == binding.E_INVALID and msg in lib.ising_last_error()
    assert bytes(e) == before


def test_xy_workspace_bytes():
    """Above L = 32 the workspace adds 64 L bytes of hand-off slots per band
    of the band-tiled form, for at most min(count L / 2, 2048) bands, and
    above L = 80 16 B of cosine and sine per site (the per-half-sweep form)."""
    assert lib.ising_xy_workspace_bytes(1, 10) == 0
    assert lib.ising_xy_workspace_bytes(130, 10) == 0
    assert lib.ising_xy_workspace_bytes(32, 0) == 0
    assert lib.ising_xy_workspace_bytes(32, 4097) == 0
    small = lib.ising_xy_workspace_bytes(32, 10)
    assert small > 0 and small % 256 == 0
    assert lib.ising_xy_workspace_bytes(2, 10) == small
    assert lib.ising_xy_workspace_bytes(34, 10) == small + 10 * 17 * 64 * 34
    assert lib.ising_xy_workspace_bytes(80, 10) == small + 10 * 40 * 64 * 80
    trig = -(-10 * 82 * 82 * 16 // 256) * 256
    assert lib.ising_xy_workspace_bytes(82, 10) == small + trig + 10 * 41 * 64 * 82
    big = lib.ising_xy_workspace_bytes(128, 4096)
    assert big == lib.ising_xy_workspace_bytes(2, 4096) + 4096 * 128 * 128 * 16 + 2048 * 64 * 128
