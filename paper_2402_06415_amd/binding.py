"""Thin ctypes binding of libising.so (declared in include/ising.h).

Functions carry the C names and only marshal arguments; every step of the
sweep runs in the HIP kernels of the library.  There is no CPU fallback: if
the library is missing or fails to load, every call raises.

Device memory and streams come from PyTorch: ``Lattice`` allocates the spin
and workspace buffers as torch tensors on the current HIP device and passes
``torch.cuda.current_stream()`` to the library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libising.so")

ABI_VERSION = 3
LAYOUT_INT8 = 0
LAYOUT_BIT1 = 1
DRAWS_SITE = 0
DRAWS_PLANE = 1
START_COLD_UP = 0
START_RANDOM = 1
OK, E_INVALID, E_UNSUPPORTED, E_HIP, E_STATE = 0, 1, 2, 3, 4
FLAG_GLOBAL_HALFSWEEP = 1
FLAG_COUNT_DRAWS = 2

EXPORTED = (
    "ising_spins_bytes", "ising_workspace_bytes", "ising_abi_version", "ising_thresholds",
    "ising_init", "ising_sweep", "ising_sweep_tiles", "ising_sweep_noalloc", "ising_measure", "ising_to_int8", "ising_from_int8",
    "ising_check_device_error", "ising_last_error", "ising_rng_blocks",
    "ising_batch_spins_bytes", "ising_batch_workspace_bytes", "ising_batch_setup",
    "ising_batch_init", "ising_batch_sweep", "ising_batch_measure", "ising_batch_sweep_index",
    "ising_batch_rng_blocks", "ising_batch_check_device_error", "ising_batch_autotune",
    "ising_nn_param_count", "ising_nn_workspace_bytes", "ising_nn_round_weights", "ising_nn_logq",
    "ising_nn_grad", "ising_nn_adam", "ising_nn_sample", "ising_batch_mh",
    "ising_ea_spins_bytes", "ising_ea_workspace_bytes", "ising_ea_setup", "ising_ea_init",
    "ising_ea_sweep", "ising_ea_measure", "ising_ea_state", "ising_ea_check_device_error",
    "ising_ea_rng_blocks", "ising_xy_workspace_bytes", "ising_xy_init", "ising_xy_sweep",
    "ising_xy_energy", "ising_xy_state", "ising_xy_check_device_error",
)
NN_CHANNELS = 16
NN_MAX_L = 64
BATCH_MAX_L = 256
BATCH_MAX_COUNT = 65536
MOMENT_FIELDS = ("E", "M", "sum_E", "sum_E2", "sum_absM", "sum_M2", "sum_M4_lo", "sum_M4_hi")


class IsingError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"libising error {code}: {message}")
        self.code = code


class ising_lattice(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("lattice_id", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("sweep_index", ctypes.c_uint64),
        ("spins", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
    ]


class ising_batch(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("count", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("lattice_id0", ctypes.c_uint32),
        ("max_L", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("groups_per_cu", ctypes.c_int32),
        ("draws", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("spins_bytes", ctypes.c_uint64),
        ("spins", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
    ]


class ising_nn(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("channels", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("master", ctypes.c_void_p),
        ("weights", ctypes.c_void_p),
        ("grad", ctypes.c_void_p),
        ("adam_m", ctypes.c_void_p),
        ("adam_v", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
    ]


class ising_xy(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("count", ctypes.c_int32),
        ("lattice_id0", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("theta", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
    ]


class ising_ea(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("replicas", ctypes.c_int32),
        ("draws", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("spins", ctypes.c_void_p),
        ("bonds", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
    ]


_lib = None


def load_library():
    """Load libising.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lat_p = P(ising_lattice)
    vp = ctypes.c_void_p
    lib.ising_spins_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.ising_spins_bytes.restype = ctypes.c_size_t
    lib.ising_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.ising_workspace_bytes.restype = ctypes.c_size_t
    lib.ising_abi_version.argtypes = []
    lib.ising_abi_version.restype = ctypes.c_int32
    lib.ising_thresholds.argtypes = [ctypes.c_double, P(ctypes.c_uint32), P(ctypes.c_uint8)]
    lib.ising_thresholds.restype = ctypes.c_int
    lib.ising_init.argtypes = [lat_p, ctypes.c_int32, vp]
    lib.ising_init.restype = ctypes.c_int
    lib.ising_sweep.argtypes = [lat_p, ctypes.c_double, ctypes.c_int64, vp, vp, vp]
    lib.ising_sweep.restype = ctypes.c_int
    lib.ising_sweep_tiles.argtypes = [lat_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, vp, vp, vp]
    lib.ising_sweep_tiles.restype = ctypes.c_int
    lib.ising_sweep_noalloc.argtypes = [lat_p, ctypes.c_double, ctypes.c_int64, vp, vp, vp, vp]
    lib.ising_sweep_noalloc.restype = ctypes.c_int
    lib.ising_measure.argtypes = [lat_p, vp, vp, vp]
    lib.ising_measure.restype = ctypes.c_int
    lib.ising_to_int8.argtypes = [lat_p, vp, vp]
    lib.ising_to_int8.restype = ctypes.c_int
    lib.ising_from_int8.argtypes = [lat_p, vp, vp]
    lib.ising_from_int8.restype = ctypes.c_int
    lib.ising_rng_blocks.argtypes = [lat_p, P(ctypes.c_uint64), vp]
    lib.ising_rng_blocks.restype = ctypes.c_int
    lib.ising_check_device_error.argtypes = [lat_p, vp]
    lib.ising_check_device_error.restype = ctypes.c_int
    lib.ising_last_error.argtypes = []
    lib.ising_last_error.restype = ctypes.c_char_p
    bat_p = P(ising_batch)
    i32p, u64p, f64p = P(ctypes.c_int32), P(ctypes.c_uint64), P(ctypes.c_double)
    lib.ising_batch_spins_bytes.argtypes = [ctypes.c_int32, i32p, u64p]
    lib.ising_batch_spins_bytes.restype = ctypes.c_size_t
    lib.ising_batch_workspace_bytes.argtypes = [ctypes.c_int32]
    lib.ising_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.ising_batch_setup.argtypes = [bat_p, i32p, f64p, vp]
    lib.ising_batch_init.argtypes = [bat_p, ctypes.c_int32, vp]
    lib.ising_batch_sweep.argtypes = [bat_p, ctypes.c_int64, vp, vp, vp]
    lib.ising_batch_measure.argtypes = [bat_p, vp, vp, vp]
    lib.ising_batch_sweep_index.argtypes = [bat_p, u64p, vp]
    lib.ising_batch_rng_blocks.argtypes = [bat_p, u64p, vp]
    lib.ising_batch_check_device_error.argtypes = [bat_p, vp]
    lib.ising_batch_autotune.argtypes = [bat_p, vp, ctypes.c_int64, f64p, ctypes.c_int32, i32p, vp]
    for name in ("ising_batch_setup", "ising_batch_init", "ising_batch_sweep", "ising_batch_measure",
                 "ising_batch_sweep_index", "ising_batch_rng_blocks",
                 "ising_batch_check_device_error", "ising_batch_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    nn_p = P(ising_nn)
    lib.ising_nn_param_count.argtypes = [ctypes.c_int32]
    lib.ising_nn_param_count.restype = ctypes.c_int32
    lib.ising_nn_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.ising_nn_workspace_bytes.restype = ctypes.c_size_t
    lib.ising_nn_round_weights.argtypes = [nn_p, vp]
    lib.ising_nn_logq.argtypes = [nn_p, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp, vp]
    lib.ising_nn_grad.argtypes = [nn_p, vp, ctypes.c_int64, ctypes.c_int32, vp, vp]
    lib.ising_nn_adam.argtypes = [nn_p, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_int32, vp]
    lib.ising_nn_sample.argtypes = [nn_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_int32, vp, ctypes.c_int64, vp, vp]
    lib.ising_batch_mh.argtypes = [bat_p, ctypes.c_int32, vp, ctypes.c_int64, vp, vp, vp,
                                   ctypes.c_uint32, vp, vp]
    for name in ("ising_nn_round_weights", "ising_nn_logq", "ising_nn_grad", "ising_nn_adam",
                 "ising_nn_sample", "ising_batch_mh"):
        getattr(lib, name).restype = ctypes.c_int
    ea_p = P(ising_ea)
    lib.ising_ea_spins_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.ising_ea_spins_bytes.restype = ctypes.c_size_t
    lib.ising_ea_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.ising_ea_workspace_bytes.restype = ctypes.c_size_t
    lib.ising_ea_setup.argtypes = [ea_p, f64p, vp]
    lib.ising_ea_init.argtypes = [ea_p, ctypes.c_int32, vp]
    lib.ising_ea_sweep.argtypes = [ea_p, ctypes.c_int64, ctypes.c_int32, vp, vp]
    lib.ising_ea_measure.argtypes = [ea_p, vp, vp]
    lib.ising_ea_state.argtypes = [ea_p, u64p, i32p, P(ctypes.c_int64), u64p, vp]
    lib.ising_ea_check_device_error.argtypes = [ea_p, vp]
    lib.ising_ea_rng_blocks.argtypes = [ea_p, u64p, vp]
    lib.ising_ea_rng_blocks.restype = ctypes.c_int
    for name in ("ising_ea_setup", "ising_ea_init", "ising_ea_sweep", "ising_ea_measure",
                 "ising_ea_state", "ising_ea_check_device_error"):
        getattr(lib, name).restype = ctypes.c_int
    xy_p = P(ising_xy)
    lib.ising_xy_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.ising_xy_workspace_bytes.restype = ctypes.c_size_t
    lib.ising_xy_init.argtypes = [xy_p, ctypes.c_int32, vp]
    lib.ising_xy_sweep.argtypes = [xy_p, ctypes.c_double, ctypes.c_int64, vp, vp]
    lib.ising_xy_energy.argtypes = [xy_p, vp, vp]
    lib.ising_xy_state.argtypes = [xy_p, u64p, u64p, vp]
    lib.ising_xy_check_device_error.argtypes = [xy_p, vp]
    for name in ("ising_xy_init", "ising_xy_sweep", "ising_xy_energy", "ising_xy_state",
                 "ising_xy_check_device_error"):
        getattr(lib, name).restype = ctypes.c_int
    if lib.ising_abi_version() != ABI_VERSION:
        raise RuntimeError("libising.so ABI version mismatch")
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise IsingError(rc, ising_last_error())


# ------------------------------------------------------------ C-named calls
def ising_last_error() -> str:
    return load_library().ising_last_error().decode()


def ising_abi_version() -> int:
    return int(load_library().ising_abi_version())


def ising_spins_bytes(dim: int, L: int, layout: int) -> int:
    return int(load_library().ising_spins_bytes(dim, L, layout))


def ising_workspace_bytes(dim: int, L: int, layout: int) -> int:
    return int(load_library().ising_workspace_bytes(dim, L, layout))


def ising_thresholds(beta: float):
    T = np.zeros(5, dtype=np.uint32)
    a = np.zeros(5, dtype=np.uint8)
    _check(load_library().ising_thresholds(
        float(beta), T.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
        a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return T, a


def ising_init(lat: ising_lattice, start: int, stream: int = 0):
    _check(load_library().ising_init(ctypes.byref(lat), start, stream))


def ising_sweep(lat: ising_lattice, beta: float, n: int, E_dev: int = 0, M_dev: int = 0,
                stream: int = 0):
    _check(load_library().ising_sweep(ctypes.byref(lat), float(beta), int(n), E_dev or None,
                                      M_dev or None, stream))


def ising_sweep_tiles(lat: ising_lattice, beta: float, n: int, rows: int, waves: int,
                      E_dev: int = 0, M_dev: int = 0, stream: int = 0):
    _check(load_library().ising_sweep_tiles(ctypes.byref(lat), float(beta), int(n), int(rows),
                                            int(waves), E_dev or None, M_dev or None, stream))


def ising_sweep_noalloc(lat: ising_lattice, beta: float, n: int, E_dev: int = 0, M_dev: int = 0,
                        status_dev: int = 0, stream: int = 0):
    _check(load_library().ising_sweep_noalloc(ctypes.byref(lat), float(beta), int(n),
                                              E_dev or None, M_dev or None, status_dev or None,
                                              stream))


def ising_measure(lat: ising_lattice, E_dev: int = 0, M_dev: int = 0, stream: int = 0):
    _check(load_library().ising_measure(ctypes.byref(lat), E_dev or None, M_dev or None, stream))


def ising_to_int8(lat: ising_lattice, out_dev: int, stream: int = 0):
    _check(load_library().ising_to_int8(ctypes.byref(lat), out_dev, stream))


def ising_from_int8(lat: ising_lattice, in_dev: int, stream: int = 0):
    _check(load_library().ising_from_int8(ctypes.byref(lat), in_dev, stream))


def ising_rng_blocks(lat: ising_lattice, stream: int = 0) -> int:
    v = ctypes.c_uint64(0)
    _check(load_library().ising_rng_blocks(ctypes.byref(lat), ctypes.byref(v), stream))
    return int(v.value)


def ising_check_device_error(lat: ising_lattice, stream: int = 0):
    _check(load_library().ising_check_device_error(ctypes.byref(lat), stream))


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def ising_batch_spins_bytes(L_host):
    """(bytes, offsets) of the spins buffer of a batch; bytes == 0 if invalid."""
    L, Lp = _i32(L_host)
    off = np.zeros(max(len(L), 1), dtype=np.uint64)
    nb = load_library().ising_batch_spins_bytes(
        len(L), Lp, off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return int(nb), off[:len(L)]


def ising_batch_workspace_bytes(count: int) -> int:
    return int(load_library().ising_batch_workspace_bytes(int(count)))


def ising_batch_setup(b: ising_batch, L_host, beta_host, stream: int = 0):
    L, Lp = _i32(L_host)
    be, bp = _f64(beta_host)
    if len(L) != b.count or len(be) != b.count:
        raise IsingError(E_INVALID, "L_host and beta_host need one entry per lattice")
    _check(load_library().ising_batch_setup(ctypes.byref(b), Lp, bp, stream))


def ising_batch_init(b: ising_batch, start: int, stream: int = 0):
    _check(load_library().ising_batch_init(ctypes.byref(b), start, stream))


def ising_batch_sweep(b: ising_batch, n: int, moments_dev: int = 0, trace_dev: int = 0,
                      stream: int = 0):
    _check(load_library().ising_batch_sweep(ctypes.byref(b), int(n), moments_dev or None,
                                            trace_dev or None, stream))


def ising_batch_measure(b: ising_batch, E_dev: int = 0, M_dev: int = 0, stream: int = 0):
    _check(load_library().ising_batch_measure(ctypes.byref(b), E_dev or None, M_dev or None,
                                              stream))


def ising_batch_sweep_index(b: ising_batch, stream: int = 0) -> int:
    v = ctypes.c_uint64(0)
    _check(load_library().ising_batch_sweep_index(ctypes.byref(b), ctypes.byref(v), stream))
    return int(v.value)


def ising_batch_rng_blocks(b: ising_batch, stream: int = 0) -> int:
    v = ctypes.c_uint64(0)
    _check(load_library().ising_batch_rng_blocks(ctypes.byref(b), ctypes.byref(v), stream))
    return int(v.value)


def ising_batch_check_device_error(b: ising_batch, stream: int = 0):
    _check(load_library().ising_batch_check_device_error(ctypes.byref(b), stream))


def ising_batch_autotune(b: ising_batch, scratch_dev: int, probe_sweeps: int, stream: int = 0):
    """Returns [(threads, groups_per_cu, ms), ...] of every shape timed."""
    times = np.zeros(3 * 64, dtype=np.float64)
    nt = ctypes.c_int32(0)
    _check(load_library().ising_batch_autotune(
        ctypes.byref(b), scratch_dev, int(probe_sweeps),
        times.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 64, ctypes.byref(nt), stream))
    t = times[:3 * nt.value].reshape(-1, 3)
    return [(int(a), int(g), float(ms)) for a, g, ms in t]


def ising_nn_param_count(channels: int = NN_CHANNELS) -> int:
    return int(load_library().ising_nn_param_count(channels))


def ising_nn_workspace_bytes(L: int, channels: int, max_batch: int) -> int:
    return int(load_library().ising_nn_workspace_bytes(L, channels, max_batch))


def ising_nn_round_weights(net: ising_nn, stream: int = 0):
    _check(load_library().ising_nn_round_weights(ctypes.byref(net), stream))


def ising_nn_logq(net: ising_nn, s_dev: int, stride: int, batch: int, logq_dev: int,
                  symmetric: int = 0, stream: int = 0):
    _check(load_library().ising_nn_logq(ctypes.byref(net), s_dev, stride, batch, symmetric,
                                        logq_dev, stream))


def ising_nn_grad(net: ising_nn, s_dev: int, stride: int, batch: int, loss_dev: int = 0,
                  stream: int = 0):
    _check(load_library().ising_nn_grad(ctypes.byref(net), s_dev, stride, batch, loss_dev or None,
                                        stream))


def ising_nn_adam(net: ising_nn, lr: float, b1: float, b2: float, eps: float, step: int,
                  stream: int = 0):
    _check(load_library().ising_nn_adam(ctypes.byref(net), lr, b1, b2, eps, step, stream))


def ising_nn_sample(net: ising_nn, batch: int, seed: int, chain0: int, draw: int, s_out: int,
                    stride: int, logq_out: int = 0, symmetric: int = 0, stream: int = 0):
    _check(load_library().ising_nn_sample(ctypes.byref(net), batch, seed, chain0, draw, symmetric,
                                          s_out, stride, logq_out or None, stream))


def ising_batch_mh(b: ising_batch, L_prop: int, prop_dev: int, prop_stride: int, logq_cur_dev: int,
                   logq_prop_dev: int, beta_dev: int, draw: int, accepted_dev: int = 0,
                   stream: int = 0):
    _check(load_library().ising_batch_mh(ctypes.byref(b), L_prop, prop_dev, prop_stride,
                                         logq_cur_dev, logq_prop_dev, beta_dev, draw,
                                         accepted_dev or None, stream))


def ising_ea_spins_bytes(L: int, replicas: int) -> int:
    return int(load_library().ising_ea_spins_bytes(L, replicas))


def ising_ea_workspace_bytes(L: int, replicas: int) -> int:
    return int(load_library().ising_ea_workspace_bytes(L, replicas))


def ising_ea_setup(ea: ising_ea, beta_host, stream: int = 0):
    b, bp = _f64(beta_host)
    if len(b) != ea.replicas:
        raise IsingError(E_INVALID, "one beta per replica")
    _check(load_library().ising_ea_setup(ctypes.byref(ea), bp, stream))


def ising_ea_init(ea: ising_ea, start: int, stream: int = 0):
    _check(load_library().ising_ea_init(ctypes.byref(ea), start, stream))


def ising_ea_sweep(ea: ising_ea, n: int, every: int, trace_dev: int = 0, stream: int = 0):
    _check(load_library().ising_ea_sweep(ctypes.byref(ea), int(n), int(every), trace_dev or None,
                                         stream))


def ising_ea_measure(ea: ising_ea, E_dev: int, stream: int = 0):
    _check(load_library().ising_ea_measure(ctypes.byref(ea), E_dev, stream))


def ising_ea_state(ea: ising_ea, stream: int = 0):
    """(t, perm [R], E [R], accepts [R-1]) read back from the device."""
    R = ea.replicas
    t = ctypes.c_uint64(0)
    perm = np.zeros(R, np.int32)
    E = np.zeros(R, np.int64)
    acc = np.zeros(max(R - 1, 1), np.uint64)
    _check(load_library().ising_ea_state(
        ctypes.byref(ea), ctypes.byref(t), perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        E.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        acc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), stream))
    return int(t.value), perm, E, acc[:max(R - 1, 0)]


def ising_ea_rng_blocks(ea: ising_ea, stream: int = 0) -> int:
    v = ctypes.c_uint64(0)
    _check(load_library().ising_ea_rng_blocks(ctypes.byref(ea), ctypes.byref(v), stream))
    return int(v.value)


def ising_ea_check_device_error(ea: ising_ea, stream: int = 0):
    _check(load_library().ising_ea_check_device_error(ctypes.byref(ea), stream))


def ising_xy_workspace_bytes(L: int, count: int) -> int:
    return int(load_library().ising_xy_workspace_bytes(L, count))


def ising_xy_init(xy: ising_xy, start: int, stream: int = 0):
    _check(load_library().ising_xy_init(ctypes.byref(xy), start, stream))


def ising_xy_sweep(xy: ising_xy, beta: float, n: int, E_trace_dev: int = 0, stream: int = 0):
    _check(load_library().ising_xy_sweep(ctypes.byref(xy), float(beta), int(n),
                                         E_trace_dev or None, stream))


def ising_xy_energy(xy: ising_xy, E_dev: int, stream: int = 0):
    _check(load_library().ising_xy_energy(ctypes.byref(xy), E_dev, stream))


def ising_xy_state(xy: ising_xy, stream: int = 0):
    t = ctypes.c_uint64(0)
    acc = np.zeros(xy.count, np.uint64)
    _check(load_library().ising_xy_state(ctypes.byref(xy), ctypes.byref(t),
                                         acc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                         stream))
    return int(t.value), acc


def ising_xy_check_device_error(xy: ising_xy, stream: int = 0):
    _check(load_library().ising_xy_check_device_error(ctypes.byref(xy), stream))


# ------------------------------------------------------------ torch-backed lattice
def _aligned_buffer(nbytes: int, device):
    """A uint8 device tensor whose data pointer is 256-byte aligned."""
    import torch

    raw = torch.zeros(max(nbytes, 1) + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw, raw[off:off + max(nbytes, 1)]


class Lattice:
    """One lattice whose spin and workspace memory are torch tensors."""

    def __init__(self, L: int, layout: str = "int8", seed: int = 1, lattice_id: int = 0,
                 start: str = "cold", device=None, init: bool = True, flags: int = 0):
        import torch

        self.device = torch.device(device or "cuda")
        lay = {"int8": LAYOUT_INT8, "bit1": LAYOUT_BIT1}[layout]
        nb = ising_spins_bytes(2, L, lay)
        if nb == 0:
            raise IsingError(E_INVALID, f"L={L} is invalid for layout {layout}")
        nw = ising_workspace_bytes(2, L, lay)
        self._spins_raw, self.spins = _aligned_buffer(nb, self.device)
        self._ws_raw, self.workspace = _aligned_buffer(nw, self.device)
        self.c = ising_lattice(ABI_VERSION, 2, L, lay, seed, lattice_id, flags, 0,
                               self.spins.data_ptr(), self.workspace.data_ptr())
        self.L = L
        self.layout = layout
        if init:
            self.init(start)

    @staticmethod
    def _stream() -> int:
        import torch

        return torch.cuda.current_stream().cuda_stream

    @property
    def sweep_index(self) -> int:
        return int(self.c.sweep_index)

    def init(self, start: str = "cold"):
        ising_init(self.c, {"cold": START_COLD_UP, "random": START_RANDOM}[start], self._stream())

    def sweep(self, beta: float, n: int, record: bool = True, tiles=None):
        """n sweeps; returns device int64 tensors (E, M) after each sweep.
        tiles = (rows, waves) runs the BIT1 tile kernel under that shape
        (ising_sweep_tiles) instead of the library's choice."""
        import torch

        E = M = None
        if record:
            E = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
            M = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        Ep, Mp = (E.data_ptr(), M.data_ptr()) if record else (0, 0)
        if tiles is None:
            ising_sweep(self.c, beta, n, Ep, Mp, self._stream())
        else:
            ising_sweep_tiles(self.c, beta, n, tiles[0], tiles[1], Ep, Mp, self._stream())
        return (E[:n], M[:n]) if record else (None, None)

    def set_sweep_index(self, t: int):
        """Resume a chain: the next sweep draws as sweep t (with
        from_int8, a checkpoint of spins and sweep index restores it)."""
        self.c.sweep_index = int(t)

    def measure(self):
        import torch

        out = torch.empty(2, dtype=torch.int64, device=self.device)
        ising_measure(self.c, out.data_ptr(), out.data_ptr() + 8, self._stream())
        return out

    def to_int8(self):
        import torch

        out = torch.empty((self.L, self.L), dtype=torch.int8, device=self.device)
        ising_to_int8(self.c, out.data_ptr(), self._stream())
        return out

    def from_int8(self, s):
        import torch

        s = s.to(device=self.device, dtype=torch.int8).contiguous()
        assert s.shape == (self.L, self.L)
        ising_from_int8(self.c, s.data_ptr(), self._stream())

    def check(self):
        ising_check_device_error(self.c, self._stream())

    def rng_blocks(self) -> int:
        return ising_rng_blocks(self.c, self._stream())


class Batch:
    """Many small INT8 lattices (sides L_list, temperatures betas) swept in
    one persistent launch; spins and workspace are torch tensors.  draws:
    "site" (per-site draws, any L % 8 == 0) or "plane" (bit-plane draws,
    L = 32 or a multiple of 64, 32 sites per lane)."""

    def __init__(self, L_list, betas, seed: int = 1, lattice_id0: int = 0, start: str = "random",
                 device=None, threads: int = 0, groups_per_cu: int = 0, init: bool = True,
                 draws: str = "site"):
        import torch

        self.device = torch.device(device or "cuda")
        self.L = np.ascontiguousarray(L_list, dtype=np.int32)
        self.count = len(self.L)
        nb, self.offsets = ising_batch_spins_bytes(self.L)
        if nb == 0 or self.count == 0:
            raise IsingError(E_INVALID, "every L must be a multiple of 8 in 8..256")
        nw = ising_batch_workspace_bytes(self.count)
        self._spins_raw, self.spins = _aligned_buffer(nb, self.device)
        self._ws_raw, self.workspace = _aligned_buffer(nw, self.device)
        self.draws = {"site": DRAWS_SITE, "plane": DRAWS_PLANE}[draws]
        self.c = ising_batch(ABI_VERSION, self.count, seed, lattice_id0, int(self.L.max()),
                             threads, groups_per_cu, self.draws, 0, nb, self.spins.data_ptr(),
                             self.workspace.data_ptr())
        self.set_beta(betas)
        if init:
            self.init(start)

    _stream = staticmethod(Lattice._stream)

    def set_beta(self, betas):
        self.beta = np.ascontiguousarray(betas, dtype=np.float64)
        ising_batch_setup(self.c, self.L, self.beta, self._stream())

    def init(self, start: str = "random"):
        ising_batch_init(self.c, {"cold": START_COLD_UP, "random": START_RANDOM}[start],
                         self._stream())

    def sweep(self, n: int, moments: bool = True, out=None, trace=None):
        """n sweeps of every lattice; returns the int64 [count, 8] moments
        (fields MOMENT_FIELDS) of this call, or None.  trace, if given, is
        an int64 tensor [n, count, 2] receiving E and M after every sweep."""
        import torch

        if moments and out is None:
            out = torch.empty((self.count, 8), dtype=torch.int64, device=self.device)
        if trace is not None:
            assert trace.dtype == torch.int64 and trace.is_contiguous() and trace.numel() >= 2 * n * self.count
        ising_batch_sweep(self.c, n, out.data_ptr() if moments else 0,
                          trace.data_ptr() if trace is not None else 0, self._stream())
        return out if moments else None

    def measure(self):
        import torch

        E = torch.empty(self.count, dtype=torch.int64, device=self.device)
        M = torch.empty(self.count, dtype=torch.int64, device=self.device)
        ising_batch_measure(self.c, E.data_ptr(), M.data_ptr(), self._stream())
        return E, M

    def lattice(self, j: int):
        """View of lattice j as an int8 [L, L] tensor."""
        import torch

        L, o = int(self.L[j]), int(self.offsets[j])
        return self.spins[o:o + L * L].view(torch.int8).view(L, L)

    def set_lattice(self, j: int, s):
        import torch

        self.lattice(j).copy_(s.to(device=self.device, dtype=torch.int8))

    @property
    def sweep_index(self) -> int:
        return ising_batch_sweep_index(self.c, self._stream())

    def rng_blocks(self) -> int:
        return ising_batch_rng_blocks(self.c, self._stream())

    def check(self):
        ising_batch_check_device_error(self.c, self._stream())

    def autotune(self, probe_sweeps: int = 20):
        import torch

        scratch_raw, scratch = _aligned_buffer(int(self.c.spins_bytes), self.device)
        times = ising_batch_autotune(self.c, scratch.data_ptr(), probe_sweeps, self._stream())
        del scratch_raw, scratch
        return times


class Net:
    """The learned proposal network on the current HIP device: float32
    master parameters, their bfloat16 copy, gradient and Adam moments, and
    the workspace, all torch tensors."""

    def __init__(self, L: int, max_batch: int, params=None, device=None):
        import torch

        self.device = torch.device(device or "cuda")
        self.L, self.max_batch = L, max_batch
        self.P = ising_nn_param_count()
        f32 = dict(dtype=torch.float32, device=self.device)
        self.master = torch.zeros(self.P, **f32)
        self.weights = torch.zeros(self.P, dtype=torch.int16, device=self.device)
        self.grad = torch.zeros(self.P, **f32)
        self.adam_m = torch.zeros(self.P, **f32)
        self.adam_v = torch.zeros(self.P, **f32)
        nw = ising_nn_workspace_bytes(L, NN_CHANNELS, max_batch)
        if nw == 0:
            raise IsingError(E_INVALID, f"L={L}, max_batch={max_batch} invalid")
        self._ws_raw, self.workspace = _aligned_buffer(nw, self.device)
        self.c = ising_nn(ABI_VERSION, L, NN_CHANNELS, max_batch, self.master.data_ptr(),
                          self.weights.data_ptr(), self.grad.data_ptr(), self.adam_m.data_ptr(),
                          self.adam_v.data_ptr(), self.workspace.data_ptr())
        self.step = 0
        if params is not None:
            self.set_params(params)

    _stream = staticmethod(Lattice._stream)

    def set_params(self, params):
        import torch

        self.master.copy_(torch.as_tensor(np.asarray(params, dtype=np.float32)))
        self.adam_m.zero_()
        self.adam_v.zero_()
        self.step = 0
        ising_nn_round_weights(self.c, self._stream())

    def bf16_params(self):
        """The bfloat16 parameters the kernels use, as float32 (host numpy)."""
        import torch

        w = self.weights.to(torch.int32).cpu().numpy().astype(np.uint32) & 0xFFFF
        return (w << 16).view(np.float32)

    @staticmethod
    def _cfg(s):
        """(pointer, stride in bytes, count) of a [B, L, L] int8 tensor, or
        of a Batch whose lattices all have side L."""
        if isinstance(s, Batch):
            if len(s.offsets) > 1:
                st = int(s.offsets[1] - s.offsets[0])
                assert all(int(s.offsets[j]) == j * st for j in range(len(s.offsets)))
            else:
                st = int(s.L[0]) ** 2
            return s.spins.data_ptr(), st, s.count
        assert s.dim() == 3 and s.stride(2) == 1 and s.stride(1) == s.shape[2]
        return s.data_ptr(), s.stride(0), s.shape[0]

    def logq(self, s, out=None, symmetric: bool = False):
        import torch

        ptr, st, B = self._cfg(s)
        if out is None:
            out = torch.empty(B, dtype=torch.float32, device=self.device)
        ising_nn_logq(self.c, ptr, st, B, out.data_ptr(), int(symmetric), self._stream())
        return out

    def loss_and_grad(self, s, loss=None):
        """Mean NLL of the batch (device tensor [1]); the gradient goes to self.grad."""
        import torch

        ptr, st, B = self._cfg(s)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        ising_nn_grad(self.c, ptr, st, B, loss.data_ptr(), self._stream())
        return loss

    def adam(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        ising_nn_adam(self.c, lr, b1, b2, eps, self.step, self._stream())

    def sample(self, batch: int, seed: int, chain0: int = 0, draw: int = 0, out=None, logq=None,
               symmetric: bool = False):
        """Draw `batch` configurations; returns (int8 [batch, L, L], float32 [batch]):
        the configurations written and their log q (log q_sym with symmetric),
        bitwise equal to logq() of the same configurations."""
        import torch

        if out is None:
            out = torch.empty((batch, self.L, self.L), dtype=torch.int8, device=self.device)
        if logq is None:
            logq = torch.empty(batch, dtype=torch.float32, device=self.device)
        ising_nn_sample(self.c, batch, seed, chain0, draw, out.data_ptr(), out.stride(0),
                        logq.data_ptr(), int(symmetric), self._stream())
        return out, logq


class SpinGlass:
    """R replicas of the 3D +-J glass (couplings `bonds`, int8 [3, L, L, L])
    on a beta ladder, with replica exchange; torch-backed buffers.  draws:
    "site" (per-site draws) or "plane" (bit-plane draws, L >= 64, 32 sites
    per lane)."""

    def __init__(self, bonds, betas, seed: int = 3, start: str = "random", device=None,
                 init: bool = True, draws: str = "site"):
        import torch

        self.device = torch.device(device or "cuda")
        bonds = np.ascontiguousarray(bonds, np.int8)
        self.L = int(bonds.shape[1])
        self.R = len(betas)
        nb = ising_ea_spins_bytes(self.L, self.R)
        nw = ising_ea_workspace_bytes(self.L, self.R)
        if nb == 0:
            raise IsingError(E_INVALID, f"L={self.L}, R={self.R} invalid")
        self._spins_raw, self.spins = _aligned_buffer(nb, self.device)
        self._bonds_raw, self.bonds = _aligned_buffer(bonds.nbytes, self.device)
        self.bonds.copy_(torch.from_numpy(bonds.reshape(-1).view(np.uint8)))
        self._ws_raw, self.workspace = _aligned_buffer(nw, self.device)
        self.draws = {"site": DRAWS_SITE, "plane": DRAWS_PLANE}[draws]
        self.c = ising_ea(ABI_VERSION, self.L, self.R, self.draws, seed, self.spins.data_ptr(),
                          self.bonds.data_ptr(), self.workspace.data_ptr())
        self.beta = np.ascontiguousarray(betas, np.float64)
        ising_ea_setup(self.c, self.beta, self._stream())
        if init:
            self.init(start)

    _stream = staticmethod(Lattice._stream)

    def init(self, start: str = "random"):
        ising_ea_init(self.c, {"cold": START_COLD_UP, "random": START_RANDOM}[start], self._stream())

    def sweep(self, n: int, every: int = 10, trace=None):
        """n sweeps; trace (int64 [n, R], optional) receives every replica's energy after each sweep."""
        if trace is not None:
            assert trace.is_contiguous() and trace.numel() >= n * self.R
        ising_ea_sweep(self.c, n, every, trace.data_ptr() if trace is not None else 0,
                       self._stream())

    def replica(self, r: int):
        import torch

        N = self.L ** 3
        return self.spins[r * N:(r + 1) * N].view(torch.int8).view(self.L, self.L, self.L)

    def measure(self):
        import torch

        E = torch.empty(self.R, dtype=torch.int64, device=self.device)
        ising_ea_measure(self.c, E.data_ptr(), self._stream())
        return E

    def state(self):
        return ising_ea_state(self.c, self._stream())

    def check(self):
        ising_ea_check_device_error(self.c, self._stream())

    def rng_blocks(self) -> int:
        return ising_ea_rng_blocks(self.c, self._stream())


class XYLattices:
    """`count` independent L x L XY lattices (double angles) on the GPU."""

    def __init__(self, L: int, count: int = 1, seed: int = 1, lattice_id0: int = 0,
                 start: str = "random", device=None, init: bool = True):
        import torch

        self.device = torch.device(device or "cuda")
        self.L, self.count = L, count
        nw = ising_xy_workspace_bytes(L, count)
        if nw == 0 or L < 2 or L % 2 or L > 128:
            raise IsingError(E_INVALID, f"L={L}, count={count} invalid")
        self._th_raw, th = _aligned_buffer(count * L * L * 8, self.device)
        self.theta = th.view(torch.float64).view(count, L, L)
        self._ws_raw, self.workspace = _aligned_buffer(nw, self.device)
        self.c = ising_xy(ABI_VERSION, L, count, lattice_id0, seed, self.theta.data_ptr(),
                          self.workspace.data_ptr())
        if init:
            self.init(start)

    _stream = staticmethod(Lattice._stream)

    def init(self, start: str = "random"):
        ising_xy_init(self.c, {"cold": START_COLD_UP, "random": START_RANDOM}[start], self._stream())

    def sweep(self, beta: float, n: int, trace: bool = True):
        """n sweeps; returns H after each sweep, double [n, count] (or None)."""
        import torch

        E = torch.empty((max(n, 1), self.count), dtype=torch.float64, device=self.device) \
            if trace else None
        ising_xy_sweep(self.c, beta, n, E.data_ptr() if trace else 0, self._stream())
        return E[:n] if trace else None

    def energy(self):
        import torch

        E = torch.empty(self.count, dtype=torch.float64, device=self.device)
        ising_xy_energy(self.c, E.data_ptr(), self._stream())
        return E

    def state(self):
        return ising_xy_state(self.c, self._stream())

    def check(self):
        ising_xy_check_device_error(self.c, self._stream())
