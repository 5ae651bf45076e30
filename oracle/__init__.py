"""CPU oracle for the checkerboard Metropolis sweep (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does.

The arithmetic lives in ``ising_oracle.c`` (plain scalar C, optional OpenMP
over rows of one colour, which is bit-identical because sites of one colour
never neighbour each other).  This module only compiles it with gcc and
marshals numpy buffers through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ising_oracle.c")
_SRC_EA = os.path.join(_HERE, "ea_oracle.c")
_SRC_XY = os.path.join(_HERE, "xy_oracle.c")
_LIB = os.path.join(_HERE, "libising_oracle.so")

MODE_SITE = 0
MODE_PLANE = 1
START_COLD_UP = 0
START_RANDOM = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               "-o", tmp, _SRC, _SRC_EA, _SRC_XY, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(f) for f in (_SRC, _SRC_EA, _SRC_XY)):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i8p = ctypes.POINTER(ctypes.c_int8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_thresholds.argtypes = [ctypes.c_double, u32p, u8p]
    lib.oracle_thresholds.restype = ctypes.c_int
    lib.oracle_accept.argtypes = [ctypes.c_int, ctypes.c_uint32, u32p, u8p]
    lib.oracle_accept.restype = ctypes.c_int
    lib.oracle_local_u.argtypes = [i8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_local_u.restype = ctypes.c_int
    lib.oracle_init.argtypes = [i8p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                ctypes.c_uint32]
    lib.oracle_init.restype = ctypes.c_int
    lib.oracle_fill_uniforms.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                         u32p, ctypes.c_int]
    lib.oracle_fill_uniforms.restype = ctypes.c_int
    lib.oracle_halfsweep.argtypes = [i8p, ctypes.c_int, ctypes.c_int, u32p, u32p, u8p,
                                     i64p, i64p, ctypes.c_int]
    lib.oracle_halfsweep.restype = ctypes.c_int
    lib.oracle_measure.argtypes = [i8p, ctypes.c_int, i64p, i64p]
    lib.oracle_measure.restype = None
    lib.oracle_sweep.argtypes = [i8p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64,
                                 ctypes.c_double, i64p, i64p, ctypes.c_int]
    lib.oracle_sweep.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    f64p = ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_ea_energy.argtypes = [i8p, i8p, ctypes.c_int]
    lib.oracle_ea_energy.restype = ctypes.c_int64
    lib.oracle_ea_local_u.argtypes = [i8p, i8p, ctypes.c_int, ctypes.c_int64]
    lib.oracle_ea_local_u.restype = ctypes.c_int
    lib.oracle_ea_thresholds.argtypes = [ctypes.c_double, u32p, u8p]
    lib.oracle_ea_thresholds.restype = ctypes.c_int
    lib.oracle_ea_swap_threshold.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                             u32p, u8p]
    lib.oracle_ea_swap_threshold.restype = None
    lib.oracle_ea_init.argtypes = [i8p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                   ctypes.c_uint32]
    lib.oracle_ea_init.restype = None
    lib.oracle_ea_halfsweep.argtypes = [i8p, i8p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, i64p,
                                        ctypes.c_int, ctypes.c_int]
    lib.oracle_ea_fill_plane.argtypes = [u32p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_ea_fill_plane.restype = None
    lib.oracle_ea_halfsweep.restype = ctypes.c_int
    lib.oracle_ea_exchange.argtypes = [i64p, i32p, ctypes.c_int, f64p, ctypes.c_uint64,
                                       ctypes.c_uint64, u64p]
    lib.oracle_ea_exchange.restype = None
    lib.oracle_ea_run.argtypes = [i8p, i8p, ctypes.c_int, ctypes.c_int, f64p, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, i32p, i64p, u64p,
                                  i64p, ctypes.c_int, ctypes.c_int]
    lib.oracle_ea_run.restype = ctypes.c_int
    lib.oracle_xy_init.argtypes = [f64p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                   ctypes.c_uint32]
    lib.oracle_xy_init.restype = None
    lib.oracle_xy_energy.argtypes = [f64p, ctypes.c_int]
    lib.oracle_xy_energy.restype = ctypes.c_double
    lib.oracle_xy_halfsweep.argtypes = [f64p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double]
    lib.oracle_xy_halfsweep.restype = ctypes.c_int64
    lib.oracle_xy_sweep.argtypes = [f64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, f64p, i64p]
    lib.oracle_xy_sweep.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one 128-bit counter under a 64-bit key (two words)."""
    lib = _load()
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                             _ptr(out, ctypes.c_uint32))
    return out


def thresholds(beta: float):
    """(T[5], always[5]) for u = -4,-2,0,2,4; raises on invalid beta."""
    lib = _load()
    T = np.zeros(5, dtype=np.uint32)
    a = np.zeros(5, dtype=np.uint8)
    if lib.oracle_thresholds(float(beta), _ptr(T, ctypes.c_uint32),
                             _ptr(a, ctypes.c_uint8)):
        raise ValueError(f"invalid beta {beta!r}")
    return T, a


def accept(u: int, r: int, T: np.ndarray, always: np.ndarray) -> bool:
    lib = _load()
    return bool(lib.oracle_accept(int(u), int(r), _ptr(T, ctypes.c_uint32),
                                  _ptr(always, ctypes.c_uint8)))


def local_u(s: np.ndarray, x: int, y: int) -> int:
    lib = _load()
    L = s.shape[0]
    return int(lib.oracle_local_u(_ptr(s, ctypes.c_int8), L, x, y))


def init(L: int, start: int, seed: int, lattice_id: int = 0) -> np.ndarray:
    lib = _load()
    s = np.zeros((L, L), dtype=np.int8)
    if lib.oracle_init(_ptr(s, ctypes.c_int8), L, start, seed, lattice_id):
        raise ValueError("oracle_init rejected its arguments")
    return s


def fill_uniforms(L: int, mode: int, seed: int, lattice_id: int, t: int, c: int,
                  nthreads: int = 1) -> np.ndarray:
    """Draws r[y, x] for the sites of colour c in half-sweep 2t+c (others 0)."""
    lib = _load()
    r = np.zeros((L, L), dtype=np.uint32)
    if lib.oracle_fill_uniforms(L, mode, seed, lattice_id, t, c,
                                _ptr(r, ctypes.c_uint32), nthreads):
        raise ValueError("oracle_fill_uniforms rejected its arguments")
    return r


def halfsweep(s: np.ndarray, c: int, r: np.ndarray, T: np.ndarray, always: np.ndarray,
              nthreads: int = 1):
    """In-place update of colour c with draws r; returns (dE, dM)."""
    lib = _load()
    L = s.shape[0]
    dE = ctypes.c_int64(0)
    dM = ctypes.c_int64(0)
    if lib.oracle_halfsweep(_ptr(s, ctypes.c_int8), L, c, _ptr(r, ctypes.c_uint32),
                            _ptr(T, ctypes.c_uint32), _ptr(always, ctypes.c_uint8),
                            ctypes.byref(dE), ctypes.byref(dM), nthreads):
        raise ValueError("oracle_halfsweep rejected its arguments")
    return dE.value, dM.value


def measure(s: np.ndarray):
    lib = _load()
    L = s.shape[0]
    E = ctypes.c_int64(0)
    M = ctypes.c_int64(0)
    lib.oracle_measure(_ptr(s, ctypes.c_int8), L, ctypes.byref(E), ctypes.byref(M))
    return E.value, M.value


def sweep(s: np.ndarray, mode: int, seed: int, lattice_id: int, t0: int, n: int,
          beta: float, record: bool = True, nthreads: int = 1):
    """n sweeps in place from sweep index t0; returns (E_trace, M_trace)."""
    lib = _load()
    L = s.shape[0]
    E = np.zeros(max(n, 0), dtype=np.int64)
    M = np.zeros(max(n, 0), dtype=np.int64)
    Ep = _ptr(E, ctypes.c_int64) if record else None
    Mp = _ptr(M, ctypes.c_int64) if record else None
    if lib.oracle_sweep(_ptr(s, ctypes.c_int8), L, mode, seed, lattice_id, t0, n,
                        float(beta), Ep, Mp, nthreads):
        raise ValueError("oracle_sweep rejected its arguments")
    return (E, M) if record else (None, None)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def moments(E_trace, M_trace) -> dict:
    """Energy and magnetisation moments of a chain segment, as exact Python
    integers: sums over the states after each sweep of E, E^2, |M|, M^2 and
    M^4, plus the last E and M.  Divided by the number of sweeps (and powers
    of L^2) they estimate U = <H>/L^2 of the Supplementary Eq. S3, the
    specific heat and the Binder cumulant."""
    E = [int(v) for v in E_trace]
    M = [int(v) for v in M_trace]
    return {
        "E": E[-1], "M": M[-1],
        "sum_E": sum(E), "sum_E2": sum(e * e for e in E),
        "sum_absM": sum(abs(m) for m in M), "sum_M2": sum(m * m for m in M),
        "sum_M4": sum(m ** 4 for m in M),
    }


def batch_sweep(states, betas, seed: int, lattice_id0: int, t0: int, n: int, nthreads: int = 1,
                mode: int = MODE_SITE):
    """A batch is a set of independent lattices: lattice j runs its own
    chain (per-site or bit-plane draws, `mode`) with lattice id
    lattice_id0 + j at betas[j].  Sweeps every state in place from sweep
    index t0 and returns the moments of each lattice over these n sweeps."""
    out = []
    for j, s in enumerate(states):
        E, M = sweep(s, mode, seed, lattice_id0 + j, t0, n, betas[j], nthreads=nthreads)
        out.append(moments(E, M))
    return out


# ------------------------------------------------------------ 3D spin glass
def ea_energy(s: np.ndarray, J: np.ndarray) -> int:
    """H = -sum_n sum_d J_d(n) s_n s_{n+e_d} of s [L, L, L] (index [z, y, x])
    with couplings J [3, L, L, L] (d = 0: x, 1: y, 2: z)."""
    s, J = np.ascontiguousarray(s, np.int8), np.ascontiguousarray(J, np.int8)
    return int(_load().oracle_ea_energy(_ptr(s, ctypes.c_int8), _ptr(J, ctypes.c_int8), s.shape[0]))


def ea_local_u(s: np.ndarray, J: np.ndarray, n: int) -> int:
    s, J = np.ascontiguousarray(s, np.int8), np.ascontiguousarray(J, np.int8)
    return int(_load().oracle_ea_local_u(_ptr(s, ctypes.c_int8), _ptr(J, ctypes.c_int8),
                                         s.shape[0], n))


def ea_thresholds(beta: float):
    T = np.zeros(3, np.uint32)
    a = np.zeros(3, np.uint8)
    if _load().oracle_ea_thresholds(float(beta), _ptr(T, ctypes.c_uint32), _ptr(a, ctypes.c_uint8)):
        raise ValueError("invalid beta")
    return T, a


def ea_swap_threshold(beta_lo: float, beta_hi: float, D: int):
    T = np.zeros(1, np.uint32)
    a = np.zeros(1, np.uint8)
    _load().oracle_ea_swap_threshold(float(beta_lo), float(beta_hi), int(D),
                                     _ptr(T, ctypes.c_uint32), _ptr(a, ctypes.c_uint8))
    return int(T[0]), bool(a[0])


def ea_init(L: int, start: int, seed: int, replica_id: int) -> np.ndarray:
    s = np.zeros((L, L, L), np.int8)
    _load().oracle_ea_init(_ptr(s, ctypes.c_int8), L, start, seed, replica_id)
    return s


def ea_fill_plane(L: int, c: int, seed: int, replica_id: int, t: int) -> np.ndarray:
    """Plane draws of half-sweep 2t + c: r [L, L, L] for the colour-c sites
    (zero elsewhere)."""
    r = np.zeros((L, L, L), np.uint32)
    _load().oracle_ea_fill_plane(_ptr(r, ctypes.c_uint32), L, c, seed, replica_id,
                                 (2 * t + c) & 0xFFFFFFFF)
    return r


def ea_halfsweep(s: np.ndarray, J: np.ndarray, c: int, seed: int, replica_id: int, t: int,
                 beta: float, nthreads: int = 1, mode: int = MODE_SITE) -> int:
    dE = ctypes.c_int64(0)
    J = np.ascontiguousarray(J, np.int8)
    if _load().oracle_ea_halfsweep(_ptr(s, ctypes.c_int8), _ptr(J, ctypes.c_int8), s.shape[0], c,
                                   seed, replica_id, t, float(beta), ctypes.byref(dE), nthreads,
                                   mode):
        raise ValueError("oracle_ea_halfsweep rejected its arguments")
    return dE.value


def ea_exchange(E: np.ndarray, perm: np.ndarray, beta, m: int, seed: int,
                accepts: np.ndarray = None):
    """Exchange number m on the ladder beta [R] (increasing): perm (int32
    [R], temperature -> replica) is updated in place from the energies E
    (int64 [R], per replica); accepts (uint64 [R-1]) counts the swaps."""
    R = len(perm)
    E = np.ascontiguousarray(E, np.int64)
    beta = np.ascontiguousarray(beta, np.float64)
    if accepts is None:
        accepts = np.zeros(max(R - 1, 1), np.uint64)
    _load().oracle_ea_exchange(_ptr(E, ctypes.c_int64), _ptr(perm, ctypes.c_int32), R,
                               _ptr(beta, ctypes.c_double), m, seed,
                               _ptr(accepts, ctypes.c_uint64))
    return accepts


def ea_run(spins: np.ndarray, J: np.ndarray, beta, seed: int, t0: int, n: int, every: int,
           perm: np.ndarray, E: np.ndarray, accepts: np.ndarray = None, trace: bool = True,
           nthreads: int = 1, mode: int = MODE_SITE):
    """n sweeps of the replicas spins [R, L, L, L] in place (replica id r),
    temperatures beta [R] increasing, exchange after every `every`-th
    sweep; perm (int32 [R], temperature -> replica), E (int64 [R], current
    energies) and accepts (uint64 [R-1]) are updated.  Returns the energy
    trace [n, R] (or None)."""
    R, L = spins.shape[0], spins.shape[1]
    beta = np.ascontiguousarray(beta, np.float64)
    J = np.ascontiguousarray(J, np.int8)
    if accepts is None:
        accepts = np.zeros(max(R - 1, 1), np.uint64)
    tr = np.zeros((max(n, 1), R), np.int64) if trace else None
    rc = _load().oracle_ea_run(_ptr(spins, ctypes.c_int8), _ptr(J, ctypes.c_int8), L, R,
                               _ptr(beta, ctypes.c_double), seed, t0, n, every,
                               _ptr(perm, ctypes.c_int32), _ptr(E, ctypes.c_int64),
                               _ptr(accepts, ctypes.c_uint64),
                               _ptr(tr, ctypes.c_int64) if trace else None, nthreads, mode)
    if rc:
        raise ValueError("oracle_ea_run rejected its arguments")
    return tr[:n] if trace else None


# ------------------------------------------------------------ 2D XY model
def xy_init(L: int, start: int, seed: int, lattice_id: int = 0) -> np.ndarray:
    th = np.zeros((L, L), np.float64)
    _load().oracle_xy_init(_ptr(th, ctypes.c_double), L, start, seed, lattice_id)
    return th


def xy_energy(theta: np.ndarray) -> float:
    theta = np.ascontiguousarray(theta, np.float64)
    return float(_load().oracle_xy_energy(_ptr(theta, ctypes.c_double), theta.shape[0]))


def xy_halfsweep(theta: np.ndarray, c: int, seed: int, lattice_id: int, t: int, beta: float) -> int:
    return int(_load().oracle_xy_halfsweep(_ptr(theta, ctypes.c_double), theta.shape[0], c, seed,
                                           lattice_id, t, float(beta)))


def xy_sweep(theta: np.ndarray, seed: int, lattice_id: int, t0: int, n: int, beta: float):
    """n sweeps in place; returns (energy after each sweep [n], accepted rotations)."""
    E = np.zeros(max(n, 1), np.float64)
    acc = ctypes.c_int64(0)
    if _load().oracle_xy_sweep(_ptr(theta, ctypes.c_double), theta.shape[0], seed, lattice_id, t0,
                               n, float(beta), _ptr(E, ctypes.c_double), ctypes.byref(acc)):
        raise ValueError("oracle_xy_sweep rejected its arguments")
    return E[:n], acc.value
