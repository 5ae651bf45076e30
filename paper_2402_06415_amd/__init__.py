"""MI355X checkerboard Metropolis sweep of the 2D Ising model.

The compute path is libising.so (HIP kernels for gfx950) behind the C ABI of
include/ising.h; ``binding`` exposes the same calls from Python and a
torch-backed ``Lattice`` convenience class.
"""
from .binding import (  # noqa: F401
    ABI_VERSION, FLAG_GLOBAL_HALFSWEEP, LAYOUT_BIT1, LAYOUT_INT8, START_COLD_UP, START_RANDOM, IsingError, Lattice,
    ising_abi_version, ising_check_device_error, ising_from_int8, ising_init, ising_lattice,
    ising_last_error, ising_measure, ising_rng_blocks, ising_spins_bytes, ising_sweep, ising_thresholds,
    ising_to_int8, ising_workspace_bytes, load_library,
)
