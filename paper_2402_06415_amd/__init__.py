"""MI355X checkerboard Metropolis sweep of the 2D Ising model.

The compute path is libising.so (HIP kernels for gfx950) behind the C ABI of
include/ising.h; ``binding`` exposes the same calls from Python and a
torch-backed ``Lattice`` convenience class.
"""
from .binding import (  # noqa: F401
    BATCH_MAX_COUNT, BATCH_MAX_L, MOMENT_FIELDS, Batch, ising_batch, ising_batch_autotune,
    ising_batch_check_device_error, ising_batch_init, ising_batch_measure, ising_batch_rng_blocks,
    ising_batch_setup, ising_batch_spins_bytes, ising_batch_sweep, ising_batch_sweep_index,
    ising_batch_workspace_bytes, NN_CHANNELS, NN_MAX_L, Net, ising_nn, ising_nn_param_count,
    ising_nn_workspace_bytes, ising_nn_round_weights, ising_nn_logq, ising_nn_grad, ising_nn_adam,
    ising_nn_sample, ising_batch_mh, SpinGlass, ising_ea, ising_ea_spins_bytes,
    ising_ea_workspace_bytes, ising_ea_setup, ising_ea_init, ising_ea_sweep, ising_ea_measure,
    ising_ea_state, ising_ea_check_device_error, ising_ea_rng_blocks, XYLattices, ising_xy,
    ising_xy_workspace_bytes, ising_xy_init, ising_xy_sweep, ising_xy_energy, ising_xy_state,
    ising_xy_check_device_error,
    ABI_VERSION, FLAG_COUNT_DRAWS, FLAG_GLOBAL_HALFSWEEP, LAYOUT_BIT1, LAYOUT_INT8, START_COLD_UP, START_RANDOM, IsingError, Lattice,
    ising_abi_version, ising_check_device_error, ising_from_int8, ising_init, ising_lattice,
    ising_last_error, ising_measure, ising_rng_blocks, ising_spins_bytes, ising_sweep,
    ising_sweep_tiles, ising_sweep_noalloc, ising_thresholds,
    ising_to_int8, ising_workspace_bytes, load_library,
)
