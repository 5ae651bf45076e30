/*
 * ising_ea.h - 3D Edwards-Anderson +-J spin glass with replica exchange
 * (C ABI of libising.so; same conventions, status codes and error
 * reporting as ising.h).
 *
 * R replicas of an L x L x L periodic simple cubic lattice share one set
 * of couplings J in {+1, -1}:
 *     H = - sum_n sum_{d = x,y,z} J_d(n) s_n s_{n + e_d}
 * Each replica runs the checkerboard Metropolis sweep of ising.h (the
 * paper's single-spin-flip trial, Fig. 2c, on the two sublattices in turn,
 * Fig. 2a-b) at the inverse temperature of its current place on a ladder
 * beta_0 < beta_1 < ... < beta_{R-1}; replica exchange swaps the places of
 * replicas at adjacent temperatures with probability
 *     min(1, exp((beta_k - beta_{k+1}) (E_k - E_{k+1}))).
 *
 * Conventions:
 *   site n = (z L + y) L + x, colour (x + y + z) & 1, colour 0 first;
 *   bonds: int8 [3][L^3], bonds[d L^3 + n] = J_d(n) couples n and n + e_d
 *   (d = 0: x, 1: y, 2: z); spins: int8 +1/-1, replica r at r L^3 bytes.
 *   u = s_n h_n with h_n the coupling-weighted sum of the six neighbours,
 *   dE = 2u in {-12..12}; u <= 0 flips without a draw; otherwise the draw
 *   is r = out[q & 3] of Philox4x32-10 counter (q >> 2, r_id, 2t + c, 0),
 *   q = n >> 1, r_id the replica's index, key (seed lo, seed hi); accepted
 *   iff r < ceil(2^32 exp(-beta dE)) (thresholds on the host in double).
 *   Random start: s = -1 iff the top bit of out[n & 3] of counter
 *   (n >> 2, r_id, 0, 2) is set.
 *   Plane draws (draws = ISING_DRAWS_PLANE, L >= 64): the colour-c sites
 *   with q >> 5 == g (one row) share the Philox blocks
 *   (g, r_id, 2t + c, 1 | b << 8), b = 0..7, and the r of lane l = q & 31
 *   has bit 31 - k equal to bit l of out[k & 3] of block k >> 2 (as the
 *   BIT1 lattices of ising.h).  The spins stay INT8 in `spins`; a sweep
 *   call packs them and the couplings into colour bit planes in the
 *   workspace, updates 32 sites per lane, and unpacks the spins at its end.
 *   Exchange after sweep t when (t + 1) % every == 0, as exchange number
 *   m = (t + 1) / every - 1, over the pairs (k, k+1) with k = m & 1,
 *   (m & 1) + 2, ...; with D = E(replica at k) - E(replica at k+1): swapped
 *   without a draw when D <= 0, else iff r < ceil(2^32 exp(-(beta_{k+1} -
 *   beta_k) D)) with r = out[0] of counter (k, m, 0, 5).  The swap
 *   thresholds are tabulated on the host in double for every D the lattice
 *   allows (D is a multiple of 4).
 */
#ifndef ISING_EA_H
#define ISING_EA_H

#include "ising.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ISING_EA_MAX_L 512
#define ISING_EA_MAX_REPLICAS 1024
#define ISING_EA_SWAP_TABLE 4096 /* swap thresholds tabulated per pair */

typedef struct ising_ea {
    int32_t abi_version;  /* must equal ISING_ABI_VERSION                     */
    int32_t L;            /* a power of two, 8..ISING_EA_MAX_L                  */
    int32_t replicas;     /* R, 1..ISING_EA_MAX_REPLICAS                        */
    int32_t draws;        /* ISING_DRAWS_SITE, or ISING_DRAWS_PLANE (L >= 64)   */
    uint64_t seed;        /* Philox key of starts, sweeps and exchanges        */
    int8_t *spins;        /* device, 256-B aligned, >= ising_ea_spins_bytes     */
    const int8_t *bonds;  /* device, 256-B aligned, int8 [3][L^3] of +1/-1      */
    void *workspace;      /* device, 256-B aligned, >= ising_ea_workspace_bytes */
} ising_ea;

ISING_API size_t ising_ea_spins_bytes(int32_t L, int32_t replicas);
/* Workspace: sweep index, ladder order, energies, thresholds, swap
 * tables, per-block energy changes, error word, and the bit planes of the
 * plane-draw mode (R L^3/8 + 3 L^3/8 bytes).  0 if invalid. */
ISING_API size_t ising_ea_workspace_bytes(int32_t L, int32_t replicas);

/* Tabulate the Metropolis thresholds of every beta and the swap thresholds
 * of every adjacent pair from beta_host[0..R-1] (strictly increasing,
 * finite, >= 0) and write them to the workspace; synchronises the stream.
 * Does not change spins, energies, order or sweep index.
 * Errors: invalid description or ladder -> ISING_E_INVALID; a pair so
 * close in beta that its swap table would exceed ISING_EA_SWAP_TABLE
 * entries -> ISING_E_UNSUPPORTED. */
ISING_API int ising_ea_setup(const ising_ea *ea, const double *beta_host, void *hip_stream);

/* Random (ISING_START_RANDOM) or all-up start of every replica; sweep
 * index 0; replica k at temperature k; energies recounted; swap counters
 * cleared.  Requires ising_ea_setup on this workspace. */
ISING_API int ising_ea_init(const ising_ea *ea, int32_t start, void *hip_stream);

/* n sweeps of all replicas from the device sweep index, with an exchange
 * step after every `every`-th sweep (every >= 1; 0 = no exchanges).  When
 * trace_dev is non-NULL it is device int64[n][R] receiving the energy of
 * every replica after every sweep.  Only kernel launches (the sweep index
 * lives on the device): the call may be captured in a HIP graph and each
 * replay continues the run.  Errors (host): invalid description, n < 0,
 * every < 0 -> ISING_E_INVALID; (device, via
 * ising_ea_check_device_error): not set up, t + n > 2^31. */
ISING_API int ising_ea_sweep(const ising_ea *ea, int64_t n, int32_t every, int64_t *trace_dev,
                             void *hip_stream);

/* Recount the energy of every replica into E_dev (device int64[R]). */
ISING_API int ising_ea_measure(const ising_ea *ea, int64_t *E_dev, void *hip_stream);

/* Read back (synchronising the stream) the sweep index, the replica at
 * each temperature (perm_host int32[R]), the running energies
 * (E_host int64[R]) and the accepted swaps of each pair
 * (accepts_host uint64[R-1]); any output may be NULL. */
ISING_API int ising_ea_state(const ising_ea *ea, uint64_t *t_host, int32_t *perm_host,
                             int64_t *E_host, uint64_t *accepts_host, void *hip_stream);

/* Read back (synchronising the stream) the Philox blocks the sweeps have
 * drawn since ising_ea_init (four sites share a block; blocks whose four
 * sites all flip without a draw are skipped).  Diagnostic only. */
ISING_API int ising_ea_rng_blocks(const ising_ea *ea, uint64_t *blocks_host, void *hip_stream);

/* Read back and clear the device error word (see ising_check_device_error). */
ISING_API int ising_ea_check_device_error(const ising_ea *ea, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ISING_EA_H */
