/*
 * ising_xy.h - Metropolis Monte Carlo of the 2D classical XY model (C ABI
 * of libising.so; same conventions, status codes and error reporting as
 * ising.h).  This is the paper's own Monte Carlo workload: Eq. (1),
 *     H = - sum_<x,delta> cos(theta_x - theta_{x+delta}),
 * on a periodic L x L square lattice, angles in double precision, with the
 * two sublattices updated alternately (Fig. 2a-b) and each single-spin
 * trial in the three steps of the Supplementary section "Detail of the MC
 * calculation for the XY model": a new angle theta' uniform in [0, 2 pi)
 * and p uniform in [0, 1); P = exp(-beta dE) with
 *     dE = - sum_delta [cos(theta' - theta_delta) - cos(theta - theta_delta)]
 * (Eq. S1 with its garbled sign read as new minus old); theta <- theta'
 * iff p < P.
 *
 * Several independent lattices (for example the paper's ten seeds) are
 * swept together: up to L = 80 one workgroup per lattice with the angles in
 * LDS for all n sweeps of a call; above that one launch per half-sweep
 * spread over many workgroups per lattice, the angles in global memory and
 * their cosines and sines in the workspace (2n + 1 launches per call, so a
 * caller of many short calls may capture them in a HIP graph).  Lattice j draws with lattice id lattice_id0 + j:
 * the trial of the site with compact index q = n >> 1 in half-sweep 2t + c
 * uses out of Philox4x32-10 counter (q, id, 2t + c, 8), key (seed lo,
 * seed hi):
 *     theta' = ((out[0] << 32 | out[1]) >> 11) 2^-53 * 2 pi,
 *     p      = ((out[2] << 32 | out[3]) >> 11) 2^-53,
 * the neighbours summed in the order right, left, down, up, every
 * floating-point operation rounded separately (no fused multiply-add).
 * The sweep keeps cos and sin of every angle (recomputed from the angles
 * at the start of each call) and forms the sum by the angle-difference
 * identity (sum_delta cos(theta' - theta_delta) = cos theta' sum cos
 * theta_delta + sin theta' sum sin theta_delta), with one sincos per trial;
 * it equals the direct sum up to rounding, so a decision can differ from the
 * direct sum's only when p lies within a few units in the last place of P.
 * Random start: theta_n from out[0], out[1] of counter (n, id, 0, 9).
 * The sweep index t lives in device memory and advances on the device.
 */
#ifndef ISING_XY_H
#define ISING_XY_H

#include "ising.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ISING_XY_MAX_L 128 /* largest side (the paper's largest lattice) */
#define ISING_XY_MAX_COUNT 4096

typedef struct ising_xy {
    int32_t abi_version;  /* must equal ISING_ABI_VERSION                    */
    int32_t L;            /* even, 2..ISING_XY_MAX_L                          */
    int32_t count;        /* lattices, 1..ISING_XY_MAX_COUNT                  */
    uint32_t lattice_id0; /* lattice j draws with id lattice_id0 + j          */
    uint64_t seed;        /* Philox key                                       */
    double *theta;        /* device, 256-B aligned: double [count][L][L]      */
    void *workspace;      /* device, 256-B aligned, >= ising_xy_workspace_bytes */
} ising_xy;

/* Workspace of count lattices of side L: sweep index, accepted-rotation
 * counters, error word, the per-lattice energy sums of the large-lattice
 * sweep and, for L > 80, the cosine and sine of every angle (16 B per site)
 * and the hand-off slots of the band-tiled sweep (64 L bytes per band, for
 * at most min(count L / 2, 2048) bands).
 * 0 for L or count out of range.  The library cannot check the size it is
 * given: a smaller workspace is undefined behaviour. */
ISING_API size_t ising_xy_workspace_bytes(int32_t L, int32_t count);

/* Random (ISING_START_RANDOM) or aligned (theta = 0, ISING_START_COLD_UP)
 * start of every lattice; sweep index 0; counters cleared. */
ISING_API int ising_xy_init(const ising_xy *xy, int32_t start, void *hip_stream);

/* n sweeps of every lattice at inverse temperature beta from the device
 * sweep index; E_trace_dev (device double[n][count], may be NULL)
 * receives H of every lattice after every sweep: H summed over the
 * lattice at the start of the call, plus the energy changes of the trials
 * accepted since (equal to a recount up to rounding).  Fewer lattices
 * than compute units with L > 32, or L > 80, run as bands of rows resident
 * for the whole call (one launch), handing edge rows to each other; many
 * lattices of L > 80 run one launch per half-sweep.  The chain is the same
 * in every form.  Errors: invalid description, beta negative or not
 * finite, n < 0 -> ISING_E_INVALID; device: workspace not initialised,
 * t + n > 2^31, or a band waited too long for a neighbour (see
 * ising_xy_check_device_error). */
ISING_API int ising_xy_sweep(const ising_xy *xy, double beta, int64_t n, double *E_trace_dev,
                             void *hip_stream);

/* H of every lattice into E_dev (device double[count]). */
ISING_API int ising_xy_energy(const ising_xy *xy, double *E_dev, void *hip_stream);

/* Read back (synchronising) the sweep index and the accepted rotations of
 * every lattice since init (accepted_host uint64[count]; either may be NULL). */
ISING_API int ising_xy_state(const ising_xy *xy, uint64_t *t_host, uint64_t *accepted_host,
                             void *hip_stream);

/* Read back and clear the device error word. */
ISING_API int ising_xy_check_device_error(const ising_xy *xy, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ISING_XY_H */
