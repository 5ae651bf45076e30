/*
 * ising.h - C ABI of the MI355X checkerboard Metropolis library (libising.so).
 *
 * The library runs the Metropolis single-spin-flip Monte Carlo of the 2D
 * Ising model H = -sum_<ij> s_i s_j on an L x L periodic square lattice,
 * updating the two checkerboard sublattices alternately.  This is the hot
 * path of "Many-body computing on Field Programmable Gate Arrays"
 * (arXiv 2402.06415): the Hamiltonian is the paper's Eq. (1) restricted to
 * theta in {0, pi}; the bipartite, alternating update is the one of the
 * Results section "Parallel design of MC simulation for the XY model" and
 * Fig. 2a-b; each trial follows the three steps of Fig. 2c and of the
 * Supplementary section "Detail of the MC calculation for the XY model":
 * draw p uniform in [0,1), compute dE and P = exp(-beta dE), accept iff p < P.
 * The per-site LCG of the paper is replaced by the counter-based
 * Philox4x32-10 generator (Salmon et al., SC'11).
 *
 * Conventions (identical in every entry point):
 *   site n = y*L + x, colour(x,y) = (x+y) & 1; colour 0 is updated first in
 *   each sweep; a sweep is one update of colour 0 then one of colour 1.
 *   Spin s = +1 or -1.  INT8 layout: s[n] as int8, row-major, L*L bytes.
 *   BIT1 layout (L % 64 == 0): two colour planes, plane c at byte offset
 *   c*L*L/16, each L rows of L/64 uint32 words; bit b of word w in row y
 *   of plane c is the colour-c site of row y with compact column 32w+b
 *   (x = 2*(32w+b) + ((y+c)&1)); bit value 1 means s = -1.
 *   Draws: p = r / 2^32, accepted iff r < T = ceil(2^32 exp(-beta dE)),
 *   thresholds computed on the host in IEEE double; dE <= 0 always flips.
 *   The Philox key is (seed lo, seed hi); the counter of a draw is
 *     INT8 (per site):  (q >> 2, lattice_id, 2t + c, 0),  r = out[q & 3],
 *     BIT1 (bit planes): (q >> 5, lattice_id, 2t + c, 1 | b << 8), and bit
 *       (31 - k) of r is bit (q & 31) of out[k & 3] of block b = k >> 2,
 *   with q = n >> 1 the compact index of site n within its colour and t
 *   the sweep index.  Random start: s = -1 iff the top bit of out[n & 3]
 *   of counter (n >> 2, lattice_id, 0, 2) is set.
 *   E = -sum over right and down bonds of s_i s_j, M = sum s_i (int64).
 *
 * Memory and streams: every device pointer is caller-owned (the Python
 * binding allocates them as torch tensors); the library allocates nothing.
 * Every call enqueues its work on the given HIP stream (NULL = the null
 * stream) and returns without synchronising; results are valid once the
 * stream has reached that point.  A lattice handle must not be used from
 * two host threads at once, and two calls on the same spins must not
 * overlap on different streams.
 *
 * Errors: every int-returning call returns ISING_OK (0) or an error code.
 * ISING_E_INVALID and ISING_E_UNSUPPORTED leave the lattice and all device
 * memory untouched.  ISING_E_HIP reports a failed HIP call (launch or
 * configuration); device contents are then undefined.  ISING_E_STATE
 * reports a device-side failure detected after the fact (see
 * ising_check_device_error).  ising_last_error() returns a thread-local
 * message describing the last failure of the calling thread.
 */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISING_ABI_VERSION 3

#if defined(__GNUC__) || defined(__clang__)
#define ISING_API __attribute__((visibility("default")))
#else
#define ISING_API
#endif

enum ising_layout { ISING_LAYOUT_INT8 = 0, ISING_LAYOUT_BIT1 = 1 };
enum ising_start { ISING_START_COLD_UP = 0, ISING_START_RANDOM = 1 };

/* Kernel-choice flags.  Every choice computes the same chain bit for bit;
 * they exist so that each variant can be tested and timed. */
enum ising_flags {
    /* one launch per half-sweep reading the spins from global memory,
     * instead of the resident single-workgroup (INT8, L <= 64, or
     * L <= 128 when L % 8 != 0) or the persistent tile-resident kernels
     * (BIT1; INT8 with L % 8 == 0 up to L = 4096) */
    ISING_FLAG_GLOBAL_HALFSWEEP = 1u,
    /* BIT1: count the Philox blocks the sweeps draw (ising_rng_blocks), a
     * diagnostic that costs a few instructions per word; without it the
     * BIT1 kernels do not count.  The INT8 kernels always count. */
    ISING_FLAG_COUNT_DRAWS = 2u
};
enum ising_status {
    ISING_OK = 0,
    ISING_E_INVALID = 1,     /* bad argument; nothing was changed          */
    ISING_E_UNSUPPORTED = 2, /* valid request this build does not run      */
    ISING_E_HIP = 3,         /* a HIP runtime call failed                  */
    ISING_E_STATE = 4        /* device reported an inconsistent state      */
};

/* Plain-old-data description of one lattice.  The caller fills every field
 * before ising_init (or ising_from_int8) and keeps it alive; the library
 * only advances sweep_index. */
typedef struct ising_lattice {
    int32_t abi_version;  /* must equal ISING_ABI_VERSION                   */
    int32_t dim;          /* 2                                              */
    int32_t L;            /* even, 4 <= L <= 65536; BIT1: L % 64 == 0       */
    int32_t layout;       /* enum ising_layout                              */
    uint64_t seed;        /* Philox key                                     */
    uint32_t lattice_id;  /* second Philox counter word                     */
    uint32_t flags;       /* ISING_FLAG_* bits; 0 = automatic kernel choice  */
    uint64_t sweep_index; /* t of the next sweep; < 2^31                    */
    void *spins;          /* device, >= ising_spins_bytes(), 256-B aligned  */
    void *workspace;      /* device, >= ising_workspace_bytes(), 256-B aligned,
                             NULL allowed when that size is 0               */
} ising_lattice;

/* Bytes of spin storage for (dim, L, layout); 0 if the combination is
 * invalid.  INT8: L*L.  BIT1: L*L/8. */
ISING_API size_t ising_spins_bytes(int32_t dim, int32_t L, int32_t layout);

/* Bytes of device workspace the calls on such a lattice need (partial
 * sums, synchronisation flags, halo rows); 0 if invalid. */
ISING_API size_t ising_workspace_bytes(int32_t dim, int32_t L, int32_t layout);

/* ABI version of the loaded library (== ISING_ABI_VERSION when matched). */
ISING_API int32_t ising_abi_version(void);

/* Host-only: acceptance table for u = s_i h_i = -4,-2,0,2,4 (index
 * (u+4)/2): T[k] = ceil(2^32 exp(-2 beta u)) for u > 0, always[k] = 1 when
 * the flip needs no draw (u <= 0, or 2^32 P rounds up to 2^32).  Follows
 * step 2 and 3 of the trial (P(dE) = exp(-beta dE), accept iff p < P).
 * Errors: beta negative, NaN or infinite -> ISING_E_INVALID. */
ISING_API int ising_thresholds(double beta, uint32_t T[5], uint8_t always_flip[5]);

/* Fill the spins: ISING_START_COLD_UP (all +1) or ISING_START_RANDOM
 * (Philox draw per site, see above) and set sweep_index = 0; also clears
 * the workspace's accumulators, device error word and draw counters.
 * Paper: the start of a Monte Carlo trajectory, fixed by its random seed
 * (Supplementary, "Detail of the MC calculation for the XY model": each
 * simulation runs from its own initial random seed, giving its own
 * trajectory).  Asynchronous on hip_stream; spins and workspace stay
 * caller-owned.
 * Errors: invalid lattice description or start -> ISING_E_INVALID, nothing
 * enqueued. */
ISING_API int ising_init(ising_lattice *lat, int32_t start, void *hip_stream);

/* Run n >= 0 sweeps at inverse temperature beta from sweep index
 * lat->sweep_index, then advance it by n.  Paper: Results, "Parallel
 * design of MC simulation for the XY model", Fig. 2a-b (sublattices A and
 * B updated alternately, each in parallel since no two sites of one
 * sublattice are neighbours), every site trial following the three steps
 * of Fig. 2c (draw p, compute dE and P = exp(-beta dE), accept iff p < P)
 * with the thresholds of ising_thresholds.  One sweep is one MC step.
 * E_dev / M_dev, when non-NULL, are device int64[n] (caller-owned)
 * receiving E and M after each sweep of this call (not the state before
 * it: that is ising_measure's).  sweep(b, n1) followed by sweep(b, n2)
 * equals sweep(b, n1 + n2) bit for bit, because the draws are keyed by
 * the sweep index.  Asynchronous on hip_stream.  Errors: beta negative,
 * NaN or infinite; n < 0; sweep_index + n > 2^31; invalid lattice ->
 * ISING_E_INVALID, nothing enqueued and sweep_index unchanged;
 * ISING_E_HIP if a launch fails (spins then undefined). */
ISING_API int ising_sweep(ising_lattice *lat, double beta, int64_t n, int64_t *E_dev,
                int64_t *M_dev, void *hip_stream);

/* ising_sweep for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  It is ising_sweep (same kernels, same chain, same E_dev /
 * M_dev contents) except that the kernels' workspace is a static device
 * array of the library, 1 KiB + 4 MiB, one copy per GPU, held until the
 * process ends; lat->workspace is not used and may be NULL.  The call
 * allocates and frees nothing.  Limit: BIT1 lattices up to L = 8192
 * (the halo slots of 1024 tiles); INT8 lattices of any valid L (above
 * L = 1024 with one launch per half-sweep when the tile kernel's halo
 * slots do not fit the scratch; the chain is the same).
 * status_dev (device uint32, may be NULL) receives 0, or the device error
 * word of this call if an inter-tile wait timed out (spins then undefined).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or host threads) race and must not be made; the
 * call clears what must start at zero, so successive calls are
 * independent.  ising_rng_blocks does not count this call's draws.
 * Errors: as ising_sweep (the workspace is not checked); a BIT1 lattice
 * above L = 8192 -> ISING_E_UNSUPPORTED; status_dev misaligned ->
 * ISING_E_INVALID; nothing is enqueued in these cases. */
ISING_API int ising_sweep_noalloc(ising_lattice *lat, double beta, int64_t n, int64_t *E_dev,
                                  int64_t *M_dev, uint32_t *status_dev, void *hip_stream);

/* ising_sweep with the persistent tile kernel under a given tile shape
 * instead of the library's choice: the lattice is cut into L / rows tiles
 * of `rows` full-width rows, one workgroup of `waves` wavefronts each,
 * resident in LDS for the whole call (BIT1: colour bit planes, any
 * L % 64 == 0; INT8: bytes, L % 8 == 0 and L <= 4096).  The chain does not
 * depend on the shape (the same draws, the same decisions): this entry
 * point exists so that the shapes can be compared, timed and tested.
 * Paper: as ising_sweep; the tile is the GPU counterpart of the paper's
 * supercell (Supplementary, "Details and comparisons of parallelization
 * strategies applied to different lattice configurations").
 * Errors: an INT8 side not a multiple of 8 or above 4096, rows not dividing
 * L into 2..1024 tiles, waves outside 1..16 (BIT1: 1..min(16, rows)) ->
 * ISING_E_INVALID; a tile above the LDS a workgroup may use (BIT1: 64 KiB)
 * or more tiles than the device holds at once -> ISING_E_UNSUPPORTED; in
 * both cases nothing is enqueued.  Otherwise as ising_sweep. */
ISING_API int ising_sweep_tiles(ising_lattice *lat, double beta, int64_t n, int32_t rows,
                                int32_t waves, int64_t *E_dev, int64_t *M_dev, void *hip_stream);

/* Recount E and M of the current spins from scratch into E_dev[0] and
 * M_dev[0] (device int64, caller-owned; either may be NULL):
 * E = -sum over right and down bonds of s_i s_j, M = sum s_i.  Paper: the
 * Hamiltonian of Eq. (1) restricted to theta in {0, pi}, whose per-site
 * mean is the internal energy U = <H>/L^2 of Supplementary Eq. (S3).
 * Asynchronous on hip_stream; uses the workspace accumulators, so it must
 * not overlap another call on the same lattice.  Errors: invalid lattice
 * -> ISING_E_INVALID. */
ISING_API int ising_measure(const ising_lattice *lat, int64_t *E_dev, int64_t *M_dev,
                  void *hip_stream);

/* Copy the spins to / from the canonical INT8 row-major form (device
 * int8[L*L] of +1/-1, 4-byte aligned).  ising_from_int8 does not change
 * sweep_index.
 * Values other than +1/-1 in the input are read as -1 if negative, else +1. */
ISING_API int ising_to_int8(const ising_lattice *lat, int8_t *out_dev, void *hip_stream);
ISING_API int ising_from_int8(ising_lattice *lat, const int8_t *in_dev, void *hip_stream);

/* Read back (synchronising hip_stream) how many Philox4x32-10 blocks
 * (128 random bits each) the sweeps on this lattice have drawn since the
 * last ising_init: the random-number work the method actually consumed,
 * which sets the integer-ALU cost of a sweep.  A BIT1 lattice counts only
 * the sweeps run with ISING_FLAG_COUNT_DRAWS; a block counts when some site
 * of its 32-site word was still undecided before it.  Diagnostic only. */
ISING_API int ising_rng_blocks(const ising_lattice *lat, uint64_t *blocks_host,
                               void *hip_stream);

/* Read back (synchronising hip_stream) the device error word written by
 * kernels that wait on each other; returns ISING_OK if clear, else
 * ISING_E_STATE with a message, and clears it. */
ISING_API int ising_check_device_error(const ising_lattice *lat, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batches of small lattices in one persistent launch.
 *
 * Many independent L x L lattices (INT8 in memory, each with its own beta),
 * for example a grid of temperatures, a set of replicas or the independent
 * chains of a finite-size study.  The update rule and observables are those
 * above, applied to every lattice; lattice j of the batch draws with
 * lattice_id = lattice_id0 + j, either per site (ISING_DRAWS_SITE: the
 * draws of an INT8 lattice, any L % 8 == 0) or as bit planes
 * (ISING_DRAWS_PLANE: the draws of a BIT1 lattice, generalised to L = 32,
 * where a group of 32 compact columns spans rows 2g and 2g + 1; every L
 * must be 32 or a multiple of 64).  Each lattice stays in LDS for all n
 * sweeps of a call, as bytes (site draws) or as two colour bit planes
 * updated 32 sites per lane (plane draws).  With site draws workgroups take
 * lattices from a device work queue, largest L first; with plane draws the
 * largest-first order is dealt out to the workgroups in a snake (positions
 * g, 2G - 1 - g, 2G + g, ... to workgroup g of G), and each workgroup sweeps
 * its lattices together, one team of lanes per lattice.
 * The sweep index t of the batch lives in device memory (in the
 * workspace) and is advanced on the device, so that the launches of
 * ising_batch_sweep can be captured once in a HIP graph and replayed: each
 * replay continues the chain.  The launch shape (threads, groups_per_cu)
 * never changes the chain, only the speed.
 * ------------------------------------------------------------------------ */

#define ISING_BATCH_MAX_L 256      /* whole lattice in LDS: L*L bytes <= 64 KiB */
enum { ISING_DRAWS_SITE = 0, ISING_DRAWS_PLANE = 1 };
#define ISING_BATCH_MAX_COUNT 65536

typedef struct ising_batch {
    int32_t abi_version;    /* must equal ISING_ABI_VERSION                    */
    int32_t count;          /* lattices, 1..ISING_BATCH_MAX_COUNT              */
    uint64_t seed;          /* Philox key shared by the batch                  */
    uint32_t lattice_id0;   /* lattice j draws with lattice_id0 + j (no wrap)  */
    int32_t max_L;          /* >= every L of the batch; sizes the LDS of the
                               sweep: L % 8 == 0, 8 <= max_L <= 256            */
    int32_t threads;        /* threads per workgroup: 0 = library choice, else
                               a multiple of 64 in 64..1024                    */
    int32_t groups_per_cu;  /* workgroups per compute unit: 0 = library choice,
                               else 1..16 (fewer if LDS or threads do not fit) */
    int32_t draws;          /* ISING_DRAWS_SITE or ISING_DRAWS_PLANE; the same
                               at setup and at every sweep                     */
    int32_t reserved;       /* 0                                               */
    uint64_t spins_bytes;   /* size of the spins buffer in bytes               */
    int8_t *spins;          /* device, 256-B aligned: lattice j at byte offset
                               offsets[j] (see ising_batch_spins_bytes),
                               INT8 row-major +1/-1                            */
    void *workspace;        /* device, 256-B aligned,
                               >= ising_batch_workspace_bytes(count)           */
} ising_batch;

/* Bytes of the spins buffer for lattices of sides L_host[0..count-1] and,
 * when offsets_host is non-NULL, the byte offset of each lattice (each a
 * multiple of 256, in order).  Every L must be a multiple of 8 in
 * 8..ISING_BATCH_MAX_L.  Returns 0 if count or an L is invalid. */
ISING_API size_t ising_batch_spins_bytes(int32_t count, const int32_t *L_host,
                                         uint64_t *offsets_host);

/* Bytes of device workspace of a batch of count lattices (0 if invalid):
 * sweep index, work queue, error word, draw counters, the per-lattice
 * descriptor table and the queue order. */
ISING_API size_t ising_batch_workspace_bytes(int32_t count);

/* Write the per-lattice descriptors into the workspace: sides L_host[j],
 * byte offsets as ising_batch_spins_bytes lays them out, and the
 * acceptance thresholds of beta_host[j] (as ising_thresholds).  Does not
 * touch the spins or the sweep index, so it may be called again between
 * sweeps to change the temperatures.  The copy is complete when the call
 * returns (it synchronises hip_stream); the host arrays may be freed then.
 * Errors: invalid batch description, an L that is invalid or above max_L
 * (or, with plane draws, neither 32 nor a multiple of 64), a beta that is
 * negative, NaN or infinite, spins_bytes too small -> ISING_E_INVALID,
 * nothing written. */
ISING_API int ising_batch_setup(const ising_batch *b, const int32_t *L_host,
                                const double *beta_host, void *hip_stream);

/* Fill every lattice (ISING_START_COLD_UP or ISING_START_RANDOM, each with
 * its own lattice id) and set the device sweep index to 0.  Requires a
 * prior ising_batch_setup on this workspace. */
ISING_API int ising_batch_init(const ising_batch *b, int32_t start, void *hip_stream);

/* Run n >= 0 sweeps of every lattice at its beta, from the device sweep
 * index t, then advance t by n on the device.  Only kernel launches are
 * enqueued (no copies, no memsets, no host reads), so the call may be
 * captured in a HIP graph.  When moments_dev is non-NULL it is device
 * int64[count][8] and receives, for lattice j and the states after each
 * of the n sweeps of this call:
 *   [0] E after the last sweep        [1] M after the last sweep
 *   [2] sum E     [3] sum E^2         [4] sum |M|     [5] sum M^2
 *   [6], [7] sum M^4 as an unsigned 128-bit integer (low, high 64 bits)
 * (exact while n * E^2 < 2^63; n < 2^29 suffices for every L <= 256).
 * When trace_dev is non-NULL it is device int64[n][count][2] and receives
 * E and M of every lattice after every sweep of this call (the time series
 * behind autocorrelation times).
 * These are the energy and magnetisation moments behind U = <H>/L^2, the
 * specific heat and the Binder cumulant.
 * Errors (host): invalid batch, n < 0 or n > 2^31 -> ISING_E_INVALID.
 * Errors (device, reported by ising_batch_check_device_error): the
 * workspace was not set up for this batch, a descriptor does not fit the
 * spins buffer or max_L, or t + n > 2^31; then no lattice is changed and
 * t is not advanced. */
ISING_API int ising_batch_sweep(const ising_batch *b, int64_t n, int64_t *moments_dev,
                                int64_t *trace_dev, void *hip_stream);

/* Recount E and M of every lattice from scratch into E_dev[j], M_dev[j]
 * (device int64[count]; either may be NULL). */
ISING_API int ising_batch_measure(const ising_batch *b, int64_t *E_dev, int64_t *M_dev,
                                  void *hip_stream);

/* Read back (synchronising hip_stream) the device sweep index. */
ISING_API int ising_batch_sweep_index(const ising_batch *b, uint64_t *t_host,
                                      void *hip_stream);

/* Read back (synchronising hip_stream) the Philox blocks drawn by the
 * batch sweeps since ising_batch_init.  Diagnostic only. */
ISING_API int ising_batch_rng_blocks(const ising_batch *b, uint64_t *blocks_host,
                                     void *hip_stream);

/* Read back (synchronising hip_stream) and clear the device error word of
 * the batch: ISING_OK if clear, else ISING_E_STATE with a message. */
ISING_API int ising_batch_check_device_error(const ising_batch *b, void *hip_stream);

/* Autotuner: time every launch shape (threads per workgroup x workgroups
 * per CU) that fits the device, each running probe_sweeps sweeps on a copy
 * of the spins in scratch_spins (device, >= spins_bytes, 256-B aligned),
 * and store the fastest in b->threads and b->groups_per_cu.  The spins,
 * the sweep index and the draw counters of the batch are not changed.
 * Synchronises hip_stream.  The chain does not depend on the shape, so a
 * tuned batch continues exactly as an untuned one would.  When
 * times_ms_host is non-NULL it receives up to max_times entries of
 * (threads, groups_per_cu, milliseconds) as three doubles each; the number
 * of shapes timed is returned in *n_times (may be NULL).
 * Errors: invalid batch, probe_sweeps < 1 or > 10^6, scratch invalid ->
 * ISING_E_INVALID. */
ISING_API int ising_batch_autotune(ising_batch *b, int8_t *scratch_spins, int64_t probe_sweeps,
                                   double *times_ms_host, int32_t max_times, int32_t *n_times,
                                   void *hip_stream);

/* Thread-local description of the last error on this thread ("" if none). */
ISING_API const char *ising_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
