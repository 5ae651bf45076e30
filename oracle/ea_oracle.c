/*
 * CPU oracle for the 3D Edwards-Anderson +-J spin glass with replica
 * exchange (parallel tempering).  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path calls, links or loads this file.
 *
 * The update is the paper's single-spin-flip Metropolis trial (Fig. 2c;
 * Supplementary, "Detail of the MC calculation": draw p, compute dE and
 * P = exp(-beta dE), accept iff p < P) on the bipartite simple cubic
 * lattice (the two sublattices updated alternately, as in Fig. 2a-b), with
 * random couplings J in {+1, -1}:
 *     H = - sum_n sum_{d = x,y,z} J_d(n) s_n s_{n + e_d},   periodic.
 * Replica exchange swaps the temperatures of replicas at adjacent betas
 * with probability min(1, exp((beta_k - beta_{k+1}) (E_k - E_{k+1}))).
 *
 * Conventions (the same readings as the 2D oracle, written out again):
 *   site n = (z L + y) L + x, colour (x + y + z) & 1, colour 0 first;
 *   J[d N + n] couples n and n + e_d (d = 0: x, 1: y, 2: z);
 *   u = s_n h_n, h_n the coupling-weighted sum of the six neighbours,
 *   dE = 2u; u <= 0 flips without a draw; otherwise the draw is
 *   r = out[q & 3] of Philox counter (q >> 2, replica id, 2t + c, 0),
 *   q = n >> 1, and the flip is accepted iff r < ceil(2^32 exp(-2 beta u)).
 *   Exchange after sweep t when (t + 1) % every == 0, as exchange number
 *   m = (t + 1) / every - 1: pairs (k, k+1) with k = m & 1, m & 1 + 2, ...;
 *   D = E(replica at k) - E(replica at k+1); accepted without a draw when
 *   D <= 0 (beta_k < beta_{k+1}), else iff r < ceil(2^32 exp(-(beta_{k+1}
 *   - beta_k) D)) with r = out[0] of counter (k, m, 0, 5).
 *   Random start: s = -1 iff the top bit of out[n & 3] of counter
 *   (n >> 2, replica id, 0, 2) is set.
 *   Plane draws (mode 1, the bit-plane layout of the 2D oracle carried to
 *   3D): the colour-c sites with q >> 5 == g form group g, lane l = q & 31;
 *   plane k (k = 0 most significant) is P_k = out[k & 3] of counter
 *   (g, replica id, 2t + c, 1 | (k >> 2) << 8), and
 *   r = sum_k ((P_k >> l) & 1) << (31 - k).  Mode 0 is the per-site draw
 *   above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);

static void ea_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                      uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

static int64_t wrap(int64_t v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

/* Neighbour of site n one step along axis d in direction dir (+1 / -1). */
static int64_t neighbour(int64_t n, int L, int d, int dir)
{
    int64_t x = n % L, y = (n / L) % L, z = n / ((int64_t)L * L);
    if (d == 0) x = wrap(x + dir, L);
    if (d == 1) y = wrap(y + dir, L);
    if (d == 2) z = wrap(z + dir, L);
    return (z * L + y) * L + x;
}

/* H = - sum_n sum_d J_d(n) s_n s_{n + e_d}. */
int64_t oracle_ea_energy(const int8_t *s, const int8_t *J, int L)
{
    int64_t N = (int64_t)L * L * L, E = 0;
    for (int64_t n = 0; n < N; ++n)
        for (int d = 0; d < 3; ++d)
            E -= (int64_t)J[d * N + n] * s[n] * s[neighbour(n, L, d, +1)];
    return E;
}

/* u = s_n h_n, h_n = sum_d [J_d(n) s_{n+e_d} + J_d(n-e_d) s_{n-e_d}]. */
int oracle_ea_local_u(const int8_t *s, const int8_t *J, int L, int64_t n)
{
    int64_t N = (int64_t)L * L * L;
    int h = 0;
    for (int d = 0; d < 3; ++d) {
        int64_t up = neighbour(n, L, d, +1), dn = neighbour(n, L, d, -1);
        h += J[d * N + n] * s[up] + J[d * N + dn] * s[dn];
    }
    return s[n] * h;
}

/* T[i] = ceil(2^32 exp(-beta dE)) for u = 2(i+1), dE = 2u; always[i] when
 * that rounds up to 2^32.  Returns nonzero for an invalid beta. */
int oracle_ea_thresholds(double beta, uint32_t T[3], uint8_t always_flip[3])
{
    if (!(beta >= 0.0) || isinf(beta))
        return 1;
    for (int i = 0; i < 3; ++i) {
        int u = 2 * (i + 1);
        double t = ceil(ldexp(exp(-beta * (double)(2 * u)), 32));
        always_flip[i] = t >= 4294967296.0;
        T[i] = always_flip[i] ? 0u : (uint32_t)t;
    }
    return 0;
}

/* Swap of the replicas at beta_lo < beta_hi with energies differing by
 * D = E_lo - E_hi: always when D <= 0, else iff r < T. */
void oracle_ea_swap_threshold(double beta_lo, double beta_hi, int64_t D, uint32_t *T,
                              uint8_t *always_flip)
{
    if (D <= 0) {
        *always_flip = 1;
        *T = 0;
        return;
    }
    double t = ceil(ldexp(exp(-(beta_hi - beta_lo) * (double)D), 32));
    *always_flip = t >= 4294967296.0;
    *T = *always_flip ? 0u : (uint32_t)t;
}

void oracle_ea_init(int8_t *s, int L, int start, uint64_t seed, uint32_t replica_id)
{
    int64_t N = (int64_t)L * L * L;
    for (int64_t n = 0; n < N; ++n) {
        if (start == 0) {
            s[n] = 1;
            continue;
        }
        uint32_t out[4];
        ea_philox(seed, (uint32_t)(n >> 2), replica_id, 0u, 2u, out);
        s[n] = (out[n & 3] >> 31) ? -1 : 1;
    }
}

/* Plane draws of half-sweep h for every colour-c site: r[n] for the sites
 * of colour c (entries of the other colour untouched). */
static void ea_fill_plane_threads(uint32_t *r, int L, int c, uint64_t seed, uint32_t replica_id,
                                  uint32_t h, int nthreads)
{
    int64_t N = (int64_t)L * L * L, half = N / 2, row = L / 2;
    int64_t groups = (half + 31) / 32;
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
    for (int64_t g = 0; g < groups; ++g) {
        uint32_t planes[32];
        for (int b = 0; b < 8; ++b) {
            uint32_t out[4];
            ea_philox(seed, (uint32_t)g, replica_id, h, 1u | ((uint32_t)b << 8), out);
            for (int j = 0; j < 4; ++j)
                planes[4 * b + j] = out[j];
        }
        for (int l = 0; l < 32; ++l) {
            int64_t q = 32 * g + l;
            if (q >= half)
                break;
            /* the colour-c site with compact index q: row q / (L/2) of the
             * (z, y) rows, column 2 (q % (L/2)) + parity */
            int64_t R = q / row, i = q % row;
            int64_t y = R % L, z = R / L;
            int64_t x = 2 * i + ((y + z + c) & 1);
            uint32_t v = 0;
            for (int k = 0; k < 32; ++k)
                v |= ((planes[k] >> l) & 1u) << (31 - k);
            r[R * L + x] = v;
        }
    }
}

void oracle_ea_fill_plane(uint32_t *r, int L, int c, uint64_t seed, uint32_t replica_id,
                          uint32_t h)
{
    ea_fill_plane_threads(r, L, c, seed, replica_id, h, 1);
}

/* Update every site of colour c of one replica at inverse temperature beta
 * (sweep index t) with per-site (mode 0) or plane (mode 1) draws; the
 * energy change goes to *dE. */
int oracle_ea_halfsweep(int8_t *s, const int8_t *J, int L, int c, uint64_t seed,
                        uint32_t replica_id, uint64_t t, double beta, int64_t *dE, int nthreads,
                        int mode)
{
    if (mode != 0 && mode != 1)
        return 1;
    uint32_t T[3];
    uint8_t always_flip[3];
    if (oracle_ea_thresholds(beta, T, always_flip))
        return 1;
    int64_t N = (int64_t)L * L * L, total = 0;
    uint32_t h = (uint32_t)(2 * t + (uint64_t)c);
    uint32_t *rp = NULL;
    if (mode == 1) {
        rp = (uint32_t *)calloc((size_t)N, sizeof(uint32_t));
        if (!rp)
            return 2;
        ea_fill_plane_threads(rp, L, c, seed, replica_id, h, nthreads < 1 ? 1 : nthreads);
    }
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) reduction(+ : total) schedule(static)
#endif
    for (int64_t n = 0; n < N; ++n) {
        int64_t x = n % L, y = (n / L) % L, z = n / ((int64_t)L * L);
        if (((x + y + z) & 1) != c)
            continue;
        int u = oracle_ea_local_u(s, J, L, n);
        int flip = u <= 0;
        if (!flip) {
            int i = u / 2 - 1;
            if (always_flip[i]) {
                flip = 1;
            } else if (mode == 1) {
                flip = rp[n] < T[i];
            } else {
                uint32_t out[4];
                uint64_t q = (uint64_t)n >> 1;
                ea_philox(seed, (uint32_t)(q >> 2), replica_id, h, 0u, out);
                flip = out[q & 3] < T[i];
            }
        }
        if (flip) {
            s[n] = (int8_t)-s[n];
            total += 2 * u;
        }
    }
    (void)nthreads;
    free(rp);
    *dE = total;
    return 0;
}

/* Exchange number m on the temperature ladder beta[0..R-1] (increasing):
 * perm[k] is the replica at temperature k; E[r] the energy of replica r. */
void oracle_ea_exchange(const int64_t *E, int32_t *perm, int R, const double *beta, uint64_t m,
                        uint64_t seed, uint64_t *accepts)
{
    for (int k = (int)(m & 1); k + 1 < R; k += 2) {
        int64_t D = E[perm[k]] - E[perm[k + 1]];
        uint32_t T;
        uint8_t always_flip;
        oracle_ea_swap_threshold(beta[k], beta[k + 1], D, &T, &always_flip);
        int swap = always_flip;
        if (!swap) {
            uint32_t out[4];
            ea_philox(seed, (uint32_t)k, (uint32_t)m, 0u, 5u, out);
            swap = out[0] < T;
        }
        if (swap) {
            int32_t a = perm[k];
            perm[k] = perm[k + 1];
            perm[k + 1] = a;
            if (accepts)
                accepts[k] += 1;
        }
    }
}

/* n sweeps of R replicas (spins[r * N ...], replica id r) from sweep index
 * t0 with an exchange after every `every`-th sweep (every >= 1; 0 means
 * none).  perm (temperature -> replica) and E (per replica, must hold the
 * current energies) are updated in place; E_trace[j * R + r], when given,
 * receives E of replica r after sweep j. */
int oracle_ea_run(int8_t *spins, const int8_t *J, int L, int R, const double *beta,
                  uint64_t seed, uint64_t t0, int64_t n, int every, int32_t *perm, int64_t *E,
                  uint64_t *accepts, int64_t *E_trace, int nthreads, int mode)
{
    if (L < 2 || (L & 1) || R < 1 || n < 0 || every < 0)
        return 1;
    if (t0 + (uint64_t)n > (1ull << 31))
        return 1;
    int64_t N = (int64_t)L * L * L;
    int32_t *tidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    if (!tidx)
        return 2;
    for (int64_t j = 0; j < n; ++j) {
        uint64_t t = t0 + (uint64_t)j;
        for (int k = 0; k < R; ++k)
            tidx[perm[k]] = k;
        for (int c = 0; c < 2; ++c)
            for (int r = 0; r < R; ++r) {
                int64_t dE = 0;
                if (oracle_ea_halfsweep(spins + (int64_t)r * N, J, L, c, seed, (uint32_t)r, t,
                                        beta[tidx[r]], &dE, nthreads, mode)) {
                    free(tidx);
                    return 1;
                }
                E[r] += dE;
            }
        if (E_trace)
            memcpy(E_trace + j * R, E, sizeof(int64_t) * (size_t)R);
        if (every > 0 && (t + 1) % (uint64_t)every == 0)
            oracle_ea_exchange(E, perm, R, beta, (t + 1) / (uint64_t)every - 1, seed, accepts);
    }
    free(tidx);
    return 0;
}
