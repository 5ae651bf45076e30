/*
 * CPU oracle for the checkerboard Metropolis sweep of the 2D Ising model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library: everything here is written out again from
 * the paper and from the published definition of Philox4x32-10.
 *
 * What it computes (paper: "Many-body computing on Field Programmable Gate
 * Arrays", arXiv 2402.06415):
 *   - Hamiltonian: Eq. (1) restricted to theta in {0, pi}, i.e. spins
 *     s = cos(theta) = +-1 and H = -sum_<ij> s_i s_j (J = 1, h = 0),
 *     periodic boundaries (Supplementary, "Detail of the MC calculation").
 *   - Bipartition: the square lattice splits into two sublattices A and B
 *     that are updated alternately (Results, "Parallel design of MC
 *     simulation for the XY model"; Fig. 2a-b).  A site's update does not
 *     change the acceptance of another site of the same sublattice
 *     (Supplementary, same section), so an in-place scan of one colour is
 *     the same as the parallel update.
 *   - One single-spin-flip trial per site in three steps (Fig. 2c;
 *     Supplementary): (1) draw a uniform p in [0,1); (2) compute the energy
 *     change dE of the proposed flip and P(dE) = exp(-beta dE); (3) accept
 *     iff p < P.
 *
 * Readings fixed here (the paper is silent on them):
 *   - colour(x,y) = (x+y)&1, colour 0 first in every sweep;
 *   - p = r / 2^32 with r a uint32, so p < P  <=>  r < ceil(2^32 P);
 *     dE <= 0 is accepted without drawing (P >= 1);
 *   - the paper's per-site LCG is replaced by Philox4x32-10 (Salmon,
 *     Moraes, Dror, Shaw, SC'11) keyed by the 64-bit seed, with counters
 *     built from (site, lattice id, half-sweep index, tag) as below.
 *
 * Parity pins: see tests/test_oracle_*.py (Philox against PyTorch's
 * independent header implementation; thresholds against the acceptance
 * rule in 80-digit arithmetic; 4x4 exact enumeration; exact detailed
 * balance of each half-sweep on 4x4; Kaufman's finite-torus energy;
 * Onsager's energy; Yang's magnetisation; the beta = 0 and Z2 special
 * cases; split-sweep invariance).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------
 * Philox4x32-10 (Salmon et al., SC'11, section 4.2).
 * State: counter (c0,c1,c2,c3), key (k0,k1).  One round:
 *   (hi0,lo0) = M0 * c0,  (hi1,lo1) = M1 * c2      (32x32 -> 64-bit)
 *   c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
 * and between rounds the key advances by the Weyl constants (W0,W1).
 * Ten rounds; the output is the final counter.
 * ------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                   uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* Counter tags (fourth counter word). */
#define TAG_SITE  0u   /* one uint32 per site, four sites per call   */
#define TAG_PLANE 1u   /* bit planes, 32 sites per call, block in bits 8.. */
#define TAG_INIT  2u   /* random start                                 */

enum { MODE_SITE = 0, MODE_PLANE = 1 };
enum { START_COLD_UP = 0, START_RANDOM = 1 };

/* ---------------------------------------------------------------------
 * Acceptance thresholds.  Step (2) of the trial: u = s_i * h_i with h_i the
 * sum of the four neighbours, dE = 2u, P = exp(-beta dE).  Step (3):
 * accept iff p < P with p = r/2^32, i.e. iff r < T[u] = ceil(2^32 P).
 * Index k = (u + 4) / 2 runs over u = -4,-2,0,2,4.  always[k] = 1 when the
 * flip is accepted without a draw (dE <= 0, or 2^32 P rounds to 2^32).
 * ------------------------------------------------------------------- */
int oracle_thresholds(double beta, uint32_t T[5], uint8_t always_flip[5])
{
    if (!(beta >= 0.0) || isinf(beta))
        return 1;
    for (int k = 0; k < 5; ++k) {
        int u = 2 * k - 4;
        T[k] = 0;
        always_flip[k] = 0;
        if (u <= 0) {
            always_flip[k] = 1;
            continue;
        }
        double P = exp(-beta * (double)(2 * u));
        double scaled = ceil(ldexp(P, 32));
        if (scaled >= 4294967296.0)
            always_flip[k] = 1;
        else
            T[k] = (uint32_t)scaled;
    }
    return 0;
}

/* Decision of step (3) for one site. */
int oracle_accept(int u, uint32_t r, const uint32_t T[5],
                  const uint8_t always_flip[5])
{
    int k = (u + 4) / 2;
    if (always_flip[k])
        return 1;
    return r < T[k];
}

/* u = s(x,y) * (sum of the four periodic neighbours). */
int oracle_local_u(const int8_t *s, int L, int x, int y)
{
    int xp = (x + 1) % L, xm = (x + L - 1) % L;
    int yp = (y + 1) % L, ym = (y + L - 1) % L;
    int h = s[(int64_t)y * L + xp] + s[(int64_t)y * L + xm] +
            s[(int64_t)yp * L + x] + s[(int64_t)ym * L + x];
    return s[(int64_t)y * L + x] * h;
}

/* ---------------------------------------------------------------------
 * Random start (step (1) of the paper's set-up draws a random angle per
 * site; the Ising restriction draws a random sign).  Site n = y*L + x;
 * counter (n>>2, lattice_id, 0, TAG_INIT); s = -1 iff the top bit of
 * out[n & 3] is set.
 * ------------------------------------------------------------------- */
int oracle_init(int8_t *s, int L, int start, uint64_t seed, uint32_t lattice_id)
{
    if (L < 4 || (L & 1))
        return 1;
    int64_t N = (int64_t)L * L;
    for (int64_t n = 0; n < N; ++n) {
        if (start == START_COLD_UP) {
            s[n] = 1;
        } else if (start == START_RANDOM) {
            uint32_t out[4];
            philox(seed, (uint32_t)(n >> 2), lattice_id, 0u, TAG_INIT, out);
            s[n] = (out[n & 3] >> 31) ? (int8_t)-1 : (int8_t)1;
        } else {
            return 1;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------
 * Uniform draws of step (1) for every site of colour c in half-sweep
 * h = 2t + c.  r is indexed by site n = y*L + x; entries of the other
 * colour are left untouched.  The compact index of a site within its
 * colour is q = n >> 1 (exact for even L).
 *
 * SITE mode : counter (q>>2, lattice_id, h, TAG_SITE), r = out[q & 3].
 * PLANE mode (L % 32 == 0): the sites with q>>5 == g form group g and lane
 *   l = q & 31 (one row holds L/2 compact indices: a group lies within one
 *   row when L % 64 == 0 and spans two consecutive rows when L % 64 == 32).  Plane k (k = 0 is the most significant bit) is
 *   P_k = out[k & 3] of counter (g, lattice_id, h, TAG_PLANE | (k>>2) << 8),
 *   and r = sum_k ((P_k >> l) & 1) << (31 - k).
 * ------------------------------------------------------------------- */
int oracle_fill_uniforms(int L, int mode, uint64_t seed, uint32_t lattice_id,
                         uint64_t t, int c, uint32_t *r, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (L < 4 || (L & 1) || (c != 0 && c != 1))
        return 1;
    if (mode == MODE_PLANE && (L % 32) != 0)
        return 1;
    if (t >= (1ull << 31))
        return 1;
    uint32_t h = (uint32_t)(2 * t + (uint64_t)c);
    int64_t N = (int64_t)L * L;
    if (mode == MODE_SITE) {
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
        for (int64_t n = 0; n < N; ++n) {
            int x = (int)(n % L), y = (int)(n / L);
            if (((x + y) & 1) != c)
                continue;
            int64_t q = n >> 1;
            uint32_t out[4];
            philox(seed, (uint32_t)(q >> 2), lattice_id, h, TAG_SITE, out);
            r[n] = out[q & 3];
        }
        return 0;
    }
    if (mode == MODE_PLANE) {
        /* Group g holds compact indices 32g .. 32g+31 of colour c, in one
         * row or (L % 64 == 32) in two; the site list below maps each back. */
        int64_t groups = N / 64; /* N/2 compact indices of colour c, 32 per group */
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
        for (int64_t g = 0; g < groups; ++g) {
            uint32_t planes[32];
            for (int b = 0; b < 8; ++b) {
                uint32_t out[4];
                philox(seed, (uint32_t)g, lattice_id, h,
                       TAG_PLANE | ((uint32_t)b << 8), out);
                for (int j = 0; j < 4; ++j)
                    planes[4 * b + j] = out[j];
            }
            for (int l = 0; l < 32; ++l) {
                int64_t q = 32 * g + l;
                /* the site of colour c with compact index q */
                int64_t y = q / (L / 2);
                int64_t i = q % (L / 2);
                int64_t x = 2 * i + ((y + c) & 1);
                int64_t n = y * L + x;
                uint32_t v = 0;
                for (int k = 0; k < 32; ++k)
                    v |= ((planes[k] >> l) & 1u) << (31 - k);
                r[n] = v;
            }
        }
        return 0;
    }
    (void)nthreads;
    return 1;
}

/* ---------------------------------------------------------------------
 * One half-sweep (update of sublattice c) with given draws r[site].
 * Steps (2) and (3) for each site of colour c; the energy and
 * magnetisation changes of the accepted flips are summed:
 * flip => dE = 2u, dM = -2 s_old.
 * ------------------------------------------------------------------- */
int oracle_halfsweep(int8_t *s, int L, int c, const uint32_t *r,
                     const uint32_t T[5], const uint8_t always_flip[5],
                     int64_t *dE_out, int64_t *dM_out, int nthreads)
{
    if (L < 4 || (L & 1) || (c != 0 && c != 1))
        return 1;
    int64_t dE = 0, dM = 0;
#ifdef _OPENMP
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) reduction(+ : dE, dM) schedule(static)
#endif
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            if (((x + y) & 1) != c)
                continue;
            int64_t n = (int64_t)y * L + x;
            int u = oracle_local_u(s, L, x, y);
            if (oracle_accept(u, r[n], T, always_flip)) {
                dE += 2 * u;
                dM += -2 * s[n];
                s[n] = (int8_t)(-s[n]);
            }
        }
    }
    (void)nthreads;
    if (dE_out)
        *dE_out = dE;
    if (dM_out)
        *dM_out = dM;
    return 0;
}

/* E = -sum over right and down bonds of s_i s_j; M = sum of s_i. */
void oracle_measure(const int8_t *s, int L, int64_t *E_out, int64_t *M_out)
{
    int64_t E = 0, M = 0;
    for (int y = 0; y < L; ++y) {
        for (int x = 0; x < L; ++x) {
            int64_t n = (int64_t)y * L + x;
            int right = s[(int64_t)y * L + (x + 1) % L];
            int down = s[(int64_t)((y + 1) % L) * L + x];
            E -= s[n] * (right + down);
            M += s[n];
        }
    }
    *E_out = E;
    *M_out = M;
}

/* ---------------------------------------------------------------------
 * n sweeps starting at sweep index t0.  A sweep is the update of
 * sublattice 0 then sublattice 1 (Fig. 2b: A and B alternately).  After
 * each sweep the running E and M (started from a full recount) are
 * written to E_trace[j], M_trace[j] when those are non-NULL.
 * ------------------------------------------------------------------- */
int oracle_sweep(int8_t *s, int L, int mode, uint64_t seed, uint32_t lattice_id,
                 uint64_t t0, int64_t n, double beta, int64_t *E_trace,
                 int64_t *M_trace, int nthreads)
{
    if (L < 4 || (L & 1) || n < 0)
        return 1;
    if (mode != MODE_SITE && mode != MODE_PLANE)
        return 1;
    if (mode == MODE_PLANE && (L % 32) != 0)
        return 1;
    if (t0 + (uint64_t)n > (1ull << 31))
        return 1;
    uint32_t T[5];
    uint8_t always_flip[5];
    if (oracle_thresholds(beta, T, always_flip))
        return 1;
    int64_t N = (int64_t)L * L;
    uint32_t *r = (uint32_t *)calloc((size_t)N, sizeof(uint32_t));
    if (!r)
        return 2;
    int64_t E = 0, M = 0;
    oracle_measure(s, L, &E, &M);
    for (int64_t j = 0; j < n; ++j) {
        uint64_t t = t0 + (uint64_t)j;
        for (int c = 0; c < 2; ++c) {
            int64_t dE = 0, dM = 0;
            oracle_fill_uniforms(L, mode, seed, lattice_id, t, c, r, nthreads);
            oracle_halfsweep(s, L, c, r, T, always_flip, &dE, &dM, nthreads);
            E += dE;
            M += dM;
        }
        if (E_trace)
            E_trace[j] = E;
        if (M_trace)
            M_trace[j] = M;
    }
    free(r);
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
