/*
 * CPU oracle for the Metropolis Monte Carlo of the 2D classical XY model
 * (the paper's own workload).  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path calls, links or loads this file.
 *
 * Hamiltonian: Eq. (1), H = - sum_<x,delta> cos(theta_x - theta_{x+delta}),
 * periodic L x L square lattice, theta in [0, 2 pi), double precision.
 * Each trial follows the Supplementary section "Detail of the MC
 * calculation for the XY model":
 *   step 1: a new angle theta' uniform in [0, 2 pi) and p uniform in [0, 1);
 *   step 2: P = exp(-beta dE) with the local energy change of the rotation
 *           (Eq. S1, whose printed sign between the two cosines is garbled;
 *           the energy change new - old is used):
 *             dE = - sum_delta [cos(theta' - theta_delta) - cos(theta - theta_delta)];
 *   step 3: theta <- theta' iff p < P.
 * The two sublattices (x + y even, then odd) are updated alternately
 * (Fig. 2a-b).  The paper's per-site LCG is replaced by Philox4x32-10:
 * the trial of the site with compact index q = n >> 1 in half-sweep 2t + c
 * of lattice `lid` uses out of counter (q, lid, 2t + c, 8):
 *   u1 = ((out[0] << 32 | out[1]) >> 11) 2^-53,  theta' = u1 * 2 pi,
 *   u2 = ((out[2] << 32 | out[3]) >> 11) 2^-53,  p = u2;
 * the neighbours are summed in the order right, left, down, up.  Random
 * start: theta_n = u1 * 2 pi from counter (n, lid, 0, 9).  Compiled without
 * floating-point contraction, so every operation is rounded separately.
 */
#include <math.h>
#include <stdint.h>

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);

static const double XY_TWO_PI = 6.283185307179586;  /* nearest double to 2 pi */

static void xy_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                      uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

static double unit53(uint32_t hi, uint32_t lo)
{
    uint64_t k = (((uint64_t)hi << 32) | lo) >> 11;
    return (double)k * 0x1.0p-53;
}

void oracle_xy_init(double *theta, int L, int start, uint64_t seed, uint32_t lid)
{
    for (int64_t n = 0; n < (int64_t)L * L; ++n) {
        if (start == 0) {
            theta[n] = 0.0;
            continue;
        }
        uint32_t out[4];
        xy_philox(seed, (uint32_t)n, lid, 0u, 9u, out);
        theta[n] = unit53(out[0], out[1]) * XY_TWO_PI;
    }
}

/* H = - sum_n [cos(theta_n - theta_right) + cos(theta_n - theta_down)]. */
double oracle_xy_energy(const double *theta, int L)
{
    double E = 0.0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            double t = theta[y * L + x];
            double r = theta[y * L + (x + 1) % L];
            double d = theta[((y + 1) % L) * L + x];
            E -= cos(t - r) + cos(t - d);
        }
    return E;
}

/* One half-sweep (colour c) of one lattice; returns the number of accepted
 * rotations. */
int64_t oracle_xy_halfsweep(double *theta, int L, int c, uint64_t seed, uint32_t lid,
                            uint64_t t, double beta)
{
    int64_t accepted = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            if (((x + y) & 1) != c)
                continue;
            int64_t n = (int64_t)y * L + x;
            uint32_t out[4];
            xy_philox(seed, (uint32_t)(n >> 1), lid, (uint32_t)(2 * t + (uint64_t)c), 8u, out);
            double th_new = unit53(out[0], out[1]) * XY_TWO_PI;
            double p = unit53(out[2], out[3]);
            double th = theta[n];
            double nb[4] = {theta[y * L + (x + 1) % L], theta[y * L + (x + L - 1) % L],
                            theta[((y + 1) % L) * L + x], theta[((y + L - 1) % L) * L + x]};
            double d = 0.0;
            for (int k = 0; k < 4; ++k)
                d += cos(th_new - nb[k]) - cos(th - nb[k]);
            double dE = -d;
            double P = exp(-beta * dE);
            if (p < P) {
                theta[n] = th_new;
                ++accepted;
            }
        }
    return accepted;
}

/* n sweeps from sweep index t0; E_trace[j] (if given) = H after sweep j. */
int oracle_xy_sweep(double *theta, int L, uint64_t seed, uint32_t lid, uint64_t t0, int64_t n,
                    double beta, double *E_trace, int64_t *accepted)
{
    if (L < 2 || (L & 1) || n < 0 || !(beta >= 0.0) || isinf(beta))
        return 1;
    int64_t acc = 0;
    for (int64_t j = 0; j < n; ++j) {
        for (int c = 0; c < 2; ++c)
            acc += oracle_xy_halfsweep(theta, L, c, seed, lid, t0 + (uint64_t)j, beta);
        if (E_trace)
            E_trace[j] = oracle_xy_energy(theta, L);
    }
    if (accepted)
        *accepted = acc;
    return 0;
}
