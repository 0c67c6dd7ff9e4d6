/*
 * xy_hmc_oracle.c -- plain FP64 CPU oracle for hybrid Monte Carlo (HMC)
 * trajectories of the 2-d XY model.
 *
 * TEST INFRASTRUCTURE ONLY, like xy_oracle.c (same library, same rules: the
 * product never links, loads or calls it; it shares nothing with the HIP path).
 *
 * The method (section 1.2): the update the paper benchmarks is HMC.  Momenta
 * are Gaussian numbers converted from flat random numbers, the equations of
 * motion are integrated with leap-frog (the parallel core of the computation),
 * and the Metropolis step is taken on global sums of the energy, which the paper
 * keeps in double precision.  Written out:
 *
 *   fields theta_i (stored as turns phi_i = theta_i / 2 pi), momenta p_i;
 *   H(theta, p) = sum_i p_i^2 / 2 + beta E(theta),
 *   E = -sum_<ij> cos(theta_i - theta_j)            (eq. 1, J = 1, bonds once);
 *   force F_i = -d(beta E)/d theta_i = -beta sum_{j nn i} sin(theta_i - theta_j);
 *   one trajectory:
 *     1. p_i ~ N(0, 1), independently per site;
 *     2. H_old = H(theta, p);
 *     3. n leap-frog steps of size eps, each p += eps/2 F(theta),
 *        theta += eps p, p += eps/2 F(theta);
 *     4. H_new = H(theta', p');
 *     5. accept theta' iff u < exp(-(H_new - H_old)), else keep theta.
 *
 * Random numbers (readings, the paper names no generator or transform):
 *   momenta: Box-Muller, cosine branch, p = sqrt(-2 ln u1) cos(2 pi u2), where
 *     (u1, u2) are the site's two uniforms of purpose 2 for counter word 0 =
 *     the trajectory index (orc_site_words, same pairing of sites as the
 *     Metropolis update);
 *   acceptance: u = u(X0) of Philox with counter (traj, 0, 3, 0).
 *
 * Everything here is FP64; angles are kept in [0, 1) turns by phi - floor(phi)
 * after every drift (the model is periodic in theta, so this changes nothing
 * but the representation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* from xy_oracle.c */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t w);
void orc_site_words(uint64_t seed, int L, int x, int y, uint32_t sweep, uint32_t purpose, uint32_t w[2]);
void orc_measure(int L, const double* phi, double out[6]);

static const double HMC_PI = 3.14159265358979323846264338327950288;
#define HMC_PURPOSE_MOMENTA 2u
#define HMC_PURPOSE_ACCEPT 3u

/* Momentum of site (x, y) at the start of trajectory traj (Box-Muller). */
double orc_hmc_momentum(uint64_t seed, int L, int x, int y, uint32_t traj)
{
    uint32_t w[2];
    orc_site_words(seed, L, x, y, traj, HMC_PURPOSE_MOMENTA, w);
    double u1 = orc_u01(w[0]), u2 = orc_u01(w[1]);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * HMC_PI * u2);
}

void orc_hmc_momenta(uint64_t seed, int L, uint32_t traj, double* p)
{
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x)
            p[y * L + x] = orc_hmc_momentum(seed, L, x, y, traj);
}

/* The uniform of the accept/reject step of trajectory traj. */
double orc_hmc_accept_uniform(uint64_t seed, uint32_t traj)
{
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { traj, 0u, HMC_PURPOSE_ACCEPT, 0u }, r[4];
    orc_philox4x32_10(ctr, key, r);
    return orc_u01(r[0]);
}

/* F_i = -beta sum_{j nn i} sin(theta_i - theta_j), periodic, natural layout. */
void orc_hmc_force(int L, double beta, const double* phi, double* F)
{
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            double t = phi[y * L + x];
            double nb[4] = { phi[y * L + (x + L - 1) % L], phi[y * L + (x + 1) % L],
                             phi[((y + L - 1) % L) * L + x], phi[((y + 1) % L) * L + x] };
            double f = 0.0;
            for (int j = 0; j < 4; ++j) f -= sin(2.0 * HMC_PI * (t - nb[j]));
            F[y * L + x] = beta * f;
        }
}

/* H = sum p^2 / 2 + beta E. */
double orc_hmc_hamiltonian(int L, double beta, const double* phi, const double* p)
{
    double m[6], k = 0.0;
    orc_measure(L, phi, m);
    for (int i = 0; i < L * L; ++i) k += 0.5 * p[i] * p[i];
    return k - beta * (m[0] + m[1]);
}

/* n leap-frog steps of size eps, in place.  Returns 0, or -1 if out of memory. */
int orc_hmc_leapfrog(int L, double beta, double eps, int n, double* phi, double* p)
{
    const int N = L * L;
    double* F = (double*)malloc(sizeof(double) * (size_t)N);
    if (!F) return -1;
    for (int s = 0; s < n; ++s) {
        orc_hmc_force(L, beta, phi, F);
        for (int i = 0; i < N; ++i) p[i] += 0.5 * eps * F[i];
        for (int i = 0; i < N; ++i) {
            double t = phi[i] + eps * p[i] / (2.0 * HMC_PI);
            phi[i] = t - floor(t);
        }
        orc_hmc_force(L, beta, phi, F);
        for (int i = 0; i < N; ++i) p[i] += 0.5 * eps * F[i];
    }
    free(F);
    return 0;
}

/* One trajectory from phi (in place).  Writes dH = H_new - H_old and, if not
 * NULL, H_old.  Returns 1 if accepted, 0 if rejected (phi restored), -1 if out
 * of memory. */
int orc_hmc_trajectory(uint64_t seed, int L, double beta, double eps, int n, uint32_t traj,
                       double* phi, double* dH_out, double* H_old_out)
{
    const int N = L * L;
    double* p = (double*)malloc(sizeof(double) * (size_t)N);
    double* old = (double*)malloc(sizeof(double) * (size_t)N);
    if (!p || !old) { free(p); free(old); return -1; }
    orc_hmc_momenta(seed, L, traj, p);
    memcpy(old, phi, sizeof(double) * (size_t)N);
    double H0 = orc_hmc_hamiltonian(L, beta, phi, p);
    if (orc_hmc_leapfrog(L, beta, eps, n, phi, p) != 0) { free(p); free(old); return -1; }
    double H1 = orc_hmc_hamiltonian(L, beta, phi, p);
    double dH = H1 - H0;
    int accept = orc_hmc_accept_uniform(seed, traj) < exp(-dH);
    if (!accept) memcpy(phi, old, sizeof(double) * (size_t)N);
    if (dH_out) *dH_out = dH;
    if (H_old_out) *H_old_out = H0;
    free(p);
    free(old);
    return accept;
}

/* n_traj trajectories with indices traj0, traj0 + 1, ...  After trajectory j
 * (1-based) with j % measure_every == 0 a record of 9 doubles is appended:
 * {trajectory count after it, accepted, dH, Cx, Cy, Ix, Iy, Mx, My} of the
 * state after the accept/reject step.  Returns the number of records, or -1. */
int64_t orc_hmc_run(uint64_t seed, int L, double beta, double eps, int n, uint32_t traj0,
                    int64_t n_traj, int64_t measure_every, double* phi, double* rec)
{
    int64_t nrec = 0;
    for (int64_t j = 1; j <= n_traj; ++j) {
        uint32_t t = traj0 + (uint32_t)(j - 1);
        double dH = 0.0;
        int acc = orc_hmc_trajectory(seed, L, beta, eps, n, t, phi, &dH, 0);
        if (acc < 0) return -1;
        if (measure_every > 0 && j % measure_every == 0) {
            double m[6];
            orc_measure(L, phi, m);
            double* r = rec + 9 * nrec;
            r[0] = (double)(t + 1u); r[1] = (double)acc; r[2] = dH;
            for (int q = 0; q < 6; ++q) r[3 + q] = m[q];
            ++nrec;
        }
    }
    return nrec;
}
