/*
 * xy_pt_oracle.c -- plain FP64 CPU oracle for parallel tempering of checkerboard
 * Metropolis lattices.
 *
 * TEST INFRASTRUCTURE ONLY, like xy_oracle.c (same library and rules).
 *
 * Section 3.2 keeps replicas of a lattice at different temperatures side by
 * side; parallel tempering lets them exchange temperatures.  One ladder of M
 * lattices of the same L: rung t (0 .. M-1) has (beta_t, delta_t); member[t] is
 * the lattice on rung t (initially lattice t).  Every round:
 *   1. every lattice i runs K Metropolis sweeps (xy_oracle.c, its own seed,
 *      sweep indices s0 .. s0+K-1, shared by all lattices) at the (beta, delta)
 *      of its rung, and its energy E_i = -(Cx + Cy) is measured after them;
 *   2. for the rungs t = p, p + 2, ... with t + 1 < M, p = round parity, the
 *      lattices a = member[t], b = member[t+1] exchange rungs iff
 *      u < exp((beta_t - beta_{t+1}) (E_a - E_b)), the standard tempering
 *      acceptance (the ratio of the two product Boltzmann weights), with u =
 *      u(X0) of Philox counter (round, ladder, 4, t), key = the tempering seed.
 * Angles are stored in the FP32 storage mode (as the device does), energies FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t w);
int64_t orc_run(uint64_t seed, int L, double beta, double delta, uint32_t sweep0, int64_t n_sweeps,
                int64_t measure_every, int prec, double* phi, double* rec);

#define PT_PURPOSE 4u

double orc_pt_uniform(uint64_t pt_seed, uint32_t round, uint32_t ladder, uint32_t rung)
{
    uint32_t key[2] = { (uint32_t)(pt_seed & 0xffffffffu), (uint32_t)(pt_seed >> 32) };
    uint32_t ctr[4] = { round, ladder, PT_PURPOSE, rung }, r[4];
    orc_philox4x32_10(ctr, key, r);
    return orc_u01(r[0]);
}

/* n_rounds rounds for a ladder of M lattices.  seeds[i], phi + i L^2: lattice i;
 * beta[t], delta[t]: rung t; member[t]: lattice on rung t (updated in place);
 * round0, sweep0: indices of the first round and sweep.  Per round r (local),
 * rec[(r * M + i) * 9 ..] = {round, sweep count after, accepts, Cx, Cy, Ix, Iy,
 * Mx, My} of lattice i, and rung_out[r * M + i] = its rung during the round.
 * Returns 0, or -1 if out of memory. */
int orc_pt_run(const uint64_t* seeds, int M, int L, const double* beta, const double* delta, int32_t* member,
               uint64_t pt_seed, uint32_t ladder, uint32_t round0, uint32_t sweep0, int64_t n_rounds, int K,
               int prec, double* phi, double* rec, int32_t* rung_out)
{
    int32_t* rung = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
    double* r8 = (double*)malloc(sizeof(double) * 8 * (size_t)(K > 0 ? 1 : 1));
    double* E = (double*)malloc(sizeof(double) * (size_t)M);
    if (!rung || !r8 || !E) { free(rung); free(r8); free(E); return -1; }
    for (int64_t r = 0; r < n_rounds; ++r) {
        for (int t = 0; t < M; ++t) rung[member[t]] = t;
        uint32_t s0 = sweep0 + (uint32_t)(r * K);
        for (int i = 0; i < M; ++i) {
            double* ph = phi + (size_t)i * (size_t)L * (size_t)L;
            orc_run(seeds[i], L, beta[rung[i]], delta[rung[i]], s0, K, K, prec, ph, r8);
            double* o = rec + ((size_t)r * M + i) * 9;
            o[0] = (double)(round0 + (uint32_t)r);
            for (int q = 0; q < 8; ++q) o[1 + q] = r8[q];
            E[i] = -(r8[2] + r8[3]);
            rung_out[r * M + i] = rung[i];
        }
        uint32_t round = round0 + (uint32_t)r;
        for (int t = (int)(round & 1u); t + 1 < M; t += 2) {
            int a = member[t], b = member[t + 1];
            double u = orc_pt_uniform(pt_seed, round, ladder, (uint32_t)t);
            if (u < exp((beta[t] - beta[t + 1]) * (E[a] - E[b]))) {
                member[t] = b;
                member[t + 1] = a;
            }
        }
    }
    free(rung);
    free(r8);
    free(E);
    return 0;
}
