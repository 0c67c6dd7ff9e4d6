/*
 * xy_oracle.c -- plain, slow, obviously-correct CPU oracle for checkerboard
 * Metropolis sweeps of the 2-d XY model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP path.
 *
 * What it computes, and where that is defined:
 *   - the model: H = -J sum_<ij> cos(theta_i - theta_j) on a periodic L x L
 *     square lattice, each nearest-neighbour pair counted once (section 1.2,
 *     eq. 1; the paper writes it as -sum sigma_i . sigma_j for unit 2-vectors,
 *     which is the same thing with J = 1);
 *   - the ensemble: Boltzmann weight exp(-beta H);
 *   - the update: single-site Metropolis with the proposal
 *     theta' = theta + delta (2 u1 - 1), accepted iff u2 < exp(-beta dE),
 *     applied to the red sites ((x+y) even) and then the black sites; for an
 *     odd L (tiny test lattices only) plain sequential raster order;
 *   - the random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11), one call per
 *     two same-colour sites, keyed by the seed, counter (sweep, colour,
 *     purpose, pair);
 *   - the observables in FP64: bond sums Cx, Cy (cosines), Ix, Iy (sines)
 *     and the magnetisation sums Mx, My.  The paper keeps global energy sums
 *     off the single-precision device for exactly this reason (section 1.2,
 *     "global sums of the energy"); here they are plain FP64 loops.
 *
 * Angle unit.  A stored angle is phi = theta / (2 pi), in turns, so
 * theta = 2 pi phi; every cosine and sine below is taken of 2 pi times a
 * difference of turns (exact in FP64 for FP32 or FP16 values).  The proposal
 * width delta is given in radians, as in the model, and converted once:
 * Delta = delta / (2 pi).
 *
 * Storage precision.  All arithmetic is FP64.  The stored angles may be kept
 * at FP64, or rounded to the stated storage format of the device path (FP32,
 * or IEEE binary16 with FP32 arithmetic for the proposal).  In the rounded
 * modes the proposal is formed by the exact same sequence of roundings the
 * storage format implies (step = rnd(Delta * r), t = rnd(phi + step), wrap by
 * rnd(t - floor(t)) kept below 1), so a stored state is reproducible bit for
 * bit; energies and decisions stay FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* pi to more digits than FP64 holds; the compiler rounds it once. */
static const double ORC_PI = 3.14159265358979323846264338327950288;

#define ORC_PREC_F64 0
#define ORC_PREC_F32 1
#define ORC_PREC_F16 2

/* ---------------------------------------------------------------------------
 * Philox4x32-10, written from the SC'11 description: each round multiplies
 * words 0 and 2 by the two round multipliers, keeps both halves of the 64-bit
 * products, and mixes the high halves with the other two words and the key;
 * the key is advanced by the two Weyl constants between rounds.
 * ------------------------------------------------------------------------- */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform on the odd grid (2 (w >> 9) + 1) 2^-24: 2^23 values in (0, 1),
 * symmetric about 1/2, exact in FP32 and FP64. */
double orc_u01(uint32_t w)
{
    return ((double)(w >> 9) * 2.0 + 1.0) * 0x1p-24;
}

/* The two 32-bit words a site draws for (sweep, purpose).
 * Even L: colour c = (x+y)&1, half-row index k = x>>1, pairs per half-row
 * P = ceil(L/4); counter (sweep, c, purpose, y*P + (k>>1)); words (X0,X1) for
 * even k, (X2,X3) for odd k.  Odd L: counter (sweep, 0, purpose+2, y*L + x),
 * words (X0,X1). */
void orc_site_words(uint64_t seed, int L, int x, int y, uint32_t sweep,
                    uint32_t purpose, uint32_t w[2])
{
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t ctr[4], r[4];
    if ((L & 1) == 0) {
        uint32_t c = (uint32_t)((x + y) & 1);
        uint32_t k = (uint32_t)(x >> 1);
        uint32_t P = (uint32_t)((L / 2 + 1) / 2);
        ctr[0] = sweep; ctr[1] = c; ctr[2] = purpose;
        ctr[3] = (uint32_t)y * P + (k >> 1);
        orc_philox4x32_10(ctr, key, r);
        if ((k & 1) == 0) { w[0] = r[0]; w[1] = r[1]; }
        else              { w[0] = r[2]; w[1] = r[3]; }
    } else {
        ctr[0] = sweep; ctr[1] = 0; ctr[2] = purpose + 2;
        ctr[3] = (uint32_t)(y * L + x);
        orc_philox4x32_10(ctr, key, r);
        w[0] = r[0]; w[1] = r[1];
    }
}

/* ---------------------------------------------------------------------------
 * Storage rounding.
 * ------------------------------------------------------------------------- */

/* Round to the nearest IEEE binary16 value, ties to even, from the format's
 * definition: 10 fraction bits, normal exponents -14..15, subnormal spacing
 * 2^-24.  Inputs here are finite and far below the overflow threshold. */
double orc_round_f16(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    frexp(fabs(v), &e);            /* |v| = f 2^e, f in [0.5, 1) -> exponent e-1 */
    int exp2 = e - 1;
    if (exp2 < -14) exp2 = -14;    /* subnormal range shares the 2^-24 quantum */
    double quantum = ldexp(1.0, exp2 - 10);
    double q = v / quantum;        /* exact: power-of-two scaling */
    double r = nearbyint(q);       /* default rounding mode: nearest, ties to even */
    return r * quantum;
}

static double round_store(double v, int prec)
{
    if (prec == ORC_PREC_F32) return (double)(float)v;
    if (prec == ORC_PREC_F16) return orc_round_f16((double)(float)v);
    return v;
}

/* Arithmetic rounding of the proposal: FP32 for the FP32 and FP16 storage
 * modes (FP16 storage keeps FP32 arithmetic), none for FP64. */
static double round_arith(double v, int prec)
{
    if (prec == ORC_PREC_F64) return v;
    return (double)(float)v;
}

/* Wrap t (|t| < 2) into [0, 1): t - floor(t) rounded once in the arithmetic
 * format, and a result that rounds up to 1 (t a tiny negative number) replaced
 * by the largest value below 1 of that format. */
static double wrap_turn(double t, int prec)
{
    double r = round_arith(t - floor(t), prec);   /* the difference is exact in FP64 */
    double below_one = (prec == ORC_PREC_F64) ? 1.0 - 0x1p-53 : 1.0 - 0x1p-24;
    return r < 1.0 ? r : below_one;
}

/* Proposal theta' = theta + delta (2 u1 - 1) in turns:
 * phi' = wrap(phi + Delta (2 u1 - 1)), Delta = delta / (2 pi) (delta <= pi, so
 * |phi'| < 1.5 before the wrap). */
double orc_propose(double phi, double delta, double u1, int prec)
{
    double r = 2.0 * u1 - 1.0;                      /* exact */
    double d = delta / (2.0 * ORC_PI);
    if (prec != ORC_PREC_F64) d = (double)(float)d;
    double step = round_arith(d * r, prec);
    double t = round_arith(phi + step, prec);
    return round_store(wrap_turn(t, prec), prec);
}

/* ---------------------------------------------------------------------------
 * Initial states.
 * ------------------------------------------------------------------------- */

/* Hot-start angle of one site (the value orc_hot_start stores there). */
double orc_hot_start_site(uint64_t seed, int L, int x, int y, int prec)
{
    uint32_t w[2];
    orc_site_words(seed, L, x, y, 0u, 1u, w);
    return round_store(orc_u01(w[0]), prec);     /* exact for FP64 and FP32 */
}

/* Hot start: phi = u(X_a), i.e. theta = 2 pi u, from the purpose-1 stream of
 * sweep 0, rounded to the storage format. */
void orc_hot_start(uint64_t seed, int L, int prec, double* phi)
{
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x)
            phi[y * L + x] = orc_hot_start_site(seed, L, x, y, prec);
}

/* ---------------------------------------------------------------------------
 * Observables (FP64, plain loops) of the angles theta = 2 pi phi: bonds
 * (x,y)-(x+1,y) and (x,y)-(x,y+1), periodic, each counted once.
 *   out[0] Cx = sum cos(theta(x,y) - theta(x+1,y))
 *   out[1] Cy = sum cos(theta(x,y) - theta(x,y+1))
 *   out[2] Ix = sum sin(theta(x,y) - theta(x+1,y))
 *   out[3] Iy = sum sin(theta(x,y) - theta(x,y+1))
 *   out[4] Mx = sum cos theta,  out[5] My = sum sin theta
 * E = -J (Cx + Cy).
 * ------------------------------------------------------------------------- */
void orc_measure(int L, const double* phi, double out[6])
{
    double cx = 0, cy = 0, ix = 0, iy = 0, mx = 0, my = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            double t = phi[y * L + x];
            double tr = phi[y * L + (x + 1) % L];
            double td = phi[((y + 1) % L) * L + x];
            cx += cos(2.0 * ORC_PI * (t - tr));
            cy += cos(2.0 * ORC_PI * (t - td));
            ix += sin(2.0 * ORC_PI * (t - tr));
            iy += sin(2.0 * ORC_PI * (t - td));
            mx += cos(2.0 * ORC_PI * t);
            my += sin(2.0 * ORC_PI * t);
        }
    out[0] = cx; out[1] = cy; out[2] = ix; out[3] = iy; out[4] = mx; out[5] = my;
}

double orc_energy(int L, const double* phi)
{
    double m[6];
    orc_measure(L, phi, m);
    return -(m[0] + m[1]);
}

/* ---------------------------------------------------------------------------
 * One Metropolis site update from explicit inputs: the site's angle t_old and
 * its four neighbours nb[] (any order), in turns.  dE = -J sum_nn
 * [cos(theta' - theta_j) - cos(theta - theta_j)]; accept iff u2 < exp(-beta dE).  Writes the angle the
 * site holds afterwards, and optionally dE, the threshold T = -ln(u2)/beta (the
 * decision is dE < T), and the proposal.  Returns 1 if accepted.
 * ------------------------------------------------------------------------- */
int orc_site_update_explicit(uint64_t seed, int L, int x, int y, uint32_t sweep, int prec,
                             double beta, double delta, double t_old, const double nb[4],
                             double* t_out, double* dE_out, double* thr_out, double* prop_out)
{
    uint32_t w[2];
    orc_site_words(seed, L, x, y, sweep, 0u, w);
    double u1 = orc_u01(w[0]);
    double u2 = orc_u01(w[1]);
    double t_new = orc_propose(t_old, delta, u1, prec);
    double dE = 0.0;
    for (int j = 0; j < 4; ++j)
        dE -= cos(2.0 * ORC_PI * (t_new - nb[j])) - cos(2.0 * ORC_PI * (t_old - nb[j]));
    int accept = u2 < exp(-beta * dE);
    if (dE_out) *dE_out = dE;
    if (thr_out) *thr_out = (beta > 0.0) ? -log(u2) / beta : INFINITY;
    if (prop_out) *prop_out = t_new;
    *t_out = accept ? t_new : t_old;
    return accept;
}

static int site_update(uint64_t seed, int L, double beta, double delta, uint32_t sweep,
                       int prec, double* phi, int x, int y,
                       double* dE_out, double* thr_out, uint8_t* dec_out, double* prop_out)
{
    int xl = (x + L - 1) % L, xr = (x + 1) % L;
    int yu = (y + L - 1) % L, yd = (y + 1) % L;
    double nb[4] = { phi[y * L + xl], phi[y * L + xr], phi[yu * L + x], phi[yd * L + x] };
    int accept = orc_site_update_explicit(seed, L, x, y, sweep, prec, beta, delta, phi[y * L + x],
                                          nb, &phi[y * L + x], dE_out, thr_out, prop_out);
    if (dec_out) *dec_out = (uint8_t)accept;
    return accept;
}

/* One sweep.  Even L: every red site ((x+y) even) in raster order, then every
 * black site.  Odd L: every site in raster order.  Updates are applied in
 * place.  Per-site diagnostic arrays (length L*L, natural layout) may be NULL.
 * Returns the number of accepted proposals. */
int64_t orc_sweep(uint64_t seed, int L, double beta, double delta, uint32_t sweep, int prec,
                  double* phi, double* dE, double* thr, uint8_t* dec, double* prop)
{
    int64_t acc = 0;
    int ncol = (L & 1) ? 1 : 2;
    for (int c = 0; c < ncol; ++c)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                if (ncol == 2 && ((x + y) & 1) != c) continue;
                int i = y * L + x;
                acc += site_update(seed, L, beta, delta, sweep, prec, phi, x, y,
                                   dE ? &dE[i] : 0, thr ? &thr[i] : 0,
                                   dec ? &dec[i] : 0, prop ? &prop[i] : 0);
            }
    return acc;
}

/* n_sweeps sweeps starting at sweep index sweep0.  After relative sweep j
 * (1-based) with j % measure_every == 0, a record of 8 doubles is appended:
 * {absolute sweep count after the sweep, accepts in that sweep,
 *  Cx, Cy, Ix, Iy, Mx, My}.  Returns the number of records written. */
int64_t orc_run(uint64_t seed, int L, double beta, double delta, uint32_t sweep0,
                int64_t n_sweeps, int64_t measure_every, int prec, double* phi, double* rec)
{
    int64_t nrec = 0;
    for (int64_t j = 1; j <= n_sweeps; ++j) {
        uint32_t s = sweep0 + (uint32_t)(j - 1);
        int64_t acc = orc_sweep(seed, L, beta, delta, s, prec, phi, 0, 0, 0, 0);
        if (measure_every > 0 && j % measure_every == 0) {
            double m[6];
            orc_measure(L, phi, m);
            double* r = rec + 8 * nrec;
            r[0] = (double)(s + 1u); r[1] = (double)acc;
            for (int q = 0; q < 6; ++q) r[2 + q] = m[q];
            ++nrec;
        }
    }
    return nrec;
}

/* ---------------------------------------------------------------------------
 * q-state clock restriction: theta = 2 pi k / q, i.e. phi = k / q turns.  The proposal moves to one
 * of the q-1 other states uniformly, k' = (k + 1 + floor(u1 (q-1))) mod q,
 * which is symmetric; acceptance as above.  Same sweep order and streams.
 * ------------------------------------------------------------------------- */
static double clock_angle(int k, int q) { return (double)k / (double)q; }

int64_t orc_clock_sweep(uint64_t seed, int L, int q, double beta, uint32_t sweep, int32_t* ks)
{
    int64_t acc = 0;
    int ncol = (L & 1) ? 1 : 2;
    for (int c = 0; c < ncol; ++c)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                if (ncol == 2 && ((x + y) & 1) != c) continue;
                uint32_t w[2];
                orc_site_words(seed, L, x, y, sweep, 0u, w);
                double u1 = orc_u01(w[0]), u2 = orc_u01(w[1]);
                int k = ks[y * L + x];
                int kn = (k + 1 + (int)floor(u1 * (double)(q - 1))) % q;
                int xl = (x + L - 1) % L, xr = (x + 1) % L;
                int yu = (y + L - 1) % L, yd = (y + 1) % L;
                int nb[4] = { ks[y * L + xl], ks[y * L + xr], ks[yu * L + x], ks[yd * L + x] };
                double dE = 0.0;
                for (int j = 0; j < 4; ++j)
                    dE -= cos(2.0 * ORC_PI * (clock_angle(kn, q) - clock_angle(nb[j], q)))
                        - cos(2.0 * ORC_PI * (clock_angle(k, q) - clock_angle(nb[j], q)));
                if (u2 < exp(-beta * dE)) { ks[y * L + x] = kn; ++acc; }
            }
    return acc;
}

int64_t orc_clock_run(uint64_t seed, int L, int q, double beta, uint32_t sweep0,
                      int64_t n_sweeps, int64_t measure_every, int32_t* ks, double* rec)
{
    int64_t nrec = 0;
    double* th = (double*)malloc(sizeof(double) * (size_t)L * (size_t)L);
    if (!th) return -1;
    for (int64_t j = 1; j <= n_sweeps; ++j) {
        uint32_t s = sweep0 + (uint32_t)(j - 1);
        int64_t acc = orc_clock_sweep(seed, L, q, beta, s, ks);
        if (measure_every > 0 && j % measure_every == 0) {
            for (int i = 0; i < L * L; ++i) th[i] = clock_angle(ks[i], q);
            double m[6];
            orc_measure(L, th, m);
            double* r = rec + 8 * nrec;
            r[0] = (double)(s + 1u); r[1] = (double)acc;
            for (int p = 0; p < 6; ++p) r[2 + p] = m[p];
            ++nrec;
        }
    }
    free(th);
    return nrec;
}
