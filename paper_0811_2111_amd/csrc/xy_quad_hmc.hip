// xy_quad_hmc.hip -- hybrid Monte Carlo (section 1.2) on the four-replica texel
// (section 3.2): the four replicas of a float4 state run their leap-frog
// trajectories together, each pass over the state advancing all four, and the
// Metropolis step is a vector of four decisions z_r, one per replica from its own FP64 dH;
// replica r then keeps z_r theta_new + (1 - z_r) theta_old.
//
// Replica r follows bit for bit the trajectory of a single lattice with seed_r,
// beta_r and the same eps and step count (xy_hmc): every per-site quantity is
// formed by the single-lattice arithmetic (xy_hmc_site.hpp) from the replica's
// own component, with the replica's key for its random numbers.  Only the
// order of the FP64 sums of H differs, so dH agrees to rounding.
//
// The angles ping-pong between the state and the quad's second buffer: one
// leap-frog step per launch (momenta updated in place), or passes of up to four
// steps on 32 x 32 tiles grown by the step count (momenta ping-pong too).
#include <hip/hip_runtime.h>

#include "xy_device.hpp"
#include "xy_hmc_site.hpp"
#include "xy_launch.hpp"
#include "xy_reduce.hpp"
#include "xy_tile4.hpp"

using namespace xyd;
using namespace xyd::hmc;

namespace xyk {

namespace {

constexpr int kQThreads = 256;

__device__ __forceinline__ int qwrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// The four replicas' angles of entry (c, y, k) and of its four neighbours in the
// other plane (the single-lattice neighbour rule, entries of 16 bytes).
struct Nb4 {
    float4 t, l, r, u, d;
};

__device__ __forceinline__ Nb4 load_nb4(const float4* __restrict__ st, int L, int Hh, int c, int y, int k)
{
    const int o = (c + y) & 1;
    const float4* oth = st + (size_t)(1 - c) * L * Hh;
    Nb4 n;
    n.t = st[((size_t)c * L + y) * Hh + k];
    n.l = oth[(size_t)y * Hh + qwrap(k + o - 1, Hh)];
    n.r = oth[(size_t)y * Hh + qwrap(k + o, Hh)];
    n.u = oth[(size_t)qwrap(y - 1, L) * Hh + k];
    n.d = oth[(size_t)qwrap(y + 1, L) * Hh + k];
    return n;
}

// Replica r's (cos, sin) of the entry and of its neighbours.
__device__ __forceinline__ Nb replica_nb(const Nb4& a, int r)
{
    Nb n;
    sincos_turn(f4c(a.t, r), n.s, n.c);
    sincos_turn(f4c(a.l, r), n.sl, n.cl);
    sincos_turn(f4c(a.r, r), n.sr, n.cr);
    sincos_turn(f4c(a.u, r), n.su, n.cu);
    sincos_turn(f4c(a.d, r), n.sd, n.cd);
    return n;
}

// A site's terms of H (as the single-lattice records): a black site adds its four
// bonds, its own spin and that of the red site to its right; every site adds p^2/2.
__device__ __forceinline__ void add_site(double v[7], const Nb& n, int c, float kin)
{
    if (c == 1) {
        Meas m{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        meas_black(m, n.c, n.s, n.cl, n.sl, n.cr, n.sr, n.cu, n.su, n.cd, n.sd);
        v[0] += (double)m.cx; v[1] += (double)m.cy; v[2] += (double)m.ix;
        v[3] += (double)m.iy; v[4] += (double)m.mx; v[5] += (double)m.my;
    }
    v[6] += (double)kin;
}

// One partial record per wave and replica: replica r's record of wave w of block
// b at rec[(r nrec + b 4 + w) 8].
__device__ __forceinline__ void write_records(double v[4][7], double* __restrict__ rec, int nrec, unsigned b)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int q = 0; q < 7; ++q) v[r][q] = wave_sum_last(v[r][q]);
        if ((threadIdx.x & 63) == 63) {
            double* o = rec + ((size_t)r * nrec + (size_t)b * (kQThreads / 64) + (threadIdx.x >> 6)) * 8;
#pragma unroll
            for (int q = 0; q < 7; ++q) o[q] = v[r][q];
            o[7] = 0.0;
        }
    }
}

// Grid of the record-writing trajectory ends: cols x rb workgroups, cols =
// 2 ceil(Hh/256), each writing one partial record per wave and replica.
struct QGrid {
    int cols, rb;
};

// One leap-frog step of every replica: p += kick_r F, then a drift of
// eps/(2 pi) p turns.  Grid (2 ceil(Hh/256), L).
__global__ void __launch_bounds__(kQThreads)
k_qhmc_step(const float4* __restrict__ src, float4* __restrict__ dst, float4* __restrict__ p, int L, float4 kick,
            float drift)
{
    const int Hh = L >> 1;
    const int k = (blockIdx.x >> 1) * kQThreads + threadIdx.x;
    if (k >= Hh) return;
    const int y = blockIdx.y, c = blockIdx.x & 1;
    const Nb4 a = load_nb4(src, L, Hh, c, y, k);
    const size_t i = ((size_t)c * L + y) * Hh + k;
    float4 pv = p[i], th;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float pn = __fmaf_rn(f4c(kick, r), sin_sum(replica_nb(a, r)), f4c(pv, r));
        f4set(pv, r, pn);
        f4set(th, r, __builtin_amdgcn_fractf(__fmaf_rn(drift, pn, f4c(a.t, r))));
    }
    p[i] = pv;
    dst[i] = th;
}

// K leap-frog steps per pass (temporal blocking, as the single lattice's passes):
// a workgroup owns a 32 x 32 tile of sites (natural coordinates) and loads the
// float4 angles and momenta of the tile grown by K sites on every side into
// registers; step q updates the sites more than q from the edge of the grown
// tile; the tile itself is then exact and is written to dst / pdst (the momenta
// ping-pong too, since other tiles read this tile's old momenta as their halo).
// The four replicas' (cos, sin) sit in one LDS buffer (32 bytes a site): every
// update of a step reads its neighbours, barrier, the new values are written,
// barrier.  Per replica and site the arithmetic is that of k_qhmc_step.
constexpr int kQTile = 32;
constexpr int kQMaxSteps = 4;

__device__ __forceinline__ unsigned qxcd_band(unsigned b, unsigned nb)
{
    if ((nb & 7u) != 0u) return b;
    return (b & 7u) * (nb >> 3) + (b >> 3);
}

template <int K>
__global__ void __launch_bounds__(kQThreads)
k_qhmc_multi(const float4* __restrict__ src, float4* __restrict__ dst, const float4* __restrict__ psrc,
             float4* __restrict__ pdst, int L, float4 kick0, float4 kick, float drift)
{
    constexpr int T = kQTile, E = T + 2 * K, NE = E * E, M = (NE + kQThreads - 1) / kQThreads;
    __shared__ float4 cs[2 * NE];          // site i: cos at 2i, sin at 2i + 1
    const int Hh = L >> 1, nt = L / T;
    const int b = (int)qxcd_band(blockIdx.x, gridDim.x);
    const int ty = b / nt, tx = b - ty * nt;
    const int x0 = tx * T - K, y0 = ty * T - K;
    float4 th[M], pm[M];
    unsigned off[M];
    int dep[M];       // distance of the slot's site from the grown tile's edge (-1: no site)
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = threadIdx.x + m * kQThreads;
        dep[m] = -1;
        if (i < NE) {
            const int ye = i / E, xe = i - ye * E;
            dep[m] = min(min(xe, E - 1 - xe), min(ye, E - 1 - ye));
            const int x = qwrap(x0 + xe, L), y = qwrap(y0 + ye, L);
            off[m] = (unsigned)((((x + y) & 1) * L + y) * Hh + (x >> 1));
            th[m] = src[off[m]];
            pm[m] = psrc[off[m]];
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = threadIdx.x + m * kQThreads;
        if (i < NE) {
            float4 c4, s4;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float sn, cn;
                sincos_turn(f4c(th[m], r), sn, cn);
                f4set(c4, r, cn);
                f4set(s4, r, sn);
            }
            cs[2 * i] = c4;
            cs[2 * i + 1] = s4;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const float4 kq = q == 0 ? kick0 : kick;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int i = threadIdx.x + m * kQThreads;
            if (dep[m] > q) {
                const float4 oc = cs[2 * i], os = cs[2 * i + 1];
                const float4 lc = cs[2 * (i - 1)], ls = cs[2 * (i - 1) + 1];
                const float4 rc = cs[2 * (i + 1)], rs = cs[2 * (i + 1) + 1];
                const float4 uc = cs[2 * (i - E)], us = cs[2 * (i - E) + 1];
                const float4 dc = cs[2 * (i + E)], ds = cs[2 * (i + E) + 1];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    Nb n;
                    n.c = f4c(oc, r); n.s = f4c(os, r);
                    n.cl = f4c(lc, r); n.sl = f4c(ls, r); n.cr = f4c(rc, r); n.sr = f4c(rs, r);
                    n.cu = f4c(uc, r); n.su = f4c(us, r); n.cd = f4c(dc, r); n.sd = f4c(ds, r);
                    const float pn = __fmaf_rn(f4c(kq, r), sin_sum(n), f4c(pm[m], r));
                    f4set(pm[m], r, pn);
                    f4set(th[m], r, __builtin_amdgcn_fractf(__fmaf_rn(drift, pn, f4c(th[m], r))));
                }
            }
        }
        if (q + 1 < K) {
            __syncthreads();          // every read of this step is done
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int i = threadIdx.x + m * kQThreads;
                if (dep[m] > q) {
                    float4 c4, s4;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float sn, cn;
                        sincos_turn(f4c(th[m], r), sn, cn);
                        f4set(c4, r, cn);
                        f4set(s4, r, sn);
                    }
                    cs[2 * i] = c4;
                    cs[2 * i + 1] = s4;
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (dep[m] >= K) {           // the tile itself
            dst[off[m]] = th[m];
            pdst[off[m]] = pm[m];
        }
    }
}

template <int K>
static void launch_qmulti(unsigned nb, hipStream_t s, const float4* src, float4* dst, const float4* psrc,
                          float4* pdst, int L, float4 kick0, float4 kick, float drift)
{
    hipLaunchKernelGGL(k_qhmc_multi<K>, dim3(nb), dim3(kQThreads), 0, s, src, dst, psrc, pdst, L, kick0, kick, drift);
}

// The trajectory ends by runs of rows.  A thread takes entry k of both planes
// down a run of consecutive rows: each plane's entries of the rows above, at and
// below sit in registers with the four replicas' (cos, sin), and each row adds
// one edge entry of each plane (k - 1 or k + 1, the side the other plane's site
// needs), so a float4 is read once as its own entry and once as an edge, and a
// replica site costs two sines and cosines (a thread per site reading its four
// neighbours costs five, and took 243 and 212 us at L = 4096 where these take
// 198 and 164).  BEGIN: momenta (Box-Muller of each replica's Philox purpose-2
// words, as the single lattice's), saved angles, partial records of H_old; else
// the final half kick and the records of H_new, and `copy` != NULL receives the
// angles (the final ones may sit in the second buffer).  Block b of the record
// grid (QGrid) takes column block b % (cols / 2) of both planes and run
// b / (cols / 2) of 2 rb runs of rows.
struct CS4 {
    float c[4], s[4];
};
__device__ __forceinline__ CS4 cs4(float4 t)
{
    CS4 q;
#pragma unroll
    for (int r = 0; r < 4; ++r) sincos_turn(f4c(t, r), q.s[r], q.c[r]);
    return q;
}
__device__ __forceinline__ Nb nb_of(const CS4& own, const CS4& l, const CS4& rt, const CS4& u, const CS4& d, int r)
{
    Nb n;
    n.c = own.c[r]; n.s = own.s[r];
    n.cl = l.c[r]; n.sl = l.s[r];
    n.cr = rt.c[r]; n.sr = rt.s[r];
    n.cu = u.c[r]; n.su = u.s[r];
    n.cd = d.c[r]; n.sd = d.s[r];
    return n;
}

template <bool BEGIN>
__global__ void __launch_bounds__(kQThreads)
k_qhmc_ends(const float4* __restrict__ st, float4* __restrict__ p, float4* __restrict__ copy, int L, uint32_t traj,
            QHmcKeys keys, float4 kick, QGrid g, double* __restrict__ rec, int nrec)
{
    const int Hh = L >> 1, P = (Hh + 1) >> 1;
    const unsigned b = blockIdx.x;
    const int cols2 = g.cols >> 1, runs = 2 * g.rb;
    const int k = (int)(b % (unsigned)cols2) * kQThreads + (int)threadIdx.x;
    const int run = (int)(b / (unsigned)cols2);
    double v[4][7] = {};
    const int R = (L + runs - 1) / runs, y0 = run * R, y1 = y0 + R < L ? y0 + R : L;
    if (k < Hh && y0 < y1) {
        const float4* pl0 = st;
        const float4* pl1 = st + (size_t)L * Hh;
        float4 t0 = pl0[(size_t)y0 * Hh + k], t1 = pl1[(size_t)y0 * Hh + k];
        const int ym = qwrap(y0 - 1, L);
        CS4 u0 = cs4(pl0[(size_t)ym * Hh + k]), u1 = cs4(pl1[(size_t)ym * Hh + k]);
        CS4 h0 = cs4(t0), h1 = cs4(t1);
        const int km = qwrap(k - 1, Hh), kp = qwrap(k + 1, Hh);
        for (int y = y0; y < y1; ++y) {
            const int yd = qwrap(y + 1, L);
            const float4 n0 = pl0[(size_t)yd * Hh + k], n1 = pl1[(size_t)yd * Hh + k];
            // plane 0's site has o = y & 1 (neighbours in plane 1 at k + o - 1 and
            // k + o), plane 1's the other parity: each needs one edge entry
            const int o = y & 1;
            const CS4 e1 = cs4(pl1[(size_t)y * Hh + (o ? kp : km)]);
            const CS4 e0 = cs4(pl0[(size_t)y * Hh + (o ? km : kp)]);
            const CS4 d0 = cs4(n0), d1 = cs4(n1);
            const size_t i0 = (size_t)y * Hh + k, i1 = ((size_t)L + y) * Hh + k;
            if (BEGIN || copy) {
                copy[i0] = t0;
                copy[i1] = t1;
            }
            float4 pv0 = make_float4(0.f, 0.f, 0.f, 0.f), pv1 = pv0, pm0, pm1;
            if constexpr (!BEGIN) {
                pv0 = p[i0];
                pv1 = p[i1];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const Nb na = nb_of(h0, o ? h1 : e1, o ? e1 : h1, u1, d1, r);
                const Nb nb = nb_of(h1, o ? e0 : h0, o ? h0 : e0, u0, d0, r);
                float pa, pb;
                if constexpr (BEGIN) {
                    const uint32_t j = (uint32_t)y * (uint32_t)P + (uint32_t)(k >> 1);
                    const u32x4 wa = philox10(traj, 0u, 2u, j, keys.k0[r], keys.k1[r]);
                    const u32x4 wb = philox10(traj, 1u, 2u, j, keys.k0[r], keys.k1[r]);
                    pa = (k & 1) ? box_muller(wa.z, wa.w) : box_muller(wa.x, wa.y);
                    pb = (k & 1) ? box_muller(wb.z, wb.w) : box_muller(wb.x, wb.y);
                } else {
                    pa = __fmaf_rn(f4c(kick, r), sin_sum(na), f4c(pv0, r));
                    pb = __fmaf_rn(f4c(kick, r), sin_sum(nb), f4c(pv1, r));
                }
                f4set(pm0, r, pa);
                f4set(pm1, r, pb);
                add_site(v[r], na, 0, __fmul_rn(0.5f, __fmul_rn(pa, pa)));
                add_site(v[r], nb, 1, __fmul_rn(0.5f, __fmul_rn(pb, pb)));
            }
            if constexpr (BEGIN) {
                p[i0] = pm0;
                p[i1] = pm1;
            }
            u0 = h0; u1 = h1;
            h0 = d0; h1 = d1;
            t0 = n0; t1 = n1;
        }
    }
    write_records(v, rec, nrec, b);       // every lane reaches the wave sums
}

// The vector Metropolis step: workgroup r sums replica r's chunk records of
// H_old and H_new in a fixed order (thread t: chunks t, t + 256, ..., then the
// workgroup sum) and takes its decision (flag[r], obs[r]).
__global__ void __launch_bounds__(kQThreads)
k_qhmc_decide(const double* __restrict__ chunk_old, const double* __restrict__ chunk_new, int nchunk, QHmcBeta beta,
              uint32_t traj, QHmcKeys keys, unsigned* __restrict__ flag, xy_hmc_obs* __restrict__ obs)
{
    __shared__ double red[4 * 7];
    const int r = (int)blockIdx.x;
    double o[7] = {}, n[7] = {};
    const double* co = chunk_old + (size_t)r * nchunk * 8;
    const double* cn = chunk_new + (size_t)r * nchunk * 8;
    for (int j = threadIdx.x; j < nchunk; j += kQThreads)
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            o[q] += co[(size_t)j * 8 + q];
            n[q] += cn[(size_t)j * 8 + q];
        }
    block_sum7_256(o, red);
    __syncthreads();                      // red is reused
    block_sum7_256(n, red);
    if (threadIdx.x == 0) decide_core(o, n, beta.b[r], traj, keys.k0[r], keys.k1[r], flag + r, obs ? obs + r : nullptr);
}

// Rejected replicas: their components of the saved angles back into the state.
__global__ void __launch_bounds__(kQThreads)
k_qhmc_restore(const unsigned* __restrict__ flag, const float4* __restrict__ saved, float4* __restrict__ st, size_t n)
{
    const unsigned z0 = flag[0], z1 = flag[1], z2 = flag[2], z3 = flag[3];
    if (z0 & z1 & z2 & z3) return;
    for (size_t i = (size_t)blockIdx.x * kQThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kQThreads) {
        const float4 a = st[i], s = saved[i];
        st[i] = make_float4(z0 ? a.x : s.x, z1 ? a.y : s.y, z2 ? a.z : s.z, z3 ? a.w : s.w);
    }
}

QGrid qgrid(int L)
{
    QGrid g;
    g.cols = 2 * (((L >> 1) + kQThreads - 1) / kQThreads);
    const int rb = 4096 / g.cols;
    g.rb = rb < L ? (rb > 0 ? rb : 1) : L;
    return g;
}

}  // namespace

int quad_hmc_records(int L)
{
    const QGrid g = qgrid(L);
    return g.cols * g.rb * (kQThreads / 64);
}

size_t quad_hmc_work_bytes(int L)
{
    const size_t st = ((size_t)L * L * sizeof(float4) + 255) & ~(size_t)255;
    const size_t nrec = (size_t)quad_hmc_records(L), nch = (nrec + 255) / 256;
    return 3 * st + 256 + 2 * 4 * (nrec + nch) * 8 * sizeof(double);
}

QuadHmcWork quad_hmc_carve(void* work, int L)
{
    const size_t st = ((size_t)L * L * sizeof(float4) + 255) & ~(size_t)255;
    const size_t nrec = (size_t)quad_hmc_records(L), nch = (nrec + 255) / 256;
    char* b = (char*)work;
    QuadHmcWork w;
    w.p = (float4*)b;
    b += st;
    w.saved = (float4*)b;
    b += st;
    w.p2 = (float4*)b;
    b += st;
    w.flag = (unsigned*)b;
    b += 256;
    w.rec_old = (double*)b;
    b += 4 * nrec * 8 * sizeof(double);
    w.rec_new = (double*)b;
    b += 4 * nrec * 8 * sizeof(double);
    w.chunk_old = (double*)b;
    b += 4 * nch * 8 * sizeof(double);
    w.chunk_new = (double*)b;
    return w;
}

hipError_t launch_quad_hmc_trajectory(float4* state, float4* pingpong, const QuadHmcWork& w, int L,
                                      const double beta[4], double eps, int n_md, int steps_per_pass, uint32_t traj,
                                      const QHmcKeys& keys, xy_hmc_obs* obs, hipStream_t s)
{
    const QGrid g = qgrid(L);
    const int nrec = quad_hmc_records(L), nchunk = (nrec + 255) / 256;
    const dim3 grec((unsigned)(g.cols * g.rb)), gstep((unsigned)g.cols, (unsigned)L), block(kQThreads);
    // the single-lattice launcher's FP32 constants, per replica
    const float drift = (float)(eps / (2.0 * 3.14159265358979323846));
    float kh[4], kf[4];
    QHmcBeta qb;
    for (int r = 0; r < 4; ++r) {
        kh[r] = (float)(-beta[r] * 0.5 * eps);
        kf[r] = (float)(-beta[r] * eps);
        qb.b[r] = beta[r];
    }
    const float4 kick_half = make_float4(kh[0], kh[1], kh[2], kh[3]);
    const float4 kick_full = make_float4(kf[0], kf[1], kf[2], kf[3]);
    hipLaunchKernelGGL(k_qhmc_ends<true>, grec, block, 0, s, state, w.p, w.saved, L, traj, keys, kick_half, g,
                       w.rec_old, nrec);
    float4* src = state;
    float4* dst = pingpong;
    float4* p = w.p;
    if (steps_per_pass > 1) {
        // passes of up to min(steps_per_pass, kQMaxSteps) steps; the momenta ping-pong between p and p2
        float4* pn = w.p2;
        const unsigned nb = (unsigned)((L / kQTile) * (L / kQTile));
        const int kmax = steps_per_pass < kQMaxSteps ? steps_per_pass : kQMaxSteps;
        for (int q = 0; q < n_md;) {
            const int k = n_md - q < kmax ? n_md - q : kmax;
            const float4 k0 = q == 0 ? kick_half : kick_full;
            switch (k) {
            case 1: launch_qmulti<1>(nb, s, src, dst, p, pn, L, k0, kick_full, drift); break;
            case 2: launch_qmulti<2>(nb, s, src, dst, p, pn, L, k0, kick_full, drift); break;
            case 3: launch_qmulti<3>(nb, s, src, dst, p, pn, L, k0, kick_full, drift); break;
            default: launch_qmulti<4>(nb, s, src, dst, p, pn, L, k0, kick_full, drift); break;
            }
            float4* t = src;
            src = dst;
            dst = t;
            t = p;
            p = pn;
            pn = t;
            q += k;
        }
    } else {
        for (int q = 0; q < n_md; ++q) {
            hipLaunchKernelGGL(k_qhmc_step, gstep, block, 0, s, src, dst, p, L, q == 0 ? kick_half : kick_full,
                               drift);
            float4* t = src;
            src = dst;
            dst = t;
        }
    }
    hipLaunchKernelGGL(k_qhmc_ends<false>, grec, block, 0, s, src, p, src == state ? nullptr : state, L, traj, keys,
                       kick_half, g, w.rec_new, nrec);
    hipError_t e = hipGetLastError();
    for (int r = 0; r < 4 && e == hipSuccess; ++r) {
        e = launch_reduce_chunks(w.rec_old + (size_t)r * nrec * 8, nrec, w.chunk_old + (size_t)r * nchunk * 8, s);
        if (e == hipSuccess)
            e = launch_reduce_chunks(w.rec_new + (size_t)r * nrec * 8, nrec, w.chunk_new + (size_t)r * nchunk * 8, s);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qhmc_decide, dim3(4), block, 0, s, w.chunk_old, w.chunk_new, nchunk, qb, traj, keys, w.flag,
                       obs);
    const size_t n = (size_t)L * (size_t)L;
    const unsigned nb = (unsigned)((n + kQThreads * 8 - 1) / (kQThreads * 8));
    hipLaunchKernelGGL(k_qhmc_restore, dim3(nb < 4096 ? nb : 4096), block, 0, s, w.flag, w.saved, state, n);
    return hipGetLastError();
}

}  // namespace xyk
