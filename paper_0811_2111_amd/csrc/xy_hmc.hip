// xy_hmc.hip -- hybrid Monte Carlo trajectories (section 1.2): Gaussian momenta,
// leap-frog integration of the equations of motion, Metropolis step on FP64
// global sums of H = sum p^2/2 + beta E, all on the device.
//
// Angles are in turns (phi = theta / 2 pi), momenta in radians per unit time,
// both FP32 in the half-lattice layout of the state.  With
//     F_i = -beta sum_{j nn i} sin(theta_i - theta_j)
//         = -beta (s_i sum_j c_j - c_i sum_j s_j),   (c, s) = (cos, sin) theta,
// one trajectory of n leap-frog steps of size eps is
//     begin : p = Box-Muller(Philox), saved = phi, H_old partials;
//     step 1: p += eps/2 F(phi), phi += eps/(2 pi) p     (kick, then drift)
//     step k: p += eps   F(phi), phi += eps/(2 pi) p     (k = 2 .. n; two half
//             kicks of neighbouring steps merged)
//     end   : p += eps/2 F(phi), H_new partials;
//     decide: dH = H_new - H_old (FP64), accept iff u < exp(-dH);
//     restore phi = saved if rejected.
// A step is a Jacobi update (every site from the same old angles), so the
// angles ping-pong between the state and a second buffer; momenta are local and
// are updated in place.
#include <hip/hip_runtime.h>

#include "xy_device.hpp"
#include "xy_hmc_site.hpp"
#include "xy_launch.hpp"
#include "xy_reduce.hpp"

using namespace xyd;
using namespace xyd::hmc;

namespace xyk {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// The angle of entry (c, y, k) and the (cos, sin) of it and of its four
// neighbours in the other plane.
__device__ __forceinline__ Nb load_nb(const float* __restrict__ st, int L, int Hh, int c, int y, int k, float& th)
{
    const int o = (c + y) & 1;
    const float* oth = st + (size_t)(1 - c) * L * Hh;
    th = st[((size_t)c * L + y) * Hh + k];
    const float tl = oth[(size_t)y * Hh + wrapi(k + o - 1, Hh)];
    const float tr = oth[(size_t)y * Hh + wrapi(k + o, Hh)];
    const float tu = oth[(size_t)wrapi(y - 1, L) * Hh + k];
    const float td = oth[(size_t)wrapi(y + 1, L) * Hh + k];
    Nb n;
    sincos_turn(th, n.s, n.c);
    sincos_turn(tl, n.sl, n.cl);
    sincos_turn(tr, n.sr, n.cr);
    sincos_turn(tu, n.su, n.cu);
    sincos_turn(td, n.sd, n.cd);
    return n;
}

// One partial record per wave: (Cx, Cy, Ix, Iy, Mx, My, K, 0).  Black sites add
// their four bonds, their own spin and that of the red site to their right (as
// the Metropolis measurement does); every site adds p^2 / 2.
__device__ __forceinline__ void write_record(double v[7], double* __restrict__ rec, unsigned b)
{
#pragma unroll
    for (int q = 0; q < 7; ++q) v[q] = wave_sum_last(v[q]);
    if ((threadIdx.x & 63) == 63) {
        double* r = rec + ((size_t)b * (kThreads / 64) + (threadIdx.x >> 6)) * 8;
#pragma unroll
        for (int q = 0; q < 7; ++q) r[q] = v[q];
        r[7] = 0.0;
    }
}

__device__ __forceinline__ void accumulate(double v[7], const Nb& n, int c, float kin)
{
    if (c == 1) {
        Meas m{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        meas_black(m, n.c, n.s, n.cl, n.sl, n.cr, n.sr, n.cu, n.su, n.cd, n.sd);
        v[0] += (double)m.cx; v[1] += (double)m.cy; v[2] += (double)m.ix;
        v[3] += (double)m.iy; v[4] += (double)m.mx; v[5] += (double)m.my;
    }
    v[6] += (double)kin;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8);
// this remap gives each XCD one contiguous band of rows (both colours), so the
// neighbour rows a block reads from the other plane are hits in that XCD's L2.
__device__ __forceinline__ unsigned xcd_band(unsigned b, unsigned nb)
{
    if ((nb & 7u) != 0u) return b;
    return (b & 7u) * (nb >> 3) + (b >> 3);
}

// Record-writing passes: 1-D grid of cols x rb workgroups, cols = 2 ceil(Hh/256)
// (column block, colour interleaved), rb row blocks; after the XCD remap t,
// column t % cols takes the run of R = ceil(L / rb) consecutive rows starting at
// (t / cols) R, so the rows above and the row itself that a thread needs from
// the other plane were loaded in its previous iteration.  Record index: t.

// Momenta, saved angles and the partial records of H_old.
__global__ void __launch_bounds__(kThreads)
k_hmc_begin(const float* __restrict__ st, float* __restrict__ p, float* __restrict__ saved, int L, uint32_t traj,
            const uint32_t* __restrict__ traj_dev, uint32_t k0, uint32_t k1, int cols, int rb,
            double* __restrict__ rec)
{
    if (traj_dev) traj = *traj_dev;
    const int Hh = L >> 1, P = (Hh + 1) >> 1;
    const unsigned t = xcd_band(blockIdx.x, gridDim.x);
    const int col = (int)(t % (unsigned)cols);
    const int k = (col >> 1) * kThreads + threadIdx.x;
    const int c = col & 1;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    const int R = (L + rb - 1) / rb, y0 = (int)(t / (unsigned)cols) * R, y1 = y0 + R < L ? y0 + R : L;
    if (k < Hh) {
        for (int y = y0; y < y1; ++y) {
            float th;
            const Nb n = load_nb(st, L, Hh, c, y, k, th);
            const size_t i = ((size_t)c * L + y) * Hh + k;
            saved[i] = th;
            const u32x4 r = philox10(traj, (uint32_t)c, 2u, (uint32_t)y * (uint32_t)P + (uint32_t)(k >> 1), k0, k1);
            const float pm = (k & 1) ? box_muller(r.z, r.w) : box_muller(r.x, r.y);
            p[i] = pm;
            accumulate(v, n, c, __fmul_rn(0.5f, __fmul_rn(pm, pm)));
        }
    }
    write_record(v, rec, t);              // every lane reaches the wave sums
}

// One leap-frog step: kick with `kick` = eps (eps/2 on the first step), then
// drift by eps/(2 pi) p turns.  Grid (2 ceil(Hh/256), L).
__global__ void __launch_bounds__(kThreads)
k_hmc_step(const float* __restrict__ src, float* __restrict__ dst, float* __restrict__ p, int L, float nbeta_kick,
           float drift)
{
    const int Hh = L >> 1;
    const int k = (blockIdx.x >> 1) * kThreads + threadIdx.x;
    if (k >= Hh) return;
    const int y = blockIdx.y, c = blockIdx.x & 1;
    float th;
    const Nb n = load_nb(src, L, Hh, c, y, k, th);
    const size_t i = ((size_t)c * L + y) * Hh + k;
    const float pn = __fmaf_rn(nbeta_kick, sin_sum(n), p[i]);
    p[i] = pn;
    dst[i] = __builtin_amdgcn_fractf(__fmaf_rn(drift, pn, th));
}

// One leap-frog step for L % 4 == 0: a thread takes the two entries 2j, 2j+1 of
// a half-row in R consecutive rows (8-byte loads and stores).  Its horizontal
// neighbours in the other plane are that plane's pair 2j, 2j+1 of the same row
// and one more entry (2j-1 if o = 0, 2j+2 if o = 1); its vertical neighbours are
// the other plane's pairs of the rows above and below, so the R rows share R + 2
// rows of the other plane.  1-D grid of 2 ceil(J/256) (L/R) workgroups, J = L/4,
// remapped by xcd_band.
template <int R>
__global__ void __launch_bounds__(kThreads)
k_hmc_step2(const float* __restrict__ src, float* __restrict__ dst, float* __restrict__ p, int L, float nbeta_kick,
            float drift)
{
    const int Hh = L >> 1, J = Hh >> 1;
    const int cols = 2 * ((J + kThreads - 1) / kThreads);
    const unsigned t = xcd_band(blockIdx.x, gridDim.x);
    const int y0 = (int)(t / (unsigned)cols) * R, col = (int)(t % (unsigned)cols);
    const int c = col & 1;
    const int j = (col >> 1) * kThreads + threadIdx.x;
    if (j >= J) return;
    const float* oth = src + (size_t)(1 - c) * L * Hh;
    float2 h[R + 2];                       // other plane, rows y0-1 .. y0+R
#pragma unroll
    for (int r = 0; r < R + 2; ++r) h[r] = ((const float2*)(oth + (size_t)wrapi(y0 - 1 + r, L) * Hh))[j];
    float2 th[R], pv[R];
    float e[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = y0 + r;
        const int o = (c + y) & 1;
        th[r] = ((const float2*)(src + ((size_t)c * L + y) * Hh))[j];
        pv[r] = ((const float2*)(p + ((size_t)c * L + y) * Hh))[j];
        e[r] = oth[(size_t)y * Hh + (o ? wrapi(2 * j + 2, Hh) : wrapi(2 * j - 1, Hh))];
    }
    float hc0[R + 2], hs0[R + 2], hc1[R + 2], hs1[R + 2];
#pragma unroll
    for (int r = 0; r < R + 2; ++r) {
        sincos_turn(h[r].x, hs0[r], hc0[r]);
        sincos_turn(h[r].y, hs1[r], hc1[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = y0 + r;
        const int o = (c + y) & 1;
        float sa, ca, sb, cb, se, ce;
        sincos_turn(th[r].x, sa, ca);
        sincos_turn(th[r].y, sb, cb);
        sincos_turn(e[r], se, ce);
        Nb na, nb;
        na.c = ca; na.s = sa;
        nb.c = cb; nb.s = sb;
        // entry 2j: left = (o ? h0 : e), right = (o ? h1 : h0); 2j+1: left = (o ? h1 : h0), right = (o ? e : h1)
        na.cl = o ? hc0[r + 1] : ce;         na.sl = o ? hs0[r + 1] : se;
        na.cr = o ? hc1[r + 1] : hc0[r + 1]; na.sr = o ? hs1[r + 1] : hs0[r + 1];
        nb.cl = o ? hc1[r + 1] : hc0[r + 1]; nb.sl = o ? hs1[r + 1] : hs0[r + 1];
        nb.cr = o ? ce : hc1[r + 1];         nb.sr = o ? se : hs1[r + 1];
        na.cu = hc0[r]; na.su = hs0[r]; nb.cu = hc1[r]; nb.su = hs1[r];
        na.cd = hc0[r + 2]; na.sd = hs0[r + 2]; nb.cd = hc1[r + 2]; nb.sd = hs1[r + 2];
        const float pa = __fmaf_rn(nbeta_kick, sin_sum(na), pv[r].x);
        const float pb = __fmaf_rn(nbeta_kick, sin_sum(nb), pv[r].y);
        ((float2*)(p + ((size_t)c * L + y) * Hh))[j] = make_float2(pa, pb);
        ((float2*)(dst + ((size_t)c * L + y) * Hh))[j] =
            make_float2(__builtin_amdgcn_fractf(__fmaf_rn(drift, pa, th[r].x)),
                        __builtin_amdgcn_fractf(__fmaf_rn(drift, pb, th[r].y)));
    }
}

constexpr int kStepRows = 4;               // rows per thread of k_hmc_step2

// K leap-frog steps per pass (temporal blocking), for L % 32 == 0.  A workgroup
// owns a 32 x 32 tile of sites (natural coordinates) and loads the angles and
// momenta of the tile grown by K sites on every side (both colours) into
// registers (ceil((32 + 2K)^2 / 256) sites per thread); step q updates the sites
// more than q sites from the edge of the grown tile, whose neighbours are then all
// up to date, so after K steps the tile itself is exact and is written to dst / pdst
// (the momenta ping-pong too: other tiles read this tile's old momenta as
// their halo).  (cos, sin) of the angles live in two LDS buffers (read one,
// write the other, one barrier per step).  Every site is updated with exactly
// the arithmetic of k_hmc_step (neighbour sums (left + right) + (up + down),
// the same fma), so the trajectory is bit for bit the one-step-per-launch one.
// kick0: the first step's kick (-beta eps/2 on a trajectory's first step),
// kick: the others'.  Grid (L/32)^2 workgroups, XCD bands of tile rows.
constexpr int kMultiTile = 32;

template <int K>
__global__ void __launch_bounds__(kThreads)
k_hmc_multi(const float* __restrict__ src, float* __restrict__ dst, const float* __restrict__ psrc,
            float* __restrict__ pdst, int L, float kick0, float kick, float drift)
{
    constexpr int T = kMultiTile, E = T + 2 * K, NE = E * E, M = (NE + kThreads - 1) / kThreads;
    __shared__ float2 cs[2][NE];
    const int Hh = L >> 1, nt = L / T;
    const int b = (int)xcd_band(blockIdx.x, gridDim.x);
    const int ty = b / nt, tx = b - ty * nt;
    const int x0 = tx * T - K, y0 = ty * T - K;
    float th[M], pm[M];
    unsigned off[M];
    int dep[M];       // distance of the slot's site from the grown tile's edge (-1: no site)
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = threadIdx.x + m * kThreads;
        dep[m] = -1;
        if (i < NE) {
            const int ye = i / E, xe = i - ye * E;
            dep[m] = min(min(xe, E - 1 - xe), min(ye, E - 1 - ye));
            const int x = wrapi(x0 + xe, L), y = wrapi(y0 + ye, L);
            off[m] = (unsigned)((((x + y) & 1) * L + y) * Hh + (x >> 1));
            th[m] = src[off[m]];
            pm[m] = psrc[off[m]];
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = threadIdx.x + m * kThreads;
        if (i < NE) {
            float sn, cn;
            sincos_turn(th[m], sn, cn);
            cs[0][i] = make_float2(cn, sn);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const float2* cur = cs[q & 1];
        float2* nxt = cs[(q + 1) & 1];
        const float kq = q == 0 ? kick0 : kick;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int i = threadIdx.x + m * kThreads;
            if (dep[m] > q) {
                const float2 own = cur[i], l = cur[i - 1], r = cur[i + 1], u = cur[i - E], d = cur[i + E];
                Nb n;
                n.c = own.x; n.s = own.y;
                n.cl = l.x; n.sl = l.y; n.cr = r.x; n.sr = r.y;
                n.cu = u.x; n.su = u.y; n.cd = d.x; n.sd = d.y;
                pm[m] = __fmaf_rn(kq, sin_sum(n), pm[m]);
                th[m] = __builtin_amdgcn_fractf(__fmaf_rn(drift, pm[m], th[m]));
                if (q + 1 < K) {
                    float sn, cn;
                    sincos_turn(th[m], sn, cn);
                    nxt[i] = make_float2(cn, sn);
                }
            }
        }
        if (q + 1 < K) __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (dep[m] >= K) {           // the tile itself
            dst[off[m]] = th[m];
            pdst[off[m]] = pm[m];
        }
    }
}

// The same pass on larger tiles: T x T sites grown by K, NT threads, and with
// SINGLE one LDS buffer of (cos, sin) (every update of a step reads its
// neighbours, barrier, the new values are written, barrier), which halves the LDS
// so that 64 x 64 tiles keep two workgroups of 1024 threads on a CU.  The grown
// tile is 1.27 times the tile at T = 64, K = 4 (1.56 at T = 32), so less of the
// work goes to the halo.  Per site the arithmetic is that of k_hmc_step.
// The pass on tile b (after the XCD remap) of one lattice; cs: the LDS buffer(s),
// (SINGLE ? 1 : 2) (T + 2K)^2 float2.
template <int K, int T, int NT, bool SINGLE>
__device__ __forceinline__ void multi_g_body(const float* __restrict__ src, float* __restrict__ dst,
                                             const float* __restrict__ psrc, float* __restrict__ pdst, int L,
                                             float kick0, float kick, float drift, int b, float2* cs)
{
    constexpr int E = T + 2 * K, NE = E * E, M = (NE + NT - 1) / NT;
    const int Hh = L >> 1, nt = L / T;
    const int ty = b / nt, tx = b - ty * nt;
    const int x0 = tx * T - K, y0 = ty * T - K;
    float th[M], pm[M];
    unsigned off[M];
    int dep[M];       // distance of the slot's site from the grown tile's edge (-1: no site)
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = threadIdx.x + m * NT;
        dep[m] = -1;
        if (i < NE) {
            const int ye = i / E, xe = i - ye * E;
            dep[m] = min(min(xe, E - 1 - xe), min(ye, E - 1 - ye));
            const int x = wrapi(x0 + xe, L), y = wrapi(y0 + ye, L);
            off[m] = (unsigned)((((x + y) & 1) * L + y) * Hh + (x >> 1));
            th[m] = src[off[m]];
            pm[m] = psrc[off[m]];
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = threadIdx.x + m * NT;
        if (i < NE) {
            float sn, cn;
            sincos_turn(th[m], sn, cn);
            cs[i] = make_float2(cn, sn);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const float2* cur = cs + (SINGLE ? 0 : (q & 1)) * NE;
        float2* nxt = cs + (SINGLE ? 0 : ((q + 1) & 1)) * NE;
        const float kq = q == 0 ? kick0 : kick;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int i = threadIdx.x + m * NT;
            if (dep[m] > q) {
                const float2 own = cur[i], l = cur[i - 1], r = cur[i + 1], u = cur[i - E], d = cur[i + E];
                Nb n;
                n.c = own.x; n.s = own.y;
                n.cl = l.x; n.sl = l.y; n.cr = r.x; n.sr = r.y;
                n.cu = u.x; n.su = u.y; n.cd = d.x; n.sd = d.y;
                pm[m] = __fmaf_rn(kq, sin_sum(n), pm[m]);
                th[m] = __builtin_amdgcn_fractf(__fmaf_rn(drift, pm[m], th[m]));
            }
        }
        if (q + 1 < K) {
            if constexpr (SINGLE) __syncthreads();
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int i = threadIdx.x + m * NT;
                if (dep[m] > q) {
                    float sn, cn;
                    sincos_turn(th[m], sn, cn);
                    nxt[i] = make_float2(cn, sn);
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

template <int K, int T, int NT, bool SINGLE>
__global__ void __launch_bounds__(NT)
k_hmc_multi_g(const float* __restrict__ src, float* __restrict__ dst, const float* __restrict__ psrc,
              float* __restrict__ pdst, int L, float kick0, float kick, float drift)
{
    constexpr int NE = (T + 2 * K) * (T + 2 * K);
    __shared__ float2 cs[(SINGLE ? 1 : 2) * NE];
    multi_g_body<K, T, NT, SINGLE>(src, dst, psrc, pdst, L, kick0, kick, drift,
                                   (int)xcd_band(blockIdx.x, gridDim.x), cs);
}

constexpr int kMaxStepsPerPass = 8;

constexpr int kWideTile = 64, kWideThreads = 1024;

// L % 64 == 0: 64 x 64 tiles, 1024 threads, one LDS buffer; else 32 x 32 tiles.
template <int K>
static void launch_multi(unsigned nb, hipStream_t s, const float* src, float* dst, const float* psrc, float* pdst,
                         int L, float kick0, float kick, float drift)
{
    if (L % kWideTile == 0) {
        const unsigned nbw = (unsigned)((L / kWideTile) * (L / kWideTile));
        hipLaunchKernelGGL((k_hmc_multi_g<K, kWideTile, kWideThreads, true>), dim3(nbw), dim3(kWideThreads), 0, s, src,
                           dst, psrc, pdst, L, kick0, kick, drift);
        return;
    }
    hipLaunchKernelGGL(k_hmc_multi<K>, dim3(nb), dim3(kThreads), 0, s, src, dst, psrc, pdst, L, kick0, kick, drift);
}

static void launch_multi_k(int k, unsigned nb, hipStream_t s, const float* src, float* dst, const float* psrc,
                           float* pdst, int L, float kick0, float kick, float drift)
{
    switch (k) {
    case 1: launch_multi<1>(nb, s, src, dst, psrc, pdst, L, kick0, kick, drift); break;
    case 2: launch_multi<2>(nb, s, src, dst, psrc, pdst, L, kick0, kick, drift); break;
    case 3: launch_multi<3>(nb, s, src, dst, psrc, pdst, L, kick0, kick, drift); break;
    case 4: launch_multi<4>(nb, s, src, dst, psrc, pdst, L, kick0, kick, drift); break;
    case 5: launch_multi<5>(nb, s, src, dst, psrc, pdst, L, kick0, kick, drift); break;
    case 6: launch_multi<6>(nb, s, src, dst, psrc, pdst, L, kick0, kick, drift); break;
    case 7: launch_multi<7>(nb, s, src, dst, psrc, pdst, L, kick0, kick, drift); break;
    default: launch_multi<8>(nb, s, src, dst, psrc, pdst, L, kick0, kick, drift); break;
    }
}

// Final half kick and the partial records of H_new; `copy` != NULL receives the
// angles (the final ones may sit in the second buffer).  Grid as k_hmc_begin.
__global__ void __launch_bounds__(kThreads)
k_hmc_end(const float* __restrict__ st, float* __restrict__ copy, const float* __restrict__ p, int L,
          float nbeta_kick, int cols, int rb, double* __restrict__ rec)
{
    const int Hh = L >> 1;
    const unsigned t = xcd_band(blockIdx.x, gridDim.x);
    const int col = (int)(t % (unsigned)cols);
    const int k = (col >> 1) * kThreads + threadIdx.x;
    const int c = col & 1;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    const int R = (L + rb - 1) / rb, y0 = (int)(t / (unsigned)cols) * R, y1 = y0 + R < L ? y0 + R : L;
    if (k < Hh) {
        for (int y = y0; y < y1; ++y) {
            float th;
            const Nb n = load_nb(st, L, Hh, c, y, k, th);
            const size_t i = ((size_t)c * L + y) * Hh + k;
            if (copy) copy[i] = th;
            const float pn = __fmaf_rn(nbeta_kick, sin_sum(n), p[i]);
            accumulate(v, n, c, __fmul_rn(0.5f, __fmul_rn(pn, pn)));
        }
    }
    write_record(v, rec, t);
}

// Begin and end of a trajectory for L % 4 == 0, by pairs: a thread takes pair j
// (entries 2j, 2j+1) of both colours in a run of consecutive rows.  Each plane's
// pair j of the rows above, at and below a row sits in registers as a rolling
// window with its (cos, sin): a row loads one new pair of each plane and one edge
// entry of each (2j-1 or 2j+2), so every angle is read from memory once (a thread
// per colour would read each plane twice, once as its own colour and once as the
// other's neighbours) and a site costs 1.5 sines and cosines.
// 1-D grid of cols2 = ceil(J/256) column blocks times the row blocks, remapped by
// xcd_band; a row block holds ends_group(L) runs side by side (one unless
// J < 256); one partial record per wave.
struct PairCS {
    float c0, s0, c1, s1;
};
__device__ __forceinline__ PairCS pair_cs(float2 t)
{
    PairCS q;
    sincos_turn(t.x, q.s0, q.c0);
    sincos_turn(t.y, q.s1, q.c1);
    return q;
}

// Neighbourhoods of the pair (entries 2j, 2j+1) of row y: own (cos, sin) in a,
// b; the other plane's row above (u), at (h) and below (d) and the edge entry e.
__device__ __forceinline__ void pair_nb(const PairCS& own, const PairCS& u, const PairCS& h, const PairCS& d,
                                       float ce, float se, int o, Nb& na, Nb& nb)
{
    na.c = own.c0; na.s = own.s0;
    nb.c = own.c1; nb.s = own.s1;
    // entry 2j: left = (o ? h0 : e), right = (o ? h1 : h0); 2j+1: left = (o ? h1 : h0), right = (o ? e : h1)
    na.cl = o ? h.c0 : ce;   na.sl = o ? h.s0 : se;
    na.cr = o ? h.c1 : h.c0; na.sr = o ? h.s1 : h.s0;
    nb.cl = o ? h.c1 : h.c0; nb.sl = o ? h.s1 : h.s0;
    nb.cr = o ? ce : h.c1;   nb.sr = o ? se : h.s1;
    na.cu = u.c0; na.su = u.s0; nb.cu = u.c1; nb.su = u.s1;
    na.cd = d.c0; na.sd = d.s0; nb.cd = d.c1; nb.sd = d.s1;
}

// Pair columns per run and runs per workgroup of the pair kernels: a lattice
// narrower than a workgroup (J < 256 pair columns) gives each workgroup
// 256 / J runs side by side instead of leaving lanes idle.
__host__ __device__ __forceinline__ int ends_group(int L)
{
    const int J = L >> 2;
    return kThreads / (J < kThreads ? (J > 0 ? J : 1) : kThreads);
}

// The pass on record block t (after the XCD remap) of one lattice, whose rows
// are cut into `runs` runs of equal length (the last may be shorter).
template <bool BEGIN>
__device__ __forceinline__ void ends2_body(const float* __restrict__ st, float* __restrict__ p,
                                           float* __restrict__ copy, int L, uint32_t traj, uint32_t k0, uint32_t k1,
                                           float nbeta_kick, int cols, int runs, double* __restrict__ rec, unsigned t)
{
    const int Hh = L >> 1, J = Hh >> 1;
    const int G = ends_group(L), JB = kThreads / G;
    const int col = (int)(t % (unsigned)cols);
    const int g = (int)threadIdx.x / JB;
    const int j = col * kThreads + (int)threadIdx.x - g * JB;
    const int run = (int)(t / (unsigned)cols) * G + g;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    const int R = (L + runs - 1) / runs, y0 = run * R, y1 = y0 + R < L ? y0 + R : L;
    if (g < G && j < J && y0 < y1) {
        const float* pl0 = st;
        const float* pl1 = st + (size_t)L * Hh;
        const float2* r0 = (const float2*)pl0;
        const float2* r1 = (const float2*)pl1;
        // windows: plane c rows y-1 (u), y (h) with angles, y+1 loaded per row
        float2 t0 = r0[(size_t)y0 * J + j], t1 = r1[(size_t)y0 * J + j];
        PairCS u0 = pair_cs(r0[(size_t)wrapi(y0 - 1, L) * J + j]), u1 = pair_cs(r1[(size_t)wrapi(y0 - 1, L) * J + j]);
        PairCS h0 = pair_cs(t0), h1 = pair_cs(t1);
        const int kl = wrapi(2 * j - 1, Hh), kr = wrapi(2 * j + 2, Hh);
        for (int y = y0; y < y1; ++y) {
            const int yd = wrapi(y + 1, L);
            const float2 n0 = r0[(size_t)yd * J + j], n1 = r1[(size_t)yd * J + j];
            const PairCS d0 = pair_cs(n0), d1 = pair_cs(n1);
            const int o = y & 1;                  // red rows: o = y & 1; black rows: 1 - o
            // edge entries: the red pair reads plane 1 at 2j+2 (o) or 2j-1; the black pair plane 0 the other way
            float se1, ce1, se0, ce0;
            sincos_turn(pl1[(size_t)y * Hh + (o ? kr : kl)], se1, ce1);
            sincos_turn(pl0[(size_t)y * Hh + (o ? kl : kr)], se0, ce0);
            Nb na0, nb0, na1, nb1;
            pair_nb(h0, u1, h1, d1, ce1, se1, o, na0, nb0);
            pair_nb(h1, u0, h0, d0, ce0, se0, 1 - o, na1, nb1);
            const size_t row0 = (size_t)y * Hh, row1 = ((size_t)L + y) * Hh;
            float pa0, pb0, pa1, pb1;
            if constexpr (BEGIN) {
                ((float2*)(copy + row0))[j] = t0;      // saved angles
                ((float2*)(copy + row1))[j] = t1;
                const u32x4 q0 = philox10(traj, 0u, 2u, (uint32_t)y * (uint32_t)J + (uint32_t)j, k0, k1);
                const u32x4 q1 = philox10(traj, 1u, 2u, (uint32_t)y * (uint32_t)J + (uint32_t)j, k0, k1);
                pa0 = box_muller(q0.x, q0.y);
                pb0 = box_muller(q0.z, q0.w);
                pa1 = box_muller(q1.x, q1.y);
                pb1 = box_muller(q1.z, q1.w);
                ((float2*)(p + row0))[j] = make_float2(pa0, pb0);
                ((float2*)(p + row1))[j] = make_float2(pa1, pb1);
            } else {
                if (copy) {
                    ((float2*)(copy + row0))[j] = t0;
                    ((float2*)(copy + row1))[j] = t1;
                }
                const float2 pv0 = ((const float2*)(p + row0))[j], pv1 = ((const float2*)(p + row1))[j];
                pa0 = __fmaf_rn(nbeta_kick, sin_sum(na0), pv0.x);
                pb0 = __fmaf_rn(nbeta_kick, sin_sum(nb0), pv0.y);
                pa1 = __fmaf_rn(nbeta_kick, sin_sum(na1), pv1.x);
                pb1 = __fmaf_rn(nbeta_kick, sin_sum(nb1), pv1.y);
            }
            accumulate(v, na0, 0, __fmul_rn(0.5f, __fmul_rn(pa0, pa0)));
            accumulate(v, nb0, 0, __fmul_rn(0.5f, __fmul_rn(pb0, pb0)));
            accumulate(v, na1, 1, __fmul_rn(0.5f, __fmul_rn(pa1, pa1)));
            accumulate(v, nb1, 1, __fmul_rn(0.5f, __fmul_rn(pb1, pb1)));
            u0 = h0; u1 = h1;
            h0 = d0; h1 = d1;
            t0 = n0; t1 = n1;
        }
    }
    write_record(v, rec, t);              // every lane reaches the wave sums
}

template <bool BEGIN>
__global__ void __launch_bounds__(kThreads)
k_hmc_ends2(const float* __restrict__ st, float* __restrict__ p, float* __restrict__ copy, int L, uint32_t traj,
            const uint32_t* __restrict__ traj_dev, uint32_t k0, uint32_t k1, float nbeta_kick, int cols, int rb,
            double* __restrict__ rec)
{
    if (BEGIN && traj_dev) traj = *traj_dev;
    ends2_body<BEGIN>(st, p, copy, L, traj, k0, k1, nbeta_kick, cols, rb, rec, xcd_band(blockIdx.x, gridDim.x));
}

// Sum of one set of records in a fixed order (thread t: records t, t + 256, ...,
// then the wave sums and the four waves in order); thread 0 gets the totals.
__device__ void sum_records(const double* __restrict__ rec, int nrec, double out[7], double* red)
{
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int r = threadIdx.x; r < nrec; r += kThreads)
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] += rec[(size_t)r * 8 + q];
#pragma unroll
    for (int q = 0; q < 7; ++q) v[q] = wave_sum(v[q]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < 7; ++q) red[(threadIdx.x >> 6) * 7 + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < 7; ++q) out[q] = (red[q] + red[7 + q]) + (red[14 + q] + red[21 + q]);
    __syncthreads();
}

// Metropolis step of the trajectory: one workgroup, on the chunk sums of the two
// record sets.
__global__ void __launch_bounds__(kThreads)
k_hmc_decide(const double* __restrict__ rec_old, const double* __restrict__ rec_new, int nrec, double beta,
             uint32_t traj, const uint32_t* __restrict__ traj_dev, uint32_t k0, uint32_t k1,
             unsigned* __restrict__ flag, xy_hmc_obs* __restrict__ obs)
{
    if (traj_dev) traj = *traj_dev;
    __shared__ double red[4 * 7];
    double o[7], n[7];
    sum_records(rec_old, nrec, o, red);
    sum_records(rec_new, nrec, n, red);
    if (threadIdx.x == 0) decide_core(o, n, beta, traj, k0, k1, flag, obs);
}

// Rejected trajectory: the saved angles back into the state.
__global__ void __launch_bounds__(kThreads)
k_hmc_restore(const unsigned* __restrict__ flag, const float* __restrict__ saved, float* __restrict__ st, size_t n)
{
    if (*flag) return;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
        st[i] = saved[i];
}

// ---------------------------------------------------------------- batches
// One launch per stage over all lattices of a batch.  A stage's grid is the
// lattices' single-lattice grids one after another, each padded to a multiple of
// 8 workgroups (so that each lattice's first workgroup goes to XCD 0 and the XCD
// remap gives it the same bands as alone); a workgroup finds its lattice by
// bisection over the stage's block offsets and runs the single-lattice pass on
// its local index.

// Lattice i with start[i] <= blk < start[i + 1].
__device__ __forceinline__ int bh_find(const uint32_t* __restrict__ start, int n, uint32_t blk)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= blk) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Trajectory ends: BEGIN draws the momenta, saves the angles and writes the H_old
// records; else the final half kick from the angles and momenta the leap-frog
// passes left in the second buffers (parity odd, angles also copied back into the
// state) or the first, and the H_new records.
template <bool BEGIN>
__global__ void __launch_bounds__(kThreads)
k_bhmc_ends(const BhLat* __restrict__ d, const uint32_t* __restrict__ start, int n,
            const uint32_t* __restrict__ traj_dev, int parity)
{
    const int i = bh_find(start, n, blockIdx.x);
    const BhLat& q = d[i];
    const int G = ends_group(q.L);
    const unsigned nb = (unsigned)(q.cols * ((q.rb + G - 1) / G)), lb = blockIdx.x - start[i];
    if (lb >= nb) return;
    const unsigned t = xcd_band(lb, nb);
    if constexpr (BEGIN)
        ends2_body<true>(q.st, q.w.p, q.w.saved, q.L, *traj_dev, q.k0, q.k1, 0.0f, q.cols, q.rb, q.w.rec_old, t);
    else
        ends2_body<false>(parity ? q.pp : q.st, parity ? q.w.p2 : q.w.p, parity ? q.st : nullptr, q.L, 0u, q.k0,
                          q.k1, q.kick_half, q.cols, q.rb, q.w.rec_new, t);
}

// K leap-frog steps of every lattice on 64 x 64 tiles; parity odd: the angles and
// momenta are read from the second buffers and written to the first.
template <int K>
__global__ void __launch_bounds__(kWideThreads)
k_bhmc_multi(const BhLat* __restrict__ d, const uint32_t* __restrict__ start, int n, int parity, int first,
             float drift)
{
    constexpr int NE = (kWideTile + 2 * K) * (kWideTile + 2 * K);
    __shared__ float2 cs[NE];
    const int i = bh_find(start, n, blockIdx.x);
    const BhLat& q = d[i];
    const int nt = q.L / kWideTile;
    const unsigned nb = (unsigned)(nt * nt), lb = blockIdx.x - start[i];
    if (lb >= nb) return;
    multi_g_body<K, kWideTile, kWideThreads, true>(parity ? q.pp : q.st, parity ? q.st : q.pp,
                                                   parity ? q.w.p2 : q.w.p, parity ? q.w.p : q.w.p2, q.L,
                                                   first ? q.kick_half : q.kick_full, q.kick_full, drift,
                                                   (int)xcd_band(lb, nb), cs);
}

// One lattice's records summed as the single-lattice trajectory sums them: chunks
// of 256 records as k_reduce_chunks forms them (into ch, LDS), then the chunk sums
// as k_hmc_decide forms them.  Thread 0 gets the totals.
__device__ void bh_sum(const double* __restrict__ rec, int nrec, double* ch, double out[7], double* red)
{
    const int nch = (nrec + 255) / 256;
    for (int c = 0; c < nch; ++c) {
        const int i = c * 256 + threadIdx.x;
        double v[7] = {0, 0, 0, 0, 0, 0, 0};
        if (i < nrec) {
            const double* r = rec + (size_t)i * 8;
#pragma unroll
            for (int k = 0; k < 7; ++k) v[k] = r[k];
        }
        block_sum7_256(v, red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 7; ++k) ch[c * 8 + k] = v[k];
            ch[c * 8 + 7] = 0.0;
        }
        __syncthreads();
    }
    sum_records(ch, nch, out, red);
}

// Metropolis step of every lattice: workgroup i on lattice i.
__global__ void __launch_bounds__(kThreads)
k_bhmc_decide(const BhLat* __restrict__ d, const uint32_t* __restrict__ traj_dev)
{
    __shared__ double red[4 * 7];
    __shared__ double ch[kHmcMaxChunks * 8];
    const BhLat& q = d[blockIdx.x];
    double o[7], nn[7];
    bh_sum(q.w.rec_old, q.nrec, ch, o, red);
    bh_sum(q.w.rec_new, q.nrec, ch, nn, red);
    if (threadIdx.x == 0) decide_core(o, nn, q.beta, *traj_dev, q.k0, q.k1, q.w.flag, q.obs);
}

// Rejected trajectories: the saved angles back into the state.
__global__ void __launch_bounds__(kThreads)
k_bhmc_restore(const BhLat* __restrict__ d, const uint32_t* __restrict__ start, int n)
{
    const int i = bh_find(start, n, blockIdx.x);
    const BhLat& q = d[i];
    if (*q.w.flag) return;
    const size_t ns = (size_t)q.L * (size_t)q.L;
    const size_t stride = (size_t)(start[i + 1] - start[i]) * kThreads;
    for (size_t j = (size_t)(blockIdx.x - start[i]) * kThreads + threadIdx.x; j < ns; j += stride)
        q.st[j] = q.w.saved[j];
}

template <int K>
static void launch_bmulti(uint32_t nb, hipStream_t s, const BhLat* d, const uint32_t* start, int n, int parity,
                          int first, float drift)
{
    hipLaunchKernelGGL(k_bhmc_multi<K>, dim3(nb), dim3(kWideThreads), 0, s, d, start, n, parity, first, drift);
}

static void launch_bmulti_k(int k, uint32_t nb, hipStream_t s, const BhLat* d, const uint32_t* start, int n,
                            int parity, int first, float drift)
{
    switch (k) {
    case 1: launch_bmulti<1>(nb, s, d, start, n, parity, first, drift); break;
    case 2: launch_bmulti<2>(nb, s, d, start, n, parity, first, drift); break;
    case 3: launch_bmulti<3>(nb, s, d, start, n, parity, first, drift); break;
    case 4: launch_bmulti<4>(nb, s, d, start, n, parity, first, drift); break;
    case 5: launch_bmulti<5>(nb, s, d, start, n, parity, first, drift); break;
    case 6: launch_bmulti<6>(nb, s, d, start, n, parity, first, drift); break;
    case 7: launch_bmulti<7>(nb, s, d, start, n, parity, first, drift); break;
    default: launch_bmulti<8>(nb, s, d, start, n, parity, first, drift); break;
    }
}

}  // namespace

// Block columns (both colours) and row blocks of the record-writing kernels: as
// many rows as keep one record set at most kHmcMaxRecords.
static int hmc_cols(int L) { return 2 * (((L >> 1) + kThreads - 1) / kThreads); }

static int hmc_row_blocks(int L)
{
    int gy = kHmcMaxRecords / (hmc_cols(L) * (kThreads / 64));
    if (gy > L) gy = L;
    return gy < 1 ? 1 : gy;
}

static bool hmc_pairs(int L) { return L % 4 == 0; }
static int hmc_cols2(int L) { return ((L >> 2) + kThreads - 1) / kThreads; }
// Row runs of the pair kernels.  Each run reads the plane rows just above and
// below it once more and starts its rolling window with their sines and
// cosines, so short runs cost traffic and arithmetic.  Lattices of more than one
// column block (L > 1024): runs of up to 32 rows, but at least about 2048
// workgroups while L allows, and at most one record per wave within the record
// buffer.  One column block (L <= 1024, where batches of many lattices supply
// the parallelism): runs of 8 rows.
static int hmc_runs2(int L)
{
    const int cols = hmc_cols2(L);
    if (cols == 1) return (L + 7) / 8;
    int gy = (2048 + cols - 1) / cols;
    if (gy < L / 32) gy = L / 32;
    const int cap = kHmcMaxRecords / (cols * (kThreads / 64));
    if (gy > cap) gy = cap;
    if (gy > L) gy = L;
    return gy < 1 ? 1 : gy;
}
// Workgroups per column block: the runs, ends_group(L) to a workgroup.
static int hmc_row_blocks2(int L)
{
    const int G = ends_group(L);
    return (hmc_runs2(L) + G - 1) / G;
}

int hmc_records(int L)
{
    if (hmc_pairs(L)) return hmc_cols2(L) * hmc_row_blocks2(L) * (kThreads / 64);
    return hmc_cols(L) * hmc_row_blocks(L) * (kThreads / 64);
}

size_t hmc_work_bytes(int L)
{
    const size_t n = (size_t)L * (size_t)L;
    return 256 + 3 * n * sizeof(float) + 2 * (size_t)(kHmcMaxRecords + kHmcMaxChunks) * 8 * sizeof(double);
}

HmcWork hmc_carve(void* work, int L)
{
    HmcWork w;
    char* b = (char*)work;
    w.flag = (unsigned*)b;
    b += 256;
    const size_t n = (size_t)L * (size_t)L;
    w.p = (float*)b;
    b += n * sizeof(float);
    w.saved = (float*)b;
    b += n * sizeof(float);
    w.p2 = (float*)b;
    b += n * sizeof(float);
    w.rec_old = (double*)b;
    b += (size_t)kHmcMaxRecords * 8 * sizeof(double);
    w.rec_new = (double*)b;
    b += (size_t)kHmcMaxRecords * 8 * sizeof(double);
    w.chunk_old = (double*)b;
    b += (size_t)kHmcMaxChunks * 8 * sizeof(double);
    w.chunk_new = (double*)b;
    return w;
}

// The same areas with the record arrays sized for this L only (batches).
size_t hmc_work_bytes_compact(int L)
{
    const size_t n = (size_t)L * (size_t)L;
    const size_t nrec = (size_t)hmc_records(L), nch = (nrec + 255) / 256;
    return 256 + 3 * n * sizeof(float) + 2 * (nrec + nch) * 8 * sizeof(double);
}

HmcWork hmc_carve_compact(void* work, int L)
{
    HmcWork w;
    char* b = (char*)work;
    const size_t n = (size_t)L * (size_t)L;
    const size_t nrec = (size_t)hmc_records(L), nch = (nrec + 255) / 256;
    w.flag = (unsigned*)b;
    b += 256;
    w.p = (float*)b;
    b += n * sizeof(float);
    w.saved = (float*)b;
    b += n * sizeof(float);
    w.p2 = (float*)b;
    b += n * sizeof(float);
    w.rec_old = (double*)b;
    b += nrec * 8 * sizeof(double);
    w.rec_new = (double*)b;
    b += nrec * 8 * sizeof(double);
    w.chunk_old = (double*)b;
    b += nch * 8 * sizeof(double);
    w.chunk_new = (double*)b;
    return w;
}

bool hmc_multi_supported(int L) { return L >= kMultiTile && L % kMultiTile == 0; }

hipError_t launch_hmc_trajectory(float* state, float* pingpong, const HmcWork& w, int L, double beta, double eps,
                                 int n_md, int steps_per_pass, uint32_t traj, uint32_t k0, uint32_t k1,
                                 xy_hmc_obs* obs, hipStream_t s, const uint32_t* traj_dev)
{
    const bool pairs2 = hmc_pairs(L);
    const int cols = pairs2 ? hmc_cols2(L) : hmc_cols(L), rb = pairs2 ? hmc_runs2(L) : hmc_row_blocks(L);
    const int nbr = pairs2 ? hmc_row_blocks2(L) : rb;     // workgroups per column block
    const dim3 grec((unsigned)(cols * nbr)), gstep(hmc_cols(L), L), block(kThreads);
    const int nrec = hmc_records(L);
    const int nchunk = (nrec + 255) / 256;
    const float drift = (float)(eps / (2.0 * 3.14159265358979323846));
    if (pairs2)
        hipLaunchKernelGGL(k_hmc_ends2<true>, grec, block, 0, s, state, w.p, w.saved, L, traj, traj_dev, k0, k1, 0.0f,
                           cols, rb, w.rec_old);
    else
        hipLaunchKernelGGL(k_hmc_begin, grec, block, 0, s, state, w.p, w.saved, L, traj, traj_dev, k0, k1, cols, rb,
                           w.rec_old);
    float* src = state;
    float* dst = pingpong;
    float* p = w.p;
    const float kick_half = (float)(-beta * 0.5 * eps), kick_full = (float)(-beta * eps);
    if (steps_per_pass > 1 && hmc_multi_supported(L)) {
        // passes of up to steps_per_pass steps; the momenta ping-pong between p and p2
        float* pn = w.p2;
        const unsigned nb = (unsigned)((L / kMultiTile) * (L / kMultiTile));
        const int kmax = steps_per_pass < kMaxStepsPerPass ? steps_per_pass : kMaxStepsPerPass;
        for (int q = 0; q < n_md;) {
            const int k = n_md - q < kmax ? n_md - q : kmax;
            launch_multi_k(k, nb, s, src, dst, p, pn, L, q == 0 ? kick_half : kick_full, kick_full, drift);
            float* t = src;
            src = dst;
            dst = t;
            t = p;
            p = pn;
            pn = t;
            q += k;
        }
    } else {
        const bool pairs = (L % (4 * kStepRows)) == 0;
        const unsigned nstep2 = (unsigned)(2 * ((L / 4 + kThreads - 1) / kThreads)) * (unsigned)(L / kStepRows);
        for (int q = 0; q < n_md; ++q) {
            const float kick = q == 0 ? kick_half : kick_full;
            if (pairs)
                hipLaunchKernelGGL(k_hmc_step2<kStepRows>, dim3(nstep2), block, 0, s, src, dst, p, L, kick, drift);
            else
                hipLaunchKernelGGL(k_hmc_step, gstep, block, 0, s, src, dst, p, L, kick, drift);
            float* t = src;
            src = dst;
            dst = t;
        }
    }
    if (pairs2)
        hipLaunchKernelGGL(k_hmc_ends2<false>, grec, block, 0, s, src, p, src == state ? nullptr : state, L, traj,
                           traj_dev, k0, k1, kick_half, cols, rb, w.rec_new);
    else
        hipLaunchKernelGGL(k_hmc_end, grec, block, 0, s, src, src == state ? nullptr : state, p, L, kick_half, cols,
                           rb, w.rec_new);
    hipError_t e = launch_reduce_chunks(w.rec_old, nrec, w.chunk_old, s);
    if (e == hipSuccess) e = launch_reduce_chunks(w.rec_new, nrec, w.chunk_new, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hmc_decide, dim3(1), block, 0, s, w.chunk_old, w.chunk_new, nchunk, beta, traj, traj_dev,
                       k0, k1, w.flag, obs);
    const size_t n = (size_t)L * (size_t)L;
    const unsigned nb = (unsigned)((n + kThreads * 8 - 1) / (kThreads * 8));
    hipLaunchKernelGGL(k_hmc_restore, dim3(nb < 4096 ? nb : 4096), block, 0, s, w.flag, w.saved, state, n);
    return hipGetLastError();
}

bool hmc_batch_supported(int L) { return L >= kWideTile && L % kWideTile == 0; }

void hmc_batch_describe(BhLat& d, int L, double beta, double eps)
{
    d.L = L;
    d.beta = beta;
    d.cols = hmc_cols2(L);
    d.rb = hmc_runs2(L);
    d.nrec = hmc_records(L);
    d.kick_half = (float)(-beta * 0.5 * eps);
    d.kick_full = (float)(-beta * eps);
}

static uint32_t pad8(uint32_t v) { return (v + 7u) & ~7u; }

void hmc_batch_blocks(int L, uint32_t nb[3])
{
    nb[0] = pad8((uint32_t)(hmc_cols2(L) * hmc_row_blocks2(L)));
    nb[1] = pad8((uint32_t)((L / kWideTile) * (L / kWideTile)));
    const size_t n = (size_t)L * (size_t)L;
    const size_t r = (n + kThreads * 8 - 1) / (kThreads * 8);
    nb[2] = pad8((uint32_t)(r < 4096 ? r : 4096));
}

hipError_t launch_hmc_batch_trajectory(const BhLat* d, const uint32_t* start, int n, const uint32_t totals[3],
                                       double eps, int n_md, int steps_per_pass, const uint32_t* traj_dev,
                                       hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const uint32_t* s_ends = start;
    const uint32_t* s_pass = start + (n + 1);
    const uint32_t* s_rest = start + 2 * (n + 1);
    const float drift = (float)(eps / (2.0 * 3.14159265358979323846));
    const dim3 block(kThreads);
    hipLaunchKernelGGL(k_bhmc_ends<true>, dim3(totals[0]), block, 0, s, d, s_ends, n, traj_dev, 0);
    const int kmax = steps_per_pass < kMaxStepsPerPass ? steps_per_pass : kMaxStepsPerPass;
    int parity = 0;
    for (int q = 0; q < n_md;) {
        const int k = n_md - q < kmax ? n_md - q : kmax;
        launch_bmulti_k(k, totals[1], s, d, s_pass, n, parity, q == 0, drift);
        parity ^= 1;
        q += k;
    }
    hipLaunchKernelGGL(k_bhmc_ends<false>, dim3(totals[0]), block, 0, s, d, s_ends, n, traj_dev, parity);
    hipLaunchKernelGGL(k_bhmc_decide, dim3((unsigned)n), block, 0, s, d, traj_dev);
    hipLaunchKernelGGL(k_bhmc_restore, dim3(totals[2]), block, 0, s, d, s_rest, n);
    return hipGetLastError();
}

}  // namespace xyk
