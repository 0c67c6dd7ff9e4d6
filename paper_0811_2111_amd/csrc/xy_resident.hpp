// xy_resident.hpp -- a whole small lattice in one workgroup's LDS for every sweep
// of a call.
//
// For L <= 128 the angles of both colours (4 L^2 bytes) and the (cos, sin) of one
// colour (4 L^2 bytes) fit in LDS, so a workgroup can run any number of sweeps
// with no halo and no HBM traffic between them: per half-sweep of colour c it
// computes the (cos, sin) of the other colour from the angles in LDS, waits, and
// updates the pairs of colour c in place (an update reads only the other
// colour's (cos, sin) and its own angle), then waits again.  The angles are read
// from HBM once at the start and written once at the end.  Every site is updated
// by xyd::site_update with neighbour sums (left + right) + (up + down) and the
// Philox words of (seed, sweep, colour, row, pair), so the trajectory is that of
// every other schedule.  A measured sweep folds its sums into the black
// half-sweep and writes the record itself (FP64 workgroup sum in a fixed order).
#pragma once

#include "xy.h"
#include "xy_tile1.hpp"

namespace xyd {

constexpr int kResidentMaxL = 128;

// LDS bytes for an L x L lattice: angles 4 L^2, (cos, sin) of one colour 4 L^2,
// then 7 doubles per wave for the record sums.
__host__ __device__ constexpr size_t resident_lds_bytes(int L, int nt)
{
    return (size_t)8 * L * L + (size_t)(nt / 64) * 7 * sizeof(double);
}

// n sweeps of the L x L lattice in src (state layout) starting at sweep index
// sweep0, result in dst (may equal src).  me > 0 and obs != NULL: after the j-th
// sweep of the call (j = 1 .. n) with j % me == 0 the record j / me - 1 goes to
// obs.  NT threads; smem: resident_lds_bytes(L, NT).
template <typename T, int NT>
__device__ __forceinline__ void resident_program(const T* __restrict__ src, T* __restrict__ dst, int L,
                                                 uint32_t sweep0, int n, int me, uint32_t k0, uint32_t k1,
                                                 const Params& p, xy_obs* __restrict__ obs, char* smem)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int Hh = L >> 1, P = Hh >> 1, half = L * Hh;
    float* ang = (float*)smem;                         // [2][L][Hh]
    float2* cs = (float2*)(smem + (size_t)4 * L * L);  // [L][Hh], one colour
    double* red = (double*)(smem + (size_t)8 * L * L);
    for (int i = tid; i < 2 * half; i += NT) ang[i] = store<T>::ld(src[i]);
    __syncthreads();
    for (int j = 1; j <= n; ++j) {
        const uint32_t sweep = sweep0 + (uint32_t)(j - 1);
        const bool meas = me > 0 && obs != nullptr && (j % me) == 0;
        int acc = 0;
        MeasAcc m;
        for (int c = 0; c < 2; ++c) {
            const float* oth = ang + (1 - c) * half;
            for (int i = tid; i < half; i += NT) {
                float sn, cn;
                sincos_turn(oth[i], sn, cn);
                cs[i] = make_float2(cn, sn);
            }
            __syncthreads();
            float* own = ang + c * half;
            for (int q = tid; q < L * P; q += NT) {
                const int y = q / P, jj = q - y * P;
                const int o = (c + y) & 1;
                const int k = 2 * jj;
                const int ku = y == 0 ? L - 1 : y - 1, kd = y == L - 1 ? 0 : y + 1;
                const float2* row = cs + y * Hh;
                // entry 2jj: left 2jj + o - 1, right 2jj + o; entry 2jj + 1: left 2jj + o, right 2jj + o + 1
                const float2 la = row[wrapi(k + o - 1, Hh)], ra = row[k + o];
                const float2 lb = row[k + o], rb = row[wrapi(k + o + 1, Hh)];
                const float2 ua = cs[ku * Hh + k], ub = cs[ku * Hh + k + 1];
                const float2 da = cs[kd * Hh + k], db = cs[kd * Hh + k + 1];
                float ta = own[y * Hh + k], tb = own[y * Hh + k + 1];
                float sa, ca, sb, cb;
                sincos_turn(ta, sa, ca);
                sincos_turn(tb, sb, cb);
                const u32x4 r = philox10(sweep, (uint32_t)c, 0u, (uint32_t)y * (uint32_t)P + (uint32_t)jj, k0, k1);
                acc += site_update<T>(ta, ca, sa, nsum(la.x, ra.x, ua.x, da.x), nsum(la.y, ra.y, ua.y, da.y), r.x, r.y,
                                      p);
                acc += site_update<T>(tb, cb, sb, nsum(lb.x, rb.x, ub.x, db.x), nsum(lb.y, rb.y, ub.y, db.y), r.z, r.w,
                                      p);
                own[y * Hh + k] = ta;
                own[y * Hh + k + 1] = tb;
                if (c == 1 && meas) {
                    meas_acc(m, ca, sa, la, ra, ua, da);
                    meas_acc(m, cb, sb, lb, rb, ub, db);
                }
            }
            __syncthreads();
        }
        if (meas) {
            double v[7] = {(double)m.cx, (double)m.cy, (double)m.ix, (double)m.iy, (double)m.mx, (double)m.my,
                           (double)acc};
#pragma unroll
            for (int q = 0; q < 7; ++q) v[q] = wave_sum(v[q]);
            if (lane == 0)
#pragma unroll
                for (int q = 0; q < 7; ++q) red[wid * 7 + q] = v[q];
            __syncthreads();
            if (tid == 0) {
                double s[7];
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    s[q] = 0.0;
                    for (int w = 0; w < NT / 64; ++w) s[q] += red[w * 7 + q];
                }
                xy_obs rec;
                rec.sweep = (uint64_t)sweep + 1u;
                rec.n_accept = (uint64_t)s[6];
                rec.cx = s[0]; rec.cy = s[1]; rec.ix = s[2]; rec.iy = s[3]; rec.mx = s[4]; rec.my = s[5];
                obs[j / me - 1] = rec;
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < 2 * half; i += NT) dst[i] = store<T>::st(ang[i]);
}

}  // namespace xyd
