// xy_tile.hpp -- one LDS-resident tile of a fused checkerboard sweep.
//
// A workgroup loads a TX x TY tile of both half-lattices plus a halo of 2M sites
// (periodic wrap) from `src`, converts every loaded angle to (cos, sin) once,
// then runs M sweeps (red, black, red, black, ...) entirely in LDS and writes the
// TX x TY interior to `dst` (the other buffer of a ping-pong pair, so that
// neighbouring tiles still read the old halo).  Sub-sweep j updates the red sites
// of the tile grown by e_r = 2(M - j) - 1 sites and the black sites grown by
// e_b = 2(M - j - 1): the halo sites are recomputed with the random numbers of
// their owners, from the same inputs, so the result equals the two-launch
// schedule bit for bit.  Bytes moved per sweep and site: (1 + halo) * 4 read,
// 4 written (FP32 storage), against 12 for two in-place half-sweep passes.
#pragma once

#include "xy_device.hpp"

namespace xyd {

template <int TX, int TY, int M, int NT>
struct TileShape {
    static_assert(TX % 4 == 0, "tile_x must hold whole Philox pairs");
    static constexpr int H = 2 * M;             // halo width in sites
    static constexpr int W = TX / 2 + 2 * M;    // LDS half-row width (entries per colour)
    static constexpr int R = TY + 2 * H;        // LDS rows
    static constexpr int PLANE = R * W;
    static constexpr size_t lds_bytes =
        (size_t)2 * PLANE * (sizeof(float2) + sizeof(float));
    static constexpr size_t red_bytes = (size_t)(NT / 64) * 7 * sizeof(double);
};

__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Sum 7 values over the workgroup (fixed order); thread 0 receives the totals.
template <int NT>
__device__ __forceinline__ void tile_block_sum7(double v[7], double* red)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 7; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 7; ++q) red[wid * 7 + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            double t = 0.0;
            for (int w = 0; w < NT / 64; ++w) t += red[w * 7 + q];
            v[q] = t;
        }
    }
    __syncthreads();
}

// Update every site of colour `col` in the tile grown by e.  Returns the number
// of accepted updates inside the tile interior (what the owner counts).
template <typename T, int TX, int TY, int M, int NT>
__device__ __forceinline__ int tile_half(float2* __restrict__ cs, float* __restrict__ th, int col, int e,
                                         int L, int x0, int y0, uint32_t sweep, uint32_t k0, uint32_t k1,
                                         const Params& p)
{
    using S = TileShape<TX, TY, M, NT>;
    const int Hh = L >> 1, P = Hh >> 1;
    const int kb = x0 >> 1;
    const int slots = TX / 4 + (e == 0 ? 0 : (e == 1 ? 1 : 2));
    const int rows = TY + 2 * e;
    float2* ocs = cs + col * S::PLANE;
    float* oth = th + col * S::PLANE;
    const float2* ncs = cs + (1 - col) * S::PLANE;
    int acc = 0;
    for (int idx = threadIdx.x; idx < rows * slots; idx += NT) {
        const int rr = idx / slots;
        const int sl = idx - rr * slots;
        const int y = y0 - e + rr;                          // unwrapped row
        const int o = (col + y) & 1;
        const int klo = kb - ((e + o) >> 1);
        const int khi = kb + TX / 2 + ((e - 1 - o) >> 1);
        const int j = (klo >> 1) + sl;                      // pair of entries 2j, 2j+1
        if (2 * j > khi) continue;
        const int yw = wrap1(y, L), jw = wrap1(j, P);
        const u32x4 r = philox10(sweep, (uint32_t)col, 0u, (uint32_t)(yw * P + jw), k0, k1);
        const int lr = y - (y0 - S::H);
        const bool row_in = (y >= y0) && (y < y0 + TY);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int k = 2 * j + q;
            if (k < klo || k > khi) continue;
            const int kr = k - (kb - M);
            const int i = lr * S::W + kr;
            const float2 l = ncs[i + o - 1], rt = ncs[i + o], u = ncs[i - S::W], d = ncs[i + S::W];
            float t = oth[i];
            float2 own = ocs[i];
            const int a = site_update<T>(t, own.x, own.y, nsum(l.x, rt.x, u.x, d.x), nsum(l.y, rt.y, u.y, d.y),
                                         q ? r.z : r.x, q ? r.w : r.y, p);
            oth[i] = t;
            ocs[i] = own;
            if (row_in && k >= kb && k < kb + TX / 2) acc += a;
        }
    }
    __syncthreads();
    return acc;
}

// FP64 observables of the tile interior after a completed sweep (black-owned
// bonds), plus the interior accept count `acc`, summed over the workgroup into
// out[0..7) on thread 0: Cx, Cy, Ix, Iy, Mx, My, accepts.
template <int TX, int TY, int M, int NT>
__device__ __forceinline__ void tile_measure(const float2* __restrict__ cs, int y0, int acc, double* red, double out[7])
{
    using S = TileShape<TX, TY, M, NT>;
    const float2* rcs = cs;
    const float2* bcs = cs + S::PLANE;
    double v[7] = {0, 0, 0, 0, 0, 0, (double)acc};
    for (int idx = threadIdx.x; idx < TY * (TX / 4); idx += NT) {
        const int rr = idx / (TX / 4);
        const int sl = idx - rr * (TX / 4);
        const int o = (1 + y0 + rr) & 1;
        const int lr = rr + S::H;
        Meas m{0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int kr = 2 * sl + q + M;
            const int i = lr * S::W + kr;
            const float2 b = bcs[i], l = rcs[i + o - 1], r = rcs[i + o], u = rcs[i - S::W], d = rcs[i + S::W];
            meas_black(m, b.x, b.y, l.x, l.y, r.x, r.y, u.x, u.y, d.x, d.y);
        }
        v[0] += (double)m.cx; v[1] += (double)m.cy; v[2] += (double)m.ix;
        v[3] += (double)m.iy; v[4] += (double)m.mx; v[5] += (double)m.my;
    }
    tile_block_sum7<NT>(v, red);
#pragma unroll
    for (int q = 0; q < 7; ++q) out[q] = v[q];
}

// Full tile program: load, M sweeps, optional measurements, write back.
// If bit j of meas_mask is set, part[j * part_stride .. +8) receives the tile's
// partial sums after sub-sweep j: Cx, Cy, Ix, Iy, Mx, My, interior accepts, 0.
// `red` is workgroup scratch of 7 doubles per wave.
template <typename T, int TX, int TY, int M, int NT>
__device__ __forceinline__ void tile_program(const T* __restrict__ src, T* __restrict__ dst, int L, int x0, int y0,
                                             uint32_t sweep0, uint32_t k0, uint32_t k1, const Params& p,
                                             unsigned meas_mask, double* part, size_t part_stride, char* smem,
                                             double* red)
{
    using S = TileShape<TX, TY, M, NT>;
    float2* cs = (float2*)smem;
    float* th = (float*)(cs + 2 * S::PLANE);
    const int Hh = L >> 1;
    const int kb = x0 >> 1;

    for (int idx = threadIdx.x; idx < 2 * S::PLANE; idx += NT) {
        const int c = idx / S::PLANE;
        const int rem = idx - c * S::PLANE;
        const int r = rem / S::W;
        const int w = rem - r * S::W;
        const int y = wrap1(y0 - S::H + r, L);
        const int k = wrap1(kb - M + w, Hh);
        const float t = store<T>::ld(src[((size_t)c * L + y) * Hh + k]);
        float s_, c_;
        sincos_turn(t, s_, c_);
        th[idx] = t;
        cs[idx] = make_float2(c_, s_);
    }
    __syncthreads();

#pragma unroll
    for (int js = 0; js < M; ++js) {
        const uint32_t sweep = sweep0 + (uint32_t)js;
        int acc = tile_half<T, TX, TY, M, NT>(cs, th, 0, 2 * (M - js) - 1, L, x0, y0, sweep, k0, k1, p);
        acc += tile_half<T, TX, TY, M, NT>(cs, th, 1, 2 * (M - js - 1), L, x0, y0, sweep, k0, k1, p);
        if (meas_mask & (1u << js)) {
            double v[7];
            tile_measure<TX, TY, M, NT>(cs, y0, acc, red, v);
            if (threadIdx.x == 0) {
                double* o = part + (size_t)js * part_stride;
#pragma unroll
                for (int q = 0; q < 7; ++q) o[q] = v[q];
                o[7] = 0.0;
            }
        }
    }

    for (int idx = threadIdx.x; idx < 2 * TY * (TX / 2); idx += NT) {
        const int c = idx / (TY * (TX / 2));
        const int rem = idx - c * (TY * (TX / 2));
        const int rr = rem / (TX / 2);
        const int w = rem - rr * (TX / 2);
        dst[((size_t)c * L + y0 + rr) * Hh + kb + w] = store<T>::st(th[c * S::PLANE + (rr + S::H) * S::W + w + M]);
    }
}

}  // namespace xyd
