// xy_tile1.hpp -- one fused sweep of one tile, register-resident angles, (cos, sin) in LDS.
//
// The single-sweep (M = 1) form of the tile program.  For a TX x TY tile at
// (x0, y0), kb = x0 / 2:
//   * black entries of rows y0-2 .. y0+TY+1 and red entries of rows y0-1 .. y0+TY,
//     columns kb-1 .. kb+TX/2, are what the sweep reads (the red ones of the outer
//     ring are recomputed with their owners' random numbers);
//   * every angle is loaded from HBM exactly once, as aligned pairs (entries 2j,
//     2j+1 of a half-row, the two sites of one Philox call) plus one column of
//     single entries on each side;
//   * a thread keeps the angles of the pairs it loads in registers and updates
//     those same pairs, so angles never pass through LDS; LDS holds only
//     (cos, sin) per entry, read as 16-byte pairs;
//   * updated angles go straight from registers to the destination buffer, and
//     the measurement of a measured sweep is folded into the black update.
// The arithmetic of every site update is xyd::site_update with the neighbour
// sums in the order (left + right) + (up + down), as in every other kernel.
#pragma once

#include "xy_device.hpp"

namespace xyd {

template <typename T> struct pair_io;
template <> struct pair_io<float> {
    using P = float2;
    static __device__ __forceinline__ float2 ld(const float* p) { return *(const float2*)p; }
    static __device__ __forceinline__ void st(float* p, float a, float b) { *(float2*)p = make_float2(a, b); }
};
template <> struct pair_io<__half> {
    using P = __half2;
    static __device__ __forceinline__ float2 ld(const __half* p)
    {
        const __half2 h = *(const __half2*)p;
        return make_float2(__low2float(h), __high2float(h));
    }
    static __device__ __forceinline__ void st(__half* p, float a, float b)
    {
        *(__half2*)p = __floats2half2_rn(a, b);
    }
};

template <int TX, int TY, int NT>
struct Tile1 {
    static_assert(TX >= 4 && (TX & (TX - 1)) == 0, "tile_x must be a power of two >= 4");
    static constexpr int TQ = TX / 4;                 // Philox pairs per core half-row
    static constexpr int LGQ = __builtin_ctz(TQ);
    static constexpr int RR = TY + 2;                 // red rows y0-1 .. y0+TY
    static constexpr int RB = TY + 4;                 // black rows y0-2 .. y0+TY+1
    static constexpr int WS = TX / 2 + 4;             // LDS row stride in (cos, sin) entries; col(k) = k - kb + 2
    static constexpr int NRED = RR * TQ;
    static constexpr int NPAIR = NRED + RB * TQ;
    static constexpr int NPI = (NPAIR + NT - 1) / NT;  // pair items per thread
    static constexpr int NEDGE = RR + 2 * RB;          // red: the one needed side per row; black: both
    static_assert(NEDGE <= NT, "edge column must fit one pass");
    static constexpr int BLACK0 = RR * WS;             // black plane offset in LDS entries
    static constexpr size_t lds_bytes = (size_t)(RR + RB) * WS * sizeof(float2);
    static constexpr size_t red_bytes = (size_t)(NT / 64) * 7 * sizeof(double);
};

// 7-value workgroup sum in a fixed order; thread 0 receives the totals.
template <int NT>
__device__ __forceinline__ void block_sum7(double v[7], double* red)
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

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Neighbour (cos, sin) of the two entries of a pair at LDS column c0 (even) of
// the other colour's row `row`: h = entries c0, c0+1 (one 16-byte read), side =
// entry c0-1 (o = 0) or c0+2 (o = 1).
struct PairNb {
    float2 la, ra, lb, rb, ua, ub, da, db;
};

__device__ __forceinline__ PairNb pair_neighbours(const float2* __restrict__ plane, int WS, int row, int c0, int o)
{
    const float4 h = *(const float4*)&plane[row * WS + c0];
    const float2 side = plane[row * WS + (o ? c0 + 2 : c0 - 1)];
    const float4 u = *(const float4*)&plane[(row - 1) * WS + c0];
    const float4 d = *(const float4*)&plane[(row + 1) * WS + c0];
    const float2 hl = make_float2(h.x, h.y), hh = make_float2(h.z, h.w);
    PairNb n;
    n.la = o ? hl : side;
    n.ra = o ? hh : hl;
    n.lb = o ? hh : hl;
    n.rb = o ? side : hh;
    n.ua = make_float2(u.x, u.y);
    n.ub = make_float2(u.z, u.w);
    n.da = make_float2(d.x, d.y);
    n.db = make_float2(d.z, d.w);
    return n;
}

template <typename T, int TX, int TY, int NT>
__device__ __forceinline__ void tile1_program(const T* __restrict__ src, T* __restrict__ dst, int L, int x0, int y0,
                                              uint32_t sweep, uint32_t k0, uint32_t k1, const Params& p, bool meas,
                                              double* part, char* smem, double* red)
{
    using S = Tile1<TX, TY, NT>;
    float2* cs = (float2*)smem;
    const int tid = threadIdx.x;
    const int Hh = L >> 1, P = Hh >> 1;
    const int kb = x0 >> 1;

    // ---- load: all pair items and this thread's edge entry, loads issued first
    float2 th[S::NPI];
#pragma unroll
    for (int q = 0; q < S::NPI; ++q) {
        const int idx = q * NT + tid;
        if (idx < S::NPAIR) {
            const bool isred = idx < S::NRED;
            const int i2 = isred ? idx : idx - S::NRED;
            const int row = i2 >> S::LGQ, s = i2 & (S::TQ - 1);
            const int y = wrapi(isred ? y0 - 1 + row : y0 - 2 + row, L);
            const int c = isred ? 0 : 1;
            th[q] = pair_io<T>::ld(src + ((size_t)c * L + y) * Hh + kb + 2 * s);
        }
    }
    const int e = NT - 1 - tid;            // red edge entries land on the last wave
    float the = 0.0f;
    int e_row = 0, e_col = 0, e_red = 0, e_k = 0;
    if (e < S::NEDGE) {
        int yl, side;
        if (e < S::RR) {                   // red row y0-1+e: the side its ring update needs
            e_red = 1;
            e_row = e;
            yl = y0 - 1 + e;
            side = ((yl & 1) == 0);        // o = 0 -> right column, o = 1 -> left column
        } else {
            const int e2 = e - S::RR;
            e_row = e2 >> 1;
            yl = y0 - 2 + e_row;
            side = e2 & 1;
        }
        e_k = side ? kb + TX / 2 : kb - 1;
        e_col = side ? TX / 2 + 2 : 1;
        the = store<T>::ld(src[((size_t)(e_red ? 0 : 1) * L + wrapi(yl, L)) * Hh + wrapi(e_k, Hh)]);
    }
#pragma unroll
    for (int q = 0; q < S::NPI; ++q) {
        const int idx = q * NT + tid;
        if (idx < S::NPAIR) {
            const bool isred = idx < S::NRED;
            const int i2 = isred ? idx : idx - S::NRED;
            const int row = i2 >> S::LGQ, s = i2 & (S::TQ - 1);
            float sa, ca, sb, cb;
            sincos_rev(th[q].x, sa, ca);
            sincos_rev(th[q].y, sb, cb);
            *(float4*)&cs[(isred ? 0 : S::BLACK0) + row * S::WS + 2 * s + 2] = make_float4(ca, sa, cb, sb);
        }
    }
    if (e < S::NEDGE) {
        float s_, c_;
        sincos_rev(the, s_, c_);
        cs[(e_red ? 0 : S::BLACK0) + e_row * S::WS + e_col] = make_float2(c_, s_);
    }
    __syncthreads();

    // ---- red half-sweep: rows y0-1 .. y0+TY, columns kb-1 .. kb+TX/2 (ring of one)
    int acc = 0;
    const float2* blk = cs + S::BLACK0;
#pragma unroll
    for (int q = 0; q < S::NPI; ++q) {
        const int idx = q * NT + tid;
        if (idx < S::NRED) {
            const int row = idx >> S::LGQ, s = idx & (S::TQ - 1);
            const int y = y0 - 1 + row;
            const int o = y & 1;
            const int c0 = 2 * s + 2;
            const PairNb n = pair_neighbours(blk, S::WS, row + 1, c0, o);
            float4 own = *(const float4*)&cs[row * S::WS + c0];
            const u32x4 r = philox10((uint32_t)(wrapi(y, L) * P + (kb >> 1) + s), sweep, 0u, 0u, k0, k1);
            float ta = th[q].x, tb = th[q].y;
            const int aa = site_update<T>(ta, own.x, own.y, nsum(n.la.x, n.ra.x, n.ua.x, n.da.x),
                                          nsum(n.la.y, n.ra.y, n.ua.y, n.da.y), r.x, r.y, p);
            const int ab = site_update<T>(tb, own.z, own.w, nsum(n.lb.x, n.rb.x, n.ub.x, n.db.x),
                                          nsum(n.lb.y, n.rb.y, n.ub.y, n.db.y), r.z, r.w, p);
            *(float4*)&cs[row * S::WS + c0] = own;
            th[q] = make_float2(ta, tb);
            if (row >= 1 && row <= TY) {
                acc += aa + ab;
                pair_io<T>::st(dst + (size_t)y * Hh + kb + 2 * s, ta, tb);
            }
        }
    }
    if (e < S::NEDGE && e_red) {
        const int y = y0 - 1 + e_row;
        const int o = y & 1;
        const int j = e_k >> 1;            // e_k = kb-1 (odd: words 2, 3) or kb+TX/2 (even: words 0, 1)
        const u32x4 r = philox10((uint32_t)(wrapi(y, L) * P + wrapi(j, P)), sweep, 0u, 0u, k0, k1);
        const int b = e_row + 1;           // black row of the same y
        const float2 l = blk[b * S::WS + e_col + o - 1], rt = blk[b * S::WS + e_col + o];
        const float2 u = blk[(b - 1) * S::WS + e_col], d = blk[(b + 1) * S::WS + e_col];
        float2 own = cs[e_row * S::WS + e_col];
        const bool odd = (e_k & 1) != 0;
        site_update<T>(the, own.x, own.y, nsum(l.x, rt.x, u.x, d.x), nsum(l.y, rt.y, u.y, d.y), odd ? r.z : r.x,
                       odd ? r.w : r.y, p);
        cs[e_row * S::WS + e_col] = own;
    }
    __syncthreads();

    // ---- black half-sweep: interior rows y0 .. y0+TY-1 (black pair items of rows 2 .. TY+1)
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < S::NPI; ++q) {
        const int idx = q * NT + tid - S::NRED - 2 * S::TQ;
        if (idx >= 0 && idx < TY * S::TQ) {
            const int rr = idx >> S::LGQ, s = idx & (S::TQ - 1);   // interior row rr, black LDS row rr + 2
            const int y = y0 + rr;
            const int o = (y + 1) & 1;
            const int c0 = 2 * s + 2;
            const PairNb n = pair_neighbours(cs, S::WS, rr + 1, c0, o);
            const float4 own = *(const float4*)&blk[(rr + 2) * S::WS + c0];
            const u32x4 r = philox10((uint32_t)(y * P + (kb >> 1) + s), sweep, 1u, 0u, k0, k1);
            float ta = th[q].x, tb = th[q].y;
            float ca = own.x, sa = own.y, cb = own.z, sb = own.w;
            const int aa = site_update<T>(ta, ca, sa, nsum(n.la.x, n.ra.x, n.ua.x, n.da.x),
                                          nsum(n.la.y, n.ra.y, n.ua.y, n.da.y), r.x, r.y, p);
            const int ab = site_update<T>(tb, cb, sb, nsum(n.lb.x, n.rb.x, n.ub.x, n.db.x),
                                          nsum(n.lb.y, n.rb.y, n.ub.y, n.db.y), r.z, r.w, p);
            acc += aa + ab;
            pair_io<T>::st(dst + ((size_t)L + y) * Hh + kb + 2 * s, ta, tb);
            if (meas) {
                Meas t{0, 0, 0, 0, 0, 0};
                meas_black(t, ca, sa, n.la.x, n.la.y, n.ra.x, n.ra.y, n.ua.x, n.ua.y, n.da.x, n.da.y);
                meas_black(t, cb, sb, n.lb.x, n.lb.y, n.rb.x, n.rb.y, n.ub.x, n.ub.y, n.db.x, n.db.y);
                v[0] += (double)t.cx; v[1] += (double)t.cy; v[2] += (double)t.ix;
                v[3] += (double)t.iy; v[4] += (double)t.mx; v[5] += (double)t.my;
            }
        }
    }
    if (meas) {
        v[6] = (double)acc;
        block_sum7<NT>(v, red);
        if (tid == 0) {
#pragma unroll
            for (int q = 0; q < 7; ++q) part[q] = v[q];
            part[7] = 0.0;
        }
    }
}

}  // namespace xyd
