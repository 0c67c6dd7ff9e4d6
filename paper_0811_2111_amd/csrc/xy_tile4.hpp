// xy_tile4.hpp -- one fused sweep of one tile of a four-replica lattice.
//
// Four lattices of the same L (the replicas, each with its own seed, beta and
// delta) share one state array: entry (c, y, k) of the half-lattice layout is a
// float4 whose component r is replica r's angle (in turns).  One 16-byte load
// brings all four replicas of a site, and everything that depends only on the
// site -- addresses, tile geometry, the halo ring -- is computed once for four
// updates.  Replica r draws exactly the numbers a single lattice with seed_r
// draws (same counter, key = seed_r), so its trajectory is bit for bit that of
// the single lattice.
//
// The tile program is the single-replica one with a float4 where that one has a
// float: a thread owns the two sites of one Philox counter (entries 2j, 2j+1 of
// a half-row) and updates both for all four replicas (eight independent
// updates); LDS holds, per entry, the four cosines and the four sines, in four
// planes (see Lds4); the red sites of the ring around the tile are recomputed
// with their owners' random numbers.
#pragma once

#include "xy_tile1.hpp"

namespace xyd {

struct Params4 {
    float delta[4];     // proposal widths in turns
    float nbl2e[4];     // -beta log2(e)
    uint32_t k0[4], k1[4];
};

__device__ __forceinline__ float f4c(const float4& v, int r) { return r == 0 ? v.x : r == 1 ? v.y : r == 2 ? v.z : v.w; }
__device__ __forceinline__ void f4set(float4& v, int r, float x)
{
    if (r == 0) v.x = x;
    else if (r == 1) v.y = x;
    else if (r == 2) v.z = x;
    else v.w = x;
}

__device__ __forceinline__ float4 ld4(__amdgpu_buffer_rsrc_t rs, unsigned entry)
{
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, entry * 16u, 0, 0));
}
__device__ __forceinline__ void st4(__amdgpu_buffer_rsrc_t rs, unsigned entry, float4 v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), rs,
                                           entry * 16u, 0, 0);
}

// LDS entry: cosines and sines of the four replicas.
struct CS4 {
    float4 c, s;
};

template <int TX, int TY, int NT>
struct Tile4 {
    static_assert(TX >= 4 && (TX & (TX - 1)) == 0 && TX <= 128, "tile_x: power of two in [4, 128]");
    static_assert(NT % 128 == 0, "at least two waves");
    static constexpr int TQ = TX / 4;
    static constexpr int LGQ = __builtin_ctz(TQ);
    static constexpr int NW = NT / 64;
    static constexpr int RP = NT / TQ;
    static constexpr int RR = TY + 2;
    static constexpr int RB = TY + 4;
    static constexpr int NQR = (RR + RP - 1) / RP;
    static constexpr int NQB = (RB + RP - 1) / RP;
    static constexpr int WS = TX / 2 + 4;
    static constexpr int NEDGE = RR + 2 * RB;
    static_assert(NEDGE <= NT, "edge columns must fit one pass");
    static constexpr size_t lds_bytes = (size_t)(RR + RB) * WS * sizeof(CS4);
};

// LDS: four planes of float4 -- cosines of even entries, cosines of odd entries,
// sines of even entries, sines of odd entries -- each RR + RB rows of WS/2; red
// row r is LDS row r, black row r is LDS row RR + r.  A lane's entries 2s+2,
// 2s+3 and their neighbours sit at consecutive 16-byte slots across the lanes
// of a wave, so every 16-byte LDS access of a wave is contiguous.
template <typename S>
struct Lds4 {
    float4* p;
    static constexpr int WSH = S::WS / 2;
    static constexpr int PS = (S::RR + S::RB) * WSH;
    __device__ __forceinline__ CS4 get(int row, int col) const
    {
        const int i = row * WSH + (col >> 1), par = col & 1;
        CS4 v;
        v.c = p[par * PS + i];
        v.s = p[(2 + par) * PS + i];
        return v;
    }
    __device__ __forceinline__ void put(int row, int col, const CS4& v) const
    {
        const int i = row * WSH + (col >> 1), par = col & 1;
        p[par * PS + i] = v.c;
        p[(2 + par) * PS + i] = v.s;
    }
};

__device__ __forceinline__ CS4 sincos4(float4 t)
{
    CS4 o;
    sincos_turn(t.x, o.s.x, o.c.x);
    sincos_turn(t.y, o.s.y, o.c.y);
    sincos_turn(t.z, o.s.z, o.c.z);
    sincos_turn(t.w, o.s.w, o.c.w);
    return o;
}

// Update the two sites (a, b) of a pair for all four replicas.  la..db: the
// neighbours' LDS entries (left, right, up, down of a and of b); words w[r] of
// replica r: (x, y) drive site a, (z, w) site b.  Angles and (cos, sin) are
// updated in place; returns the accepted proposals of replica r in bits
// 8r .. 8r+7.
__device__ __forceinline__ int pair_update4(float4& ta, float4& tb, CS4& a, CS4& b, const CS4& la, const CS4& ra,
                                            const CS4& ua, const CS4& da, const CS4& lb, const CS4& rb,
                                            const CS4& ub, const CS4& db, const u32x4 (&w)[4], const Params4& p)
{
    int acc = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const Params pr{p.delta[r], p.nbl2e[r]};
        float t1 = f4c(ta, r), c1 = f4c(a.c, r), s1 = f4c(a.s, r);
        acc += site_update<float>(t1, c1, s1, nsum(f4c(la.c, r), f4c(ra.c, r), f4c(ua.c, r), f4c(da.c, r)),
                                  nsum(f4c(la.s, r), f4c(ra.s, r), f4c(ua.s, r), f4c(da.s, r)), w[r].x, w[r].y, pr)
               << (8 * r);
        f4set(ta, r, t1); f4set(a.c, r, c1); f4set(a.s, r, s1);
        float t2 = f4c(tb, r), c2 = f4c(b.c, r), s2 = f4c(b.s, r);
        acc += site_update<float>(t2, c2, s2, nsum(f4c(lb.c, r), f4c(rb.c, r), f4c(ub.c, r), f4c(db.c, r)),
                                  nsum(f4c(lb.s, r), f4c(rb.s, r), f4c(ub.s, r), f4c(db.s, r)), w[r].z, w[r].w, pr)
               << (8 * r);
        f4set(tb, r, t2); f4set(b.c, r, c2); f4set(b.s, r, s2);
    }
    return acc;
}

// Measurement accumulators of the four replicas (as MeasAcc, per replica).
struct MeasAcc4 {
    MeasAcc m[4];
};

__device__ __forceinline__ void meas_acc4(MeasAcc4& m, const CS4& b, const CS4& l, const CS4& r, const CS4& u,
                                          const CS4& d)
{
#pragma unroll
    for (int q = 0; q < 4; ++q)
        meas_acc(m.m[q], f4c(b.c, q), f4c(b.s, q), make_float2(f4c(l.c, q), f4c(l.s, q)),
                 make_float2(f4c(r.c, q), f4c(r.s, q)), make_float2(f4c(u.c, q), f4c(u.s, q)),
                 make_float2(f4c(d.c, q), f4c(d.s, q)));
}

// Red half-sweep; O = parity of this thread's red rows (left/right neighbours of
// entry k are the other colour's entries k + O - 1 and k + O).
template <int TX, int TY, int NT, int O, bool KEEP>
__device__ __forceinline__ int tile4_red(const T1Geom& g, Lds4<Tile4<TX, TY, NT>> cs, __amdgpu_buffer_rsrc_t src,
                                         __amdgpu_buffer_rsrc_t dst, uint32_t sweep, const Params4& p, float4 the,
                                         int e, int e_row, int e_col, int e_red, int e_k,
                                         const float4 (&tr)[Tile4<TX, TY, NT>::NQR][2])
{
    using S = Tile4<TX, TY, NT>;
    constexpr int FULL = TY / S::RP;
    const int c0 = 2 * g.s + 2;
    const unsigned jb = (unsigned)((g.kb >> 1) + g.s);
    int acc = 0;
#pragma unroll
    for (int q = 0; q < S::NQR; ++q) {
        if (!red_valid<S>(g, q)) continue;
        const int row = red_row<S>(g, q);
        const int y = g.y0 - 1 + row;
        const int yw = g.edge_tile ? wrapi(y, g.L) : y;
        const unsigned at = (unsigned)yw * (unsigned)g.Hh + (unsigned)(g.kb + 2 * g.s);
        // KEEP: the angles the fill loaded, kept in registers across the barrier;
        // else reloaded (an L2 hit), so no angles stay live across it
        float4 ta, tb;
        if constexpr (KEEP) {
            ta = tr[q][0];
            tb = tr[q][1];
        } else {
            ta = ld4(src, at);
            tb = ld4(src, at + 1u);
        }
        u32x4 w[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) w[r] = philox10(sweep, 0u, 0u, (uint32_t)yw * (uint32_t)g.P + jb, p.k0[r], p.k1[r]);
        const int nb = S::RR + row + 1;                   // black row of the same y
        const CS4 h0 = cs.get(nb, c0), h1 = cs.get(nb, c0 + 1);
        const CS4 side = cs.get(nb, O ? c0 + 2 : c0 - 1);
        const CS4 u0 = cs.get(nb - 1, c0), u1 = cs.get(nb - 1, c0 + 1);
        const CS4 d0 = cs.get(nb + 1, c0), d1 = cs.get(nb + 1, c0 + 1);
        CS4 a = cs.get(row, c0), b = cs.get(row, c0 + 1);
        const int ac = pair_update4(ta, tb, a, b, O ? h0 : side, O ? h1 : h0, u0, d0, O ? h1 : h0,
                                    O ? side : h1, u1, d1, w, p);
        cs.put(row, c0, a);
        cs.put(row, c0 + 1, b);
        if (q < FULL || (row >= 1 && row <= TY)) {     // halo rows only feed the black half-sweep
            acc += ac;
            st4(dst, at, ta);
            st4(dst, at + 1u, tb);
        }
        // eight updates per item are enough independent work; keeping the items
        // apart holds the live registers to one item's
        __builtin_amdgcn_sched_barrier(0);
    }
    if (e < S::NEDGE && e_red) {          // the one ring entry of red row e_row
        const int y = g.y0 - 1 + e_row;
        const int o = y & 1;
        const int j = e_k >> 1;
        const bool odd = (e_k & 1) != 0;
        const int bl = S::RR + e_row + 1;
        const CS4 l = cs.get(bl, e_col + o - 1), rt = cs.get(bl, e_col + o);
        const CS4 u = cs.get(bl - 1, e_col), d = cs.get(bl + 1, e_col);
        CS4 own = cs.get(e_row, e_col);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const u32x4 w = philox10(sweep, 0u, 0u, (uint32_t)wrapi(y, g.L) * (uint32_t)g.P + (uint32_t)wrapi(j, g.P),
                                     p.k0[r], p.k1[r]);
            const Params pr{p.delta[r], p.nbl2e[r]};
            float t = f4c(the, r), c = f4c(own.c, r), s = f4c(own.s, r);
            site_update<float>(t, c, s, nsum(f4c(l.c, r), f4c(rt.c, r), f4c(u.c, r), f4c(d.c, r)),
                               nsum(f4c(l.s, r), f4c(rt.s, r), f4c(u.s, r), f4c(d.s, r)), odd ? w.z : w.x,
                               odd ? w.w : w.y, pr);
            f4set(own.c, r, c); f4set(own.s, r, s);
        }
        cs.put(e_row, e_col, own);
    }
    return acc;
}

// Black half-sweep of the interior rows; O = parity of this thread's black rows.
template <int TX, int TY, int NT, int O, bool MEAS, bool KEEP>
__device__ __forceinline__ int tile4_black(const T1Geom& g, Lds4<Tile4<TX, TY, NT>> cs, __amdgpu_buffer_rsrc_t src,
                                           __amdgpu_buffer_rsrc_t dst, uint32_t sweep, const Params4& p, MeasAcc4& m,
                                           const float4 (&tb)[Tile4<TX, TY, NT>::NQB][2])
{
    using S = Tile4<TX, TY, NT>;
    constexpr int FULL = TY / S::RP;
    const int c0 = 2 * g.s + 2;
    const unsigned jb = (unsigned)((g.kb >> 1) + g.s);
    int acc = 0;
#pragma unroll
    for (int q = 0; q < S::NQB; ++q) {
        const int row = black_row<S>(g, q);
        if (!(q < FULL || (black_valid<S>(g, q) && row >= 2 && row < TY + 2))) continue;
        const int y = g.y0 - 2 + row;      // interior: never wraps
        const unsigned at = ((unsigned)g.L + (unsigned)y) * (unsigned)g.Hh + (unsigned)(g.kb + 2 * g.s);
        float4 t0, t1;
        if constexpr (KEEP) {
            t0 = tb[q][0];
            t1 = tb[q][1];
        } else {
            t0 = ld4(src, at);
            t1 = ld4(src, at + 1u);
        }
        u32x4 w[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) w[r] = philox10(sweep, 1u, 0u, (uint32_t)y * (uint32_t)g.P + jb, p.k0[r], p.k1[r]);
        const int nr = row - 1;                           // red row of the same y
        const CS4 h0 = cs.get(nr, c0), h1 = cs.get(nr, c0 + 1);
        const CS4 side = cs.get(nr, O ? c0 + 2 : c0 - 1);
        const CS4 u0 = cs.get(nr - 1, c0), u1 = cs.get(nr - 1, c0 + 1);
        const CS4 d0 = cs.get(nr + 1, c0), d1 = cs.get(nr + 1, c0 + 1);
        CS4 a = cs.get(S::RR + row, c0), b = cs.get(S::RR + row, c0 + 1);
        const CS4 la = O ? h0 : side, ra = O ? h1 : h0, lb = O ? h1 : h0, rb = O ? side : h1;
        acc += pair_update4(t0, t1, a, b, la, ra, u0, d0, lb, rb, u1, d1, w, p);
        st4(dst, at, t0);
        st4(dst, at + 1u, t1);
        if constexpr (MEAS) {
            meas_acc4(m, a, la, ra, u0, d0);
            meas_acc4(m, b, lb, rb, u1, d1);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    return acc;
}

// One tile of a four-replica lattice; src/dst are the two float4 state buffers.
// MEAS: one partial record per wave and replica, replica-major:
// part[(r * rec_stride + wave) * 8 ..] = (Cx, Cy, Ix, Iy, Mx, My, accepts, 0)
// of replica r, `part` already offset to this tile's first wave.
template <int TX, int TY, int NT, bool MEAS>
__device__ __forceinline__ void tile4_program(const float4* __restrict__ src, float4* __restrict__ dst,
                                              unsigned state_bytes, int L, int x0, int y0, uint32_t sweep,
                                              const Params4& p, double* part, size_t rec_stride, char* smem)
{
    using S = Tile4<TX, TY, NT>;
    const Lds4<S> cs{(float4*)smem};
    const int tid = threadIdx.x;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, state_bytes);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(dst, state_bytes);

    T1Geom g;
    g.L = L;
    g.Hh = L >> 1;
    g.P = g.Hh >> 1;
    g.kb = x0 >> 1;
    g.x0 = x0;
    g.y0 = y0;
    {
        const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar row work
        g.s = lane & (S::TQ - 1);
        const int i = lane >> S::LGQ;
        g.rt = 2 * (i * (S::NW / 2) + (w >> 1)) + (w & 1);
    }
    g.edge_tile = (y0 < 2) || (y0 + TY + 2 > L);

    // fill: (cos, sin) of every loaded entry
    float4 tr[S::NQR][2], tb[S::NQB][2];
    const unsigned col = (unsigned)(g.kb + 2 * g.s);
#pragma unroll
    for (int q = 0; q < S::NQR; ++q) {
        if (red_valid<S>(g, q)) {
            const int yr = y0 - 1 + red_row<S>(g, q);
            const unsigned base = (unsigned)(g.edge_tile ? wrapi(yr, L) : yr) * (unsigned)g.Hh + col;
            tr[q][0] = ld4(rs, base);
            tr[q][1] = ld4(rs, base + 1u);
        }
    }
#pragma unroll
    for (int q = 0; q < S::NQB; ++q) {
        if (black_valid<S>(g, q)) {
            const int yb = y0 - 2 + black_row<S>(g, q);
            const unsigned base = ((unsigned)L + (unsigned)(g.edge_tile ? wrapi(yb, L) : yb)) * (unsigned)g.Hh + col;
            tb[q][0] = ld4(rs, base);
            tb[q][1] = ld4(rs, base + 1u);
        }
    }
    const int e = NT - 1 - tid;
    float4 the = make_float4(0.f, 0.f, 0.f, 0.f);
    int e_row = 0, e_col = 0, e_red = 0, e_k = 0;
    if (e < S::NEDGE) {
        int yl, side;
        if (e < S::RR) {
            e_red = 1;
            e_row = e;
            yl = y0 - 1 + e;
            side = ((yl & 1) == 0);
        } else {
            const int e2 = e - S::RR;
            e_row = e2 >> 1;
            yl = y0 - 2 + e_row;
            side = e2 & 1;
        }
        e_k = side ? g.kb + TX / 2 : g.kb - 1;
        e_col = side ? TX / 2 + 2 : 1;
        the = ld4(rs, ((unsigned)(e_red ? 0 : L) + (unsigned)wrapi(yl, L)) * (unsigned)g.Hh +
                          (unsigned)wrapi(e_k, g.Hh));
    }
#pragma unroll
    for (int q = 0; q < S::NQR; ++q)
        if (red_valid<S>(g, q)) {
            const int row = red_row<S>(g, q);
            cs.put(row, 2 * g.s + 2, sincos4(tr[q][0]));
            cs.put(row, 2 * g.s + 3, sincos4(tr[q][1]));
        }
#pragma unroll
    for (int q = 0; q < S::NQB; ++q)
        if (black_valid<S>(g, q)) {
            const int row = black_row<S>(g, q);
            cs.put(S::RR + row, 2 * g.s + 2, sincos4(tb[q][0]));
            cs.put(S::RR + row, 2 * g.s + 3, sincos4(tb[q][1]));
        }
    if (e < S::NEDGE) cs.put((e_red ? 0 : S::RR) + e_row, e_col, sincos4(the));
    __syncthreads();

    // The unmeasured sweep keeps the loaded angles in registers through both
    // phases: the tile's LDS already limits a CU to three workgroups, i.e. three
    // waves per SIMD, so registers up to 168 per lane cost no occupancy, and the
    // updates then wait on no reload.  The measured sweep, with its sums, has no
    // registers to spare and reloads them.
    constexpr bool KEEP = !MEAS;
    MeasAcc4 m;
    int acc = 0;
    const bool red_odd = __builtin_amdgcn_readfirstlane((y0 + g.rt) & 1) != 0;
    if (red_odd)
        acc += tile4_red<TX, TY, NT, 1, KEEP>(g, cs, rs, rd, sweep, p, the, e, e_row, e_col, e_red, e_k, tr);
    else
        acc += tile4_red<TX, TY, NT, 0, KEEP>(g, cs, rs, rd, sweep, p, the, e, e_row, e_col, e_red, e_k, tr);
    __syncthreads();
    if (red_odd)
        acc += tile4_black<TX, TY, NT, 0, MEAS, KEEP>(g, cs, rs, rd, sweep, p, m, tb);
    else
        acc += tile4_black<TX, TY, NT, 1, MEAS, KEEP>(g, cs, rs, rd, sweep, p, m, tb);
    if constexpr (MEAS) {
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double v[7] = {(double)m.m[r].cx, (double)m.m[r].cy, (double)m.m[r].ix, (double)m.m[r].iy,
                           (double)m.m[r].mx, (double)m.m[r].my, (double)((acc >> (8 * r)) & 0xff)};
#pragma unroll
            for (int q = 0; q < 7; ++q) v[q] = wave_sum_last(v[q]);
            if (lane == 63) {
                double* w = part + ((size_t)r * rec_stride + (size_t)wv) * 8;
#pragma unroll
                for (int q = 0; q < 7; ++q) w[q] = v[q];
                w[7] = 0.0;
            }
        }
    }
}

}  // namespace xyd
