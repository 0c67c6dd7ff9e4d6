// xy_tile1.hpp -- one fused sweep of one tile, register-resident angles, (cos, sin) in LDS.
//
// The single-sweep form of the tile program.  For a TX x TY tile at (x0, y0),
// kb = x0 / 2:
//   * the sweep reads black entries of rows y0-2 .. y0+TY+1 and red entries of
//     rows y0-1 .. y0+TY, columns kb-1 .. kb+TX/2 (the red ones of the outer ring
//     are recomputed with their owners' random numbers, so the tile needs no
//     other tile's results);
//   * every angle is loaded once, as aligned pairs (entries 2j, 2j+1 of a
//     half-row, the two sites of one Philox call) plus a column of single
//     entries on each side;
//   * the thread that loads a pair keeps its angles in registers and updates it,
//     so angles never pass through LDS; LDS holds (cos, sin) per entry, read as
//     16-byte pairs;
//   * lanes are laid out so that all rows a wave touches have the same parity:
//     the position of a site's horizontal neighbours in the other half-lattice
//     depends only on that parity, so a whole wave takes one branch and needs no
//     per-lane selects;
//   * global traffic uses buffer instructions with 32-bit offsets (the state must
//     be below 4 GiB), updated angles go straight from registers to the
//     destination, and a measured sweep folds its sums into the black update.
// Every site update is xyd::site_update with neighbour sums in the order
// (left + right) + (up + down), as in every other kernel.
#pragma once

#include "xy_device.hpp"

namespace xyd {

typedef unsigned int xu2 __attribute__((ext_vector_type(2)));

// Loads and stores of the state.  ST = true sets the non-temporal hint (cache
// policy bit NT): the L2 keeps such lines only briefly, so a kernel that streams
// a lattice larger than the caches through once per sweep does not push out the
// lines it means to reuse (a strip's edge columns, a tile's halo rows).
constexpr int kCpolNT = 2;

template <typename T> struct bio;
template <> struct bio<float> {
    template <bool ST = false>
    static __device__ __forceinline__ float2 ld2(__amdgpu_buffer_rsrc_t r, unsigned off_elems)
    {
        const xu2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off_elems * 4u, 0, ST ? kCpolNT : 0);
        return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
    }
    static __device__ __forceinline__ float ld1(__amdgpu_buffer_rsrc_t r, unsigned off_elems)
    {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off_elems * 4u, 0, 0));
    }
    template <bool ST = false>
    static __device__ __forceinline__ void st2(__amdgpu_buffer_rsrc_t r, unsigned off_elems, float a, float b)
    {
        xu2 v;
        v.x = __float_as_uint(a);
        v.y = __float_as_uint(b);
        __builtin_amdgcn_raw_buffer_store_b64(v, r, off_elems * 4u, 0, ST ? kCpolNT : 0);
    }
    static constexpr unsigned bytes = 4;
};
template <> struct bio<__half> {
    template <bool ST = false>
    static __device__ __forceinline__ float2 ld2(__amdgpu_buffer_rsrc_t r, unsigned off_elems)
    {
        const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, off_elems * 2u, 0, ST ? kCpolNT : 0);
        return make_float2(__half2float(__ushort_as_half((unsigned short)(v & 0xffffu))),
                           __half2float(__ushort_as_half((unsigned short)(v >> 16))));
    }
    static __device__ __forceinline__ float ld1(__amdgpu_buffer_rsrc_t r, unsigned off_elems)
    {
        const unsigned short v = __builtin_amdgcn_raw_buffer_load_b16(r, off_elems * 2u, 0, 0);
        return __half2float(__ushort_as_half(v));
    }
    template <bool ST = false>
    static __device__ __forceinline__ void st2(__amdgpu_buffer_rsrc_t r, unsigned off_elems, float a, float b)
    {
        const unsigned v = (unsigned)__half_as_ushort(__float2half_rn(a)) |
                           ((unsigned)__half_as_ushort(__float2half_rn(b)) << 16);
        __builtin_amdgcn_raw_buffer_store_b32(v, r, off_elems * 2u, 0, ST ? kCpolNT : 0);
    }
    static constexpr unsigned bytes = 2;
};

// Raw buffer resource over `bytes` bytes at `base` (gfx9 descriptor word 3).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <int TX, int TY, int NT>
struct Tile1 {
    static_assert(TX >= 4 && (TX & (TX - 1)) == 0 && TX <= 256, "tile_x: power of two in [4, 256]");
    static_assert(NT % 128 == 0, "at least two waves");
    static constexpr int TQ = TX / 4;                  // Philox pairs per core half-row
    static constexpr int LGQ = __builtin_ctz(TQ);
    static constexpr int NW = NT / 64;                 // waves
    static constexpr int RP = NT / TQ;                 // rows covered by one pass of the workgroup
    static constexpr int RR = TY + 2;                  // red rows y0-1 .. y0+TY
    static constexpr int RB = TY + 4;                  // black rows y0-2 .. y0+TY+1
    static constexpr int NQR = (RR + RP - 1) / RP;     // red pair items per thread
    static constexpr int NQB = (RB + RP - 1) / RP;     // black pair items per thread
    static constexpr int WS = TX / 2 + 4;              // LDS row stride in (cos, sin) entries; col(k) = k - kb + 2
    static constexpr int NEDGE = RR + 2 * RB;          // red: the one needed side per row; black: both
    static_assert(NEDGE <= NT, "edge columns must fit one pass");
    static constexpr int BLACK0 = RR * WS;             // black plane offset in LDS entries
    static constexpr size_t lds_bytes = (size_t)(RR + RB) * WS * sizeof(float2);
    static constexpr size_t red_bytes = (size_t)NW * 7 * sizeof(double);
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

// Neighbours of the pair at LDS column c0 (even) in the other colour's row `row`.
// O = row parity of the updated sites: left/right neighbours of entry k are the
// other colour's entries k + O - 1 and k + O.
template <int O>
struct PairNb {
    float2 la, ra, lb, rb, ua, ub, da, db;
    PairNb() = default;
    __device__ __forceinline__ PairNb(const float2* __restrict__ plane, int WS, int row, int c0)
    {
        const float4 h = *(const float4*)&plane[row * WS + c0];
        const float2 side = plane[row * WS + (O ? c0 + 2 : c0 - 1)];
        const float4 u = *(const float4*)&plane[(row - 1) * WS + c0];
        const float4 d = *(const float4*)&plane[(row + 1) * WS + c0];
        const float2 hl = make_float2(h.x, h.y), hh = make_float2(h.z, h.w);
        la = O ? hl : side;
        ra = O ? hh : hl;
        lb = O ? hh : hl;
        rb = O ? side : hh;
        ua = make_float2(u.x, u.y);
        ub = make_float2(u.z, u.w);
        da = make_float2(d.x, d.y);
        db = make_float2(d.z, d.w);
    }
};

struct MeasAcc {
    float cx = 0.f, cy = 0.f, ix = 0.f, iy = 0.f, mx = 0.f, my = 0.f;
};

// A black site's four bonds from the neighbour sums the update already formed:
//   cos(tl - tb) + cos(tb - tr) = cb (cl + cr) + sb (sl + sr)
//   sin(tl - tb) + sin(tb - tr) = cb (sl - sr) + sb (cr - cl)
// and the same with up/down for the y bonds; plus its own spin and that of the red
// site to its right.
// Each bond term goes into the FP32 accumulator as two fused multiply-adds; the
// sums l + r and u + d are the ones the update's neighbour sums already formed.
__device__ __forceinline__ void meas_acc(MeasAcc& m, float cb, float sb, float2 l, float2 r, float2 u, float2 d)
{
    m.cx = __fmaf_rn(sb, __fadd_rn(l.y, r.y), __fmaf_rn(cb, __fadd_rn(l.x, r.x), m.cx));
    m.cy = __fmaf_rn(sb, __fadd_rn(u.y, d.y), __fmaf_rn(cb, __fadd_rn(u.x, d.x), m.cy));
    m.ix = __fmaf_rn(sb, __fsub_rn(r.x, l.x), __fmaf_rn(cb, __fsub_rn(l.y, r.y), m.ix));
    m.iy = __fmaf_rn(sb, __fsub_rn(d.x, u.x), __fmaf_rn(cb, __fsub_rn(u.y, d.y), m.iy));
    m.mx = __fadd_rn(__fadd_rn(m.mx, cb), r.x);
    m.my = __fadd_rn(__fadd_rn(m.my, sb), r.y);
}

// Running sums of a measured sweep, made to exist in registers at this point.
// Without it the compiler sinks the bond arithmetic of a step past the step
// boundary, keeping that step's neighbour (cos, sin) live across the next
// step's updates: the measured strip kernel then needs 133 VGPRs (three waves
// per SIMD) instead of 84 (five).
__device__ __forceinline__ void pin_sums(int& acc) { asm volatile("" : "+v"(acc)); }
__device__ __forceinline__ void pin_sums(MeasAcc& m, int& acc)
{
    asm volatile("" : "+v"(m.cx), "+v"(m.cy), "+v"(m.ix), "+v"(m.iy), "+v"(m.mx), "+v"(m.my), "+v"(acc));
}

// Per-thread geometry shared by both phases.
//
// Work items are pairs of a core half-row.  A pass of the workgroup covers RP
// rows; item q of a thread lies in row 1 + q*RP + rt of the red plane (rows
// wrap: RR -> 0) and in row 2 + q*RP + rt of the black plane (RB, RB+1 -> 0, 1).
// So the first TY/RP passes cover exactly the tile interior and need no bounds
// test (their Philox chains share one basic block and interleave), and only the
// last pass carries the halo rows.  rt has the parity of the wave, so every row a
// wave touches in one plane has the same parity.
struct T1Geom {
    int L, Hh, P, kb, y0, x0;
    int s;           // pair slot within a core half-row
    int rt;          // row offset of this thread within a pass
    bool edge_tile;  // rows wrap around the lattice
};

template <typename S> __device__ __forceinline__ bool red_valid(const T1Geom& g, int q)
{
    return q < S::RR / S::RP || q * S::RP + g.rt < S::RR;
}
template <typename S> __device__ __forceinline__ int red_row(const T1Geom& g, int q)
{
    const int r = 1 + q * S::RP + g.rt;
    return (q < S::RR / S::RP - 1 || r < S::RR) ? r : r - S::RR;
}
template <typename S> __device__ __forceinline__ bool black_valid(const T1Geom& g, int q)
{
    return q < S::RB / S::RP || q * S::RP + g.rt < S::RB;
}
template <typename S> __device__ __forceinline__ int black_row(const T1Geom& g, int q)
{
    const int r = 2 + q * S::RP + g.rt;
    return (q < S::RB / S::RP - 1 || r < S::RB) ? r : r - S::RB;
}

// Red half-sweep (rows y0-1 .. y0+TY, columns kb-1 .. kb+TX/2); O = parity of this
// thread's red rows.
template <typename T, int TX, int TY, int NT, int O, bool ST>
__device__ __forceinline__ void tile1_red(const T1Geom& g, float2* __restrict__ cs, float2 (&thr)[Tile1<TX, TY, NT>::NQR],
                                          __amdgpu_buffer_rsrc_t dst, uint32_t sweep, uint32_t k0, uint32_t k1,
                                          const Params& p, float the, int e, int e_row, int e_col, int e_red, int e_k,
                                          int& acc)
{
    using S = Tile1<TX, TY, NT>;
    constexpr int FULL = TY / S::RP;           // passes entirely inside rows 1 .. TY
    const float2* blk = cs + S::BLACK0;
    const int c0 = 2 * g.s + 2;
    const unsigned jb = (unsigned)((g.kb >> 1) + g.s);
    // All of this thread's Philox calls first: independent ten-round chains the
    // scheduler interleaves (the interior passes share one basic block).
    u32x4 rr[S::NQR];
#pragma unroll
    for (int q = 0; q < S::NQR; ++q) {
        if (red_valid<S>(g, q)) {
            const int y = g.y0 - 1 + red_row<S>(g, q);
            const int yw = g.edge_tile ? wrapi(y, g.L) : y;
            rr[q] = philox10(sweep, 0u, 0u, (uint32_t)yw * (uint32_t)g.P + jb, k0, k1);
        }
    }
#pragma unroll
    for (int q = 0; q < S::NQR; ++q) {
        if (red_valid<S>(g, q)) {
            const int row = red_row<S>(g, q);
            const PairNb<O> n(blk, S::WS, row + 1, c0);
            float4 own = *(const float4*)&cs[row * S::WS + c0];
            const u32x4 r = rr[q];
            float ta = thr[q].x, tb = thr[q].y;
            const int aa = site_update<T>(ta, own.x, own.y, nsum(n.la.x, n.ra.x, n.ua.x, n.da.x),
                                          nsum(n.la.y, n.ra.y, n.ua.y, n.da.y), r.x, r.y, p);
            const int ab = site_update<T>(tb, own.z, own.w, nsum(n.lb.x, n.rb.x, n.ub.x, n.db.x),
                                          nsum(n.lb.y, n.rb.y, n.ub.y, n.db.y), r.z, r.w, p);
            *(float4*)&cs[row * S::WS + c0] = own;
            if (q < FULL || (row >= 1 && row <= TY)) {
                acc += aa + ab;
                bio<T>::template st2<ST>(dst, (unsigned)(g.y0 - 1 + row) * (unsigned)g.Hh +
                                                  (unsigned)(g.kb + 2 * g.s), ta, tb);
            }
        }
    }
    if (e < S::NEDGE && e_red) {          // the one ring entry of red row e_row
        const int y = g.y0 - 1 + e_row;
        const int o = y & 1;
        const int j = e_k >> 1;            // e_k = kb-1 (odd: words 2, 3) or kb+TX/2 (even: words 0, 1)
        const u32x4 r = philox10(sweep, 0u, 0u, (uint32_t)wrapi(y, g.L) * (uint32_t)g.P + (uint32_t)wrapi(j, g.P),
                                 k0, k1);
        const int b = e_row + 1;           // black row of the same y
        const float2 l = blk[b * S::WS + e_col + o - 1], rt = blk[b * S::WS + e_col + o];
        const float2 u = blk[(b - 1) * S::WS + e_col], d = blk[(b + 1) * S::WS + e_col];
        float2 own = cs[e_row * S::WS + e_col];
        const bool odd = (e_k & 1) != 0;
        site_update<T>(the, own.x, own.y, nsum(l.x, rt.x, u.x, d.x), nsum(l.y, rt.y, u.y, d.y), odd ? r.z : r.x,
                       odd ? r.w : r.y, p);
        cs[e_row * S::WS + e_col] = own;
    }
}

// Black half-sweep of the interior rows y0 .. y0+TY-1 (black LDS rows 2 .. TY+1);
// O = parity of this thread's black rows.
template <typename T, int TX, int TY, int NT, int O, bool MEAS, bool ST>
__device__ __forceinline__ void tile1_black(const T1Geom& g, const float2* __restrict__ cs,
                                            float2 (&thb)[Tile1<TX, TY, NT>::NQB], __amdgpu_buffer_rsrc_t dst,
                                            uint32_t sweep, uint32_t k0, uint32_t k1, const Params& p, int& acc,
                                            MeasAcc& m)
{
    using S = Tile1<TX, TY, NT>;
    constexpr int FULL = TY / S::RP;           // passes entirely inside rows 2 .. TY+1
    const float2* blk = cs + S::BLACK0;
    const int c0 = 2 * g.s + 2;
    const unsigned jb = (unsigned)((g.kb >> 1) + g.s);
    u32x4 rb[S::NQB];
#pragma unroll
    for (int q = 0; q < S::NQB; ++q) {
        const int row = black_row<S>(g, q);
        if (q < FULL || (black_valid<S>(g, q) && row >= 2 && row < TY + 2))
            rb[q] = philox10(sweep, 1u, 0u, (uint32_t)(g.y0 - 2 + row) * (uint32_t)g.P + jb, k0, k1);
    }
#pragma unroll
    for (int q = 0; q < S::NQB; ++q) {
        const int row = black_row<S>(g, q);
        if (q < FULL || (black_valid<S>(g, q) && row >= 2 && row < TY + 2)) {
            const int y = g.y0 - 2 + row;  // interior: never wraps
            const PairNb<O> n(cs, S::WS, row - 1, c0);
            const float4 own = *(const float4*)&blk[row * S::WS + c0];
            const u32x4 r = rb[q];
            float ta = thb[q].x, tb = thb[q].y;
            float ca = own.x, sa = own.y, cb = own.z, sb = own.w;
            const int aa = site_update<T>(ta, ca, sa, nsum(n.la.x, n.ra.x, n.ua.x, n.da.x),
                                          nsum(n.la.y, n.ra.y, n.ua.y, n.da.y), r.x, r.y, p);
            const int ab = site_update<T>(tb, cb, sb, nsum(n.lb.x, n.rb.x, n.ub.x, n.db.x),
                                          nsum(n.lb.y, n.rb.y, n.ub.y, n.db.y), r.z, r.w, p);
            acc += aa + ab;
            bio<T>::template st2<ST>(dst, ((unsigned)g.L + (unsigned)y) * (unsigned)g.Hh + (unsigned)(g.kb + 2 * g.s),
                                     ta, tb);
            if constexpr (MEAS) {
                meas_acc(m, ca, sa, n.la, n.ra, n.ua, n.da);
                meas_acc(m, cb, sb, n.lb, n.rb, n.ub, n.db);
            }
        }
    }
}

// Per-tile geometry: the tile at (x0, y0) of an L x L lattice.
template <int TX, int TY, int NT>
__device__ __forceinline__ T1Geom tile1_geom(int L, int x0, int y0)
{
    using S = Tile1<TX, TY, NT>;
    const int tid = threadIdx.x;
    T1Geom g;
    g.L = L;
    g.Hh = L >> 1;
    g.P = g.Hh >> 1;
    g.kb = x0 >> 1;
    g.x0 = x0;
    g.y0 = y0;
    // The wave index is uniform; read through the scalar unit, so that for
    // 256-wide tiles (one half-row per wave) every row index, its wrap and the
    // row part of each address are scalar work.
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    g.s = lane & (S::TQ - 1);
    const int i = lane >> S::LGQ;
    g.rt = 2 * (i * (S::NW / 2) + (w >> 1)) + (w & 1);   // parity of the wave
    g.edge_tile = (y0 < 2) || (y0 + TY + 2 > L);
    return g;
}

// The angles one thread loads for a tile: its red and black pairs and, for the
// threads e = NT-1-tid < NEDGE, one edge entry (red edge entries land on the last
// wave).
template <int TX, int TY, int NT>
struct T1Regs {
    float2 thr[Tile1<TX, TY, NT>::NQR], thb[Tile1<TX, TY, NT>::NQB];
    float the;
    int e_row, e_col, e_red, e_k;
};

// Issue every load of the tile (no wait).
template <typename T, int TX, int TY, int NT>
__device__ __forceinline__ void tile1_load(const T1Geom& g, __amdgpu_buffer_rsrc_t rs, T1Regs<TX, TY, NT>& a)
{
    using S = Tile1<TX, TY, NT>;
    const int L = g.L, y0 = g.y0;
    const unsigned col = (unsigned)(g.kb + 2 * g.s);
#pragma unroll
    for (int q = 0; q < S::NQR; ++q) {
        if (red_valid<S>(g, q)) {
            const int y0r = y0 - 1 + red_row<S>(g, q);
            const int y = g.edge_tile ? wrapi(y0r, L) : y0r;
            a.thr[q] = bio<T>::ld2(rs, (unsigned)y * (unsigned)g.Hh + col);
        }
    }
#pragma unroll
    for (int q = 0; q < S::NQB; ++q) {
        if (black_valid<S>(g, q)) {
            const int y0b = y0 - 2 + black_row<S>(g, q);
            const int y = g.edge_tile ? wrapi(y0b, L) : y0b;
            a.thb[q] = bio<T>::ld2(rs, ((unsigned)L + (unsigned)y) * (unsigned)g.Hh + col);
        }
    }
    const int e = NT - 1 - (int)threadIdx.x;
    a.the = 0.0f;
    a.e_row = 0; a.e_col = 0; a.e_red = 0; a.e_k = 0;
    if (e < S::NEDGE) {
        int yl, side;
        if (e < S::RR) {                   // red row y0-1+e: the side its ring update needs
            a.e_red = 1;
            a.e_row = e;
            yl = y0 - 1 + e;
            side = ((yl & 1) == 0);        // o = 0 -> right column, o = 1 -> left column
        } else {
            const int e2 = e - S::RR;
            a.e_row = e2 >> 1;
            yl = y0 - 2 + a.e_row;
            side = e2 & 1;
        }
        a.e_k = side ? g.kb + TX / 2 : g.kb - 1;
        a.e_col = side ? TX / 2 + 2 : 1;
        a.the = bio<T>::ld1(rs, ((unsigned)(a.e_red ? 0 : L) + (unsigned)wrapi(yl, L)) * (unsigned)g.Hh +
                                    (unsigned)wrapi(a.e_k, g.Hh));
    }
}

// (cos, sin) of every loaded entry into LDS (waits for the loads); the caller
// places the barrier.
template <int TX, int TY, int NT>
__device__ __forceinline__ void tile1_fill(const T1Geom& g, float2* __restrict__ cs, const T1Regs<TX, TY, NT>& a)
{
    using S = Tile1<TX, TY, NT>;
#pragma unroll
    for (int q = 0; q < S::NQR; ++q) {
        if (red_valid<S>(g, q)) {
            float sa, ca, sb, cb;
            sincos_turn(a.thr[q].x, sa, ca);
            sincos_turn(a.thr[q].y, sb, cb);
            *(float4*)&cs[red_row<S>(g, q) * S::WS + 2 * g.s + 2] = make_float4(ca, sa, cb, sb);
        }
    }
#pragma unroll
    for (int q = 0; q < S::NQB; ++q) {
        if (black_valid<S>(g, q)) {
            float sa, ca, sb, cb;
            sincos_turn(a.thb[q].x, sa, ca);
            sincos_turn(a.thb[q].y, sb, cb);
            *(float4*)&cs[S::BLACK0 + black_row<S>(g, q) * S::WS + 2 * g.s + 2] = make_float4(ca, sa, cb, sb);
        }
    }
    if (NT - 1 - (int)threadIdx.x < S::NEDGE) {
        float s_, c_;
        sincos_turn(a.the, s_, c_);
        cs[(a.e_red ? 0 : S::BLACK0) + a.e_row * S::WS + a.e_col] = make_float2(c_, s_);
    }
}

// Both half-sweeps of a filled tile (after the fill's barrier); the updated angles
// go to rd.  MEAS and ST as for tile1_program.  Ends with the black updates (no barrier).
template <typename T, int TX, int TY, int NT, int MEAS, bool ST = false>
__device__ __forceinline__ void tile1_sweep(const T1Geom& g, float2* __restrict__ cs, T1Regs<TX, TY, NT>& a,
                                            __amdgpu_buffer_rsrc_t rd, uint32_t sweep, uint32_t k0, uint32_t k1,
                                            const Params& p, bool meas, double* part, double* red)
{
    const int tid = threadIdx.x;
    const int e = NT - 1 - tid;
    int acc = 0;
    MeasAcc m;
    // wave-uniform (rt has the wave's parity): made scalar so both phases branch per
    // wave instead of running both parity variants under exec masks
    const bool red_odd = __builtin_amdgcn_readfirstlane((g.y0 + g.rt) & 1) != 0;
    if (red_odd)
        tile1_red<T, TX, TY, NT, 1, ST>(g, cs, a.thr, rd, sweep, k0, k1, p, a.the, e, a.e_row, a.e_col, a.e_red, a.e_k,
                                    acc);
    else
        tile1_red<T, TX, TY, NT, 0, ST>(g, cs, a.thr, rd, sweep, k0, k1, p, a.the, e, a.e_row, a.e_col, a.e_red, a.e_k,
                                    acc);
    __syncthreads();
    if (MEAS == 1 || (MEAS == -1 && meas)) {
        if (red_odd)
            tile1_black<T, TX, TY, NT, 0, true, ST>(g, cs, a.thb, rd, sweep, k0, k1, p, acc, m);
        else
            tile1_black<T, TX, TY, NT, 1, true, ST>(g, cs, a.thb, rd, sweep, k0, k1, p, acc, m);
        double v[7] = {(double)m.cx, (double)m.cy, (double)m.ix, (double)m.iy, (double)m.mx, (double)m.my,
                       (double)acc};
        if constexpr (MEAS == 1) {
#pragma unroll
            for (int q = 0; q < 7; ++q) v[q] = wave_sum_last(v[q]);
            if ((tid & 63) == 63) {
                double* w = part + (size_t)(tid >> 6) * 8;
#pragma unroll
                for (int q = 0; q < 7; ++q) w[q] = v[q];
                w[7] = 0.0;
            }
        } else {
            block_sum7<NT>(v, red);
            if (tid == 0) {
#pragma unroll
                for (int q = 0; q < 7; ++q) part[q] = v[q];
                part[7] = 0.0;
            }
        }
    } else {
        if (red_odd)
            tile1_black<T, TX, TY, NT, 0, false, ST>(g, cs, a.thb, rd, sweep, k0, k1, p, acc, m);
        else
            tile1_black<T, TX, TY, NT, 1, false, ST>(g, cs, a.thb, rd, sweep, k0, k1, p, acc, m);
    }
}

// src/dst: the two state buffers (same layout); `state_bytes` bounds the buffer
// descriptors.  MEAS selects the measurement at compile time:
//   MEAS = 0 : never measure;
//   MEAS = 1 : always measure, one partial record per wave at part[wave * 8 ..]
//              (no barrier and no cross-wave step: the records are summed later in
//              a fixed order);
//   MEAS = -1: measure if `meas`, one partial record per tile at part[0 .. 8].
// A record is (Cx, Cy, Ix, Iy, Mx, My, accepts, 0).
// ST: the updated angles are stored with the non-temporal hint (for lattices
// larger than the caches: the stored lines are read again only a sweep later).
template <typename T, int TX, int TY, int NT, int MEAS = -1, bool ST = false>
__device__ __forceinline__ void tile1_program(const T* __restrict__ src, T* __restrict__ dst, unsigned state_bytes,
                                              int L, int x0, int y0, uint32_t sweep, uint32_t k0, uint32_t k1,
                                              const Params& p, bool meas, double* part, char* smem, double* red)
{
    float2* cs = (float2*)smem;
    const T1Geom g = tile1_geom<TX, TY, NT>(L, x0, y0);
    T1Regs<TX, TY, NT> a;
    // The fill (loads, sin/cos, LDS writes) holds up the whole workgroup at its
    // barrier; its waves issue ahead of other workgroups' update work on the same
    // SIMD (measured: +2% on a sweep with records every 10, neutral otherwise).
    __builtin_amdgcn_s_setprio(2);
    tile1_load<T, TX, TY, NT>(g, make_rsrc(src, state_bytes), a);
    tile1_fill<TX, TY, NT>(g, cs, a);
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    tile1_sweep<T, TX, TY, NT, MEAS, ST>(g, cs, a, make_rsrc(dst, state_bytes), sweep, k0, k1, p, meas, part,
                                         red);
}

}  // namespace xyd
