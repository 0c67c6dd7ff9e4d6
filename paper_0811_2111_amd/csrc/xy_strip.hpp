// xy_strip.hpp -- one sweep of a vertical strip segment, rows streamed through LDS rings.
//
// A workgroup owns TX columns (half-row entries kb .. kb+TX/2-1 of each colour,
// kb = x0/2) and rows y0 .. y0+SH-1, and walks down the segment R rows at a time.
// Step j:
//   * red rows y0-1+jR .. y0-1+jR+R-1 are updated (row y0-1 and row y0+SH are the
//     ring rows above and below, recomputed with their owners' random numbers and
//     not stored); they read the black rows one above to one below, which are
//     still old;
//   * black rows y0+(j-1)R .. y0+jR-1 are updated (from step 1 on); they read the
//     new red rows one above to one below, the last of which the red part of the
//     same step has just produced.
// Black (cos, sin) of the rows the red updates read live in a ring of 4R LDS rows,
// new red (cos, sin) in a ring of 2R rows; the angles a thread updates stay in its
// registers from load to store, and the loads of step j+D are issued in step j,
// so their latency overlaps D steps of arithmetic.
//
// The columns just outside the strip are handled once, before the walk: the black
// entries kb-1 and kb+TX/2 of rows y0-2 .. y0+SH+1 (their (cos, sin) into an LDS
// column pair) and, for each red row y0-1 .. y0+SH, the one red entry outside the
// strip that a black site inside needs (kb-1 for odd rows, kb+TX/2 for even rows),
// updated from its own black neighbours.  Each step copies these into the pad
// columns of its ring rows, so every pair in the strip reads its neighbours the
// same way.  Per sweep the strip recomputes SH+2 red rows and SH+2 ring entries
// for SH rows, against TY+2 rows per TY in a square tile.
//
// The edge columns are read before the walk, while the strips beside read the same
// cache lines as their walks reach those rows; the lines are L2 hits for them only
// if the L2 still holds them then.  So the walk's row loads and all its stores
// carry the non-temporal hint: the rows streamed through once per sweep leave the
// L2 early and more of the edge lines stay (at L = 16384: 2-3% less time per
// sweep, reads 1.26 -> 1.22 x one load per angle with the same XCD mapping).
//
// As in every other kernel, a site is updated by xyd::site_update with neighbour
// sums (left + right) + (up + down), and the random numbers of a site depend only
// on (seed, sweep, colour, row, pair), so the trajectory is that of any other
// schedule.
#pragma once

#include "xy_tile1.hpp"

namespace xyd {

template <int TX, int SH, int NT>
struct Strip {
    static_assert(TX == 128 || TX == 256 || TX == 512, "strip width: 128, 256 or 512");
    static_assert(NT == 256, "four waves");
    static constexpr int TQ = TX / 4;                  // Philox pairs per half-row
    static constexpr int LGQ = __builtin_ctz(TQ);
    static constexpr int NW = NT / 64;
    static constexpr int R = NT / TQ;                  // rows of each colour per step
    static_assert(SH % R == 0 && SH >= 2 * R, "segment height: a multiple of R, at least 2R");
    static constexpr int NS = SH / R + 1;              // steps
    static constexpr int WS = TX / 2 + 4;              // LDS row stride (float2); col(k) = k - kb + 2
    static constexpr int NB = 4 * R;                   // black ring rows
    static constexpr int NR = 2 * R;                   // red ring rows
    static constexpr int NEB = SH + 4;                 // black edge rows y0-2 .. y0+SH+1
    static constexpr int NER = SH + 2;                 // red ring rows y0-1 .. y0+SH
    static constexpr int RED0 = NB * WS;               // offsets in float2 entries
    static constexpr int BE0 = RED0 + NR * WS;
    static constexpr int RE0 = BE0 + 2 * NEB;
    static constexpr size_t lds_bytes = (size_t)(RE0 + NER) * sizeof(float2);
    static constexpr int D = 2;                        // prefetch depth in steps
};

// Neighbours of the pair at LDS column c0 (even) whose own row of the other colour
// is `mid`, with the rows above and below it at `up` and `dn` (ring rows need not
// be adjacent in LDS).  O = parity of the updated sites' row offset o, as in PairNb.
template <int O>
struct PairNbR {
    float2 la, ra, lb, rb, ua, ub, da, db;
    __device__ __forceinline__ PairNbR(const float2* __restrict__ mid, const float2* __restrict__ up,
                                       const float2* __restrict__ dn, int c0)
    {
        const float4 h = *(const float4*)&mid[c0];
        const float2 side = mid[O ? c0 + 2 : c0 - 1];
        const float4 u = *(const float4*)&up[c0];
        const float4 d = *(const float4*)&dn[c0];
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

struct StripGeom {
    int L, Hh, P, kb, y0;
    int s;     // pair slot within a half-row
    int rt;    // row offset of this thread within a step
};

// The walk for threads whose red rows have parity O (wave-uniform); their black
// rows have the other parity, so the horizontal neighbour offset o of both the red
// and the black sites they update is O.  Step j takes its pairs from register slot
// j % 3 and issues the loads of step j + 2 into slot (j + 2) % 3; the loop is
// unrolled by three so the slots are fixed registers and no copy has to wait for a
// load in flight.  Only the first and the last two steps have rows outside the
// segment's range or no loads to issue; the steps between them load and store
// unconditionally, so the compiler can count the memory operations in flight
// exactly and waits only for the loads a step consumes.
template <typename T, int TX, int SH, int NT, int O, bool MEAS>
struct StripWalk {
    using S = Strip<TX, SH, NT>;
    static_assert(S::D == 2, "three register slots");
    const StripGeom& g;
    float2* bring;
    float2* rring;
    const float2* be;
    const float2* re;
    __amdgpu_buffer_rsrc_t rs, rd;
    uint32_t sweep, k0, k1;
    const Params& p;
    int c0;
    unsigned col, jb, Hh, Lu;
    float2 pr[3], pb[3];   // red row y0-1+rel and black row y0+rel of step j, rel = jR + rt
    float2 ub;             // black pair of the previous step, updated in this one
    int acc;
    MeasAcc m;

    __device__ __forceinline__ StripWalk(const StripGeom& g_, float2* cs, __amdgpu_buffer_rsrc_t rs_,
                                         __amdgpu_buffer_rsrc_t rd_, uint32_t sweep_, uint32_t k0_, uint32_t k1_,
                                         const Params& p_)
        : g(g_), bring(cs), rring(cs + S::RED0), be(cs + S::BE0), re(cs + S::RE0), rs(rs_), rd(rd_),
          sweep(sweep_), k0(k0_), k1(k1_), p(p_), c0(2 * g_.s + 2), col((unsigned)(g_.kb + 2 * g_.s)),
          jb((unsigned)((g_.kb >> 1) + g_.s)), Hh((unsigned)g_.Hh), Lu((unsigned)g_.L), ub(make_float2(0.f, 0.f)),
          acc(0)
    {
    }

    // rows past the segment's halo (last step only) are loaded too, wrapped into
    // the lattice, and never used
    __device__ __forceinline__ void load(int j, float2& r, float2& b)
    {
        const int rel = j * S::R + g.rt;
        const int yr = wrapi(g.y0 - 1 + rel, g.L), yb = wrapi(g.y0 + rel, g.L);
        r = bio<T>::template ld2<true>(rs, (unsigned)yr * Hh + col);
        b = bio<T>::template ld2<true>(rs, (Lu + (unsigned)yb) * Hh + col);
    }

    // KIND: 0 = step 0 (no black update; red row y0-1 not stored); 1 = a step
    // inside the segment that issues the loads of step j + 2; 2 = the same without
    // loads (step NS-2); 3 = the last step (only the red rows y0+SH-1, y0+SH, and
    // only the first of them stored).
    template <int C, int KIND>
    __device__ __forceinline__ void step(int j)
    {
        constexpr int N2 = (C + 2) % 3;
        const int rel = j * S::R + g.rt;   // red ring row of this thread's red row
        const bool live = KIND != 3 || rel <= SH + 1;
        // nothing moves across a step boundary: a load hoisted above the previous
        // step's use of the same slot would force a register copy that waits for it
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (KIND <= 1) load(j + 2, pr[N2], pb[N2]);
        const int yr = wrapi(g.y0 - 1 + rel, g.L);
        const int ybu = g.y0 + rel - S::R;   // black row updated in this step (j >= 1)
        u32x4 wr, wb;
        if (live) wr = philox10(sweep, 0u, 0u, (uint32_t)yr * (uint32_t)g.P + jb, k0, k1);
        if constexpr (KIND != 0) wb = philox10(sweep, 1u, 0u, (uint32_t)ybu * (uint32_t)g.P + jb, k0, k1);

        // black row y0+rel: (cos, sin) into its ring row, edge columns into the pads
        float cra = 0.f, sra = 0.f, crb = 0.f, srb = 0.f;
        if (live) {
            float sa, ca, sb, cb;
            sincos_turn(pb[C].x, sa, ca);
            sincos_turn(pb[C].y, sb, cb);
            float2* row = bring + ((rel + 2) & (S::NB - 1)) * S::WS;
            *(float4*)&row[c0] = make_float4(ca, sa, cb, sb);
            if (g.s == 0) row[1] = be[rel + 2];
            if (g.s == S::TQ - 1) row[TX / 2 + 2] = be[S::NEB + rel + 2];
            sincos_turn(pr[C].x, sra, cra);
            sincos_turn(pr[C].y, srb, crb);
        }
        __syncthreads();

        // red row y0-1+rel
        if (live) {
            const PairNbR<O> n(bring + ((rel + 1) & (S::NB - 1)) * S::WS, bring + (rel & (S::NB - 1)) * S::WS,
                               bring + ((rel + 2) & (S::NB - 1)) * S::WS, c0);
            float ta = pr[C].x, tb = pr[C].y;
            const int aa = site_update<T>(ta, cra, sra, nsum(n.la.x, n.ra.x, n.ua.x, n.da.x),
                                          nsum(n.la.y, n.ra.y, n.ua.y, n.da.y), wr.x, wr.y, p);
            const int ab = site_update<T>(tb, crb, srb, nsum(n.lb.x, n.rb.x, n.ub.x, n.db.x),
                                          nsum(n.lb.y, n.rb.y, n.ub.y, n.db.y), wr.z, wr.w, p);
            float2* row = rring + (rel & (S::NR - 1)) * S::WS;
            *(float4*)&row[c0] = make_float4(cra, sra, crb, srb);
            // the ring entry of this row: left of the strip for odd rows (O = 1), right for even
            if (O ? g.s == 0 : g.s == S::TQ - 1) row[O ? 1 : TX / 2 + 2] = re[rel];
            if (KIND == 1 || KIND == 2 || (rel >= 1 && rel <= SH)) {
                acc += aa + ab;
                bio<T>::template st2<true>(rd, (unsigned)(g.y0 - 1 + rel) * Hh + col, ta, tb);
            }
            if constexpr (MEAS) pin_sums(acc);
        }
        __syncthreads();

        // black row y0+rel-R (ring rows: own rel-R+2 in the black ring; red rel-R+1 +- 1)
        if constexpr (KIND != 0) {
            const float4 own = *(const float4*)&bring[((rel - S::R + 2) & (S::NB - 1)) * S::WS + c0];
            const PairNbR<O> n(rring + ((rel - S::R + 1) & (S::NR - 1)) * S::WS,
                               rring + ((rel - S::R) & (S::NR - 1)) * S::WS,
                               rring + ((rel - S::R + 2) & (S::NR - 1)) * S::WS, c0);
            float ta = ub.x, tb = ub.y;
            float ca = own.x, sa = own.y, cb = own.z, sb = own.w;
            const int aa = site_update<T>(ta, ca, sa, nsum(n.la.x, n.ra.x, n.ua.x, n.da.x),
                                          nsum(n.la.y, n.ra.y, n.ua.y, n.da.y), wb.x, wb.y, p);
            const int ab = site_update<T>(tb, cb, sb, nsum(n.lb.x, n.rb.x, n.ub.x, n.db.x),
                                          nsum(n.lb.y, n.rb.y, n.ub.y, n.db.y), wb.z, wb.w, p);
            acc += aa + ab;
            bio<T>::template st2<true>(rd, (Lu + (unsigned)ybu) * Hh + col, ta, tb);
            if constexpr (MEAS) {
                meas_acc(m, ca, sa, n.la, n.ra, n.ua, n.da);
                meas_acc(m, cb, sb, n.lb, n.rb, n.ub, n.db);
                pin_sums(m, acc);
            }
        }
        ub = pb[C];   // already consumed above, so no wait
    }

    __device__ __forceinline__ void run()
    {
        constexpr int NS = S::NS;
        constexpr int M = NS - 3;            // steps 1 .. NS-3 load ahead
        load(0, pr[0], pb[0]);
        load(1, pr[1], pb[1]);
        step<0, 0>(0);
        int j = 1;
        for (int t = 0; t < M / 3; ++t, j += 3) {
            step<1, 1>(j);
            step<2, 1>(j + 1);
            step<0, 1>(j + 2);
        }
        if constexpr (M % 3 >= 1) step<1, 1>(j);
        if constexpr (M % 3 == 2) step<2, 1>(j + 1);
        step<(NS - 2) % 3, 2>(NS - 2);
        step<(NS - 1) % 3, 3>(NS - 1);
    }
};

// One sweep of the segment (x0, y0) from src to dst (same layout; `state_bytes`
// bounds the buffer descriptors).  MEAS: one partial record (Cx, Cy, Ix, Iy, Mx,
// My, accepts, 0) per wave at part[wave * 8 ..], no barrier.
template <typename T, int TX, int SH, int NT, bool MEAS>
__device__ __forceinline__ void strip_program(const T* __restrict__ src, T* __restrict__ dst, unsigned state_bytes,
                                              int L, int x0, int y0, uint32_t sweep, uint32_t k0, uint32_t k1,
                                              const Params& p, double* part, char* smem)
{
    using S = Strip<TX, SH, NT>;
    float2* cs = (float2*)smem;
    // wave index through the scalar unit: row indices and their wraps are scalar work
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, state_bytes);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(dst, state_bytes);

    StripGeom g;
    g.L = L;
    g.Hh = L >> 1;
    g.P = g.Hh >> 1;
    g.kb = x0 >> 1;
    g.y0 = y0;
    if constexpr (S::TQ <= 64) {
        g.s = lane & (S::TQ - 1);
        g.rt = 4 * (lane >> S::LGQ) + w;   // wave w: rows w, w + 4 (same parity)
    } else {                               // a half-row spans two waves: waves 2r, 2r+1 take row r
        g.s = (w & 1) * 64 + lane;
        g.rt = w >> 1;
    }

    // ---- edge columns: black entries kb-1 (side 0) and kb+TX/2 (side 1) of rows
    // y0-2 .. y0+SH+1; then the ring red entries of rows y0-1 .. y0+SH
    float2* be = cs + S::BE0;
    float2* re = cs + S::RE0;
    const int kl = wrapi(g.kb - 1, g.Hh), kr = wrapi(g.kb + TX / 2, g.Hh);
    for (int t = tid; t < 2 * S::NEB; t += NT) {
        const int side = t >= S::NEB, rel = side ? t - S::NEB : t;
        const int y = wrapi(y0 - 2 + rel, L);
        const float a = bio<T>::ld1(rs, ((unsigned)L + (unsigned)y) * (unsigned)g.Hh + (unsigned)(side ? kr : kl));
        float sn, cn;
        sincos_turn(a, sn, cn);
        be[t] = make_float2(cn, sn);
    }
    // ring entries i = lane * NW + wave + q NT (row y0-1+i), so every wave takes a share
    constexpr int NQE = (S::NER + NT - 1) / NT;
    const int ie0 = lane * S::NW + w;
    float th_e[NQE], tin[NQE];
    u32x4 we[NQE];
#pragma unroll
    for (int q = 0; q < NQE; ++q) {
        const int ie = ie0 + q * NT;
        if (ie < S::NER) {
            const int y = y0 - 1 + ie, yw = wrapi(y, L);
            const int odd = y & 1;         // odd rows: entry kb-1, inside neighbour kb; even: kb+TX/2, kb+TX/2-1
            const int k = odd ? kl : kr, kin = odd ? g.kb : g.kb + TX / 2 - 1;
            th_e[q] = bio<T>::ld1(rs, (unsigned)yw * (unsigned)g.Hh + (unsigned)k);
            tin[q] = bio<T>::ld1(rs, ((unsigned)L + (unsigned)yw) * (unsigned)g.Hh + (unsigned)kin);
            we[q] = philox10(sweep, 0u, 0u, (uint32_t)yw * (uint32_t)g.P + (uint32_t)(k >> 1), k0, k1);
        }
    }
    // black rows y0-2, y0-1 (black ring rows 0, 1) on the threads with rt = R-2, R-1
    const bool pre = g.rt >= S::R - 2;
    float4 pre_cs;
    if (pre) {
        const int y = wrapi(y0 - 2 + g.rt - (S::R - 2), L);
        const float2 b = bio<T>::ld2(rs, ((unsigned)L + (unsigned)y) * (unsigned)g.Hh + (unsigned)(g.kb + 2 * g.s));
        sincos_turn(b.x, pre_cs.y, pre_cs.x);
        sincos_turn(b.y, pre_cs.w, pre_cs.z);
    }
    __syncthreads();
    if (pre) {
        const int rel = g.rt - (S::R - 2);
        float2* row = cs + rel * S::WS;
        *(float4*)&row[2 * g.s + 2] = pre_cs;
        if (g.s == 0) row[1] = be[rel];
        if (g.s == S::TQ - 1) row[TX / 2 + 2] = be[S::NEB + rel];
    }
#pragma unroll
    for (int q = 0; q < NQE; ++q) {
        const int ie = ie0 + q * NT;
        if (ie < S::NER) {
            const int y = y0 - 1 + ie;
            const int odd = y & 1, side = !odd;
            float sn, cn, si, ci;
            sincos_turn(th_e[q], sn, cn);
            sincos_turn(tin[q], si, ci);
            const float2 in = make_float2(ci, si), out = be[side * S::NEB + ie + 1];
            const float2 u = be[side * S::NEB + ie], d = be[side * S::NEB + ie + 2];
            // red entry (y, k), o = y & 1: left (y, k+o-1), right (y, k+o)
            const float2 l = odd ? out : in, r = odd ? in : out;
            site_update<T>(th_e[q], cn, sn, nsum(l.x, r.x, u.x, d.x), nsum(l.y, r.y, u.y, d.y),
                           odd ? we[q].z : we[q].x, odd ? we[q].w : we[q].y, p);
            re[ie] = make_float2(cn, sn);
        }
    }
    // (the walk's first barrier orders these LDS writes before their readers)

    int acc;
    MeasAcc m;
    const bool red_odd = __builtin_amdgcn_readfirstlane((y0 - 1 + g.rt) & 1) != 0;
    if (red_odd) {
        StripWalk<T, TX, SH, NT, 1, MEAS> wk(g, cs, rs, rd, sweep, k0, k1, p);
        wk.run();
        acc = wk.acc;
        m = wk.m;
    } else {
        StripWalk<T, TX, SH, NT, 0, MEAS> wk(g, cs, rs, rd, sweep, k0, k1, p);
        wk.run();
        acc = wk.acc;
        m = wk.m;
    }

    if constexpr (MEAS) {
        double v[7] = {(double)m.cx, (double)m.cy, (double)m.ix, (double)m.iy, (double)m.mx, (double)m.my,
                       (double)acc};
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] = wave_sum_last(v[q]);
        if (lane == 63) {
            double* o = part + (size_t)w * 8;
#pragma unroll
            for (int q = 0; q < 7; ++q) o[q] = v[q];
            o[7] = 0.0;
        }
    }
}

}  // namespace xyd
