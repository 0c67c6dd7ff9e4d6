// xy_device.hpp -- device-side building blocks shared by every sweep kernel.
//
// Every kernel updates a site through xy_site_update() below, with the
// neighbour sums formed in one fixed order, so the trajectory is bitwise the
// same whatever kernel, tile shape or batch runs it.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xyd {

// --------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): ten rounds of two 32x32->64 products of
// words 0 and 2 with the round multipliers, high halves mixed into the other
// words with the key, key advanced by the Weyl increments between rounds.
// The counter is (sweep, colour, purpose, pair): the three uniform words and
// the key stay in scalar registers and the per-lane pair index enters through
// the last word, which the first rounds only xor in, so the early rounds are
// mostly scalar work.  From the fifth round on every word is per-lane and a
// round costs two v_mad_u64_u32 and two three-input xors (v_bitop3_b32 with
// truth table 0x96 = a ^ b ^ c, which the compiler does not form by itself).
struct u32x4 {
    uint32_t x, y, z, w;
};

template <bool VEC>
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    if constexpr (VEC) return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
    else return a ^ b ^ c;
}

template <int R>
__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                             uint32_t k0, uint32_t k1)
{
    // With a per-lane last counter word, word 1 is uniform up to round 3 and
    // word 3 up to round 2: until then those xors have two scalar operands,
    // which the compiler folds with one s_xor (the builtin would need them
    // both on the vector unit).
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3<(R >= 4)>((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = xor3<(R >= 3)>((uint32_t)(p0 >> 32), c3, k1);
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
}

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    philox_round<0>(c0, c1, c2, c3, k0, k1);
    philox_round<1>(c0, c1, c2, c3, k0 + 1 * W0, k1 + 1 * W1);
    philox_round<2>(c0, c1, c2, c3, k0 + 2 * W0, k1 + 2 * W1);
    philox_round<3>(c0, c1, c2, c3, k0 + 3 * W0, k1 + 3 * W1);
    philox_round<4>(c0, c1, c2, c3, k0 + 4 * W0, k1 + 4 * W1);
    philox_round<5>(c0, c1, c2, c3, k0 + 5 * W0, k1 + 5 * W1);
    philox_round<6>(c0, c1, c2, c3, k0 + 6 * W0, k1 + 6 * W1);
    philox_round<7>(c0, c1, c2, c3, k0 + 7 * W0, k1 + 7 * W1);
    philox_round<8>(c0, c1, c2, c3, k0 + 8 * W0, k1 + 8 * W1);
    philox_round<9>(c0, c1, c2, c3, k0 + 9 * W0, k1 + 9 * W1);
    return {c0, c1, c2, c3};
}

// f = 1 + (w >> 9) 2^-23 in [1, 2): the top 23 bits of w as the mantissa of a
// float with exponent 0, built by one funnel shift (alignbit).
__device__ __forceinline__ float one_two(uint32_t w)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, w, 9));
}

// u = (2 (w >> 9) + 1) 2^-24 = f - (1 - 2^-24), exact in FP32 (Sterbenz).
__device__ __forceinline__ float u01(uint32_t w)
{
    return __fsub_rn(one_two(w), 0x1.fffffep-1f);
}

// 2u - 1 = (2 (w >> 9) + 1 - 2^23) 2^-23 = (2f - 3) + 2^-23, each step exact.
__device__ __forceinline__ float sym11(uint32_t w)
{
    return __fadd_rn(__fmaf_rn(one_two(w), 2.0f, -3.0f), 0x1p-23f);
}

// ------------------------------------------------------------- sin / cos / exp
// Angles are stored in turns, phi = theta / (2 pi), in [0, 1], which is the
// argument the hardware transcendental unit takes: no scaling, no range
// reduction.
__device__ __forceinline__ void sincos_turn(float phi, float& s, float& c)
{
    s = __builtin_amdgcn_sinf(phi);
    c = __builtin_amdgcn_cosf(phi);
}

// ------------------------------------------------------------------- storage
template <typename T> struct store;
template <> struct store<float> {
    static __device__ __forceinline__ float ld(float v) { return v; }
    static __device__ __forceinline__ float st(float v) { return v; }
    // value as it will be stored (FP32: unchanged)
    static __device__ __forceinline__ float rnd(float v) { return v; }
};
template <> struct store<__half> {
    static __device__ __forceinline__ float ld(__half v) { return __half2float(v); }
    static __device__ __forceinline__ __half st(float v) { return __float2half_rn(v); }
    static __device__ __forceinline__ float rnd(float v) { return __half2float(__float2half_rn(v)); }
};

struct Params {
    float delta;    // FP32 rounding of delta / (2 pi): the proposal width in turns
    float nbl2e;    // -beta * log2(e), FP32
};

// One Metropolis update.  th is the angle in turns, (c, s) its (cos, sin);
// (sx, sy) = sums of the four neighbours' (cos, sin), formed by the caller as
// (left + right) + (up + down).  w1 drives the proposal, w2 the acceptance.
// The proposal th + delta (2 u1 - 1) is wrapped by v_fract_f32, which returns
// t - floor(t) rounded once and, where that rounds up to 1 (t a tiny negative
// number), the largest float below 1.  Returns 1 if the proposal is accepted;
// the new angle and its (cos, sin) come back in th, c, s.
template <typename T>
__device__ __forceinline__ int site_update(float& th, float& c, float& s, float sx, float sy,
                                           uint32_t w1, uint32_t w2, const Params& p,
                                           float* dE_out = nullptr)
{
    const float step = __fmul_rn(p.delta, sym11(w1));
    float t = __builtin_amdgcn_fractf(__fadd_rn(th, step));
    t = store<T>::rnd(t);
    float sn, cn;
    sincos_turn(t, sn, cn);
    const float dc = __fsub_rn(cn, c);
    const float ds = __fsub_rn(sn, s);
    const float dE = -__fmaf_rn(dc, sx, __fmul_rn(ds, sy));
    if (dE_out) *dE_out = dE;
    const int acc = u01(w2) < __builtin_amdgcn_exp2f(__fmul_rn(p.nbl2e, dE));
    th = acc ? t : th;
    c = acc ? cn : c;
    s = acc ? sn : s;
    return acc;
}

__device__ __forceinline__ float nsum(float l, float r, float u, float d)
{
    return __fadd_rn(__fadd_rn(l, r), __fadd_rn(u, d));
}

// Bond and magnetisation terms a black site contributes to a measurement: its
// four bonds (every bond has exactly one black end) and its own spin plus that
// of the red site to its right (a bijection black -> red).
struct Meas {
    float cx, cy, ix, iy, mx, my;
};

__device__ __forceinline__ void meas_black(Meas& m, float cb, float sb, float cl, float sl, float cr,
                                           float sr, float cu, float su, float cd, float sd)
{
    // bond (x-1 -> x): cos(tl - tb), sin(tl - tb); bond (x -> x+1): cos(tb - tr), sin(tb - tr)
    m.cx += __fmaf_rn(cl, cb, __fmul_rn(sl, sb)) + __fmaf_rn(cb, cr, __fmul_rn(sb, sr));
    m.ix += __fmaf_rn(sl, cb, -__fmul_rn(cl, sb)) + __fmaf_rn(sb, cr, -__fmul_rn(cb, sr));
    m.cy += __fmaf_rn(cu, cb, __fmul_rn(su, sb)) + __fmaf_rn(cb, cd, __fmul_rn(sb, sd));
    m.iy += __fmaf_rn(su, cb, -__fmul_rn(cu, sb)) + __fmaf_rn(sb, cd, -__fmul_rn(cb, sd));
    m.mx += cb + cr;
    m.my += sb + sr;
}

// ------------------------------------------------------------ reductions
// v moved across lanes by a DPP permutation within each row of 16 lanes (both
// 32-bit halves), on the vector unit instead of through the LDS crossbar.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// As dpp_f64, for the row broadcasts: rows outside ROWS receive 0.0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64_rows(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave, in a fixed order; every lane gets the result.
// Call with all lanes active.  Within a row of 16 lanes: partner lane ^ 1, ^ 2
// (quad permutations), then the mirror in each half-row (quad q <-> its other
// quad) and in the row (half-row <-> half-row); a + b = b + a, so all lanes of a
// row then hold the same row sum.  The four row sums are read as scalars and
// added as (r0 + r1) + (r2 + r3).
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// The same sum, valid in lane 63 only (other lanes hold partial sums): after the
// four steps within rows, row 1 adds row 0 and row 3 adds row 2 (row_bcast:15,
// the last lane of the row below), then rows 2 and 3 add lane 31 (row_bcast:31),
// so lane 63 ends with (r2 + r3) + (r0 + r1).  Call with all lanes active.
__device__ __forceinline__ double wave_sum_last(double v)
{
    v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    v += dpp_f64_rows<0x142, 0xA>(v);   // row_bcast:15 into rows 1, 3
    v += dpp_f64_rows<0x143, 0xC>(v);   // row_bcast:31 into rows 2, 3
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace xyd
