// xy_hmc_site.hpp -- per-site arithmetic of a hybrid Monte Carlo trajectory
// (section 1.2), shared by the single-lattice and the four-replica kernels so
// that a replica follows bit for bit the trajectory of the same lattice alone
// (its FP64 sums are taken in another order, so dH agrees to rounding).
#pragma once

#include "xy.h"
#include "xy_device.hpp"

namespace xyd {
namespace hmc {

constexpr float kMinus2Ln2 = -1.38629436111989061883f;   // -2 ln 2

// Box-Muller, cosine branch: sqrt(-2 ln u1) cos(2 pi u2); the hardware log is
// base 2 and the hardware cosine takes turns, so 2 pi u2 turns is u2.
__device__ __forceinline__ float box_muller(uint32_t w1, uint32_t w2)
{
    const float r2 = kMinus2Ln2 * __builtin_amdgcn_logf(u01(w1));
    return __builtin_sqrtf(r2) * __builtin_amdgcn_cosf(u01(w2));
}

// (cos, sin) of entry (c, y, k) and of its four neighbours in the other plane.
struct Nb {
    float c, s;                    // the site
    float cl, sl, cr, sr, cu, su, cd, sd;
};

// s_i sum c_j - c_i sum s_j = sum_j sin(theta_i - theta_j); F = -beta times this.
__device__ __forceinline__ float sin_sum(const Nb& n)
{
    const float sc = nsum(n.cl, n.cr, n.cu, n.cd);
    const float ss = nsum(n.sl, n.sr, n.su, n.sd);
    return __fmaf_rn(n.s, sc, -__fmul_rn(n.c, ss));
}

// dH = H_new - H_old from the two sums (slot 6 = sum p^2/2, slots 0, 1 = the bond
// cosines, H = K + beta E with E = -(Cx + Cy)); accept iff u < exp(-dH), u from
// Philox (traj, 0, 3, 0).
__device__ __forceinline__ void decide_core(const double o[7], const double n[7], double beta, uint32_t traj,
                                            uint32_t k0, uint32_t k1, unsigned* __restrict__ flag,
                                            xy_hmc_obs* __restrict__ obs)
{
    const double h_old = o[6] - beta * (o[0] + o[1]);
    const double h_new = n[6] - beta * (n[0] + n[1]);
    const double dH = h_new - h_old;
    const u32x4 r = philox10(traj, 0u, 3u, 0u, k0, k1);
    const double u = (double)u01(r.x);           // exact in FP32
    const unsigned acc = u < exp(-dH) ? 1u : 0u;
    *flag = acc;
    if (obs) {
        const double* s = acc ? n : o;
        obs->traj = (uint64_t)traj + 1u;
        obs->accepted = acc;
        obs->dH = dH;
        obs->cx = s[0]; obs->cy = s[1]; obs->ix = s[2]; obs->iy = s[3]; obs->mx = s[4]; obs->my = s[5];
    }
}

}  // namespace hmc
}  // namespace xyd
