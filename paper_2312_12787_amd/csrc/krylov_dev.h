// krylov_dev.h -- device helpers shared by the Krylov-step kernels of
// linalg.hip and the step product of matvec.hip, so that both form the norm
// of a Krylov vector with the same arithmetic in the same order.
#pragma once

#include <hip/hip_runtime.h>

namespace bemk {
namespace dev {

// Move a double between lanes with a DPP pattern (two 32-bit moves); lanes
// whose row is masked off or whose source is out of range receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false));
}

// Sum over the 64 lanes of a wave, returned in every lane (GFX9 DPP: quad
// swaps, half-row and row mirrors give each 16-lane row its sum; the row
// broadcasts of lanes 15 and 31 then collect the four rows into row 3, and
// lane 63 is read out).
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xf>(v);  // row_half_mirror
    v += dpp_f64<0x140, 0xf>(v);  // row_mirror
    v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// beta = |w| from the nu partial sums of |w|^2 that the update blocks wrote
// for one right-hand side (p = norm_part + r * nu): lane l adds partials
// l, l + 64, ... in order, then the wave sum.  Called by a whole wave; the
// result is in every lane.
__device__ __forceinline__ double step_beta(const double* __restrict__ p, int nu)
{
    double v = 0.0;
    for (int b = threadIdx.x & 63; b < nu; b += 64) v += p[b];
    return sqrt(wave_sum(v));
}

// 1 / beta, 0 when the Krylov space ended (beta = 0)
__device__ __forceinline__ double inv_beta(double beta) { return beta > 0.0 ? 1.0 / beta : 0.0; }

// `active` value of a column that stops at the current step: marked while the
// update blocks of the same launch may still read it, cleared by the
// normalisation that follows
constexpr int STOPPING = 2;

}  // namespace dev
}  // namespace bemk
