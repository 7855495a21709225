// Cross-lane sums of a wavefront on VALU permutations (DPP and the gfx950
// permlane swaps).  A __shfl_xor butterfly runs through the LDS crossbar
// (ds_bpermute): six dependent LDS round trips per 32-bit value, which in a
// per-quartet reduction leaves the wavefront waiting on LDS latency.
#pragma once

#include <hip/hip_runtime.h>

namespace ks {

// Sum over the four rows of 16 lanes, left in every lane: the gfx950
// permlane swaps (v_permlane16_swap / v_permlane32_swap, VALU, no LDS
// traffic) exchange odd and even rows, then the two halves of the wave; with
// both operands the same value the two results add to x + x(lane ^ 16),
// then to the sum over lane ^ 32.  FP64 values travel as two 32-bit halves.
__device__ __forceinline__ float sum_rows(float x)
{
    const unsigned int u = __builtin_bit_cast(unsigned int, x);
    const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    x = __builtin_bit_cast(float, (unsigned int)a[0]) + __builtin_bit_cast(float, (unsigned int)a[1]);
    const unsigned int v = __builtin_bit_cast(unsigned int, x);
    const auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return __builtin_bit_cast(float, (unsigned int)b[0]) + __builtin_bit_cast(float, (unsigned int)b[1]);
}
__device__ __forceinline__ double swap_rows(double x, bool wide, double& other)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned int lo = (unsigned int)u, hi = (unsigned int)(u >> 32);
    unsigned int a0, a1, b0, b1;
    if (wide) {
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        a0 = l[0]; a1 = l[1]; b0 = h[0]; b1 = h[1];
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        a0 = l[0]; a1 = l[1]; b0 = h[0]; b1 = h[1];
    }
    other = __builtin_bit_cast(double, (unsigned long long)a1 | ((unsigned long long)b1 << 32));
    return __builtin_bit_cast(double, (unsigned long long)a0 | ((unsigned long long)b0 << 32));
}
__device__ __forceinline__ double sum_rows(double x)
{
    double o;
    double s = swap_rows(x, false, o);
    x = s + o;
    s = swap_rows(x, true, o);
    return s + o;
}

// One DPP move of a double (both 32-bit halves with the same control).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

// Sum over all 64 lanes, left in every lane: quad permutations [1,0,3,2]
// and [2,3,0,1] give each lane its quad's sum, the half-row mirror (lane i
// of 8 with lane 7 - i) pairs the two quads of 8 lanes, the row mirror
// (i with 15 - i) the two halves of a row of 16, and sum_rows the four rows.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_f64<0xB1>(x);
    x += dpp_f64<0x4E>(x);
    x += dpp_f64<0x141>(x);
    x += dpp_f64<0x140>(x);
    return sum_rows(x);
}

}  // namespace ks
