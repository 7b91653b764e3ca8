// Device helpers shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace nuosc {

// sin and cos of x: x = k pi/2 + r, pi/2 split into three doubles whose
// products with k are subtracted with one rounding each (fma; the reduction
// of Cody and Waite, exact in k P1 and k P2 for |k| < 2^53, so accurate to
// |x| ~ 7e15, beyond which the ulp of x itself exceeds pi), then the Taylor
// series of sin and cos to r^17 and r^18 on |r| <= pi/4 (truncation below
// 1e-19) and the quadrant k mod 4.  NaN in, NaN out.
__device__ __forceinline__ void fast_sincos(double x, double& s, double& c)
{
    const double k = rint(x * 0.6366197723675814);  // 2 / pi
    double r = fma(-k, 1.5707963267948966, x);
    r = fma(-k, 6.123233995736766e-17, r);
    r = fma(-k, -1.4973849048591698e-33, r);
    const double z = r * r;
    // (-1)^n / (2n+1)!, n = 1..8, and (-1)^n / (2n)!, n = 1..9
    double ps = 2.8114572543455206e-15;
    ps = fma(ps, z, -7.647163731819816e-13);
    ps = fma(ps, z, 1.6059043836821613e-10);
    ps = fma(ps, z, -2.505210838544172e-08);
    ps = fma(ps, z, 2.7557319223985893e-06);
    ps = fma(ps, z, -0.0001984126984126984);
    ps = fma(ps, z, 0.008333333333333333);
    ps = fma(ps, z, -0.16666666666666666);
    const double sr = fma(r * z, ps, r);
    double pc = -1.5619206968586225e-16;
    pc = fma(pc, z, 4.779477332387385e-14);
    pc = fma(pc, z, -1.1470745597729725e-11);
    pc = fma(pc, z, 2.08767569878681e-09);
    pc = fma(pc, z, -2.755731922398589e-07);
    pc = fma(pc, z, 2.48015873015873e-05);
    pc = fma(pc, z, -0.001388888888888889);
    pc = fma(pc, z, 0.041666666666666664);
    pc = fma(pc, z, -0.5);
    const double cr = fma(z, pc, 1.0);
    const int q = (int)fma(-4.0, floor(0.25 * k), k);  // k mod 4 in [0, 4), exact for integer k
    s = (q & 1) ? cr : sr;
    c = (q & 1) ? sr : cr;
    if (q == 1 || q == 2) c = -c;
    if (q & 2) s = -s;
}

// x of the lane that the DPP control CTRL selects (a pattern within each row
// of 16 lanes), the whole wavefront active; a double moves as its two halves.
template <int CTRL>
__device__ __forceinline__ double dpp_pick(double x)
{
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum of x over the 16 lanes of each row, the same bits in every lane of the
// row: rotations of the row by 8 and by 4 lanes, then the swaps of lanes 2
// apart and 1 apart within each quad.  Cross-lane moves of the vector ALU,
// no LDS traffic.
__device__ __forceinline__ double row_sum16(double x)
{
    x += dpp_pick<0x128>(x);  // row_ror:8
    x += dpp_pick<0x124>(x);  // row_ror:4
    x += dpp_pick<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dpp_pick<0xB1>(x);   // quad_perm [1,0,3,2]
    return x;
}

// x of lane l (l wave-uniform), as a wave-uniform value.
__device__ __forceinline__ double lane_value(double x, int l)
{
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum of x over the wavefront, the same bits in every lane: the row sums,
// then (row 0 + row 1) + (row 2 + row 3).
__device__ __forceinline__ double wave_sum_rows(double x)
{
    x = row_sum16(x);
    return (lane_value(x, 0) + lane_value(x, 16)) + (lane_value(x, 32) + lane_value(x, 48));
}

// Maximum of x over the wavefront (fmax: a NaN is dropped while a number is
// left), the same in every lane.
__device__ __forceinline__ double wave_max_rows(double x)
{
    x = fmax(x, dpp_pick<0x128>(x));
    x = fmax(x, dpp_pick<0x124>(x));
    x = fmax(x, dpp_pick<0x4E>(x));
    x = fmax(x, dpp_pick<0xB1>(x));
    return fmax(fmax(lane_value(x, 0), lane_value(x, 16)), fmax(lane_value(x, 32), lane_value(x, 48)));
}

// v of the even row (first) and of the odd row (second) of each pair of rows
// (lanes 32k .. 32k+15 and 32k+16 .. 32k+31), in every lane of the pair: one
// v_permlane16_swap per 32-bit half, the whole wavefront active.
__device__ __forceinline__ void row_pair(float v, float& even, float& odd)
{
    const unsigned b = __builtin_bit_cast(unsigned, v);
    const auto r = __builtin_amdgcn_permlane16_swap(b, b, false, false);
    even = __builtin_bit_cast(float, (unsigned)r[0]);
    odd = __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ void row_pair(double v, double& even, double& odd)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    even = __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi[0] << 32) | (unsigned)lo[0]);
    odd = __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi[1] << 32) | (unsigned)lo[1]);
}

}  // namespace nuosc
