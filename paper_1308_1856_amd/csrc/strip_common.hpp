// Helpers shared by the wave-strip kernels (k_strip.hip, k_pstrip.hip):
// storage widening, the zero row, DPP whole-wave shifts of FP64 values and
// register copies that the compiler cannot fold.
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace tdse {

template <typename C> __device__ __forceinline__ C zero_c();
template <> __device__ __forceinline__ float2 zero_c<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 zero_c<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ c48 zero_c<c48>() { return c48{0u, 0u, 0u}; }
__device__ __forceinline__ double2 widen(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double2 widen(double2 v) { return v; }
__device__ __forceinline__ double2 widen(c48 v) { return widen48(v); }
// The all-zero row (at least max N complex FP64 values) as a row of storage
// type T.
template <typename T> __device__ __forceinline__ auto zero_rowt(const SweepGeom& g)
{
    if constexpr (std::is_same<T, s48>::value) {
        void* z = const_cast<void*>(g.zero_row);
        return P48{static_cast<uint2*>(z), static_cast<unsigned*>(z)};
    } else {
        return static_cast<const typename Cplx<T>::type*>(g.zero_row);
    }
}
__device__ __forceinline__ double2 pick2(bool c, double2 a, double2 b)
{
    return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
// Radial neighbours across the wave by DPP whole-wave shifts (a VALU move,
// no LDS round trip): wave_shr:1 gives lane i the value of lane i-1,
// wave_shl:1 the value of lane i+1.  The end lanes receive 0 (bound_ctrl: the
// move writes zero where the source lane does not exist, so the destination
// needs no initial value); they are outside the strip's exact region anyway.
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ double2 dpp_shift2(double2 v)
{
    return make_double2(dpp_shift<CTRL>(v.x), dpp_shift<CTRL>(v.y));
}
// The same shift, with the lane that has no source (lane 0 for wave_shr,
// lane 63 for wave_shl) keeping its value of `edge` instead of zero.
template <int CTRL>
__device__ __forceinline__ double dpp_shift_edge(double v, double edge)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned long long e = (unsigned long long)__double_as_longlong(edge);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)e, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(e >> 32), (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf,
                                               false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ double2 dpp_shift2_edge(double2 v, double2 edge)
{
    return make_double2(dpp_shift_edge<CTRL>(v.x, edge.x), dpp_shift_edge<CTRL>(v.y, edge.y));
}
// A copy of v in registers of its own (an actual move, which the compiler
// cannot fold into v's registers), ordered before every later memory access:
// the registers of v are then free for a reload of v's variable, so a loop
// that reloads it needs no register copy at its end (a copy that would wait
// for the reload just issued).
__device__ __forceinline__ double2 take(double2 v)
{
    double2 r;
    asm volatile("v_mov_b64 %0, %1" : "=&v"(r.x) : "v"(v.x) : "memory");
    asm volatile("v_mov_b64 %0, %1" : "=&v"(r.y) : "v"(v.y) : "memory");
    return r;
}
__device__ __forceinline__ float2 take(float2 v)
{
    float2 r;
    asm volatile("v_mov_b32 %0, %1" : "=&v"(r.x) : "v"(v.x) : "memory");
    asm volatile("v_mov_b32 %0, %1" : "=&v"(r.y) : "v"(v.y) : "memory");
    return r;
}
__device__ __forceinline__ c48 take(c48 v)
{
    c48 r;
    asm volatile("v_mov_b32 %0, %1" : "=&v"(r.hx) : "v"(v.hx) : "memory");
    asm volatile("v_mov_b32 %0, %1" : "=&v"(r.hy) : "v"(v.hy) : "memory");
    asm volatile("v_mov_b32 %0, %1" : "=&v"(r.l) : "v"(v.l) : "memory");
    return r;
}
// value of lane - d / lane + d (d = 1 or 2)
__device__ __forceinline__ double2 lane_below(double2 v, int d)
{
    v = dpp_shift2<kDppWaveShr1>(v);
    return d == 2 ? dpp_shift2<kDppWaveShr1>(v) : v;
}
__device__ __forceinline__ double2 lane_above(double2 v, int d)
{
    v = dpp_shift2<kDppWaveShl1>(v);
    return d == 2 ? dpp_shift2<kDppWaveShl1>(v) : v;
}

}  // namespace tdse
