// Device helpers: complex loads/stores with FP64 registers, wave64/block
// reductions in FP64 with a fixed (timing-independent) order.
#pragma once

#include "tdse_internal.hpp"

namespace tdse {

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

__device__ __forceinline__ double2 ldc(const double2* p, int64_t k) { return p[k]; }
__device__ __forceinline__ double2 ldc(const float2* p, int64_t k)
{
    const float2 v = p[k];
    return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void stc(double2* p, int64_t k, double2 v) { p[k] = v; }
__device__ __forceinline__ void stc(float2* p, int64_t k, double2 v)
{
    p[k] = make_float2((float)v.x, (float)v.y);
}

__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }

// A value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ double wave_uniform(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Block-wide sums of NQ values for a kBlock-thread block.  Thread q < NQ of
// the block receives the sum of value q in `out_q` (others get 0).  The
// summation tree depends only on thread indices, so results are bitwise
// reproducible.  The butterfly runs stage by stage over groups of up to 4
// values (not value by value), so the independent shuffles of a stage overlap
// instead of paying the shuffle latency once per value; each value's tree is the xor
// butterfly 32, 16, ..., 1 over the wave's lanes.  Must be reached by every
// thread of the block.
template <int NQ>
__device__ __forceinline__ double block_sum(double (&v)[NQ], double* lds /* [kBlock/64][NQ] */)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // groups of (at most) 4 values: independent shuffles per stage to hide
    // their latency, few enough not to raise the register count of the caller
    constexpr int G = NQ < 4 ? NQ : 4;
#pragma unroll
    for (int q0 = 0; q0 < NQ; q0 += G) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
            for (int q = q0; q < q0 + G && q < NQ; ++q) v[q] += __shfl_xor(v[q], off, 64);
        }
        // each group's totals leave the registers at once
        if (lane == 0) {
#pragma unroll
            for (int q = q0; q < q0 + G && q < NQ; ++q) lds[wave * NQ + q] = v[q];
        }
    }
    __syncthreads();
    double out = 0.0;
    if (threadIdx.x < NQ) {
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) out += lds[w * NQ + threadIdx.x];
    }
    __syncthreads();
    return out;
}

// The tile handled by this workgroup.  order 0: tile = blockIdx.x (the
// hardware deals workgroup b to XCD b mod 8, so consecutive tiles land on
// different XCDs).  order 1: each XCD gets a contiguous run of tiles, so the
// radial and l halos of neighbouring tiles meet in that XCD's L2.  Both are
// bijections of [0, n_tiles); which one streams faster depends on the shape
// and is left to the autotuner.
__device__ __forceinline__ int my_tile_index(const SweepGeom& g)
{
    const int b = (int)blockIdx.x;
    if (g.order == 0) return b;
    const int q = g.n_tiles >> 3, rem = g.n_tiles & 7;
    const int x = b & 7, j = b >> 3;
    return x * q + min(x, rem) + j;
}
__device__ __forceinline__ Tile my_tile(const SweepGeom& g) { return g.tiles[my_tile_index(g)]; }

// A load through the constant address space, for tables that no launch
// writes, read at wave-uniform indexes: it becomes a scalar load, which is
// counted apart from the vector loads in flight, so using the value does not
// wait for them (a plain load after a store in the same kernel stays a vector
// load: the compiler cannot tell that the store does not reach the table).
template <typename X>
__device__ __forceinline__ X ld_const(const X* p, int64_t i)
{
    return ((const __attribute__((address_space(4))) X*)p)[i];
}

// Stencil weights of -1/2 D2 (zero-padded 3- or 5-point second difference).
template <int S> struct Kin;
template <> struct Kin<1> {
    static constexpr double c0 = 1.0, c1 = -0.5, c2 = 0.0;
};
template <> struct Kin<2> {
    static constexpr double c0 = 30.0 / 24.0, c1 = -16.0 / 24.0, c2 = 1.0 / 24.0;
};

// Per-thread radial constants.
struct RadialPoint {
    double r, inv_r2, z_over_r;
};
__device__ __forceinline__ RadialPoint radial_point(const Tile& I, int i)
{
    RadialPoint p;
    p.r = (double)(i + 1) * I.dr;
    const double inv_r = 1.0 / p.r;
    p.inv_r2 = inv_r * inv_r;
    p.z_over_r = I.z * inv_r;
    return p;
}

// Diagonal potential of row l: l(l+1)/(2 r^2) - Z/r.  l(l+1)/2 is formed in
// integers (exact; scalar unit when l is wave-uniform) and converted once.
__device__ __forceinline__ double row_potential(int l, double inv_r2, double z_over_r)
{
    return fma((double)((l * (l + 1)) >> 1), inv_r2, -z_over_r);
}

// (H f)_{l,i} from the centre value, its radial neighbours (already zero
// outside the box) and the values of rows l-1, l+1 at the same radius.
// Every multiply-add is an explicit fma in a fixed order (the library is
// built without implicit contraction), so every kernel that evaluates H
// through this function rounds identically, whatever its loop shape.
template <int S>
__device__ __forceinline__ double2 h_point(double2 cur, double2 m1, double2 p1, double2 m2, double2 p2,
                                           double2 lm, double2 lp, double kin_scale, double v,
                                           double er, double kl, double klp)
{
    const double d0 = fma(Kin<S>::c0, kin_scale, v);
    const double d1 = Kin<S>::c1 * kin_scale;
    const double d2 = Kin<S>::c2 * kin_scale;
    const double ekl = er * kl, eklp = er * klp;
    double hx = eklp * lp.x, hy = eklp * lp.y;
    hx = fma(ekl, lm.x, hx);
    hy = fma(ekl, lm.y, hy);
    if (S == 2) {
        hx = fma(d2, m2.x + p2.x, hx);
        hy = fma(d2, m2.y + p2.y, hy);
    }
    hx = fma(d1, m1.x + p1.x, hx);
    hy = fma(d1, m1.y + p1.y, hy);
    hx = fma(d0, cur.x, hx);
    hy = fma(d0, cur.y, hy);
    return make_double2(hx, hy);
}

// One Horner term: psi + (-i c) h, with (-i c)(x + i y) = c y - i c x.
__device__ __forceinline__ double2 horner_update(double2 psi, double2 h, double c)
{
    return make_double2(fma(c, h.y, psi.x), fma(-c, h.x, psi.y));
}

// Radial neighbours of element i of a row (zero outside [0, n)).
template <int S, typename C>
struct Neighbours {
    double2 m1, p1, m2, p2;
    __device__ __forceinline__ void load(const C* row, int i, int n)
    {
        m1 = (i >= 1) ? ldc(row, i - 1) : zero2();
        p1 = (i + 1 < n) ? ldc(row, i + 1) : zero2();
        if (S == 2) {
            m2 = (i >= 2) ? ldc(row, i - 2) : zero2();
            p2 = (i + 2 < n) ? ldc(row, i + 2) : zero2();
        } else {
            m2 = p2 = zero2();
        }
    }
};

}  // namespace tdse
