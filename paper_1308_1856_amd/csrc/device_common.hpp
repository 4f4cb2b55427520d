// Device helpers: complex loads/stores with FP64 registers, wave64/block
// reductions in FP64 with a fixed (timing-independent) order.
#pragma once

#include "tdse_internal.hpp"

namespace tdse {

// Storage precisions: T = double (16 B per complex element), float (8 B) or
// s48 (12 B).  s48 keeps each FP64 component rounded to 36 mantissa bits
// (relative rounding error at most 2^-37): the upper 32-bit word of the FP64
// bit pattern in plane h (8 B per element: re, im) and the next 16 bits in
// plane l (4 B per element: re in the low half, im in the high half).  A
// state-shaped vector of s48 storage is [plane h | plane l], plane l starting
// 8 * plane bytes after plane h (SweepGeom::plane elements per plane).
struct s48 {};
struct c48 {
    unsigned hx, hy, l;
};
struct P48 {
    uint2* h;
    unsigned* l;
    __host__ __device__ __forceinline__ P48 operator+(int64_t k) const { return P48{h + k, l + k}; }
    __host__ __device__ __forceinline__ P48 operator-(int64_t k) const { return P48{h - k, l - k}; }
    __device__ __forceinline__ c48 operator[](int64_t k) const
    {
        const uint2 a = h[k];
        return c48{a.x, a.y, l[k]};
    }
};

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<s48> { using type = c48; };

// Kernel-argument types of state-shaped vectors and their construction from
// the launchers' untyped pointers (the s48 planes from one base address, or,
// for a run of vectors stored plane by plane, from the two plane bases).
template <typename T> struct Stor {
    using C = typename Cplx<T>::type;
    using cptr = const C* __restrict__;
    using ptr = C* __restrict__;
    using aptr = C*;          // may alias another argument
    using captr = const C*;   // read-only, may alias another argument
    static const C* cmake(const void* p, int64_t) { return static_cast<const C*>(p); }
    static C* make(void* p, int64_t) { return static_cast<C*>(p); }
};
template <> struct Stor<s48> {
    using C = c48;
    using cptr = P48;
    using ptr = P48;
    using aptr = P48;
    using captr = P48;
    static P48 cmake(const void* p, int64_t plane)
    {
        char* b = static_cast<char*>(const_cast<void*>(p));
        return P48{reinterpret_cast<uint2*>(b), reinterpret_cast<unsigned*>(b + 8 * plane)};
    }
    static P48 make(void* p, int64_t plane) { return cmake(p, plane); }
};

// s48 conversions: the FP64 value from its stored words, and the stored words
// of an FP64 value rounded to nearest (ties away from zero) at bit 16.
__device__ __forceinline__ double2 widen48(c48 v)
{
    const unsigned lox = v.l << 16, loy = v.l & 0xffff0000u;
    return make_double2(__hiloint2double((int)v.hx, (int)lox), __hiloint2double((int)v.hy, (int)loy));
}
__device__ __forceinline__ c48 narrow48(double2 v)
{
    const unsigned long long a = (unsigned long long)__double_as_longlong(v.x) + 0x8000ull;
    const unsigned long long b = (unsigned long long)__double_as_longlong(v.y) + 0x8000ull;
    return c48{(unsigned)(a >> 32), (unsigned)(b >> 32), ((unsigned)a >> 16) | ((unsigned)b & 0xffff0000u)};
}

__device__ __forceinline__ double2 ldc(const double2* p, int64_t k) { return p[k]; }
__device__ __forceinline__ double2 ldc(const float2* p, int64_t k)
{
    const float2 v = p[k];
    return make_double2((double)v.x, (double)v.y);
}
// Stores of state-shaped vectors are non-temporal (streaming: the line is
// not kept in the caches for reuse).  A sweep writes each element once and
// reads it, if at all, in a later launch; with ordinary stores the written
// lines displaced the rows still to be read, and the 25.7M-unknown H-psi
// apply took 81 instead of 59 us.
typedef double dvec2_t __attribute__((ext_vector_type(2)));
typedef float fvec2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void stc(double2* p, int64_t k, double2 v)
{
    const dvec2_t w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<dvec2_t*>(p + k));
}
__device__ __forceinline__ void stc(float2* p, int64_t k, double2 v)
{
    const fvec2_t w = {(float)v.x, (float)v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<fvec2_t*>(p + k));
}
__device__ __forceinline__ double2 ldc(P48 p, int64_t k) { return widen48(p[k]); }
typedef unsigned uvec2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void stc(P48 p, int64_t k, double2 v)
{
    const c48 c = narrow48(v);
    const uvec2_t w = {c.hx, c.hy};
    __builtin_nontemporal_store(w, reinterpret_cast<uvec2_t*>(p.h + k));
    __builtin_nontemporal_store(c.l, p.l + k);
}
// The value a store of v keeps, as FP64.
template <typename T> __device__ __forceinline__ double2 stored_value(double2 v);
template <> __device__ __forceinline__ double2 stored_value<double>(double2 v) { return v; }
template <> __device__ __forceinline__ double2 stored_value<float>(double2 v)
{
    return make_double2((double)(float)v.x, (double)(float)v.y);
}
template <> __device__ __forceinline__ double2 stored_value<s48>(double2 v) { return widen48(narrow48(v)); }
// Ordinary stores, for vectors read again while still cache-resident (the
// Lanczos w and basis vectors, reread by the next sweep; measured 2.6% more
// steps per second than with streaming stores).
__device__ __forceinline__ void stc_keep(double2* p, int64_t k, double2 v) { p[k] = v; }
__device__ __forceinline__ void stc_keep(float2* p, int64_t k, double2 v)
{
    p[k] = make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ void stc_keep(P48 p, int64_t k, double2 v)
{
    const c48 c = narrow48(v);
    p.h[k] = make_uint2(c.hx, c.hy);
    p.l[k] = c.l;
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

// A lane's value of v, as a wave-uniform (scalar) value.
__device__ __forceinline__ double lane_value(double v, int lane)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// DPP lane permutations inside each row of 16 lanes (every source lane exists).
constexpr int kDppQuadXor1 = 0xB1;       // quad_perm [1,0,3,2]: lane ^ 1
constexpr int kDppQuadXor2 = 0x4E;       // quad_perm [2,3,0,1]: lane ^ 2
constexpr int kDppRowHalfMirror = 0x141; // lane 7 - i within each 8 lanes
constexpr int kDppRowMirror = 0x140;     // lane 15 - i within each 16 lanes
// Across rows: lane 15 of row r to every lane of row r + 1, lane 31 to rows 2
// and 3 (only the rows enabled by the row mask are written).
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// v of the lane that the row broadcast CTRL names, in the rows ROW_MASK
// enables; 0 in the other rows.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_bcast(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum of v over the 64 lanes of the wave, in registers (no LDS round trip),
// returned as a wave-uniform value.  Inside each row of 16 lanes, v is added
// to its partner at lane ^ 1, then at lane ^ 2, then at its mirror in the half
// row and in the row: each step adds two values that the partner lane adds in
// the other order, and a + b = b + a exactly, so every lane of row r ends
// with the same row sum s_r.  Then rows 1 and 3 add the sums of rows 0 and 2,
// and row 3 adds the result of row 1: lane 63 holds
// (s_2 + s_3) + (s_0 + s_1).  Every lane of the wave must be active.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_row<kDppQuadXor1>(v);
    v += dpp_row<kDppQuadXor2>(v);
    v += dpp_row<kDppRowHalfMirror>(v);
    v += dpp_row<kDppRowMirror>(v);
    v += dpp_bcast<kDppRowBcast15, 0xa>(v);   // rows 1, 3; rows 0, 2 add +0 (exact)
    v += dpp_bcast<kDppRowBcast31, 0xc>(v);   // rows 2, 3
    return lane_value(v, 63);
}

// Block-wide sums of NQ values for a kBlock-thread block.  Thread q < NQ of
// the block receives the sum of value q (others get 0): wave_sum in each
// wave, then the kBlock / 64 wave sums in wave order.  The summation tree
// depends only on lane and wave indices, so results are bitwise reproducible.
// Values go through in groups of 4, each group's sums stored before the next
// group starts, so few sums are held in registers at once.  Must be reached by
// every thread of the block.
template <int NQ>
__device__ __forceinline__ double block_sum(double (&v)[NQ], double* lds /* [kBlock/64][NQ] */)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr int G = NQ < 4 ? NQ : 4;
#pragma unroll
    for (int q0 = 0; q0 < NQ; q0 += G) {
        double s[G];
#pragma unroll
        for (int q = q0; q < q0 + G && q < NQ; ++q) s[q - q0] = wave_sum(v[q]);
        if (lane == 0) {
#pragma unroll
            for (int q = q0; q < q0 + G && q < NQ; ++q) lds[wave * NQ + q] = s[q - q0];
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
// radial and l halos of neighbouring tiles meet in that XCD's L2.  order 2:
// runs of kXcdGroup consecutive tiles go to one XCD, the runs dealt round
// the XCDs: the 8 XCDs still sweep neighbouring tiles at the same time (as
// order 0), and the radial halos inside a run meet in one L2 (the tiles
// past the last whole round of runs keep order 0).  All are bijections of
// [0, n_tiles); which one streams faster depends on the shape and is left to
// the autotuner.
constexpr int kXcdGroup = 4;
__device__ __forceinline__ int my_tile_index(const SweepGeom& g)
{
    const int b = (int)blockIdx.x;
    if (g.order == 0) return b;
    const int x = b & 7, j = b >> 3;
    if (g.order == 2) {
        constexpr int round = 8 * kXcdGroup;
        if (b >= g.n_tiles / round * round) return b;
        return (j / kXcdGroup) * round + x * kXcdGroup + j % kXcdGroup;
    }
    const int q = g.n_tiles >> 3, rem = g.n_tiles & 7;
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
    double r, inv_r, inv_r2, z_over_r;
};
__device__ __forceinline__ RadialPoint radial_point(const Tile& I, int i)
{
    RadialPoint p;
    p.r = (double)(i + 1) * I.dr;
    p.inv_r = 1.0 / p.r;
    p.inv_r2 = p.inv_r * p.inv_r;
    p.z_over_r = I.z * p.inv_r;
    return p;
}

// The diagonal of H on row l at one radius, kinetic centre weight included:
//   d0 = l(l+1)/(2 r^2) + (c0 / dr^2 - Z/r),
// as fma(L, 1/r^2, base) with L = l(l+1)/2 (formed in integers, exact; the
// scalar unit when l is wave-uniform, then one conversion) and base =
// fma(c0, 1/dr^2, -Z/r), formed once per radius.
__device__ __forceinline__ double half_ll(int l) { return (double)((l * (l + 1)) >> 1); }
template <int S>
__device__ __forceinline__ double diag_base(double kin_scale, double z_over_r);
__device__ __forceinline__ double row_diag(double half_ll_l, double inv_r2, double base)
{
    return fma(half_ll_l, inv_r2, base);
}

template <int S>
__device__ __forceinline__ double diag_base(double kin_scale, double z_over_r)
{
    return fma(Kin<S>::c0, kin_scale, -z_over_r);
}

// (H f)_{l,i} from the centre value, its radial neighbours (already zero
// outside the box), the values of rows l-1, l+1 at the same radius and the
// diagonal d0 of row l (row_diag).  Every multiply-add is an explicit fma in
// a fixed order (the library is built without implicit contraction), so
// every kernel that evaluates H through this function rounds identically,
// whatever its loop shape.
template <int S>
__device__ __forceinline__ double2 h_point(double2 cur, double2 m1, double2 p1, double2 m2, double2 p2,
                                           double2 lm, double2 lp, double kin_scale, double d0,
                                           double er, double kl, double klp)
{
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

// The diffusion step's Horner term: psi - c h.
__device__ __forceinline__ double2 horner_update_imag(double2 psi, double2 h, double c)
{
    return make_double2(fma(-c, h.x, psi.x), fma(-c, h.y, psi.y));
}

// Radial neighbours of element i of a row (zero outside [0, n)).
template <int S>
struct Neighbours {
    double2 m1, p1, m2, p2;
    __device__ __forceinline__ void zero() { m1 = p1 = m2 = p2 = zero2(); }
    template <typename P>
    __device__ __forceinline__ void load(P row, int i, int n)
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

// First radial derivative of a row at the point whose neighbours are nb, of
// the stencil's order (Sec. 2): (f_{i+1} - f_{i-1}) / (2 dr), or the
// fourth-order (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2}) / (12 dr).
template <int S>
__device__ __forceinline__ double2 first_derivative(const Neighbours<S>& nb, double inv_dr)
{
    if (S == 1) {
        const double s = 0.5 * inv_dr;
        return make_double2((nb.p1.x - nb.m1.x) * s, (nb.p1.y - nb.m1.y) * s);
    }
    const double s = inv_dr * (1.0 / 12.0);
    return make_double2(fma(8.0, nb.p1.x - nb.m1.x, nb.m2.x - nb.p2.x) * s,
                        fma(8.0, nb.p1.y - nb.m1.y, nb.m2.y - nb.p2.y) * s);
}

// Velocity-gauge coupling of row l (Sec. 2, the V form of the radial TDSE:
// A/c p_z in partial waves):
//   -i a [kappa_l (d/dr - l/r) f_{l-1} + kappa_{l+1} (d/dr + (l+1)/r) f_{l+1}]
// from the values fm, fp of rows l - 1, l + 1 at this radius and their
// radial neighbours (zeros for rows outside [0, lmax]); a = A/c.
template <int S>
__device__ __forceinline__ double2 vel_coupling(double2 fm, const Neighbours<S>& nbm, double2 fp,
                                                const Neighbours<S>& nbp, int l, double inv_r, double inv_dr,
                                                double a, double kl, double klp)
{
    const double2 dm = first_derivative<S>(nbm, inv_dr);
    const double2 dp = first_derivative<S>(nbp, inv_dr);
    const double cm = (double)l * inv_r, cp = (double)(l + 1) * inv_r;
    double cx = kl * fma(-cm, fm.x, dm.x), cy = kl * fma(-cm, fm.y, dm.y);
    cx = fma(klp, fma(cp, fp.x, dp.x), cx);
    cy = fma(klp, fma(cp, fp.y, dp.y), cy);
    return make_double2(a * cy, -(a * cx));   // -i a (cx + i cy)
}

}  // namespace tdse
