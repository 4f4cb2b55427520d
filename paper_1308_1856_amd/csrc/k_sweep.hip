// Sweep kernels: H.psi (Sec. 2, eq. h_matrix), one fused Horner term of the
// Taylor step (Sec. 5.2, eq. Taylor) and the fused classic RK4 stage
// (Sec. 5.2, eq. RKDeriv).
//
// Work decomposition: a workgroup of 256 threads owns a radial segment of
// rows [l0, l1) of one instance.  Each thread walks down its rows keeping
// f_{l-1}, f_l, f_{l+1} at its radii in registers, so the l +- 1 coupling
// costs one new load per row.  All arithmetic is FP64; storage is FP64 or
// FP32.  HBM traffic per unknown and term: read `in` once, read psi once,
// write out once.
//
// Two sweep shapes (the autotuner picks per problem shape):
//   k_hsweep       one radius per thread (256 radii per tile); the radial
//                  neighbours come from the same row through L1.
//   k_hsweep_pair  two adjacent radii per thread (512 radii per tile): one
//                  16-byte FP32 (or two 16-byte FP64) load per row and
//                  stream, radial neighbours from the adjacent lanes by
//                  shuffles, only the first and last lane of a wave load a
//                  neighbour from memory.  Twice the bytes in flight per
//                  wave, which the FP32 sweep needs to approach the HBM
//                  ceiling; values are held in storage precision until use
//                  to keep the register count (and so the occupancy) up.
// Both evaluate H through h_point and the term through horner_update, so
// they agree bit for bit.
#include <type_traits>

#include "device_common.hpp"

namespace tdse {

// IMAG (term < 0): the Horner term of the diffusion (imaginary-time) step,
// out = psi - (dtau / |term|) H in (the factor -i of the Taylor step replaced
// by -1; Sec. 4, ground state calculation).
// VG: the velocity gauge (the kEMid slot holds A/c; the coupling takes the
// radial neighbours of rows l -+ 1, kept from the rows before and after).
template <int S, typename T, bool IMAG = false, bool VG = false>
__global__ void __launch_bounds__(kBlock)
k_hsweep(SweepGeom g, typename Stor<T>::cptr in, typename Stor<T>::cptr psi, typename Stor<T>::ptr out,
         const double* __restrict__ step, int term)
{
    const Tile I = my_tile(g);
    const int n = I.n;
    const int i = I.r0 + (int)threadIdx.x;
    if (i >= n) return;
    const RadialPoint rp = radial_point(I, i);
    const double fld = step_value(step, g.n_inst, kEMid, I.inst);
    const double er = VG ? 0.0 : fld * rp.r;
    const double inv_dr = 1.0 / I.dr;
    const double c = IMAG ? step_value(step, g.n_inst, kDt, I.inst) / (double)(-term)
                          : (term > 0) ? step_value(step, g.n_inst, kDt, I.inst) / (double)term : 0.0;
    const int64_t base = I.off;
    double2 prev = (I.l0 > 0) ? ldc(in, base + (int64_t)(I.l0 - 1) * n + i) : zero2();
    double2 cur = ldc(in, base + (int64_t)I.l0 * n + i);
    Neighbours<S> nbm, nb;   // rows l - 1 and l (velocity gauge)
    if (VG) {
        nbm.zero();
        if (I.l0 > 0) nbm.load(in + (base + (int64_t)(I.l0 - 1) * n), i, n);
        nb.load(in + (base + (int64_t)I.l0 * n), i, n);
    }
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t row = base + (int64_t)l * n;
        const double2 next = (l < I.lmax) ? ldc(in, row + n + i) : zero2();
        Neighbours<S> nbp;
        if (VG) {
            nbp.zero();
            if (l < I.lmax) nbp.load(in + (row + n), i, n);
        } else {
            nb.load(in + row, i, n);
        }
        const double d0 = row_diag(half_ll(l), rp.inv_r2, diag_base<S>(I.inv_dr2, rp.z_over_r));
        double2 h = h_point<S>(cur, nb.m1, nb.p1, nb.m2, nb.p2, prev, next, I.inv_dr2, d0, er,
                               g.kappa[l], g.kappa[l + 1]);
        if (VG) {
            const double2 w = vel_coupling<S>(prev, nbm, next, nbp, l, rp.inv_r, inv_dr, fld, g.kappa[l],
                                              g.kappa[l + 1]);
            h.x += w.x;
            h.y += w.y;
            nbm = nb;
            nb = nbp;
        }
        if (IMAG)
            stc(out, row + i, horner_update_imag(ldc(psi, row + i), h, c));
        else if (term > 0)
            stc(out, row + i, horner_update(ldc(psi, row + i), h, c));
        else
            stc(out, row + i, h);
        prev = cur;
        cur = next;
    }
}

// Two adjacent elements of a row, kept in storage precision.
template <typename C> struct PairReg;
template <> struct PairReg<float2> {
    float2 a, b;
    __device__ __forceinline__ double2 da() const { return make_double2((double)a.x, (double)a.y); }
    __device__ __forceinline__ double2 db() const { return make_double2((double)b.x, (double)b.y); }
};
template <> struct PairReg<double2> {
    double2 a, b;
    __device__ __forceinline__ double2 da() const { return a; }
    __device__ __forceinline__ double2 db() const { return b; }
};
// Four floats at 8-byte alignment: one 16-byte access for an FP32 pair whose
// first element sits at an odd element offset (rows of odd length).
struct alignas(8) Float4a8 {
    float x, y, z, w;
};

// Loads elements k, k + 1 (both < the row end when `full`; only k when only
// `live`; none otherwise, giving zeros).
template <typename C>
__device__ __forceinline__ void load_pair(const C* p, int64_t k, bool full, bool live, PairReg<C>& v)
{
    if (full) {
        if constexpr (sizeof(C) == 8) {
            const Float4a8 w = *reinterpret_cast<const Float4a8*>(p + k);
            v.a = make_float2(w.x, w.y);
            v.b = make_float2(w.z, w.w);
        } else {
            v.a = p[k];
            v.b = p[k + 1];
        }
    } else if (live) {
        v.a = p[k];
        v.b = C{};
    } else {
        v.a = C{};
        v.b = C{};
    }
}
// (non-temporal, as stc)
typedef float fvec4a8_t __attribute__((ext_vector_type(4), aligned(8)));
__device__ __forceinline__ void store_pair(float2* p, int64_t k, double2 a, double2 b)
{
    const fvec4a8_t w = {(float)a.x, (float)a.y, (float)b.x, (float)b.y};
    __builtin_nontemporal_store(w, reinterpret_cast<fvec4a8_t*>(p + k));
}
__device__ __forceinline__ void store_pair(double2* p, int64_t k, double2 a, double2 b)
{
    stc(p, k, a);
    stc(p, k + 1, b);
}
__device__ __forceinline__ double2 from_lane_below(double2 v)
{
    return make_double2(__shfl_up(v.x, 1, 64), __shfl_up(v.y, 1, 64));
}
__device__ __forceinline__ double2 from_lane_above(double2 v)
{
    return make_double2(__shfl_down(v.x, 1, 64), __shfl_down(v.y, 1, 64));
}

// Thread t of a tile owns radii e = r0 + 2t and e + 1 (tiles are 512 radii
// wide).  Row values of the pair: a = f(e), b = f(e + 1); the neighbours
// e - 1, e - 2 are lane t-1's b, a and e + 2, e + 3 are lane t+1's a, b.
// Every lane executes the shuffles (no early exit); lanes past the row end
// hold zeros and store nothing.
template <int S, typename T, bool TERM>
__global__ void __launch_bounds__(kBlock)
k_hsweep_pair(SweepGeom g, const typename Cplx<T>::type* __restrict__ in,
              const typename Cplx<T>::type* __restrict__ psi, typename Cplx<T>::type* __restrict__ out,
              const double* __restrict__ step, int term)
{
    using C = typename Cplx<T>::type;
    const Tile I = my_tile(g);
    const int n = I.n;
    const int lane = (int)threadIdx.x & 63;
    const int e = I.r0 + 2 * (int)threadIdx.x;
    const bool live = e < n, full = e + 1 < n;
    const int ec = live ? e : 0;
    const double ra = (double)(ec + 1) * I.dr, rb = (double)(ec + 2) * I.dr;
    const double ira = 1.0 / ra, irb = 1.0 / rb;
    const double ira2 = ira * ira, irb2 = irb * irb, zra = I.z * ira, zrb = I.z * irb;
    const double ef = step_value(step, g.n_inst, kEMid, I.inst);
    // wave-uniform: kept in scalar registers
    const double c = TERM ? wave_uniform(step_value(step, g.n_inst, kDt, I.inst) / (double)term) : 0.0;
    const C* in_i = in + I.off;
    const C* psi_i = psi + I.off;
    C* out_i = out + I.off;

    PairReg<C> P, Cu, N, Q;
    P.a = P.b = N.a = N.b = Q.a = Q.b = C{};
    if (I.l0 > 0) load_pair(in_i, (int64_t)(I.l0 - 1) * n + ec, full, live, P);
    load_pair(in_i, (int64_t)I.l0 * n + ec, full, live, Cu);
    if (I.l0 < I.lmax) load_pair(in_i, (int64_t)(I.l0 + 1) * n + ec, full, live, N);
    if (TERM) load_pair(psi_i, (int64_t)I.l0 * n + ec, full, live, Q);
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t row = (int64_t)l * n;
        const double2 ca = Cu.da(), cb = Cu.db();
        double2 xm1 = from_lane_below(cb), xp2 = from_lane_above(ca), xm2 = zero2(), xp3 = zero2();
        if (S == 2) {
            xm2 = from_lane_below(ca);
            xp3 = from_lane_above(cb);
        }
        if (lane == 0) {
            xm1 = (live && ec >= 1) ? ldc(in_i, row + ec - 1) : zero2();
            if (S == 2) xm2 = (live && ec >= 2) ? ldc(in_i, row + ec - 2) : zero2();
        }
        if (lane == 63) {
            xp2 = (live && ec + 2 < n) ? ldc(in_i, row + ec + 2) : zero2();
            if (S == 2) xp3 = (live && ec + 3 < n) ? ldc(in_i, row + ec + 3) : zero2();
        }
        const double kl = g.kappa[l], klp = g.kappa[l + 1];
        const double2 ha = h_point<S>(ca, xm1, cb, xm2, xp2, P.da(), N.da(), I.inv_dr2,
                                      row_diag(half_ll(l), ira2, diag_base<S>(I.inv_dr2, zra)), ef * ra, kl, klp);
        const double2 hb = h_point<S>(cb, ca, xp2, xm1, xp3, P.db(), N.db(), I.inv_dr2,
                                      row_diag(half_ll(l), irb2, diag_base<S>(I.inv_dr2, zrb)), ef * rb, kl, klp);
        const double2 oa = TERM ? horner_update(Q.da(), ha, c) : ha;
        const double2 ob = TERM ? horner_update(Q.db(), hb, c) : hb;
        if (full)
            store_pair(out_i, row + ec, oa, ob);
        else if (live)
            stc(out_i, row + ec, oa);
        P = Cu;
        Cu = N;
        if (l + 2 <= I.lmax) load_pair(in_i, row + 2 * (int64_t)n + ec, full, live, N);
        else N.a = N.b = C{};
        if (TERM && l + 1 < I.l1) load_pair(psi_i, row + n + ec, full, live, Q);
    }
}

// Classic RK4 with k_s = -i H(t_s) g_s:
//   stage 0: g = psi                 acc  = psi + dt/6 k, gout = psi + dt/2 k
//   stage 1: g = gin                 acc += dt/3 k,       gout = psi + dt/2 k
//   stage 2: g = gin                 acc += dt/3 k,       gout = psi + dt k
//   stage 3: g = gin                 psi  = acc + dt/6 k
// H is taken at t_n (stage 0), t_n + dt/2 (stages 1, 2) and t_n + dt (stage 3).
template <int S, typename T, int STAGE, bool VG = false>
__global__ void __launch_bounds__(kBlock)
k_rk4_stage(SweepGeom g, typename Stor<T>::cptr gin, typename Stor<T>::aptr psi, typename Stor<T>::aptr acc,
            typename Stor<T>::ptr gout, const double* __restrict__ step)
{
    const Tile I = my_tile(g);
    const int n = I.n;
    const int i = I.r0 + (int)threadIdx.x;
    if (i >= n) return;
    const RadialPoint rp = radial_point(I, i);
    const int slot = (STAGE == 0) ? kEStart : (STAGE == 3 ? kEEnd : kEMid);
    const double fld = step_value(step, g.n_inst, slot, I.inst);
    const double er = VG ? 0.0 : fld * rp.r;
    const double inv_dr = 1.0 / I.dr;
    const double dt = step_value(step, g.n_inst, kDt, I.inst);
    const double bw = (STAGE == 0 || STAGE == 3) ? dt / 6.0 : dt / 3.0;
    const double aw = (STAGE == 2) ? dt : 0.5 * dt;
    const int64_t base = I.off;
    constexpr bool kReadAcc = STAGE > 0;
    constexpr bool kReadPsi = STAGE == 1 || STAGE == 2;

    // software pipeline: row l + 1's loads go out before row l
    // is stored (acc and psi are read and written only at a thread's own
    // elements, one row apart)
    const auto row0 = gin + base + (int64_t)I.l0 * n;
    double2 prev = (I.l0 > 0) ? ldc(row0 - n, i) : zero2();
    double2 cur = ldc(row0, i);
    double2 next = (I.l0 < I.lmax) ? ldc(row0 + n, i) : zero2();
    Neighbours<S> nb, nbm;   // rows l and (velocity gauge) l - 1
    nb.load(row0, i, n);
    if (VG) {
        nbm.zero();
        if (I.l0 > 0) nbm.load(row0 - n, i, n);
    }
    double2 a = kReadAcc ? ldc(acc, base + (int64_t)I.l0 * n + i) : zero2();
    double2 p = kReadPsi ? ldc(psi, base + (int64_t)I.l0 * n + i) : zero2();
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t row = base + (int64_t)l * n;
        const bool more = l + 1 < I.l1;
        const double2 next2 = (l + 2 <= I.lmax) ? ldc(gin, row + 2 * n + i) : zero2();
        Neighbours<S> nb_next;
        // the velocity gauge needs row l + 1's neighbours also past the tile
        const bool want_next = VG ? (l + 1 <= I.lmax) : more;
        if (VG) nb_next.zero();
        if (want_next) nb_next.load(gin + row + n, i, n);
        const double2 a_next = (kReadAcc && more) ? ldc(acc, row + n + i) : zero2();
        const double2 p_next = (kReadPsi && more) ? ldc(psi, row + n + i) : zero2();

        const double d0 = row_diag(half_ll(l), rp.inv_r2, diag_base<S>(I.inv_dr2, rp.z_over_r));
        double2 h = h_point<S>(cur, nb.m1, nb.p1, nb.m2, nb.p2, prev, next, I.inv_dr2, d0, er,
                               g.kappa[l], g.kappa[l + 1]);
        if (VG) {
            const double2 w = vel_coupling<S>(prev, nbm, next, nb_next, l, rp.inv_r, inv_dr, fld, g.kappa[l],
                                              g.kappa[l + 1]);
            h.x += w.x;
            h.y += w.y;
            nbm = nb;
        }
        // x + w k with k = -i h
        if (STAGE == 0) {
            stc(acc, row + i, horner_update(cur, h, bw));
            stc(gout, row + i, horner_update(cur, h, aw));
        } else if (STAGE < 3) {
            stc(acc, row + i, horner_update(a, h, bw));
            stc(gout, row + i, horner_update(p, h, aw));
        } else {
            stc(psi, row + i, horner_update(a, h, bw));
        }
        prev = cur;
        cur = next;
        next = next2;
        if (more) nb = nb_next;
        a = a_next;
        p = p_next;
    }
}

__device__ __forceinline__ void copy_elem(const double2* src, double2* dst, int64_t k) { dst[k] = src[k]; }
__device__ __forceinline__ void copy_elem(const float2* src, float2* dst, int64_t k) { dst[k] = src[k]; }
__device__ __forceinline__ void copy_elem(P48 src, P48 dst, int64_t k)
{
    dst.h[k] = src.h[k];
    dst.l[k] = src.l[k];
}

// Stage i of an explicit Runge-Kutta step given by its tableau (see
// launch_rk_stage): H at the stage's time on g_i, k_i = -i H g_i, then the
// combination of the stage weights in stage order, j = 0..i.
template <int S, typename T, bool VG = false>
__global__ void __launch_bounds__(kBlock)
k_rk_stage(SweepGeom g, typename Stor<T>::cptr gin, typename Stor<T>::cptr psi, typename Stor<T>::aptr kv,
           int64_t kstride, typename Stor<T>::ptr next, const double* __restrict__ step, RkStage A,
           double* __restrict__ err_partial)
{
    __shared__ double lds[kBlock / 64];
    const int t = my_tile_index(g);
    const Tile I = g.tiles[t];
    const int n = I.n;
    const int i = I.r0 + (int)threadIdx.x;
    double acc[1] = {0.0};
    if (i < n) {
        const RadialPoint rp = radial_point(I, i);
        const double fld = step_value(step, g.n_inst, A.slot, I.inst);
        const double er = VG ? 0.0 : fld * rp.r;
        const double inv_dr = 1.0 / I.dr;
        const double dt = step_value(step, g.n_inst, kDt, I.inst);
        const int64_t base = I.off;
        double2 prev = (I.l0 > 0) ? ldc(gin, base + (int64_t)(I.l0 - 1) * n + i) : zero2();
        double2 cur = ldc(gin, base + (int64_t)I.l0 * n + i);
        Neighbours<S> nbm, nb;   // rows l - 1 and l (velocity gauge)
        if (VG) {
            nbm.zero();
            if (I.l0 > 0) nbm.load(gin + (base + (int64_t)(I.l0 - 1) * n), i, n);
            nb.load(gin + (base + (int64_t)I.l0 * n), i, n);
        }
        for (int l = I.l0; l < I.l1; ++l) {
            const int64_t row = base + (int64_t)l * n;
            const double2 nx = (l < I.lmax) ? ldc(gin, row + n + i) : zero2();
            Neighbours<S> nbp;
            if (VG) {
                nbp.zero();
                if (l < I.lmax) nbp.load(gin + (row + n), i, n);
            } else {
                nb.load(gin + row, i, n);
            }
            const double d0 = row_diag(half_ll(l), rp.inv_r2, diag_base<S>(I.inv_dr2, rp.z_over_r));
            double2 h = h_point<S>(cur, nb.m1, nb.p1, nb.m2, nb.p2, prev, nx, I.inv_dr2, d0, er,
                                   g.kappa[l], g.kappa[l + 1]);
            if (VG) {
                const double2 w = vel_coupling<S>(prev, nbm, nx, nbp, l, rp.inv_r, inv_dr, fld, g.kappa[l],
                                                  g.kappa[l + 1]);
                h.x += w.x;
                h.y += w.y;
                nbm = nb;
                nb = nbp;
            }
            const double2 ki = make_double2(h.y, -h.x);      // -i h
            if (!A.last) stc(kv + (int64_t)A.stage * kstride, row + i, ki);
            double2 sum = zero2(), dev = zero2();
#pragma unroll
            for (int j = 0; j < kRkMax; ++j) {
                if (j < A.stage) {
                    const double2 kj = ldc(kv + (int64_t)j * kstride, row + i);
                    sum = make_double2(fma(A.w[j], kj.x, sum.x), fma(A.w[j], kj.y, sum.y));
                    if (A.err) dev = make_double2(fma(A.we[j], kj.x, dev.x), fma(A.we[j], kj.y, dev.y));
                }
            }
            sum = make_double2(fma(A.w[A.stage], ki.x, sum.x), fma(A.w[A.stage], ki.y, sum.y));
            const double2 p = ldc(psi, row + i);
            stc(next, row + i, make_double2(fma(dt, sum.x, p.x), fma(dt, sum.y, p.y)));
            if (A.err) {
                dev = make_double2(fma(A.we[A.stage], ki.x, dev.x), fma(A.we[A.stage], ki.y, dev.y));
                const double dx = dt * dev.x, dy = dt * dev.y;
                acc[0] = fma(dx, dx, fma(dy, dy, acc[0]));
            }
            prev = cur;
            cur = nx;
        }
    }
    if (A.err) {   // uniform over the launch
        const double s = block_sum<1>(acc, lds);
        if (threadIdx.x == 0) err_partial[t] = s;
    }
}

// One workgroup per instance: sigma[k] += sqrt(sum_t partial[t] / U_k) over
// the instance's sweep tiles (each thread adds its tiles in order, then the
// fixed block tree).
__global__ void __launch_bounds__(kBlock)
k_rk_sigma(SweepGeom g, const double* __restrict__ partial, double* __restrict__ sigma)
{
    __shared__ double lds[kBlock / 64];
    const int k = blockIdx.x;
    const Inst& I = g.inst[k];
    double acc[1] = {0.0};
    for (int t = I.tbegin[kSweepTiles] + (int)threadIdx.x; t < I.tend[kSweepTiles]; t += kBlock) acc[0] += partial[t];
    const double s = block_sum<1>(acc, lds);
    if (threadIdx.x == 0) sigma[k] += sqrt(s / ((double)(I.lmax + 1) * (double)I.n));
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_copy(SweepGeom g, typename Stor<T>::cptr src, typename Stor<T>::ptr dst)
{
    const Tile I = my_tile(g);
    const int i = I.r0 + (int)threadIdx.x;
    if (i >= I.n) return;
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t k = I.off + (int64_t)l * I.n + i;
        copy_elem(src, dst, k);
    }
}

__device__ __forceinline__ bool bits_differ(double2 a, double2 b)
{
    return __double_as_longlong(a.x) != __double_as_longlong(b.x) ||
           __double_as_longlong(a.y) != __double_as_longlong(b.y);
}
__device__ __forceinline__ bool bits_differ(float2 a, float2 b)
{
    return __float_as_uint(a.x) != __float_as_uint(b.x) || __float_as_uint(a.y) != __float_as_uint(b.y);
}
__device__ __forceinline__ bool bits_differ(c48 a, c48 b) { return a.hx != b.hx || a.hy != b.hy || a.l != b.l; }

// Counts elements (over the tiles of g) whose stored values differ bit for bit.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_count_diff(SweepGeom g, typename Stor<T>::cptr a, typename Stor<T>::cptr b, unsigned int* __restrict__ count)
{
    const Tile I = my_tile(g);
    const int i = I.r0 + (int)threadIdx.x;
    if (i >= I.n) return;
    unsigned int d = 0;
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t k = I.off + (int64_t)l * I.n + i;
        d += bits_differ(a[k], b[k]) ? 1u : 0u;
    }
    if (d) atomicAdd(count, d);
}

// out[0] += sum |a - b|^2, out[1] += sum |b|^2 over the tiles of g (FP64).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_diff_norm(SweepGeom g, typename Stor<T>::cptr a, typename Stor<T>::cptr b, double* __restrict__ out)
{
    __shared__ double lds[(kBlock / 64) * 2];
    const Tile I = my_tile(g);
    const int i = I.r0 + (int)threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (i < I.n) {
        for (int l = I.l0; l < I.l1; ++l) {
            const int64_t k = I.off + (int64_t)l * I.n + i;
            const double2 x = ldc(a, k), y = ldc(b, k);
            const double dx = x.x - y.x, dy = x.y - y.y;
            acc[0] += dx * dx + dy * dy;
            acc[1] += y.x * y.x + y.y * y.y;
        }
    }
    const double s = block_sum<2>(acc, lds);
    if (threadIdx.x < 2) atomicAdd(&out[threadIdx.x], s);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int S, typename T>
static hipError_t hsweep_t(const SweepGeom& g, const void* in, const void* psi, void* out,
                           const double* step, int term, hipStream_t st)
{
    using C = typename Cplx<T>::type;
    if (g.gauge != 0) {   // velocity gauge: one radius per thread, real-time terms and H only
        if (g.variant != 0 || term < 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_hsweep<S, T, false, true>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(in, g.plane), Stor<T>::cmake(psi, g.plane), Stor<T>::make(out, g.plane),
                           step, term);
        return hipGetLastError();
    }
    if (term < 0) {   // the diffusion step's Horner terms: one radius per thread
        if (g.variant != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_hsweep<S, T, true>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::cmake(in, g.plane),
                           Stor<T>::cmake(psi, g.plane), Stor<T>::make(out, g.plane), step, term);
        return hipGetLastError();
    }
    if constexpr (std::is_same<T, s48>::value) {
        if (g.variant == 1) return hipErrorInvalidValue;   // two-radii sweeps: FP64 and FP32 storage only
    } else {
        if (g.variant == 1 && term > 0)
            hipLaunchKernelGGL((k_hsweep_pair<S, T, true>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                               static_cast<const C*>(in), static_cast<const C*>(psi), static_cast<C*>(out),
                               step, term);
        else if (g.variant == 1)
            hipLaunchKernelGGL((k_hsweep_pair<S, T, false>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                               static_cast<const C*>(in), static_cast<const C*>(psi), static_cast<C*>(out),
                               step, term);
        if (g.variant == 1) return hipGetLastError();
    }
    hipLaunchKernelGGL((k_hsweep<S, T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::cmake(in, g.plane),
                       Stor<T>::cmake(psi, g.plane), Stor<T>::make(out, g.plane), step, term);
    return hipGetLastError();
}

hipError_t launch_hsweep(int prec, int S, const SweepGeom& g, const void* in, const void* psi,
                         void* out, const double* step, int term, hipStream_t st)
{
    if (g.set == kApplyTiles && g.gauge != 0) return hipErrorInvalidValue;
    if (g.set == kApplyTiles) return launch_strip_sweep(prec, S, g, in, psi, out, step, term, st);
    if (prec == 0) return S == 1 ? hsweep_t<1, double>(g, in, psi, out, step, term, st)
                                 : hsweep_t<2, double>(g, in, psi, out, step, term, st);
    if (prec == 2) return S == 1 ? hsweep_t<1, s48>(g, in, psi, out, step, term, st)
                                 : hsweep_t<2, s48>(g, in, psi, out, step, term, st);
    return S == 1 ? hsweep_t<1, float>(g, in, psi, out, step, term, st)
                  : hsweep_t<2, float>(g, in, psi, out, step, term, st);
}

template <int S, typename T, int STAGE>
static hipError_t rk4_t(const SweepGeom& g, const void* gin, const void* psi, void* acc, void* gout,
                        const double* step, hipStream_t st)
{
    if (g.gauge != 0)
        hipLaunchKernelGGL((k_rk4_stage<S, T, STAGE, true>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(gin, g.plane), Stor<T>::make(const_cast<void*>(psi), g.plane),
                           Stor<T>::make(acc, g.plane), Stor<T>::make(gout, g.plane), step);
    else
        hipLaunchKernelGGL((k_rk4_stage<S, T, STAGE>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(gin, g.plane), Stor<T>::make(const_cast<void*>(psi), g.plane),
                           Stor<T>::make(acc, g.plane), Stor<T>::make(gout, g.plane), step);
    return hipGetLastError();
}

template <int S, typename T>
static hipError_t rk4_s(const SweepGeom& g, int stage, const void* gin, const void* psi, void* acc,
                        void* gout, const double* step, hipStream_t st)
{
    switch (stage) {
        case 0: return rk4_t<S, T, 0>(g, gin, psi, acc, gout, step, st);
        case 1: return rk4_t<S, T, 1>(g, gin, psi, acc, gout, step, st);
        case 2: return rk4_t<S, T, 2>(g, gin, psi, acc, gout, step, st);
        default: return rk4_t<S, T, 3>(g, gin, psi, acc, gout, step, st);
    }
}

hipError_t launch_rk4_stage(int prec, int S, const SweepGeom& g, int stage, const void* gin,
                            const void* psi, void* acc, void* gout, const double* step,
                            hipStream_t st)
{
    if (prec == 0) return S == 1 ? rk4_s<1, double>(g, stage, gin, psi, acc, gout, step, st)
                                 : rk4_s<2, double>(g, stage, gin, psi, acc, gout, step, st);
    if (prec == 2) return S == 1 ? rk4_s<1, s48>(g, stage, gin, psi, acc, gout, step, st)
                                 : rk4_s<2, s48>(g, stage, gin, psi, acc, gout, step, st);
    return S == 1 ? rk4_s<1, float>(g, stage, gin, psi, acc, gout, step, st)
                  : rk4_s<2, float>(g, stage, gin, psi, acc, gout, step, st);
}

template <int S, typename T>
static hipError_t rk_stage_t(const SweepGeom& g, const void* gin, const void* psi, void* kv, int64_t kstride, int nk,
                             void* next, const double* step, const RkStage& a, double* err_partial, hipStream_t st)
{
    typename Stor<T>::aptr k;
    if constexpr (std::is_same<T, s48>::value) {
        char* b = static_cast<char*>(kv);
        k = P48{reinterpret_cast<uint2*>(b), reinterpret_cast<unsigned*>(b + 8 * kstride * (int64_t)max(nk, 0))};
    } else {
        k = static_cast<typename Cplx<T>::type*>(kv);
    }
    if (g.gauge != 0)
        hipLaunchKernelGGL((k_rk_stage<S, T, true>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(gin, g.plane), Stor<T>::cmake(psi, g.plane), k, kstride,
                           Stor<T>::make(next, g.plane), step, a, err_partial);
    else
        hipLaunchKernelGGL((k_rk_stage<S, T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::cmake(gin, g.plane),
                           Stor<T>::cmake(psi, g.plane), k, kstride, Stor<T>::make(next, g.plane), step, a,
                           err_partial);
    return hipGetLastError();
}

hipError_t launch_rk_stage(int prec, int S, const SweepGeom& g, const void* gin, const void* psi, void* kv,
                           int64_t kstride, int nk, void* next, const double* step, const RkStage& a,
                           double* err_partial, hipStream_t st)
{
    if (g.variant != 0 || a.stage < 0 || a.stage >= kRkMax) return hipErrorInvalidValue;
    if (prec == 0) return S == 1 ? rk_stage_t<1, double>(g, gin, psi, kv, kstride, nk, next, step, a, err_partial, st)
                                 : rk_stage_t<2, double>(g, gin, psi, kv, kstride, nk, next, step, a, err_partial, st);
    if (prec == 2) return S == 1 ? rk_stage_t<1, s48>(g, gin, psi, kv, kstride, nk, next, step, a, err_partial, st)
                                 : rk_stage_t<2, s48>(g, gin, psi, kv, kstride, nk, next, step, a, err_partial, st);
    return S == 1 ? rk_stage_t<1, float>(g, gin, psi, kv, kstride, nk, next, step, a, err_partial, st)
                  : rk_stage_t<2, float>(g, gin, psi, kv, kstride, nk, next, step, a, err_partial, st);
}

hipError_t launch_rk_sigma(const SweepGeom& g, const double* err_partial, double* sigma, hipStream_t st)
{
    hipLaunchKernelGGL(k_rk_sigma, dim3(g.n_inst), dim3(kBlock), 0, st, g, err_partial, sigma);
    return hipGetLastError();
}

template <typename T>
static hipError_t count_diff_t(const SweepGeom& g, const void* a, const void* b, unsigned int* count,
                               hipStream_t st)
{
    hipLaunchKernelGGL((k_count_diff<T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::cmake(a, g.plane),
                       Stor<T>::cmake(b, g.plane), count);
    return hipGetLastError();
}
hipError_t launch_count_diff(int prec, const SweepGeom& g, const void* a, const void* b,
                             unsigned int* count, hipStream_t st)
{
    if (prec == 0) return count_diff_t<double>(g, a, b, count, st);
    if (prec == 2) return count_diff_t<s48>(g, a, b, count, st);
    return count_diff_t<float>(g, a, b, count, st);
}

template <typename T>
static hipError_t diff_norm_t(const SweepGeom& g, const void* a, const void* b, double* out, hipStream_t st)
{
    hipLaunchKernelGGL((k_diff_norm<T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::cmake(a, g.plane),
                       Stor<T>::cmake(b, g.plane), out);
    return hipGetLastError();
}
hipError_t launch_diff_norm(int prec, const SweepGeom& g, const void* a, const void* b, double* out,
                            hipStream_t st)
{
    if (prec == 0) return diff_norm_t<double>(g, a, b, out, st);
    if (prec == 2) return diff_norm_t<s48>(g, a, b, out, st);
    return diff_norm_t<float>(g, a, b, out, st);
}

template <typename T>
static hipError_t copy_t(const SweepGeom& g, const void* src, void* dst, hipStream_t st)
{
    hipLaunchKernelGGL((k_copy<T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::cmake(src, g.plane),
                       Stor<T>::make(dst, g.plane));
    return hipGetLastError();
}
hipError_t launch_copy(int prec, const SweepGeom& g, const void* src, void* dst, hipStream_t st)
{
    if (prec == 0) return copy_t<double>(g, src, dst, st);
    if (prec == 2) return copy_t<s48>(g, src, dst, st);
    return copy_t<float>(g, src, dst, st);
}

}  // namespace tdse
