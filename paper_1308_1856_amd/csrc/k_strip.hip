// K consecutive Horner terms of the Taylor step (Sec. 5.2, eq. Taylor) in one
// launch, computed by independent wave-wide radial strips with no LDS and no
// barriers.
//
//   v_0 = in,  v_k = psi + (-i dt / t_k) H v_{k-1}   (k = 1..K, t_k = first_term - k + 1)
//   out = v_K
//
// A wave owns 64 consecutive radii j = o - Kt s + lane (s = 1 or 2 for the
// 3- or 5-point stencil; Kt >= K is the term count the tile set was built
// for, passed in g.variant) and writes level K on the middle 64 - 2 Kt s of
// them: every level needs its radial neighbours (lane +- 1, +- 2 by
// shuffles), so the lanes whose values are exact shrink by s per side and
// level.  Adjacent strips overlap by 2 Kt s radii; each output radius is
// written by exactly one strip.  Along l, level k runs one row behind level k-1 within an iteration:
//   rho_k(it) = l0 - K + 2 - k + it,   it = 0 .. (l1 - l0) + 2K - 3,
// so level k at row rho needs level k-1 at rows rho-1 (two iterations ago),
// rho (one iteration ago) and rho+1 (this iteration): each level keeps its
// last two rows in registers, per thread.  Level k is skipped while
// it < 2(k-1) (rows no output depends on).  The input rows and psi are read
// once per iteration with one iteration of prefetch; psi(rho_1) is passed
// down a shift register to the later levels.
//
// Every element is computed by h_point and horner_update, the functions of
// the single-term sweeps, from the same FP64 operands, so FP64 results are
// bit-identical to K single-term launches; with FP32 storage the
// intermediate levels stay FP64.  Rows outside [0, lmax] and radii outside
// [0, N) are zero at every level, as in the single-term sweep.  HBM traffic
// per unknown and launch: read `in` and psi once (plus the row and radial
// overlaps), write out once.  `out` must not alias `in` or `psi`.
#include "device_common.hpp"

namespace tdse {

template <typename C> __device__ __forceinline__ C zero_c();
template <> __device__ __forceinline__ float2 zero_c<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 zero_c<double2>() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 widen(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double2 widen(double2 v) { return v; }
__device__ __forceinline__ double2 pick2(bool c, double2 a, double2 b)
{
    return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
__device__ __forceinline__ double2 lane_below(double2 v, int d)
{
    return make_double2(__shfl_up(v.x, d, 64), __shfl_up(v.y, d, 64));
}
__device__ __forceinline__ double2 lane_above(double2 v, int d)
{
    return make_double2(__shfl_down(v.x, d, 64), __shfl_down(v.y, d, 64));
}

template <int S, typename T, int K>
__global__ void __launch_bounds__(kBlock)
k_horner_strip(SweepGeom g, const typename Cplx<T>::type* __restrict__ in,
               const typename Cplx<T>::type* __restrict__ psi, typename Cplx<T>::type* __restrict__ out,
               const double* __restrict__ step, int first_term)
{
    using C = typename Cplx<T>::type;
    const int halo = g.variant * S;             // >= K * S: lanes lost per side after K levels
    const int valid = 64 - 2 * halo;            // output radii per wave
    const Tile I = my_tile(g);
    const int n = I.n, lmax = I.lmax;
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
    const int j = I.r0 + wave * valid - halo + lane;    // this lane's radius
    const bool inside = j >= 0 && j < n;
    const int jc = min(max(j, 0), n - 1);               // clamped: every load is in bounds
    const bool writes = inside && lane >= halo && lane < 64 - halo;

    const double r = (double)(jc + 1) * I.dr;
    const double inv_r = 1.0 / r;
    const double inv_r2 = inv_r * inv_r;
    const double z_over_r = I.z * inv_r;
    const double er = step_value(step, g.n_inst, kEMid, I.inst) * r;
    const double dt = step_value(step, g.n_inst, kDt, I.inst);
    double coef[K];
#pragma unroll
    for (int k = 0; k < K; ++k) coef[k] = wave_uniform(dt / (double)(first_term - k));

    const C* in_i = in + I.off;
    const C* psi_i = psi + I.off;
    C* out_i = out + I.off;
    auto row_of = [&](int rr) -> int64_t { return (int64_t)min(max(rr, 0), lmax) * n + jc; };

    const int rho0 = I.l0 - K + 1;              // level-1 row at it = 0
    // input rows rho-1, rho, rho+1 of the current iteration (raw), prefetched rho+2
    C x_m = in_i[row_of(rho0 - 1)];
    C x_c = in_i[row_of(rho0)];
    C x_p = in_i[row_of(rho0 + 1)];
    // psi(rho_k) for level k = 1..K: pr[k-1]; pr[0] arrives one iteration ahead
    C pr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) pr[k] = zero_c<C>();
    pr[0] = psi_i[row_of(rho0)];
    // level k (1..K-1): a = row rho_k - 1, b = row rho_k - 2 (FP64)
    double2 ra[K > 1 ? K - 1 : 1], rb[K > 1 ? K - 1 : 1];
#pragma unroll
    for (int k = 0; k < (K > 1 ? K - 1 : 1); ++k) ra[k] = rb[k] = zero2();

    const int iters = (I.l1 - I.l0) + 2 * K - 2;
    for (int it = 0; it < iters; ++it) {
        const int rho = rho0 + it;
        // prefetch for the next iteration (clamped rows; zeroed at use)
        const C x_n = in_i[row_of(rho + 2)];
        const C p_n = psi_i[row_of(rho + 1)];

        // ---- level 1 from the input ----------------------------------------
        double2 up;   // the newest level value, passed to the next level as its row rho_k + 1
        {
            const bool ok_c = inside && rho >= 0 && rho <= lmax;
            const double2 c = pick2(ok_c, widen(x_c), zero2());
            const double2 lm = pick2(inside && rho - 1 >= 0 && rho - 1 <= lmax, widen(x_m), zero2());
            const double2 lp = pick2(inside && rho + 1 >= 0 && rho + 1 <= lmax, widen(x_p), zero2());
            const double2 m1 = lane_below(c, 1), p1 = lane_above(c, 1);
            double2 m2 = zero2(), p2 = zero2();
            if (S == 2) {
                m2 = lane_below(c, 2);
                p2 = lane_above(c, 2);
            }
            const int rk = min(max(rho, 0), lmax);
            const double2 h = h_point<S>(c, m1, p1, m2, p2, lm, lp, I.inv_dr2,
                                         row_potential(rk, inv_r2, z_over_r), er, g.kappa[rk],
                                         g.kappa[rk + 1]);
            const double2 v = horner_update(widen(pr[0]), h, coef[0]);
            up = pick2(ok_c, v, zero2());
        }
        if (K == 1) {
            if (writes && rho >= I.l0 && rho < I.l1) stc(out_i, (int64_t)rho * n + jc, up);
        }
        // ---- levels 2..K from the registers of the level below -------------
#pragma unroll
        for (int k = 2; k <= K; ++k) {
            const int rk_row = rho - (k - 1);
            double2 v = zero2();
            if (it >= 2 * (k - 1)) {
                const bool ok = inside && rk_row >= 0 && rk_row <= lmax;
                const double2 c = ra[k - 2];              // level k-1 at row rk_row
                const double2 lm = rb[k - 2];             // level k-1 at row rk_row - 1
                const double2 lp = up;                    // level k-1 at row rk_row + 1
                const double2 m1 = lane_below(c, 1), p1 = lane_above(c, 1);
                double2 m2 = zero2(), p2 = zero2();
                if (S == 2) {
                    m2 = lane_below(c, 2);
                    p2 = lane_above(c, 2);
                }
                const int rk = min(max(rk_row, 0), lmax);
                const double2 h = h_point<S>(c, m1, p1, m2, p2, lm, lp, I.inv_dr2,
                                             row_potential(rk, inv_r2, z_over_r), er, g.kappa[rk],
                                             g.kappa[rk + 1]);
                v = pick2(ok, horner_update(widen(pr[k - 1]), h, coef[k - 1]), zero2());
            }
            // the level below moves on by one row
            rb[k - 2] = ra[k - 2];
            ra[k - 2] = up;
            up = v;
            if (k == K && writes && rk_row >= I.l0 && rk_row < I.l1) stc(out_i, (int64_t)rk_row * n + jc, v);
        }
        // shift the window and the psi register
        x_m = x_c;
        x_c = x_p;
        x_p = x_n;
#pragma unroll
        for (int k = K - 1; k > 0; --k) pr[k] = pr[k - 1];
        pr[0] = p_n;
    }
}

template <int S, typename T, int K>
static hipError_t strip_t(const SweepGeom& g, const void* in, const void* psi, void* out,
                          const double* step, int first_term, hipStream_t st)
{
    using C = typename Cplx<T>::type;
    hipLaunchKernelGGL((k_horner_strip<S, T, K>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                       static_cast<const C*>(in), static_cast<const C*>(psi), static_cast<C*>(out),
                       step, first_term);
    return hipGetLastError();
}

template <int S, typename T>
static hipError_t strip_k(int K, const SweepGeom& g, const void* in, const void* psi, void* out,
                          const double* step, int first_term, hipStream_t st)
{
    switch (K) {
        case 1: return strip_t<S, T, 1>(g, in, psi, out, step, first_term, st);
        case 2: return strip_t<S, T, 2>(g, in, psi, out, step, first_term, st);
        case 3: return strip_t<S, T, 3>(g, in, psi, out, step, first_term, st);
        case 4: return strip_t<S, T, 4>(g, in, psi, out, step, first_term, st);
        case 5: return strip_t<S, T, 5>(g, in, psi, out, step, first_term, st);
        case 6: return strip_t<S, T, 6>(g, in, psi, out, step, first_term, st);
        case 7: return strip_t<S, T, 7>(g, in, psi, out, step, first_term, st);
        case 8: return strip_t<S, T, 8>(g, in, psi, out, step, first_term, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_horner_strip(int prec, int S, int K, const SweepGeom& g, const void* in,
                               const void* psi, void* out, const double* step, int first_term,
                               hipStream_t st)
{
    if (prec == 0) return S == 1 ? strip_k<1, double>(K, g, in, psi, out, step, first_term, st)
                                 : strip_k<2, double>(K, g, in, psi, out, step, first_term, st);
    return S == 1 ? strip_k<1, float>(K, g, in, psi, out, step, first_term, st)
                  : strip_k<2, float>(K, g, in, psi, out, step, first_term, st);
}

}  // namespace tdse
