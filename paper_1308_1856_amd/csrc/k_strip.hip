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
// written by exactly one strip.  The shuffles are DPP whole-wave shifts.  Along l, level k runs one row behind level k-1 within an iteration:
//   rho_k(it) = l0 - K + 2 - k + it,   it = 0 .. (l1 - l0) + 2K - 3,
// so level k at row rho needs level k-1 at rows rho-1 (two iterations ago),
// rho (one iteration ago) and rho+1 (this iteration): each level keeps its
// last two rows in registers, per thread.  Level k is skipped while
// it < 2(k-1) (rows no output depends on).  The input rows and psi are read
// once per iteration, one iteration ahead of use; psi(rho_1) is passed down a
// shift register to the later levels.
//
// Every element is computed by h_point and horner_update, the functions of
// the single-term sweeps, from the same FP64 operands, so FP64 results are
// bit-identical to K single-term launches; with FP32 storage the
// intermediate levels stay FP64.  Rows outside [0, lmax] and radii outside
// [0, N) are zero at every level, as in the single-term sweep.  HBM traffic
// per unknown and launch: read `in` and psi once (plus the row and radial
// overlaps), write out once.  `out` must not alias `in` or `psi`.
#include <type_traits>

#include "strip_common.hpp"

namespace tdse {

// The strip loop.  MASKED: some lanes of this wave lie outside [0, N) and
// their values are forced to zero at every level; waves wholly inside skip
// those selects.  Rows outside [0, lmax] cost no vector work: their input and
// psi values are read from the all-zero row (a wave-uniform pointer choice),
// and their l couplings are zero, so every level is exactly +0 there, as the
// single-term sweep's zero padding in l.  For the valid rows the coupling
// coefficients are the sweep's (kappa_{lmax+1} multiplies the zero row above
// lmax in the sweep; zero here gives the same bits).
constexpr int kStripDepth = 3;   // iterations of row loads in flight per wave (measured: 3 beats 2 and 4)
// the plain H.psi apply on aligned strips: six rows of loads in flight (on
// 4-row tiles of the 104M-unknown batch 541 us against 570 us with three)
constexpr int kApplyDepth = 6;

// The observables' partial sums of the rows a strip writes (OBS below): the
// wave's sums of norm, p_ion, dipole and acceleration terms go to
// partial[q * stride + unit] (q = 0..3); r is the lane's radius, outer: the
// radius lies beyond r_ion.
struct StripObs {
    double* partial = nullptr;
    int64_t stride = 0, unit = 0;
    double r = 0.0;
    bool outer = false;
    int lane = 0;
};

// Radii just outside an aligned strip (ALIGNED below): lanes 0..31 hold
// j0 - 1 (e1) and j0 - 2 (e2), lanes 32..63 j0 + 64 and j0 + 65, clamped into
// [0, N); in1 / in2: the unclamped radius lies in [0, N).
struct StripEdge {
    int e1 = 0, e2 = 0;
    bool in1 = false, in2 = false;
};

// APPLY (K = 1 only): out = H in, with no psi (the plain H-psi sweep).
// ALIGNED (K = 1 only): the wave writes all 64 of its radii; the radial
// neighbours beyond its ends are read per row as two (s = 2: four) extra
// values and enter the DPP shifts as the end lanes' values, so strips need
// not overlap, and each wave's loads and stores cover whole aligned lines.
// OBS (not with APPLY or ALIGNED): the strip also sums the observables of
// the level-K rows it writes (the stored values, so FP32 storage rounds
// first), as the observables pass does per element: |f|^2 (all radii and
// those beyond r_ion) and, for each pair of rows (l, l+1) at one radius,
// kappa_{l+1} Re(f_l* f_{l+1}) weighted by r and by 1/r^2.  The pair
// (l1 - 1, l1) needs row l1 of level K, which the next tile writes: one more
// iteration computes it (the same bits) without storing it.
template <int S, typename T, int K, bool MASKED, bool APPLY = false, bool ALIGNED = false, int D = kStripDepth,
          bool OBS = false>
__device__ __forceinline__ void strip_loop(const SweepGeom& g, const Tile& I, typename Stor<T>::cptr in_i,
                                           typename Stor<T>::cptr psi_i, typename Stor<T>::ptr out_i,
                                           int jc, bool inside, bool writes, double er, double inv_r2,
                                           double z_over_r, const double (&coef)[K], StripEdge edge = {},
                                           StripObs ob = {})
{
    static_assert(!OBS || !(APPLY || ALIGNED), "observables ride on the Horner strips");
    static_assert(!(APPLY || ALIGNED) || K == 1, "the plain sweep and the aligned strips have one level");
    using C = typename Cplx<T>::type;
    const int n = I.n, lmax = I.lmax;
    const auto zrow = zero_rowt<T>(g);
    using RowP = decltype(zrow + 0);
    auto rowp = [&](RowP base, int rr) -> RowP {
        return (rr >= 0 && rr <= lmax) ? base + (int64_t)rr * n : zrow;
    };
    auto widen_lane = [&](C raw) -> double2 {
        const double2 v = widen(raw);
        return MASKED ? pick2(inside, v, zero2()) : v;
    };
    // kappa_l for 1 <= l <= lmax, else 0 (the index is clamped so the load
    // itself is always in bounds)
    auto kap = [&](int l) -> double {
        const double v = ld_const(g.kappa, min(max(l, 0), lmax));  // a scalar load
        return (l >= 1 && l <= lmax) ? v : 0.0;
    };
    // the radius' part of the diagonal
    const double dbase = diag_base<S>(I.inv_dr2, z_over_r);
    // H at row rr of the level below: centre c, rows rr-1 / rr+1 at this
    // radius; the coupling to row rr-1 is kl = kappa_rr, to row rr+1
    // klp = kappa_{rr+1} (zero where the other row is outside [0, lmax])
    auto h_row = [&](double2 c, double2 lm, double2 lp, int rr, double kl, double klp) -> double2 {
        const double2 m1 = lane_below(c, 1), p1 = lane_above(c, 1);
        double2 m2 = zero2(), p2 = zero2();
        if (S == 2) {
            m2 = lane_below(c, 2);
            p2 = lane_above(c, 2);
        }
        return h_point<S>(c, m1, p1, m2, p2, lm, lp, I.inv_dr2, row_diag(half_ll(rr), inv_r2, dbase), er, kl, klp);
    };
    // the same with the centre row's values beyond the wave ends (c1: one
    // radius out, c2: two)
    auto h_row_edge = [&](double2 c, double2 c1, double2 c2, double2 lm, double2 lp, int rr, double kl,
                          double klp) -> double2 {
        const double2 m1 = dpp_shift2_edge<kDppWaveShr1>(c, c1), p1 = dpp_shift2_edge<kDppWaveShl1>(c, c1);
        double2 m2 = zero2(), p2 = zero2();
        if (S == 2) {
            m2 = dpp_shift2_edge<kDppWaveShr1>(m1, c2);
            p2 = dpp_shift2_edge<kDppWaveShl1>(p1, c2);
        }
        return h_point<S>(c, m1, p1, m2, p2, lm, lp, I.inv_dr2, row_diag(half_ll(rr), inv_r2, dbase), er, kl, klp);
    };
    auto widen_edge = [&](C raw, bool in) -> double2 {
        const double2 v = widen(raw);
        return MASKED ? pick2(in, v, zero2()) : v;
    };

    const int rho0 = I.l0 - K + 1;              // level-1 row at it = 0
    // A tile of the Horner strips from row 0 starts at iteration it0 = K - 1
    // (rounded down to a loop trip): before it every level works on rows
    // below 0, which are zero; the kept rows of the skipped iterations are
    // the zeros they start with.
    const int it0 = (!APPLY && !ALIGNED && I.l0 == 0) ? (K - 1) / D * D : 0;
    // input rows rho-1, rho (FP64) of the current iteration
    double2 xm = widen_lane(rowp(in_i, rho0 + it0 - 1)[jc]);
    double2 xc = widen_lane(rowp(in_i, rho0 + it0)[jc]);
    // ALIGNED: row rho's values beyond the wave ends
    double2 xc1 = zero2(), xc2 = zero2();
    if (ALIGNED) {
        xc1 = widen_edge(rowp(in_i, rho0)[edge.e1], edge.in1);
        if (S == 2) xc2 = widen_edge(rowp(in_i, rho0)[edge.e2], edge.in2);
    }
    // Rows are loaded D iterations ahead, into D register slots
    // that the iterations take in turn (iteration it uses slot it mod D): the
    // slot holds input row rho+1 and psi(rho) and is reloaded, in place, with
    // the rows of iteration it+D.  One iteration of loads in flight per wave
    // is too little to cover the memory latency (with 8-byte FP32 elements
    // above all).
    //
    // Iterations it = 0 .. iters-1 run (loop trips below).  Their last reads
    // the input row rho0 + iters and the psi row rho0 + iters - 1: the
    // prefetches of later rows, for iterations that never run, read the zero
    // row instead (no HBM traffic for rows the tile does not use).
    const int warm_trips_end = (2 * (K - 1) + D - 1) / D * D;
    const int iters = max((I.l1 - I.l0) + 2 * K - 2, warm_trips_end);
    const int xhi = min(lmax, rho0 + iters + (OBS ? 1 : 0));
    const int phi = min(lmax, rho0 + iters - 1 + (OBS ? 1 : 0));
    auto rowp_x = [&](int rr) -> RowP { return (unsigned)rr <= (unsigned)xhi ? in_i + (int64_t)rr * n : zrow; };
    auto rowp_p = [&](int rr) -> RowP { return (unsigned)rr <= (unsigned)phi ? psi_i + (int64_t)rr * n : zrow; };
    struct Slot {
        C x, p, x1, x2;   // x1, x2: row rho+1 beyond the wave ends (ALIGNED)
    };
    Slot sl[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
        const RowP xr = rowp_x(rho0 + it0 + 1 + u);
        sl[u] = Slot{xr[jc], APPLY ? zero_c<C>() : rowp_p(rho0 + it0 + u)[jc], ALIGNED ? xr[edge.e1] : zero_c<C>(),
                     ALIGNED && S == 2 ? xr[edge.e2] : zero_c<C>()};
    }
    // psi(rho_k) for level k = 1..K: pr[k-1]
    C pr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) pr[k] = zero_c<C>();
    // level k (1..K-1): a = row rho_k - 1, b = row rho_k - 2 (FP64)
    double2 ra[K > 1 ? K - 1 : 1], rb[K > 1 ? K - 1 : 1];
#pragma unroll
    for (int k = 0; k < (K > 1 ? K - 1 : 1); ++k) ra[k] = rb[k] = zero2();
    // kappa of rows rho + 1 - j, j = 0..K (wave-uniform, scalar registers):
    // the rows of an iteration's levels and their upper neighbours.  One new
    // value per iteration, loaded an iteration ahead (kn).
    double kq[K + 1];
#pragma unroll
    for (int j = 0; j <= K; ++j) kq[j] = kap(rho0 + it0 + 1 - j);
    double kn = kap(rho0 + it0 + 2);
    // element offsets of the rows an iteration reloads (input row rho+1+D,
    // psi row rho+D) and stores (level K at rho-(K-1)); each advances by one
    // row per iteration
    int64_t ox = (int64_t)(rho0 + it0 + 1 + D) * n, op = (int64_t)(rho0 + it0 + D) * n;
    int64_t os = (int64_t)(rho0 + it0 - (K - 1)) * n + jc;

    // OBS: sums per lane over the rows, and the previous level-K row as stored.
    // Level K is zero at the rows below l0 (not yet started), so the pair
    // (l0 - 1, l0) adds exactly zero; only rows from l1 on (the extra
    // iteration, a short tile's padding) need excluding, and only checked
    // iterations reach them.  p_ion: |f|^2 times 1 or 0 (exact).
    double oacc[kObsMainQ] = {0.0, 0.0, 0.0, 0.0};
    double2 fprev = zero2();
    const double outer1 = ob.outer ? 1.0 : 0.0;
    auto obs_row = [&](double2 v, int rk, auto check) {
        if (!OBS) return;
        constexpr bool CHECK = decltype(check)::value;
        const double2 vs = stored_value<T>(v);
        if (!CHECK || rk <= I.l1) {             // the pair (rk - 1, rk) is the tile's
            const double re = fma(fprev.x, vs.x, fprev.y * vs.y) * kq[K];
            oacc[2] = fma(ob.r, re, oacc[2]);
            oacc[3] = fma(re, inv_r2, oacc[3]);
        }
        if (!CHECK || rk < I.l1) {              // row rk is the tile's
            const double a2 = fma(vs.x, vs.x, vs.y * vs.y);
            oacc[0] += a2;
            oacc[1] = fma(outer1, a2, oacc[1]);
        }
        fprev = vs;
    };

    // Rows outside [0, lmax] of every level are zero (their psi rows and
    // couplings are), so the checked iterations skip them: at a member's
    // first and last rows the level pipeline's ramps would otherwise compute
    // K - k zero rows of level k at each end.
    auto live = [&](int rr) { return rr >= 0 && rr <= lmax; };
    // one iteration; CHECK: some levels may not have reached their first row
    // yet, or may work on rows outside [0, lmax]
    auto body = [&](int it, Slot& sl, auto check) {
        constexpr bool CHECK = decltype(check)::value;
        const int rho = rho0 + it;
        // move the slot's rows out, then reload the slot for iteration it+D
        const C xo = take(sl.x);
        const C po = APPLY ? zero_c<C>() : take(sl.p);
        const C xo1 = ALIGNED ? take(sl.x1) : zero_c<C>();
        const C xo2 = ALIGNED && S == 2 ? take(sl.x2) : zero_c<C>();
        const RowP xr = (unsigned)(rho + 1 + D) <= (unsigned)xhi ? in_i + ox : zrow;
        sl.x = xr[jc];
        if (!APPLY) sl.p = ((unsigned)(rho + D) <= (unsigned)phi ? psi_i + op : zrow)[jc];
        if (ALIGNED) sl.x1 = xr[edge.e1];
        if (ALIGNED && S == 2) sl.x2 = xr[edge.e2];
        ox += n;
        op += n;
        const double2 xp = widen_lane(xo);
        const double2 xp1 = ALIGNED ? widen_edge(xo1, edge.in1) : zero2();
        const double2 xp2 = ALIGNED && S == 2 ? widen_edge(xo2, edge.in2) : zero2();
#pragma unroll
        for (int k = K - 1; k > 0; --k) pr[k] = pr[k - 1];
        pr[0] = po;

        // level 1 from the input
        double2 up = zero2();
        if (!CHECK || live(rho)) {
            const double2 h1 = ALIGNED ? h_row_edge(xc, xc1, xc2, xm, xp, rho, kq[1], kq[0])
                                       : h_row(xc, xm, xp, rho, kq[1], kq[0]);
            up = APPLY ? h1 : horner_update(widen(pr[0]), h1, coef[0]);
            if (MASKED) up = pick2(inside, up, zero2());
        }
        // the stored row: in [l0, l1) at every iteration past the warm-up trips
        auto store_row = [&](int rr) { return !CHECK || (rr >= I.l0 && rr < I.l1); };
        if (K == 1 && writes && store_row(rho)) stc(out_i, os, up);
        if (K == 1) obs_row(up, rho, check);
        // levels 2..K from the registers of the level below
#pragma unroll
        for (int k = 2; k <= K; ++k) {
            const int rk = rho - (k - 1);
            double2 v = zero2();
            if (!CHECK || (it >= 2 * (k - 1) && live(rk))) {
                // level k-1 at rows rk (ra), rk - 1 (rb) and rk + 1 (this iteration)
                v = horner_update(widen(pr[k - 1]), h_row(ra[k - 2], rb[k - 2], up, rk, kq[k], kq[k - 1]), coef[k - 1]);
                if (MASKED) v = pick2(inside, v, zero2());
            }
            rb[k - 2] = ra[k - 2];
            ra[k - 2] = up;
            up = v;
            if (k == K && writes && store_row(rk)) stc(out_i, os, v);
            if (k == K) obs_row(v, rk, check);
        }
        // shift the window and the kappa register; fetch kappa for it + 2
#pragma unroll
        for (int j = K; j > 0; --j) kq[j] = kq[j - 1];
        kq[0] = kn;
        kn = kap(rho + 3);
        os += n;
        xm = xc;
        xc = xp;
        xc1 = xp1;
        xc2 = xp2;
        // keep the iterations of a loop trip apart: interleaving them would
        // hold several iterations' values in registers at once
        __builtin_amdgcn_sched_barrier(0);
    };
    // Loop trips of D iterations (iteration it + u takes slot u): first the
    // trips that hold the warm-up iterations it < 2(K-1) (levels still
    // starting; kept rolled, as the trip count is a constant and the
    // straight-line code of a full unroll would be scheduled into many more
    // live registers), then the steady trips, then checked trips once level
    // 1 passes lmax, then a tail of fewer than D iterations.  A tile too
    // short to reach the end of the warm-up trips runs on to it: the extra
    // iterations compute rows past l1 (inputs outside [0, lmax] read as zero)
    // and store nothing.
    int it = it0;
#pragma clang loop unroll(disable)
    for (; it < warm_trips_end; it += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) body(it + u, sl[u], std::true_type{});
    }
    // unchecked while every level's row lies in [0, lmax] (level 1 leads:
    // row rho0 + it), checked from there to the end
    const int steady_end = max(warm_trips_end, min(iters, lmax - rho0 + 1) / D * D);
    for (; it + D <= steady_end; it += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) body(it + u, sl[u], std::false_type{});
    }
#pragma clang loop unroll(disable)
    for (; it + D <= iters; it += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) body(it + u, sl[u], std::true_type{});
    }
#pragma unroll
    for (int u = 0; u < D - 1; ++u)
        if (it + u < iters) body(it + u, sl[u], std::true_type{});
    if (OBS) {
        // the iteration past the last (slot iters - it < D): level K at row
        // l1 for the last pair, checked so that it stores nothing
        Slot last = sl[0];
#pragma unroll
        for (int u = 1; u < D; ++u)
            if (it + u == iters) last = sl[u];
        body(iters, last, std::true_type{});
#pragma unroll
        for (int q = 0; q < kObsMainQ; ++q) {
            const double sq = wave_sum(writes ? oacc[q] : 0.0);
            if (ob.lane == 0) ob.partial[(int64_t)q * ob.stride + ob.unit] = sq;
        }
    }
}

template <int S, typename T, int K, bool OBS>
__global__ void __launch_bounds__(kBlock)
k_horner_strip(SweepGeom g, typename Stor<T>::cptr in, typename Stor<T>::cptr psi, typename Stor<T>::ptr out,
               const double* __restrict__ step, int first_term, double* __restrict__ obs_partial,
               const int* __restrict__ perm)
{
    const int halo = g.variant * S;             // >= K * S: lanes lost per side after K levels
    const int valid = 64 - 2 * halo;            // output radii per wave
    // the tile: perm gives the launch order, else g.order maps the block
    const int t = perm ? perm[blockIdx.x] : my_tile_index(g);
    const Tile I = g.tiles[t];
    const int n = I.n;
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
    const int j0 = I.r0 + wave * valid - halo;  // radius of lane 0
    const int j = j0 + lane;                    // this lane's radius
    const bool inside = j >= 0 && j < n;
    const int jc = min(max(j, 0), n - 1);       // clamped: every load is in bounds
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

    const auto in_i = in + I.off;
    const auto psi_i = psi + I.off;
    const auto out_i = out + I.off;
    StripObs ob;
    if (OBS) {
        ob.partial = obs_partial;
        ob.stride = (int64_t)g.n_tiles * kStripWaves;
        ob.unit = (int64_t)t * kStripWaves + wave;
        ob.r = r;
        ob.outer = jc >= I.i_ion;
        ob.lane = lane;
    }
    if (j0 >= 0 && j0 + 63 < n)   // wave-uniform
        strip_loop<S, T, K, false, false, false, kStripDepth, OBS>(g, I, in_i, psi_i, out_i, jc, inside, writes, er,
                                                                   inv_r2, z_over_r, coef, {}, ob);
    else
        strip_loop<S, T, K, true, false, false, kStripDepth, OBS>(g, I, in_i, psi_i, out_i, jc, inside, writes, er,
                                                                  inv_r2, z_over_r, coef, {}, ob);
}

template <int S, typename T, int K>
static hipError_t strip_t(const SweepGeom& g, const void* in, const void* psi, void* out,
                          const double* step, int first_term, double* obs_partial, const int* perm, hipStream_t st)
{
    if (obs_partial)
        hipLaunchKernelGGL((k_horner_strip<S, T, K, true>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(in, g.plane), Stor<T>::cmake(psi, g.plane), Stor<T>::make(out, g.plane),
                           step, first_term, obs_partial, perm);
    else
        hipLaunchKernelGGL((k_horner_strip<S, T, K, false>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(in, g.plane), Stor<T>::cmake(psi, g.plane), Stor<T>::make(out, g.plane),
                           step, first_term, obs_partial, perm);
    return hipGetLastError();
}

template <int S, typename T>
static hipError_t strip_k(int K, const SweepGeom& g, const void* in, const void* psi, void* out,
                          const double* step, int first_term, double* obs_partial, const int* perm,
                          hipStream_t st)
{
    switch (K) {
        case 1: return strip_t<S, T, 1>(g, in, psi, out, step, first_term, obs_partial, perm, st);
        case 2: return strip_t<S, T, 2>(g, in, psi, out, step, first_term, obs_partial, perm, st);
        case 3: return strip_t<S, T, 3>(g, in, psi, out, step, first_term, obs_partial, perm, st);
        case 4: return strip_t<S, T, 4>(g, in, psi, out, step, first_term, obs_partial, perm, st);
        case 5: return strip_t<S, T, 5>(g, in, psi, out, step, first_term, obs_partial, perm, st);
        case 6: return strip_t<S, T, 6>(g, in, psi, out, step, first_term, obs_partial, perm, st);
        case 7: return strip_t<S, T, 7>(g, in, psi, out, step, first_term, obs_partial, perm, st);
        case 8: return strip_t<S, T, 8>(g, in, psi, out, step, first_term, obs_partial, perm, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_horner_strip(int prec, int S, int K, const SweepGeom& g, const void* in,
                               const void* psi, void* out, const double* step, int first_term,
                               hipStream_t st, double* obs_partial, const int* perm)
{
    if (g.gauge != 0) return hipErrorInvalidValue;   // length gauge only
    if (prec == 0) return S == 1 ? strip_k<1, double>(K, g, in, psi, out, step, first_term, obs_partial, perm, st)
                                 : strip_k<2, double>(K, g, in, psi, out, step, first_term, obs_partial, perm, st);
    if (prec == 2) return S == 1 ? strip_k<1, s48>(K, g, in, psi, out, step, first_term, obs_partial, perm, st)
                                 : strip_k<2, s48>(K, g, in, psi, out, step, first_term, obs_partial, perm, st);
    return S == 1 ? strip_k<1, float>(K, g, in, psi, out, step, first_term, obs_partial, perm, st)
                  : strip_k<2, float>(K, g, in, psi, out, step, first_term, obs_partial, perm, st);
}

// The plain H-psi sweep (term 0: out = H(E_mid) in) and single Horner terms
// (term >= 1: out = psi + (-i dt / term) H(E_mid) in) on aligned wave strips
// of one level: a tile is 4 waves of 64 consecutive radii from a multiple of
// 256, each wave writing all of its radii (the radial neighbours beyond its
// ends come from two (s = 2: four) extra values per row).  The elements are
// those of the workgroup sweeps of k_sweep.hip, bit for bit.
template <int S, typename T, bool APPLY>
__global__ void __launch_bounds__(kBlock)
k_sweep_strip(SweepGeom g, typename Stor<T>::cptr in, typename Stor<T>::cptr psi, typename Stor<T>::ptr out,
              const double* __restrict__ step, int term)
{
    const Tile I = my_tile(g);
    const int n = I.n;
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
    const int j0 = I.r0 + wave * 64;            // radius of lane 0
    if (j0 >= n) return;                        // wave-uniform; no LDS, no barrier
    const int j = j0 + lane;
    const bool inside = j < n;
    const int jc = min(j, n - 1);
    StripEdge edge;
    {
        const int e1 = lane < 32 ? j0 - 1 : j0 + 64;
        const int e2 = lane < 32 ? j0 - 2 : j0 + 65;
        edge.in1 = e1 >= 0 && e1 < n;
        edge.in2 = e2 >= 0 && e2 < n;
        edge.e1 = min(max(e1, 0), n - 1);
        edge.e2 = min(max(e2, 0), n - 1);
    }
    const double r = (double)(jc + 1) * I.dr;
    const double inv_r = 1.0 / r;
    const double inv_r2 = inv_r * inv_r;
    const double z_over_r = I.z * inv_r;
    const double er = step_value(step, g.n_inst, kEMid, I.inst) * r;
    const double coef[1] = {APPLY ? 0.0 : wave_uniform(step_value(step, g.n_inst, kDt, I.inst) / (double)term)};
    const auto in_i = in + I.off;
    const auto psi_i = psi + I.off;
    const auto out_i = out + I.off;
    if (j0 - S >= 0 && j0 + 63 + S < n)   // wave-uniform: every value the wave reads is inside
        strip_loop<S, T, 1, false, APPLY, true, APPLY ? kApplyDepth : kStripDepth>(
            g, I, in_i, psi_i, out_i, jc, inside, inside, er, inv_r2, z_over_r, coef, edge);
    else
        strip_loop<S, T, 1, true, APPLY, true, APPLY ? kApplyDepth : kStripDepth>(
            g, I, in_i, psi_i, out_i, jc, inside, inside, er, inv_r2, z_over_r, coef, edge);
}

template <int S, typename T>
static hipError_t sweep_strip_t(const SweepGeom& g, const void* in, const void* psi, void* out, const double* step,
                                int term, hipStream_t st)
{
    if (term == 0)
        hipLaunchKernelGGL((k_sweep_strip<S, T, true>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(in, g.plane), Stor<T>::cmake(in, g.plane), Stor<T>::make(out, g.plane), step,
                           term);
    else
        hipLaunchKernelGGL((k_sweep_strip<S, T, false>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(in, g.plane), Stor<T>::cmake(psi, g.plane), Stor<T>::make(out, g.plane), step,
                           term);
    return hipGetLastError();
}

hipError_t launch_strip_sweep(int prec, int S, const SweepGeom& g, const void* in, const void* psi, void* out,
                              const double* step, int term, hipStream_t st)
{
    if (g.gauge != 0) return hipErrorInvalidValue;   // length gauge only
    if (g.variant != 1 || term < 0) return hipErrorInvalidValue;   // aligned tiles of one level
    if (prec == 0) return S == 1 ? sweep_strip_t<1, double>(g, in, psi, out, step, term, st)
                                 : sweep_strip_t<2, double>(g, in, psi, out, step, term, st);
    if (prec == 2) return S == 1 ? sweep_strip_t<1, s48>(g, in, psi, out, step, term, st)
                                 : sweep_strip_t<2, s48>(g, in, psi, out, step, term, st);
    return S == 1 ? sweep_strip_t<1, float>(g, in, psi, out, step, term, st)
                  : sweep_strip_t<2, float>(g, in, psi, out, step, term, st);
}

// One classic RK4 step (eq. RKDeriv) per launch on the wave strips, the four
// stages being the levels of the strip (each one row behind the last):
//   stage s at row r_s = rho - s:  k_s = -i H(t_s) g_s  (g_0 = psi),
//     g_{s+1} = psi + a_s dt k_s                (a = 1/2, 1/2, 1),
//     acc_0 = psi + dt/6 k_0,  acc_s = acc_{s-1} + dt/3 k_s  (s = 1, 2),
//     psi' = acc_2 + dt/6 k_3,
// with t_0 = t_n, t_1 = t_2 = t_n + dt/2, t_3 = t_n + dt.  Stage s reads g_s
// at rows r_s - 1, r_s, r_s + 1 (two from its registers, one just computed by
// stage s-1) and radial neighbours by DPP shifts; the acc of a row passes from
// stage s to stage s+1 in a register (stage s+1 reaches the row one iteration
// later).  psi is the input and the base of every stage: read once per row,
// rows rho-3 .. rho+1 kept in registers.  Every element is computed by
// h_point and horner_update from the same FP64 operands as the four stage
// launches (k_rk4_stage), so FP64 results are bit-identical to them; with
// FP32 storage g and acc stay FP64 between stages.  HBM traffic per unknown
// and step: read psi, write psi' (2c, against 16c for the stage launches).
template <int S, typename T, bool MASKED>
__device__ __forceinline__ void rk4_strip_loop(const SweepGeom& g, const Tile& I, typename Stor<T>::cptr in_i,
                                               typename Stor<T>::ptr out_i, int jc, bool inside, bool writes,
                                               const double (&er)[4], double inv_r2, double z_over_r, double dt)
{
    using C = typename Cplx<T>::type;
    constexpr int K = 4;
    const int n = I.n, lmax = I.lmax;
    const auto zrow = zero_rowt<T>(g);
    using RowP = decltype(zrow + 0);
    auto rowp = [&](RowP base, int rr) -> RowP {
        return (rr >= 0 && rr <= lmax) ? base + (int64_t)rr * n : zrow;
    };
    auto widen_lane = [&](C raw) -> double2 {
        const double2 v = widen(raw);
        return MASKED ? pick2(inside, v, zero2()) : v;
    };
    auto kap = [&](int l) -> double {
        const double v = ld_const(g.kappa, min(max(l, 0), lmax));  // a scalar load
        return (l >= 1 && l <= lmax) ? v : 0.0;
    };
    // the radius' part of the diagonal
    const double dbase = diag_base<S>(I.inv_dr2, z_over_r);
    auto h_row = [&](double2 c, double2 lm, double2 lp, int rr, double kl, double klp, double e_r) -> double2 {
        const double2 m1 = lane_below(c, 1), p1 = lane_above(c, 1);
        double2 m2 = zero2(), p2 = zero2();
        if (S == 2) {
            m2 = lane_below(c, 2);
            p2 = lane_above(c, 2);
        }
        return h_point<S>(c, m1, p1, m2, p2, lm, lp, I.inv_dr2, row_diag(half_ll(rr), inv_r2, dbase), e_r, kl, klp);
    };
    // the stage weights, as the stage launches form them
    const double b06 = dt / 6.0, b13 = dt / 3.0, a_half = 0.5 * dt;

    const int rho0 = I.l0 - K + 1;              // stage-0 row at it = 0
    // psi rows rho-3 .. rho (FP64)
    double2 x3 = widen_lane(rowp(in_i, rho0 - 3)[jc]);
    double2 x2 = widen_lane(rowp(in_i, rho0 - 2)[jc]);
    double2 xm = widen_lane(rowp(in_i, rho0 - 1)[jc]);
    double2 xc = widen_lane(rowp(in_i, rho0)[jc]);
    // psi row rho+1, loaded D iterations ahead into D slots (as in strip_loop,
    // with rows past the last one the tile's iterations read taken from the
    // zero row)
    constexpr int D = kStripDepth;
    const int warm_trips_end = (2 * (K - 1) + D - 1) / D * D;
    const int iters = max((I.l1 - I.l0) + 2 * K - 2, warm_trips_end);
    const int xhi = min(lmax, rho0 + iters);
    C sl[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
        const int rr = rho0 + 1 + u;
        sl[u] = ((unsigned)rr <= (unsigned)xhi ? in_i + (int64_t)rr * n : zrow)[jc];
    }
    // g_{s} (s = 1..3) at rows r_s (ra) and r_s - 1 (rb); acc of stage s-1
    // for the row stage s takes (acc_in[s-1])
    double2 ra[3], rb[3], acc_in[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) ra[s] = rb[s] = acc_in[s] = zero2();
    double kq[K + 1];
#pragma unroll
    for (int j = 0; j <= K; ++j) kq[j] = kap(rho0 + 1 - j);
    double kn = kap(rho0 + 2);
    int64_t ox = (int64_t)(rho0 + 1 + D) * n;
    int64_t os = (int64_t)(rho0 - (K - 1)) * n + jc;

    auto body = [&](int it, C& slot, auto check) {
        constexpr bool CHECK = decltype(check)::value;
        const int rho = rho0 + it;
        const C xo = take(slot);
        slot = ((unsigned)(rho + 1 + D) <= (unsigned)xhi ? in_i + ox : zrow)[jc];
        ox += n;
        const double2 xp = widen_lane(xo);

        // stage 0 at row rho, from psi
        const double2 h0 = h_row(xc, xm, xp, rho, kq[1], kq[0], er[0]);
        double2 acc_new[3];
        acc_new[0] = horner_update(xc, h0, b06);
        double2 up = horner_update(xc, h0, a_half);     // g_1 at row rho
        if (MASKED) up = pick2(inside, up, zero2());
        // stages 1..3 at rows rho - s
        const double2 psi_s[3] = {xm, x2, x3};
#pragma unroll
        for (int st = 1; st <= 3; ++st) {
            const int rs = rho - st;
            double2 v = zero2();
            if (!CHECK || it >= 2 * st) {
                const double2 hs = h_row(ra[st - 1], rb[st - 1], up, rs, kq[st + 1], kq[st], er[st]);
                if (st < 3) {
                    acc_new[st] = horner_update(acc_in[st - 1], hs, b13);
                    v = horner_update(psi_s[st - 1], hs, st == 2 ? dt : a_half);
                    if (MASKED) v = pick2(inside, v, zero2());
                } else if (writes && (!CHECK || (rs >= I.l0 && rs < I.l1))) {
                    stc(out_i, os, horner_update(acc_in[2], hs, b06));
                }
            } else if (st < 3) {
                acc_new[st] = zero2();
            }
            rb[st - 1] = ra[st - 1];
            ra[st - 1] = up;
            up = v;
        }
#pragma unroll
        for (int st = 0; st < 3; ++st) acc_in[st] = acc_new[st];
#pragma unroll
        for (int j = K; j > 0; --j) kq[j] = kq[j - 1];
        kq[0] = kn;
        kn = kap(rho + 3);
        os += n;
        x3 = x2;
        x2 = xm;
        xm = xc;
        xc = xp;
        __builtin_amdgcn_sched_barrier(0);
    };
    int it = 0;
#pragma clang loop unroll(disable)
    for (; it < warm_trips_end; it += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) body(it + u, sl[u], std::true_type{});
    }
    for (; it + D <= iters; it += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) body(it + u, sl[u], std::false_type{});
    }
#pragma unroll
    for (int u = 0; u < D - 1; ++u)
        if (it + u < iters) body(it + u, sl[u], std::false_type{});
}

template <int S, typename T>
__global__ void __launch_bounds__(kBlock)
k_rk4_strip(SweepGeom g, typename Stor<T>::cptr in, typename Stor<T>::ptr out, const double* __restrict__ step)
{
    const int halo = g.variant * S;             // = 4 S: lanes lost per side after the four stages
    const int valid = 64 - 2 * halo;
    const Tile I = my_tile(g);
    const int n = I.n;
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
    const int j0 = I.r0 + wave * valid - halo;
    const int j = j0 + lane;
    const bool inside = j >= 0 && j < n;
    const int jc = min(max(j, 0), n - 1);
    const bool writes = inside && lane >= halo && lane < 64 - halo;

    const double r = (double)(jc + 1) * I.dr;
    const double inv_r = 1.0 / r;
    const double inv_r2 = inv_r * inv_r;
    const double z_over_r = I.z * inv_r;
    const double e_mid = step_value(step, g.n_inst, kEMid, I.inst) * r;
    const double er[4] = {step_value(step, g.n_inst, kEStart, I.inst) * r, e_mid, e_mid,
                          step_value(step, g.n_inst, kEEnd, I.inst) * r};
    const double dt = step_value(step, g.n_inst, kDt, I.inst);

    const auto in_i = in + I.off;
    const auto out_i = out + I.off;
    if (j0 >= 0 && j0 + 63 < n)   // wave-uniform
        rk4_strip_loop<S, T, false>(g, I, in_i, out_i, jc, inside, writes, er, inv_r2, z_over_r, dt);
    else
        rk4_strip_loop<S, T, true>(g, I, in_i, out_i, jc, inside, writes, er, inv_r2, z_over_r, dt);
}

template <int S, typename T>
static hipError_t rk4_strip_t(const SweepGeom& g, const void* in, void* out, const double* step, hipStream_t st)
{
    hipLaunchKernelGGL((k_rk4_strip<S, T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::cmake(in, g.plane),
                       Stor<T>::make(out, g.plane), step);
    return hipGetLastError();
}

hipError_t launch_rk4_strip(int prec, int S, const SweepGeom& g, const void* in, void* out, const double* step,
                            hipStream_t st)
{
    if (g.gauge != 0) return hipErrorInvalidValue;   // length gauge only
    if (g.variant != 4) return hipErrorInvalidValue;   // tiles built for the four stages
    if (prec == 0) return S == 1 ? rk4_strip_t<1, double>(g, in, out, step, st) : rk4_strip_t<2, double>(g, in, out, step, st);
    if (prec == 2) return S == 1 ? rk4_strip_t<1, s48>(g, in, out, step, st) : rk4_strip_t<2, s48>(g, in, out, step, st);
    return S == 1 ? rk4_strip_t<1, float>(g, in, out, step, st) : rk4_strip_t<2, float>(g, in, out, step, st);
}

}  // namespace tdse
