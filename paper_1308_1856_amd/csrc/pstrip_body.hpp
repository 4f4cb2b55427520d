// K consecutive Horner terms of the Taylor step (Sec. 5.2, eq. Taylor) in one
// launch on wave strips of two radii per lane ("pair strips"), the levels
// split between two waves:
//
//   v_0 = in,  v_k = psi + (-i dt / t_k) H v_{k-1}   (k = 1..K, t_k = first_term - k + 1)
//   out = v_K
//
// The wave-strip kernel of k_strip.hip holds one radius per lane, so each
// level shifts the centre values by one lane both ways (and twice more for
// the 5-point stencil): eight (sixteen) 32-bit DPP moves per FP64 complex
// element and level, about a third of the VALU work of a level, and a strip
// of 64 radii keeps only 64 - 2 K s of them exact after K levels.  Here lane
// L holds the adjacent radii a = j0 + 2L and b = a + 1: the inner neighbours
// of the pair are in the lane itself, only b of the lane below and a of the
// lane above cross lanes (5-point: also a of the lane below and b of the
// lane above), half the moves per element; and a strip of 128 radii keeps
// 128 - 2 K s of them exact.
//
// Twice the radii per lane would need twice the level registers (each level
// keeps its last two rows), more than a wave has.  So each strip is worked
// by two waves of the workgroup: the producer computes levels 1..K1 (K1 =
// ceil(K/2)) from the input, the consumer levels K1+1..K, one row-iteration
// behind, from the level-K1 row the producer hands over through LDS.  The psi
// rows the levels add pass through a ring of K+1 rows in LDS written by the
// producer (which loads psi once).  One workgroup barrier per row-iteration
// orders the hand-over (double-buffered) and the ring; every wave of the
// workgroup runs the same number of iterations.
//
// Rows march along l as in the one-radius kernel: at producer iteration it
// (rho = l0 - K + 1 + it) level k works on row rho - (k-1) from the rows
// rho - k, rho - k + 1 (kept) and rho - k + 2 (just computed by level k-1);
// the consumer at its iteration it plays producer iteration it - 1.
//
// Every element is computed by h_point and horner_update from the same FP64
// operands as the other sweeps, so FP64 results are bit-identical to K
// single-term launches.  HBM traffic per unknown and launch: read `in` and
// psi once (plus the row and radial overlaps), write out once.  `out` must
// not alias `in` or `psi`.
#pragma once
#include <algorithm>
#include <utility>

#include "strip_common.hpp"

namespace tdse {

template <typename T> struct type_tag { using type = T; };

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>), in order.
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// A lane's two radii.
struct Pair {
    double2 a, b;
};
__device__ __forceinline__ Pair zero_pair() { return Pair{zero2(), zero2()}; }

// H at one row of the level below on both radii of each lane: c at that row,
// lm / lp at the rows below and above (same radii); d0a / d0b the diagonal.
template <int S>
__device__ __forceinline__ Pair h_pair(const Pair& c, const Pair& lm, const Pair& lp, double inv_dr2, double d0a,
                                       double d0b, double era, double erb, double kl, double klp)
{
    const double2 b_below = dpp_shift2<kDppWaveShr1>(c.b);   // radius a - 1
    const double2 a_above = dpp_shift2<kDppWaveShl1>(c.a);   // radius b + 1
    double2 a_below = zero2(), b_above = zero2();
    if (S == 2) {
        a_below = dpp_shift2<kDppWaveShr1>(c.a);             // radius a - 2
        b_above = dpp_shift2<kDppWaveShl1>(c.b);             // radius b + 2
    }
    Pair h;
    h.a = h_point<S>(c.a, b_below, c.b, a_below, a_above, lm.a, lp.a, inv_dr2, d0a, era, kl, klp);
    h.b = h_point<S>(c.b, c.a, a_above, b_below, b_above, lm.b, lp.b, inv_dr2, d0b, erb, kl, klp);
    return h;
}

// Per-lane constants of the two radii.
struct PairLane {
    int jca = 0, jcb = 0;          // radii clamped into [0, N) (every load in bounds)
    bool ina = false, inb = false; // the radius lies in [0, N)
    bool wa = false, wb = false;   // the lane writes the radius
    double inv_r2a = 0.0, inv_r2b = 0.0, dba = 0.0, dbb = 0.0, era = 0.0, erb = 0.0;
    double ra = 0.0, rb = 0.0;     // radii (observables)
    bool outa = false, outb = false;
};

// The LDS of one strip: the psi ring (K + 1 rows of 128 radii in storage
// type; per row the a values of the 64 lanes, then the b values: 16-byte
// strides for FP64) and the double-buffered hand-over row (FP64, same order).
template <typename C, int K>
struct StripLds {
    C ring[(K + 1) * 128];
    double2 hand[2 * 128];
};

template <int S, typename T, int K, bool MASKED, int D, bool OBS, bool PRODUCER>
__device__ __forceinline__ void pair_loop(const SweepGeom& g, const Tile& I, typename Stor<T>::cptr in_i,
                                          typename Stor<T>::cptr psi_i, typename Stor<T>::ptr out_i,
                                          const PairLane& P, const double (&coef)[K],
                                          StripLds<typename Cplx<T>::type, K>& L, int lane, double* obs_partial,
                                          int64_t obs_stride, int64_t obs_unit)
{
    using C = typename Cplx<T>::type;
    constexpr int K1 = (K + 1) / 2;                        // producer levels 1..K1
    constexpr int KLO = PRODUCER ? 1 : K1 + 1;             // this wave's levels KLO..KHI
    constexpr int KHI = PRODUCER ? K1 : K;
    constexpr bool WRITES = PRODUCER ? (K1 == K) : (K > K1);   // this wave computes level K
    constexpr int NR = (KHI - KLO + 1) > 0 ? (KHI - KLO + 1) : 1;
    constexpr int R = K + 1;                                // psi ring rows
    constexpr int LAG = PRODUCER ? 0 : 1;                  // the consumer plays producer iteration it - 1
    const int n = I.n, lmax = I.lmax;
    const auto zrow = zero_rowt<T>(g);
    using RowP = decltype(zrow + 0);
    auto wa2 = [&](C raw) -> double2 {
        const double2 v = widen(raw);
        return MASKED ? pick2(P.ina, v, zero2()) : v;
    };
    auto wb2 = [&](C raw) -> double2 {
        const double2 v = widen(raw);
        return MASKED ? pick2(P.inb, v, zero2()) : v;
    };
    auto mask = [&](Pair v) -> Pair {
        if (MASKED) {
            v.a = pick2(P.ina, v.a, zero2());
            v.b = pick2(P.inb, v.b, zero2());
        }
        return v;
    };
    auto kap = [&](int l) -> double {
        const double v = ld_const(g.kappa, min(max(l, 0), lmax));  // a scalar load
        return (l >= 1 && l <= lmax) ? v : 0.0;
    };
    auto h_row = [&](const Pair& c, const Pair& lm, const Pair& lp, int rr, double kl, double klp) -> Pair {
        const double cl = half_ll(rr);
        return h_pair<S>(c, lm, lp, I.inv_dr2, row_diag(cl, P.inv_r2a, P.dba), row_diag(cl, P.inv_r2b, P.dbb), P.era,
                         P.erb, kl, klp);
    };
    auto horner = [&](const Pair& p, const Pair& h, double c) -> Pair {
        return Pair{horner_update(p.a, h.a, c), horner_update(p.b, h.b, c)};
    };
    auto ring_a = [&](int slot) -> C& { return L.ring[(slot * 2) * 64 + lane]; };
    auto ring_b = [&](int slot) -> C& { return L.ring[(slot * 2 + 1) * 64 + lane]; };

    const int rho0 = I.l0 - K + 1;
    // iterations: level K reaches row l1 - 1 at it = (l1 - l0) + 2K - 3, one
    // later on the consumer (none for K = 1: the producer computes it); the
    // warm-up iterations (levels not all started) come first, D at a time
    constexpr int KLAG = (K > K1) ? 1 : 0;
    const int warm_trips_end = (2 * K - 2 + KLAG + D - 1) / D * D;
    const int iters = max((I.l1 - I.l0) + 2 * K - 2 + KLAG, warm_trips_end);
    const int xhi = min(lmax, rho0 + iters + (OBS ? 1 : 0));
    const int phi = min(lmax, rho0 + iters - 1 + (OBS ? 1 : 0));
    // A tile from row 0 starts at iteration it0 = K - 1 (rounded down to a
    // loop trip): before it every level works on rows below 0, which are
    // zero, so the iterations would only load zero rows and meet at the
    // barrier.  Both waves skip the same count (their barriers stay paired);
    // the kept rows of the skipped iterations are the zeros they start with.
    const int it0 = (I.l0 == 0) ? (K - 1) / D * D : 0;
    auto rowp_x = [&](int rr) -> RowP { return (unsigned)rr <= (unsigned)xhi ? in_i + (int64_t)rr * n : zrow; };
    auto rowp_p = [&](int rr) -> RowP { return (unsigned)rr <= (unsigned)phi ? psi_i + (int64_t)rr * n : zrow; };

    // producer: input rows rho - 1, rho and the prefetch slots (input row
    // rho + 1, psi row rho; iteration it takes slot it mod D)
    struct Slot {
        C xa, xb, pa, pb;
    };
    Slot sl[D];
    // Rows kept from one iteration to the next swap roles with the
    // iteration's parity instead of being copied: at parity p the centre row
    // of level 1 is xw[p] and the row below it xw[1 - p], which the new input
    // row then replaces (the next iteration's centre); likewise lv[p][j] and
    // lv[1 - p][j] for level j's rows of the level below.  D is even, so every
    // loop trip starts at parity 0.
    static_assert(D % 2 == 0, "the row roles alternate over loop trips of D iterations");
    Pair xw[2] = {zero_pair(), zero_pair()};
    int64_t ox = 0, op = 0;
    if (PRODUCER) {
        xw[1] = Pair{wa2(rowp_x(rho0 + it0 - 1)[P.jca]), wb2(rowp_x(rho0 + it0 - 1)[P.jcb])};
        xw[0] = Pair{wa2(rowp_x(rho0 + it0)[P.jca]), wb2(rowp_x(rho0 + it0)[P.jcb])};
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const RowP xr = rowp_x(rho0 + it0 + 1 + u);
            const RowP pr = rowp_p(rho0 + it0 + u);
            sl[u] = Slot{xr[P.jca], xr[P.jcb], pr[P.jca], pr[P.jcb]};
        }
        ox = (int64_t)(rho0 + it0 + 1 + D) * n;
        op = (int64_t)(rho0 + it0 + D) * n;
    }
    // for each of this wave's levels, the two older rows of the level below
    // (the centre row r and the row r - 1 of the level's row r); the
    // producer's level 1 uses the input rows instead
    Pair lv[2][NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) lv[0][j] = lv[1][j] = zero_pair();
    // kappa window: kq[j] = kappa(rho + 1 - j), j = 0..K, rho of the
    // producer iteration played
    double kq[K + 1];
#pragma unroll
    for (int j = 0; j <= K; ++j) kq[j] = kap(rho0 + it0 - LAG + 1 - j);
    double kn = kap(rho0 + it0 - LAG + 2);
    int64_t os = (int64_t)(rho0 + it0 - LAG - (K - 1)) * n;   // the level-K row's offset

    double oacc[kObsMainQ] = {0.0, 0.0, 0.0, 0.0};
    Pair fprev = zero_pair();
    const double fa = P.wa ? 1.0 : 0.0, fb = P.wb ? 1.0 : 0.0;
    const double oa = P.outa ? fa : 0.0, ob = P.outb ? fb : 0.0;
    auto obs_row = [&](const Pair& v, int rk, auto check) {
        if (!OBS || !WRITES) return;
        constexpr bool CHECK = decltype(check)::value;
        const double2 va = stored_value<T>(v.a), vb = stored_value<T>(v.b);
        if (!CHECK || rk <= I.l1) {             // the pair (rk - 1, rk) is the tile's
            const double rea = fa * fma(fprev.a.x, va.x, fprev.a.y * va.y) * kq[K];
            const double reb = fb * fma(fprev.b.x, vb.x, fprev.b.y * vb.y) * kq[K];
            oacc[2] = fma(P.rb, reb, fma(P.ra, rea, oacc[2]));
            oacc[3] = fma(reb, P.inv_r2b, fma(rea, P.inv_r2a, oacc[3]));
        }
        if (!CHECK || rk < I.l1) {              // row rk is the tile's
            const double a2 = fma(va.x, va.x, va.y * va.y), b2 = fma(vb.x, vb.x, vb.y * vb.y);
            oacc[0] = fma(fb, b2, fma(fa, a2, oacc[0]));
            oacc[1] = fma(ob, b2, fma(oa, a2, oacc[1]));
        }
        fprev = Pair{va, vb};
    };

    // Rows outside [0, lmax] of every level are zero (their psi rows and
    // couplings are), so the checked iterations skip them: at a member's
    // first and last rows the level pipeline's ramps would otherwise compute
    // K - k zero rows of level k at each end.
    auto live = [&](int rr) { return rr >= 0 && rr <= lmax; };

    // The stores are plain (cached) ones: a lane writes the two radii of its
    // 32-byte pair in two instructions, and the L2 joins the halves of each
    // line before writing it back; streaming stores wrote the halves out one
    // by one (a third more HBM writes).
    //
    // one iteration (it: this wave's count; CHECK: some levels may not have
    // reached their first row or may work on rows outside [0, lmax], and rows
    // past the tile are not stored)
    auto body = [&](int it, Slot& s, auto check, auto parity) {
        constexpr bool CHECK = decltype(check)::value;
        constexpr int PAR = decltype(parity)::value;   // it mod 2
        const int pit = it - LAG;                // the producer iteration this one plays
        const int rho = rho0 + pit;
        auto store_row = [&](int rr) { return !CHECK || (rr >= I.l0 && rr < I.l1); };
        Pair up;
        if (PRODUCER) {
            const C xoa = take(s.xa), xob = take(s.xb), poa = take(s.pa), pob = take(s.pb);
            const RowP xr = (unsigned)(rho + 1 + D) <= (unsigned)xhi ? in_i + ox : zrow;
            const RowP pr = (unsigned)(rho + D) <= (unsigned)phi ? psi_i + op : zrow;
            s.xa = xr[P.jca];
            s.xb = xr[P.jcb];
            s.pa = pr[P.jca];
            s.pb = pr[P.jcb];
            ox += n;
            op += n;
            const Pair xp{wa2(xoa), wb2(xob)};
            // psi(rho) into the ring for the levels below
            const int wslot = it % R;
            ring_a(wslot) = poa;
            ring_b(wslot) = pob;
            up = zero_pair();
            if (!CHECK || live(rho))
                up = mask(horner(Pair{widen(poa), widen(pob)}, h_row(xw[PAR], xw[1 - PAR], xp, rho, kq[1], kq[0]),
                                 coef[0]));
            xw[1 - PAR] = xp;
            if (WRITES && KHI == 1) {
                if (store_row(rho)) {
                    if (P.wa) stc_keep(out_i, os + P.jca, up.a);
                    if (P.wb) stc_keep(out_i, os + P.jcb, up.b);
                }
                obs_row(up, rho, check);
            }
        } else {
            // the producer's level-K1 row of the iteration before (row rho -
            // (K1 - 1)); none before the first iteration (a row below 0)
            const int hs = (it + 1) & 1;
            if (CHECK && it == it0)
                up = zero_pair();
            else
                up = Pair{L.hand[hs * 128 + lane], L.hand[hs * 128 + 64 + lane]};
        }
#pragma unroll
        for (int k = KLO + (PRODUCER ? 1 : 0); k <= KHI; ++k) {
            const int j = k - KLO;               // register index of level k
            const int rk = rho - (k - 1);
            Pair v = zero_pair();
            if (!CHECK || (pit >= 2 * (k - 1) && live(rk))) {
                // psi(rk), written by the producer at its iteration pit - (k - 1)
                const int rslot = (pit - (k - 1) + 2 * R) % R;
                const Pair pk{widen(ring_a(rslot)), widen(ring_b(rslot))};
                v = mask(horner(pk, h_row(lv[PAR][j], lv[1 - PAR][j], up, rk, kq[k], kq[k - 1]), coef[k - 1]));
            }
            lv[1 - PAR][j] = up;
            up = v;
            if (k == K && store_row(rk)) {
                if (P.wa) stc_keep(out_i, os + P.jca, v.a);
                if (P.wb) stc_keep(out_i, os + P.jcb, v.b);
            }
            if (k == K) obs_row(v, rk, check);
        }
        if (PRODUCER && !WRITES) {
            // hand the level-K1 row to the consumer
            const int hs = it & 1;
            L.hand[hs * 128 + lane] = up.a;
            L.hand[hs * 128 + 64 + lane] = up.b;
        }
#pragma unroll
        for (int jj = K; jj > 0; --jj) kq[jj] = kq[jj - 1];
        kq[0] = kn;
        kn = kap(rho + 3);
        os += n;
        // the hand-over and the ring of this iteration are complete before
        // either wave of the strip goes on
        __syncthreads();
    };
    // D iterations from ib (a multiple of D), slot u and parity u mod 2 each
    auto trip = [&](int ib, auto check) {
        static_for<D>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            body(ib + u, sl[u], check, std::integral_constant<int, u % 2>{});
        });
    };
    int it = it0;
#pragma clang loop unroll(disable)
    for (; it < warm_trips_end; it += D) trip(it, std::true_type{});
    // unchecked while every level's row lies in [0, lmax] (level 1 leads:
    // row rho0 + it - LAG), checked from there to the end
    const int steady_end = max(warm_trips_end, min(iters, lmax - rho0 + 1 + LAG) / D * D);
#pragma clang loop unroll(disable)
    for (; it + D <= steady_end; it += D) trip(it, std::false_type{});
#pragma clang loop unroll(disable)
    for (; it + D <= iters; it += D) trip(it, std::true_type{});
    static_for<D - 1>([&](auto uc) {
        constexpr int u = decltype(uc)::value;
        if (it + u < iters) body(it + u, sl[u], std::true_type{}, std::integral_constant<int, u % 2>{});
    });
    if (OBS) {
        // the iteration past the last: level K at row l1 for the last pair,
        // checked so that it stores nothing (every wave runs it: one barrier)
        Slot last = sl[0];
#pragma unroll
        for (int u = 1; u < D; ++u)
            if (it + u == iters) last = sl[u];
        if ((iters - it) & 1)
            body(iters, last, std::true_type{}, std::integral_constant<int, 1>{});
        else
            body(iters, last, std::true_type{}, std::integral_constant<int, 0>{});
        if (WRITES) {
#pragma unroll
            for (int q = 0; q < kObsMainQ; ++q) {
                const double sq = wave_sum(oacc[q]);
                if (lane == 0) obs_partial[(int64_t)q * obs_stride + obs_unit] = sq;
            }
        }
    }
}

constexpr int kPairDepth = 2;     // iterations of row loads in flight per producer wave
constexpr int kPairBlock = 128 * kPairStrips;   // threads per workgroup

// One tile of the strip tile set (tile index t) by the workgroup.
template <int S, typename T, int K, bool OBS>
__device__ __forceinline__ void pstrip_tile(const SweepGeom& g, int t, typename Stor<T>::cptr in,
                                            typename Stor<T>::cptr psi, typename Stor<T>::ptr out,
                                            const double* __restrict__ step, int first_term,
                                            double* __restrict__ obs_partial,
                                            StripLds<typename Cplx<T>::type, K>* lds)
{
    const int halo = g.variant * S;             // >= K * S: radii lost per side after K levels
    const int valid = 128 - 2 * halo;           // output radii per strip
    const Tile I = g.tiles[t];
    const int n = I.n;
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
    const int strip = wave >> 1;
    const bool producer = (wave & 1) == 0;
    const int j0 = I.r0 + strip * valid - halo;  // radius a of lane 0
    const int ja = j0 + 2 * lane, jb = ja + 1;
    PairLane P;
    P.ina = ja >= 0 && ja < n;
    P.inb = jb >= 0 && jb < n;
    P.jca = min(max(ja, 0), n - 1);
    P.jcb = min(max(jb, 0), n - 1);
    P.wa = P.ina && 2 * lane >= halo && 2 * lane < 128 - halo;
    P.wb = P.inb && 2 * lane + 1 >= halo && 2 * lane + 1 < 128 - halo;
    const double e_mid = step_value(step, g.n_inst, kEMid, I.inst);
    {
        const double r = (double)(P.jca + 1) * I.dr;
        const double inv_r = 1.0 / r;
        P.ra = r;
        P.inv_r2a = inv_r * inv_r;
        P.dba = diag_base<S>(I.inv_dr2, I.z * inv_r);
        P.era = e_mid * r;
        P.outa = P.jca >= I.i_ion;
    }
    {
        const double r = (double)(P.jcb + 1) * I.dr;
        const double inv_r = 1.0 / r;
        P.rb = r;
        P.inv_r2b = inv_r * inv_r;
        P.dbb = diag_base<S>(I.inv_dr2, I.z * inv_r);
        P.erb = e_mid * r;
        P.outb = P.jcb >= I.i_ion;
    }
    const double dt = step_value(step, g.n_inst, kDt, I.inst);
    double coef[K];
#pragma unroll
    for (int k = 0; k < K; ++k) coef[k] = wave_uniform(dt / (double)(first_term - k));
    const int64_t stride = (int64_t)g.n_tiles * kStripWaves;
    // one partial per strip, in the first kPairStrips units of the tile's
    // four; the others hold zeros (the finish sums all four)
    const int64_t unit = (int64_t)t * kStripWaves + strip;
    if (OBS && producer && lane == 0) {
        for (int u = kPairStrips + strip; u < kStripWaves; u += kPairStrips)
#pragma unroll
            for (int q = 0; q < kObsMainQ; ++q)
                obs_partial[(int64_t)q * stride + (int64_t)t * kStripWaves + u] = 0.0;
    }
    const bool full = j0 >= 0 && j0 + 127 < n;   // wave-uniform, and the same for both waves of a strip
    auto run = [&](auto prod, auto masked) {
        constexpr bool PR = decltype(prod)::value, MK = decltype(masked)::value;
        pair_loop<S, T, K, MK, kPairDepth, OBS, PR>(g, I, in + I.off, psi + I.off, out + I.off, P, coef, lds[strip],
                                                    lane, obs_partial, stride, unit);
    };
    if (producer) {
        if (full) run(std::true_type{}, std::false_type{});
        else run(std::true_type{}, std::true_type{});
    } else {
        if (full) run(std::false_type{}, std::false_type{});
        else run(std::false_type{}, std::true_type{});
    }
}

// PERSIST false: one workgroup per tile (block b -> tile perm[b], or by
// g.order without perm).  PERSIST true: a persistent launch: each workgroup
// takes tiles from the work queue (queue[0] counts the tiles taken; the q-th
// taken is perm[q]) until none is left, then counts itself out in queue[1];
// the last one out resets both counters to zero for the next launch.  The
// queue holds no waits: a workgroup never depends on another, whatever the
// grid size.
template <int S, typename T, int K, bool OBS, bool PERSIST>
__global__ void __launch_bounds__(kPairBlock, 2)
k_horner_pstrip(SweepGeom g, typename Stor<T>::cptr in, typename Stor<T>::cptr psi, typename Stor<T>::ptr out,
                const double* __restrict__ step, int first_term, double* __restrict__ obs_partial,
                unsigned* __restrict__ queue, const int* __restrict__ perm)
{
    using C = typename Cplx<T>::type;
    __shared__ StripLds<C, K> lds[kPairStrips];
    if (!PERSIST) {
        const int t = perm ? perm[blockIdx.x] : my_tile_index(g);
        pstrip_tile<S, T, K, OBS>(g, t, in, psi, out, step, first_term, obs_partial, lds);
        return;
    }
    __shared__ int q_next;
    for (;;) {
        // the previous tile's LDS and the last q_next read are done first
        __syncthreads();
        if (threadIdx.x == 0) q_next = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int q = q_next;
        if (q >= g.n_tiles) break;
        pstrip_tile<S, T, K, OBS>(g, perm[q], in, psi, out, step, first_term, obs_partial, lds);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(queue + 1, 1u) == gridDim.x - 1) {
            atomicExch(queue, 0u);
            atomicExch(queue + 1, 0u);
        }
    }
}

// Workgroups of a persistent launch: those resident at once on the device
// (at least one), at most one per tile.
template <typename F>
static hipError_t resident_grid(F kernel, int n_tiles, int* grid)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kPairBlock, 0);
    if (e != hipSuccess) return e;
    *grid = std::max(1, std::min(n_tiles, std::max(1, per_cu) * std::max(1, cus)));
    return hipSuccess;
}

template <int S, typename T, int K, bool OBS, bool PERSIST>
static hipError_t pstrip_o(const SweepGeom& g, const void* in, const void* psi, void* out, const double* step,
                           int first_term, double* obs_partial, unsigned* queue, const int* perm, hipStream_t st)
{
    auto kernel = k_horner_pstrip<S, T, K, OBS, PERSIST>;
    int grid = g.n_tiles;
    if (PERSIST) {
        hipError_t e = resident_grid(kernel, g.n_tiles, &grid);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kPairBlock), 0, st, g, Stor<T>::cmake(in, g.plane),
                       Stor<T>::cmake(psi, g.plane), Stor<T>::make(out, g.plane), step, first_term, obs_partial,
                       queue, perm);
    return hipGetLastError();
}

// Every term count, storage type and stencil of one launch form (PERSIST).
template <bool PERSIST>
static hipError_t pstrip_dispatch(int prec, int S, int K, const SweepGeom& g, const void* in, const void* psi,
                                  void* out, const double* step, int first_term, hipStream_t st,
                                  double* obs_partial, unsigned* queue, const int* perm)
{
    auto by_k = [&](auto s_tag, auto t_tag) -> hipError_t {
        constexpr int SS = decltype(s_tag)::value;
        using TT = typename decltype(t_tag)::type;
        auto one = [&](auto k_tag) -> hipError_t {
            constexpr int KK = decltype(k_tag)::value;
            return obs_partial
                       ? pstrip_o<SS, TT, KK, true, PERSIST>(g, in, psi, out, step, first_term, obs_partial, queue,
                                                             perm, st)
                       : pstrip_o<SS, TT, KK, false, PERSIST>(g, in, psi, out, step, first_term, obs_partial, queue,
                                                              perm, st);
        };
        switch (K) {
            case 1: return one(std::integral_constant<int, 1>{});
            case 2: return one(std::integral_constant<int, 2>{});
            case 3: return one(std::integral_constant<int, 3>{});
            case 4: return one(std::integral_constant<int, 4>{});
            case 5: return one(std::integral_constant<int, 5>{});
            case 6: return one(std::integral_constant<int, 6>{});
            case 7: return one(std::integral_constant<int, 7>{});
            case 8: return one(std::integral_constant<int, 8>{});
            default: return hipErrorInvalidValue;
        }
    };
    using S1 = std::integral_constant<int, 1>;
    using S2 = std::integral_constant<int, 2>;
    if (prec == 0) return S == 1 ? by_k(S1{}, type_tag<double>{}) : by_k(S2{}, type_tag<double>{});
    if (prec == 2) return S == 1 ? by_k(S1{}, type_tag<s48>{}) : by_k(S2{}, type_tag<s48>{});
    return S == 1 ? by_k(S1{}, type_tag<float>{}) : by_k(S2{}, type_tag<float>{});
}

}  // namespace tdse
