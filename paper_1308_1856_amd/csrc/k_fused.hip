// K consecutive Horner terms of the Taylor step (Sec. 5.2, eq. Taylor) in one
// launch, with the intermediate vectors kept on chip.
//
//   v_0 = in,  v_k = psi + (-i dt / t_k) H v_{k-1}   (k = 1..K, t_k = first_term - k + 1)
//   out = v_K
//
// A workgroup owns 256 consecutive radii (columns c0 .. c0+255) and output rows
// [l0, l1).  Level k needs the rows [l0 - (K-k), l1 - 1 + (K-k)] of level k
// (the l +- 1 coupling widens the range by one row per level), and level k
// must run one row ahead of level k+1.  Both hold with the schedule
//   rho_k(it) = l0 - K + 2 - k + it,   it = 0 .. (l1 - l0) + 2K - 3,
// in which level k works once it >= 2(k-1) (its first needed row) and level
// 1 reads input row rho_1 + 1 from memory.  Levels 1..K-1 keep their last four
// rows in LDS rings; a barrier after each level's write orders it before the
// next level's reads, and a slot is only rewritten two iterations after its
// last read (with barriers in between).  Radial halos: level 1 reads its
// radial neighbours from memory; level k >= 2 reads them from the LDS row of
// level k-1, which is valid on columns [c0 + (k-1)s, c0 + 256 - (k-1)s), so a
// tile writes only the columns [c0 + (K-1)s, c0 + 256 - (K-1)s) and
// neighbouring tiles overlap by 2(K-1)s columns (c0 may be negative).  Rows
// outside [0, lmax] and radii outside [0, N) are zero, as in the single-term
// sweep.
//
// Every element of every level is computed by the same functions (h_point,
// horner_update) as in the single-term sweeps, so FP64 results are
// bit-identical to K single-term launches; in
// FP32 storage mode the intermediates stay FP64 (rounded once per launch).
// HBM traffic per unknown and launch: read `in` and psi once, write out once,
// instead of K times each.  `out` must not alias `in` or `psi`.
#include "device_common.hpp"

namespace tdse {

template <int S, typename T, int K>
__global__ void __launch_bounds__(kBlock)
k_horner_fused(SweepGeom g, const typename Cplx<T>::type* __restrict__ in,
               const typename Cplx<T>::type* __restrict__ psi, typename Cplx<T>::type* __restrict__ out,
               const double* __restrict__ step, int first_term)
{
    constexpr int kSlotsPerLevel = 4;
    // LDS: levels 1..K-1, four rows of 256 complex FP64 each
    __shared__ double2 ring[(K > 1 ? K - 1 : 1) * kSlotsPerLevel * kBlock];

    const Tile I = my_tile(g);
    const int n = I.n;
    const int lmax = I.lmax;
    const int tid = (int)threadIdx.x;
    const int j = I.r0 + tid;             // this thread's radius (may lie outside [0, n))
    const bool inside = j >= 0 && j < n;
    const int jc = inside ? j : 0;        // clamped index for the (unused) loads of outside lanes
    const int lo_out = (K - 1) * S, hi_out = kBlock - (K - 1) * S;
    const bool writes = inside && tid >= lo_out && tid < hi_out;

    const double r = (double)(jc + 1) * I.dr;
    const double inv_r = 1.0 / r;
    const double inv_r2 = inv_r * inv_r;
    const double z_over_r = I.z * inv_r;
    const double er = step_value(step, g.n_inst, kEMid, I.inst) * r;
    const double dt = step_value(step, g.n_inst, kDt, I.inst);
    const int64_t base = I.off;

    // level-0 sliding window at this radius (rows rho_1 - 1, rho_1, rho_1 + 1)
    auto load_in = [&](int l) -> double2 {
        return (inside && l >= 0 && l <= lmax) ? ldc(in, base + (int64_t)l * n + jc) : zero2();
    };
    auto load_psi = [&](int l) -> double2 {
        return (inside && l >= 0 && l <= lmax) ? ldc(psi, base + (int64_t)l * n + jc) : zero2();
    };
    // level-0 sliding window at this radius: rows rho_1 - 1, rho_1 (rho_1 = l0 - K + 1 at it = 0)
    double2 in_prev = load_in(I.l0 - K);
    double2 in_cur = load_in(I.l0 - K + 1);
    // psi at rows rho_1 .. rho_K of the current iteration (pr[k-1] = psi(rho_k))
    double2 pr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) pr[k] = zero2();

    const int iters = (I.l1 - I.l0) + 2 * K - 2;
    for (int it = 0; it < iters; ++it) {
        // ---- level 1: from the input (memory) --------------------------------
        {
            const int rho = I.l0 - K + 1 + it;
            const double2 in_next = load_in(rho + 1);
#pragma unroll
            for (int k = K - 1; k > 0; --k) pr[k] = pr[k - 1];
            pr[0] = load_psi(rho);
            double2 v = zero2();
            if (inside && rho >= 0 && rho <= lmax) {
                Neighbours<S> nb;
                nb.load(in + base + (int64_t)rho * n, jc, n);
                const double d0 = row_diag(half_ll(rho), inv_r2, diag_base<S>(I.inv_dr2, z_over_r));
                const double2 h = h_point<S>(in_cur, nb.m1, nb.p1, nb.m2, nb.p2, in_prev, in_next,
                                             I.inv_dr2, d0, er, g.kappa[rho], g.kappa[rho + 1]);
                v = horner_update(pr[0], h, dt / (double)first_term);
            }
            in_prev = in_cur;
            in_cur = in_next;
            if (K == 1) {
                if (writes && rho >= I.l0 && rho < I.l1) stc(out, base + (int64_t)rho * n + jc, v);
            } else {
                ring[((rho + 4 * K) & 3) * kBlock + tid] = v;
            }
        }
        // ---- levels 2..K: from the LDS ring of the level below ---------------
#pragma unroll
        for (int k = 2; k <= K; ++k) {
            __syncthreads();
            const int rho = I.l0 - K + 2 - k + it;
            const bool active = it >= 2 * (k - 1);       // rho >= first row level k needs
            const double2* below = ring + (size_t)(k - 2) * kSlotsPerLevel * kBlock;
            double2 v = zero2();
            if (active && inside && rho >= 0 && rho <= lmax) {
                const double2* rowm = below + ((rho - 1 + 4 * K) & 3) * kBlock;
                const double2* row0 = below + ((rho + 4 * K) & 3) * kBlock;
                const double2* rowp = below + ((rho + 1 + 4 * K) & 3) * kBlock;
                const double2 cur = row0[tid];
                const double2 lm = (rho > 0) ? rowm[tid] : zero2();
                const double2 lp = (rho < lmax) ? rowp[tid] : zero2();
                // radial neighbours from LDS (zero beyond the box, because the
                // level below stored zeros there; beyond the tile they are only
                // needed by columns this level does not keep valid)
                const double2 m1 = (tid >= 1) ? row0[tid - 1] : zero2();
                const double2 p1 = (tid + 1 < kBlock) ? row0[tid + 1] : zero2();
                double2 m2 = zero2(), p2 = zero2();
                if (S == 2) {
                    m2 = (tid >= 2) ? row0[tid - 2] : zero2();
                    p2 = (tid + 2 < kBlock) ? row0[tid + 2] : zero2();
                }
                const double d0 = row_diag(half_ll(rho), inv_r2, diag_base<S>(I.inv_dr2, z_over_r));
                const double2 h = h_point<S>(cur, m1, p1, m2, p2, lm, lp, I.inv_dr2, d0, er,
                                             g.kappa[rho], g.kappa[rho + 1]);
                v = horner_update(pr[k - 1], h, dt / (double)(first_term - k + 1));
            }
            if (k == K) {
                if (writes && active && rho >= I.l0 && rho < I.l1) stc(out, base + (int64_t)rho * n + jc, v);
            } else {
                ring[((k - 1) * kSlotsPerLevel + ((rho + 4 * K) & 3)) * kBlock + tid] = v;
            }
        }
    }
}

template <int S, typename T, int K>
static hipError_t fused_t(const SweepGeom& g, const void* in, const void* psi, void* out,
                          const double* step, int first_term, hipStream_t st)
{
    using C = typename Cplx<T>::type;
    hipLaunchKernelGGL((k_horner_fused<S, T, K>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                       static_cast<const C*>(in), static_cast<const C*>(psi), static_cast<C*>(out),
                       step, first_term);
    return hipGetLastError();
}

template <int S, typename T>
static hipError_t fused_k(int K, const SweepGeom& g, const void* in, const void* psi, void* out,
                          const double* step, int first_term, hipStream_t st)
{
    switch (K) {
        case 1: return fused_t<S, T, 1>(g, in, psi, out, step, first_term, st);
        case 2: return fused_t<S, T, 2>(g, in, psi, out, step, first_term, st);
        case 3: return fused_t<S, T, 3>(g, in, psi, out, step, first_term, st);
        case 4: return fused_t<S, T, 4>(g, in, psi, out, step, first_term, st);
        case 5: return fused_t<S, T, 5>(g, in, psi, out, step, first_term, st);
        case 6: return fused_t<S, T, 6>(g, in, psi, out, step, first_term, st);
        case 7: return fused_t<S, T, 7>(g, in, psi, out, step, first_term, st);
        case 8: return fused_t<S, T, 8>(g, in, psi, out, step, first_term, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_horner_fused(int prec, int S, int K, const SweepGeom& g, const void* in,
                               const void* psi, void* out, const double* step, int first_term,
                               hipStream_t st)
{
    if (g.gauge != 0) return hipErrorInvalidValue;   // length gauge only
    if (prec == 0) return S == 1 ? fused_k<1, double>(K, g, in, psi, out, step, first_term, st)
                                 : fused_k<2, double>(K, g, in, psi, out, step, first_term, st);
    if (prec != 1) return hipErrorInvalidValue;   // LDS-ring kernel: FP64 and FP32 storage only
    return S == 1 ? fused_k<1, float>(K, g, in, psi, out, step, first_term, st)
                  : fused_k<2, float>(K, g, in, psi, out, step, first_term, st);
}

}  // namespace tdse
