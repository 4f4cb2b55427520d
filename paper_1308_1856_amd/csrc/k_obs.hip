// Observables of Sec. 4 as FP64 reductions in a fixed order:
//   norm, p_ion (eq. yield_1), <z> (eq. Dipole), <z''> (eq. DipoleAccel),
//   p_g (eq. p_g) and the bound-state projections P_nl.
// Pass 1 writes kObsQ partial sums per tile; pass 2 (one workgroup per
// instance) adds the partials of the instance's tiles in tile order and
// forms the record, so results do not depend on scheduling.
#include "device_common.hpp"

namespace tdse {

// partial layout per tile: 0 sum|f|^2, 1 sum_{r>r_b}|f|^2, 2 sum kappa r Re(f_l* f_l+1),
// 3 sum kappa Re(f_l* f_l+1)/r^2, 4/5 sum u0 f_0 (re, im), 6+2k/7+2k sum phi_k f_l(k)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_obs_partial(SweepGeom g, const double* __restrict__ radial, const typename Cplx<T>::type* __restrict__ psi,
              double* __restrict__ partial)
{
    __shared__ double lds[(kBlock / 64) * kObsQ];
    const int t = my_tile_index(g);
    const Tile tile = g.tiles[t];
    const Inst& I = g.inst[tile.inst];
    const int n = I.n;
    const int i = tile.r0 + (int)threadIdx.x;
    double acc[kObsQ];
#pragma unroll
    for (int q = 0; q < kObsQ; ++q) acc[q] = 0.0;
    if (i < n) {
        const RadialPoint rp = radial_point(I, i);
        const double* tab = radial + I.tab_off;
        const bool outer = i >= I.i_ion;
        double2 cur = ldc(psi, I.off + (int64_t)tile.l0 * n + i);
        for (int l = tile.l0; l < tile.l1; ++l) {
            const int64_t row = I.off + (int64_t)l * n;
            const double2 next = (l < I.lmax) ? ldc(psi, row + n + i) : zero2();
            const double a2 = cur.x * cur.x + cur.y * cur.y;
            acc[0] += a2;
            if (outer) acc[1] += a2;
            const double re = cur.x * next.x + cur.y * next.y;
            const double kp = g.kappa[l + 1];
            acc[2] += kp * rp.r * re;
            acc[3] += kp * re * rp.inv_r2;
            if (l == 0) {
                const double u = tab[i];
                acc[4] += u * cur.x;
                acc[5] += u * cur.y;
            }
            if (l <= 4) {
                // states ordered l-major: l = 0 -> 0..4, 1 -> 5..8, 2 -> 9..11, 3 -> 12..13, 4 -> 14
#pragma unroll
                for (int k = 0; k < kMaxStates; ++k) {
                    const int kl = (k < 5) ? 0 : (k < 9) ? 1 : (k < 12) ? 2 : (k < 14) ? 3 : 4;
                    if (kl == l && k < I.n_states) {
                        const double ph = tab[(int64_t)(1 + k) * n + i];
                        acc[6 + 2 * k] += ph * cur.x;
                        acc[7 + 2 * k] += ph * cur.y;
                    }
                }
            }
            cur = next;
        }
    }
    const double s = block_sum<kObsQ>(acc, lds);
    if (threadIdx.x < kObsQ) partial[(int64_t)t * kObsQ + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
k_obs_finish(SweepGeom g, const double* __restrict__ partial, const double* __restrict__ step,
             int64_t rec_stride, double* __restrict__ records)
{
    __shared__ double lds[(kBlock / 64) * kObsQ];
    __shared__ double tot[kObsQ];
    const int k = blockIdx.x;
    const Inst& I = g.inst[k];
    double acc[kObsQ];
#pragma unroll
    for (int q = 0; q < kObsQ; ++q) acc[q] = 0.0;
    for (int t = I.tile_begin + (int)threadIdx.x; t < I.tile_end; t += kBlock) {
#pragma unroll
        for (int q = 0; q < kObsQ; ++q) acc[q] += partial[(int64_t)t * kObsQ + q];
    }
    const double s = block_sum<kObsQ>(acc, lds);
    if (threadIdx.x < kObsQ) tot[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double dr = I.dr;
        const double e = step_value(step, g.n_inst, kEEnd, k);
        double* rec = records + (int64_t)k * rec_stride;
        rec[0] = step_value(step, g.n_inst, kTEnd, k);
        rec[1] = e;
        rec[2] = dr * tot[0];
        const double pgr = dr * tot[4], pgi = dr * tot[5];
        rec[3] = pgr * pgr + pgi * pgi;
        double pb = 0.0;
        for (int q = 0; q < kMaxStates; ++q) {
            double pop = 0.0;
            if (q < I.n_states) {
                const double a = dr * tot[6 + 2 * q], b = dr * tot[7 + 2 * q];
                pop = a * a + b * b;
            }
            rec[8 + q] = pop;
            pb += pop;
        }
        rec[4] = pb;
        rec[5] = dr * tot[1];
        rec[6] = 2.0 * dr * tot[2];
        rec[7] = -e - 2.0 * I.z * dr * tot[3];
    }
}

hipError_t launch_obs_partial(int prec, const SweepGeom& g, const double* radial_tab,
                              const void* psi, double* partial, hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL((k_obs_partial<double>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           radial_tab, static_cast<const double2*>(psi), partial);
    else
        hipLaunchKernelGGL((k_obs_partial<float>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           radial_tab, static_cast<const float2*>(psi), partial);
    return hipGetLastError();
}

hipError_t launch_obs_finish(const SweepGeom& g, const double* partial, const double* step,
                             int64_t rec_stride, double* out_records, hipStream_t st)
{
    hipLaunchKernelGGL(k_obs_finish, dim3(g.n_inst), dim3(kBlock), 0, st, g, partial, step,
                       rec_stride, out_records);
    return hipGetLastError();
}

}  // namespace tdse
