// Observables of Sec. 4 as FP64 reductions in a fixed order:
//   norm, p_ion (eq. yield_1), <z> (eq. Dipole), <z''> (eq. DipoleAccel),
//   p_g (eq. p_g) and the bound-state projections P_nl.
// Pass 1 has two roles in one launch: the first workgroups each take one
// population tile (rows l <= 4 of 256 radial points) and sum the 32
// projection values; the others each stream the rows of one tile of the
// observables' tile set (at most kObsRows rows) and sum 4 values.  Partials are stored [q][tile] so that pass 2 (one
// workgroup per instance, adding its tiles in tile order) reads them
// coalesced.  Results do not depend on scheduling.
#include "device_common.hpp"

namespace tdse {

template <typename T>
__device__ __forceinline__ void obs_main(const SweepGeom& g, int t, typename Stor<T>::cptr psi,
                                         double* __restrict__ partial, double* lds)
{
    const Tile I = g.tiles[t];
    const int n = I.n;
    const int i = I.r0 + (int)threadIdx.x;
    double acc[kObsMainQ] = {0.0, 0.0, 0.0, 0.0};
    if (i < n) {
        const RadialPoint rp = radial_point(I, i);
        const bool outer = i >= I.i_ion;
        // all rows of the tile (at most kObsRows) and the row above it are
        // loaded before any is used: one memory latency per tile
        const int nr = I.l1 - I.l0;
        const int last = min(I.l1, I.lmax);     // the highest row the tile reads
        double2 r[kObsRows + 1];
#pragma unroll
        for (int u = 0; u <= kObsRows; ++u) {
            const int l = I.l0 + u;
            r[u] = (u <= nr && l <= I.lmax) ? ldc(psi, I.off + (int64_t)min(l, last) * n + i) : zero2();
        }
#pragma unroll
        for (int u = 0; u < kObsRows; ++u) {
            if (u < nr) {
                const int l = I.l0 + u;
                const double a2 = fma(r[u].x, r[u].x, r[u].y * r[u].y);
                acc[0] += a2;
                if (outer) acc[1] += a2;
                const double re = fma(r[u].x, r[u + 1].x, r[u].y * r[u + 1].y) * ld_const(g.kappa, l + 1);
                acc[2] = fma(rp.r, re, acc[2]);
                acc[3] = fma(re, rp.inv_r2, acc[3]);
            }
        }
    }
    const double s = block_sum<kObsMainQ>(acc, lds);
    if (threadIdx.x < kObsMainQ) partial[(int64_t)threadIdx.x * g.n_tiles + t] = s;
}

template <typename T>
__device__ __forceinline__ void obs_pop(const SweepGeom& g, int t, const double* __restrict__ radial,
                                        typename Stor<T>::cptr psi, double* __restrict__ partial, double* lds)
{
    const Tile I = g.tiles[t];
    const int n = I.n;
    const int i = I.r0 + (int)threadIdx.x;
    double acc[kObsPopQ];
#pragma unroll
    for (int q = 0; q < kObsPopQ; ++q) acc[q] = 0.0;
    if (i < n) {
        const double* tab = radial + I.tab_off;
        const double2 f0 = ldc(psi, I.off + i);
        const double u = tab[i];
        acc[0] = u * f0.x;
        acc[1] = u * f0.y;
        // states ordered l-major: l = 0 -> 0..4, 1 -> 5..8, 2 -> 9..11, 3 -> 12..13, 4 -> 14
#pragma unroll
        for (int k = 0; k < kMaxStates; ++k) {
            const int kl = (k < 5) ? 0 : (k < 9) ? 1 : (k < 12) ? 2 : (k < 14) ? 3 : 4;
            if (k < I.n_states) {
                const double2 f = ldc(psi, I.off + (int64_t)kl * n + i);
                const double ph = tab[(int64_t)(1 + k) * n + i];
                acc[2 + 2 * k] = ph * f.x;
                acc[3 + 2 * k] = ph * f.y;
            }
        }
    }
    const double s = block_sum<kObsPopQ>(acc, lds);
    if (threadIdx.x < kObsPopQ) partial[(int64_t)threadIdx.x * g.n_tiles + t] = s;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_obs_partial(SweepGeom red, SweepGeom pop, const double* __restrict__ radial,
              typename Stor<T>::cptr psi, double* __restrict__ partial_main,
              double* __restrict__ partial_pop)
{
    __shared__ double lds[(kBlock / 64) * kObsPopQ];
    // the population tiles (more loads and sums each) go first, so they are
    // not the last workgroups of the launch
    if ((int)blockIdx.x < pop.n_tiles)
        obs_pop<T>(pop, (int)blockIdx.x, radial, psi, partial_pop, lds);
    else
        obs_main<T>(red, (int)blockIdx.x - pop.n_tiles, psi, partial_main, lds);
}

constexpr int kFinishU = 8;

__global__ void __launch_bounds__(kBlock)
k_obs_finish(SweepGeom red, SweepGeom pop, const double* __restrict__ pmain,
             const double* __restrict__ ppop, const double* __restrict__ step, int64_t rec_stride,
             double* __restrict__ records, int main_set, int main_upt, int64_t main_stride)
{
    constexpr int Q = kObsMainQ + kObsPopQ;
    __shared__ double lds[(kBlock / 64) * Q];
    __shared__ double tot[Q];
    const int k = blockIdx.x;
    const Inst& I = red.inst[k];
    // the step scalars of the record, loaded now rather than after the sums
    const double t_end = step_value(step, red.n_inst, kTEnd, k);
    const double e = step_value(step, red.n_inst, kEEnd, k);
    const int64_t ridx = (int64_t)step_value(step, red.n_inst, kRec, k);
    double acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = 0.0;
    // up to kFinishU tiles per thread per pass, loaded before any is added:
    // the partials come from every XCD, so each pass costs one memory latency
    const int tb = I.tbegin[main_set] * main_upt, te = I.tend[main_set] * main_upt;
    for (int t0 = tb + (int)threadIdx.x; t0 < te; t0 += kFinishU * kBlock) {
        double v[kFinishU][kObsMainQ];
#pragma unroll
        for (int u = 0; u < kFinishU; ++u) {
            const int t = t0 + u * kBlock;
#pragma unroll
            for (int q = 0; q < kObsMainQ; ++q) v[u][q] = (t < te) ? pmain[(int64_t)q * main_stride + t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinishU; ++u) {
#pragma unroll
            for (int q = 0; q < kObsMainQ; ++q) acc[q] += v[u][q];
        }
    }
    for (int t = I.tbegin[kPopTiles] + (int)threadIdx.x; t < I.tend[kPopTiles]; t += kBlock) {
#pragma unroll
        for (int q = 0; q < kObsPopQ; ++q) acc[kObsMainQ + q] += ppop[(int64_t)q * pop.n_tiles + t];
    }
    const double s = block_sum<Q>(acc, lds);
    if (threadIdx.x < Q) tot[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double dr = I.dr;
        double* rec = records + (int64_t)k * rec_stride + ridx * kObsRecord;
        const double* pp = tot + kObsMainQ;
        rec[0] = t_end;
        rec[1] = e;
        rec[2] = dr * tot[0];
        const double pgr = dr * pp[0], pgi = dr * pp[1];
        rec[3] = pgr * pgr + pgi * pgi;
        double pb = 0.0;
        for (int q = 0; q < kMaxStates; ++q) {
            double popq = 0.0;
            if (q < I.n_states) {
                const double a = dr * pp[2 + 2 * q], b = dr * pp[3 + 2 * q];
                popq = a * a + b * b;
            }
            rec[8 + q] = popq;
            pb += popq;
        }
        rec[4] = pb;
        rec[5] = dr * tot[1];
        rec[6] = 2.0 * dr * tot[2];
        rec[7] = -e - 2.0 * I.z * dr * tot[3];
    }
}

template <typename T>
static hipError_t obs_partial_t(const SweepGeom& red, const SweepGeom& pop, const double* radial_tab,
                                const void* psi, double* partial_main, double* partial_pop, hipStream_t st)
{
    const dim3 grid(red.n_tiles + pop.n_tiles);
    hipLaunchKernelGGL((k_obs_partial<T>), grid, dim3(kBlock), 0, st, red, pop, radial_tab,
                       Stor<T>::cmake(psi, red.plane), partial_main, partial_pop);
    return hipGetLastError();
}

hipError_t launch_obs_partial(int prec, const SweepGeom& red, const SweepGeom& pop,
                              const double* radial_tab, const void* psi, double* partial_main,
                              double* partial_pop, hipStream_t st)
{
    if (prec == 0) return obs_partial_t<double>(red, pop, radial_tab, psi, partial_main, partial_pop, st);
    if (prec == 2) return obs_partial_t<s48>(red, pop, radial_tab, psi, partial_main, partial_pop, st);
    return obs_partial_t<float>(red, pop, radial_tab, psi, partial_main, partial_pop, st);
}

hipError_t launch_obs_finish(const SweepGeom& red, const SweepGeom& pop, const double* partial_main,
                             const double* partial_pop, const double* step, int64_t rec_stride,
                             double* out_records, hipStream_t st, int main_set, int main_upt,
                             int64_t main_stride)
{
    if (main_stride < 0) main_stride = red.n_tiles;
    hipLaunchKernelGGL(k_obs_finish, dim3(red.n_inst), dim3(kBlock), 0, st, red, pop, partial_main,
                       partial_pop, step, rec_stride, out_records, main_set, main_upt, main_stride);
    return hipGetLastError();
}

}  // namespace tdse
