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
    const double e = step_value(step, red.n_inst, kEObs, k);
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

// ---------------------------------------------------------------------------
// absorbing mask (Sec. 2.1) and radial current (Sec. 4, eq. flux)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_mask(SweepGeom g, typename Stor<T>::aptr psi)
{
    const Tile I = my_tile(g);
    const Inst& J = g.inst[I.inst];
    const double rb = J.r_abs;
    if (!(rb > 0.0)) return;   // uniform over the workgroup
    const int i = I.r0 + (int)threadIdx.x;
    if (i >= I.n) return;
    const double r = (double)(i + 1) * I.dr;
    const double m = (r >= rb) ? 0.0 : 1.0 - pow(cos(0.5 * M_PI * (1.0 - r / rb)), J.p_abs);
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t k = I.off + (int64_t)l * I.n + i;
        const double2 v = ldc(psi, k);
        stc(psi, k, make_double2(m * v.x, m * v.y));
    }
}

template <typename T>
static hipError_t mask_t(const SweepGeom& g, void* psi, hipStream_t st)
{
    hipLaunchKernelGGL((k_mask<T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::make(psi, g.plane));
    return hipGetLastError();
}
hipError_t launch_mask(int prec, const SweepGeom& g, void* psi, hipStream_t st)
{
    if (prec == 0) return mask_t<double>(g, psi, st);
    if (prec == 2) return mask_t<s48>(g, psi, st);
    return mask_t<float>(g, psi, st);
}

template <int S, typename T, bool VG>
__global__ void __launch_bounds__(kBlock)
k_flux(SweepGeom g, typename Stor<T>::cptr psi, const double* __restrict__ step, int init,
       double* __restrict__ j_prev, double* __restrict__ yield)
{
    __shared__ double lds[kBlock / 64];
    const int k = blockIdx.x;
    const Inst& I = g.inst[k];
    const int j = I.i_flux;
    if (j < 0) return;   // uniform over the workgroup
    // velocity gauge: A/c at the state's time (the step's start for the
    // first point of the trapezoid, its end after the step)
    const double a = VG ? step_value(step, g.n_inst, init ? kEStart : kEEnd, k) : 0.0;
    double acc[1] = {0.0};
    for (int l = (int)threadIdx.x; l <= I.lmax; l += kBlock) {
        const int64_t row = I.off + (int64_t)l * I.n;
        auto at = [&](int i) { return (i >= 0 && i < I.n) ? ldc(psi, row + i) : zero2(); };
        auto at_row = [&](int r) { return ldc(psi, I.off + (int64_t)r * I.n + j); };
        const double2 f = at(j);
        double2 d;
        if (S == 1) {
            const double2 a = at(j + 1), b = at(j - 1);
            const double s = 1.0 / (2.0 * I.dr);
            d = make_double2((a.x - b.x) * s, (a.y - b.y) * s);
        } else {
            const double2 m2 = at(j - 2), m1 = at(j - 1), p1 = at(j + 1), p2 = at(j + 2);
            const double s = 1.0 / (12.0 * I.dr);
            d = make_double2((m2.x - 8.0 * m1.x + 8.0 * p1.x - p2.x) * s, (m2.y - 8.0 * m1.y + 8.0 * p1.y - p2.y) * s);
        }
        acc[0] += fma(f.x, d.y, -(f.y * d.x));   // Im(conj(f) d)
        if (VG && l < I.lmax) {
            // + 2 (A/c) kappa_{l+1} Re(conj(f_l) f_{l+1})
            const double2 fp = at_row(l + 1);
            acc[0] += 2.0 * a * g.kappa[l + 1] * fma(f.x, fp.x, f.y * fp.y);
        }
    }
    const double cur = block_sum<1>(acc, lds);
    if (threadIdx.x == 0) {
        if (!init) yield[k] += 0.5 * step_value(step, g.n_inst, kDt, k) * (j_prev[k] + cur);
        j_prev[k] = cur;
    }
}

template <int S, typename T>
static hipError_t flux_t(const SweepGeom& g, const void* psi, const double* step, int init, double* j_prev,
                         double* yield, hipStream_t st)
{
    if (g.gauge != 0)
        hipLaunchKernelGGL((k_flux<S, T, true>), dim3(g.n_inst), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(psi, g.plane), step, init, j_prev, yield);
    else
        hipLaunchKernelGGL((k_flux<S, T, false>), dim3(g.n_inst), dim3(kBlock), 0, st, g,
                           Stor<T>::cmake(psi, g.plane), step, init, j_prev, yield);
    return hipGetLastError();
}
hipError_t launch_flux(int prec, int S, const SweepGeom& g, const void* psi, const double* step, int init,
                       double* j_prev, double* yield, hipStream_t st)
{
    if (prec == 0) return S == 1 ? flux_t<1, double>(g, psi, step, init, j_prev, yield, st)
                                 : flux_t<2, double>(g, psi, step, init, j_prev, yield, st);
    if (prec == 2) return S == 1 ? flux_t<1, s48>(g, psi, step, init, j_prev, yield, st)
                                 : flux_t<2, s48>(g, psi, step, init, j_prev, yield, st);
    return S == 1 ? flux_t<1, float>(g, psi, step, init, j_prev, yield, st)
                  : flux_t<2, float>(g, psi, step, init, j_prev, yield, st);
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
