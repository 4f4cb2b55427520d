// Sweep kernels: H.psi (Sec. 2, eq. h_matrix), one fused Horner term of the
// Taylor step (Sec. 5.2, eq. Taylor) and the fused classic RK4 stage
// (Sec. 5.2, eq. RKDeriv).
//
// Work decomposition: a workgroup of 256 threads owns 256 consecutive radial
// points of rows [l0, l1) of one instance.  Each thread walks down its rows
// keeping f_{l-1}, f_l, f_{l+1} at its radius in registers, so the l +- 1
// coupling costs one new load per row; the radial neighbours come from the
// same row through the L1/L2 caches.  All arithmetic is FP64; storage is FP64
// or FP32.  HBM traffic per unknown and term: read `in` once, read psi once,
// write out once.
#include "device_common.hpp"

namespace tdse {

template <int S, typename T, bool PIPE>
__global__ void __launch_bounds__(kBlock)
k_hsweep(SweepGeom g, const typename Cplx<T>::type* __restrict__ in,
         const typename Cplx<T>::type* psi, typename Cplx<T>::type* out,
         const double* __restrict__ step, int term)
{
    using C = typename Cplx<T>::type;
    const Tile I = my_tile(g);
    const int n = I.n;
    const int i = I.r0 + (int)threadIdx.x;
    if (i >= n) return;
    const RadialPoint rp = radial_point(I, i);
    const double e = step_value(step, g.n_inst, kEMid, I.inst);
    const double er = e * rp.r;
    // Horner term: out = psi + (-i dt/term) h;  (-i c)(x + i y) = c y - i c x
    const double c = (term > 0) ? step_value(step, g.n_inst, kDt, I.inst) / (double)term : 0.0;
    const int64_t base = I.off;

    if (!PIPE) {
        // plain loop: one row at a time (fewer registers, more waves)
        double2 prev = (I.l0 > 0) ? ldc(in, base + (int64_t)(I.l0 - 1) * n + i) : zero2();
        double2 cur = ldc(in, base + (int64_t)I.l0 * n + i);
        for (int l = I.l0; l < I.l1; ++l) {
            const int64_t row = base + (int64_t)l * n;
            const double2 next = (l < I.lmax) ? ldc(in, row + n + i) : zero2();
            Neighbours<S, C> nb;
            nb.load(in + row, i, n);
            const double v = 0.5 * (double)l * (double)(l + 1) * rp.inv_r2 - rp.z_over_r;
            const double2 h = h_point<S>(cur, nb.m1, nb.p1, nb.m2, nb.p2, prev, next, I.inv_dr2, v,
                                         er, g.kappa[l], g.kappa[l + 1]);
            if (term > 0) {
                const double2 p = ldc(psi, row + i);
                stc(out, row + i, make_double2(p.x + c * h.y, p.y - c * h.x));
            } else {
                stc(out, row + i, h);
            }
            prev = cur;
            cur = next;
        }
        return;
    }
    // Software pipeline: the loads row l + 1 needs (the input two rows ahead,
    // the radial neighbours of row l + 1, psi of row l + 1) are issued before
    // row l is computed and stored.  Safe when out == psi: a thread reads
    // psi(l + 1, i) and writes out(l, i), never the same element.
    const C* row0 = in + base + (int64_t)I.l0 * n;
    double2 prev = (I.l0 > 0) ? ldc(row0 - n, i) : zero2();
    double2 cur = ldc(row0, i);
    double2 next = (I.l0 < I.lmax) ? ldc(row0 + n, i) : zero2();
    Neighbours<S, C> nb;
    nb.load(row0, i, n);
    double2 p = (term > 0) ? ldc(psi + base + (int64_t)I.l0 * n, i) : zero2();
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t row = base + (int64_t)l * n;
        const bool more = l + 1 < I.l1;
        const double2 next2 = (l + 2 <= I.lmax) ? ldc(in, row + 2 * n + i) : zero2();
        Neighbours<S, C> nb_next;
        if (more) nb_next.load(in + row + n, i, n);
        const double2 p_next = (more && term > 0) ? ldc(psi, row + n + i) : zero2();

        const double v = 0.5 * (double)l * (double)(l + 1) * rp.inv_r2 - rp.z_over_r;
        const double2 h = h_point<S>(cur, nb.m1, nb.p1, nb.m2, nb.p2, prev, next, I.inv_dr2, v, er,
                                     g.kappa[l], g.kappa[l + 1]);
        if (term > 0)
            stc(out, row + i, make_double2(p.x + c * h.y, p.y - c * h.x));
        else
            stc(out, row + i, h);
        prev = cur;
        cur = next;
        next = next2;
        if (more) nb = nb_next;
        p = p_next;
    }
}

// Classic RK4 with k_s = -i H(t_s) g_s:
//   stage 0: g = psi                 acc  = psi + dt/6 k, gout = psi + dt/2 k
//   stage 1: g = gin                 acc += dt/3 k,       gout = psi + dt/2 k
//   stage 2: g = gin                 acc += dt/3 k,       gout = psi + dt k
//   stage 3: g = gin                 psi  = acc + dt/6 k
// H is taken at t_n (stage 0), t_n + dt/2 (stages 1, 2) and t_n + dt (stage 3).
template <int S, typename T, int STAGE>
__global__ void __launch_bounds__(kBlock)
k_rk4_stage(SweepGeom g, const typename Cplx<T>::type* __restrict__ gin,
            typename Cplx<T>::type* psi, typename Cplx<T>::type* acc,
            typename Cplx<T>::type* __restrict__ gout, const double* __restrict__ step)
{
    using C = typename Cplx<T>::type;
    const Tile I = my_tile(g);
    const int n = I.n;
    const int i = I.r0 + (int)threadIdx.x;
    if (i >= n) return;
    const RadialPoint rp = radial_point(I, i);
    const int slot = (STAGE == 0) ? kEStart : (STAGE == 3 ? kEEnd : kEMid);
    const double er = step_value(step, g.n_inst, slot, I.inst) * rp.r;
    const double dt = step_value(step, g.n_inst, kDt, I.inst);
    const double bw = (STAGE == 0 || STAGE == 3) ? dt / 6.0 : dt / 3.0;
    const double aw = (STAGE == 2) ? dt : 0.5 * dt;
    const int64_t base = I.off;
    constexpr bool kReadAcc = STAGE > 0;
    constexpr bool kReadPsi = STAGE == 1 || STAGE == 2;

    // software pipeline as in k_hsweep: row l + 1's loads go out before row l
    // is stored (acc and psi are read and written only at a thread's own
    // elements, one row apart)
    const C* row0 = gin + base + (int64_t)I.l0 * n;
    double2 prev = (I.l0 > 0) ? ldc(row0 - n, i) : zero2();
    double2 cur = ldc(row0, i);
    double2 next = (I.l0 < I.lmax) ? ldc(row0 + n, i) : zero2();
    Neighbours<S, C> nb;
    nb.load(row0, i, n);
    double2 a = kReadAcc ? ldc(acc, base + (int64_t)I.l0 * n + i) : zero2();
    double2 p = kReadPsi ? ldc(psi, base + (int64_t)I.l0 * n + i) : zero2();
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t row = base + (int64_t)l * n;
        const bool more = l + 1 < I.l1;
        const double2 next2 = (l + 2 <= I.lmax) ? ldc(gin, row + 2 * n + i) : zero2();
        Neighbours<S, C> nb_next;
        if (more) nb_next.load(gin + row + n, i, n);
        const double2 a_next = (kReadAcc && more) ? ldc(acc, row + n + i) : zero2();
        const double2 p_next = (kReadPsi && more) ? ldc(psi, row + n + i) : zero2();

        const double v = 0.5 * (double)l * (double)(l + 1) * rp.inv_r2 - rp.z_over_r;
        const double2 h = h_point<S>(cur, nb.m1, nb.p1, nb.m2, nb.p2, prev, next, I.inv_dr2, v, er,
                                     g.kappa[l], g.kappa[l + 1]);
        const double2 k = make_double2(h.y, -h.x);  // -i h
        if (STAGE == 0) {
            stc(acc, row + i, make_double2(cur.x + bw * k.x, cur.y + bw * k.y));
            stc(gout, row + i, make_double2(cur.x + aw * k.x, cur.y + aw * k.y));
        } else if (STAGE < 3) {
            stc(acc, row + i, make_double2(a.x + bw * k.x, a.y + bw * k.y));
            stc(gout, row + i, make_double2(p.x + aw * k.x, p.y + aw * k.y));
        } else {
            stc(psi, row + i, make_double2(a.x + bw * k.x, a.y + bw * k.y));
        }
        prev = cur;
        cur = next;
        next = next2;
        if (more) nb = nb_next;
        a = a_next;
        p = p_next;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_copy(SweepGeom g, const typename Cplx<T>::type* __restrict__ src, typename Cplx<T>::type* __restrict__ dst)
{
    const Tile I = my_tile(g);
    const int i = I.r0 + (int)threadIdx.x;
    if (i >= I.n) return;
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t k = I.off + (int64_t)l * I.n + i;
        dst[k] = src[k];
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

// Counts elements (over the tiles of g) whose stored values differ bit for bit.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_count_diff(SweepGeom g, const typename Cplx<T>::type* __restrict__ a,
             const typename Cplx<T>::type* __restrict__ b, unsigned int* __restrict__ count)
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
k_diff_norm(SweepGeom g, const typename Cplx<T>::type* __restrict__ a,
            const typename Cplx<T>::type* __restrict__ b, double* __restrict__ out)
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
    if (g.variant == 1)
        hipLaunchKernelGGL((k_hsweep<S, T, true>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           static_cast<const C*>(in), static_cast<const C*>(psi), static_cast<C*>(out),
                           step, term);
    else
        hipLaunchKernelGGL((k_hsweep<S, T, false>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           static_cast<const C*>(in), static_cast<const C*>(psi), static_cast<C*>(out),
                           step, term);
    return hipGetLastError();
}

hipError_t launch_hsweep(int prec, int S, const SweepGeom& g, const void* in, const void* psi,
                         void* out, const double* step, int term, hipStream_t st)
{
    if (prec == 0) return S == 1 ? hsweep_t<1, double>(g, in, psi, out, step, term, st)
                                 : hsweep_t<2, double>(g, in, psi, out, step, term, st);
    return S == 1 ? hsweep_t<1, float>(g, in, psi, out, step, term, st)
                  : hsweep_t<2, float>(g, in, psi, out, step, term, st);
}

template <int S, typename T, int STAGE>
static hipError_t rk4_t(const SweepGeom& g, const void* gin, const void* psi, void* acc, void* gout,
                        const double* step, hipStream_t st)
{
    using C = typename Cplx<T>::type;
    hipLaunchKernelGGL((k_rk4_stage<S, T, STAGE>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                       static_cast<const C*>(gin), static_cast<C*>(const_cast<void*>(psi)),
                       static_cast<C*>(acc), static_cast<C*>(gout), step);
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
    return S == 1 ? rk4_s<1, float>(g, stage, gin, psi, acc, gout, step, st)
                  : rk4_s<2, float>(g, stage, gin, psi, acc, gout, step, st);
}

hipError_t launch_count_diff(int prec, const SweepGeom& g, const void* a, const void* b,
                             unsigned int* count, hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL((k_count_diff<double>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           static_cast<const double2*>(a), static_cast<const double2*>(b), count);
    else
        hipLaunchKernelGGL((k_count_diff<float>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           static_cast<const float2*>(a), static_cast<const float2*>(b), count);
    return hipGetLastError();
}

hipError_t launch_diff_norm(int prec, const SweepGeom& g, const void* a, const void* b, double* out,
                            hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL((k_diff_norm<double>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           static_cast<const double2*>(a), static_cast<const double2*>(b), out);
    else
        hipLaunchKernelGGL((k_diff_norm<float>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           static_cast<const float2*>(a), static_cast<const float2*>(b), out);
    return hipGetLastError();
}

hipError_t launch_copy(int prec, const SweepGeom& g, const void* src, void* dst, hipStream_t st)
{
    if (prec == 0)
        hipLaunchKernelGGL((k_copy<double>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           static_cast<const double2*>(src), static_cast<double2*>(dst));
    else
        hipLaunchKernelGGL((k_copy<float>), dim3(g.n_tiles), dim3(kBlock), 0, st, g,
                           static_cast<const float2*>(src), static_cast<float2*>(dst));
    return hipGetLastError();
}

}  // namespace tdse
