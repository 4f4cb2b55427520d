// Lanczos propagator (Sec. 5.2 Lanczos.c; appendix "Lanczos methods").
// All its kernels run over the reduce tile set (at most 16 rows per tile), so
// the per-tile partial sums of the 2m dot products stay small.
//
// Per step and instance: q_0 = F/||F||; for j = 0..m-1:
//   sweep A:  w = H(t_mid) q_j, partial sums of h_i = <q_i, w>, i <= j
//   finish A: h_i, alpha_j = Re h_j
//   sweep B:  q_{j+1} <- w - sum_i h_i q_i  (one classical Gram-Schmidt pass
//             against every earlier vector: three-term recurrence plus full
//             re-orthogonalisation), partial sums of ||.||^2
//   finish B: beta_j, scale of q_{j+1} = 1/beta_j, breakdown test
// then c = ||F|| exp(-i T dt) e_1 for the tridiagonal T (one workgroup per
// instance, scaling and squaring in LDS) and F <- sum_k c_k q_k.
//
// Basis vectors are stored unnormalised (FP64 or FP32) and scaled on load by
// FP64 factors; q_0 is the state buffer itself.  All inner products, norms
// and coefficients are FP64.
#include <type_traits>

#include "device_common.hpp"

namespace tdse {

// Vector j of the basis: the state for j = 0, else stored vector j at
// basis + (j - 1) stride elements (with s48 storage the basis vectors are
// stored plane by plane: their h planes one after another, then their l
// planes, so the same element arithmetic reaches both).
template <typename P>
__device__ __forceinline__ P basis_vec(P psi, P basis, int64_t stride, int j)
{
    return (j == 0) ? psi : basis + (int64_t)(j - 1) * stride;
}
template <typename C> __device__ __forceinline__ const C* cview(const C* p) { return p; }
__device__ __forceinline__ P48 cview(P48 p) { return p; }

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_lz_norm(SweepGeom g, typename Stor<T>::cptr psi, double* __restrict__ partial)
{
    __shared__ double lds[kBlock / 64];
    const int t = my_tile_index(g);
    const Tile I = g.tiles[t];
    const Tile& tile = I;
    const int i = tile.r0 + (int)threadIdx.x;
    double acc[1] = {0.0};
    if (i < I.n) {
        for (int l = tile.l0; l < tile.l1; ++l) {
            const double2 v = ldc(psi, I.off + (int64_t)l * I.n + i);
            acc[0] = fma(v.x, v.x, fma(v.y, v.y, acc[0]));
        }
    }
    const double s = block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partial[t] = s;
}

// One workgroup per instance: sum nq partials over the instance's tiles in a
// fixed order (partial q of tile t at partial[q * stride + t]: the tiles of one
// q are contiguous, so the loads of a wave are coalesced); thread q < nq
// receives sum q.
template <int NQ>
__device__ __forceinline__ double instance_sum(const Inst& I, const double* partial, int stride,
                                               int nq, double* lds)
{
    // U tiles per thread per pass, all loaded before any is added (the
    // partials come from every XCD: one memory latency per pass); each thread
    // still adds its tiles in increasing order
    constexpr int U = NQ >= 8 ? 4 : 8;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    const int tb = I.tbegin[kReduceTiles], te = I.tend[kReduceTiles];
    for (int t0 = tb + (int)threadIdx.x; t0 < te; t0 += U * kBlock) {
        double v[U][NQ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * kBlock;
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[u][q] = (t < te && q < nq) ? partial[(int64_t)q * stride + t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (t0 + u * kBlock < te) {
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (q < nq) acc[q] += v[u][q];
            }
        }
    }
    return block_sum<NQ>(acc, lds);
}

__global__ void __launch_bounds__(kBlock)
k_lz_norm_finish(SweepGeom g, const double* __restrict__ partial, LanczosScalars* __restrict__ scs)
{
    __shared__ double lds[kBlock / 64];
    const int k = blockIdx.x;
    const double s = instance_sum<1>(g.inst[k], partial, 1, 1, lds);
    if (threadIdx.x == 0) {
        LanczosScalars& sc = scs[k];
        const double nrm = sqrt(s);
        sc.norm0 = nrm;
        sc.meff = 0;
        sc.done = (nrm > 0.0) ? 0 : 1;
        sc.scale[0] = (nrm > 0.0) ? 1.0 / nrm : 0.0;
    }
}

// Sweep A for iteration j: w = H q_j over the tile rows, then the partial
// sums of <q_i, w> for i <= j (w re-read from the lines this thread just
// wrote, eight basis vectors at a time).
template <int S, typename T, bool VG = false>
__global__ void __launch_bounds__(kBlock)
k_lz_sweep_a(SweepGeom g, int j, int m, typename Stor<T>::captr psi, typename Stor<T>::captr basis, int64_t stride,
             typename Stor<T>::aptr w, const double* __restrict__ step, const LanczosScalars* __restrict__ scs,
             double* __restrict__ partial)
{
    constexpr int JB = 8;
    __shared__ double lds[(kBlock / 64) * 2 * JB];
    const int t = my_tile_index(g);
    const Tile I = g.tiles[t];
    const Tile& tile = I;
    const LanczosScalars& sc = scs[tile.inst];
    if (sc.done) return;  // uniform over the workgroup
    const int n = I.n;
    const int i = tile.r0 + (int)threadIdx.x;
    const bool active = i < n;
    const auto qj = basis_vec(psi, basis, stride, j);
    const double sj = sc.scale[j];

    if (active) {
        const RadialPoint rp = radial_point(I, i);
        const double fld = step_value(step, g.n_inst, kEMid, tile.inst);
        const double er = VG ? 0.0 : fld * rp.r;
        const double inv_dr = 1.0 / I.dr;
        const int64_t base = I.off;
        double2 prev = (tile.l0 > 0) ? ldc(qj, base + (int64_t)(tile.l0 - 1) * n + i) : zero2();
        double2 cur = ldc(qj, base + (int64_t)tile.l0 * n + i);
        Neighbours<S> nbm, nb;   // rows l - 1 and l (velocity gauge)
        if (VG) {
            nbm.zero();
            if (tile.l0 > 0) nbm.load(qj + (base + (int64_t)(tile.l0 - 1) * n), i, n);
            nb.load(qj + (base + (int64_t)tile.l0 * n), i, n);
        }
        for (int l = tile.l0; l < tile.l1; ++l) {
            const int64_t row = base + (int64_t)l * n;
            const double2 next = (l < I.lmax) ? ldc(qj, row + n + i) : zero2();
            Neighbours<S> nbp;
            if (VG) {
                nbp.zero();
                if (l < I.lmax) nbp.load(qj + (row + n), i, n);
            } else {
                nb.load(qj + row, i, n);
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
            h.x *= sj;
            h.y *= sj;
            stc_keep(w, row + i, h);
            prev = cur;
            cur = next;
        }
    }
    for (int i0 = 0; i0 <= j; i0 += JB) {
        double acc[2 * JB];
#pragma unroll
        for (int q = 0; q < 2 * JB; ++q) acc[q] = 0.0;
        if (active) {
            // the group's scale factors, read once (not per row)
            double su[JB];
#pragma unroll
            for (int u = 0; u < JB; ++u) su[u] = (i0 + u <= j) ? sc.scale[i0 + u] : 0.0;
            for (int l = tile.l0; l < tile.l1; ++l) {
                const int64_t k = I.off + (int64_t)l * n + i;
                const double2 wv = ldc(w, k);
#pragma unroll
                for (int u = 0; u < JB; ++u) {
                    if (i0 + u <= j) {
                        const double s = su[u];
                        const double2 q = ldc(basis_vec(psi, basis, stride, i0 + u), k);
                        // conj(s q) w
                        acc[2 * u] = fma(s, fma(q.x, wv.x, q.y * wv.y), acc[2 * u]);
                        acc[2 * u + 1] = fma(s, fma(q.x, wv.y, -(q.y * wv.x)), acc[2 * u + 1]);
                    }
                }
            }
        }
        const double s = block_sum<2 * JB>(acc, lds);
        if ((int)threadIdx.x < 2 * JB && i0 + (int)threadIdx.x / 2 <= j)
            partial[(int64_t)(2 * i0 + threadIdx.x) * g.n_tiles + t] = s;
    }
}

__global__ void __launch_bounds__(kBlock)
k_lz_finish_a(SweepGeom g, int j, int m, const double* __restrict__ partial,
              LanczosScalars* __restrict__ scs)
{
    constexpr int JB = 8;
    __shared__ double lds[(kBlock / 64) * 2 * JB];
    const int k = blockIdx.x;
    LanczosScalars& sc = scs[k];
    if (sc.done) return;
    const Inst& I = g.inst[k];
    // workgroup (k, y) sums the products i0 = y JB .. i0 + JB - 1 (all groups
    // of an instance run side by side)
    const int i0 = (int)blockIdx.y * JB;
    if (i0 > j) return;
    const int nq = min(2 * JB, 2 * (j + 1 - i0));
    const double s = instance_sum<2 * JB>(I, partial + (int64_t)2 * i0 * g.n_tiles, g.n_tiles, nq, lds);
    if ((int)threadIdx.x < nq) sc.h[2 * i0 + threadIdx.x] = s;
    // Re <q_j, H q_j>, from the one group that holds product j
    if (j - i0 < JB && (int)threadIdx.x == 2 * (j - i0)) sc.alpha[j] = s;
    if (blockIdx.y == 0 && threadIdx.x == 0) sc.meff = j + 1;
}

// q_{j+1} (stored unnormalised) = w - sum_{i<=j} h_i q_i, and ||.||^2 partials.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_lz_sweep_b(SweepGeom g, int j, typename Stor<T>::captr psi, typename Stor<T>::aptr basis, int64_t stride,
             typename Stor<T>::cptr w, const LanczosScalars* __restrict__ scs, double* __restrict__ partial)
{
    __shared__ double lds[kBlock / 64];
    const int t = my_tile_index(g);
    const Tile I = g.tiles[t];
    const Tile& tile = I;
    const LanczosScalars& sc = scs[tile.inst];
    if (sc.done) return;
    const int i = tile.r0 + (int)threadIdx.x;
    const auto out = basis + (int64_t)j * stride;  // vector j+1
    double acc[1] = {0.0};
    if (i < I.n) {
        for (int l = tile.l0; l < tile.l1; ++l) {
            const int64_t k = I.off + (int64_t)l * I.n + i;
            double2 v = ldc(w, k);
            for (int q = 0; q <= j; ++q) {
                const double s = sc.scale[q];
                const double hr = s * sc.h[2 * q], hi = s * sc.h[2 * q + 1];
                const double2 b = ldc(basis_vec(psi, cview(basis), stride, q), k);
                v.x = fma(-hr, b.x, fma(hi, b.y, v.x));
                v.y = fma(-hr, b.y, fma(-hi, b.x, v.y));
            }
            stc_keep(out, k, v);
            // the norm is taken of the stored (possibly rounded) vector
            const double2 vs = ldc(out, k);
            acc[0] = fma(vs.x, vs.x, fma(vs.y, vs.y, acc[0]));
        }
    }
    const double s = block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partial[t] = s;
}

__global__ void __launch_bounds__(kBlock)
k_lz_finish_b(SweepGeom g, int j, const double* __restrict__ partial, LanczosScalars* __restrict__ scs)
{
    __shared__ double lds[kBlock / 64];
    const int k = blockIdx.x;
    LanczosScalars& sc = scs[k];
    if (sc.done) return;
    const double s = instance_sum<1>(g.inst[k], partial, 1, 1, lds);
    if (threadIdx.x == 0) {
        const double b = sqrt(s);
        sc.beta[j] = b;
        if (!(b > g.inst[k].breakdown)) {
            sc.done = 1;  // invariant subspace: keep meff = j + 1
        } else {
            sc.scale[j + 1] = 1.0 / b;
        }
    }
}

// Exponential of the Krylov matrix, c = ||F|| exp(-i T dt) e_1 (Sec. 5.2 and
// the appendix on Lanczos methods; the exponential by scaling and squaring):
//   B = T dt / 2^s with ||B||_inf <= 1/2,
//   exp(-i B) = X - i Y,  X = sum_{k even} (-1)^{k/2} B^k / k!,
//                         Y = sum_{k odd} (-1)^{(k-1)/2} B^k / k!  (k <= 17;
//   the remainder is below 0.5^18 / 18! < 1e-21),
//   then s squarings (X - iY)^2 = (X^2 - Y^2) - i (XY + YX).
// One workgroup per instance; the m x m real matrices live in LDS, each
// thread computes a fixed set of entries of every product (fixed summation
// order: results do not depend on scheduling).  Every matrix is a polynomial
// in the symmetric B, so each product is formed on the upper triangle and
// mirrored, X and Y commute (XY + YX = 2XY), and the Taylor products P B take
// three terms per entry (B is tridiagonal).  T is exponentiated as a
// whole; no eigen-decomposition, unlike the oracle, which diagonalises T.
constexpr int kExpmTerms = 17;
constexpr int kExpmPerThread = (kMaxKrylov * kMaxKrylov + kBlock - 1) / kBlock;
constexpr int kExpmUpper = (kMaxKrylov * (kMaxKrylov + 1) / 2 + kBlock - 1) / kBlock;   // upper-triangle entries per thread

// Row r of L times column c of R, with four independent partial sums (a
// fixed order, so the result does not depend on scheduling).
__device__ __forceinline__ double lds_dot(const double* L, const double* R, int m, int r, int c)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = 0;
    for (; j + 3 < m; j += 4) {
        a0 = fma(L[r * m + j], R[j * m + c], a0);
        a1 = fma(L[r * m + j + 1], R[(j + 1) * m + c], a1);
        a2 = fma(L[r * m + j + 2], R[(j + 2) * m + c], a2);
        a3 = fma(L[r * m + j + 3], R[(j + 3) * m + c], a3);
    }
    for (; j < m; ++j) a0 = fma(L[r * m + j], R[j * m + c], a0);
    return (a0 + a1) + (a2 + a3);
}

__global__ void __launch_bounds__(kBlock)
k_lz_expm(SweepGeom g, const double* __restrict__ step, LanczosScalars* __restrict__ scs)
{
    __shared__ double Bm[kMaxKrylov * kMaxKrylov];
    __shared__ double Pm[kMaxKrylov * kMaxKrylov];
    __shared__ double Xm[kMaxKrylov * kMaxKrylov];
    __shared__ double Ym[kMaxKrylov * kMaxKrylov];
    const int inst = blockIdx.x;
    LanczosScalars& sc = scs[inst];
    const int m = sc.meff;
    const int mm = m * m;
    const int tid = (int)threadIdx.x;
    // the dimension the step used, for the breakdown report of the call
    if (tid == 0) sc.meff_min = min(sc.meff_min, m);
    const double dt = step_value(step, g.n_inst, kDt, inst);

    // ||T dt||_inf and the number of squarings (the same in every thread)
    double tn = 0.0;
    for (int k = 0; k < m; ++k) {
        double row = fabs(sc.alpha[k]);
        if (k > 0) row += fabs(sc.beta[k - 1]);
        if (k + 1 < m) row += fabs(sc.beta[k]);
        tn = fmax(tn, row);
    }
    tn *= dt;
    int nsq = 0;
    while (tn > 0.5 && nsq < 60) {
        tn *= 0.5;
        ++nsq;
    }
    const double scl = ldexp(dt, -nsq);

    for (int e = 0; e < kExpmPerThread; ++e) {
        const int idx = tid + e * kBlock;
        if (idx < mm) {
            const int r = idx / m, c = idx - r * m;
            double v = 0.0;
            if (r == c) v = sc.alpha[r];
            else if (c == r + 1) v = sc.beta[r];
            else if (r == c + 1) v = sc.beta[c];
            v *= scl;
            Bm[idx] = v;
            Pm[idx] = v;
            Xm[idx] = (r == c) ? 1.0 : 0.0;
            Ym[idx] = v;
        }
    }
    // Every matrix here is a polynomial in the symmetric B: symmetric, and X
    // and Y commute.  Each product is formed on the upper triangle (entry
    // (r, c), r <= c, the thread's fixed entries) and mirrored.
    const int nut = m * (m + 1) / 2;
    int ur[kExpmUpper], uc[kExpmUpper];
    for (int e = 0; e < kExpmUpper; ++e) {
        int t = tid + e * kBlock, r = 0;
        ur[e] = uc[e] = 0;
        if (t < nut) {
            while (t >= m - r) {
                t -= m - r;
                ++r;
            }
            ur[e] = r;
            uc[e] = r + t;
        }
    }
    __syncthreads();
    // Taylor terms: P <- P B / k, added to X (even k) or Y (odd k) with sign
    for (int k = 2; k <= kExpmTerms; ++k) {
        double nv[kExpmUpper];
        const double inv_k = 1.0 / (double)k;
        for (int e = 0; e < kExpmUpper; ++e) {
            nv[e] = 0.0;
            if (tid + e * kBlock < nut) {
                // (P B)[r][c] with B tridiagonal: three terms
                const int r = ur[e], c = uc[e];
                double v = Pm[r * m + c] * Bm[c * m + c];
                if (c > 0) v = fma(Pm[r * m + c - 1], Bm[(c - 1) * m + c], v);
                if (c + 1 < m) v = fma(Pm[r * m + c + 1], Bm[(c + 1) * m + c], v);
                nv[e] = v * inv_k;
            }
        }
        __syncthreads();
        const double sgn = ((k / 2) & 1) ? -1.0 : 1.0;   // (-1)^{k/2} even, (-1)^{(k-1)/2} odd
        for (int e = 0; e < kExpmUpper; ++e) {
            if (tid + e * kBlock < nut) {
                const int a = ur[e] * m + uc[e], b = uc[e] * m + ur[e];
                Pm[a] = Pm[b] = nv[e];
                if (k & 1) Ym[a] = Ym[b] = fma(sgn, nv[e], Ym[a]);
                else Xm[a] = Xm[b] = fma(sgn, nv[e], Xm[a]);
            }
        }
        __syncthreads();
    }
    // squarings: (X - iY)^2 = (X^2 - Y^2) - i 2XY
    for (int q = 0; q < nsq; ++q) {
        double nx[kExpmUpper], ny[kExpmUpper];
        for (int e = 0; e < kExpmUpper; ++e) {
            nx[e] = ny[e] = 0.0;
            if (tid + e * kBlock < nut) {
                const int r = ur[e], c = uc[e];
                nx[e] = lds_dot(Xm, Xm, m, r, c) - lds_dot(Ym, Ym, m, r, c);
                ny[e] = 2.0 * lds_dot(Xm, Ym, m, r, c);
            }
        }
        __syncthreads();
        for (int e = 0; e < kExpmUpper; ++e) {
            if (tid + e * kBlock < nut) {
                const int a = ur[e] * m + uc[e], b = uc[e] * m + ur[e];
                Xm[a] = Xm[b] = nx[e];
                Ym[a] = Ym[b] = ny[e];
            }
        }
        __syncthreads();
    }
    // c_k = ||F|| scale_k (X[k][0] - i Y[k][0])
    if (tid < m) {
        const double f = sc.norm0 * sc.scale[tid];
        sc.coef[2 * tid] = f * Xm[tid * m];
        sc.coef[2 * tid + 1] = -f * Ym[tid * m];
    }
}

// F <- sum_k coef_k stored_k  (stored_0 is F itself: read before written).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_lz_recombine(SweepGeom g, typename Stor<T>::aptr psi, typename Stor<T>::cptr basis, int64_t stride,
               const LanczosScalars* __restrict__ scs)
{
    const Tile I = my_tile(g);
    const Tile& tile = I;
    const LanczosScalars& sc = scs[tile.inst];
    const int i = tile.r0 + (int)threadIdx.x;
    if (i >= I.n) return;
    const int m = sc.meff;
    for (int l = tile.l0; l < tile.l1; ++l) {
        const int64_t k = I.off + (int64_t)l * I.n + i;
        double2 v = zero2();
        for (int q = 0; q < m; ++q) {
            const double cr = sc.coef[2 * q], ci = sc.coef[2 * q + 1];
            const double2 b = ldc(basis_vec(cview(psi), basis, stride, q), k);
            v.x = fma(cr, b.x, fma(-ci, b.y, v.x));
            v.y = fma(cr, b.y, fma(ci, b.x, v.y));
        }
        stc_keep(psi, k, v);
    }
}

// ---------------------------------------------------------------------------
// The diffusion (imaginary-time) step's renormalisation (Sec. 4, ground state
// calculation; eq. e_g): the norm of the step's output from the lz_norm
// partials, the energy estimate -ln(n2) / (2 dtau), and the scale 1/sqrt(n2).
__global__ void __launch_bounds__(kBlock)
k_imag_finish(SweepGeom g, const double* __restrict__ partial, const double* __restrict__ step, int record,
              double* __restrict__ energy, int64_t e_stride, int64_t e_index, LanczosScalars* __restrict__ scs)
{
    __shared__ double lds[kBlock / 64];
    const int k = blockIdx.x;
    const Inst& I = g.inst[k];
    const double s = instance_sum<1>(I, partial, 1, 1, lds);
    if (threadIdx.x == 0) {
        const double n2 = I.dr * s;
        scs[k].norm0 = 1.0 / sqrt(n2);
        if (record && energy)
            energy[(int64_t)k * e_stride + e_index] = -log(n2) / (2.0 * step_value(step, g.n_inst, kDt, k));
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_imag_scale(SweepGeom g, typename Stor<T>::cptr src, typename Stor<T>::ptr dst, const LanczosScalars* __restrict__ scs)
{
    const Tile I = my_tile(g);
    const int i = I.r0 + (int)threadIdx.x;
    if (i >= I.n) return;
    const double f = scs[I.inst].norm0;
    for (int l = I.l0; l < I.l1; ++l) {
        const int64_t k = I.off + (int64_t)l * I.n + i;
        const double2 v = ldc(src, k);
        stc(dst, k, make_double2(f * v.x, f * v.y));
    }
}

hipError_t launch_imag_finish(const SweepGeom& g, const double* partial, const double* step, int record,
                              double* energy, int64_t e_stride, int64_t e_index, LanczosScalars* sc,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_imag_finish, dim3(g.n_inst), dim3(kBlock), 0, st, g, partial, step, record, energy,
                       e_stride, e_index, sc);
    return hipGetLastError();
}

template <typename T>
static hipError_t imag_scale_t(const SweepGeom& g, const void* src, void* dst, const LanczosScalars* sc,
                               hipStream_t st)
{
    hipLaunchKernelGGL((k_imag_scale<T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::cmake(src, g.plane),
                       Stor<T>::make(dst, g.plane), sc);
    return hipGetLastError();
}
hipError_t launch_imag_scale(int prec, const SweepGeom& g, const void* src, void* dst, const LanczosScalars* sc,
                             hipStream_t st)
{
    if (prec == 0) return imag_scale_t<double>(g, src, dst, sc, st);
    if (prec == 2) return imag_scale_t<s48>(g, src, dst, sc, st);
    return imag_scale_t<float>(g, src, dst, sc, st);
}

// ---------------------------------------------------------------------------
// Launchers.  The basis vectors 1..m-1 start at `basis`, vec_stride elements
// apart (with s48 storage, vec_stride is the plane length and the m - 1
// vectors are stored plane by plane, see basis_vec).
template <typename T>
static typename Stor<T>::aptr basis_ptr(const SweepGeom& g, const void* basis, int64_t vec_stride, int m)
{
    if constexpr (std::is_same<T, s48>::value) {
        char* b = static_cast<char*>(const_cast<void*>(basis));
        return P48{reinterpret_cast<uint2*>(b), reinterpret_cast<unsigned*>(b + 8 * vec_stride * (int64_t)max(m - 1, 0))};
    } else {
        (void)g, (void)vec_stride, (void)m;
        return static_cast<typename Cplx<T>::type*>(const_cast<void*>(basis));
    }
}

template <typename T>
static hipError_t lz_norm_t(const SweepGeom& g, const void* psi, double* partial, hipStream_t st)
{
    hipLaunchKernelGGL((k_lz_norm<T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::cmake(psi, g.plane),
                       partial);
    return hipGetLastError();
}
hipError_t launch_lz_norm(int prec, const SweepGeom& g, const void* psi, double* partial,
                          hipStream_t st)
{
    if (prec == 0) return lz_norm_t<double>(g, psi, partial, st);
    if (prec == 2) return lz_norm_t<s48>(g, psi, partial, st);
    return lz_norm_t<float>(g, psi, partial, st);
}

hipError_t launch_lz_norm_finish(const SweepGeom& g, const double* partial, LanczosScalars* sc,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(k_lz_norm_finish, dim3(g.n_inst), dim3(kBlock), 0, st, g, partial, sc);
    return hipGetLastError();
}

template <int S, typename T>
static hipError_t sweep_a_t(const SweepGeom& g, int j, int m, const void* psi, const void* basis,
                            int64_t stride, void* w, const double* step, const LanczosScalars* sc,
                            double* partial, hipStream_t st)
{
    if (g.gauge != 0)
        hipLaunchKernelGGL((k_lz_sweep_a<S, T, true>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, j, m,
                           Stor<T>::cmake(psi, g.plane), basis_ptr<T>(g, basis, stride, m), stride,
                           Stor<T>::make(w, g.plane), step, sc, partial);
    else
        hipLaunchKernelGGL((k_lz_sweep_a<S, T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, j, m,
                           Stor<T>::cmake(psi, g.plane), basis_ptr<T>(g, basis, stride, m), stride,
                           Stor<T>::make(w, g.plane), step, sc, partial);
    return hipGetLastError();
}

hipError_t launch_lz_sweep_a(int prec, int S, const SweepGeom& g, int j, int m, const void* psi,
                             const void* basis, int64_t vec_stride, void* w, const double* step,
                             const LanczosScalars* sc, double* partial, hipStream_t st)
{
    if (prec == 0)
        return S == 1 ? sweep_a_t<1, double>(g, j, m, psi, basis, vec_stride, w, step, sc, partial, st)
                      : sweep_a_t<2, double>(g, j, m, psi, basis, vec_stride, w, step, sc, partial, st);
    if (prec == 2)
        return S == 1 ? sweep_a_t<1, s48>(g, j, m, psi, basis, vec_stride, w, step, sc, partial, st)
                      : sweep_a_t<2, s48>(g, j, m, psi, basis, vec_stride, w, step, sc, partial, st);
    return S == 1 ? sweep_a_t<1, float>(g, j, m, psi, basis, vec_stride, w, step, sc, partial, st)
                  : sweep_a_t<2, float>(g, j, m, psi, basis, vec_stride, w, step, sc, partial, st);
}

hipError_t launch_lz_finish_a(const SweepGeom& g, int j, int m, const double* partial,
                              LanczosScalars* sc, hipStream_t st)
{
    constexpr int JB = 8;
    hipLaunchKernelGGL(k_lz_finish_a, dim3(g.n_inst, (j + JB) / JB), dim3(kBlock), 0, st, g, j, m, partial, sc);
    return hipGetLastError();
}

template <typename T>
static hipError_t sweep_b_t(const SweepGeom& g, int j, int m, const void* psi, const void* basis, int64_t stride,
                            const void* w, const LanczosScalars* sc, double* partial, hipStream_t st)
{
    hipLaunchKernelGGL((k_lz_sweep_b<T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, j, Stor<T>::cmake(psi, g.plane),
                       basis_ptr<T>(g, basis, stride, m), stride, Stor<T>::cmake(w, g.plane), sc, partial);
    return hipGetLastError();
}
hipError_t launch_lz_sweep_b(int prec, const SweepGeom& g, int j, int m, const void* psi,
                             const void* basis, int64_t vec_stride, const void* w,
                             const LanczosScalars* sc, double* partial, hipStream_t st)
{
    if (prec == 0) return sweep_b_t<double>(g, j, m, psi, basis, vec_stride, w, sc, partial, st);
    if (prec == 2) return sweep_b_t<s48>(g, j, m, psi, basis, vec_stride, w, sc, partial, st);
    return sweep_b_t<float>(g, j, m, psi, basis, vec_stride, w, sc, partial, st);
}

hipError_t launch_lz_finish_b(const SweepGeom& g, int j, const double* partial,
                              LanczosScalars* sc, hipStream_t st)
{
    hipLaunchKernelGGL(k_lz_finish_b, dim3(g.n_inst), dim3(kBlock), 0, st, g, j, partial, sc);
    return hipGetLastError();
}

__global__ void k_lz_reset(int n_inst, int m, LanczosScalars* __restrict__ scs)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < n_inst) scs[k].meff_min = m;
}

hipError_t launch_lz_reset(const SweepGeom& g, int m, LanczosScalars* sc, hipStream_t st)
{
    hipLaunchKernelGGL(k_lz_reset, dim3((g.n_inst + kBlock - 1) / kBlock), dim3(kBlock), 0, st, g.n_inst, m, sc);
    return hipGetLastError();
}

hipError_t launch_lz_expm(const SweepGeom& g, const double* step, LanczosScalars* sc,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_lz_expm, dim3(g.n_inst), dim3(kBlock), 0, st, g, step, sc);
    return hipGetLastError();
}

template <typename T>
static hipError_t recombine_t(const SweepGeom& g, int m, void* psi, const void* basis, int64_t stride,
                              const LanczosScalars* sc, hipStream_t st)
{
    hipLaunchKernelGGL((k_lz_recombine<T>), dim3(g.n_tiles), dim3(kBlock), 0, st, g, Stor<T>::make(psi, g.plane),
                       basis_ptr<T>(g, basis, stride, m), stride, sc);
    return hipGetLastError();
}
hipError_t launch_lz_recombine(int prec, const SweepGeom& g, int m, void* psi, const void* basis,
                               int64_t vec_stride, const LanczosScalars* sc, hipStream_t st)
{
    if (prec == 0) return recombine_t<double>(g, m, psi, basis, vec_stride, sc, st);
    if (prec == 2) return recombine_t<s48>(g, m, psi, basis, vec_stride, sc, st);
    return recombine_t<float>(g, m, psi, basis, vec_stride, sc, st);
}

}  // namespace tdse
