// Host FP64 eigenvectors of the field-free radial blocks h_l (Sec. 2,
// eq. tdse-radial-field on the finite-difference grid): a real symmetric
// banded N x N matrix with half-bandwidth s = 1 (3-point) or 2 (5-point).
//
// The k lowest eigenvalues are isolated by bisection on the inertia of
// h_l - sigma I (Sylvester: the number of negative pivots of its banded
// LDL^T factorisation counts the eigenvalues below sigma); each eigenvector
// then follows from three steps of inverse iteration with a banded LU
// factorisation with partial pivoting.  Used once at context creation for the
// bound-state populations; the time stepping never calls it.
#include "host_eigen.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

namespace tdse {

namespace {

struct Band {
    int n, s;
    std::vector<double> diag;     // main diagonal
    double off[3];                // off[1], off[2]: constant off-diagonals
};

Band radial_band(int n, int stencil, double dr, double z, int l)
{
    Band b;
    b.n = n;
    b.s = (stencil == 3) ? 1 : 2;
    const double h2 = dr * dr;
    double d0;
    if (stencil == 3) {
        d0 = 1.0 / h2;
        b.off[1] = -0.5 / h2;
        b.off[2] = 0.0;
    } else {
        d0 = 30.0 / (24.0 * h2);
        b.off[1] = -16.0 / (24.0 * h2);
        b.off[2] = 1.0 / (24.0 * h2);
    }
    b.off[0] = 0.0;
    b.diag.resize(n);
    for (int i = 0; i < n; ++i) {
        const double r = (double)(i + 1) * dr;
        b.diag[i] = d0 + 0.5 * (double)l * (double)(l + 1) / (r * r) - z / r;
    }
    return b;
}

// Number of eigenvalues of B below sigma (negative pivots of LDL^T of B - sigma I).
int count_below(const Band& B, double sigma)
{
    const double tiny = 1e-300;
    int neg = 0;
    if (B.s == 1) {
        double d = 0.0;
        const double b1 = B.off[1];
        for (int i = 0; i < B.n; ++i) {
            d = (B.diag[i] - sigma) - ((i > 0) ? b1 * b1 / d : 0.0);
            if (d == 0.0) d = -tiny;
            if (d < 0.0) ++neg;
        }
        return neg;
    }
    // half-bandwidth 2: A = L D L^T, L unit lower with two sub-diagonals
    double d1 = 0.0, d2 = 0.0;      // d_{i-1}, d_{i-2}
    double l21 = 0.0;               // L(i-1, i-2)
    const double a1 = B.off[1], a2 = B.off[2];
    for (int i = 0; i < B.n; ++i) {
        const double li2 = (i >= 2) ? a2 / d2 : 0.0;                       // L(i, i-2)
        const double li1 = (i >= 1) ? (a1 - ((i >= 2) ? li2 * d2 * l21 : 0.0)) / d1 : 0.0;  // L(i, i-1)
        double d = (B.diag[i] - sigma) - ((i >= 1) ? li1 * li1 * d1 : 0.0) - ((i >= 2) ? li2 * li2 * d2 : 0.0);
        if (d == 0.0) d = -tiny;
        if (d < 0.0) ++neg;
        d2 = d1;
        d1 = d;
        l21 = li1;
    }
    return neg;
}

// Banded LU with partial pivoting of B - sigma I (storage of columns with
// kl = s sub-diagonals and up to 2s super-diagonals after fill-in).
struct BandLU {
    int n, kl, ku;               // ku includes fill-in
    std::vector<double> ab;      // (2 kl + ku0 + 1) x n, column-major band
    std::vector<int> piv;
    int ld;
    double& at(int i, int j) { return ab[(size_t)j * ld + (ku + i - j)]; }

    void factor(const Band& B, double sigma)
    {
        n = B.n;
        kl = B.s;
        ku = 2 * B.s;
        ld = kl + ku + 1;
        ab.assign((size_t)ld * n, 0.0);
        piv.assign(n, 0);
        for (int j = 0; j < n; ++j) {
            for (int i = std::max(0, j - B.s); i <= std::min(n - 1, j + B.s); ++i) {
                const int d = std::abs(i - j);
                at(i, j) = (d == 0) ? B.diag[i] - sigma : B.off[d];
            }
        }
        double scale = 0.0;
        for (int i = 0; i < n; ++i) scale = std::max(scale, std::fabs(B.diag[i] - sigma));
        scale = std::max(scale, std::fabs(B.off[1]) + std::fabs(B.off[2]));
        const double floor = std::numeric_limits<double>::epsilon() * scale;
        for (int j = 0; j < n; ++j) {
            const int last = std::min(n - 1, j + kl);
            int p = j;
            for (int i = j + 1; i <= last; ++i)
                if (std::fabs(at(i, j)) > std::fabs(at(p, j))) p = i;
            piv[j] = p;
            const int cend = std::min(n - 1, j + ku);
            if (p != j)
                for (int c = j; c <= cend; ++c) std::swap(at(p, c), at(j, c));
            if (std::fabs(at(j, j)) < floor) at(j, j) = (at(j, j) < 0.0) ? -floor : floor;
            const double inv = 1.0 / at(j, j);
            for (int i = j + 1; i <= last; ++i) at(i, j) *= inv;
            for (int c = j + 1; c <= cend; ++c) {
                const double u = at(j, c);
                if (u == 0.0) continue;
                for (int i = j + 1; i <= last; ++i) at(i, c) -= at(i, j) * u;
            }
        }
    }

    void solve(std::vector<double>& x)
    {
        for (int j = 0; j < n; ++j) {
            if (piv[j] != j) std::swap(x[j], x[piv[j]]);
            const int last = std::min(n - 1, j + kl);
            for (int i = j + 1; i <= last; ++i) x[i] -= at(i, j) * x[j];
        }
        for (int j = n - 1; j >= 0; --j) {
            x[j] /= at(j, j);
            const int first = std::max(0, j - ku);
            for (int i = first; i < j; ++i) x[i] -= at(i, j) * x[j];
        }
    }
};

}  // namespace

void lowest_radial_states(int n, int stencil, double dr, double z, int l, int count,
                          std::vector<double>& energies, std::vector<double>& vectors)
{
    const Band B = radial_band(n, stencil, dr, z, l);
    double lo = std::numeric_limits<double>::max(), hi = -lo;
    const double offsum = 2.0 * (std::fabs(B.off[1]) + std::fabs(B.off[2]));
    for (int i = 0; i < n; ++i) {
        lo = std::min(lo, B.diag[i] - offsum);
        hi = std::max(hi, B.diag[i] + offsum);
    }
    energies.assign(count, 0.0);
    vectors.assign((size_t)count * n, 0.0);
    BandLU lu;
    for (int k = 0; k < count; ++k) {
        // bisection for the k-th lowest eigenvalue: count_below(a) <= k < count_below(b)
        double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (a + b);
            if (count_below(B, mid) > k) b = mid; else a = mid;
            if (b - a <= 1e-10 * std::max(std::fabs(a), std::fabs(b))) break;
        }
        const double sigma = 0.5 * (a + b);
        lu.factor(B, sigma);
        std::vector<double> x(n);
        for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.25 * std::sin(0.37 * (double)i);
        for (int it = 0; it < 3; ++it) {
            lu.solve(x);
            double nrm = 0.0;
            for (double v : x) nrm += v * v;
            nrm = std::sqrt(nrm);
            for (double& v : x) v /= nrm;
        }
        // Rayleigh quotient for the energy; normalise dr * sum phi^2 = 1 with
        // the largest component positive
        double num = 0.0, den = 0.0;
        for (int i = 0; i < n; ++i) {
            double hx = B.diag[i] * x[i];
            for (int d = 1; d <= B.s; ++d) {
                if (i - d >= 0) hx += B.off[d] * x[i - d];
                if (i + d < n) hx += B.off[d] * x[i + d];
            }
            num += x[i] * hx;
            den += x[i] * x[i];
        }
        energies[k] = num / den;
        int imax = 0;
        for (int i = 1; i < n; ++i)
            if (std::fabs(x[i]) > std::fabs(x[imax])) imax = i;
        const double sgn = (x[imax] < 0.0) ? -1.0 : 1.0;
        const double norm = sgn / std::sqrt(dr * den);
        for (int i = 0; i < n; ++i) vectors[(size_t)k * n + i] = x[i] * norm;
    }
}

}  // namespace tdse
