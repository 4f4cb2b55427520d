/*
 * Plain FP64 CPU oracle for the finite-difference TDSE of arXiv:1308.1856.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg to check the GPU library; never by the product
 * path.  Deliberately slow and literal: loops over l then r, no blocking, no
 * fusion, no SIMD, built with -ffp-contract=off.  Every function follows the
 * passage of the paper named in its comment.
 */
#include "tdse_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Threads: the loops over partial waves of H f and the element-wise vector
 * updates may run on several OpenMP threads (each element is computed by one
 * thread with the same operations, so the results do not depend on the
 * thread count); every sum over elements (norms, inner products, observables)
 * runs on one thread in index order. */
static int default_threads = 1;
/* At load: remember the OpenMP default (OMP_NUM_THREADS, else the cores) and
 * run on one thread until told otherwise (the tests call the oracle on small
 * grids, where thread start-up costs more than the loops). */
__attribute__((constructor)) static void orc_threads_init(void)
{
    default_threads = omp_get_max_threads();
    omp_set_num_threads(1);
}
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return default_threads; }

/* Sec. 2, grid definition: uniform points, the first one a spacing away from
 * the origin ("Start = 1"), optionally displaced by the "Offset" setting. */
double orc_radius(const orc_grid* g, int i) { return (double)(i + 1) * g->dr + g->r_shift; }

/* Sec. 2, angular coupling k_{l,l'}(m) for m = 0 and l_> = l:
 * kappa_l = sqrt(l^2 / (4 l^2 - 1)). */
double orc_kappa(int l)
{
    if (l <= 0) return 0.0;
    double ll = (double)l;
    return sqrt(ll * ll / (4.0 * ll * ll - 1.0));
}

/* Sec. 3, field with the Hann (sine-squared) envelope: E0 f(tau) cos(w tau +
 * phi), f = sin^2(pi tau / T), T = 2 pi n_c / w, zero outside the pulse.
 * Shape 1 ("SineA" of Sec. 3, eq. VecSinSinCosE): the envelope sits on the
 * vector potential, A/c = -E0 sin^2(W tau) sin(w tau + phi) with W = pi / T,
 * and E = -d(A/c)/dt = E0 sin(W tau) [w sin(W tau) cos(w tau + phi)
 * + 2 W cos(W tau) sin(w tau + phi)]. */
double orc_field(const orc_pulse* p, double t)
{
    double tau = t - p->t_on;
    double period = 2.0 * M_PI * p->n_cycles / p->omega;
    if (!(tau >= 0.0 && tau <= period)) return 0.0;
    double s = sin(M_PI * tau / period);
    if (p->shape == 1) {
        const double w_env = M_PI / period;
        const double c = cos(M_PI * tau / period);
        return p->e0 * s * (p->omega * s * cos(p->omega * tau + p->cep) + 2.0 * w_env * c * sin(p->omega * tau + p->cep));
    }
    return p->e0 * s * s * cos(p->omega * tau + p->cep);
}

/* 5-point Gauss-Legendre rule on [-1, 1] (nodes: 0 and the roots
 * +-(1/3) sqrt(5 -+ 2 sqrt(10/7)) of P_5; weights 128/225 and
 * (322 +- 13 sqrt(70)) / 900), nodes in increasing order. */
static void gauss_legendre5(double x[5], double w[5])
{
    const double a = sqrt(5.0 - 2.0 * sqrt(10.0 / 7.0)) / 3.0;
    const double b = sqrt(5.0 + 2.0 * sqrt(10.0 / 7.0)) / 3.0;
    const double wa = (322.0 + 13.0 * sqrt(70.0)) / 900.0;
    const double wb = (322.0 - 13.0 * sqrt(70.0)) / 900.0;
    x[0] = -b; x[1] = -a; x[2] = 0.0; x[3] = a; x[4] = b;
    w[0] = wb; w[1] = wa; w[2] = 128.0 / 225.0; w[3] = wa; w[4] = wb;
}

double orc_vector_potential_step(const orc_pulse* p, double t, double h)
{
    double x[5], w[5];
    gauss_legendre5(x, w);
    double sum = 0.0;
    for (int j = 0; j < 5; ++j) sum += w[j] * orc_field(p, t + 0.5 * h * (1.0 + x[j]));
    return -0.5 * h * sum;
}

double orc_vector_potential_at(const orc_pulse* p, double t0, double dt)
{
    if (!(t0 > p->t_on)) return 0.0;
    const double span = t0 - p->t_on;
    int64_t m = (int64_t)ceil(span / dt - 1e-9);
    if (m < 1) m = 1;
    const double piece = span / (double)m;
    double a = 0.0;
    for (int64_t q = 0; q < m; ++q) a += orc_vector_potential_step(p, p->t_on + (double)q * piece, piece);
    return a;
}

static double complex value_at(const orc_grid* g, const double complex* row, int i)
{
    /* Sec. 2.1: the finite-difference terms beyond the box edges are zero */
    if (i < 0 || i >= g->n) return 0.0;
    return row[i];
}

/* First radial derivative of a row at point i, of the stencil's order: the
 * central difference (f_{i+1} - f_{i-1}) / (2 dr) with the 3-point Laplacian,
 * the fourth-order (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2}) / (12 dr) of
 * Sec. 2 with the 5-point one (its printed 1/(12 h^2) read as 1/(12 h)). */
static double complex first_derivative(const orc_grid* g, const double complex* f, int i)
{
    if (g->stencil == 3) return (value_at(g, f, i + 1) - value_at(g, f, i - 1)) / (2.0 * g->dr);
    return (value_at(g, f, i - 2) - 8.0 * value_at(g, f, i - 1) + 8.0 * value_at(g, f, i + 1)
            - value_at(g, f, i + 2)) / (12.0 * g->dr);
}

/* H(t) f (Sec. 2, radial TDSE in the L and V gauges, with the field-free
 * block h_l and the matrix layout of eq. h_matrix):
 *   (H f)_l = -1/2 D2 f_l + [l(l+1)/(2 r^2) - z/r] f_l + coupling,
 * length gauge (g->gauge 0, `field` = E):
 *   coupling = E r [kappa_l f_{l-1} + kappa_{l+1} f_{l+1}],
 * velocity gauge (g->gauge 1, `field` = A~ = A/c):
 *   coupling = -i A~ [kappa_l (d/dr - l/r) f_{l-1}
 *                     + kappa_{l+1} (d/dr + (l+1)/r) f_{l+1}],
 * the partial-wave form of A~ p_z on f_l / r (the signs of the l/r terms as
 * p_z acting on (f/r) Y_l0 gives them; the paper prints them the other way
 * round).  D2 is the 3-point second difference or the 5-point fourth-order
 * formula of Sec. 2, d/dr the first derivative of the same order. */
void orc_apply_h(const orc_grid* g, double efield, const double complex* f, double complex* hf)
{
    const int n = g->n;
    const double h2 = g->dr * g->dr;
#pragma omp parallel for schedule(static)
    for (int l = 0; l <= g->lmax; ++l) {
        const double complex* fl = f + (size_t)l * n;
        const double complex* flm = (l > 0) ? f + (size_t)(l - 1) * n : NULL;
        const double complex* flp = (l < g->lmax) ? f + (size_t)(l + 1) * n : NULL;
        const double kl = orc_kappa(l);
        const double klp = orc_kappa(l + 1);
        const double centrifugal = 0.5 * (double)l * (double)(l + 1);
        for (int i = 0; i < n; ++i) {
            double complex d2;
            if (g->stencil == 3) {
                d2 = (value_at(g, fl, i + 1) - 2.0 * fl[i] + value_at(g, fl, i - 1)) / h2;
            } else {
                d2 = (-value_at(g, fl, i + 2) + 16.0 * value_at(g, fl, i + 1) - 30.0 * fl[i]
                      + 16.0 * value_at(g, fl, i - 1) - value_at(g, fl, i - 2))
                     / (12.0 * h2);
            }
            const double r = orc_radius(g, i);
            const double v = centrifugal / (r * r) - g->z / r;
            double complex coupling = 0.0;
            if (g->gauge == 1) {
                if (flm) coupling += kl * (first_derivative(g, flm, i) - ((double)l / r) * flm[i]);
                if (flp) coupling += klp * (first_derivative(g, flp, i) + ((double)(l + 1) / r) * flp[i]);
                hf[(size_t)l * n + i] = -0.5 * d2 + v * fl[i] + (-I * efield) * coupling;
            } else {
                if (flm) coupling += kl * flm[i];
                if (flp) coupling += klp * flp[i];
                hf[(size_t)l * n + i] = -0.5 * d2 + v * fl[i] + efield * r * coupling;
            }
        }
    }
}

/* Gershgorin bound on the spectral radius of H(E) (length gauge; H(A~) in
 * the velocity gauge): the largest absolute row sum of the matrix of eq.
 * h_matrix.  Used as the scale of the Lanczos breakdown test and of the
 * explicit-step stability limit. */
double orc_h_bound(const orc_grid* g, double efield)
{
    const double h2 = g->dr * g->dr;
    const double diag_kin = (g->stencil == 3) ? 1.0 / h2 : 30.0 / (24.0 * h2);
    const double off_kin = (g->stencil == 3) ? 1.0 / h2 : (32.0 + 2.0) / (24.0 * h2);
    const double d1 = (g->stencil == 3) ? 1.0 / g->dr : 18.0 / (12.0 * g->dr);   /* sum |first-derivative weights| */
    double bound = 0.0;
    for (int l = 0; l <= g->lmax; ++l) {
        const double klm = orc_kappa(l), klp = (l < g->lmax) ? orc_kappa(l + 1) : 0.0;
        const double coup = klm + klp;
        for (int i = 0; i < g->n; ++i) {
            const double r = orc_radius(g, i);
            const double d = diag_kin + 0.5 * (double)l * (double)(l + 1) / (r * r) - g->z / r;
            const double cpl = (g->gauge == 1) ? fabs(efield) * (klm * (d1 + (double)l / r) + klp * (d1 + (double)(l + 1) / r))
                                               : fabs(efield) * r * coup;
            const double row = fabs(d) + off_kin + cpl;
            if (row > bound) bound = row;
        }
    }
    return bound;
}

static size_t state_len(const orc_grid* g) { return (size_t)(g->lmax + 1) * (size_t)g->n; }

/* Sec. 5.2 (Taylor.c), eq. Taylor with the recurrence divisor read as p+1:
 *   F_{n+1} = sum_{p=0..P} F^(p),  F^(0) = F_n,  F^(p+1) = (-i dt/(p+1)) H F^(p)
 * H is frozen at the field value passed in (the step midpoint). */
void orc_taylor_step(const orc_grid* g, double efield, double dt, int order, double complex* psi)
{
    const size_t len = state_len(g);
    double complex* term = malloc(len * sizeof *term);
    double complex* next = malloc(len * sizeof *next);
    memcpy(term, psi, len * sizeof *term);
    for (int p = 0; p < order; ++p) {
        orc_apply_h(g, efield, term, next);
        const double complex factor = -I * dt / (double)(p + 1);
#pragma omp parallel for schedule(static)
        for (size_t k = 0; k < len; ++k) {
            term[k] = factor * next[k];
            psi[k] += term[k];
        }
    }
    free(term);
    free(next);
}

/* Sec. 5.2 (RungeKutta.c), eq. RKDeriv with the classic fourth-order tableau
 * (c = 0, 1/2, 1/2, 1; b = 1/6, 1/3, 1/3, 1/6) applied to dF/dt = -i H(t) F
 * (eq. tdse_matrix).  The field values at the stage times are passed in. */
static void rk4_step_fields(const orc_grid* g, double e_start, double e_mid, double e_end,
                            double dt, double complex* psi)
{
    const size_t len = state_len(g);
    double complex* k = malloc(len * sizeof *k);
    double complex* y = malloc(len * sizeof *y);
    double complex* acc = malloc(len * sizeof *acc);
    const double a[4] = {0.0, 0.5, 0.5, 1.0};
    const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double e[4] = {e_start, e_mid, e_mid, e_end};
    memcpy(acc, psi, len * sizeof *acc);
    memcpy(y, psi, len * sizeof *y);
    for (int s = 0; s < 4; ++s) {
        if (s > 0) {
#pragma omp parallel for schedule(static)
            for (size_t j = 0; j < len; ++j) y[j] = psi[j] + a[s] * dt * k[j];
        }
        orc_apply_h(g, e[s], y, k);
#pragma omp parallel for schedule(static)
        for (size_t j = 0; j < len; ++j) {
            k[j] = -I * k[j];
            acc[j] += b[s] * dt * k[j];
        }
    }
    memcpy(psi, acc, len * sizeof *acc);
    free(k);
    free(y);
    free(acc);
}

/* The coupling scalar of the gauge at time t_n + frac dt inside the step
 * starting at t_n: E(t_lg) in the length gauge (t_lg that time as the caller
 * forms it), A~(t_n) - int_{t_n}^{t_n + frac dt} E in the velocity gauge
 * (a_n = A~(t_n); eq. VectorStep applied from the step start to each stage
 * time, as the appendix describes for the Runge-Kutta stages). */
static double coupling_at(const orc_grid* g, const orc_pulse* p, double t_n, double a_n, double frac, double dt,
                          double t_lg)
{
    if (g->gauge == 1) return a_n + orc_vector_potential_step(p, t_n, frac * dt);
    return orc_field(p, t_lg);
}

static double start_potential(const orc_grid* g, const orc_pulse* p, double t0, double dt)
{
    return (g->gauge == 1) ? orc_vector_potential_at(p, t0, dt) : 0.0;
}

void orc_rk4_step(const orc_grid* g, const orc_pulse* p, double t, double dt, double complex* psi)
{
    const double a = start_potential(g, p, t, dt);
    rk4_step_fields(g, coupling_at(g, p, t, a, 0.0, dt, t), coupling_at(g, p, t, a, 0.5, dt, t + 0.5 * dt),
                    coupling_at(g, p, t, a, 1.0, dt, t + dt), dt, psi);
}

/* Appendix "Runge-Kutta" and Sec. 5.2 (RungeKutta.c, eq. RKDeriv): explicit
 * Runge-Kutta methods given by their Butcher tableaux, the published ones:
 * Euler; the classic fourth-order method; Fehlberg's 4(5) pair; the
 * Cash-Karp 5(4) pair; the Dormand-Prince 5(4) pair; Merson's 4(3) method.
 * b: the weights of the solution carried forward (the higher order of a
 * pair); bhat: the weights of the embedded solution of the other order
 * (zero rows for the methods without one). */
int orc_rk_tableau(int method, double* c, double* a /* [ORC_RK_MAX][ORC_RK_MAX] */, double* b, double* bhat)
{
    const int M = ORC_RK_MAX;
    for (int i = 0; i < M; ++i) {
        c[i] = b[i] = bhat[i] = 0.0;
        for (int j = 0; j < M; ++j) a[i * M + j] = 0.0;
    }
#define A_(i, j, v) a[(i) * M + (j)] = (v)
    switch (method) {
    case ORC_RK_EULER:
        b[0] = 1.0;
        return 1;
    case ORC_RK_CLASSIC4:
        c[1] = 0.5; c[2] = 0.5; c[3] = 1.0;
        A_(1, 0, 0.5); A_(2, 1, 0.5); A_(3, 2, 1.0);
        b[0] = 1.0 / 6.0; b[1] = 1.0 / 3.0; b[2] = 1.0 / 3.0; b[3] = 1.0 / 6.0;
        return 4;
    case ORC_RK_FEHLBERG45:
        c[1] = 1.0 / 4.0; c[2] = 3.0 / 8.0; c[3] = 12.0 / 13.0; c[4] = 1.0; c[5] = 1.0 / 2.0;
        A_(1, 0, 1.0 / 4.0);
        A_(2, 0, 3.0 / 32.0); A_(2, 1, 9.0 / 32.0);
        A_(3, 0, 1932.0 / 2197.0); A_(3, 1, -7200.0 / 2197.0); A_(3, 2, 7296.0 / 2197.0);
        A_(4, 0, 439.0 / 216.0); A_(4, 1, -8.0); A_(4, 2, 3680.0 / 513.0); A_(4, 3, -845.0 / 4104.0);
        A_(5, 0, -8.0 / 27.0); A_(5, 1, 2.0); A_(5, 2, -3544.0 / 2565.0); A_(5, 3, 1859.0 / 4104.0);
        A_(5, 4, -11.0 / 40.0);
        b[0] = 16.0 / 135.0; b[2] = 6656.0 / 12825.0; b[3] = 28561.0 / 56430.0; b[4] = -9.0 / 50.0;
        b[5] = 2.0 / 55.0;
        bhat[0] = 25.0 / 216.0; bhat[2] = 1408.0 / 2565.0; bhat[3] = 2197.0 / 4104.0; bhat[4] = -1.0 / 5.0;
        return 6;
    case ORC_RK_CASHKARP:
        c[1] = 1.0 / 5.0; c[2] = 3.0 / 10.0; c[3] = 3.0 / 5.0; c[4] = 1.0; c[5] = 7.0 / 8.0;
        A_(1, 0, 1.0 / 5.0);
        A_(2, 0, 3.0 / 40.0); A_(2, 1, 9.0 / 40.0);
        A_(3, 0, 3.0 / 10.0); A_(3, 1, -9.0 / 10.0); A_(3, 2, 6.0 / 5.0);
        A_(4, 0, -11.0 / 54.0); A_(4, 1, 5.0 / 2.0); A_(4, 2, -70.0 / 27.0); A_(4, 3, 35.0 / 27.0);
        A_(5, 0, 1631.0 / 55296.0); A_(5, 1, 175.0 / 512.0); A_(5, 2, 575.0 / 13824.0);
        A_(5, 3, 44275.0 / 110592.0); A_(5, 4, 253.0 / 4096.0);
        b[0] = 37.0 / 378.0; b[2] = 250.0 / 621.0; b[3] = 125.0 / 594.0; b[5] = 512.0 / 1771.0;
        bhat[0] = 2825.0 / 27648.0; bhat[2] = 18575.0 / 48384.0; bhat[3] = 13525.0 / 55296.0;
        bhat[4] = 277.0 / 14336.0; bhat[5] = 1.0 / 4.0;
        return 6;
    case ORC_RK_DORMANDPRINCE:
        c[1] = 1.0 / 5.0; c[2] = 3.0 / 10.0; c[3] = 4.0 / 5.0; c[4] = 8.0 / 9.0; c[5] = 1.0; c[6] = 1.0;
        A_(1, 0, 1.0 / 5.0);
        A_(2, 0, 3.0 / 40.0); A_(2, 1, 9.0 / 40.0);
        A_(3, 0, 44.0 / 45.0); A_(3, 1, -56.0 / 15.0); A_(3, 2, 32.0 / 9.0);
        A_(4, 0, 19372.0 / 6561.0); A_(4, 1, -25360.0 / 2187.0); A_(4, 2, 64448.0 / 6561.0);
        A_(4, 3, -212.0 / 729.0);
        A_(5, 0, 9017.0 / 3168.0); A_(5, 1, -355.0 / 33.0); A_(5, 2, 46732.0 / 5247.0); A_(5, 3, 49.0 / 176.0);
        A_(5, 4, -5103.0 / 18656.0);
        A_(6, 0, 35.0 / 384.0); A_(6, 2, 500.0 / 1113.0); A_(6, 3, 125.0 / 192.0); A_(6, 4, -2187.0 / 6784.0);
        A_(6, 5, 11.0 / 84.0);
        b[0] = 35.0 / 384.0; b[2] = 500.0 / 1113.0; b[3] = 125.0 / 192.0; b[4] = -2187.0 / 6784.0;
        b[5] = 11.0 / 84.0;
        bhat[0] = 5179.0 / 57600.0; bhat[2] = 7571.0 / 16695.0; bhat[3] = 393.0 / 640.0;
        bhat[4] = -92097.0 / 339200.0; bhat[5] = 187.0 / 2100.0; bhat[6] = 1.0 / 40.0;
        return 7;
    case ORC_RK_MERSON:
        c[1] = 1.0 / 3.0; c[2] = 1.0 / 3.0; c[3] = 1.0 / 2.0; c[4] = 1.0;
        A_(1, 0, 1.0 / 3.0);
        A_(2, 0, 1.0 / 6.0); A_(2, 1, 1.0 / 6.0);
        A_(3, 0, 1.0 / 8.0); A_(3, 2, 3.0 / 8.0);
        A_(4, 0, 1.0 / 2.0); A_(4, 2, -3.0 / 2.0); A_(4, 3, 2.0);
        b[0] = 1.0 / 6.0; b[3] = 2.0 / 3.0; b[4] = 1.0 / 6.0;
        bhat[0] = 1.0 / 10.0; bhat[2] = 3.0 / 10.0; bhat[3] = 2.0 / 5.0; bhat[4] = 1.0 / 5.0;
        return 5;
    default:
        return 0;
    }
#undef A_
}

/* One step of the method from psi at t: k_i = -i H(t + c_i dt) g_i with
 * g_i = F_n + dt sum_{j<i} a_ij k_j; F_{n+1} = F_n + dt sum_i b_i k_i.  For a
 * pair, the local deviation Delta = dt sum_i (b_i - bhat_i) k_i gives
 * sigma_n = sqrt(sum_e |Delta_e|^2 / U) over the U elements of the state (the
 * root mean square over the solution vector); returned (0 without a pair). */
static double rk_step_a(const orc_grid* g, const orc_pulse* p, int method, double t, double dt, double a_n,
                        double complex* psi)
{
    const int M = ORC_RK_MAX;
    double c[ORC_RK_MAX], a[ORC_RK_MAX * ORC_RK_MAX], b[ORC_RK_MAX], bh[ORC_RK_MAX];
    const int stages = orc_rk_tableau(method, c, a, b, bh);
    const size_t len = state_len(g);
    double complex* k = malloc((size_t)stages * len * sizeof *k);
    double complex* y = malloc(len * sizeof *y);
    for (int i = 0; i < stages; ++i) {
#pragma omp parallel for schedule(static)
        for (size_t e = 0; e < len; ++e) {
            double complex acc = 0.0;
            for (int j = 0; j < i; ++j) acc += a[i * M + j] * k[(size_t)j * len + e];
            y[e] = psi[e] + dt * acc;
        }
        double complex* ki = k + (size_t)i * len;
        orc_apply_h(g, coupling_at(g, p, t, a_n, c[i], dt, t + c[i] * dt), y, ki);
#pragma omp parallel for schedule(static)
        for (size_t e = 0; e < len; ++e) ki[e] = -I * ki[e];
    }
    double d2 = 0.0;
    for (size_t e = 0; e < len; ++e) {
        double complex acc = 0.0, dev = 0.0;
        for (int i = 0; i < stages; ++i) {
            acc += b[i] * k[(size_t)i * len + e];
            dev += (b[i] - bh[i]) * k[(size_t)i * len + e];
        }
        psi[e] += dt * acc;
        dev *= dt;
        d2 += creal(dev) * creal(dev) + cimag(dev) * cimag(dev);
    }
    free(k);
    free(y);
    int pair = 0;
    for (int i = 0; i < stages; ++i) pair = pair || (bh[i] != 0.0);
    return pair ? sqrt(d2 / (double)len) : 0.0;
}

double orc_rk_step(const orc_grid* g, const orc_pulse* p, int method, double t, double dt,
                   double complex* psi)
{
    return rk_step_a(g, p, method, t, dt, start_potential(g, p, t, dt), psi);
}

/* nsteps steps of method from t0 with observables every obs_every steps (as
 * orc_propagate); returns sigma = sum_n sigma_n, the passive global
 * truncation estimate of the appendix. */
double orc_propagate_rk(const orc_grid* g, const orc_pulse* p, int method, double t0, double dt,
                        int64_t nsteps, int64_t obs_every, double r_ion, const double* u0, int n_states,
                        const int32_t* state_l, const double* phi, double complex* psi, double* obs_out)
{
    const int rec = ORC_OBS_FIXED + n_states;
    int64_t n_obs = 0;
    double sigma = 0.0;
    double a_n = start_potential(g, p, t0, dt);
    for (int64_t s = 0; s < nsteps; ++s) {
        const double t_n = t0 + (double)s * dt;
        sigma += rk_step_a(g, p, method, t_n, dt, a_n, psi);
        if (g->gauge == 1) a_n += orc_vector_potential_step(p, t_n, dt);
        if (obs_every > 0 && (s + 1) % obs_every == 0 && obs_out) {
            orc_observables(g, p, t0 + (double)(s + 1) * dt, r_ion, u0, n_states, state_l, phi, psi,
                            obs_out + (size_t)n_obs * rec);
            ++n_obs;
        }
    }
    return sigma;
}

/* Cyclic-by-row Jacobi method for a dense symmetric matrix (the rotation of
 * Golub & Van Loan, Matrix Computations, Sec. 8.5).  Each rotation zeroes one
 * off-diagonal pair; sweeps repeat until the off-diagonal part vanishes. */
void orc_jacobi_eig(int m, double* a, double* v)
{
#define A(i, j) a[(size_t)(i) * m + (j)]
#define V(i, j) v[(size_t)(i) * m + (j)]
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) V(i, j) = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < m; ++i) {
            diag += A(i, i) * A(i, i);
            for (int j = i + 1; j < m; ++j) off += A(i, j) * A(i, j);
        }
        if (off == 0.0 || off <= 1e-36 * diag) break;
        for (int p = 0; p < m - 1; ++p) {
            for (int q = p + 1; q < m; ++q) {
                const double apq = A(p, q);
                if (apq == 0.0) continue;
                const double tau = (A(q, q) - A(p, p)) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                for (int k = 0; k < m; ++k) { /* A <- A J */
                    const double akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * akq;
                    A(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) { /* A <- J^T A */
                    const double apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * aqk;
                    A(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) { /* V <- V J */
                    const double vkp = V(k, p), vkq = V(k, q);
                    V(k, p) = c * vkp - s * vkq;
                    V(k, q) = s * vkp + c * vkq;
                }
            }
        }
    }
#undef A
#undef V
}

/* Appendix "Lanczos methods" and Sec. 5.2 (Lanczos.c): the Hermitian Lanczos
 * process builds an orthonormal Krylov basis q_1..q_m of H (frozen at the
 * field passed in) from q_1 = F/||F|| together with the tridiagonal matrix
 * T (alpha on the diagonal, beta beside it).  Each new direction w = H q_j is
 * orthogonalised against every earlier basis vector in one classical
 * Gram-Schmidt pass (this contains the three-term recurrence of the
 * listing); alpha_j = <q_j, H q_j>, beta_j = ||w||.  The process stops early
 * (the listing's "beta = 0" exit) when beta_j is below 1e-12 times the
 * Gershgorin bound of the field-free H, i.e. at round-off level for this
 * operator.  The subspace propagator
 * exp(-i T dt) e_1 is formed from the eigen-decomposition of T, and the
 * state is expanded back: F_{n+1} = ||F|| sum_k c_k q_k. */
int orc_lanczos_step(const orc_grid* g, double efield, double dt, int m, double complex* psi)
{
    const size_t len = state_len(g);
    double complex* q = malloc((size_t)m * len * sizeof *q);
    double complex* w = malloc(len * sizeof *w);
    double complex* h = malloc((size_t)m * sizeof *h);
    double* alpha = calloc((size_t)m, sizeof *alpha);
    double* beta = calloc((size_t)m, sizeof *beta);

    double norm2 = 0.0;
    for (size_t k = 0; k < len; ++k) norm2 += creal(psi[k]) * creal(psi[k]) + cimag(psi[k]) * cimag(psi[k]);
    const double norm = sqrt(norm2);
    for (size_t k = 0; k < len; ++k) q[k] = psi[k] / norm;

    const double breakdown = 1e-12 * orc_h_bound(g, 0.0);
    int meff = 0;
    for (int j = 0; j < m; ++j) {
        double complex* qj = q + (size_t)j * len;
        orc_apply_h(g, efield, qj, w);
        for (int i = 0; i <= j; ++i) {
            const double complex* qi = q + (size_t)i * len;
            double complex dot = 0.0;
            for (size_t k = 0; k < len; ++k) dot += conj(qi[k]) * w[k];
            h[i] = dot;
        }
#pragma omp parallel for schedule(static)
        for (size_t k = 0; k < len; ++k)
            for (int i = 0; i <= j; ++i) w[k] -= h[i] * q[(size_t)i * len + k];
        alpha[j] = creal(h[j]);
        double b2 = 0.0;
        for (size_t k = 0; k < len; ++k) b2 += creal(w[k]) * creal(w[k]) + cimag(w[k]) * cimag(w[k]);
        beta[j] = sqrt(b2);
        meff = j + 1;
        if (j == m - 1) break;
        if (beta[j] <= breakdown) break; /* invariant subspace found */
        double complex* qn = q + (size_t)(j + 1) * len;
#pragma omp parallel for schedule(static)
        for (size_t k = 0; k < len; ++k) qn[k] = w[k] / beta[j];
    }

    double* tmat = calloc((size_t)meff * meff, sizeof *tmat);
    double* s = malloc((size_t)meff * meff * sizeof *s);
    for (int j = 0; j < meff; ++j) {
        tmat[(size_t)j * meff + j] = alpha[j];
        if (j + 1 < meff) {
            tmat[(size_t)j * meff + j + 1] = beta[j];
            tmat[(size_t)(j + 1) * meff + j] = beta[j];
        }
    }
    orc_jacobi_eig(meff, tmat, s);
    /* c = S exp(-i Lambda dt) S^T e_1 */
    double complex* c = calloc((size_t)meff, sizeof *c);
    for (int k = 0; k < meff; ++k) {
        double complex acc = 0.0;
        for (int j = 0; j < meff; ++j) {
            const double lam = tmat[(size_t)j * meff + j];
            acc += s[(size_t)k * meff + j] * cexp(-I * lam * dt) * s[(size_t)0 * meff + j];
        }
        c[k] = acc;
    }
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < len; ++k) {
        double complex acc = 0.0;
        for (int j = 0; j < meff; ++j) acc += c[j] * q[(size_t)j * len + k];
        psi[k] = norm * acc;
    }
    free(c);
    free(s);
    free(tmat);
    free(q);
    free(w);
    free(h);
    free(alpha);
    free(beta);
    return meff;
}

/* Sec. 4 "Ground state calculation": the diffusion equation, i.e. the TDSE
 * with the time derivative taken in imaginary time (the factor -i of the
 * propagator replaced, read here as dF/dtau = -H F), field free, propagated by
 * the Taylor series of eq. Taylor with that factor:
 *   F_{n+1} = sum_{p=0..P} F^(p),  F^(0) = F_n,  F^(p+1) = (-dtau/(p+1)) H F^(p),
 * the partial waves renormalised after every step.  For a normalised F_n the
 * loss of unitarity gives the energy, eq. e_g read with the factor 2 of a
 * squared norm: E = -ln <F_{n+1}|F_{n+1}> / (2 dtau).  Returns E and leaves the
 * renormalised F_{n+1} in psi (the input is assumed normalised). */
double orc_imag_step(const orc_grid* g, double dtau, int order, double complex* psi)
{
    const size_t len = state_len(g);
    double complex* term = malloc(len * sizeof *term);
    double complex* next = malloc(len * sizeof *next);
    memcpy(term, psi, len * sizeof *term);
    for (int p = 0; p < order; ++p) {
        orc_apply_h(g, 0.0, term, next);
        const double factor = -dtau / (double)(p + 1);
#pragma omp parallel for schedule(static)
        for (size_t k = 0; k < len; ++k) {
            term[k] = factor * next[k];
            psi[k] += term[k];
        }
    }
    double n2 = 0.0;
    for (size_t k = 0; k < len; ++k) n2 += creal(psi[k]) * creal(psi[k]) + cimag(psi[k]) * cimag(psi[k]);
    n2 *= g->dr;
    const double scale = 1.0 / sqrt(n2);
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < len; ++k) psi[k] *= scale;
    free(term);
    free(next);
    return -log(n2) / (2.0 * dtau);
}

/* nsteps diffusion steps from psi, normalised first; energy[s] receives the
 * estimate of step s. */
void orc_imag_propagate(const orc_grid* g, double dtau, int order, int64_t nsteps, double complex* psi,
                        double* energy)
{
    const size_t len = state_len(g);
    double n2 = 0.0;
    for (size_t k = 0; k < len; ++k) n2 += creal(psi[k]) * creal(psi[k]) + cimag(psi[k]) * cimag(psi[k]);
    const double scale = 1.0 / sqrt(g->dr * n2);
    for (size_t k = 0; k < len; ++k) psi[k] *= scale;
    for (int64_t s = 0; s < nsteps; ++s) energy[s] = orc_imag_step(g, dtau, order, psi);
}

/* Sec. 2.1 "Absorbing potential": W(r) = (i/dt) ln{1 - cos^p[(pi/2)(1 - r/r_b)]}
 * added to V.  Over a step of length dt its propagator factor exp(-i W dt) is
 * exactly the mask M(r) = 1 - cos^p[(pi/2)(1 - r/r_b)] (taken as 0 from r_b
 * on): the potential is split off the step and applied as M to every partial
 * wave after it. */
double orc_mask(double r, double r_b, double p)
{
    if (r >= r_b) return 0.0;
    return 1.0 - pow(cos(0.5 * M_PI * (1.0 - r / r_b)), p);
}

void orc_apply_mask(const orc_grid* g, double r_b, double p, double complex* psi)
{
    for (int l = 0; l <= g->lmax; ++l)
        for (int i = 0; i < g->n; ++i) psi[(size_t)l * g->n + i] *= orc_mask(orc_radius(g, i), r_b, p);
}

/* Sec. 4, eq. flux and eq. yield in the length gauge (no vector-potential
 * term): the radial probability current through the sphere r = r_j,
 *   J = sum_l Im[f_l^*(r_j) df_l/dr(r_j)],
 * the first derivative of the stencil's order, zero beyond the box:
 * (f_{j+1} - f_{j-1}) / (2 dr) with the 3-point stencil and the 4th-order
 * (f_{j-2} - 8 f_{j-1} + 8 f_{j+1} - f_{j+2}) / (12 dr) of Sec. 2 with the
 * 5-point stencil. */
double orc_radial_current(const orc_grid* g, int j, const double complex* psi)
{
    double sum = 0.0;
    for (int l = 0; l <= g->lmax; ++l) {
        const double complex* f = psi + (size_t)l * g->n;
        sum += cimag(conj(f[j]) * first_derivative(g, f, j));
    }
    return sum;
}

/* The velocity-gauge current (Sec. 4, eq. yield with its vector-potential
 * term): J + 2 A~ sum_l kappa_{l+1} Re[f_l^*(r_j) f_{l+1}(r_j)], the flux of
 * Re{psi^* (p + A/c) psi} through the sphere; equal to the length-gauge
 * current of the gauge-transformed state. */
double orc_radial_current_vel(const orc_grid* g, int j, double a_tilde, const double complex* psi)
{
    double extra = 0.0;
    for (int l = 0; l < g->lmax; ++l)
        extra += orc_kappa(l + 1) * creal(conj(psi[(size_t)l * g->n + j]) * psi[(size_t)(l + 1) * g->n + j]);
    return orc_radial_current(g, j, psi) + 2.0 * a_tilde * extra;
}

/* Initial state: the hydrogenic 1s radial function u(r) ~ r exp(-z r)
 * (Fig. "1sHydroRad": density 4 r^2 exp(-2r) for z = 1), normalised on the
 * grid, placed in the l = 0 partial wave.  u0 receives the normalised l = 0
 * row (the reference state of eq. p_g). */
void orc_initial_state(const orc_grid* g, double complex* psi, double* u0)
{
    double sum = 0.0;
    for (int i = 0; i < g->n; ++i) {
        const double r = orc_radius(g, i);
        u0[i] = r * exp(-g->z * r);
        sum += u0[i] * u0[i];
    }
    const double scale = 1.0 / sqrt(g->dr * sum);
    for (int i = 0; i < g->n; ++i) u0[i] *= scale;
    memset(psi, 0, state_len(g) * sizeof *psi);
    for (int i = 0; i < g->n; ++i) psi[i] = u0[i];
}

/* Sec. 4 observables, radial integrals by the rectangle rule dr * sum:
 *   norm  = sum_l int |f_l|^2
 *   p_g   = |<psi(0)|psi(t)>|^2 with psi(0) the l = 0 row u0 (eq. p_g)
 *   P_nl  = |<phi_nl|f_l>|^2 for the bound eigenvectors supplied by the caller
 *   p_ion = sum_l int_{r > r_b} |f_l|^2   (eq. yield_1)
 *   <z>   = 2 sum_l kappa_{l+1} Re int r f_l^* f_{l+1}           (eq. Dipole)
 *   <z''> = -E(t) - 2 z sum_l kappa_{l+1} Re int f_l^* f_{l+1} / r^2
 *                                                           (eq. DipoleAccel) */
void orc_observables(const orc_grid* g, const orc_pulse* p, double t, double r_ion,
                     const double* u0, int n_states, const int32_t* state_l, const double* phi,
                     const double complex* psi, double* out)
{
    const int n = g->n;
    const double dr = g->dr;
    double norm = 0.0, outer = 0.0, dip = 0.0, acc = 0.0;
    for (int l = 0; l <= g->lmax; ++l) {
        const double complex* fl = psi + (size_t)l * n;
        for (int i = 0; i < n; ++i) {
            const double a2 = creal(fl[i]) * creal(fl[i]) + cimag(fl[i]) * cimag(fl[i]);
            norm += a2;
            if (orc_radius(g, i) > r_ion) outer += a2;
        }
        if (l < g->lmax) {
            const double complex* fn = psi + (size_t)(l + 1) * n;
            double sd = 0.0, sa = 0.0;
            for (int i = 0; i < n; ++i) {
                const double r = orc_radius(g, i);
                const double re = creal(conj(fl[i]) * fn[i]);
                sd += r * re;
                sa += re / (r * r);
            }
            dip += orc_kappa(l + 1) * sd;
            acc += orc_kappa(l + 1) * sa;
        }
    }
    double complex proj0 = 0.0;
    for (int i = 0; i < n; ++i) proj0 += u0[i] * psi[i];
    proj0 *= dr;
    const double efield = orc_field(p, t);

    out[0] = t;
    out[1] = efield;
    out[2] = dr * norm;
    out[3] = creal(proj0) * creal(proj0) + cimag(proj0) * cimag(proj0);
    double pbound = 0.0;
    for (int k = 0; k < n_states; ++k) {
        const double complex* fl = psi + (size_t)state_l[k] * n;
        const double* ph = phi + (size_t)k * n;
        double complex proj = 0.0;
        for (int i = 0; i < n; ++i) proj += ph[i] * fl[i];
        proj *= dr;
        const double pop = creal(proj) * creal(proj) + cimag(proj) * cimag(proj);
        out[ORC_OBS_FIXED + k] = pop;
        pbound += pop;
    }
    out[4] = pbound;
    out[5] = dr * outer;
    out[6] = 2.0 * dr * dip;
    out[7] = -efield - 2.0 * g->z * dr * acc;
}

/* orc_propagate with the absorbing mask (r_abs > 0) applied after every step
 * and, for flux_j >= 0, the ionisation yield of eq. yield: the current J at
 * r_{flux_j} after every step (and at the start) integrated over time by the
 * trapezoid rule, returned in *flux. */
int orc_propagate_abs(const orc_grid* g, const orc_pulse* p, int method, int order_or_m, double t0,
                      double dt, int64_t nsteps, int64_t obs_every, double r_ion, const double* u0,
                      int n_states, const int32_t* state_l, const double* phi, double r_abs, double p_abs,
                      int flux_j, double complex* psi, double* obs_out, double* flux)
{
    const int rec = ORC_OBS_FIXED + n_states;
    int64_t n_obs = 0;
    int min_m = (method == ORC_LANCZOS) ? order_or_m : 0;
    double a_n = start_potential(g, p, t0, dt);
    double j_prev = (flux_j >= 0) ? orc_radial_current_vel(g, flux_j, a_n, psi) : 0.0;
    double yield = 0.0;
    for (int64_t s = 0; s < nsteps; ++s) {
        const double t_start = t0 + (double)s * dt;
        const double t_mid = t0 + ((double)s + 0.5) * dt;
        const double t_end = t0 + (double)(s + 1) * dt;
        const double c_mid = coupling_at(g, p, t_start, a_n, 0.5, dt, t_mid);
        if (method == ORC_TAYLOR) {
            orc_taylor_step(g, c_mid, dt, order_or_m, psi);
        } else if (method == ORC_RK4) {
            rk4_step_fields(g, coupling_at(g, p, t_start, a_n, 0.0, dt, t_start), c_mid,
                            coupling_at(g, p, t_start, a_n, 1.0, dt, t_end), dt, psi);
        } else {
            const int used = orc_lanczos_step(g, c_mid, dt, order_or_m, psi);
            if (used < min_m) min_m = used;
        }
        if (g->gauge == 1) a_n += orc_vector_potential_step(p, t_start, dt);
        if (r_abs > 0.0) orc_apply_mask(g, r_abs, p_abs, psi);
        if (flux_j >= 0) {
            const double j_new = orc_radial_current_vel(g, flux_j, a_n, psi);
            yield += 0.5 * dt * (j_prev + j_new);
            j_prev = j_new;
        }
        if (obs_every > 0 && (s + 1) % obs_every == 0 && obs_out) {
            orc_observables(g, p, t_end, r_ion, u0, n_states, state_l, phi, psi, obs_out + (size_t)n_obs * rec);
            ++n_obs;
        }
    }
    if (flux) *flux = yield;
    return min_m;
}

int orc_propagate(const orc_grid* g, const orc_pulse* p, int method, int order_or_m, double t0,
                  double dt, int64_t nsteps, int64_t obs_every, double r_ion, const double* u0,
                  int n_states, const int32_t* state_l, const double* phi, double complex* psi,
                  double* obs_out)
{
    const int rec = ORC_OBS_FIXED + n_states;
    int64_t n_obs = 0;
    int min_m = (method == ORC_LANCZOS) ? order_or_m : 0;
    double a_n = start_potential(g, p, t0, dt);
    for (int64_t s = 0; s < nsteps; ++s) {
        const double t_start = t0 + (double)s * dt;
        const double t_mid = t0 + ((double)s + 0.5) * dt;
        const double t_end = t0 + (double)(s + 1) * dt;
        const double c_mid = coupling_at(g, p, t_start, a_n, 0.5, dt, t_mid);
        if (method == ORC_TAYLOR) {
            orc_taylor_step(g, c_mid, dt, order_or_m, psi);
        } else if (method == ORC_RK4) {
            rk4_step_fields(g, coupling_at(g, p, t_start, a_n, 0.0, dt, t_start), c_mid,
                            coupling_at(g, p, t_start, a_n, 1.0, dt, t_end), dt, psi);
        } else {
            const int used = orc_lanczos_step(g, c_mid, dt, order_or_m, psi);
            if (used < min_m) min_m = used;
        }
        if (g->gauge == 1) a_n += orc_vector_potential_step(p, t_start, dt);
        if (obs_every > 0 && (s + 1) % obs_every == 0 && obs_out) {
            orc_observables(g, p, t_end, r_ion, u0, n_states, state_l, phi, psi,
                            obs_out + (size_t)n_obs * rec);
            ++n_obs;
        }
    }
    return min_m;
}
