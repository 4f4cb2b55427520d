/*
 * Plain FP64 CPU oracle for the finite-difference, length-gauge, partial-wave
 * TDSE of hydrogen-like atoms (O Broin & Nikolopoulos, arXiv:1308.1856).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; it is
 * never called by the product path.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no source with the
 * GPU library.
 *
 * Conventions (each a reading of the paper where it is silent):
 *   state      psi[l*n + i] = f_l(r_i), l = 0..lmax, i = 0..n-1, complex128
 *   grid       r_i = (i+1)*dr + r_shift   (Sec. 2 grid, "Start"/"Offset" of
 *              the FD settings group); f = 0 outside [0, n)  (Sec. 2.1: the FD
 *              terms beyond the fixed boundary are zero)
 *   inner prod <u|v> = dr * sum conj(u) v   (rectangle rule)
 */
#ifndef TDSE_ORACLE_H
#define TDSE_ORACLE_H

#include <complex.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;        /* radial points per partial wave                    */
    int32_t lmax;     /* highest partial wave                              */
    int32_t stencil;  /* 3 (2nd order) or 5 (4th order, Sec. 2)            */
    int32_t gauge;    /* 0 length, 1 velocity (Sec. 2, the two forms of d) */
    double dr;        /* grid spacing (au)                                 */
    double z;         /* nuclear charge, V(r) = -z/r                       */
    double r_shift;   /* grid offset added to every radius (normally 0)    */
} orc_grid;

typedef struct {
    double e0;        /* peak field (au)                                   */
    double omega;     /* carrier angular frequency (au)                    */
    double n_cycles;  /* number of carrier cycles under the envelope       */
    double cep;       /* carrier-envelope phase                            */
    double t_on;      /* pulse start time (au)                             */
    int32_t shape;    /* 0 sin^2 envelope on E, 1 on A/c (Sec. 3, "SineA") */
    int32_t pad_;
} orc_pulse;

/* Observable record, in this order (all FP64):
 *   0 t, 1 E(t), 2 norm, 3 p_g, 4 p_bound (sum of P_nl), 5 p_ion(r_b),
 *   6 <z>, 7 <z''>, 8.. the populations P_nl (n_states of them)          */
#define ORC_OBS_FIXED 8

enum { ORC_TAYLOR = 0, ORC_RK4 = 1, ORC_LANCZOS = 2 };

double orc_radius(const orc_grid* g, int i);
double orc_kappa(int l);
double orc_field(const orc_pulse* p, double t);

/* Sec. 3, eq. VectorStep with A~ = A/c: -int_t^{t+h} E by the 5-point
 * Gauss-Legendre rule, the increment of A~ over [t, t + h]. */
double orc_vector_potential_step(const orc_pulse* p, double t, double h);
/* A~(t0) = -int_{t_on}^{t0} E (0 for t0 <= t_on) by the same rule over
 * M = ceil((t0 - t_on)/dt) equal pieces, summed in time order: the value the
 * per-step increments reach when the steps start at t_on. */
double orc_vector_potential_at(const orc_pulse* p, double t0, double dt);

double orc_h_bound(const orc_grid* g, double efield);

/* OpenMP threads of the element-wise loops (results do not depend on it:
 * every sum over elements runs on one thread, in index order).  One thread
 * after loading; orc_max_threads gives the OpenMP default of the process
 * (OMP_NUM_THREADS, else the cores). */
void orc_set_threads(int n);
int orc_max_threads(void);

void orc_apply_h(const orc_grid* g, double efield,
                 const double complex* f, double complex* hf);

void orc_taylor_step(const orc_grid* g, double efield, double dt, int order,
                     double complex* psi);
void orc_rk4_step(const orc_grid* g, const orc_pulse* p, double t, double dt,
                  double complex* psi);
/* returns the Krylov dimension actually used (smaller than m on breakdown) */
int orc_lanczos_step(const orc_grid* g, double efield, double dt, int m,
                     double complex* psi);

/* Diffusion (imaginary-time) step of the ground-state search: order-P
 * Taylor polynomial of exp(-dtau H) with E = 0, renormalised; returns the
 * energy estimate -ln||F'||^2 / (2 dtau) (input assumed normalised). */
double orc_imag_step(const orc_grid* g, double dtau, int order, double complex* psi);
/* normalises psi, then nsteps steps; energy[s] per step */
void orc_imag_propagate(const orc_grid* g, double dtau, int order, int64_t nsteps,
                        double complex* psi, double* energy);

/* Explicit Runge-Kutta methods of the appendix "Runge-Kutta" (tableaux). */
#define ORC_RK_MAX 8
enum { ORC_RK_EULER = 0, ORC_RK_CLASSIC4 = 1, ORC_RK_FEHLBERG45 = 2, ORC_RK_CASHKARP = 3,
       ORC_RK_DORMANDPRINCE = 4, ORC_RK_MERSON = 5 };
/* fills c[ORC_RK_MAX], a[ORC_RK_MAX][ORC_RK_MAX] (row-major), b, bhat;
 * returns the number of stages (0: unknown method) */
int orc_rk_tableau(int method, double* c, double* a, double* b, double* bhat);
/* one step; returns sigma_n (0 for methods without an embedded pair) */
double orc_rk_step(const orc_grid* g, const orc_pulse* p, int method, double t, double dt,
                   double complex* psi);
/* returns sigma = sum of sigma_n over the steps */
double orc_propagate_rk(const orc_grid* g, const orc_pulse* p, int method, double t0, double dt,
                        int64_t nsteps, int64_t obs_every, double r_ion, const double* u0,
                        int n_states, const int32_t* state_l, const double* phi,
                        double complex* psi, double* obs_out);

/* Eigen-decomposition of a dense real symmetric m x m matrix (row-major) by
 * cyclic Jacobi rotations: on return a holds the eigenvalues on its diagonal
 * and v (row-major) the eigenvectors as columns. */
void orc_jacobi_eig(int m, double* a, double* v);

void orc_initial_state(const orc_grid* g, double complex* psi, double* u0);

void orc_observables(const orc_grid* g, const orc_pulse* p, double t,
                     double r_ion, const double* u0, int n_states,
                     const int32_t* state_l, const double* phi,
                     const double complex* psi, double* out);

/* Sec. 2.1 absorbing mask M(r) = 1 - cos^p[(pi/2)(1 - r/r_b)] (0 from r_b
 * on), the one-step factor of the absorbing potential W; applied in place */
double orc_mask(double r, double r_b, double p);
void orc_apply_mask(const orc_grid* g, double r_b, double p, double complex* psi);
/* radial current J = sum_l Im[f_l^* df_l/dr] at grid point j (eq. flux) */
double orc_radial_current(const orc_grid* g, int j, const double complex* psi);
/* The velocity-gauge current: orc_radial_current plus the vector-potential
 * term of eq. yield, 2 A~ sum_l kappa_{l+1} Re[f_l^* f_{l+1}] at r_j. */
double orc_radial_current_vel(const orc_grid* g, int j, double a_tilde, const double complex* psi);
/* orc_propagate plus the mask after every step (r_abs > 0) and the
 * trapezoid-rule time integral of J at point flux_j (>= 0) in *flux */
int orc_propagate_abs(const orc_grid* g, const orc_pulse* p, int method, int order_or_m,
                      double t0, double dt, int64_t nsteps, int64_t obs_every, double r_ion,
                      const double* u0, int n_states, const int32_t* state_l,
                      const double* phi, double r_abs, double p_abs, int flux_j,
                      double complex* psi, double* obs_out, double* flux);

/* Runs nsteps steps of the chosen method from t0.  After every obs_every-th
 * step the observables are appended to obs_out (record length
 * ORC_OBS_FIXED + n_states).  Returns the smallest Krylov dimension used
 * (Lanczos) or 0. */
int orc_propagate(const orc_grid* g, const orc_pulse* p, int method,
                  int order_or_m, double t0, double dt, int64_t nsteps,
                  int64_t obs_every, double r_ion, const double* u0,
                  int n_states, const int32_t* state_l, const double* phi,
                  double complex* psi, double* obs_out);

#ifdef __cplusplus
}
#endif
#endif
