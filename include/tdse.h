/*
 * tdse.h -- C ABI of the MI355X (gfx950) finite-difference TDSE library.
 *
 * What it computes (arXiv:1308.1856, O Broin & Nikolopoulos):
 *   the length-gauge, m = 0 partial-wave TDSE of a hydrogen-like atom,
 *     i d/dt F = H(t) F              (Sec. 2, eq. tdse_matrix)
 *   with F = [f_0(r_1..r_N), ..., f_lmax(r_1..r_N)] and H(t) the block-
 *   tridiagonal matrix of eq. h_matrix:
 *     (H F)_l = -1/2 D2 f_l + [l(l+1)/(2r^2) - Z/r] f_l
 *               + E(t) r [kappa_l f_{l-1} + kappa_{l+1} f_{l+1}]
 *   D2 is the 3-point or the 5-point (4th-order, Sec. 2) second difference
 *   with zero values beyond the box (Sec. 2.1); kappa_l = l / sqrt(4l^2 - 1);
 *   r_i = (i+1) dr, i = 0..N-1.  The field is the Hann-envelope pulse of
 *   Sec. 3 (eq. EField):  E(t) = E0 sin^2(pi tau/T) cos(w tau + cep),
 *   tau = t - t_on in [0, T], T = 2 pi n_cycles / w, zero outside.
 *
 * Memory and ownership
 *   The library never allocates device memory.  The caller owns the state
 *   buffer, the workspace, the observable buffers and the HIP stream; the
 *   library owns only its opaque host context (and small pinned host
 *   staging buffers).  All device work is enqueued on the stream given to
 *   tdse_bind and is asynchronous unless a function says it synchronises.
 *
 * State layout (device)
 *   Instances are concatenated; instance k starts at element offset
 *   tdse_state_offset(ctx, k) (a multiple of 64 elements).  Within an
 *   instance, element (l, i) sits at offset + l*N + i.  An element is an
 *   interleaved complex number: 16 bytes (re, im as double) for
 *   TDSE_FP64, 8 bytes (re, im as float) for TDSE_FP32; TDSE_FP48 splits
 *   the vector into two planes (see tdse_precision).  In the TDSE_FP32 and
 *   TDSE_FP48 modes every sweep reads and writes values of that storage
 *   precision but computes in FP64, and all reductions (norms, inner
 *   products, observables, Lanczos coefficients, the tridiagonal
 *   exponential) are FP64.
 *
 * Errors
 *   Every function returning tdse_status returns TDSE_OK (0) or a negative
 *   code; nothing throws across the ABI.  tdse_last_error() gives a message
 *   for the last failing call on a context.  On an error nothing has been
 *   enqueued unless the code is TDSE_E_HIP.
 */
#ifndef TDSE_H
#define TDSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tdse_status;
enum {
    TDSE_OK = 0,
    TDSE_E_INVALID = -1,    /* bad argument (null pointer, size, range)            */
    TDSE_E_NOMEM = -2,      /* host allocation failed                              */
    TDSE_E_HIP = -3,        /* a HIP runtime call failed                           */
    TDSE_E_UNSTABLE = -4,   /* explicit step would exceed its stability limit      */
    TDSE_E_BREAKDOWN = -5,  /* information, not a failure: a Lanczos step stopped
                               early at an invariant subspace (tdse_lanczos_dims) */
    TDSE_E_NONFINITE = -6,  /* a norm came out NaN or Inf                          */
    TDSE_E_WORKSPACE = -7,  /* bound workspace smaller than the method needs       */
    TDSE_E_UNBOUND = -8     /* no device memory bound yet (tdse_bind)              */
};

/* Storage precision of state-shaped vectors (arithmetic and reductions are
 * FP64 in all three).  TDSE_FP48: each FP64 component rounded to nearest at
 * 36 mantissa bits (relative rounding error <= 2^-37, against 2^-24 for
 * FP32), 12 bytes per complex element, stored in two planes: plane h holds
 * the upper 32-bit words of (re, im) of every element (8 bytes per element),
 * plane l, from byte 8 * P of the vector on, the next 16 bits of re (low
 * half) and im (high half) of every element (4 bytes), with P the element
 * count rounded up to a multiple of 64.  Rounding an FP32 state once per
 * step drifts coherently at the small steps explicit methods need on these
 * grids (the state changes by a few FP32 ulp per step); the 48-bit state
 * keeps that drift 2^13 times smaller.  The two-radii sweeps and the
 * LDS-ring fused kernel are FP64/FP32 only. */
typedef enum { TDSE_FP64 = 0, TDSE_FP32 = 1, TDSE_FP48 = 2 } tdse_precision;
/* TDSE_METHOD_TUNE only sizes the workspace the autotuners need (four
 * state-shaped vectors); TDSE_METHOD_RK_TABLEAU sizes tdse_step_rk's (its
 * order_or_m argument is the tdse_rk_method: stages + 1 vectors). */
typedef enum { TDSE_METHOD_TAYLOR = 0, TDSE_METHOD_RK4 = 1, TDSE_METHOD_LANCZOS = 2,
               TDSE_METHOD_TUNE = 3, TDSE_METHOD_RK_TABLEAU = 4 } tdse_method;
/* Explicit Runge-Kutta methods of tdse_step_rk (appendix "Runge-Kutta"): the
 * published tableaux of Euler (1 stage, order 1), the classic fourth-order
 * method (4, 4), Fehlberg's pair (6 stages, orders 5 and 4), the Cash-Karp
 * pair (6; 5, 4), the Dormand-Prince pair (7; 5, 4) and Merson's method
 * (5; 4, 3).  The solution carried forward is the higher order of a pair. */
typedef enum { TDSE_RK_EULER = 0, TDSE_RK_CLASSIC4 = 1, TDSE_RK_FEHLBERG45 = 2, TDSE_RK_CASHKARP = 3,
               TDSE_RK_DORMANDPRINCE = 4, TDSE_RK_MERSON = 5 } tdse_rk_method;

/* One instance (one radial grid and partial-wave set).  All instances of a
 * context must share stencil and precision. */
typedef struct {
    int32_t n_r;        /* radial points N, >= 8                                  */
    int32_t lmax;       /* highest partial wave, 0..1023                          */
    int32_t stencil;    /* 3 or 5                                                 */
    int32_t precision;  /* tdse_precision (TDSE_FP64, TDSE_FP32 or TDSE_FP48)     */
    double dr;          /* grid spacing (au), > 0                                 */
    double z_nuc;       /* nuclear charge Z (> 0)                                 */
    double r_ion;       /* ionisation radius r_b (au) for p_ion                   */
} tdse_grid_desc;

/* Sec. 3 pulse with the Hann (sine-squared) envelope over T = 2 pi n_c / w
 * from t_on (tau = t - t_on, zero outside [0, T]), in one of two shapes:
 *   TDSE_PULSE_SINE2_E  E = E0 sin^2(pi tau / T) cos(w tau + phi)  (eq. EField)
 *   TDSE_PULSE_SINE2_A  A/c = -E0 sin^2(W tau) sin(w tau + phi), W = pi / T,
 *                       E = -d(A/c)/dt  (the "SineA" form, eq. VecSinSinCosE;
 *                       A(T) = 0, so the gauges agree after the pulse) */
#define TDSE_PULSE_SINE2_E 0
#define TDSE_PULSE_SINE2_A 1
typedef struct {
    double e0;          /* field amplitude E0 (au)                                */
    double omega;       /* carrier angular frequency (au), > 0                    */
    double n_cycles;    /* carrier cycles under the envelope, > 0                 */
    double cep;         /* carrier-envelope phase (a sine carrier is -pi/2)       */
    double t_on;        /* start of the pulse (au)                                */
    int32_t shape;      /* TDSE_PULSE_SINE2_E or TDSE_PULSE_SINE2_A               */
    int32_t pad_;
} tdse_pulse;

#define TDSE_MAX_STATES 15
/* Observables at one time (Sec. 4), all FP64 with radial integrals dr*sum:
 *   norm    = sum_l int |f_l|^2
 *   p_g     = |<u0|f_0>|^2, u0 the normalised analytic 1s (eq. p_g, read as
 *             a probability)
 *   pop[k]  = |<phi_k|f_l(k)>|^2, phi_k the k-th bound eigenvector of the
 *             field-free block h_l, states ordered 1s 2s 3s 4s 5s 2p 3p 4p
 *             5p 3d 4d 5d 4f 5f 5g (fewer if lmax < 4; unused entries are 0)
 *   p_bound = sum_k pop[k]
 *   p_ion   = sum_l int_{r > r_ion} |f_l|^2                  (eq. yield_1)
 *   dipole  = 2 sum_l kappa_{l+1} Re int r f_l^* f_{l+1}      (eq. Dipole)
 *   accel   = -E(t) - 2 Z sum_l kappa_{l+1} Re int f_l^* f_{l+1} / r^2
 *                                                        (eq. DipoleAccel) */
typedef struct {
    double t, e_field, norm, p_g, p_bound, p_ion, dipole, accel;
    double pop[TDSE_MAX_STATES];
} tdse_obs;

typedef struct tdse_ctx tdse_ctx;

/* Creates a context for n_inst instances (n_inst = 1 for a single run; every
 * other call takes per-instance arrays of length n_inst).  Computes on the
 * host, in FP64: the instance and tile tables, kappa_l, the normalised 1s
 * row u0 and the bound eigenvectors phi_nl (n <= 5) of each h_l.  Touches no
 * device memory.  *out receives the context (NULL on error). */
tdse_status tdse_init_grid(const tdse_grid_desc* grids, int32_t n_inst, tdse_ctx** out);

/* Frees the host context (never the caller's device memory). */
void tdse_destroy(tdse_ctx* ctx);

const char* tdse_last_error(const tdse_ctx* ctx);

int32_t tdse_num_instances(const tdse_ctx* ctx);
/* Element offset of instance k in the state (and in any state-shaped vector). */
int64_t tdse_state_offset(const tdse_ctx* ctx, int32_t inst);
/* Bytes of one state-shaped device vector (all instances). */
size_t tdse_state_bytes(const tdse_ctx* ctx);
/* Workspace bytes needed by a method (order_or_m: Taylor order, ignored for
 * RK4, Krylov dimension for Lanczos).  The largest of the methods a caller
 * uses is enough for all of them. */
size_t tdse_workspace_bytes(const tdse_ctx* ctx, int32_t method, int32_t order_or_m);

/* Binds caller-owned device memory and a HIP stream (hipStream_t, may be
 * NULL for the null stream).  d_state: tdse_state_bytes bytes, 256-byte
 * aligned.  d_work: work_bytes >= tdse_workspace_bytes for every method used,
 * 256-byte aligned.  Uploads the tables into the workspace and synchronises
 * the stream.  May be called again to rebind. */
tdse_status tdse_bind(tdse_ctx* ctx, void* d_state, void* d_work, size_t work_bytes,
                      void* hip_stream);

/* Host <-> device copies of one instance's state as complex128 (interleaved
 * re, im doubles, (lmax+1)*N of them).  host_c128 == NULL in set_state puts
 * the normalised 1s state u0 in l = 0 and zeros elsewhere.  Both synchronise
 * the stream. */
tdse_status tdse_set_state(tdse_ctx* ctx, int32_t inst, const double* host_c128);
tdse_status tdse_get_state(tdse_ctx* ctx, int32_t inst, double* host_c128);

/* d_out = H(E) d_in for every instance, with e_field[k] the field of
 * instance k (Sec. 2, eq. h_matrix; A/c in the velocity gauge, see
 * tdse_set_gauge).  d_in and d_out are caller-owned
 * state-shaped device vectors in the context's precision; they must not
 * overlap.  Asynchronous. */
tdse_status tdse_apply_H(tdse_ctx* ctx, const double* e_field, const void* d_in, void* d_out);

/* Taylor propagator of order `order` (1..16), Sec. 5.2 eq. Taylor:
 *   F <- sum_{p=0..P} (-i dt H(t_s + dt/2))^p / p! F
 * evaluated in Horner form, one fused sweep per term (or several terms per
 * launch, see tdse_set_taylor_fusion).  Within the call psi rotates through
 * the state and the first two workspace vectors (no launch writes a buffer
 * it reads); the state buffer holds the result once the call's launches
 * have completed.  For each instance k
 * advances the bound state by nsteps steps of dt[k] from t0[k]; step s
 * spans [t0 + s dt, t0 + (s+1) dt].  If obs_every > 0 and d_obs != NULL the
 * observables after every obs_every-th step are written to d_obs (device
 * memory, [n_inst][nsteps / obs_every] records).  Returns TDSE_E_UNSTABLE
 * (and enqueues nothing) if dt[k] times tdse_lambda_max_bound(k, c_k)
 * exceeds the imaginary-axis stability limit of the order-P polynomial, with
 * c_k the pulse's bound on the coupling scalar of the gauge (length gauge:
 * |E0|, or |E0| (w + w / (2 n_c)) for TDSE_PULSE_SINE2_A; velocity gauge:
 * see tdse_set_gauge).  Returns TDSE_E_INVALID for an unknown pulse shape.
 * Asynchronous. */
tdse_status tdse_step_taylor(tdse_ctx* ctx, const tdse_pulse* pulses, const double* t0,
                             const double* dt, int32_t order, int32_t nsteps, int32_t obs_every,
                             tdse_obs* d_obs);

/* Classic fourth-order Runge-Kutta (Sec. 5.2 eq. RKDeriv, tableau c = 0, 1/2,
 * 1/2, 1; b = 1/6, 1/3, 1/3, 1/6) on dF/dt = -i H(t) F.  Arguments,
 * stability check and observables as tdse_step_taylor (limit of order 4).
 * By default one launch per step computes the four stages on wave strips
 * (see tdse_set_rk4_fusion); with FP64 storage its results are bit-identical
 * to four stage launches. */
tdse_status tdse_step_rk4(tdse_ctx* ctx, const tdse_pulse* pulses, const double* t0,
                          const double* dt, int32_t nsteps, int32_t obs_every, tdse_obs* d_obs);

/* Explicit Runge-Kutta propagator of the appendix "Runge-Kutta" (eq.
 * RKDeriv) with the tableau of `method` (tdse_rk_method): per step
 *   k_i = -i H(t_s + c_i dt) (F + dt sum_{j<i} a_ij k_j),  F <- F + dt sum_i b_i k_i,
 * one launch per stage.  For the embedded pairs and d_sigma != NULL (device
 * memory, n_inst FP64 values), the passive truncation estimate of the
 * appendix is accumulated: d_sigma[k] += sigma_n for every step, sigma_n =
 * sqrt(sum_e |Delta_e|^2 / U_k) the root mean square over the U_k elements of
 * instance k of the pair's difference Delta = dt sum_i (b_i - bhat_i) k_i (the
 * caller zeroes d_sigma to start a sum).  Arguments, observables and errors as
 * tdse_step_taylor; TDSE_E_UNSTABLE if dt[k] tdse_lambda_max_bound(k, c_k)
 * exceeds tdse_rk_stability_limit(method).  Needs the TDSE_METHOD_RK_TABLEAU
 * workspace of the method.  Asynchronous. */
tdse_status tdse_step_rk(tdse_ctx* ctx, const tdse_pulse* pulses, const double* t0, const double* dt,
                         int32_t method, int32_t nsteps, int32_t obs_every, tdse_obs* d_obs, double* d_sigma);
/* Imaginary-axis stability limit of the method's stability polynomial
 * R(z) = 1 + sum_k (b^T A^(k-1) 1) z^k: the largest y with |R(i y')| <=
 * 1 + 1e-12 for all y' <= y (0 for an unknown method). */
double tdse_rk_stability_limit(int32_t method);

/* Lanczos propagator (Sec. 5.2 Lanczos.c, appendix "Lanczos methods"): an
 * m-dimensional Krylov basis of H(t_s + dt/2) from F/||F||, each new
 * direction orthogonalised against all earlier basis vectors in one
 * classical Gram-Schmidt pass with FP64 coefficients (this contains the
 * three-term recurrence), and F <- ||F|| Q exp(-i T dt) e1.  The exponential
 * of the m x m tridiagonal T is taken by scaling and squaring, in FP64 on
 * one workgroup per instance: B = T dt / 2^s with ||B||_inf <= 1/2,
 * exp(-i B) = cos B - i sin B by their Taylor series to degree 17 (remainder
 * below 1e-21), then s complex squarings (no eigen-decomposition; the
 * paper's subspace Taylor series alone diverges for the Ritz values of stiff
 * grids, lambda dt ~ 1e3).  The process stops early at breakdown (beta_j <=
 * 1e-12 times the Gershgorin bound of the field-free H) and the step is then
 * exact in the invariant subspace found; since the call is asynchronous,
 * breakdown is reported afterwards by tdse_lanczos_dims.  m in 1..64.  No
 * stability limit.  Asynchronous. */
tdse_status tdse_step_lanczos(tdse_ctx* ctx, const tdse_pulse* pulses, const double* t0,
                              const double* dt, int32_t m, int32_t nsteps, int32_t obs_every,
                              tdse_obs* d_obs);

/* Ground-state search by the diffusion equation (Sec. 4, "Ground state
 * calculation"; eq. e_g): the TDSE in imaginary time, dF/dtau = -H F with no
 * field, advanced by nsteps steps of dtau[k] from the bound state of every
 * instance.  The state is first normalised; each step then applies the
 * order-P Taylor polynomial of exp(-dtau H) in Horner form,
 *   w_P = F - (dtau/P) H F, ..., w_1 = F - dtau H w_2,
 * takes n2 = ||w_1||^2 (FP64, dr * sum |w|^2), records the energy estimate
 * E = -ln(n2) / (2 dtau) (the loss of norm of a normalised state over one
 * step; the factor 2 of a squared norm) at d_energy[k * nsteps + s] (device
 * memory, FP64; may be NULL), and stores F = w_1 / sqrt(n2).  Repeated steps
 * converge to the lowest state of the discrete H within the symmetry of the
 * start (no field couples partial waves).  Returns TDSE_E_UNSTABLE (and
 * enqueues nothing) if dtau[k] times tdse_lambda_max_bound(k, 0) exceeds
 * tdse_taylor_real_stability_limit(order).  Needs the Taylor workspace of
 * the same order.  Asynchronous. */
tdse_status tdse_step_imag(tdse_ctx* ctx, const double* dtau, int32_t order, int32_t nsteps, double* d_energy);

/* Gauge of the atom-field coupling (Sec. 2, the L and V forms of the radial
 * TDSE in the dipole approximation):
 *   length    (H f)_l += E r [kappa_l f_{l-1} + kappa_{l+1} f_{l+1}]
 *   velocity  (H f)_l += -i (A/c) [kappa_l (d/dr - l/r) f_{l-1}
 *                                  + kappa_{l+1} (d/dr + (l+1)/r) f_{l+1}]
 * with d/dr the first derivative of the stencil's order ((f_{i+1} -
 * f_{i-1}) / (2 dr), or the fourth-order 5-point formula of Sec. 2 whose
 * printed 1/(12 h^2) is read as 1/(12 h)) and the l/r signs of p_z acting
 * on (f/r) Y_l0 (printed the other way round in the paper).  In the velocity
 * gauge A/c = -int_{t_on}^t E comes from eq. VectorStep (Sec. 3): A/c at the
 * start of a step call is the 5-point Gauss-Legendre quadrature of -E over
 * ceil((t0 - t_on) / dt) equal pieces from t_on (0 for t0 <= t_on), then each
 * step adds the quadrature over its own span, and every stage (midpoint,
 * Runge-Kutta stage times t_n + c_i dt) takes A/c(t_n) plus the quadrature
 * from t_n to its time.  The steps then run the workgroup sweeps (one launch
 * per Horner term; RK4 in four stage launches; the fusion settings are kept
 * for the length gauge), tdse_apply_H takes A/c in place of E, and
 * tdse_lambda_max_bound takes a bound on |A/c| (the step calls bound it by
 * |E0| for TDSE_PULSE_SINE2_A, by 3 |E0| / w for TDSE_PULSE_SINE2_E).  The
 * observables are the same sums (the norm, p_ion, dipole and acceleration
 * do not depend on the gauge; the populations agree once A = 0), and the
 * flux current gains its A term.  The diffusion steps have no field.  The
 * autotuners time the length-gauge kernels (the context is in the length
 * gauge while they run).  Returns TDSE_E_INVALID for another value. */
#define TDSE_GAUGE_LENGTH 0
#define TDSE_GAUGE_VELOCITY 1
tdse_status tdse_set_gauge(tdse_ctx* ctx, int32_t gauge);
int32_t tdse_gauge(const tdse_ctx* ctx);

/* Absorbing boundary (Sec. 2, "Absorbing potential"): the imaginary
 * potential W(r) of that subsection, split off every real-time step
 * (tdse_step_taylor, _rk4, _rk, _lanczos; not the diffusion steps) and
 * applied after it as its exact one-step factor, the mask
 *   M(r) = 1 - cos^p[(pi/2)(1 - r/r_b)]   (0 from r_b on),
 * multiplying every partial wave at radius r.  r_abs[k] is r_b of instance
 * k (au; <= 0: no absorber), p_abs[k] its exponent p (> 0 where r_abs[k] >
 * 0); host arrays of n_inst, copied.  The mask is 1 to FP64 precision well
 * inside r_b for the usual large p, so the loss of norm it causes measures
 * the probability that reached the absorber.  While any instance absorbs,
 * the Taylor path sums its observables in their own pass (after the mask)
 * instead of in the step's last launch.  Returns TDSE_E_UNBOUND before
 * tdse_bind, TDSE_E_INVALID for a non-finite r_abs or a p_abs <= 0 where
 * r_abs > 0 (nothing changed).  Synchronises the stream. */
tdse_status tdse_set_absorber(tdse_ctx* ctx, const double* r_abs, const double* p_abs);

/* Ionisation yield by the radial probability current (Sec. 4, "Ionisation
 * yield and angular distribution"; eq. yield): for each instance with
 * i_flux[k] >= 0, after every real-time step (after the absorbing mask)
 *   J = sum_l Im[f_l^*(r_j) df_l/dr(r_j)],   r_j = (i_flux[k] + 1) dr,
 * plus, in the velocity gauge, the vector-potential term
 * 2 (A/c) sum_l kappa_{l+1} Re[f_l^*(r_j) f_{l+1}(r_j)] (A/c at the state's time),
 * with the first derivative of the stencil's order ((f_{j+1} - f_{j-1}) /
 * (2 dr) with the 3-point Laplacian, the 4th-order 5-point derivative with
 * the 5-point one; values beyond the box are 0), integrated over time by the
 * trapezoid rule from the current of the state each step call starts from.
 * The yields accumulate on the device across step calls; this call sets
 * the flux points (host array of n_inst, -1: none) and resets every yield
 * to 0.  Returns TDSE_E_UNBOUND before tdse_bind, TDSE_E_INVALID for an
 * index outside [-1, n_r) (nothing changed).  Asynchronous, except for the
 * table upload. */
tdse_status tdse_set_flux(tdse_ctx* ctx, const int32_t* i_flux);

/* The accumulated flux yields, copied to host_yield[n_inst] (0 for the
 * instances without a flux point).  Synchronises the stream. */
tdse_status tdse_get_flux(tdse_ctx* ctx, double* host_yield);

/* Smallest Krylov dimension each instance used over the steps of the last
 * tdse_step_lanczos call, copied to host_meff[n_inst].  Synchronises the
 * stream.  Returns TDSE_E_BREAKDOWN (information: the results are valid) if
 * any instance stopped below the requested m, TDSE_E_INVALID if no Lanczos
 * step ran since the context was bound. */
tdse_status tdse_lanczos_dims(tdse_ctx* ctx, int32_t* host_meff);

/* Observables of the bound state at time t[k] (E(t) from pulses[k]) for
 * every instance, copied to host_out[n_inst].  Synchronises the stream.
 * Returns TDSE_E_NONFINITE if any norm is not finite. */
tdse_status tdse_observables(tdse_ctx* ctx, const tdse_pulse* pulses, const double* t,
                             tdse_obs* host_out);

/* For callers that cannot allocate device memory, or bind a workspace for
 * scratch (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the observables of tdse_observables, computed by the
 * same kernels in the same order (bit-identical records), with the call's
 * scratch (the step scalars of the record, the per-tile partial sums and the
 * records before their copy to host_out) in a static device buffer of the
 * library, TDSE_NOALLOC_SCRATCH_BYTES bytes per GPU, held until the process
 * ends, instead of the bound workspace; the context's tables still come from
 * the workspace bound by tdse_bind.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).  The current device must
 * be the one of the bound stream.  Returns TDSE_E_WORKSPACE (before any
 * device work) if the context's grids need more scratch than that,
 * TDSE_E_NONFINITE if any norm is not finite.  Every call on one GPU uses the
 * same buffer: calls that overlap on one GPU (other threads, other streams)
 * race.  Synchronises the stream. */
#define TDSE_NOALLOC_SCRATCH_BYTES (8u << 20)
tdse_status tdse_observables_noalloc(tdse_ctx* ctx, const tdse_pulse* pulses, const double* t,
                                     tdse_obs* host_out);

/* Gershgorin bound on the spectral radius of H for instance k when the
 * coupling scalar of the context's gauge is at most e_max in magnitude (|E|
 * in the length gauge, |A/c| in the velocity gauge): the largest absolute
 * row sum of eq. h_matrix. */
double tdse_lambda_max_bound(const tdse_ctx* ctx, int32_t inst, double e_max);

/* Imaginary-axis stability limit y_P of the degree-P Taylor polynomial: the
 * largest y with |sum_{k<=P} (i y')^k / k!| <= 1 + 1e-12 for all y' <= y. */
double tdse_taylor_stability_limit(int32_t order);

/* Real-axis stability limit x_P of the diffusion step's polynomial: the
 * largest x with |sum_{k<=P} (-x')^k / k!| <= 1 + 1e-12 for all 0 <= x' <= x. */
double tdse_taylor_real_stability_limit(int32_t order);

/* Autotuner for the sweep kernels (H.psi, Horner terms; RK4 stages take the
 * row count): times a Horner-term sweep of the bound state for each tile
 * shape (1, 2, 4, 8, 16 or 32 rows per workgroup) and each sweep variant
 * (bit 0: one radius per thread on 256-radius tiles, or two adjacent radii
 * per thread on 512-radius tiles; bit 1: workgroups take tiles in order, or
 * each XCD takes a contiguous run of tiles; bit 2: instead of either, wave
 * strips of 64 radii with radial neighbours by lane shifts (the values just
 * beyond a strip's ends read per row) and rows loaded three rows ahead, four
 * strips per 256-radius tile, with bit 1 runs of four tiles per XCD;
 * variants 0, 1, 2, 3, 4 and 6 are timed), checks that every choice
 * produces bit-identical results to the current one (a sweep's arithmetic
 * depends on neither), keeps the fastest and appends it to the tuning
 * cache named by the environment variable TDSE_TUNE_CACHE (if set; read by
 * tdse_init_grid for grids of the same shape class).  Needs the Taylor
 * workspace (two state-shaped vectors, overwritten); leaves the state
 * untouched.  *rows_out (may be NULL) receives the choice.  Synchronises. */
tdse_status tdse_autotune(tdse_ctx* ctx, int32_t* rows_out);
/* Autotuner for the Taylor step of order `order` (1..16): times whole steps
 * of the bound state (field-free, stable dt) with one launch per Horner term
 * (the sweep tiles in use) and with K = 2..min(order, 8) terms per fused
 * launch (ceil(order/K) launches per step), for both fused kernels (kind 0: workgroup tiles of 256
 * radii with the intermediate levels in LDS rings, 8, 16 or 32 rows; kind 1:
 * independent 64-radius wave strips with the intermediate levels in
 * registers, 8, 16, 32 or 64 rows; kind 2: 128-radius pair strips, two
 * adjacent radii per lane, the psi rows of the levels in an LDS ring, 8, 16,
 * 32 or 64 rows; kind 3: the pair strips in a persistent launch, as many
 * workgroups as are resident at once taking the tiles from a work queue in
 * the workspace, most rows first, 16, 32 or 64 rows), verifies each
 * candidate's step against
 * the one-launch-per-term step (bit for bit in FP64; relative 2-norm
 * difference <= 1e-6 with FP32 storage, where the fused launches keep their
 * intermediates in FP64), and keeps the fastest for later tdse_step_taylor
 * calls.  With a strip kernel (kind 1..3) chosen it then times 8 steps with a
 * record after each, the main observables summed in the step's last launch
 * and by their own pass (tdse_set_obs_fusion), for each strip kernel whose
 * candidates at the chosen K all passed, at the chosen strip height and at
 * 16, 32 and 64 rows, and the fastest strip shapes of the two next-fastest
 * term counts (the fastest of four timed passes each), and keeps the fastest
 * term count, kernel, height and mode (when work vector 3 holds
 * the 8 records of every instance; else the settings stay).  Needs the TDSE_METHOD_TUNE workspace; the state is restored.
 * *fuse_k_out (0: one launch per term) and *rows_out (may be NULL) receive
 * the choice; tdse_taylor_fusion_kind gives the kernel.  Synchronises. */
tdse_status tdse_autotune_taylor(tdse_ctx* ctx, int32_t order, int32_t* fuse_k_out, int32_t* rows_out);
/* Horner terms per fused Taylor launch in use (0: one launch per term), the
 * fused kernel in use (0 LDS rings, 1 wave strips, 2 pair strips, 3 pair
 * strips in a persistent launch), and an explicit choice:
 * k = 0 (one launch per term) or 1..8 terms per fused launch of kernel
 * `kind` on tiles of `rows` rows (1..64); tdse_step_taylor then makes
 * ceil(order/k) launches per step, the last one with the remaining terms.
 * Synchronises. */
int32_t tdse_taylor_fusion(const tdse_ctx* ctx);
int32_t tdse_taylor_fusion_kind(const tdse_ctx* ctx);
tdse_status tdse_set_taylor_fusion(tdse_ctx* ctx, int32_t k, int32_t rows, int32_t kind);

/* Rows per workgroup of the sweep tile set in use, and the sweep variant
 * (0..7, bits as in tdse_autotune); and an explicit choice of both (rows
 * 1..32), e.g. to reproduce a tuned shape.  Results do not depend on it.
 * Synchronises. */
int32_t tdse_tile_rows(const tdse_ctx* ctx);
int32_t tdse_sweep_variant(const tdse_ctx* ctx);
tdse_status tdse_set_sweep_shape(tdse_ctx* ctx, int32_t rows, int32_t variant);

/* Step-loop replay through HIP graphs (default off).  When on, and timing is
 * off, and the bound stream is not the null stream, each step call captures
 * the launches of a 256-step chunk once into a hipGraph and replays it for
 * every chunk with the same launch pattern; results are bitwise identical to
 * direct launches.  Graphs are cached per (method, order, chunk length,
 * observable spacing, d_obs) and dropped on rebind.  Synchronises the stream. */
tdse_status tdse_use_graphs(tdse_ctx* ctx, int32_t enable);

/* Observables beside the next step (default on).  With the Taylor methods the
 * observables of step s (the Sec. 4 reductions over the state after step s)
 * run on a second stream of the library, concurrently with step s+1: the
 * state rotates through three buffers and the one holding psi(s) is first
 * overwritten in step s+2, which waits for them.  The second stream rejoins
 * the bound stream before a step call returns (and at the end of every
 * 256-step chunk, so captured graphs contain both branches).  Off: every
 * launch goes to the bound stream in order.  Results are bitwise identical
 * either way.  Synchronises the bound stream; drops captured graphs. */
tdse_status tdse_set_obs_overlap(tdse_ctx* ctx, int32_t enable);

/* Observables summed inside the Taylor step (default on): with the wave-strip
 * fused kernel in use, the last launch of a step whose record is due also
 * sums the norm, p_ion, dipole and acceleration terms of the rows it writes
 * (one partial sum per strip; the strip computes one row past its tile,
 * unstored, for the l-coupling of its last row), so the observables' own pass
 * reads only the rows l <= 4 of the populations; the finish adds the strips'
 * partials in strip order.  Off: the observables pass reads the whole state
 * (Sec. 4 reductions over its own tiles).  The two orders of summation differ
 * by FP64 rounding only.  Other step methods and kernels always use the pass.
 * tdse_obs_fusion gives the setting.  Synchronises the bound stream and the
 * observables stream; drops captured graphs. */
tdse_status tdse_set_obs_fusion(tdse_ctx* ctx, int32_t enable);
int32_t tdse_obs_fusion(const tdse_ctx* ctx);

/* RK4 in one launch per step (default on: the four stages as the levels of
 * wave strips, reading the state once and writing the new state once, the
 * stage vectors and the accumulator held in FP64 registers) or in four stage
 * launches (off: each stage reads and writes state-shaped vectors in the
 * storage precision).  tdse_rk4_fusion gives the setting.  Synchronises the
 * bound stream; drops captured graphs. */
tdse_status tdse_set_rk4_fusion(tdse_ctx* ctx, int32_t enable);
int32_t tdse_rk4_fusion(const tdse_ctx* ctx);

/* Kernel timing with HIP events recorded around every launch of the named
 * kernel family on the bound stream ("taylor_term", "rk4_stage",
 * "observables", "lanczos_sweep_a", "apply_h", "taylor_fused").  tdse_timing_enable(ctx, 1)
 * clears the counters; tdse_timing_read synchronises the stream and returns
 * the number of launches and their summed duration in milliseconds. */
tdse_status tdse_timing_enable(tdse_ctx* ctx, int32_t enable);
tdse_status tdse_timing_read(tdse_ctx* ctx, const char* kernel, int64_t* launches,
                             double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* TDSE_H */
