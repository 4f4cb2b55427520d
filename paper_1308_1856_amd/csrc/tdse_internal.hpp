// Internal structures shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tdse {

constexpr int kBlock = 256;         // threads per workgroup of the sweep kernels (4 wave64)
constexpr int kMaxStates = 15;      // bound states n <= 5
constexpr int kMaxKrylov = 64;      // largest Lanczos dimension

// Tile sets: sweeps at 256 radii per tile (also RK4 stages), reductions
// (Lanczos, copies), populations, fused Horner terms (LDS rings), sweeps at
// 512 radii per tile (two radii per thread), fused Horner terms on wave
// strips, the observables' norm / dipole pass (taller tiles: fewer partial
// sums to finish), RK4 steps on wave strips (built for the four stages) and
// the H sweeps on aligned wave strips of one level.
enum TileSetId {
    kSweepTiles = 0, kReduceTiles = 1, kPopTiles = 2, kFusedTiles = 3, kPairTiles = 4, kStripTiles = 5,
    kObsTiles = 6, kRk4Tiles = 7, kApplyTiles = 8, kNumTileSets = 9
};
constexpr int kMaxFused = 8;        // most Horner terms per fused launch

// One instance (grid) as the per-instance kernels see it.
struct Inst {
    int64_t off;        // element offset of (l = 0, i = 0) in every state-shaped vector
    int64_t tab_off;    // offset (doubles) of this instance's u0 row in the radial table
    int32_t n;          // radial points
    int32_t lmax;
    int32_t n_states;   // bound states tracked (<= 15)
    int32_t i_ion;      // first radial index with r_i > r_ion
    int32_t tbegin[kNumTileSets];  // tiles [tbegin, tend) of each tile set
    int32_t tend[kNumTileSets];
    double dr;
    double inv_dr2;     // 1 / dr^2
    double z;
    double breakdown;   // Lanczos breakdown threshold: 1e-12 * Gershgorin bound of H
    double r_abs;       // absorbing mask reaching 0 at r_abs (<= 0: none)
    double p_abs;       // its exponent
    int32_t i_flux;     // grid point of the flux sphere (-1: none)
    int32_t pad_;
};

// A workgroup's share of a sweep: radial points [r0, r0 + kBlock) of rows
// [l0, l1) of one instance, with the instance fields the kernels need, so a
// workgroup starts with one uniform (scalar) load.
struct Tile {
    int64_t off;
    int64_t tab_off;
    int32_t inst, r0, l0, l1;
    int32_t n, lmax, i_ion, n_states;
    double dr, inv_dr2, z, pad_;
};

// Lanczos scalars per instance (FP64, device).
struct LanczosScalars {
    double norm0;                  // ||F|| at the start of the step
    double scale[kMaxKrylov];      // q_j = scale[j] * stored_j
    double alpha[kMaxKrylov];
    double beta[kMaxKrylov];
    double h[2 * kMaxKrylov];      // <q_i, H q_j> of the current iteration (re, im)
    double coef[2 * kMaxKrylov];   // recombination weights (re, im), include norm0 and scale
    int32_t meff;                  // Krylov dimension in use (grows; frozen at breakdown)
    int32_t done;                  // breakdown reached
    int32_t meff_min;              // smallest Krylov dimension over the steps of the current call
    int32_t pad_;
};

// ----------------------------------------------------------------------------
// Launchers (defined next to their kernels).  `prec` is the storage precision
// (0: FP64, 1: FP32, 2: 48-bit, see device_common.hpp); `S` is the stencil
// half-width (1 or 2).  Launchers of kernels without a 48-bit form return
// hipErrorInvalidValue for prec 2.
// ----------------------------------------------------------------------------
struct SweepGeom {
    const Inst* inst;      // device instance table
    const Tile* tiles;     // device tile table of the tile set used by the launch
    const double* kappa;   // device kappa_l table (lmax_max + 2 entries)
    int32_t n_tiles;
    int32_t n_inst;
    int32_t set;           // TileSetId of `tiles`
    int32_t variant;       // H sweep: 0 one radius per thread, 1 two radii per thread;
                           // strip sets: the level count the tiles were built for
    int32_t order;         // block -> tile map: 0 identity, 1 XCD-contiguous runs, 2 short runs dealt round the XCDs
    const void* zero_row;  // device zeros, at least max N complex FP64 values
    int64_t plane;         // s48 storage: elements per plane of a state-shaped vector
    int32_t gauge;         // 0 length (the field slots hold E), 1 velocity (they hold A/c)
    int32_t pad_;
};

// Per-step scalars, FP64, laid out [slot][instance] with these slots:
// kEStart, kEMid, kEEnd: the coupling scalar of the gauge at t_n, t_n + dt/2
// and t_n + dt (E in the length gauge, A/c in the velocity gauge).
// kRec: index of the observable record written after this step (-1: none).
// kEObs: the field E at t_n + dt (the observables' record, both gauges).
// kEStage0 + i: the coupling scalar at t_n + c_i dt for stage i of an
// explicit Runge-Kutta method given by its tableau (zero for other methods).
constexpr int kRkMax = 8;           // most stages of a tableau
enum StepSlot { kEStart = 0, kEMid = 1, kEEnd = 2, kTEnd = 3, kDt = 4, kRec = 5, kEObs = 6, kEStage0 = 7,
                kSlots = kEStage0 + kRkMax };
__host__ __device__ inline double step_value(const double* st, int n_inst, int slot, int inst)
{
    return st[slot * n_inst + inst];
}

// out = H(E_mid) in                              (term == 0)
// out = psi + (-i dt / term) H(E_mid) in         (term >= 1: one Horner term)
// out = psi - (dt / |term|) H(E_mid) in          (term <= -1: a Horner term of the
//                                                 diffusion step; g.variant 0 only)
// `out` must not overlap `in` or `psi` (`in` may equal `psi`).
hipError_t launch_hsweep(int prec, int S, const SweepGeom& g, const void* in, const void* psi,
                         void* out, const double* step, int term, hipStream_t st);

// K (1..kMaxFused) consecutive Horner terms first_term, first_term-1, ... in
// one launch over the fused tile set built for K; `out` must not alias `in`
// or `psi` (`in` may equal `psi`).
hipError_t launch_horner_fused(int prec, int S, int K, const SweepGeom& g, const void* in,
                               const void* psi, void* out, const double* step, int first_term,
                               hipStream_t st);
// The same K terms on the wave-strip tile set built for Kt >= K terms
// (g.variant = Kt; tiles of 4 strips of 64 - 2 Kt s output radii); same
// aliasing rules.  With obs_partial, the launch also writes the observables'
// main partial sums of its output (norm, p_ion, dipole, acceleration), one
// per strip: obs_partial[q * 4 n_tiles + 4 tile + wave], q < kObsMainQ.
// perm: the tiles in launch order (workgroup b takes tile perm[b]); without
// it, g.order maps blocks to tiles.
hipError_t launch_horner_strip(int prec, int S, int K, const SweepGeom& g, const void* in,
                               const void* psi, void* out, const double* step, int first_term,
                               hipStream_t st, double* obs_partial = nullptr, const int* perm = nullptr);
constexpr int kStripWaves = kBlock / 64;   // strips per strip tile
// The same K terms on pair strips: lane L holds radii 2L and 2L + 1 of a
// strip of 128, two waves per strip (levels 1..ceil(K/2) and the rest, the
// level rows handed over and the psi rows kept in LDS), tiles of kPairStrips
// strips of 128 - 2 Kt s output radii (g.variant = Kt >= K), 128 threads per
// strip; same results and aliasing rules as launch_horner_strip; the
// observables' partial sums in the first kPairStrips units of each tile's
// four (the others zero).
constexpr int kPairStrips = 1;   // pair strips per workgroup (two waves each)
// perm: the tiles in launch order (workgroup b takes tile perm[b]; without
// it, g.order maps blocks to tiles).  queue (needs perm): a persistent launch
// of the workgroups resident at once, which take the tiles in the order
// perm[0..n_tiles) from the counters queue[0..1] (zero before the launch,
// zero again after it).
hipError_t launch_horner_pstrip(int prec, int S, int K, const SweepGeom& g, const void* in, const void* psi,
                                void* out, const double* step, int first_term, hipStream_t st,
                                double* obs_partial = nullptr, unsigned* queue = nullptr,
                                const int* perm = nullptr);
// An H sweep (term 0) or one Horner term on the aligned strip tile set of one
// level (g.variant = 1; tiles of 4 waves of 64 radii from a multiple of 256);
// same results and aliasing rules as launch_hsweep.
hipError_t launch_strip_sweep(int prec, int S, const SweepGeom& g, const void* in, const void* psi, void* out,
                              const double* step, int term, hipStream_t st);
// One RK4 step on the strip tile set built for four levels (g.variant = 4):
// reads psi from `in`, writes the new psi to `out` (must not alias `in`).
hipError_t launch_rk4_strip(int prec, int S, const SweepGeom& g, const void* in, void* out, const double* step,
                            hipStream_t st);

// RK4 stage s (0..3); see the kernel for the buffer roles.
hipError_t launch_rk4_stage(int prec, int S, const SweepGeom& g, int stage, const void* gin,
                            const void* psi, void* acc, void* gout, const double* step,
                            hipStream_t st);

// Stage i of an explicit Runge-Kutta step (appendix "Runge-Kutta", eq.
// RKDeriv) over the sweep tiles (one radius per thread, g.variant 0):
//   k_i = -i H(t_n + c_i dt) g_i            (g_i read from gin; E from slot)
//   next = psi + dt sum_{j<=i} w_j k_j      (g_{i+1}, or the new state when last)
// k_i is stored at kv + i kstride unless last (k_0..k_{i-1} are read there);
// with err, the last stage also adds dt sum_j we_j k_j (the pair's deviation)
// as |.|^2 to a per-tile partial, err_partial[tile].  With 48-bit storage the
// nk stored k vectors are laid out plane by plane (kstride = plane length).
struct RkStage {
    int32_t stage, last, err, slot;
    double w[kRkMax];
    double we[kRkMax];
};
hipError_t launch_rk_stage(int prec, int S, const SweepGeom& g, const void* gin, const void* psi, void* kv,
                           int64_t kstride, int nk, void* next, const double* step, const RkStage& a,
                           double* err_partial, hipStream_t st);
// sigma[k] += sqrt(sum of instance k's err partials (sweep tiles) / U_k),
// U_k = (lmax + 1) N: the root mean square deviation of the step.
hipError_t launch_rk_sigma(const SweepGeom& g, const double* err_partial, double* sigma, hipStream_t st);

// Sec. 2.1 absorbing potential as its one-step factor: psi *= M(r) =
// 1 - cos^p[(pi/2)(1 - r/r_abs)] (0 from r_abs on) for the instances with
// r_abs > 0, in place, over the reduce tiles.
hipError_t launch_mask(int prec, const SweepGeom& g, void* psi, hipStream_t st);
// Sec. 4 eq. flux / eq. yield: one workgroup per instance with i_flux >= 0,
// J = sum_l Im[f_l^* df_l/dr] at point i_flux (the stencil's first
// derivative).  init: j_prev[k] = J; else yield[k] += dt (j_prev[k] + J) / 2
// and j_prev[k] = J (dt from the step table).
hipError_t launch_flux(int prec, int S, const SweepGeom& g, const void* psi, const double* step, int init,
                       double* j_prev, double* yield, hipStream_t st);

// Observables: per-tile partial sums of norm, p_ion, dipole and acceleration
// over the reduce tiles (kObsMainQ per tile, stored [q][tile]) and of p_g and
// the projections over the population tiles (kObsPopQ per tile, [q][tile]).
constexpr int kObsMainQ = 4;
constexpr int kObsRows = 16;   // most rows per tile of the observables' tile set
constexpr int kObsRecord = 8 + kMaxStates;   // doubles per tdse_obs record
constexpr int kObsPopQ = 2 + 2 * kMaxStates;
hipError_t launch_obs_partial(int prec, const SweepGeom& red, const SweepGeom& pop,
                              const double* radial_tab, const void* psi, double* partial_main,
                              double* partial_pop, hipStream_t st);
// One block per instance: sums the partials in tile order and writes the
// record of instance k at records + k * rec_stride + 23 * rec, with rec the
// record index of the step (kRec slot).  The main partials of instance k are
// units [upt * tbegin[main_set], upt * tend[main_set]) at stride main_stride
// (the observables pass: the kObsTiles set, one unit per tile; the Horner
// strips: the kStripTiles set, one unit per strip).
hipError_t launch_obs_finish(const SweepGeom& red, const SweepGeom& pop, const double* partial_main,
                             const double* partial_pop, const double* step, int64_t rec_stride,
                             double* out_records, hipStream_t st, int main_set = kObsTiles, int main_upt = 1,
                             int64_t main_stride = -1);

// Lanczos pieces (basis vector j >= 1 lives at basis + (j-1)*vec_stride
// elements; vector 0 is the state itself; with 48-bit storage vec_stride is
// the plane length and the m - 1 basis vectors are stored plane by plane).
hipError_t launch_lz_norm(int prec, const SweepGeom& g, const void* psi, double* partial,
                          hipStream_t st);
hipError_t launch_lz_norm_finish(const SweepGeom& g, const double* partial, LanczosScalars* sc,
                                 hipStream_t st);
hipError_t launch_lz_sweep_a(int prec, int S, const SweepGeom& g, int j, int m, const void* psi,
                             const void* basis, int64_t vec_stride, void* w, const double* step,
                             const LanczosScalars* sc, double* partial, hipStream_t st);
hipError_t launch_lz_finish_a(const SweepGeom& g, int j, int m, const double* partial,
                              LanczosScalars* sc, hipStream_t st);
hipError_t launch_lz_sweep_b(int prec, const SweepGeom& g, int j, int m, const void* psi,
                             const void* basis, int64_t vec_stride, const void* w,
                             const LanczosScalars* sc, double* partial, hipStream_t st);
hipError_t launch_lz_finish_b(const SweepGeom& g, int j, const double* partial,
                              LanczosScalars* sc, hipStream_t st);
hipError_t launch_lz_expm(const SweepGeom& g, const double* step, LanczosScalars* sc,
                          hipStream_t st);
// meff_min = m for every instance (before the first step of a call).
hipError_t launch_lz_reset(const SweepGeom& g, int m, LanczosScalars* sc, hipStream_t st);
hipError_t launch_lz_recombine(int prec, const SweepGeom& g, int m, void* psi, const void* basis,
                               int64_t vec_stride, const LanczosScalars* sc, hipStream_t st);

// The diffusion (imaginary-time) step's renormalisation, over the reduce
// tiles.  finish: per instance, n2 = dr * (sum of the lz_norm partials);
// scale_k = 1 / sqrt(n2) kept in sc[k].norm0; with energy != nullptr also
// energy[k * e_stride + e_index] = -ln(n2) / (2 dtau) (dtau from the step
// table) when `record` is set.  scale: dst = scale_k * src.
hipError_t launch_imag_finish(const SweepGeom& g, const double* partial, const double* step, int record,
                              double* energy, int64_t e_stride, int64_t e_index, LanczosScalars* sc,
                              hipStream_t st);
hipError_t launch_imag_scale(int prec, const SweepGeom& g, const void* src, void* dst, const LanczosScalars* sc,
                             hipStream_t st);

// Number of elements whose stored values differ bit for bit, added to *count.
hipError_t launch_count_diff(int prec, const SweepGeom& g, const void* a, const void* b,
                             unsigned int* count, hipStream_t st);

// out[0] += sum |a - b|^2, out[1] += sum |b|^2 (FP64, atomic accumulation).
hipError_t launch_diff_norm(int prec, const SweepGeom& g, const void* a, const void* b, double* out,
                            hipStream_t st);

// dst = src over every tile (state-shaped vectors).
hipError_t launch_copy(int prec, const SweepGeom& g, const void* src, void* dst, hipStream_t st);

}  // namespace tdse
