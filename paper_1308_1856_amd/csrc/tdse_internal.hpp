// Internal structures shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tdse {

constexpr int kBlock = 256;         // threads per workgroup of the sweep kernels (4 wave64)
constexpr int kMaxStates = 15;      // bound states n <= 5
constexpr int kMaxKrylov = 64;      // largest Lanczos dimension
constexpr int kObsQ = 6 + 2 * kMaxStates;  // per-tile partial sums of the observables

// One instance (grid) as the kernels see it.
struct Inst {
    int64_t off;        // element offset of (l = 0, i = 0) in every state-shaped vector
    int64_t tab_off;    // offset (doubles) of this instance's u0 row in the radial table
    int32_t n;          // radial points
    int32_t lmax;
    int32_t n_states;   // bound states tracked (<= 15)
    int32_t i_ion;      // first radial index with r_i > r_ion
    int32_t tile_begin; // tiles [tile_begin, tile_end) of the sweep tile table
    int32_t tile_end;
    double dr;
    double inv_dr2;     // 1 / dr^2
    double z;
    double breakdown;   // Lanczos breakdown threshold: 1e-12 * Gershgorin bound of H
};

// A workgroup's share of a sweep: radial points [r0, r0 + kBlock) of rows [l0, l1).
struct Tile {
    int32_t inst;
    int32_t r0;
    int32_t l0;
    int32_t l1;
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
    int32_t pad_[2];
};

// ----------------------------------------------------------------------------
// Launchers (defined next to their kernels).  `T` is double (FP64 storage) or
// float (FP32 storage); `S` is the stencil half-width (1 or 2).
// ----------------------------------------------------------------------------
struct SweepGeom {
    const Inst* inst;      // device instance table
    const Tile* tiles;     // device tile table
    const int32_t* order;  // device block -> tile permutation (XCD-aware)
    const double* kappa;   // device kappa_l table (lmax_max + 2 entries)
    int32_t n_tiles;
    int32_t n_inst;
};

// Per-step scalars, FP64, laid out [slot][instance] with these slots:
enum StepSlot { kEStart = 0, kEMid = 1, kEEnd = 2, kTEnd = 3, kDt = 4, kSlots = 5 };
__host__ __device__ inline double step_value(const double* st, int n_inst, int slot, int inst)
{
    return st[slot * n_inst + inst];
}

// out = H(E_mid) in                              (term == 0)
// out = psi + (-i dt / term) H(E_mid) in         (term >= 1: one Horner term)
// `in` must not overlap `out`; `out` may equal `psi`.
hipError_t launch_hsweep(int prec, int S, const SweepGeom& g, const void* in, const void* psi,
                         void* out, const double* step, int term, hipStream_t st);

// RK4 stage s (0..3); see the kernel for the buffer roles.
hipError_t launch_rk4_stage(int prec, int S, const SweepGeom& g, int stage, const void* gin,
                            const void* psi, void* acc, void* gout, const double* step,
                            hipStream_t st);

// Per-tile partial sums of the observables of `psi` (kObsQ per tile).
hipError_t launch_obs_partial(int prec, const SweepGeom& g, const double* radial_tab,
                              const void* psi, double* partial, hipStream_t st);
// One block per instance: sums the partials in tile order and writes the
// record of instance k at out_records + k * rec_stride (doubles).
hipError_t launch_obs_finish(const SweepGeom& g, const double* partial, const double* step,
                             int64_t rec_stride, double* out_records, hipStream_t st);

// Lanczos pieces (basis vector j >= 1 lives at basis + (j-1)*vec_stride
// elements; vector 0 is the state itself).
hipError_t launch_lz_norm(int prec, const SweepGeom& g, const void* psi, double* partial,
                          hipStream_t st);
hipError_t launch_lz_norm_finish(const SweepGeom& g, const double* partial, LanczosScalars* sc,
                                 hipStream_t st);
hipError_t launch_lz_sweep_a(int prec, int S, const SweepGeom& g, int j, int m, const void* psi,
                             const void* basis, int64_t vec_stride, void* w, const double* step,
                             const LanczosScalars* sc, double* partial, hipStream_t st);
hipError_t launch_lz_finish_a(const SweepGeom& g, int j, int m, const double* partial,
                              LanczosScalars* sc, hipStream_t st);
hipError_t launch_lz_sweep_b(int prec, const SweepGeom& g, int j, const void* psi,
                             const void* basis, int64_t vec_stride, const void* w,
                             const LanczosScalars* sc, double* partial, hipStream_t st);
hipError_t launch_lz_finish_b(const SweepGeom& g, int j, const double* partial,
                              LanczosScalars* sc, hipStream_t st);
hipError_t launch_lz_expm(const SweepGeom& g, const double* step, LanczosScalars* sc,
                          hipStream_t st);
hipError_t launch_lz_recombine(int prec, const SweepGeom& g, int m, void* psi, const void* basis,
                               int64_t vec_stride, const LanczosScalars* sc, hipStream_t st);

// dst = src over every tile (state-shaped vectors).
hipError_t launch_copy(int prec, const SweepGeom& g, const void* src, void* dst, hipStream_t st);

}  // namespace tdse
