// The persistent launch of the pair-strip Taylor kernel (pstrip_body.hpp):
// the workgroups resident at once take the tiles from a work queue.  Its
// own translation unit, so that it builds beside the one-workgroup-per-tile
// form.
#include "pstrip_body.hpp"

namespace tdse {

hipError_t launch_horner_pstrip_q(int prec, int S, int K, const SweepGeom& g, const void* in, const void* psi,
                                  void* out, const double* step, int first_term, hipStream_t st,
                                  double* obs_partial, unsigned* queue, const int* perm)
{
    if (!queue || !perm) return hipErrorInvalidValue;
    return pstrip_dispatch<true>(prec, S, K, g, in, psi, out, step, first_term, st, obs_partial, queue, perm);
}

}  // namespace tdse
