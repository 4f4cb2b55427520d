// Launches of the pair-strip Taylor kernel with one workgroup per tile; the
// persistent form is built in k_pstrip_q.hip.  The kernel itself is in
// pstrip_body.hpp.
#include "pstrip_body.hpp"

namespace tdse {

hipError_t launch_horner_pstrip_q(int prec, int S, int K, const SweepGeom& g, const void* in, const void* psi,
                                  void* out, const double* step, int first_term, hipStream_t st,
                                  double* obs_partial, unsigned* queue, const int* perm);

hipError_t launch_horner_pstrip(int prec, int S, int K, const SweepGeom& g, const void* in, const void* psi,
                                void* out, const double* step, int first_term, hipStream_t st, double* obs_partial,
                                unsigned* queue, const int* perm)
{
    if (g.gauge != 0) return hipErrorInvalidValue;   // length gauge only
    if (K < 1 || g.variant < K || g.variant * S * 2 >= 128) return hipErrorInvalidValue;
    if (queue && !perm) return hipErrorInvalidValue;
    if (queue) return launch_horner_pstrip_q(prec, S, K, g, in, psi, out, step, first_term, st, obs_partial, queue, perm);
    return pstrip_dispatch<false>(prec, S, K, g, in, psi, out, step, first_term, st, obs_partial, nullptr, perm);
}

}  // namespace tdse
