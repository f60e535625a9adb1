// Clamp of a Gram-form distance (Eq. 4) before it is stored.
//
// N_i + N_j - 2 <x_i, x_j> evaluated in finite precision can dip slightly
// below zero for near-identical fields; such values become 0. A non-finite
// value (NaN or -inf, from non-finite inputs or an FP16 overflow when
// |x - mean| >= 65504) becomes +inf, so that a poisoned pair is never ranked
// as a near neighbour: +inf and the NaN window sums it leads to never pass a
// top-k bound. Plain C++, so the host tests compile it too.
#pragma once

#if defined(__HIPCC__)
#define TRAKNN_HOST_DEVICE __host__ __device__
#else
#define TRAKNN_HOST_DEVICE
#endif

namespace traknn {

TRAKNN_HOST_DEVICE inline float clamp_distance(float v) {
  return v > 0.f ? v : ((v != v || v == -__builtin_inff()) ? __builtin_inff() : 0.f);
}

}  // namespace traknn
