// af_weights.h -- fixed evolution stencils (host side).
#pragma once

#include "af_internal.h"

namespace af {

// a_dtdx = a dt / dx, b_dtdy = b dt / dy.
template <typename T>
void make_adv_weights(double a_dtdx, double b_dtdy, AdvWeights<T>* W);

// c_dtdx = c dt / dx, c_dtdy = c dt / dy.
template <typename T>
void make_ac_weights(double c_dtdx, double c_dtdy, AcWeights<T>* W);

// The same stencils in mirror-orbit form (af_internal.h); false if the
// FP64 stencils do not have the mirror symmetry to 1e-12 of their largest
// weight (they have it in exact arithmetic for any dx, dy).
template <typename T>
bool make_ac_orbit_weights(double c_dtdx, double c_dtdy, AcOrbitWeights<T>* W);

// Reconstruction weights for the coarse -> fine fill (Sec. 3.1): values at
// the quarter-step points of the reference square and quarter averages.
void make_fill_weights(FillWeights* W);

}  // namespace af
