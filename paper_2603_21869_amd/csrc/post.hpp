// Post-processing of the fields on the device.
#pragma once
#include <hip/hip_runtime.h>

#include "nfvm_internal.hpp"

namespace nfvm {

// lambda2 vortex criterion (Sec. 3.2, after Jeong and Hussain): the middle
// eigenvalue of S^2 + W^2 per cell, S and W the symmetric and antisymmetric
// parts of the central velocity gradient with boundary ghosts (the gradient
// of the destruction step, Algorithm 3); zero on non-fluid cells.  Written
// dense, [nz][ny][nx] FP64, to `out` (ncells values).
template <class V>
void launch_lambda2(const Geom& g, const Phys& ph, const uint8_t* type, const DevPatch* pt,
                    const V* u, const V* v, const V* w, double* out, hipStream_t s);

// Line probes (Sec. 3.1): at n points (pts: 3n FP64 metres, x y z) the
// velocity magnitude, the temperature T_ref + theta, k and omega, each by
// trilinear interpolation between the cell centres over the fluid cells
// among the eight around the point (weights renormalised; NaN where none is
// fluid), the point clamped into the box of cell centres.  out: 4n FP64.
template <class V, class F>
void launch_probe(const Geom& g, const uint8_t* type, const V* u, const V* v, const V* w,
                  const F* T, const F* k, const F* om, double T_ref, const double* pts, int n,
                  double* out, hipStream_t s);

}  // namespace nfvm
