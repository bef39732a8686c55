// The Metropolis proposal shared by the real and the complex sweeps (device code).
#pragma once
#include "common.hpp"
#include "kernels.hpp"

namespace vmc {

// The Metropolis move of electron e of walker w in sweep s.sweep: r' = r + delta (u - 1/2)
// wrapped into the box, with the acceptance uniform; Philox key (seed, traj), counter
// (step, w, sweep N + e, 0 | 1).
__device__ __forceinline__ void draw_move(const SweepArgs& s, int w, int N, int e, const double* po, double delta,
                                          double L, double invL, double& xn, double& yn, double& zn, double& ru3) {
  const uint32_t ctr2 = (uint32_t)(s.sweep * N + e);
  const u32x4 o0 = philox(s.step, (uint32_t)w, ctr2, 0u, s.seed, s.traj);
  const u32x4 o1 = philox(s.step, (uint32_t)w, ctr2, 1u, s.seed, s.traj);
  xn = wrap_box(po[0] + delta * (u01(o0.x, o0.y) - 0.5), L, invL);
  yn = wrap_box(po[1] + delta * (u01(o0.z, o0.w) - 0.5), L, invL);
  zn = wrap_box(po[2] + delta * (u01(o1.x, o1.y) - 0.5), L, invL);
  ru3 = u01(o1.z, o1.w);
}

}  // namespace vmc
