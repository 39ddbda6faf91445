// Prescribed foil kinematics, shared by the marker kernels (positions for
// a window of steps) and the host (the pose of each step, passed to the
// interpolation and spreading kernels).
#pragma once

#include <cmath>

#include "marker_args.h"

namespace ibmk {

// Chord angle, its rate, pivot position and velocity at time t
// (Eqs. 20-21, 23; ABS_SIN takes the forward derivative at the kinks, the
// kink located from the half-period phase so that every side agrees).
__host__ __device__ inline void wing_pose(const WingDev& w, double t, double& th, double& thd, double& hx,
                          double& hy, double& vx, double& vy) {
  double al = w.mean, ald = 0.0;
  if (w.shape != 0) {
    const double om = 2.0 * M_PI / w.period;
    if (w.shape == 1) {
      const double arg = om * t + w.phase;
      al = w.mean + w.amp * sin(arg);
      ald = w.amp * om * cos(arg);
    } else {
      const double psi = t / w.period + w.phase / (2.0 * M_PI);
      const double h = psi - floor(2.0 * psi) / 2.0;
      al = w.mean + w.amp * sin(2.0 * M_PI * h);
      ald = w.amp * om * cos(2.0 * M_PI * h);
    }
  }
  th = w.theta0 + w.sense * al;
  thd = w.sense * ald;
  hx = w.hinge0[0];
  hy = w.hinge0[1];
  vx = 0.0;
  vy = 0.0;
  if (w.tamp != 0.0) {
    const double om = 2.0 * M_PI / w.period;
    const double arg = om * t + w.phase;
    const double cb = cos(w.tang), sb = sin(w.tang);
    hx += w.tamp * cos(arg) * cb;
    hy += w.tamp * cos(arg) * sb;
    vx = -w.tamp * om * sin(arg) * cb;
    vy = -w.tamp * om * sin(arg) * sb;
  }
}

}  // namespace ibmk
