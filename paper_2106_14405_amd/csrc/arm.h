// arm.h -- forward kinematics of the kinematic 7-link capsule arm (float32,
// device), shared by the step and the batched collision queries.
#pragma once
#include "geom.h"

namespace rbs {

// Arm forward kinematics: joint axes z, y, z, y, z, y, z in each parent frame,
// link k spans joint k to joint k+1 along its local z.  Produces link centres
// c, orientations q (w x y z), world joint origins o and axes ax.
__device__ inline void arm_chain(const float* base, const float* th, const float* len, V3* c, float (*q)[4], V3* o, V3* ax) {
  float q0 = 1.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
  V3 p = v3(base[0], base[1], base[2]);
#pragma unroll
  for (int k = 0; k < 7; k++) {
    float sn, cs;
    sincosf(0.5f * th[k], &sn, &cs);
    // q (x) (cs, 0, 0, sn) for z joints; q (x) (cs, 0, sn, 0) for y joints
    float w, x, y, z;
    if ((k & 1) == 0) {
      w = q0 * cs - q3 * sn; x = q1 * cs + q2 * sn; y = q2 * cs - q1 * sn; z = q3 * cs + q0 * sn;
    } else {
      w = q0 * cs - q2 * sn; x = q1 * cs - q3 * sn; y = q2 * cs + q0 * sn; z = q3 * cs + q1 * sn;
    }
    q0 = w; q1 = x; q2 = y; q3 = z;
    M3 R = quat_R(w, x, y, z);
    V3 zl = col(R, 2);
    ax[k] = (k & 1) ? col(R, 1) : zl;
    o[k] = p;
    c[k] = p + zl * (0.5f * len[k]);
    q[k][0] = w; q[k][1] = x; q[k][2] = y; q[k][3] = z;
    p = p + zl * len[k];
  }
}

}  // namespace rbs
