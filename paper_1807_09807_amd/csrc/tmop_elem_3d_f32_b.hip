// Element kernels, 3D, float contractions: mu_7.
#include "tmop_launch.h"

namespace tmop {
int launch_elem_3d_f32_b(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  return launch_dispatch<3, float, 1>(p, Q, metric, op, lp, s, grid);
}
}  // namespace tmop
