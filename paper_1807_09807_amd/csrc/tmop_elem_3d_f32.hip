// Element kernels, 3D, float contractions: mu_302, mu_303 and the 3D replication metric.
#include "tmop_launch.h"

namespace tmop {
int launch_elem_3d_f32(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  if (metric == MU7_3D && op != OP_SIZE && op != OP_JINV) return launch_elem_3d_f32_b(p, Q, metric, op, lp, s, grid);
  return launch_dispatch<3, float>(p, Q, metric, op, lp, s, grid);
}
}  // namespace tmop
