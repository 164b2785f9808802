// Element kernels, 2D, float contractions: metrics mu_1, mu_2, mu_7, mu_9.
#include "tmop_launch.h"

namespace tmop {
int launch_elem_2d_f32(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  if (op != OP_SIZE && op != OP_JINV && (metric == 14 || metric == 77 || metric == 98)) return launch_elem_2d_f32_b(p, Q, metric, op, lp, s, grid);
  return launch_dispatch<2, float, 0>(p, Q, metric, op, lp, s, grid);
}
}  // namespace tmop
