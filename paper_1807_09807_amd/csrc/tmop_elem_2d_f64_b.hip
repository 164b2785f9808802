// Element kernels, 2D, double contractions: metrics mu_14, mu_77, mu_98.
#include "tmop_launch.h"

namespace tmop {
int launch_elem_2d_f64_b(int p, int Q, int metric, int op, const LaunchParams& lp, hipStream_t s, int* grid) {
  return launch_dispatch<2, double, 1>(p, Q, metric, op, lp, s, grid);
}
}  // namespace tmop
