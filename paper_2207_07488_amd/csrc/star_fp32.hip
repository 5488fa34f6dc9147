// FP32 star sweeps (mixed form).
#include "star_kernel.hpp"

namespace spnet {
void launch_star_fp32(const StarArgs &a, bool wide, int maxn, const double *r, const CgScalars *sc, int check, hipStream_t s) {
  launch_star_t<float>(a, wide, maxn, r, sc, check, s);
}
}  // namespace spnet
