// FP64 star sweeps (plain form).
#include "star_kernel.hpp"

namespace spnet {
void launch_star_fp64(const StarArgs &a, bool wide, int maxn, const double *r, const CgScalars *sc, int check, hipStream_t s) {
  launch_star_t<double>(a, wide, maxn, r, sc, check, s);
}
}  // namespace spnet
