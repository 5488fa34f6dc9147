// Explicit instantiation of the star sweep launcher for one factor precision
// (STAR_T) and one column count (STAR_KC); the build compiles this file once
// per pair so that the variants compile in parallel.
#include "star_kernel.hpp"

#ifndef STAR_T
#error "STAR_T (float or double) must be defined"
#endif
#ifndef STAR_KC
#error "STAR_KC (1, 2, 4, 8 or 16) must be defined"
#endif

namespace spnet {
template void launch_star_t<STAR_T, STAR_KC>(const StarArgs &, bool, const double *, const CgScalars *, int,
                                             hipStream_t);
}  // namespace spnet
