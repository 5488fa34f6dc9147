// Explicit instantiation of the star kernel launchers for one factor precision
// (STAR_T) and one column count (STAR_KC): the band sweep, and the supernodal
// solve for every column count per wavefront (1, 2, 4) up to STAR_KC; the
// build compiles this file once per pair so that the variants compile in
// parallel.
#include "star_band.hpp"
#include "star_sn.hpp"

#ifndef STAR_T
#error "STAR_T (float or double) must be defined"
#endif
#ifndef STAR_KC
#error "STAR_KC (1, 2, 4, 8 or 16) must be defined"
#endif

namespace spnet {
template void launch_star_t<STAR_T, STAR_KC>(const StarArgs &, bool, const double *, const CgScalars *, int,
                                             hipStream_t);
template void launch_twin_t<STAR_T, STAR_KC>(const StarArgs &, const double *, const CgScalars *, int, hipStream_t);
template void launch_sn_t<STAR_T, STAR_KC, 1>(const SnArgs &, int, bool, const double *, const CgScalars *,
                                                int, hipStream_t);
#if STAR_KC >= 2
template void launch_sn_t<STAR_T, STAR_KC, 2>(const SnArgs &, int, bool, const double *, const CgScalars *,
                                                int, hipStream_t);
#endif
#if STAR_KC >= 4
template void launch_sn_t<STAR_T, STAR_KC, 4>(const SnArgs &, int, bool, const double *, const CgScalars *,
                                                int, hipStream_t);
#endif
}  // namespace spnet
