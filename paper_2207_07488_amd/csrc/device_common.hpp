// Types shared by the gfx950 kernels of the spnet library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>

#include "internal.hpp"

namespace spnet {

#define HIPCHK(x)                                                                                \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) fail(SN_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));      \
  } while (0)

// ---------------------------------------------------------------------------
// device scalars of one PCG recurrence
// ---------------------------------------------------------------------------
struct CgScalars {
  double rho, alpha, beta, pq, rr, rz, f2, tol2;
  double tmp;  // scratch dot result
  int32_t iters, done, max_iter, fixed, first, pad0;
};

// Arguments of the star sweep kernel (see star_kernel.hpp).
struct StarArgs {
  int32_t nstars;
  const int32_t *order;    // stars, longest first
  const int32_t *st_n;     // positions of the star
  const int32_t *st_vb;    // base in the per-position arrays
  const int32_t *st_q;     // window registers
  const int32_t *st_gb;    // base in the per-group header arrays
  const int64_t *st_fb;    // forward stream value base
  const int64_t *st_bb;    // backward stream value base
  const int32_t *pos_dof;  // global dof of each position (factor order)
  const uint32_t *f_hdr, *b_hdr;             // per group: width << 21 | offset (16-byte units)
  const void *f_inv, *b_inv;                 // 1/pivot per step (T)
  const void *f_val, *b_val;                 // packed stream values (T)
  void *slots;                               // T, per position
  int32_t pad;                               // LDS zero padding each side (elements)
};

// one launch over the stars of a.order, narrow (windows of 1-2 registers) or
// wide (4-16); defined in star_fp32.hip / star_fp64.hip
void launch_star_fp32(const StarArgs &a, bool wide, int maxn, const double *r, const CgScalars *sc, int check,
                      hipStream_t s);
void launch_star_fp64(const StarArgs &a, bool wide, int maxn, const double *r, const CgScalars *sc, int check,
                      hipStream_t s);

}  // namespace spnet
