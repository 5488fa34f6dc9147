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
// Device state of one PCG column (one right-hand side), Sec. 4.2. A batch of KC
// columns keeps one of these per column; the kernels read the flags to decide
// which columns they advance.
//
//   active  the column holds a right-hand side
//   fresh   the next iteration skips its first half (q = K p ... convergence)
//           and only computes z = B r, rho = r.z and p = z: a column joins a
//           running batch this way
//   done    the recurrence has stopped (tolerance, max_iter or fixed count)
//   verify  stopped, its true residual f - K u is still to be checked
//   restart the check asked for a restart from the true residual
// ---------------------------------------------------------------------------
// rho = r.z is kept twice, by the parity of the iteration count: the kernel
// that computes a new rho (every block redundantly) stores it in
// rho[iters & 1] while its blocks still read the previous one from the other
// slot. first_it: the iteration count at which the recurrence (re)starts
// (beta = 0 there).
struct CgScalars {
  double rho[2], alpha, beta, rr, f2, tol2, t2, rtol;
  double tmp, pq, rz;
  int32_t iters, done, max_iter, fixed, first_it, fresh, verify, restart, replacements, active, pad1, pad2;
};

__device__ __forceinline__ double cg_alpha(const CgScalars &x, double pq) { return x.rho[x.iters & 1] / pq; }
__device__ __forceinline__ double cg_beta(const CgScalars &x, double rz) {
  return x.first_it == x.iters ? 0.0 : rz / x.rho[(x.iters & 1) ^ 1];
}

// which columns a kernel works on
enum ColumnSel : int32_t {
  SEL_ALL = 0,      // every column (apply_K / apply_B / set-up)
  SEL_FIRST = 1,    // first half of an iteration: active, not done, not fresh
  SEL_SECOND = 2,   // second half: active, not done
  SEL_VERIFY = 3,   // stopped columns whose true residual is pending
  SEL_RESTART = 4,  // columns restarting from their true residual
  SEL_MASK = 5,     // the columns of an explicit bit mask
};

__device__ __forceinline__ bool column_selected(const CgScalars &s, int sel, uint32_t mask, int c) {
  switch (sel) {
    case SEL_ALL: return true;
    case SEL_FIRST: return s.active && !s.done && !s.fresh;
    case SEL_SECOND: return s.active && !s.done;
    case SEL_VERIFY: return s.active && s.verify;
    case SEL_RESTART: return s.active && s.restart;
    default: return (mask >> c) & 1u;
  }
}

// Device layout of one star's factor (a "blob", 16-byte aligned; see
// factor.cpp and star_kernel.hpp). The index part (header, level table,
// position records, 16-bit index lists) comes first, padded to 16 bytes,
// then the values of the matrices S_k.
struct SnHeader {
  uint32_t n, nsn, nu, nlev;   // positions, supernodes, u-slots, levels
  uint32_t idx_bytes;          // bytes of the index part (multiple of 16)
  uint32_t val_bytes;          // bytes of the values (multiple of 16)
  uint32_t off_lev;            // uint32 [nlev + 1]: first position of each level
  uint32_t off_pos;            // SnPos [n]
  uint32_t off_R;              // uint16 [nu]: the position each u-slot updates
  uint32_t off_alist;          // uint16 [nu]: per position (ranges in SnPos), the u-slots aimed at it
  uint32_t pad[6];
};
static_assert(sizeof(SnHeader) == 64, "blob header");

// the supernode of a position and the u-slots aimed at it
struct SnPos {
  uint32_t sbase;  // first value of its supernode's S_k (elements of T from the start of the values)
  uint16_t c0;     // first position of the supernode
  uint16_t w;      // positions of the supernode (columns of its diagonal block)
  uint16_t h;      // rows below the diagonal block
  uint16_t ubase;  // first u-slot of the supernode
  uint16_t a0, a1; // alist[a0 .. a1-1]: the u-slots aimed at this position, ascending
};
static_assert(sizeof(SnPos) == 16, "position record");

// LDS a star workgroup may use: the 160 KB of a gfx950 compute unit
constexpr int kStarMaxLds = 160 * 1024;

// Arguments of the star kernel (see star_kernel.hpp).
struct SnArgs {
  int32_t nstars;                 // workgroups of the launch
  int32_t lds_bytes;              // dynamic LDS per workgroup
  const int32_t *order;           // star of each workgroup
  const unsigned char *blob;      // all blobs
  const int64_t *st_blob;         // byte offset of each star's blob
  const int32_t *st_pos;          // first slot of each star (its positions are consecutive slots)
  const int32_t *pos_dof;         // dof of every slot
  void *slots;                    // T, KC values per slot
  unsigned char *vscratch;        // vectors of the stars solved from global memory
  const int64_t *st_vs;           // byte offset of each such star's vectors in vscratch
};

// one launch over the stars of a.order: k_star with nteam wavefronts per
// workgroup, or (global) k_star_global with 256 threads per star; defined in
// star_inst.hip (one object per precision, column count and columns per
// wavefront)
template <typename T, int KC, int CW>
void launch_star_t(const SnArgs &a, int nteam, bool global, const double *r, const CgScalars *sc, int sel,
                   hipStream_t s);

}  // namespace spnet
