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

// N consecutive values of type T, moved with the widest aligned accesses
template <typename T, int N>
struct Row {
  T v[N];
  static constexpr int BYTES = N * (int)sizeof(T);
  static constexpr int CH = BYTES >= 16 ? 16 : BYTES;  // chunk bytes
  __device__ __forceinline__ void load(const T *p) {
    if constexpr (CH == 16) {
#pragma unroll
      for (int i = 0; i < BYTES / 16; ++i) {
        const float4 c = reinterpret_cast<const float4 *>(p)[i];
        __builtin_memcpy(reinterpret_cast<char *>(v) + 16 * i, &c, 16);
      }
    } else if constexpr (CH == 8) {
      const float2 c = *reinterpret_cast<const float2 *>(p);
      __builtin_memcpy(v, &c, 8);
    } else {
      v[0] = p[0];
    }
  }
  __device__ __forceinline__ void store(T *p) const {
    if constexpr (CH == 16) {
#pragma unroll
      for (int i = 0; i < BYTES / 16; ++i) {
        float4 c;
        __builtin_memcpy(&c, reinterpret_cast<const char *>(v) + 16 * i, 16);
        reinterpret_cast<float4 *>(p)[i] = c;
      }
    } else if constexpr (CH == 8) {
      float2 c;
      __builtin_memcpy(&c, v, 8);
      *reinterpret_cast<float2 *>(p) = c;
    } else {
      p[0] = v[0];
    }
  }
};

// Arguments of the band sweep kernel (see star_band.hpp).
// counters of the persistent band sweeps' star queues (k_star_queue): up to
// kQueues queues, one int32 each kQueueStride entries apart, then the count of
// wavefronts that have left
constexpr int kQueues = 8, kQueueStride = 64;

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
  const uint16_t *f_hdr, *b_hdr;             // per group: width in 16-byte slots (groups are contiguous)
  const void *f_inv, *b_inv;                 // 1/pivot per step (T)
  const void *f_val, *b_val;                 // packed stream values (T)
  int64_t f_zero, b_zero;                    // element offset of a zero region (16 KB) in f_val / b_val
  int32_t lds_reserve;                       // dynamic LDS per workgroup: caps waves per CU
  int32_t maxn;                              // largest star (positions)
  int32_t use_lds;                           // working vectors in LDS where they fit
  int32_t n_prio;                            // the first n_prio stars of order run at raised issue priority
  int32_t n_resident;                        // > 0: narrow sweeps as that many persistent wavefronts
  int32_t *queue;                            // their queue counters (k_star_queue; all 0 at rest)
  void *slots;                               // T, per position and column (position-major)
  // two-chain stars (k_star_twin; order then lists twin ids)
  int32_t unit0;                             // the chains of twin t are units unit0 + 2 t and unit0 + 2 t + 1
  const int32_t *tw_star, *tw_K;             // per twin: its star, the step where the chains meet
  const int32_t *pos_map;                    // per chain position: the star's band position, -1: not owned
  const int64_t *tw_vs;                      // per twin: first position of its two vectors in tw_scratch
  void *tw_scratch;                          // T, the chains' working vectors
};

// one band launch over the stars of a.order, narrow (windows of 1-2
// registers) or wide (4-16), for kc columns; defined in star_inst.hip (one
// object per precision and column count)
// per precision and column count
template <typename T, int KC>
void launch_star_t(const StarArgs &a, bool wide, const double *r, const CgScalars *sc, int sel, hipStream_t s);
// one launch over the two-chain stars of a.order (twin ids)
template <typename T, int KC>
void launch_twin_t(const StarArgs &a, const double *r, const CgScalars *sc, int sel, hipStream_t s);

// Device layout of one star's supernodal factor (a "blob", 16-byte aligned;
// see factor.cpp and star_sn.hpp). The index part (header, level table,
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
  uint32_t off_bpos;           // uint16 [n]: the star's slot (band position) of each position
  uint32_t pad[5];
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

// Arguments of the supernodal star kernels (see star_sn.hpp).
struct SnArgs {
  int32_t nstars;                 // workgroups of the launch
  int32_t lds_bytes;              // dynamic LDS per workgroup
  const int32_t *order;           // star of each workgroup
  const unsigned char *blob;      // all blobs
  const int64_t *st_blob;         // byte offset of each star's blob
  const int32_t *st_pos;          // first slot of each star (its slots are consecutive)
  const int32_t *pos_dof;         // dof of every slot (band order)
  void *slots;                    // T, KC values per slot
  unsigned char *vscratch;        // vectors of the stars solved from global memory
  const int64_t *st_vs;           // byte offset of each such star's vectors in vscratch
};

// one supernodal launch over the stars of a.order: k_sn with nteam
// wavefronts per workgroup, or (global) k_sn_global with 256 threads per star;
// defined in star_inst.hip (one object per precision, column count and
// columns per wavefront)
template <typename T, int KC, int CW>
void launch_sn_t(const SnArgs &a, int nteam, bool global, const double *r, const CgScalars *sc, int sel,
                 hipStream_t s);

}  // namespace spnet
