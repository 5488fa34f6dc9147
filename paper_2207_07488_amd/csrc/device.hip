// GPU hot path for gfx950 (MI355X): PCG on P = BK (Sec. 4.2) with the
// two-level additive Schwarz preconditioner B = P K_0^{-1} P^T +
// sum_j R_j^T K_j^{-1} R_j (Sec. 4.1), for KC right-hand sides at once.
//
// Every column runs its own recurrence (alpha, beta, convergence per column);
// the columns share the reads of the matrix, the star factors and the coarse
// operator. A vector of the batch is npad x KC, position-major (the KC values
// of a dof are adjacent). Per iteration:
//   first half   q = K p (sliced ELL, 64-row slices) and p.q   -> alpha
//                u += alpha p, r -= alpha q, r.r, convergence
//   second half  star sweeps z_j = K_j^{-1} r[S_j] (one wavefront per star)
//                r_H = P^T r, c = K_0^{-1} r_H (dense inverse, matrix cores)
//                z = P c + sum of the star slots of every dof, r.z -> beta
//                p = z + beta p
// Dot products are reduced per block in a fixed order and the partials are
// combined in a fixed order, per column: by a one-block kernel, by every block
// of the consuming kernel redundantly (alpha, beta for few columns), or by
// block 0 of the restriction (the convergence test, when the coarse solve runs
// first); always with the same arithmetic for every column and every KC, so a
// column's iterates do not depend on the other columns of its batch. The star
// sweeps live in star_kernel.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "device_common.hpp"

namespace spnet {

constexpr int kBlock = 256;     // threads of the vector kernels
constexpr int kSlice = 64;      // rows per ELL slice (one wavefront)
constexpr int kMaxGrid = 2048;  // blocks of the grid-stride vector kernels (= partial sums per column)
constexpr int kMaxCols = 16;

// Workspace of the entry points that allocate nothing (sn_apply_K_noalloc):
// one array per GPU, held until the process ends. Host code never uses the
// array's name as an address: each device's address comes from
// hipGetSymbolAddress (scratch_ptr) and is passed to the kernels.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

enum ScalarOp { OP_ALPHA = 0, OP_CONV = 1, OP_BETA = 2, OP_F2 = 3, OP_R2 = 4, OP_TRUE = 5, OP_DOT = 6 };

// ---------------------------------------------------------------------------
// KC adjacent doubles
// ---------------------------------------------------------------------------
template <int KC>
struct Vec {
  double v[KC];
  __device__ __forceinline__ void load(const double *p) {
    if constexpr (KC == 1) {
      v[0] = p[0];
    } else {
#pragma unroll
      for (int i = 0; i < KC / 2; ++i) {
        const double2 t = reinterpret_cast<const double2 *>(p)[i];
        v[2 * i] = t.x;
        v[2 * i + 1] = t.y;
      }
    }
  }
  __device__ __forceinline__ void store(double *p) const {
    if constexpr (KC == 1) {
      p[0] = v[0];
    } else {
#pragma unroll
      for (int i = 0; i < KC / 2; ++i) reinterpret_cast<double2 *>(p)[i] = double2{v[2 * i], v[2 * i + 1]};
    }
  }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < KC; ++c) v[c] = 0.0;
  }
};

template <typename TS, int KC>
struct SlotVec;
template <int KC>
struct SlotVec<double, KC> : Vec<KC> {};
template <int KC>
struct SlotVec<float, KC> {
  float v[KC];
  __device__ __forceinline__ void load(const float *p) {
    if constexpr (KC == 1) {
      v[0] = p[0];
    } else if constexpr (KC == 2) {
      const float2 t = *reinterpret_cast<const float2 *>(p);
      v[0] = t.x;
      v[1] = t.y;
    } else {
#pragma unroll
      for (int i = 0; i < KC / 4; ++i) {
        const float4 t = reinterpret_cast<const float4 *>(p)[i];
        v[4 * i] = t.x;
        v[4 * i + 1] = t.y;
        v[4 * i + 2] = t.z;
        v[4 * i + 3] = t.w;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// reductions: per-block partials in a fixed order, then one block combines
// them in a fixed order, so every result is independent of scheduling
// ---------------------------------------------------------------------------
// one DPP step on both halves of a double: the value of the lane `ctrl` names
// (0 where that lane is outside the row or masked)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double(((long long)(uint32_t)hi << 32) | (long long)(uint32_t)lo);
}

// sum over the wavefront in a fixed tree, in every lane: shifts by 1, 2, 4, 8
// inside each 16-lane row (lane 15 of a row then holds the row), then row 1
// takes row 0's and row 3 row 2's total (row_bcast:15), then rows 2-3 take
// lane 31's (row_bcast:31); lane 63 holds the total, which is broadcast
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __longlong_as_double(((long long)(uint32_t)hi << 32) | (long long)(uint32_t)lo);
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  __syncthreads();
  return s;  // thread 0
}

// per-column block sums of a kBlock-thread block; results in thread 0, which
// writes them to partials[c * kMaxGrid + blockIdx.x]
template <int KC>
__device__ __forceinline__ void block_partials(const Vec<KC> &v, double *partials) {
  __shared__ double sh[kBlock / 64][KC];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const double s = wave_sum(v.v[c]);
    if (lane == 0) sh[w][c] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      double s = 0.0;
      for (int i = 0; i < kBlock / 64; ++i) s += sh[i][c];
      partials[c * kMaxGrid + blockIdx.x] = s;
    }
  }
}

// thread t adds partials t, t+256, ... of every column in order; IB of them are
// loaded before the first is added (entries past nparts are skipped by a zero
// factor: adding +0 leaves a sum unchanged)
template <int KC>
__device__ __forceinline__ void partial_sums(const double *__restrict__ partials, int nparts, int t, Vec<KC> &sum) {
  constexpr int IB = KC <= 4 ? 8 : (KC <= 8 ? 4 : 2);
  static_assert(kMaxGrid % (kBlock * IB) == 0, "batches of partials");
  for (int i0 = 0; i0 < nparts; i0 += kBlock * IB) {
    double v[IB][KC];
#pragma unroll
    for (int u = 0; u < IB; ++u) {
      const int i = i0 + kBlock * u + t;
      const double m = i < nparts ? 1.0 : 0.0;
#pragma unroll
      for (int c = 0; c < KC; ++c) v[u][c] = partials[c * kMaxGrid + min(i, kMaxGrid - 1)] * m;
    }
#pragma unroll
    for (int u = 0; u < IB; ++u)
#pragma unroll
      for (int c = 0; c < KC; ++c) sum.v[c] += v[u][c];
  }
}

// the per-column totals of partials, as k_scalar forms them (same order), in
// every thread of the block: lets a consumer kernel reduce redundantly in each
// block instead of a one-block kernel in between
template <int KC>
__device__ __forceinline__ void block_totals(const double *__restrict__ partials, int nparts, const bool (&on)[KC],
                                             double (&tot)[KC]) {
  __shared__ double sh[kBlock / 64][KC];
  __shared__ double res[KC];
  Vec<KC> sum;
  sum.zero();
  partial_sums<KC>(partials, nparts, (int)threadIdx.x, sum);
  (void)on;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const double v = wave_sum(sum.v[c]);
    if (lane == 0) sh[w][c] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < KC; ++c) {
      double t = 0.0;
      for (int i = 0; i < kBlock / 64; ++i) t += sh[i][c];
      res[c] = t;
    }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < KC; ++c) tot[c] = res[c];
}

// few columns: alpha and beta are reduced inside the update kernels
template <int KC>
constexpr bool kFuseScalars = KC <= 2;

template <int KC>
__device__ __forceinline__ bool any_selected(const CgScalars *sc, int sel, uint32_t mask) {
  if (sel == SEL_ALL) return true;
  bool any = false;
#pragma unroll
  for (int c = 0; c < KC; ++c) any |= column_selected(sc[c], sel, mask, c);
  return any;
}

// the scalar update of one column from the total of its partials
__device__ __forceinline__ void apply_scalar(CgScalars &x, int op, double tot) {
  switch (op) {
    case OP_ALPHA:
      x.pq = tot;
      x.alpha = cg_alpha(x, tot);
      break;
    case OP_CONV: {
      x.rr = tot;
      const int it = x.iters + 1;
      x.iters = it;
      const bool stop = x.fixed > 0 ? it >= x.fixed : (tot <= x.tol2 || it >= x.max_iter);
      if (stop) {
        x.done = 1;
        x.verify = 1;
      }
      break;
    }
    case OP_BETA:
      x.rz = tot;
      x.beta = cg_beta(x, tot);
      x.rho[x.iters & 1] = tot;
      x.fresh = 0;
      x.restart = 0;
      break;
    case OP_F2:
      x.f2 = tot;
      x.tol2 = x.rtol * x.rtol * tot;
      break;
    case OP_R2:
      x.rr = tot;
      if (x.fixed == 0 && (tot <= x.tol2 || x.f2 == 0.0)) {
        // nothing to iterate: r^(0) is the true residual
        x.done = 1;
        x.t2 = tot;
      }
      break;
    case OP_TRUE: {
      // The recurrence stopped; t2 = ||f - K u||^2. When it exceeds the
      // tolerance by a small factor the recurrence has drifted: restart from
      // the true residual. A true residual far above the tolerance is the
      // attainable accuracy of the system in FP64, which a restart cannot
      // improve.
      x.t2 = tot;
      x.verify = 0;
      if (x.fixed == 0 && x.rr <= x.tol2 && x.iters < x.max_iter && tot > x.tol2 * 1.0000001 &&
          tot < 100.0 * x.tol2 && x.replacements < 3) {
        x.replacements += 1;
        x.rr = tot;
        x.done = 0;
        x.first_it = x.iters;
        x.fresh = 1;
        x.restart = 1;
      }
      break;
    }
    default:
      x.tmp = tot;
  }
}

// one block: combine the partials of the previous kernel per column and update
// the scalars of the selected columns. Every column is summed like a single
// one (thread t adds partials t, t+256, ... in order, then a fixed block tree).
// Columns come in groups of at most four, one group per 256 threads.
template <int KC>
constexpr int scalar_groups() {
  return KC > 4 ? KC / 4 : 1;
}

template <int KC>
__global__ __launch_bounds__(kBlock * 4) void k_scalar(const double *__restrict__ partials, int nparts, CgScalars *sc,
                                                       int op, int sel, uint32_t mask) {
  constexpr int NG = scalar_groups<KC>(), CPG = KC / NG;
  __shared__ double sh[NG][kBlock / 64][CPG];
  bool any = false;
#pragma unroll
  for (int c = 0; c < KC; ++c) any |= column_selected(sc[c], sel, mask, c);
  if (!any) return;
  const int g = threadIdx.x / kBlock, t = threadIdx.x % kBlock;
  // every column of the group is loaded (the sums of unselected ones are not
  // used), so that all loads of a thread are in flight together
  Vec<CPG> sum;
  sum.zero();
  partial_sums<CPG>(partials + (size_t)g * CPG * kMaxGrid, nparts, t, sum);
  const int lane = t & 63, w = t >> 6;
#pragma unroll
  for (int c = 0; c < CPG; ++c) {
    const double v = wave_sum(sum.v[c]);
    if (lane == 0) sh[g][w][c] = v;
  }
  __syncthreads();
  if (t != 0) return;
  for (int cc = 0; cc < CPG; ++cc) {
    const int c = g * CPG + cc;
    if (!column_selected(sc[c], sel, mask, c)) continue;
    double tot = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) tot += sh[g][i][cc];
    apply_scalar(sc[c], op, tot);
  }
}

// ---------------------------------------------------------------------------
// sliced ELL SpMV: y = K x for KC columns, optionally x.y partials
// ---------------------------------------------------------------------------
struct Sell {
  const int32_t *sptr;  // slice start (elements)
  const int32_t *slen;  // slice width
  const int32_t *col;
  const double *val;
};

// A slice is one wavefront, so its width is uniform across the wavefront; the
// entries of a row are fetched U at a time (column indices, then the gathers of
// x) with clamped unconditional loads, so that the loads of a chunk overlap.
// Entries past the width are masked by a zero factor (padding entries already
// hold zeros), which leaves the sum unchanged.
template <int KC>
__global__ __launch_bounds__(kBlock) void k_spmv(Sell A, const double *__restrict__ x, double *__restrict__ y,
                                                 int nrows, const CgScalars *sc, int sel, double *partials) {
  if (!any_selected<KC>(sc, sel, 0u)) return;
  constexpr int U = KC <= 2 ? 8 : 4;
  Vec<KC> dot;
  dot.zero();
  for (int row = blockIdx.x * kBlock + threadIdx.x; row < nrows; row += gridDim.x * kBlock) {
    const int s = row >> 6, lane = row & 63;
    const int base = A.sptr[s], len = A.slen[s];
    Vec<KC> xr;
    if (partials) xr.load(x + (size_t)row * KC);
    Vec<KC> acc;
    acc.zero();
    for (int c0 = 0; c0 < len; c0 += U) {
      int cl[U];
      double a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + min(c0 + u, len - 1) * kSlice + lane;
        // the matrix is read once per application: non-temporal loads
        cl[u] = __builtin_nontemporal_load(A.col + e);
        a[u] = __builtin_nontemporal_load(A.val + e) * (c0 + u < len ? 1.0 : 0.0);
      }
      Vec<KC> xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u].load(x + (size_t)cl[u] * KC);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < KC; ++k) acc.v[k] = __builtin_fma(a[u], xv[u].v[k], acc.v[k]);
    }
    acc.store(y + (size_t)row * KC);
    if (partials) {
#pragma unroll
      for (int k = 0; k < KC; ++k) dot.v[k] = __builtin_fma(xr.v[k], acc.v[k], dot.v[k]);
    }
  }
  if (partials) block_partials<KC>(dot, partials);
}

// first-half columns: u += alpha p, r -= alpha q, r.r partials (rr_parts);
// with few columns alpha = rho / p.q is reduced here from the SpMV's partials
template <int KC>
__global__ __launch_bounds__(kBlock) void k_cg_update(double *u, double *r, const double *p, const double *q, int n,
                                                      CgScalars *sc, const double *__restrict__ pq_parts, int nparts,
                                                      double *rr_parts) {
  bool on[KC];
  bool any = false;
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    on[c] = column_selected(sc[c], SEL_FIRST, 0u, c);
    any |= on[c];
  }
  if (!any) return;
  // the first element's operands are fetched before the partials are added,
  // so that both latencies overlap
  const int i0 = blockIdx.x * kBlock + threadIdx.x;
  Vec<KC> uv, rv, pv, qv;
  if (i0 < n) {
    uv.load(u + (size_t)i0 * KC);
    rv.load(r + (size_t)i0 * KC);
    pv.load(p + (size_t)i0 * KC);
    qv.load(q + (size_t)i0 * KC);
  }
  double a[KC];
  if constexpr (kFuseScalars<KC>) {
    double tot[KC];
    block_totals<KC>(pq_parts, nparts, on, tot);
#pragma unroll
    for (int c = 0; c < KC; ++c) a[c] = on[c] ? cg_alpha(sc[c], tot[c]) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0)
      for (int c = 0; c < KC; ++c)
        if (on[c]) {
          sc[c].pq = tot[c];
          sc[c].alpha = a[c];
        }
  } else {
#pragma unroll
    for (int c = 0; c < KC; ++c) a[c] = sc[c].alpha;
  }
  Vec<KC> rr;
  rr.zero();
  for (int i = i0; i < n; i += gridDim.x * kBlock) {
    if (i != i0) {
      uv.load(u + (size_t)i * KC);
      rv.load(r + (size_t)i * KC);
      pv.load(p + (size_t)i * KC);
      qv.load(q + (size_t)i * KC);
    }
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      if (!on[c]) continue;
      uv.v[c] = __builtin_fma(a[c], pv.v[c], uv.v[c]);
      rv.v[c] = __builtin_fma(-a[c], qv.v[c], rv.v[c]);
      rr.v[c] = __builtin_fma(rv.v[c], rv.v[c], rr.v[c]);
    }
    uv.store(u + (size_t)i * KC);
    rv.store(r + (size_t)i * KC);
  }
  block_partials<KC>(rr, rr_parts);
}

// z = P c + sum of the star slots of every dof (ascending star order), r.z partials.
// The NV prolongation entries and slot indices of a dof are adjacent (vector
// loads); absent ones (index -1, weight 0) are read at index 0 and masked by a
// zero factor, so every gather is issued before the first one is used.
template <typename TS, int KC, int NV>
__global__ __launch_bounds__(kBlock) void k_reduce(double *z, const double *r, const TS *__restrict__ slots,
                                                   const int32_t *__restrict__ slot_of,
                                                   const int32_t *__restrict__ Pc, const double *__restrict__ Pw,
                                                   const double *__restrict__ cvec, int n,
                                                   const CgScalars *sc, int sel, double *partials) {
  if (!any_selected<KC>(sc, sel, 0u)) return;
  Vec<KC> rz;
  rz.zero();
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int pc[NV], so[NV];
    double pw[NV];
#pragma unroll
    for (int b = 0; b < NV; b += 4) {
      // the prolongation and slot lists are read once per application:
      // non-temporal loads
      typedef int i4 __attribute__((ext_vector_type(4)));
      typedef double d2 __attribute__((ext_vector_type(2)));
      const i4 c4 = __builtin_nontemporal_load(reinterpret_cast<const i4 *>(Pc + (size_t)i * NV + b));
      const i4 s4 = __builtin_nontemporal_load(reinterpret_cast<const i4 *>(slot_of + (size_t)i * NV + b));
      const d2 w0 = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(Pw + (size_t)i * NV + b));
      const d2 w1 = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(Pw + (size_t)i * NV + b + 2));
      pc[b] = c4.x;
      pc[b + 1] = c4.y;
      pc[b + 2] = c4.z;
      pc[b + 3] = c4.w;
      so[b] = s4.x;
      so[b + 1] = s4.y;
      so[b + 2] = s4.z;
      so[b + 3] = s4.w;
      pw[b] = w0.x;
      pw[b + 1] = w0.y;
      pw[b + 2] = w1.x;
      pw[b + 3] = w1.y;
    }
    Vec<KC> cv[NV];
    SlotVec<TS, KC> sv[NV];
#pragma unroll
    for (int b = 0; b < NV; ++b) {
      cv[b].load(cvec + (size_t)max(pc[b], 0) * KC);
      sv[b].load(slots + (size_t)max(so[b], 0) * KC);
    }
    Vec<KC> rv;
    if (partials) rv.load(r + (size_t)i * KC);
    Vec<KC> acc;
    acc.zero();
#pragma unroll
    for (int b = 0; b < NV; ++b)
#pragma unroll
      for (int k = 0; k < KC; ++k) acc.v[k] = __builtin_fma(pw[b], cv[b].v[k], acc.v[k]);
#pragma unroll
    for (int b = 0; b < NV; ++b) {
      const double m = so[b] >= 0 ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < KC; ++k) acc.v[k] += m * (double)sv[b].v[k];
    }
    acc.store(z + (size_t)i * KC);
    if (partials) {
#pragma unroll
      for (int k = 0; k < KC; ++k) rz.v[k] = __builtin_fma(rv.v[k], acc.v[k], rz.v[k]);
    }
  }
  if (partials) block_partials<KC>(rz, partials);
}

// second-half columns: p = z + beta p; with few columns beta = r.z / rho is
// reduced here from the accumulation's partials, and block 0 records the new
// rho (in the other parity slot than the one the blocks read)
template <int KC>
__global__ __launch_bounds__(kBlock) void k_p_update(double *p, const double *z, int n, CgScalars *sc,
                                                     const double *__restrict__ rz_parts, int nparts) {
  bool on[KC];
  bool any = false;
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    on[c] = column_selected(sc[c], SEL_SECOND, 0u, c);
    any |= on[c];
  }
  if (!any) return;
  // the first element's operands are fetched before the partials are added
  const int i0 = blockIdx.x * kBlock + threadIdx.x;
  Vec<KC> pv, zv;
  if (i0 < n) {
    pv.load(p + (size_t)i0 * KC);
    zv.load(z + (size_t)i0 * KC);
  }
  double b[KC];
  if constexpr (kFuseScalars<KC>) {
    double tot[KC];
    block_totals<KC>(rz_parts, nparts, on, tot);
#pragma unroll
    for (int c = 0; c < KC; ++c) b[c] = on[c] ? cg_beta(sc[c], tot[c]) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0)
      for (int c = 0; c < KC; ++c)
        if (on[c]) {
          CgScalars &x = sc[c];
          x.rz = tot[c];
          x.beta = b[c];
          x.rho[x.iters & 1] = tot[c];
          x.fresh = 0;
          x.restart = 0;
        }
  } else {
#pragma unroll
    for (int c = 0; c < KC; ++c) b[c] = sc[c].beta;
  }
  for (int i = i0; i < n; i += gridDim.x * kBlock) {
    if (i != i0) {
      pv.load(p + (size_t)i * KC);
      zv.load(z + (size_t)i * KC);
    }
#pragma unroll
    for (int c = 0; c < KC; ++c)
      if (on[c]) pv.v[c] = __builtin_fma(b[c], pv.v[c], zv.v[c]);
    pv.store(p + (size_t)i * KC);
  }
}

// r_H = P^T r: one wavefront per coarse dof (four per block); lane l sums the
// entries l, l+64, ... of the dof's list, then a fixed wavefront tree. The
// entries of a lane are fetched U at a time (indices, then the gathers), so
// that the dependent loads overlap.
template <int KC>
__global__ __launch_bounds__(kBlock) void k_restrict(const int32_t *__restrict__ ptr, const int32_t *__restrict__ dof,
                                                     const double *__restrict__ w, const double *__restrict__ r,
                                                     double *rH, int m0, CgScalars *sc, int sel,
                                                     const double *__restrict__ rr_parts, int nparts) {
  constexpr int U = KC <= 2 ? 8 : 4;
  if (rr_parts && blockIdx.x == 0) {
    // the first half's convergence test (what k_scalar does with OP_CONV), by
    // block 0 only. The other blocks may read a column's flags before or after
    // this update: the update only ever stops a column, and a stopped column's
    // r_H is not used, so skipping or computing it is correct either way.
    bool on[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) on[c] = column_selected(sc[c], SEL_FIRST, 0u, c);
    double tot[KC];
    block_totals<KC>(rr_parts, nparts, on, tot);
    if (threadIdx.x == 0)
      for (int c = 0; c < KC; ++c)
        if (on[c]) apply_scalar(sc[c], OP_CONV, tot[c]);
  }
  if (!any_selected<KC>(sc, sel, 0u)) return;
  const int g = (blockIdx.x * kBlock + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (g >= m0) return;
  Vec<KC> acc;
  acc.zero();
  const int q0 = ptr[g], q1 = ptr[g + 1];
  for (int qb = q0 + lane; qb < q1; qb += 64 * U) {
    int idx[U];
    double wq[U];
    // clamped unconditional loads; entries past the list are masked by a zero
    // weight, which leaves the sum unchanged
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = qb + 64 * u, qc = min(q, q1 - 1);
      idx[u] = __builtin_nontemporal_load(dof + qc);
      wq[u] = __builtin_nontemporal_load(w + qc) * (q < q1 ? 1.0 : 0.0);
    }
    Vec<KC> rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) rv[u].load(r + (size_t)idx[u] * KC);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < KC; ++k) acc.v[k] = __builtin_fma(wq[u], rv[u].v[k], acc.v[k]);
  }
  Vec<KC> out;
#pragma unroll
  for (int k = 0; k < KC; ++k) out.v[k] = wave_sum(acc.v[k]);
  if (lane == 0) out.store(rH + (size_t)g * KC);
}

// c = K_0^{-1} r_H on the matrix cores: v_mfma_f64_4x4x4_4b_f64 computes four
// independent 4 x 4 by 4 x 4 products (blocks y = 0..3) per instruction,
// accumulated in FP64. Lane l = 16 k + 4 y + i supplies A_y[i][k] and
// B_y[k][j = i]; the result D_y[i][j] sits in lane 16 i + 4 y + j (layout
// checked on the device). The inverse is stored symmetric, padded with zeros
// to ld x ld (ld a multiple of 64), in TA (double, or float in the mixed form,
// converted exactly on load); r_H and c have ld rows (r_H zero past m0).
// A workgroup of 16 wavefronts owns 8 rows: wavefront w takes rows
// 4 (w mod 2) .. + 3 and the (w / 2)-th eighth of the 64-column chunks (two
// workgroups per compute unit, for more loads in flight). In a chunk, lane
// (k, y, i) loads 4 adjacent columns 16 y + 4 k .. + 3 of its row (a load
// instruction reads 4 rows x 64 contiguous columns) and the four instructions
// s = 0..3 of the chunk take one of them each; block y thus sums the columns
// 16 y .. 16 y + 15 of every chunk. Column j NG + g of r_H (j = 0..3) goes to
// accumulator g, NG = ceil(KC / 4) accumulators; with fewer than four columns,
// positions past KC repeat column KC - 1 and are discarded. The partial
// products are added in LDS in a fixed order (column part, then block), so
// every column is computed by the same instructions whatever KC is and a
// batched column equals the single-column result bit for bit.
constexpr int kMmWaves = 16;

template <typename TA>
struct MmLoad;
template <>
struct MmLoad<double> {
  static __device__ __forceinline__ void load(const double *p, double (&a)[4]) {
    const double2 u = *reinterpret_cast<const double2 *>(p);
    const double2 v = *reinterpret_cast<const double2 *>(p + 2);
    a[0] = u.x;
    a[1] = u.y;
    a[2] = v.x;
    a[3] = v.y;
  }
};
// the packed coarse product streams its tiles once per application: loads
// marked non-temporal, so that they displace less of the local solves' factor
// streams from the caches
template <typename TA>
struct MmLoadNT;
template <>
struct MmLoadNT<double> {
  typedef double d2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ void load(const double *p, double (&a)[4]) {
    const d2 u = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p));
    const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p + 2));
    a[0] = u.x;
    a[1] = u.y;
    a[2] = v.x;
    a[3] = v.y;
  }
};
template <>
struct MmLoadNT<float> {
  typedef float f4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ void load(const float *p, float (&a)[4]) {
    const f4 u = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p));
    a[0] = u.x;
    a[1] = u.y;
    a[2] = u.z;
    a[3] = u.w;
  }
};
// FP32 values stay FP32 until the product that uses them converts them
template <>
struct MmLoad<float> {
  static __device__ __forceinline__ void load(const float *p, float (&a)[4]) {
    const float4 u = *reinterpret_cast<const float4 *>(p);
    a[0] = u.x;
    a[1] = u.y;
    a[2] = u.z;
    a[3] = u.w;
  }
};

template <typename TA, int KC>
__global__ __launch_bounds__(64 * kMmWaves) void k_coarse_mm(const TA *__restrict__ Kinv, int ld,
                                                             const double *__restrict__ rH, double *cvec, int m0,
                                                             const CgScalars *sc, int sel) {
  static_assert(KC >= 1 && KC <= 16, "up to four groups of four columns");
  constexpr int NG = (KC + 3) / 4;  // column groups
  constexpr int UC = (NG >= 3 || sizeof(TA) == 8) ? 2 : 4;  // chunks loaded before their products
  __shared__ double part[kMmWaves][4][4 * NG * 4];  // [wave][block][row * 4 NG + column]
  if (!any_selected<KC>(sc, sel, 0u)) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int i = lane & 3, y = (lane >> 2) & 3, k = lane >> 4;
  const int rt = wv & 1, qt = wv >> 1;  // row tile, column part
  const int row0 = blockIdx.x * 8 + 4 * rt;
  const int chunks = ld / 64, cpw = (chunks + 7) / 8;
  const int c0 = min(chunks, qt * cpw), c1 = min(chunks, c0 + cpw);
  const int col_l = 16 * y + 4 * k;  // the lane's first column in a chunk
  const TA *arow = Kinv + (size_t)(row0 + i) * ld + col_l;
  double acc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) acc[g] = 0.0;
  for (int c = c0; c < c1; c += UC) {
    TA a[UC][4];
    double b[UC][NG][4];
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      // a short last batch repeats the wavefront's last chunk with a zero factor
      const int cc = min(c + u, c1 - 1);
      MmLoad<TA>::load(arow + (size_t)cc * 64, a[u]);
      const int kb = cc * 64 + col_l;
      if constexpr (KC == 1) {
        const double2 p = *reinterpret_cast<const double2 *>(rH + kb);
        const double2 q = *reinterpret_cast<const double2 *>(rH + kb + 2);
        b[u][0][0] = p.x;
        b[u][0][1] = p.y;
        b[u][0][2] = q.x;
        b[u][0][3] = q.y;
      } else if constexpr (NG == 1) {
#pragma unroll
        for (int s = 0; s < 4; ++s) b[u][0][s] = rH[(size_t)(kb + s) * KC + min(i, KC - 1)];
      } else {
        // column j NG + g of r_H goes to accumulator g: a lane's NG columns are adjacent
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int g = 0; g < NG; g += 2) {
            const double2 v = *reinterpret_cast<const double2 *>(rH + (size_t)(kb + s) * KC + NG * i + g);
            b[u][g][s] = v.x;
            b[u][g + 1][s] = v.y;
          }
      }
    }
    // every load of the batch is issued before the first product waits
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const double m = c + u < c1 ? 1.0 : 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double av = (double)a[u][s] * m;
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, b[u][g][s], acc[g], 0, 0, 0);
      }
    }
  }
  // lane l = 16 i' + 4 y' + j' holds block y', row i', column j' of each group
  {
    const int ir = lane >> 4, yb = (lane >> 2) & 3, jc = lane & 3;
#pragma unroll
    for (int g = 0; g < NG; ++g) part[wv][yb][ir * 4 * NG + NG * jc + g] = acc[g];
  }
  __syncthreads();
  // rows 4 rt + i'' of the workgroup, columns: quarters in order, blocks in order
  for (int t = threadIdx.x; t < 8 * 4 * NG; t += 64 * kMmWaves) {
    const int row = t / (4 * NG), col = t % (4 * NG), rtt = row >> 2, ir = row & 3;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int yb = 0; yb < 4; ++yb) sum += part[2 * q + rtt][yb][ir * 4 * NG + col];
    const int grow = blockIdx.x * 8 + row;
    if (col < KC && grow < m0) cvec[(size_t)grow * KC + col] = sum;
  }
}

// The same product with one wavefront per four rows, for launches that share
// the device with the star sweeps (a one-wavefront workgroup takes whatever
// wave slot a SIMD has left). The wavefront runs the eight column parts of the
// workgroup form itself, QB parts at a time (their chunk loads in flight
// together), keeps each part's accumulators apart, and adds them in the
// workgroup form's order (part, then block) through lane shuffles, so every
// output equals the workgroup form's bit for bit (a chunk past a part's end is
// read in bounds and multiplied by zero, which leaves an accumulator as it is).
template <typename TA, int KC>
__global__ __launch_bounds__(64) void k_coarse_mm1(const TA *__restrict__ Kinv, int ld,
                                                   const double *__restrict__ rH, double *cvec, int m0,
                                                   const CgScalars *sc, int sel) {
  static_assert(KC >= 1 && KC <= 16, "up to four groups of four columns");
  constexpr int NG = (KC + 3) / 4;
  constexpr int NP = kMmWaves / 2;  // column parts of the workgroup form
  constexpr int QB = NG == 1 ? 4 : 2;
  if (!any_selected<KC>(sc, sel, 0u)) return;
  const int lane = threadIdx.x & 63;
  const int i = lane & 3, y = (lane >> 2) & 3, k = lane >> 4;
  const int row0 = blockIdx.x * 4;
  const int chunks = ld / 64, cpw = (chunks + NP - 1) / NP;
  const int col_l = 16 * y + 4 * k;
  const TA *arow = Kinv + (size_t)(row0 + i) * ld + col_l;
  double acc[NP][NG];
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[q][g] = 0.0;
  for (int t = 0; t < cpw; ++t) {
#pragma unroll
    for (int q0 = 0; q0 < NP; q0 += QB) {
      TA a[QB][4];
      double b[QB][NG][4];
#pragma unroll
      for (int u = 0; u < QB; ++u) {
        const int cq = (q0 + u) * cpw + t;
        const int cc = min(cq, chunks - 1);
        MmLoad<TA>::load(arow + (size_t)cc * 64, a[u]);
        const int kb = cc * 64 + col_l;
        if constexpr (KC == 1) {
          const double2 p = *reinterpret_cast<const double2 *>(rH + kb);
          const double2 r2 = *reinterpret_cast<const double2 *>(rH + kb + 2);
          b[u][0][0] = p.x;
          b[u][0][1] = p.y;
          b[u][0][2] = r2.x;
          b[u][0][3] = r2.y;
        } else if constexpr (NG == 1) {
#pragma unroll
          for (int s = 0; s < 4; ++s) b[u][0][s] = rH[(size_t)(kb + s) * KC + min(i, KC - 1)];
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int g = 0; g < NG; g += 2) {
              const double2 v = *reinterpret_cast<const double2 *>(rH + (size_t)(kb + s) * KC + NG * i + g);
              b[u][g][s] = v.x;
              b[u][g + 1][s] = v.y;
            }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < QB; ++u) {
        const double m = (q0 + u) * cpw + t < chunks ? 1.0 : 0.0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double av = (double)a[u][s] * m;
#pragma unroll
          for (int g = 0; g < NG; ++g)
            acc[q0 + u][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, b[u][g][s], acc[q0 + u][g], 0, 0, 0);
        }
      }
    }
  }
  // lane 16 i' + 4 y' + j' holds block y', row i', column j' of each group;
  // every lane forms the sum of its row and column over parts and blocks
  const int ir = lane >> 4, jc = lane & 3;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int yb = 0; yb < 4; ++yb) sum += __shfl(acc[q][g], 16 * ir + 4 * yb + jc, 64);
    const int col = NG * jc + g, grow = row0 + ir;
    if (y == 0 && col < KC && grow < m0) cvec[(size_t)grow * KC + col] = sum;
  }
}

// The product with the symmetric inverse stored once: the upper triangle in
// 64 x 64 tiles (I <= J), each tile in 16 strips of 4 rows, strip p holding for
// lane l = 16 k + 4 y + i the four values of row 4 p + i, columns
// 16 y + 4 k .. + 3 (one 16- or 32-byte load per lane, a whole strip per
// load instruction). One wavefront per tile computes
//   A_IJ r_J   (the strip's rows; the same MFMA operands as k_coarse_mm)
//   A_IJ^T r_I (I < J: the values moved to lane 16 i + 4 y + k, which makes
//               them the A operand of the transposed 4 x 4 products)
// and writes them as the (I, J) and (J, I) blocks of 64 x KC partial sums;
// k_coarse_fold adds the blocks of each row in order. Every column is computed
// by the same instructions whatever KC is.
constexpr int kSymTile = 64 * 64;

template <typename TA, int KC>
__global__ __launch_bounds__(64) void k_coarse_sym(const TA *__restrict__ Ks, const int2 *__restrict__ tiles, int T,
                                                   const double *__restrict__ rH, double *part,
                                                   const CgScalars *sc, int sel) {
  static_assert(KC >= 1 && KC <= 16, "up to four groups of four columns");
  constexpr int NG = (KC + 3) / 4;
  if (!any_selected<KC>(sc, sel, 0u)) return;
  const int lane = threadIdx.x & 63;
  const int i = lane & 3, y = (lane >> 2) & 3, k = lane >> 4;
  const int2 t = tiles[blockIdx.x];
  const int I = t.x, J = t.y;
  const TA *tp = Ks + (size_t)blockIdx.x * kSymTile + lane * 4;
  auto col_of = [&](int j, int g) { return KC == 1 ? 0 : (NG == 1 ? min(j, KC - 1) : NG * j + g); };
  // B operand of the direct product: r_J at rows 16 y + 4 k + s
  double bn[4][NG];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int g = 0; g < NG; ++g) bn[s][g] = rH[(size_t)(64 * J + 16 * y + 4 * k + s) * KC + col_of(i, g)];
  const int src = 16 * i + 4 * y + k;  // lane whose value is this lane's transposed operand
  const int ir = lane >> 4, jc = lane & 3;
  double acc_t[4][NG];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc_t[s][g] = 0.0;
  double *pdir = part + ((size_t)I * T + J) * 64 * KC;
  // the whole tile is loaded before the first product (one wavefront per
  // tile and about two tiles per SIMD: the loads are the parallelism)
  constexpr int H = (NG >= 3) ? 2 : 1;  // halves for the widest batches (registers)
#pragma unroll 1
  for (int h = 0; h < H; ++h) {
    constexpr int QN = 16 / H;
    TA a[QN][4];
    double bt[QN][NG];
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      MmLoadNT<TA>::load(tp + (size_t)(QN * h + q) * 256, a[q]);
#pragma unroll
      for (int g = 0; g < NG; ++g) bt[q][g] = rH[(size_t)(64 * I + 4 * (QN * h + q) + k) * KC + col_of(i, g)];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int p = QN * h + q;
      double an[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) an[g] = 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double av = (double)a[q][s];
#pragma unroll
        for (int g = 0; g < NG; ++g) an[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bn[s][g], an[g], 0, 0, 0);
      }
      // rows 4 p + ir: the four blocks added in order
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        double sum = 0.0;
#pragma unroll
        for (int yb = 0; yb < 4; ++yb) sum += __shfl(an[g], 16 * ir + 4 * yb + jc, 64);
        const int col = NG * jc + g;
        if (y == 0 && col < KC) pdir[(size_t)(4 * p + ir) * KC + col] = sum;
      }
      if (I != J) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double at = __shfl((double)a[q][s], src, 64);
#pragma unroll
          for (int g = 0; g < NG; ++g)
            acc_t[s][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(at, bt[q][g], acc_t[s][g], 0, 0, 0);
        }
      }
    }
  }
  if (I != J) {
    // lane 16 i' + 4 y' + j holds rows 16 y' + 4 i' + s of the (J, I) block
    double *ptr = part + ((size_t)J * T + I) * 64 * KC;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const int col = NG * jc + g;
        if (col < KC) ptr[(size_t)(16 * y + 4 * ir + s) * KC + col] = acc_t[s][g];
      }
  }
}

// c (rows below m0) = the sum of the T partial blocks of each block row R:
// one workgroup of four wavefronts per block row; lane r of wavefront w adds
// row r of the blocks C = w, w + 4, w + 8, ... in that order (one coalesced
// access per lane and block, eight blocks in flight), then the four wavefront
// sums are added in the order w = 0, 1, 2, 3 (the same order for every KC).
template <int KC>
__global__ __launch_bounds__(kBlock) void k_coarse_fold(const double *__restrict__ part, int T, double *cvec, int m0,
                                                        const CgScalars *sc, int sel) {
  static_assert(kBlock == 256, "four wavefronts per block row");
  if (!any_selected<KC>(sc, sel, 0u)) return;
  __shared__ double red[3][64 * KC];
  const int R = blockIdx.x, w = threadIdx.x >> 6, r = threadIdx.x & 63;
  const double *pp = part + ((size_t)R * T * 64 + r) * KC;
  Vec<KC> acc;
  acc.zero();
  for (int C0 = w; C0 < T; C0 += 32) {
    Vec<KC> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u].load(pp + (size_t)min(C0 + 4 * u, T - 1) * 64 * KC);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (C0 + 4 * u < T) {
#pragma unroll
        for (int c = 0; c < KC; ++c) acc.v[c] += v[u].v[c];
      }
  }
  if (w > 0) {
#pragma unroll
    for (int c = 0; c < KC; ++c) red[w - 1][r * KC + c] = acc.v[c];
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int ww = 0; ww < 3; ++ww)
#pragma unroll
      for (int c = 0; c < KC; ++c) acc.v[c] += red[ww][r * KC + c];
    const int row = R * 64 + r;
    if (row < m0) acc.store(cvec + (size_t)row * KC);
  }
}

// a.b partials per column
template <int KC>
__global__ __launch_bounds__(kBlock) void k_dot(const double *a, const double *b, int n, double *partials,
                                                const CgScalars *sc, int sel, uint32_t mask) {
  if (!any_selected<KC>(sc, sel, mask)) return;
  Vec<KC> s;
  s.zero();
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    Vec<KC> av, bv;
    av.load(a + (size_t)i * KC);
    bv.load(b + (size_t)i * KC);
#pragma unroll
    for (int k = 0; k < KC; ++k) s.v[k] = __builtin_fma(av.v[k], bv.v[k], s.v[k]);
  }
  block_partials<KC>(s, partials);
}

// y = a - b on the selected columns (others untouched), y.y partials
template <int KC>
__global__ __launch_bounds__(kBlock) void k_sub_dot(double *y, const double *a, const double *b, int n,
                                                    const CgScalars *sc, int sel, uint32_t mask, double *partials) {
  if (!any_selected<KC>(sc, sel, mask)) return;
  bool on[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) on[c] = column_selected(sc[c], sel, mask, c);
  Vec<KC> s;
  s.zero();
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    Vec<KC> yv, av, bv;
    yv.load(y + (size_t)i * KC);
    av.load(a + (size_t)i * KC);
    bv.load(b + (size_t)i * KC);
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      if (!on[c]) continue;
      yv.v[c] = av.v[c] - bv.v[c];
      s.v[c] = __builtin_fma(yv.v[c], yv.v[c], s.v[c]);
    }
    yv.store(y + (size_t)i * KC);
  }
  if (partials) block_partials<KC>(s, partials);
}

// dst = src on the selected columns
template <int KC>
__global__ __launch_bounds__(kBlock) void k_copy_sel(double *dst, const double *src, int n, const CgScalars *sc,
                                                     int sel, uint32_t mask) {
  if (!any_selected<KC>(sc, sel, mask)) return;
  bool on[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) on[c] = column_selected(sc[c], sel, mask, c);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    Vec<KC> dv, sv;
    dv.load(dst + (size_t)i * KC);
    sv.load(src + (size_t)i * KC);
#pragma unroll
    for (int c = 0; c < KC; ++c)
      if (on[c]) dv.v[c] = sv.v[c];
    dv.store(dst + (size_t)i * KC);
  }
}

// Start column `col` from column j of the n x k block `src` (canonical dof
// order; perm maps internal to canonical): f = r = src, u = p = 0 (rows
// n..npad-1 zero).
template <int KC>
__global__ __launch_bounds__(kBlock) void k_admit(double *f, double *r, double *u, double *p, const double *src,
                                                  const int32_t *__restrict__ perm, int n, int npad, int k, int j,
                                                  int col) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < npad; i += gridDim.x * kBlock) {
    const double v = i < n ? src[(size_t)perm[i] * k + j] : 0.0;
    const size_t o = (size_t)i * KC + col;
    f[o] = v;
    r[o] = v;
    u[o] = 0.0;
    p[o] = 0.0;
  }
}

// column col of a batch vector (internal order) <-> column j of an n x k
// block (canonical order)
template <int KC>
__global__ __launch_bounds__(kBlock) void k_col_in(double *dst, const double *src, const int32_t *__restrict__ perm,
                                                   int n, int npad, int k, int j, int col) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < npad; i += gridDim.x * kBlock)
    dst[(size_t)i * KC + col] = i < n ? src[(size_t)perm[i] * k + j] : 0.0;
}
template <int KC>
__global__ __launch_bounds__(kBlock) void k_col_out(double *dst, const double *src, const int32_t *__restrict__ perm,
                                                    int n, int k, int j, int col) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    dst[(size_t)perm[i] * k + j] = src[(size_t)i * KC + col];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {
// The caller's device allocator (sn_set_allocator), or none: hipMalloc.
struct Allocator {
  sn_alloc_fn alloc = nullptr;
  sn_free_fn free = nullptr;
  void *ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;

Allocator current_allocator() {
  std::lock_guard<std::mutex> g(g_alloc_mu);
  return g_alloc;
}

// Device memory of `bytes` from the current allocator on the current device;
// `owner` and `dev` record where it must go back.
void *device_alloc(size_t bytes, Allocator &owner, int &dev) {
  owner = current_allocator();
  HIPCHK(hipGetDevice(&dev));
  void *p = nullptr;
  if (!owner.alloc) {
    if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  } else {
    p = owner.alloc(bytes, dev, owner.ctx);
    if (p && reinterpret_cast<uintptr_t>(p) % 256 != 0) {
      owner.free(p, bytes, dev, owner.ctx);
      fail(SN_EINVAL, "the device allocator returned a pointer not aligned to 256 bytes");
    }
  }
  if (!p) fail(SN_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  return p;
}

// hipFree waits for the device; a caller's pool may hand the block out again
// at once, so the library's queued work on that device is drained first.
void device_free(void *p, size_t bytes, const Allocator &owner, int dev) {
  if (!p) return;
  if (owner.free) {
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    if (cur != dev) (void)hipSetDevice(cur);
    owner.free(p, bytes, dev, owner.ctx);
  } else {
    (void)hipFree(p);
  }
}
}  // namespace

template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  Allocator owner;
  int dev = 0;
  void alloc(size_t cnt) {
    release();
    if (cnt) {
      p = static_cast<T *>(device_alloc(cnt * sizeof(T), owner, dev));
      n = cnt;
    }
  }
  void upload(const std::vector<T> &h) {
    alloc(h.size());
    if (n) HIPCHK(hipMemcpy(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice));
  }
  void zero() {
    if (n) HIPCHK(hipMemset(p, 0, n * sizeof(T)));
  }
  void release() {
    device_free(p, n * sizeof(T), owner, dev);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
  ~DBuf() { release(); }
};

void set_device_allocator(sn_alloc_fn alloc, sn_free_fn free_, void *ctx) {
  if ((alloc == nullptr) != (free_ == nullptr)) fail(SN_EINVAL, "alloc and free_ must both be set or both be NULL");
  std::lock_guard<std::mutex> g(g_alloc_mu);
  g_alloc = Allocator{alloc, free_, alloc ? ctx : nullptr};
}

struct DeviceState {
  int device = 0;
  int precision = 0;
  int64_t n = 0, npad = 0, m0 = 0;
  int nv = 4;
  // matrix
  int nslices = 0;
  DBuf<int32_t> sptr, slen, col;
  DBuf<double> val;
  // stars: slots = the positions of all stars back to back, each star's in
  // its band (RCM) order; st_vb[s] is the first slot of star s
  int32_t nstars = 0, maxn = 0, maxlev = 0;
  int64_t slot_count = 0;
  DBuf<int32_t> st_vb, pos_dof, slot_of;
  std::vector<int32_t> h_n;            // per star: positions
  // band layout (star_band.hpp): windows of Q registers, packed streams
  std::vector<int32_t> h_q;            // per star: window registers (0: band beyond 1024, supernodal only)
  DBuf<int32_t> st_n, st_q, st_gb;
  DBuf<int64_t> st_fb, st_bb;
  DBuf<uint16_t> f_hdr, b_hdr;
  DBuf<float> f_inv32, b_inv32, f_val32, b_val32;
  DBuf<double> f_inv64, b_inv64, f_val64, b_val64;
  int64_t f_zero = 0, b_zero = 0;
  // supernodal layout (star_sn.hpp): one blob per star (index part, then values)
  DBuf<unsigned char> blob;
  DBuf<int64_t> st_blob;
  std::vector<uint32_t> h_idx, h_val, h_nu;  // per star: blob part bytes, u-slots
  std::vector<uint8_t> h_sn_ok;               // per star: the supernodal layout holds it
  std::vector<int64_t> h_bytes_band, h_bytes_sn;  // per star: algorithmic bytes of one solve of one column
  // two-chain band stars: per star its twin id (-1: none), per twin its chain
  // length and algorithmic bytes; the chains are units nstars + 2 t (+ 1) of
  // the per-star device arrays
  std::vector<int32_t> h_twin, h_twin_len;
  std::vector<int64_t> h_bytes_twin;
  DBuf<int32_t> tw_star, tw_K, pos_map;
  int32_t ntwin = 0;
  // twins on: stars with at least twin_min positions and a two-chain factor
  // run k_star_twin; per preconditioner like the split (the two forms round
  // differently); -1: measured at the first engine, 0: off
  int64_t twin_min = -1;
  // stars on the supernodal path besides those the band kernel cannot take:
  // measured when the first engine is created (or set by the caller) and then
  // shared by every engine, since the two kernels round differently and a
  // column's iterates must not depend on its batch; -1: not yet chosen
  int64_t split = -1;
  int32_t coarse_launch = -1;  // fixed coarse kernel and placement (kernel + 2 placement), -1: measured
  int32_t sn_beyond = -1;      // supernodal stars beyond LDS: 0 global memory, 1 vectors in LDS, -1 measured
  int64_t twin_force = -1;     // caller's twin threshold (0 off, > 0 positions), -1: measured
  int32_t queue_force = -1;    // caller's persistent band wavefronts (0 off), -1: measured
  // coarse
  // K_0^{-1}, symmetric, zero-padded to ld0 x ld0 (ld0 a multiple of 64): FP32 in the mixed form
  // unless the coarse factor's pivot ratio rules it out, else FP64
  DBuf<double> Kinv64, PTw, Pw;
  DBuf<float> Kinv32;
  // the same inverse stored once, in 64 x 64 tiles of its upper triangle
  DBuf<double> Ksym64;
  DBuf<float> Ksym32;
  DBuf<int2> sym_tiles;  // (I, J) of every tile
  int32_t sym_T = 0;     // ld0 / 64
  int64_t ld0 = 0;
  bool coarse32 = false;
  DBuf<int32_t> PTptr, PTdof, Pc;
  // internal dof order: free nodes grouped by coarse element (gather
  // locality); perm[internal] = canonical dof, iperm the inverse
  DBuf<int32_t> perm;
  std::vector<int32_t> perm_h, iperm_h;
  int64_t bytes = 0;
  // engines of sn_solve / sn_apply_*, one per width
  std::unique_ptr<Engine> solve_engine[5];
  // profiling
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free, ev_coarse;
  int64_t prof_iters = 0;
  ~DeviceState();
};

// Everything a batch of KC columns writes: vectors, per-column scalars, star
// slots, captured iteration graphs and streams. Engines never share these, so
// engines on the same preconditioner can run side by side.
struct Engine {
  Precond *pre = nullptr;
  DeviceState *d = nullptr;
  int kc = 1;
  DBuf<double> u, r, p, q, z, f, rH, c, partials, partials2;
  DBuf<double> cpart;  // 64 x KC partial blocks of the packed coarse product (T x T)
  DBuf<CgScalars> sc;
  DBuf<float> slots32;
  DBuf<double> slots64;
  CgScalars *host_sc = nullptr;  // pinned: last read-back, and the source of uploads
  // local solves, chosen by measurement (see tune_stars): the stars with the
  // longest band sweeps (and every star whose band exceeds 1024) run the
  // supernodal kernel on aux3, the others the band kernel on the solve stream
  // (narrow windows) and aux (wide windows)
  int32_t n_sn = 0;                            // stars on the supernodal path
  std::vector<int32_t> sn_list;                // those stars, longest first
  int64_t sweep_bytes = 0;                     // algorithmic bytes of one application (one column)
  // band launches: stars of the band path, narrow and wide windows, longest first
  DBuf<int32_t> b_narrow, b_wide;
  int32_t n_narrow = 0, n_wide = 0;
  // two-chain stars (twin ids, longest first), their vectors
  DBuf<int32_t> b_twin;
  int32_t n_twin = 0;
  DBuf<int64_t> tw_vs;
  DBuf<unsigned char> tw_scratch;
  int32_t star_cap = 0, star_lds = 0;          // resident band wavefronts per SIMD (0: no limit) and its LDS reservation
  bool star_lv = true;                         // band working vectors in LDS (where they fit)
  int32_t star_prio = 0;                       // band wavefronts of the longest stars at raised issue priority
  int32_t star_resident = 0;                   // > 0: narrow band sweeps as that many persistent wavefronts
  DBuf<int32_t> squeue;                        // their star queues (counters, zero between launches)
  // supernodal launches: 0 (lds_cap per workgroup), 1 (more LDS), 2 (global memory)
  struct StarLaunch {
    DBuf<int32_t> order;
    int32_t count = 0, lds = 0;
  } sl[3];
  DBuf<unsigned char> vscratch;                // vectors of the launch-2 stars
  DBuf<int64_t> st_vs;
  int32_t star_cw = 1, star_nteam = 1, star_lcap = 0;
  int32_t star_gteam = 4;                      // wavefronts per star of the global-memory launch (4 or 16)
  bool sn_iglobal = false;                     // stars beyond LDS: vectors in LDS, index part in global memory
  int32_t star_iglobal = 0;                    // such stars in the plan
  double star_us = 0.0;
  bool coarse_first = false;  // coarse solve before the sweeps rather than beside them
  bool coarse_w1 = false;     // one-wavefront coarse kernel (else 16-wavefront workgroups)
  bool coarse_sym = false;    // the packed symmetric coarse kernel (fixed per preconditioner)
  bool coarse_late = false;   // beside the sweeps: queued after them (else before)
  double b_us = 0.0;
  bool sc_dirty = false;         // host_sc changed since the last upload
  hipStream_t own = nullptr;     // the engine's stream (and graph capture)
  hipStream_t aux = nullptr;     // wide band stars run beside the narrow ones
  hipStream_t aux2 = nullptr;    // the coarse solve runs beside the star sweeps
  hipStream_t aux3 = nullptr;    // the supernodal stars run beside the band ones
  hipStream_t aux4 = nullptr;    // the two-chain stars run beside the other band stars
  hipEvent_t fork4 = nullptr, join4 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, fork2 = nullptr, join2 = nullptr, fork3 = nullptr, join3 = nullptr;
  hipEvent_t tick_done = nullptr;
  bool in_flight = false;
  std::vector<hipGraphExec_t> graphs;  // graphs[i] runs 2^i iterations on `own`-captured work
  std::vector<hipGraph_t> graph_defs;
  int64_t bytes = 0;
  ~Engine() {
    if (in_flight && tick_done) (void)hipEventSynchronize(tick_done);
    for (auto &g : graphs)
      if (g) (void)hipGraphExecDestroy(g);
    for (auto &g : graph_defs)
      if (g) (void)hipGraphDestroy(g);
    if (host_sc) (void)hipHostFree(host_sc);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (fork2) (void)hipEventDestroy(fork2);
    if (join2) (void)hipEventDestroy(join2);
    if (fork3) (void)hipEventDestroy(fork3);
    if (join3) (void)hipEventDestroy(join3);
    if (aux3) (void)hipStreamDestroy(aux3);
    if (fork4) (void)hipEventDestroy(fork4);
    if (join4) (void)hipEventDestroy(join4);
    if (aux4) (void)hipStreamDestroy(aux4);
    if (tick_done) (void)hipEventDestroy(tick_done);
    if (aux2) (void)hipStreamDestroy(aux2);
    if (aux) (void)hipStreamDestroy(aux);
    if (own) (void)hipStreamDestroy(own);
  }
};

DeviceState::~DeviceState() {
  for (auto &e : solve_engine) e.reset();
  for (auto &e : ev_used) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto &e : ev_coarse) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto &e : ev_free) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (the array's name is a host-side stand-in, not a device address).
void *scratch_ptr() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(SN_EDEVICE, "device id out of range for the workspace table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      fail(SN_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

void device_release(DeviceState *d) { delete d; }
void DeviceDeleter::operator()(DeviceState *d) const { delete d; }

namespace {

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
inline unsigned grid_for(int64_t n) { return std::max(1u, std::min<unsigned>(kMaxGrid, nblk(n))); }

int window_regs(int band) {
  const int q = (band + 63) / 64;
  for (int w = 1; w <= 16; w *= 2)
    if (q <= w) return w;
  return -1;
}

// Pack one sweep stream of a star: steps in groups of SG (the first step of
// every group a multiple of SG), values divided by the step's pivot. Lane l
// and window register q read slot u = ((l - j0 - 1) mod 64) + 64 q of the group
// with first step j0 (mod 64); slot u holds, for k = 0..SG-1, entry
// t = 64 q + ((u mod 64 - k) mod 64) of step j0 + k (zero past the step's width).
// The group stores slots 0..W-1, W one past the last non-zero slot, right after
// the previous group; `widths` gets W (16-bit) per group, so a group's offset is
// the sum of the widths before it.
template <typename T>
void pack_stream(const std::vector<int32_t> &width, const std::vector<double> &vals, const std::vector<double> &inv,
                 int SG, int Q, std::vector<T> &out, std::vector<uint16_t> &widths) {
  const int n = (int)width.size();
  std::vector<int64_t> start((size_t)n + 1, 0);
  for (int j = 0; j < n; ++j) start[j + 1] = start[j] + width[j];
  auto entry = [&](int j, int slot, int k) -> double {
    const int jj = j + k;
    if (jj >= n) return 0.0;
    const int q = slot / 64, u = slot % 64;
    const int t = 64 * q + ((u - k) & 63);
    if (t >= width[jj]) return 0.0;
    return vals[(size_t)(start[jj] + t)] * inv[jj];
  };
  for (int j0 = 0; j0 < n; j0 += SG) {
    int W = 0;
    for (int slot = 0; slot < 64 * Q; ++slot)
      for (int k = 0; k < SG; ++k)
        if (entry(j0, slot, k) != 0.0) W = slot + 1;
    widths.push_back((uint16_t)W);
    for (int slot = 0; slot < W; ++slot)
      for (int k = 0; k < SG; ++k) out.push_back((T)entry(j0, slot, k));
  }
  // zero widths past the end: the sweep reads whole blocks of widths up to
  // four blocks ahead
  const int GPB = 64 / SG;
  const size_t ng = (size_t)(n + SG - 1) / SG;
  const size_t padded = (ng + GPB - 1) / GPB * GPB + 4 * GPB;
  widths.resize(widths.size() + (padded - ng), 0);
}

// One star's supernodal blob: header, level table, position records, 16-bit index lists
// (padded to 16 bytes: the index part), then the values of the S_k in T
// (padded to 16 bytes).
// The supernodal layout indexes positions and update slots with 16 bits and
// the values of a star with 31.
bool sn_layout_fits(const SnFactor &F) {
  return F.n < 65536 && F.nu < 65536 && (int64_t)F.S.size() < ((int64_t)1 << 31);
}

template <typename T>
void pack_blob(const SnFactor &F, const std::vector<int32_t> &bpos, std::vector<unsigned char> &out,
               uint32_t &idx_bytes, uint32_t &val_bytes) {
  if (F.n >= 65536 || F.nu >= 65536)
    fail(SN_EINVAL, "star too large for 16-bit local indices (" + std::to_string(F.n) + " positions, " +
                        std::to_string(F.nu) + " updates)");
  if ((int64_t)F.S.size() >= (int64_t)1 << 31) fail(SN_EINVAL, "star factor too large");
  auto a16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
  SnHeader h{};
  h.n = (uint32_t)F.n;
  h.nsn = (uint32_t)F.nsn;
  h.nu = (uint32_t)F.nu;
  h.nlev = (uint32_t)F.nlev;
  size_t off = sizeof(SnHeader);
  h.off_lev = (uint32_t)off;
  off = a16(off + 4 * ((size_t)F.nlev + 1));
  h.off_pos = (uint32_t)off;
  off += sizeof(SnPos) * (size_t)F.n;
  h.off_R = (uint32_t)off;
  off += 2 * (size_t)F.nu;
  h.off_alist = (uint32_t)off;
  off += 2 * (size_t)F.nu;
  h.off_bpos = (uint32_t)off;
  off += 2 * (size_t)F.n;
  h.idx_bytes = (uint32_t)a16(off);
  h.val_bytes = (uint32_t)a16(F.S.size() * sizeof(T));
  const size_t base = out.size();
  out.resize(base + h.idx_bytes + h.val_bytes, 0);
  unsigned char *b = out.data() + base;
  std::memcpy(b, &h, sizeof(h));
  uint32_t *lev = reinterpret_cast<uint32_t *>(b + h.off_lev);
  for (int32_t l = 0; l <= F.nlev; ++l) lev[l] = (uint32_t)F.lev_pos[l];
  for (int32_t p = 0; p < F.n; ++p) {
    const int32_t k = F.snpos[p];
    SnPos r{};
    r.sbase = (uint32_t)F.sbase[k];
    r.c0 = (uint16_t)F.c0[k];
    r.w = (uint16_t)F.w[k];
    r.h = (uint16_t)F.h[k];
    r.ubase = (uint16_t)F.ubase[k];
    r.a0 = (uint16_t)F.aptr[p];
    r.a1 = (uint16_t)F.aptr[p + 1];
    std::memcpy(b + h.off_pos + sizeof(SnPos) * (size_t)p, &r, sizeof(r));
  }
  auto put16 = [&](uint32_t o, const std::vector<int32_t> &v) {
    uint16_t *d16 = reinterpret_cast<uint16_t *>(b + o);
    for (size_t i = 0; i < v.size(); ++i) d16[i] = (uint16_t)v[i];
  };
  put16(h.off_R, F.R);
  put16(h.off_alist, F.alist);
  put16(h.off_bpos, bpos);
  T *val = reinterpret_cast<T *>(b + h.idx_bytes);
  for (size_t i = 0; i < F.S.size(); ++i) val[i] = (T)F.S[i];
  idx_bytes = h.idx_bytes;
  val_bytes = h.val_bytes;
}

// Both layouts of every star. Slots follow the band order of each star; the
// supernodal blob maps its positions to them (bpos). Per star the algorithmic
// bytes of one solve of one column are kept for each path: the structural
// non-zeros of that path's factor times the factor precision (twice for the
// band path, whose two sweeps stream their own copies; once for the supernodal
// path, which reads its factor from HBM once and keeps it in LDS or cache for
// the second solve), and per position the dof index, the FP64 gather of r and
// the slot write.
template <typename T>
void upload_stars(DeviceState &d, const Precond &pre, const HostFactors &hf, sn_factor_info &fi) {
  constexpr int SG = 16 / (int)sizeof(T);
  const int64_t ns = (int64_t)hf.stars.size();
  const int64_t sT = sizeof(T);
  std::vector<int32_t> st_n(ns), st_vb(ns), st_q(ns), st_gb(ns), pos_dof;
  std::vector<uint16_t> f_hdr, b_hdr;
  std::vector<int64_t> st_fb(ns), st_bb(ns), st_blob(ns);
  std::vector<T> f_val, b_val, f_inv, b_inv;
  std::vector<unsigned char> blob;
  d.h_n.assign((size_t)ns, 0);
  d.h_q.assign((size_t)ns, 0);
  d.h_idx.assign((size_t)ns, 0);
  d.h_val.assign((size_t)ns, 0);
  d.h_nu.assign((size_t)ns, 0);
  d.h_sn_ok.assign((size_t)ns, 0);
  d.h_bytes_band.assign((size_t)ns, 0);
  d.h_bytes_sn.assign((size_t)ns, 0);
  int64_t tot = 0, nnz_md = 0, nnz_rcm = 0, env = 0, stored = 0, idx_tot = 0;
  int maxband = 0;
  for (int64_t s = 0; s < ns; ++s) {
    const StarFactor &F = hf.stars[s];
    const int q = window_regs(std::max(F.band, 1));
    st_n[s] = F.n;
    st_vb[s] = (int32_t)tot;
    st_q[s] = q < 0 ? 0 : q;
    d.h_q[s] = st_q[s];
    d.h_n[s] = F.n;
    st_gb[s] = (int32_t)f_hdr.size();
    maxband = std::max(maxband, F.band);
    d.maxn = std::max(d.maxn, F.n);
    // band streams (empty for a star whose band no window covers)
    std::vector<double> finv(F.invdiag), binv((size_t)F.n);
    for (int p = 0; p < F.n; ++p) binv[p] = F.invdiag[F.n - 1 - p];
    st_fb[s] = (int64_t)f_val.size();
    st_bb[s] = (int64_t)b_val.size();
    if (q > 0) {
      pack_stream<T>(F.width_fwd, F.colvals, finv, SG, q, f_val, f_hdr);
      pack_stream<T>(F.width_bwd, F.rowvals, binv, SG, q, b_val, b_hdr);
      if (f_hdr.size() != b_hdr.size()) fail(SN_EINVAL, "internal: header arrays out of step");
    }
    const int32_t *dofs = &pre.star_dofs[pre.star_ptr[s]];
    for (int p = 0; p < F.n; ++p) {
      pos_dof.push_back(d.iperm_h[dofs[F.perm[p]]]);
      f_inv.push_back((T)finv[p]);
      b_inv.push_back((T)binv[p]);
    }
    // supernodal blob, when the layout holds the star (else the star stays on
    // the band path); bpos maps its positions to the band positions (slots)
    d.h_bytes_band[s] = 2 * F.nnz_rcm * sT + (int64_t)F.n * (4 + 8 + sT);
    d.h_sn_ok[s] = sn_layout_fits(F.sn) ? 1 : 0;
    if (q <= 0 && !d.h_sn_ok[s])
      fail(SN_EINVAL, "star " + std::to_string(s) + " fits neither local-solve layout (band " +
                          std::to_string(F.band) + ", " + std::to_string(F.sn.nu) + " supernodal updates)");
    st_blob[s] = (int64_t)blob.size();
    if (d.h_sn_ok[s]) {
      std::vector<int32_t> band_of((size_t)F.n), bpos((size_t)F.n);
      for (int p = 0; p < F.n; ++p) band_of[F.perm[p]] = p;
      for (int p = 0; p < F.n; ++p) bpos[p] = band_of[F.sn.perm[p]];
      pack_blob<T>(F.sn, bpos, blob, d.h_idx[s], d.h_val[s]);
      d.h_nu[s] = (uint32_t)F.sn.nu;
      d.maxlev = std::max(d.maxlev, F.sn.nlev);
      d.h_bytes_sn[s] = F.sn.nnz * sT + (int64_t)F.n * (4 + 8 + sT);
      stored += (int64_t)F.sn.S.size();
      idx_tot += d.h_idx[s];
    } else {
      d.h_bytes_sn[s] = d.h_bytes_band[s];
    }
    tot += F.n;
    nnz_md += F.sn.nnz;
    nnz_rcm += F.nnz_rcm;
    env += F.env;
  }
  // the two chains of every star that has them (windows of 1-2 registers),
  // after the stars' own entries; pos_map gives each chain position the band
  // position it owns in its star (pads and the second chain's separator copy
  // own none)
  std::vector<int32_t> tw_star, tw_K, pos_map((size_t)tot, -1);
  d.h_twin.assign((size_t)ns, -1);
  d.h_twin_len.clear();
  d.h_bytes_twin.clear();
  int64_t ext = tot;
  for (int64_t s = 0; s < ns; ++s) {
    const StarFactor &F = hf.stars[s];
    const BandTwin &TW = F.twin;
    if (TW.K <= 0) continue;
    const int q2 = window_regs(std::max({TW.c[0].band, TW.c[1].band, 1}));
    if (q2 < 1 || q2 > 2) continue;
    const int32_t t = (int32_t)tw_star.size();
    const int32_t n2 = TW.K + TW.s;
    tw_star.push_back((int32_t)s);
    tw_K.push_back(TW.K);
    d.h_twin[s] = t;
    d.h_twin_len.push_back(n2);
    d.h_bytes_twin.push_back(2 * (TW.c[0].nnz + TW.c[1].nnz) * sT + (int64_t)F.n * (4 + 8 + sT));
    const int32_t *dofs = &pre.star_dofs[pre.star_ptr[s]];
    for (int c = 0; c < 2; ++c) {
      const BandChain &C = TW.c[c];
      st_n.push_back(n2);
      st_vb.push_back((int32_t)ext);
      st_q.push_back(q2);
      st_gb.push_back((int32_t)f_hdr.size());
      st_fb.push_back((int64_t)f_val.size());
      st_bb.push_back((int64_t)b_val.size());
      std::vector<double> binv((size_t)n2);
      for (int p = 0; p < n2; ++p) binv[p] = C.invdiag[n2 - 1 - p];
      pack_stream<T>(C.width_fwd, C.colvals, C.invdiag, SG, q2, f_val, f_hdr);
      pack_stream<T>(C.width_bwd, C.rowvals, binv, SG, q2, b_val, b_hdr);
      if (f_hdr.size() != b_hdr.size()) fail(SN_EINVAL, "internal: header arrays out of step");
      for (int p = 0; p < n2; ++p) {
        const int32_t bp = C.bpos[p];
        const bool own = bp >= 0 && !(c == 1 && p >= TW.K);
        pos_dof.push_back(own ? d.iperm_h[dofs[F.perm[bp]]] : -1);
        pos_map.push_back(own ? bp : -1);
        f_inv.push_back((T)C.invdiag[p]);
        b_inv.push_back((T)binv[p]);
      }
      ext += n2;
    }
  }
  d.ntwin = (int32_t)tw_star.size();
  if (ext >= (int64_t)1 << 31 || (int64_t)std::max(f_val.size(), b_val.size()) >= (int64_t)1 << 31)
    fail(SN_EINVAL, "star streams too large for 32-bit offsets");
  // zero region: band lanes past a group's width load from here (64*Q lanes of
  // SG values, Q <= 16)
  const size_t slack = (size_t)64 * 16 * SG + 64;
  d.f_zero = (int64_t)f_val.size();
  d.b_zero = (int64_t)b_val.size();
  f_val.resize(f_val.size() + slack, T(0));
  b_val.resize(b_val.size() + slack, T(0));
  // dof -> slots in ascending star order
  std::vector<int32_t> slot_of((size_t)d.npad * d.nv, -1);
  {
    std::vector<int32_t> cnt((size_t)d.n, 0);
    for (int64_t s = 0; s < ns; ++s)
      for (int p = 0; p < st_n[s]; ++p) {
        const int32_t dof = pos_dof[st_vb[s] + p];
        if (cnt[dof] >= d.nv) fail(SN_EINVAL, "a dof lies in more stars than its element has mesh nodes");
        slot_of[(size_t)dof * d.nv + cnt[dof]++] = st_vb[s] + p;
      }
  }
  d.nstars = (int32_t)ns;
  d.slot_count = tot;
  d.st_n.upload(st_n);
  d.st_vb.upload(st_vb);
  d.st_q.upload(st_q);
  d.st_gb.upload(st_gb);
  d.st_fb.upload(st_fb);
  d.st_bb.upload(st_bb);
  d.pos_dof.upload(pos_dof);
  d.pos_map.upload(pos_map);
  d.tw_star.upload(tw_star);
  d.tw_K.upload(tw_K);
  d.f_hdr.upload(f_hdr);
  d.b_hdr.upload(b_hdr);
  d.slot_of.upload(slot_of);
  d.blob.upload(blob);
  d.st_blob.upload(st_blob);
  int64_t stream_bytes;
  if constexpr (sizeof(T) == 4) {
    d.f_inv32.upload(f_inv);
    d.b_inv32.upload(b_inv);
    d.f_val32.upload(f_val);
    d.b_val32.upload(b_val);
    stream_bytes = (int64_t)(d.f_val32.bytes() + d.b_val32.bytes());
  } else {
    d.f_inv64.upload(f_inv);
    d.b_inv64.upload(b_inv);
    d.f_val64.upload(f_val);
    d.b_val64.upload(b_val);
    stream_bytes = (int64_t)(d.f_val64.bytes() + d.b_val64.bytes());
  }
  fi.star_factor_nnz = nnz_md;
  fi.star_rcm_nnz = nnz_rcm;
  fi.star_envelope = env;
  fi.star_stored = stored;
  fi.star_blob_bytes = (int64_t)blob.size();
  fi.star_index_bytes = idx_tot;
  fi.star_stream_bytes = stream_bytes;
  fi.max_levels = d.maxlev;
  fi.max_band = maxband;
  fi.max_star_dofs = d.maxn;
  fi.sweep_bytes = 0;
  for (int64_t s = 0; s < ns; ++s) fi.sweep_bytes += d.h_q[s] > 0 ? d.h_bytes_band[s] : d.h_bytes_sn[s];
  fi.sweep_bytes_sn = 0;
  for (int64_t s = 0; s < ns; ++s) fi.sweep_bytes_sn += d.h_bytes_sn[s];
  fi.sweep_flops = 4 * nnz_md;
}

}  // namespace

void device_setup(Precond &pre, const HostFactors &hf, int precision) {
  double max_ratio = 1.0;
  for (const StarFactor &F : hf.stars) max_ratio = std::max({max_ratio, F.pivot_ratio, F.sn.pivot_ratio});
  const int requested = precision;
  if (precision != SN_PREC_FP64 && precision != SN_PREC_FP32_STARS && precision != SN_PREC_FP32_STARS_COARSE)
    fail(SN_EINVAL, "unknown precision " + std::to_string(precision));
  const bool want_coarse32 = precision == SN_PREC_FP32_STARS_COARSE;
  if (precision == SN_PREC_FP32_STARS_COARSE) precision = SN_PREC_FP32_STARS;
  if (precision == SN_PREC_FP32_STARS && max_ratio * std::ldexp(1.0, -24) > 0.05) precision = SN_PREC_FP64;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(SN_EDEVICE, "no HIP device available");
  auto d = std::make_unique<DeviceState>();
  HIPCHK(hipGetDevice(&d->device));
  (void)scratch_ptr();  // the workspace address of this device, while it is current
  const System &sys = *pre.sys;
  d->precision = precision;
  d->n = sys.n;
  d->npad = (sys.n + kBlock - 1) / kBlock * kBlock;
  d->m0 = pre.m0;
  d->nv = pre.nvert_per_elem;
  if (d->nv != 4 && d->nv != 8) fail(SN_EINVAL, "coarse elements must have 4 (2D) or 8 (3D) vertices");
  const int64_t n = sys.n, npad = d->npad;
  if (n >= (int64_t)1 << 30) fail(SN_EINVAL, "system too large for 32-bit indices");
  sn_factor_info fi{};

  // internal order: free nodes sorted by the mesh element that holds them
  // (lexicographic), then by index; the components of a node stay together.
  // Rows, star gathers and the slot accumulation then touch nearby memory.
  {
    const Network &net = *sys.net;
    const int dim = net.dim, nc = sys.ncomp;
    const int64_t nf = (int64_t)sys.free_node.size();
    std::vector<int64_t> cell((size_t)nf);
    for (int64_t f = 0; f < nf; ++f) {
      const double *x = &net.x[(size_t)sys.free_node[f] * dim];
      int64_t c = 0;
      for (int k = dim - 1; k >= 0; --k) {
        int64_t e = (int64_t)std::floor(x[k] * pre.nH);
        e = std::min<int64_t>(std::max<int64_t>(e, 0), pre.nH - 1);
        c = c * pre.nH + e;
      }
      cell[f] = c;
    }
    std::vector<int32_t> order((size_t)nf);
    for (int64_t f = 0; f < nf; ++f) order[f] = (int32_t)f;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cell[a] < cell[b]; });
    d->perm_h.assign((size_t)n, 0);
    d->iperm_h.assign((size_t)n, 0);
    for (int64_t i = 0; i < nf; ++i)
      for (int c = 0; c < nc; ++c) {
        const int32_t can = (int32_t)(order[i] * nc + c), in = (int32_t)(i * nc + c);
        d->perm_h[in] = can;
        d->iperm_h[can] = in;
      }
    d->perm.upload(d->perm_h);
  }
  const std::vector<int32_t> &iperm = d->iperm_h, &perm = d->perm_h;

  // sliced ELL
  {
    const int ns = (int)(npad / kSlice);
    d->nslices = ns;
    std::vector<int32_t> sptr(ns), slen(ns);
    int64_t tot = 0;
    for (int s = 0; s < ns; ++s) {
      int w = 0;
      for (int l = 0; l < kSlice; ++l) {
        const int64_t ri = (int64_t)s * kSlice + l;
        if (ri < n) {
          const int64_t r = perm[ri];
          w = std::max<int>(w, (int)(sys.rowptr[r + 1] - sys.rowptr[r]));
        }
      }
      sptr[s] = (int32_t)tot;
      slen[s] = w;
      tot += (int64_t)w * kSlice;
    }
    if (tot >= (int64_t)1 << 31) fail(SN_EINVAL, "matrix too large for 32-bit offsets");
    std::vector<int32_t> col((size_t)tot);
    std::vector<double> val((size_t)tot, 0.0);
    for (int s = 0; s < ns; ++s)
      for (int l = 0; l < kSlice; ++l) {
        const int64_t ri = (int64_t)s * kSlice + l;
        const int64_t r = ri < n ? perm[ri] : 0;
        const int64_t len = ri < n ? sys.rowptr[r + 1] - sys.rowptr[r] : 0;
        for (int c = 0; c < slen[s]; ++c) {
          const size_t e = (size_t)sptr[s] + (size_t)c * kSlice + l;
          if (c < len) {
            col[e] = iperm[sys.col[sys.rowptr[r] + c]];
            val[e] = sys.val[sys.rowptr[r] + c];
          } else {
            col[e] = (int32_t)std::min<int64_t>(ri, n - 1);
            val[e] = 0.0;
          }
        }
      }
    d->sptr.upload(sptr);
    d->slen.upload(slen);
    d->col.upload(col);
    d->val.upload(val);
  }

  // stars
  if (precision == SN_PREC_FP32_STARS) upload_stars<float>(*d, pre, hf, fi);
  else upload_stars<double>(*d, pre, hf, fi);

  // coarse operator
  const int nc = sys.ncomp, nv = d->nv;
  if (d->m0 > 0) {
    // symmetric (the mean of the two computed triangles) and padded
    const int64_t m0 = d->m0, ld = (m0 + 63) / 64 * 64;
    d->ld0 = ld;
    d->coarse32 = want_coarse32 && precision == SN_PREC_FP32_STARS &&
                  hf.coarse_pivot_ratio * std::ldexp(1.0, -24) <= 0.05;
    auto sym = [&](int64_t i, int64_t j) {
      return 0.5 * (hf.coarse_inv[(size_t)(i * m0 + j)] + hf.coarse_inv[(size_t)(j * m0 + i)]);
    };
    if (d->coarse32) {
      std::vector<float> A((size_t)(ld * ld), 0.0f);
      for (int64_t i = 0; i < m0; ++i)
        for (int64_t j = 0; j < m0; ++j) A[(size_t)(i * ld + j)] = (float)sym(i, j);
      d->Kinv32.upload(A);
    } else {
      std::vector<double> A((size_t)(ld * ld), 0.0);
      for (int64_t i = 0; i < m0; ++i)
        for (int64_t j = 0; j < m0; ++j) A[(size_t)(i * ld + j)] = sym(i, j);
      d->Kinv64.upload(A);
    }
    // tiles (I <= J) of the upper triangle: strip p, lane l = 16 k + 4 y + i,
    // value s is row 4 p + i, column 16 y + 4 k + s of the tile
    {
      const int64_t T = ld / 64;
      d->sym_T = (int32_t)T;
      std::vector<int2> tiles;
      for (int64_t I = 0; I < T; ++I)
        for (int64_t J = I; J < T; ++J) tiles.push_back(make_int2((int)I, (int)J));
      auto fill_tiles = [&](auto *out) {
        for (size_t q = 0; q < tiles.size(); ++q)
          for (int p = 0; p < 16; ++p)
            for (int l = 0; l < 64; ++l)
              for (int sv = 0; sv < 4; ++sv) {
                const int ii = l & 3, yy = (l >> 2) & 3, kk = l >> 4;
                const int64_t row = 64 * (int64_t)tiles[q].x + 4 * p + ii;
                const int64_t col = 64 * (int64_t)tiles[q].y + 16 * yy + 4 * kk + sv;
                const double v = row < m0 && col < m0 ? sym(row, col) : 0.0;
                out[q * kSymTile + (size_t)p * 256 + (size_t)l * 4 + sv] = (std::remove_pointer_t<decltype(out)>)v;
              }
      };
      if (d->coarse32) {
        std::vector<float> A(tiles.size() * kSymTile);
        fill_tiles(A.data());
        d->Ksym32.upload(A);
      } else {
        std::vector<double> A(tiles.size() * kSymTile);
        fill_tiles(A.data());
        d->Ksym64.upload(A);
      }
      d->sym_tiles.upload(tiles);
    }
    // P per dof (npad x nv) and P^T as CSR over coarse dofs
    std::vector<int32_t> Pc((size_t)npad * nv, -1);
    std::vector<double> Pw((size_t)npad * nv, 0.0);
    std::vector<int32_t> cnt((size_t)d->m0 + 1, 0);
    const int64_t nf = (int64_t)sys.free_node.size();
    for (int64_t f = 0; f < nf; ++f)
      for (int b = 0; b < nv; ++b) {
        const int32_t g = pre.vert_coarse[pre.Pvert[(size_t)f * nv + b]];
        if (g < 0) continue;
        for (int c = 0; c < nc; ++c) {
          const int64_t dof = iperm[f * nc + c];
          Pc[(size_t)dof * nv + b] = g * nc + c;
          Pw[(size_t)dof * nv + b] = pre.Pphi[(size_t)f * nv + b];
          ++cnt[(size_t)g * nc + c + 1];
        }
      }
    for (int64_t c = 0; c < d->m0; ++c) cnt[c + 1] += cnt[c];
    std::vector<int32_t> PTdof((size_t)cnt[d->m0]);
    std::vector<double> PTw((size_t)cnt[d->m0]);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t dof = 0; dof < n; ++dof)
      for (int b = 0; b < nv; ++b) {
        const int32_t c = Pc[(size_t)dof * nv + b];
        if (c < 0) continue;
        PTdof[fill[c]] = (int32_t)dof;
        PTw[fill[c]++] = Pw[(size_t)dof * nv + b];
      }
    d->Pc.upload(Pc);
    d->Pw.upload(Pw);
    d->PTptr.upload(cnt);
    d->PTdof.upload(PTdof);
    d->PTw.upload(PTw);
  } else {
    d->Pc.upload(std::vector<int32_t>((size_t)npad * nv, -1));
    d->Pw.upload(std::vector<double>((size_t)npad * nv, 0.0));
  }
  HIPCHK(hipDeviceSynchronize());
  d->bytes = (int64_t)(d->sptr.bytes() + d->slen.bytes() + d->col.bytes() + d->val.bytes() + d->perm.bytes() +
                       d->st_vb.bytes() + d->pos_dof.bytes() + d->slot_of.bytes() + d->st_n.bytes() +
                       d->st_q.bytes() + d->st_gb.bytes() + d->st_fb.bytes() + d->st_bb.bytes() + d->f_hdr.bytes() +
                       d->b_hdr.bytes() + d->f_inv32.bytes() + d->b_inv32.bytes() + d->f_val32.bytes() +
                       d->b_val32.bytes() + d->f_inv64.bytes() + d->b_inv64.bytes() + d->f_val64.bytes() +
                       d->b_val64.bytes() + d->blob.bytes() + d->st_blob.bytes() + d->Kinv64.bytes() +
                       d->Kinv32.bytes() + d->Ksym64.bytes() + d->Ksym32.bytes() + d->sym_tiles.bytes() +
                       d->Pc.bytes() + d->Pw.bytes() + d->PTptr.bytes() + d->PTdof.bytes() +
                       d->PTw.bytes());
  const int64_t nnz = (int64_t)sys.col.size();
  fi.spmv_bytes = nnz * (8 + 4 + 8) + n * 8;
  fi.max_pivot_ratio = max_ratio;
  fi.star_precision = precision;
  fi.coarse_bytes = (int64_t)(d->Kinv64.bytes() + d->Kinv32.bytes() + d->Ksym64.bytes() + d->Ksym32.bytes());
  fi.coarse_precision = d->coarse32 ? SN_PREC_FP32_STARS_COARSE : SN_PREC_FP64;
  fi.coarse_pivot_ratio = hf.coarse_pivot_ratio;
  fi.device_bytes = d->bytes;
  fi.factor_seconds = hf.seconds;
  pre.finfo = fi;
  pre.precision = requested;
  pre.dev.reset(d.release());
}

// ---------------------------------------------------------------------------
// star kernel dispatch over the column counts (instantiated in star_inst.hip)
// ---------------------------------------------------------------------------
template <typename T>
static void launch_band_kc(int kc, const StarArgs &a, bool wide, const double *r, const CgScalars *sc, int sel,
                           hipStream_t s) {
  switch (kc) {
    case 1: launch_star_t<T, 1>(a, wide, r, sc, sel, s); break;
    case 2: launch_star_t<T, 2>(a, wide, r, sc, sel, s); break;
    case 4: launch_star_t<T, 4>(a, wide, r, sc, sel, s); break;
    case 8: launch_star_t<T, 8>(a, wide, r, sc, sel, s); break;
    case 16: launch_star_t<T, 16>(a, wide, r, sc, sel, s); break;
    default: fail(SN_EINVAL, "unsupported column count");
  }
}
template <typename T, int KC>
static void launch_sn_cw(int cw, const SnArgs &a, int nteam, bool global, const double *r, const CgScalars *sc,
                         int sel, hipStream_t s) {
  if (cw == 1) launch_sn_t<T, KC, 1>(a, nteam, global, r, sc, sel, s);
  else if constexpr (KC >= 2) {
    if (cw == 2) launch_sn_t<T, KC, 2>(a, nteam, global, r, sc, sel, s);
    else if constexpr (KC >= 4) {
      if (cw == 4) launch_sn_t<T, KC, 4>(a, nteam, global, r, sc, sel, s);
      else fail(SN_EINVAL, "unsupported columns per wavefront");
    } else fail(SN_EINVAL, "unsupported columns per wavefront");
  } else fail(SN_EINVAL, "unsupported columns per wavefront");
}
template <typename T>
static void launch_sn_kc(int kc, int cw, const SnArgs &a, int nteam, bool global, const double *r,
                         const CgScalars *sc, int sel, hipStream_t s) {
  switch (kc) {
    case 1: launch_sn_cw<T, 1>(cw, a, nteam, global, r, sc, sel, s); break;
    case 2: launch_sn_cw<T, 2>(cw, a, nteam, global, r, sc, sel, s); break;
    case 4: launch_sn_cw<T, 4>(cw, a, nteam, global, r, sc, sel, s); break;
    case 8: launch_sn_cw<T, 8>(cw, a, nteam, global, r, sc, sel, s); break;
    case 16: launch_sn_cw<T, 16>(cw, a, nteam, global, r, sc, sel, s); break;
    default: fail(SN_EINVAL, "unsupported column count");
  }
}

namespace {

template <typename F>
void with_kc(int kc, F &&f) {
  switch (kc) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: fail(SN_EINVAL, "unsupported column count " + std::to_string(kc));
  }
}

template <typename T>
static void launch_twin_kc(int kc, const StarArgs &a, const double *r, const CgScalars *sc, int sel, hipStream_t s) {
  switch (kc) {
    case 1: launch_twin_t<T, 1>(a, r, sc, sel, s); break;
    case 2: launch_twin_t<T, 2>(a, r, sc, sel, s); break;
    case 4: launch_twin_t<T, 4>(a, r, sc, sel, s); break;
    case 8: launch_twin_t<T, 8>(a, r, sc, sel, s); break;
    case 16: launch_twin_t<T, 16>(a, r, sc, sel, s); break;
    default: fail(SN_EINVAL, "unsupported column count");
  }
}

StarArgs band_args(DeviceState &d, Engine &e, bool wide) {
  StarArgs a{};
  a.nstars = wide ? e.n_wide : e.n_narrow;
  a.order = wide ? e.b_wide.p : e.b_narrow.p;
  a.st_n = d.st_n.p;
  a.st_vb = d.st_vb.p;
  a.st_q = d.st_q.p;
  a.st_gb = d.st_gb.p;
  a.st_fb = d.st_fb.p;
  a.st_bb = d.st_bb.p;
  a.pos_dof = d.pos_dof.p;
  a.f_hdr = d.f_hdr.p;
  a.b_hdr = d.b_hdr.p;
  a.f_zero = d.f_zero;
  a.b_zero = d.b_zero;
  a.lds_reserve = e.star_lds;
  a.maxn = d.maxn;
  a.use_lds = e.star_lv ? 1 : 0;
  a.n_prio = e.star_prio;
  a.n_resident = wide ? 0 : e.star_resident;
  a.queue = e.squeue.p;
  a.unit0 = d.nstars;
  a.tw_star = d.tw_star.p;
  a.tw_K = d.tw_K.p;
  a.pos_map = d.pos_map.p;
  a.tw_vs = e.tw_vs.p;
  a.tw_scratch = e.tw_scratch.p;
  if (d.precision == SN_PREC_FP32_STARS) {
    a.f_inv = d.f_inv32.p;
    a.b_inv = d.b_inv32.p;
    a.f_val = d.f_val32.p;
    a.b_val = d.b_val32.p;
    a.slots = e.slots32.p;
  } else {
    a.f_inv = d.f_inv64.p;
    a.b_inv = d.b_inv64.p;
    a.f_val = d.f_val64.p;
    a.b_val = d.b_val64.p;
    a.slots = e.slots64.p;
  }
  return a;
}

SnArgs sn_args(DeviceState &d, Engine &e, int which) {
  SnArgs a{};
  a.nstars = e.sl[which].count;
  a.lds_bytes = e.sl[which].lds;
  a.order = e.sl[which].order.p;
  a.blob = d.blob.p;
  a.st_blob = d.st_blob.p;
  a.st_pos = d.st_vb.p;
  a.pos_dof = d.pos_dof.p;
  a.slots = d.precision == SN_PREC_FP32_STARS ? (void *)e.slots32.p : (void *)e.slots64.p;
  a.vscratch = e.vscratch.p;
  a.st_vs = e.st_vs.p;
  return a;
}

// band sweeps: narrow windows on s, wide windows beside them on aux
void launch_band(Engine &e, const double *r, int sel, hipStream_t s) {
  DeviceState &d = *e.d;
  const bool f32 = d.precision == SN_PREC_FP32_STARS;
  auto L = [&](bool wide, hipStream_t st) {
    const StarArgs a = band_args(d, e, wide);
    if (f32) launch_band_kc<float>(e.kc, a, wide, r, e.sc.p, sel, st);
    else launch_band_kc<double>(e.kc, a, wide, r, e.sc.p, sel, st);
  };
  // the two-chain stars (the longest) first, beside the others on aux4
  if (e.n_twin > 0) {
    StarArgs a = band_args(d, e, false);
    a.nstars = e.n_twin;
    a.order = e.b_twin.p;
    const bool alone = e.n_wide == 0 && e.n_narrow == 0;
    const hipStream_t ts = alone ? s : e.aux4;
    if (!alone) {
      HIPCHK(hipEventRecord(e.fork4, s));
      HIPCHK(hipStreamWaitEvent(e.aux4, e.fork4, 0));
    }
    if (f32) launch_twin_kc<float>(e.kc, a, r, e.sc.p, sel, ts);
    else launch_twin_kc<double>(e.kc, a, r, e.sc.p, sel, ts);
    if (!alone) HIPCHK(hipEventRecord(e.join4, e.aux4));
  }
  if (e.n_wide > 0 && e.n_narrow > 0) {
    HIPCHK(hipEventRecord(e.fork, s));
    HIPCHK(hipStreamWaitEvent(e.aux, e.fork, 0));
    L(true, e.aux);
    HIPCHK(hipEventRecord(e.join, e.aux));
    L(false, s);
    HIPCHK(hipStreamWaitEvent(s, e.join, 0));
  } else if (e.n_wide > 0) {
    L(true, s);
  } else if (e.n_narrow > 0) {
    L(false, s);
  }
  if (e.n_twin > 0 && (e.n_wide > 0 || e.n_narrow > 0)) HIPCHK(hipStreamWaitEvent(s, e.join4, 0));
}

// supernodal solves: the launches that need the most resources first
void launch_sn(Engine &e, const double *r, int sel, hipStream_t s) {
  DeviceState &d = *e.d;
  const bool f32 = d.precision == SN_PREC_FP32_STARS;
  for (int which = 2; which >= 0; --which) {
    if (e.sl[which].count == 0) continue;
    const SnArgs a = sn_args(d, e, which);
    const int nt = which == 2 ? e.star_gteam : e.star_nteam;
    if (f32) launch_sn_kc<float>(e.kc, e.star_cw, a, nt, which == 2, r, e.sc.p, sel, s);
    else launch_sn_kc<double>(e.kc, e.star_cw, a, nt, which == 2, r, e.sc.p, sel, s);
  }
}

// local solves of the selected columns (a workgroup returns at once when none
// of its columns is selected): the supernodal stars on aux3 beside the band
// stars
void launch_stars(Engine &e, const double *r, int sel, hipStream_t s) {
  DeviceState &d = *e.d;
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (d.profiling) {
    if (d.ev_free.empty()) {
      HIPCHK(hipEventCreate(&ev.first));
      HIPCHK(hipEventCreate(&ev.second));
    } else {
      ev = d.ev_free.back();
      d.ev_free.pop_back();
    }
    HIPCHK(hipEventRecord(ev.first, s));
  }
  const bool band = e.n_narrow + e.n_wide + e.n_twin > 0, sn = e.n_sn > 0;
  if (band && sn) {
    HIPCHK(hipEventRecord(e.fork3, s));
    HIPCHK(hipStreamWaitEvent(e.aux3, e.fork3, 0));
    launch_sn(e, r, sel, e.aux3);
    HIPCHK(hipEventRecord(e.join3, e.aux3));
    launch_band(e, r, sel, s);
    HIPCHK(hipStreamWaitEvent(s, e.join3, 0));
  } else if (sn) {
    launch_sn(e, r, sel, s);
  } else {
    launch_band(e, r, sel, s);
  }
  if (d.profiling) {
    HIPCHK(hipEventRecord(ev.second, s));
    d.ev_used.push_back(ev);
  }
}

// z = B r on the selected columns; with dot, r.z -> rho, beta (second half)
// conv: the convergence test of the first half (r.r partials in partials2) is
// left to the restriction, which then runs before everything else of B
bool coarse_runs_first(const Engine &e) { return e.d->m0 > 0 && (e.coarse_first || e.d->profiling); }

void launch_B(Engine &e, const double *r, double *z, int sel, bool dot, hipStream_t s, bool conv) {
  DeviceState &d = *e.d;
  if (conv && !coarse_runs_first(e))
    fail(SN_EINVAL, "internal: convergence test in a restriction that does not run first");
  auto coarse = [&](hipStream_t cs) {
    with_kc(e.kc, [&](auto K) {
      constexpr int KC = decltype(K)::value;
      hipLaunchKernelGGL(k_restrict<KC>, dim3(nblk(d.m0 * 64)), dim3(kBlock), 0, cs, d.PTptr.p, d.PTdof.p, d.PTw.p,
                         r, e.rH.p, (int)d.m0, e.sc.p, sel, conv ? e.partials2.p : nullptr, (int)grid_for(d.npad));
      const unsigned gb = (unsigned)(d.ld0 / 8);
      std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
      if (d.profiling) {
        if (d.ev_free.empty()) {
          HIPCHK(hipEventCreate(&ev.first));
          HIPCHK(hipEventCreate(&ev.second));
        } else {
          ev = d.ev_free.back();
          d.ev_free.pop_back();
        }
        HIPCHK(hipEventRecord(ev.first, cs));
      }
      const unsigned g1 = (unsigned)(d.ld0 / 4);
      const unsigned gs = (unsigned)((int64_t)d.sym_T * (d.sym_T + 1) / 2);
      if (e.coarse_sym) {
        if (d.coarse32)
          hipLaunchKernelGGL((k_coarse_sym<float, KC>), dim3(gs), dim3(64), 0, cs, d.Ksym32.p, d.sym_tiles.p,
                             (int)d.sym_T, e.rH.p, e.cpart.p, e.sc.p, sel);
        else
          hipLaunchKernelGGL((k_coarse_sym<double, KC>), dim3(gs), dim3(64), 0, cs, d.Ksym64.p, d.sym_tiles.p,
                             (int)d.sym_T, e.rH.p, e.cpart.p, e.sc.p, sel);
        hipLaunchKernelGGL(k_coarse_fold<KC>, dim3((unsigned)d.sym_T), dim3(kBlock), 0, cs, e.cpart.p,
                           (int)d.sym_T, e.c.p, (int)d.m0, e.sc.p, sel);
      } else if (d.coarse32 && e.coarse_w1)
        hipLaunchKernelGGL((k_coarse_mm1<float, KC>), dim3(g1), dim3(64), 0, cs, d.Kinv32.p, (int)d.ld0, e.rH.p,
                           e.c.p, (int)d.m0, e.sc.p, sel);
      else if (d.coarse32)
        hipLaunchKernelGGL((k_coarse_mm<float, KC>), dim3(gb), dim3(64 * kMmWaves), 0, cs, d.Kinv32.p, (int)d.ld0,
                           e.rH.p, e.c.p, (int)d.m0, e.sc.p, sel);
      else if (e.coarse_w1)
        hipLaunchKernelGGL((k_coarse_mm1<double, KC>), dim3(g1), dim3(64), 0, cs, d.Kinv64.p, (int)d.ld0, e.rH.p,
                           e.c.p, (int)d.m0, e.sc.p, sel);
      else
        hipLaunchKernelGGL((k_coarse_mm<double, KC>), dim3(gb), dim3(64 * kMmWaves), 0, cs, d.Kinv64.p, (int)d.ld0,
                           e.rH.p, e.c.p, (int)d.m0, e.sc.p, sel);
      if (d.profiling) {
        HIPCHK(hipEventRecord(ev.second, cs));
        d.ev_coarse.push_back(ev);
      }
    });
  };
  // while profiling, the coarse solve always runs first, so that the timed
  // sweeps have the device to themselves
  if (coarse_runs_first(e)) {
    // the coarse solve first, on the whole device, then the star sweeps
    coarse(s);
    launch_stars(e, r, sel, s);
  } else if (d.m0 > 0) {
    // the coarse solve is independent of the local solves (the preconditioner
    // is additive): it runs on its own stream beside the star sweeps
    // (queued before the sweeps, or after them so that the sweeps' long
    // stars start first and the coarse wavefronts fill the SIMDs they leave)
    HIPCHK(hipEventRecord(e.fork2, s));
    HIPCHK(hipStreamWaitEvent(e.aux2, e.fork2, 0));
    if (e.coarse_late) {
      launch_stars(e, r, sel, s);
      coarse(e.aux2);
    } else {
      coarse(e.aux2);
      launch_stars(e, r, sel, s);
    }
    HIPCHK(hipEventRecord(e.join2, e.aux2));
    HIPCHK(hipStreamWaitEvent(s, e.join2, 0));
  } else {
    launch_stars(e, r, sel, s);
  }
  with_kc(e.kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    const unsigned G = grid_for(d.npad);
    double *parts = dot ? e.partials.p : nullptr;
    auto red = [&](auto nvc) {
      constexpr int NV = decltype(nvc)::value;
      if (d.precision == SN_PREC_FP32_STARS)
        hipLaunchKernelGGL((k_reduce<float, KC, NV>), dim3(G), dim3(kBlock), 0, s, z, r, e.slots32.p, d.slot_of.p,
                           d.Pc.p, d.Pw.p, e.c.p, (int)d.npad, e.sc.p, sel, parts);
      else
        hipLaunchKernelGGL((k_reduce<double, KC, NV>), dim3(G), dim3(kBlock), 0, s, z, r, e.slots64.p, d.slot_of.p,
                           d.Pc.p, d.Pw.p, e.c.p, (int)d.npad, e.sc.p, sel, parts);
    };
    if (d.nv == 4) red(std::integral_constant<int, 4>{});
    else red(std::integral_constant<int, 8>{});
    if (dot && !kFuseScalars<KC>)
      hipLaunchKernelGGL(k_scalar<KC>, dim3(1), dim3(kBlock * scalar_groups<KC>()), 0, s,
                       e.partials.p, (int)G, e.sc.p, (int)OP_BETA, sel, 0u);
  });
}

// y = K x on the selected columns; with dot, x.y -> alpha (first half)
void launch_spmv(Engine &e, const double *x, double *y, int sel, bool dot, hipStream_t s) {
  DeviceState &d = *e.d;
  Sell A{d.sptr.p, d.slen.p, d.col.p, d.val.p};
  const unsigned G = grid_for(d.npad);
  with_kc(e.kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    hipLaunchKernelGGL(k_spmv<KC>, dim3(G), dim3(kBlock), 0, s, A, x, y, (int)d.npad, e.sc.p, sel,
                       dot ? e.partials.p : nullptr);
    if (dot && !kFuseScalars<KC>)
      hipLaunchKernelGGL(k_scalar<KC>, dim3(1), dim3(kBlock * scalar_groups<KC>()), 0, s,
                       e.partials.p, (int)G, e.sc.p, (int)OP_ALPHA, sel, 0u);
  });
}

void launch_iteration(Engine &e, hipStream_t s) {
  DeviceState &d = *e.d;
  if (d.profiling) ++d.prof_iters;
  const unsigned G = grid_for(d.npad);
  launch_spmv(e, e.p.p, e.q.p, SEL_FIRST, true, s);
  with_kc(e.kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    hipLaunchKernelGGL(k_cg_update<KC>, dim3(G), dim3(kBlock), 0, s, e.u.p, e.r.p, e.p.p, e.q.p, (int)d.npad, e.sc.p,
                       e.partials.p, (int)G, e.partials2.p);
    // the convergence test: by the restriction when the coarse solve runs first
    // (one launch fewer), else by a one-block kernel before the fork
    if (!coarse_runs_first(e))
      hipLaunchKernelGGL(k_scalar<KC>, dim3(1), dim3(kBlock * scalar_groups<KC>()), 0, s,
                         e.partials2.p, (int)G, e.sc.p, (int)OP_CONV,
                         (int)SEL_FIRST, 0u);
  });
  launch_B(e, e.r.p, e.z.p, SEL_SECOND, true, s, coarse_runs_first(e));
  with_kc(e.kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    hipLaunchKernelGGL(k_p_update<KC>, dim3(G), dim3(kBlock), 0, s, e.p.p, e.z.p, (int)d.npad, e.sc.p, e.partials.p,
                       (int)G);
  });
}

// true residual of the stopped columns: restart or final (see OP_TRUE)
void launch_verify(Engine &e, hipStream_t s) {
  DeviceState &d = *e.d;
  const unsigned G = grid_for(d.npad);
  launch_spmv(e, e.u.p, e.q.p, SEL_VERIFY, false, s);
  with_kc(e.kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    hipLaunchKernelGGL(k_sub_dot<KC>, dim3(G), dim3(kBlock), 0, s, e.q.p, e.f.p, e.q.p, (int)d.npad, e.sc.p,
                       (int)SEL_VERIFY, 0u, e.partials.p);
    hipLaunchKernelGGL(k_scalar<KC>, dim3(1), dim3(kBlock * scalar_groups<KC>()), 0, s,
                       e.partials.p, (int)G, e.sc.p, (int)OP_TRUE,
                       (int)SEL_VERIFY, 0u);
    hipLaunchKernelGGL(k_copy_sel<KC>, dim3(G), dim3(kBlock), 0, s, e.r.p, e.q.p, (int)d.npad, e.sc.p,
                       (int)SEL_RESTART, 0u);
  });
}

// f.f -> f2, tol2 and r.r -> rr (done at once when nothing is to iterate) for
// the columns of `mask`
void launch_start_dots(Engine &e, uint32_t mask, hipStream_t s) {
  DeviceState &d = *e.d;
  const unsigned G = grid_for(d.npad);
  with_kc(e.kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    hipLaunchKernelGGL(k_dot<KC>, dim3(G), dim3(kBlock), 0, s, e.f.p, e.f.p, (int)d.npad, e.partials.p, e.sc.p,
                       (int)SEL_MASK, mask);
    hipLaunchKernelGGL(k_scalar<KC>, dim3(1), dim3(kBlock * scalar_groups<KC>()), 0, s,
                       e.partials.p, (int)G, e.sc.p, (int)OP_F2,
                       (int)SEL_MASK, mask);
    hipLaunchKernelGGL(k_dot<KC>, dim3(G), dim3(kBlock), 0, s, e.r.p, e.r.p, (int)d.npad, e.partials.p, e.sc.p,
                       (int)SEL_MASK, mask);
    hipLaunchKernelGGL(k_scalar<KC>, dim3(1), dim3(kBlock * scalar_groups<KC>()), 0, s,
                       e.partials.p, (int)G, e.sc.p, (int)OP_R2,
                       (int)SEL_MASK, mask);
  });
}

// run m iterations: as captured graphs of 2^i iterations, or launch by launch
void run_iterations(Engine &e, int m, bool use_graph, hipStream_t s) {
  if (!use_graph || e.d->profiling) {
    for (int it = 0; it < m; ++it) launch_iteration(e, s);
    return;
  }
  for (int i = 0; m > 0; ++i) {
    if (!(m & (1 << i))) continue;
    if ((int)e.graphs.size() <= i) {
      e.graphs.resize(i + 1, nullptr);
      e.graph_defs.resize(i + 1, nullptr);
    }
    if (!e.graphs[i]) {
      // capture on the engine's own stream, replay on the caller's
      HIPCHK(hipStreamSynchronize(s));
      HIPCHK(hipStreamBeginCapture(e.own, hipStreamCaptureModeRelaxed));
      for (int it = 0; it < (1 << i); ++it) launch_iteration(e, e.own);
      HIPCHK(hipStreamEndCapture(e.own, &e.graph_defs[i]));
      HIPCHK(hipGraphInstantiate(&e.graphs[i], e.graph_defs[i], nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(e.graphs[i], s));
    m -= 1 << i;
  }
}

void upload_scalars(Engine &e, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(e.sc.p, e.host_sc, (size_t)e.kc * sizeof(CgScalars), hipMemcpyHostToDevice, s));
  e.sc_dirty = false;
}

// iterations, true-residual checks and the asynchronous read-back of the
// column states
void tick(Engine &e, int iters, bool use_graph, hipStream_t s) {
  if (e.sc_dirty) upload_scalars(e, s);
  if (iters > 0) run_iterations(e, iters, use_graph, s);
  launch_verify(e, s);
  HIPCHK(hipMemcpyAsync(e.host_sc, e.sc.p, (size_t)e.kc * sizeof(CgScalars), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(e.tick_done, s));
  e.in_flight = true;
}

void wait_tick(Engine &e) {
  if (!e.in_flight) return;
  HIPCHK(hipEventSynchronize(e.tick_done));
  e.in_flight = false;
}

CgScalars column_init(double rtol, int64_t max_iter, int64_t fixed) {
  CgScalars x;
  std::memset(&x, 0, sizeof(x));
  x.rtol = rtol;
  x.max_iter = (int32_t)std::min<int64_t>(max_iter > 0 ? max_iter : 1000, 1 << 30);
  x.fixed = (int32_t)std::max<int64_t>(std::min<int64_t>(fixed, 1 << 30), 0);
  x.active = 1;
  x.first_it = 0;
  x.fresh = 1;
  return x;
}

int kc_index(int kc) {
  switch (kc) {
    case 1: return 0;
    case 2: return 1;
    case 4: return 2;
    case 8: return 3;
    default: return 4;
  }
}

Engine &solve_engine(Precond &pre, int k) {
  DeviceState &d = *pre.dev;
  const int kc = engine_width_for(k);
  auto &slot = d.solve_engine[kc_index(kc)];
  if (!slot) slot.reset(engine_create(pre, kc));
  return *slot;
}

// host n x k block -> staging buffer (the engine's q); returns the device source
const double *stage_block(Engine &e, const double *src, int k, bool dev_ptrs, hipStream_t s) {
  if (dev_ptrs) return src;
  HIPCHK(hipMemcpyAsync(e.q.p, src, (size_t)e.d->n * k * sizeof(double), hipMemcpyHostToDevice, s));
  return e.q.p;
}

// batch vector columns 0..k-1 -> n x k block (host or device)
void store_block(Engine &e, double *dst, const double *src, int k, bool dev_ptrs, hipStream_t s) {
  DeviceState &d = *e.d;
  if (dev_ptrs) {
    with_kc(e.kc, [&](auto K) {
      constexpr int KC = decltype(K)::value;
      for (int j = 0; j < k; ++j)
        hipLaunchKernelGGL(k_col_out<KC>, dim3(grid_for(d.n)), dim3(kBlock), 0, s, dst, src, d.perm.p, (int)d.n, k, j,
                           j);
    });
    HIPCHK(hipStreamSynchronize(s));
    return;
  }
  std::vector<double> tmp((size_t)d.n * e.kc);
  HIPCHK(hipMemcpyAsync(tmp.data(), src, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int64_t i = 0; i < d.n; ++i)
    for (int j = 0; j < k; ++j) dst[(size_t)d.perm_h[i] * k + j] = tmp[(size_t)i * e.kc + j];
}

// n x k block (device) -> batch vector columns 0..k-1 (the rest zero)
void load_block(Engine &e, double *dst, const double *src_dev, int k, hipStream_t s) {
  DeviceState &d = *e.d;
  with_kc(e.kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    for (int j = 0; j < e.kc; ++j) {
      if (j < k)
        hipLaunchKernelGGL(k_col_in<KC>, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, dst, src_dev, d.perm.p,
                           (int)d.n, (int)d.npad, k, j, j);
      else
        hipLaunchKernelGGL(k_col_in<KC>, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, dst, src_dev, d.perm.p, 0,
                           (int)d.npad, k, 0, j);
    }
  });
}

// Split of the stars between the two local-solve kernels: of the `nsn` stars
// with the longest band sweeps (2n dependent steps) those the supernodal
// layout holds, and every star whose band no window covers, go to the
// supernodal path, the others to the band path (narrow and wide windows in
// separate launches, longest first).
void plan_split(Engine &e, int64_t nsn) {
  DeviceState &d = *e.d;
  std::vector<int32_t> by_len((size_t)d.nstars);
  for (int32_t s = 0; s < d.nstars; ++s) by_len[s] = s;
  std::stable_sort(by_len.begin(), by_len.end(), [&](int32_t a, int32_t b) { return d.h_n[a] > d.h_n[b]; });
  std::vector<int32_t> narrow, wide, twin;
  std::vector<int64_t> vs;
  int64_t tw_pos = 0;
  e.sn_list.clear();
  e.sweep_bytes = 0;
  for (int64_t i = 0; i < d.nstars; ++i) {
    const int32_t s = by_len[i];
    if (d.h_q[s] == 0 || (i < nsn && d.h_sn_ok[s])) {
      e.sn_list.push_back(s);
      e.sweep_bytes += d.h_bytes_sn[s];
    } else if (d.twin_min > 0 && d.h_twin[s] >= 0 && d.h_n[s] >= d.twin_min) {
      const int32_t t = d.h_twin[s];
      twin.push_back(t);
      e.sweep_bytes += d.h_bytes_twin[t];
    } else {
      (d.h_q[s] <= 2 ? narrow : wide).push_back(s);
      e.sweep_bytes += d.h_bytes_band[s];
    }
  }
  // vectors of the twin stars: two chains each, per twin in twin-id order
  vs.assign((size_t)d.ntwin, 0);
  for (const int32_t t : twin) {
    vs[t] = tw_pos;
    tw_pos += 2 * (int64_t)d.h_twin_len[t];
  }
  const int64_t ts = d.precision == SN_PREC_FP32_STARS ? 4 : 8;
  const int64_t need = tw_pos * e.kc * ts;
  if ((int64_t)e.tw_scratch.n < need) {
    e.tw_scratch.alloc((size_t)need);
    e.bytes += need;
  }
  e.tw_vs.upload(vs);
  e.b_twin.upload(twin);
  e.n_twin = (int32_t)twin.size();
  e.b_narrow.upload(narrow);
  e.b_wide.upload(wide);
  e.n_narrow = (int32_t)narrow.size();
  e.n_wide = (int32_t)wide.size();
  e.n_sn = (int32_t)e.sn_list.size();
}

// Supernodal launch plan for the stars of sn_list, an LDS cap (bytes per
// workgroup), CW columns per wavefront and nteam wavefronts per workgroup. A
// star needs its index part plus nteam sets of vectors (x and y: n x CW, u:
// nu x CW) in LDS, and its values too if they are to be staged; the kernel
// stages them when they fit the launch's LDS. Stars whose index part and
// vectors fit the cap go to launch 0, the others to launch 1 with as much LDS
// as its largest star wants (at most 160 KB), and stars beyond that to launch
// 2, solved from global memory. Each launch takes its stars longest first.
void plan_sn(Engine &e, int lcap, int cw, int nteam) {
  DeviceState &d = *e.d;
  const int64_t ts = d.precision == SN_PREC_FP32_STARS ? 4 : 8;
  const int64_t kMaxLds = kStarMaxLds;
  std::vector<int32_t> o[3];
  std::vector<int64_t> vs((size_t)d.nstars, -1);
  int64_t l1 = 0, vbytes = 0;
  int32_t nig = 0;
  // more wavefronts than column chunks: the workgroup solves the chunks
  // together, with one set of vectors
  const int64_t vsets = nteam > e.kc / cw ? 1 : nteam;
  for (const int32_t s : e.sn_list) {
    const int64_t xb = (d.h_n[s] * cw * ts + 15) & ~15, ub = (d.h_nu[s] * cw * ts + 15) & ~15;
    const int64_t vec = vsets * (2 * xb + ub), need = d.h_idx[s] + vec;
    if (need <= lcap) {
      o[0].push_back(s);
    } else if (need <= kMaxLds) {
      o[1].push_back(s);
      l1 = std::max(l1, std::min(kMaxLds, need + d.h_val[s]));
    } else if (e.sn_iglobal && vec <= kMaxLds) {
      // vectors in LDS, index part and values read from global memory
      o[1].push_back(s);
      l1 = std::max(l1, vec);
      ++nig;
    } else if (e.sn_iglobal && vsets == 1 && nteam > e.kc / cw && 2 * xb <= kMaxLds) {
      // x and y in LDS, the update slots in global memory (workgroup teams
      // only: their phases end in workgroup barriers)
      o[1].push_back(s);
      l1 = std::max(l1, 2 * xb);
      vs[s] = vbytes;
      vbytes += ub;
      ++nig;
    } else {
      o[2].push_back(s);
      vs[s] = vbytes;
      vbytes += 2 * xb + ub;
    }
  }
  for (int w = 0; w < 3; ++w) {
    e.sl[w].order.upload(o[w]);
    e.sl[w].count = (int32_t)o[w].size();
  }
  e.sl[0].lds = lcap;
  e.sl[1].lds = (int32_t)l1;
  e.sl[2].lds = 0;
  if ((int64_t)e.vscratch.n < vbytes) {
    e.vscratch.alloc((size_t)vbytes);
    e.bytes += vbytes;
  }
  e.st_vs.upload(vs);
  e.star_cw = cw;
  e.star_nteam = nteam;
  e.star_lcap = lcap;
  e.star_iglobal = nig;
}

// The local-solve launch shape is measured: every candidate solves all stars
// (zero input) a few times and the fastest wins (a candidate must beat the
// best by 2%, since a three-launch timing moves by a few percent). In turn:
// the band occupancy limit (few resident band wavefronts per SIMD leave the
// hardware to hand out the remaining, shorter stars as waves finish; many hide
// more latency) and where the band working vectors live, with every star on
// the band path; then the split between the paths; then the supernodal LDS
// cap and launch shape at that split; then the band occupancy again.
void tune_stars(Engine &e) {
  DeviceState &d = *e.d;
  if (d.nstars == 0) return;
  const bool prof = d.profiling;
  d.profiling = false;
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  auto time_it = [&]() -> double {
    for (int w = 0; w < 2; ++w) launch_stars(e, e.r.p, SEL_ALL, e.own);
    HIPCHK(hipEventRecord(t0, e.own));
    for (int it = 0; it < 3; ++it) launch_stars(e, e.r.p, SEL_ALL, e.own);
    HIPCHK(hipEventRecord(t1, e.own));
    HIPCHK(hipEventSynchronize(t1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    return 1e3 * ms / 3.0;
  };
  auto set_cap = [&](int cap) {
    e.star_cap = cap;
    e.star_lds = cap == 0 ? 0 : (160 * 1024 / (4 * cap)) & ~511;
  };
  // supernodal defaults
  int lcap = 24 << 10, cw = std::min(e.kc, 4), nt = 1;
  if (d.twin_force >= 0) d.twin_min = d.twin_force;
  // 1. band occupancy and vector placement, all stars on the band path
  plan_split(e, 0);
  plan_sn(e, lcap, cw, nt);
  double best = 1e30;
  int bcap = 0;
  if (e.n_narrow + e.n_wide > 0) {
    for (int cap : {0, 4, 3, 2, 1}) {
      set_cap(cap);
      const double us = time_it();
      if (us < 0.98 * best) {
        best = us;
        bcap = cap;
      }
    }
    set_cap(bcap);
    e.star_lv = false;
    const double us = time_it();
    e.star_lv = !(us < 0.95 * best);
    if (!e.star_lv) best = us;
  }
  // 2. the split: the longest stars to the supernodal path (once per
  //    preconditioner); stars beyond LDS keep their vectors there unless the
  //    caller fixed otherwise
  e.sn_iglobal = d.sn_beyond != 0;
  if (d.split < 0) {
    int64_t bsplit = 0;
    // each candidate with one wavefront per column chunk and with four
    // wavefronts solving the chunks together
    std::vector<int> teams{nt};
    for (const int w : {4, 16})
      if (w > e.kc / cw) teams.push_back(w);
    for (const double f : {0.01, 0.025, 0.05, 0.1, 0.2, 0.4, 1.0}) {
      const int64_t k = std::max<int64_t>(1, (int64_t)std::llround(f * d.nstars));
      plan_split(e, k);
      for (const int w : teams) {
        plan_sn(e, lcap, cw, w);
        const double us = time_it();
        if (us < 0.98 * best) {
          best = us;
          bsplit = k;
        }
      }
    }
    d.split = bsplit;
  }
  plan_split(e, d.split);
  // 3. supernodal LDS cap and launch shape at that split
  if (e.n_sn > 0) {
    std::vector<std::pair<int, int>> shapes;  // (cw, nteam)
    for (int c = 1; c <= std::min(e.kc, 4); c *= 2)
      for (int w = 1; w <= 16; w *= 2)
        if (w <= std::min(e.kc / c, 4) || (w > e.kc / c && w >= 4))  // w > kc / c: the chunks solved together
          shapes.push_back({c, w});
    const int caps[] = {12 << 10, 16 << 10, 24 << 10, 32 << 10, 48 << 10, 64 << 10};
    double sbest = 1e30;
    auto try_sn = [&](int cap, int c, int w) {
      plan_sn(e, cap, c, w);
      const double us = time_it();
      if (us < 0.98 * sbest) {
        sbest = us;
        lcap = cap;
        cw = c;
        nt = w;
      }
    };
    for (int cap : caps) try_sn(cap, cw, nt);
    for (auto &sh : shapes) try_sn(lcap, sh.first, sh.second);
    plan_sn(e, lcap, cw, nt);
    // the stars beyond LDS: vectors in LDS with the index part and values
    // read from global memory, or everything in global memory
    if (d.sn_beyond >= 0) {
      e.sn_iglobal = d.sn_beyond == 1;
      plan_sn(e, lcap, cw, nt);
    } else {
      e.sn_iglobal = true;
      plan_sn(e, lcap, cw, nt);
      if (e.star_iglobal > 0) {
        // both settings give the same bits: keep the faster
        const double t_ig = time_it();
        e.sn_iglobal = false;
        plan_sn(e, lcap, cw, nt);
        const double t_g = time_it();
        e.sn_iglobal = t_ig <= t_g;
        sbest = std::min(sbest, std::min(t_ig, t_g));
        plan_sn(e, lcap, cw, nt);
      }
    }
    // the stars solved from global memory: four or sixteen wavefronts each
    if (e.sl[2].count > 0) {
      e.star_gteam = 16;
      const double us = time_it();
      if (us < 0.98 * sbest) sbest = us;
      else e.star_gteam = 4;
    }
    best = sbest;
  }
  plan_sn(e, lcap, cw, nt);
  // 4. band occupancy again at that split
  if (e.n_narrow + e.n_wide > 0) {
    double bb = 1e30;
    for (int cap : {0, 4, 3, 2, 1}) {
      set_cap(cap);
      const double us = time_it();
      if (us < 0.98 * bb) {
        bb = us;
        bcap = cap;
      }
    }
    set_cap(bcap);
    best = bb;
    // 5. issue priority for the wavefronts of the longest band stars (the
    //    same arithmetic, a different schedule)
    int bprio = 0;
    for (const int np : {16, 64, 256, 1024}) {
      if (np > std::max(e.n_narrow, e.n_wide)) break;
      e.star_prio = np;
      const double us = time_it();
      if (us < 0.98 * best) {
        best = us;
        bprio = np;
      }
    }
    e.star_prio = bprio;
  }
  // 6. the two-chain form for the longest band stars (once per
  //    preconditioner: it rounds differently from the single chain)
  if (d.twin_min < 0) {
    int64_t bmin = 0;
    int32_t maxn = 0;
    for (int32_t s = 0; s < d.nstars; ++s)
      if (d.h_twin[s] >= 0) maxn = std::max(maxn, d.h_n[s]);
    if (maxn > 0 && e.n_narrow + e.n_wide > 0) {
      for (const double f : {0.8, 0.6, 0.45, 0.3}) {
        d.twin_min = std::max<int64_t>(1, std::llround(f * maxn));
        plan_split(e, d.split);
        if (e.n_twin == 0) continue;
        const double us = time_it();
        if (us < 0.98 * best) {
          best = us;
          bmin = d.twin_min;
        }
      }
    }
    d.twin_min = bmin;
    plan_split(e, d.split);
  }
  // 7. the narrow band sweeps as one persistent launch: 1-6 resident
  //    wavefronts per SIMD taking the stars, longest first, from a queue (the
  //    same arithmetic, a different schedule)
  e.star_resident = 0;
  if (d.queue_force >= 0) {
    e.star_resident = d.queue_force;
  } else if (e.n_narrow > 0) {
    int cus = 0;
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d.device));
    int bres = 0;
    for (const int per_simd : {1, 2, 3, 4, 6}) {
      const int nres = per_simd * 4 * cus;
      if (nres >= e.n_narrow) break;
      e.star_resident = nres;
      const double us = time_it();
      if (us < 0.98 * best) {
        best = us;
        bres = nres;
      }
    }
    e.star_resident = bres;
  }
  e.star_us = best;
  // the coarse kernel's placement: before the sweeps, or beside them on a
  // second stream, queued before or after them (the packed kernel unless a
  // launch is fixed; the dense kernels are chosen only explicitly, since they
  // round differently). The second half of an iteration is timed: with the
  // coarse solve first the restriction also runs the convergence test, beside
  // it a one-block kernel does (no column is active here, so neither changes a
  // column's state). A candidate must beat the best so far by 2%.
  if (d.m0 > 0) {
    auto set_mode = [&](int mode) {
      // 0..5: dense kernel (mode & 1) and placement (mode / 2); 6..8: packed, placement mode - 6
      e.coarse_sym = mode >= 6;
      e.coarse_w1 = !e.coarse_sym && (mode & 1) != 0;
      const int place = e.coarse_sym ? mode - 6 : mode / 2;
      e.coarse_first = place == 0;
      e.coarse_late = place == 2;
    };
    double bbest = 1e30;
    // measured: the packed kernel in its three placements (all three give the
    // same bits, so every batch width of the preconditioner rounds alike)
    const std::vector<int> modes =
        d.coarse_launch >= 0 ? std::vector<int>{d.coarse_launch} : std::vector<int>{7, 6, 8};
    int bmode = modes.front();
    for (const int mode : modes) {
      set_mode(mode);
      auto half = [&]() {
        if (!e.coarse_first)
          with_kc(e.kc, [&](auto K) {
            constexpr int KC = decltype(K)::value;
            hipLaunchKernelGGL(k_scalar<KC>, dim3(1), dim3(kBlock * scalar_groups<KC>()), 0, e.own,
                               e.partials2.p, (int)grid_for(d.npad), e.sc.p, (int)OP_CONV, (int)SEL_FIRST, 0u);
          });
        launch_B(e, e.r.p, e.z.p, SEL_ALL, false, e.own, e.coarse_first);
      };
      for (int w = 0; w < 2; ++w) half();
      HIPCHK(hipEventRecord(t0, e.own));
      for (int it = 0; it < 3; ++it) half();
      HIPCHK(hipEventRecord(t1, e.own));
      HIPCHK(hipEventSynchronize(t1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, t0, t1));
      const double us = 1e3 * ms / 3.0;
      if (us < 0.98 * bbest) {
        bbest = us;
        bmode = mode;
      }
    }
    set_mode(bmode);
    e.b_us = bbest;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  d.profiling = prof;
}

}  // namespace

// ---------------------------------------------------------------------------
// engines
// ---------------------------------------------------------------------------
int engine_width_for(int k) {
  if (k < 1 || k > kMaxCols) fail(SN_EINVAL, "k must be in 1..16");
  int w = 1;
  while (w < k) w *= 2;
  return w;
}

int64_t engine_footprint(const Precond &pre, int kc) {
  const int64_t n = pre.sys->n, npad = (n + kBlock - 1) / kBlock * kBlock;
  const int64_t m0 = (std::max<int64_t>(pre.m0, 1) + 63) / 64 * 64;
  const int prec = pre.dev ? pre.finfo.star_precision : pre.precision;
  const int64_t ts = prec == SN_PREC_FP64 ? 8 : 4;
  const int64_t T = pre.m0 > 0 ? m0 / 64 : 0;
  // vectors of the supernodal stars kept in global memory: at most x, y and
  // the update slots of every star (about twice as many updates as positions
  // before factoring)
  int64_t vsc = 0;
  if (pre.dev) {
    for (size_t st = 0; st < pre.dev->h_n.size(); ++st)
      vsc += ((2 * (int64_t)pre.dev->h_n[st] + (int64_t)pre.dev->h_nu[st]) * kc * ts + 48);
    for (const int32_t len : pre.dev->h_twin_len) vsc += 2 * (int64_t)len * kc * ts;  // two-chain vectors
  } else {
    vsc = (int64_t)pre.star_dofs.size() * 5 * kc * ts;
  }
  return (6 * npad * kc + 2 * m0 * kc + (int64_t)2 * kc * kMaxGrid + T * T * 64 * kc) * 8 +
         kc * (int64_t)sizeof(CgScalars) + (int64_t)pre.star_dofs.size() * kc * ts + vsc;
}

Engine *engine_create(Precond &pre, int kc) {
  if (!pre.dev) fail(SN_EINVAL, "preconditioner not factored");
  (void)engine_width_for(kc);
  if (engine_width_for(kc) != kc) fail(SN_EINVAL, "engine width must be 1, 2, 4, 8 or 16");
  DeviceState &d = *pre.dev;
  std::unique_ptr<Engine> e(new Engine);
  e->pre = &pre;
  e->d = &d;
  e->kc = kc;
  const size_t np = (size_t)d.npad * kc;
  for (auto *b : {&e->u, &e->r, &e->p, &e->q, &e->z, &e->f}) {
    b->alloc(np);
    b->zero();
  }
  // r_H and c padded to the coarse operator's 64-row chunks; the padding of r_H
  // stays zero (the restriction writes rows below m0 only)
  const size_t nm = (size_t)std::max<int64_t>(d.ld0, 64) * kc;
  e->rH.alloc(nm);
  e->c.alloc(nm);
  e->rH.zero();
  e->c.zero();
  if (d.sym_T > 0) {
    e->cpart.alloc((size_t)d.sym_T * d.sym_T * 64 * kc);
    e->cpart.zero();
  }
  e->squeue.alloc((size_t)kQueueStride * (kQueues + 1));
  e->squeue.zero();
  e->partials.alloc((size_t)kc * kMaxGrid);
  e->partials.zero();
  e->partials2.alloc((size_t)kc * kMaxGrid);
  e->partials2.zero();
  e->sc.alloc((size_t)kc);
  e->sc.zero();
  if (d.precision == SN_PREC_FP32_STARS) {
    e->slots32.alloc((size_t)std::max<int64_t>(d.slot_count, 1) * kc);
    e->slots32.zero();
  } else {
    e->slots64.alloc((size_t)std::max<int64_t>(d.slot_count, 1) * kc);
    e->slots64.zero();
  }
  HIPCHK(hipHostMalloc((void **)&e->host_sc, (size_t)kc * sizeof(CgScalars), hipHostMallocDefault));
  std::memset(e->host_sc, 0, (size_t)kc * sizeof(CgScalars));
  HIPCHK(hipStreamCreateWithFlags(&e->own, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&e->aux, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&e->fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&e->join, hipEventDisableTiming));
  HIPCHK(hipStreamCreateWithFlags(&e->aux2, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&e->aux3, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&e->aux4, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&e->fork4, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&e->join4, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&e->fork3, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&e->join3, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&e->fork2, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&e->join2, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&e->tick_done, hipEventDisableTiming));
  HIPCHK(hipDeviceSynchronize());
  e->bytes = (int64_t)(6 * np * 8 + 2 * nm * 8 + 2 * e->partials.bytes() + e->sc.bytes() + e->slots32.bytes() +
                       e->slots64.bytes());
  tune_stars(*e);
  return e.release();
}

void engine_destroy(Engine *e) { delete e; }
int engine_width(const Engine *e) { return e->kc; }

void engine_admit(Engine *e, int k, const int32_t *cols, const double *f, const double *rtol,
                  const int64_t *max_iter) {
  if (e->in_flight) fail(SN_EINVAL, "internal: admission into a running engine");
  if (k < 1 || k > e->kc) fail(SN_EINVAL, "internal: bad admission size");
  DeviceState &d = *e->d;
  const hipStream_t s = e->own;
  const double *src = stage_block(*e, f, k, false, s);
  uint32_t mask = 0;
  with_kc(e->kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    for (int j = 0; j < k; ++j) {
      const int c = cols[j];
      if (c < 0 || c >= e->kc || e->host_sc[c].active) fail(SN_EINVAL, "internal: column not free");
      hipLaunchKernelGGL(k_admit<KC>, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, e->f.p, e->r.p, e->u.p, e->p.p,
                         src, d.perm.p, (int)d.n, (int)d.npad, k, j, c);
      e->host_sc[c] = column_init(rtol[j], max_iter[j], 0);
      mask |= 1u << c;
    }
  });
  // Upload the new columns' states only: an earlier admission in the same
  // idle period has queued its own start-up kernels, which must not see their
  // columns reset by this upload. Retired columns (sc_dirty) go up with the
  // whole array before any start-up work of this period.
  if (e->sc_dirty) {
    upload_scalars(*e, s);
  } else {
    for (int j = 0; j < k; ++j)
      HIPCHK(hipMemcpyAsync(e->sc.p + cols[j], &e->host_sc[cols[j]], sizeof(CgScalars), hipMemcpyHostToDevice, s));
  }
  launch_start_dots(*e, mask, s);
}

void engine_tick(Engine *e, int iters, bool use_graph) {
  if (e->in_flight) fail(SN_EINVAL, "internal: tick on a running engine");
  tick(*e, iters, use_graph, e->own);
}

bool engine_query(Engine *e) {
  if (!e->in_flight) return true;
  const hipError_t r = hipEventQuery(e->tick_done);
  if (r == hipErrorNotReady) return false;
  HIPCHK(r);
  e->in_flight = false;
  return true;
}

void engine_wait(Engine *e) { wait_tick(*e); }

void engine_status(const Engine *e, ColumnStatus *out) {
  for (int c = 0; c < e->kc; ++c) {
    const CgScalars &x = e->host_sc[c];
    out[c].iters = x.iters;
    out[c].rr = x.rr;
    out[c].f2 = x.f2;
    out[c].tol2 = x.tol2;
    out[c].t2 = x.t2;
    out[c].active = x.active;
    out[c].done = x.done;
    out[c].verify = x.verify;
    out[c].replacements = x.replacements;
    out[c].fixed = x.fixed;
  }
}

void engine_retire(Engine *e, int c, double *u, int64_t ld) {
  if (e->in_flight) fail(SN_EINVAL, "internal: retire on a running engine");
  DeviceState &d = *e->d;
  const hipStream_t s = e->own;
  with_kc(e->kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    hipLaunchKernelGGL(k_col_out<KC>, dim3(grid_for(d.n)), dim3(kBlock), 0, s, e->q.p, e->u.p, d.perm.p, (int)d.n, 1,
                       0, c);
  });
  std::vector<double> tmp((size_t)d.n);
  HIPCHK(hipMemcpyAsync(tmp.data(), e->q.p, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int64_t i = 0; i < d.n; ++i) u[(size_t)i * ld] = tmp[i];
  std::memset(&e->host_sc[c], 0, sizeof(CgScalars));
  e->sc_dirty = true;
}

// ---------------------------------------------------------------------------
// sn_solve / sn_apply_* on the per-width engines of the preconditioner
// ---------------------------------------------------------------------------
void device_profile(Precond &pre, int enable) {
  DeviceState &d = *pre.dev;
  HIPCHK(hipDeviceSynchronize());
  for (auto &e : d.ev_used) d.ev_free.push_back(e);
  for (auto &e : d.ev_coarse) d.ev_free.push_back(e);
  d.ev_used.clear();
  d.ev_coarse.clear();
  d.prof_iters = 0;
  d.profiling = enable != 0;
}

void device_stats(Precond &pre, sn_kernel_stats *st) {
  DeviceState &d = *pre.dev;
  double ms = 0.0;
  for (auto &e : d.ev_used) {
    HIPCHK(hipEventSynchronize(e.second));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e.first, e.second));
    ms += t;
  }
  st->sweep_launches = (int64_t)d.ev_used.size();
  st->sweep_ms = ms;
  st->iterations = d.prof_iters;
  double cms = 0.0;
  for (auto &e : d.ev_coarse) {
    HIPCHK(hipEventSynchronize(e.second));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e.first, e.second));
    cms += t;
  }
  st->coarse_launches = (int64_t)d.ev_coarse.size();
  st->coarse_ms = cms;
  st->coarse_flops = 2 * d.m0 * d.m0;
}

int64_t device_bytes(const Precond &pre) { return pre.dev ? pre.dev->bytes : 0; }

int device_current() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  return dev;
}

void device_bind(int dev) { HIPCHK(hipSetDevice(dev)); }

void device_set_star_split(Precond &pre, int64_t n_sn) {
  DeviceState &d = *pre.dev;
  for (auto &e : d.solve_engine) {
    if (e) wait_tick(*e);
    e.reset();
  }
  d.split = n_sn < 0 ? -1 : std::min<int64_t>(n_sn, d.nstars);
}

void device_set_band_twins(Precond &pre, int64_t min_positions) {
  DeviceState &d = *pre.dev;
  for (auto &e : d.solve_engine) {
    if (e) wait_tick(*e);
    e.reset();
  }
  d.twin_force = min_positions < 0 ? -1 : min_positions;
  d.twin_min = d.twin_force;
}

void device_set_band_queue(Precond &pre, int32_t waves) {
  DeviceState &d = *pre.dev;
  for (auto &e : d.solve_engine) {
    if (e) wait_tick(*e);
    e.reset();
  }
  d.queue_force = waves < 0 ? -1 : waves;
}

void device_set_sn_beyond_lds(Precond &pre, int mode) {
  DeviceState &d = *pre.dev;
  for (auto &e : d.solve_engine) {
    if (e) wait_tick(*e);
    e.reset();
  }
  d.sn_beyond = mode < 0 ? -1 : mode;
}

void device_set_coarse_launch(Precond &pre, int mode) {
  DeviceState &d = *pre.dev;
  for (auto &e : d.solve_engine) {
    if (e) wait_tick(*e);
    e.reset();
  }
  d.coarse_launch = mode < 0 ? -1 : mode;
}

void device_engine_info(Precond &pre, int k, sn_engine_info *info) {
  Engine &e = solve_engine(pre, k);
  std::memset(info, 0, sizeof(*info));
  info->star_sn = e.n_sn;
  info->star_waves_per_simd = e.star_cap;
  info->star_band_lds = e.star_lv ? 1 : 0;
  info->star_lds_bytes = e.star_lcap;
  info->star_cols_per_wave = e.star_cw;
  info->star_waves = e.star_nteam;
  info->star_big = e.sl[1].count;
  info->star_big_lds_bytes = e.sl[1].lds;
  info->star_global = e.sl[2].count;
  info->star_band_prio = e.star_prio;
  info->star_band_queue = e.star_resident;
  info->star_global_waves = e.star_gteam;
  info->star_big_index_global = e.star_iglobal;
  info->star_twins = e.n_twin;
  info->coarse_first = e.coarse_first ? 1 : 0;
  info->coarse_kernel = e.coarse_sym ? 2 : (e.coarse_w1 ? 1 : 0);
  info->coarse_late = e.coarse_late ? 1 : 0;
  info->sweep_bytes = e.sweep_bytes;
  info->star_sweep_us = e.star_us;
  info->b_apply_us = e.b_us;
}

void device_apply_K(Precond &pre, int k, const double *x, double *y, int device_ptrs, void *stream) {
  Engine &e = solve_engine(pre, k);
  wait_tick(e);
  const hipStream_t s = stream ? (hipStream_t)stream : e.own;
  const double *src = stage_block(e, x, k, device_ptrs != 0, s);
  load_block(e, e.p.p, src, k, s);
  launch_spmv(e, e.p.p, e.z.p, SEL_ALL, false, s);
  store_block(e, y, e.z.p, k, device_ptrs != 0, s);
}

// y = K x (device pointers, n x k) through the workspace: x in the internal
// dof order, then the SpMV, then y back in the canonical order, all queued on
// `stream` without waiting and without allocating. Calls that overlap on one
// GPU share the workspace and race.
void device_apply_K_noalloc(Precond &pre, int k, const double *x, double *y, void *stream) {
  DeviceState &d = *pre.dev;
  const int kc = engine_width_for(k);
  const size_t vec = (size_t)d.npad * kc * sizeof(double);
  const size_t need = 2 * vec + 256 + (size_t)kc * sizeof(CgScalars);
  if (need > kScratchBytes)
    fail(SN_EINVAL, "apply_K without allocation needs " + std::to_string(need) + " bytes of workspace, more than its " +
                        std::to_string(kScratchBytes) + " (fewer columns or sn_apply_K)");
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != d.device) fail(SN_EINVAL, "the preconditioner lives on another device than the current one");
  unsigned char *ws = static_cast<unsigned char *>(scratch_ptr());
  double *xs = reinterpret_cast<double *>(ws);
  double *ys = reinterpret_cast<double *>(ws + vec);
  const CgScalars *scs = reinterpret_cast<const CgScalars *>(ws + ((2 * vec + 255) & ~(size_t)255));
  const hipStream_t s = (hipStream_t)stream;
  Sell A{d.sptr.p, d.slen.p, d.col.p, d.val.p};
  with_kc(kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    // every column of xs is written (past k: zeros), so the workspace needs no clearing
    for (int j = 0; j < kc; ++j)
      hipLaunchKernelGGL(k_col_in<KC>, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, xs, x, d.perm.p,
                         j < k ? (int)d.n : 0, (int)d.npad, k, j < k ? j : 0, j);
    hipLaunchKernelGGL(k_spmv<KC>, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, A, xs, ys, (int)d.npad, scs,
                       (int)SEL_ALL, nullptr);
    for (int j = 0; j < k; ++j)
      hipLaunchKernelGGL(k_col_out<KC>, dim3(grid_for(d.n)), dim3(kBlock), 0, s, y, ys, d.perm.p, (int)d.n, k, j,
                         j);
  });
  HIPCHK(hipGetLastError());
}

void device_apply_B(Precond &pre, int k, const double *r, double *z, int device_ptrs, void *stream) {
  Engine &e = solve_engine(pre, k);
  wait_tick(e);
  const hipStream_t s = stream ? (hipStream_t)stream : e.own;
  const double *src = stage_block(e, r, k, device_ptrs != 0, s);
  load_block(e, e.r.p, src, k, s);
  launch_B(e, e.r.p, e.z.p, SEL_ALL, false, s, false);
  store_block(e, z, e.z.p, k, device_ptrs != 0, s);
}

void device_solve(Precond &pre, int k, const double *f, double *u, const sn_solve_opts &o, sn_solve_info *info) {
  const auto t0 = std::chrono::steady_clock::now();
  Engine &e = solve_engine(pre, k);
  wait_tick(e);
  DeviceState &d = *e.d;
  const hipStream_t s = o.stream ? (hipStream_t)o.stream : e.own;
  const bool dev = o.device_ptrs != 0;
  const int check = o.check_every > 0 ? o.check_every : 8;
  // start the k columns: f = r = f_j, u = p = 0; unused columns stay inactive
  const double *src = stage_block(e, f, k, dev, s);
  uint32_t mask = 0;
  with_kc(e.kc, [&](auto K) {
    constexpr int KC = decltype(K)::value;
    for (int j = 0; j < e.kc; ++j)
      hipLaunchKernelGGL(k_admit<KC>, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, e.f.p, e.r.p, e.u.p, e.p.p, src,
                         d.perm.p, j < k ? (int)d.n : 0, (int)d.npad, k, j < k ? j : 0, j);
  });
  for (int j = 0; j < e.kc; ++j) {
    if (j < k) {
      e.host_sc[j] = column_init(o.rtol, o.max_iter, o.fixed_iters);
      mask |= 1u << j;
    } else {
      std::memset(&e.host_sc[j], 0, sizeof(CgScalars));
    }
  }
  upload_scalars(e, s);
  if (o.use_u0) {
    // r = f - K u0
    const double *usrc = stage_block(e, u, k, dev, s);
    load_block(e, e.u.p, usrc, k, s);
    launch_spmv(e, e.u.p, e.q.p, SEL_ALL, false, s);
    with_kc(e.kc, [&](auto K) {
      constexpr int KC = decltype(K)::value;
      hipLaunchKernelGGL(k_sub_dot<KC>, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, e.r.p, e.f.p, e.q.p,
                         (int)d.npad, e.sc.p, (int)SEL_MASK, mask, (double *)nullptr);
    });
  }
  launch_start_dots(e, mask, s);
  // iterations queued between read-backs: first `check`, then the number the
  // observed contraction of ||r||^2 predicts the slowest column still needs
  // (at least 1, at most 4 check); one at a time while kernels are timed, so
  // that no timed launch runs after convergence
  std::vector<double> prev_rr(k, 0.0);
  std::vector<int64_t> prev_it(k, 0);
  int block = o.fixed_iters > 0 ? (int)std::min<int64_t>(check, o.fixed_iters + 1) : check;
  int64_t since_replace = 0;
  bool first_tick = true;
  for (;;) {
    if (d.profiling) block = 1;
    tick(e, block, o.use_graph != 0, s);
    wait_tick(e);
    since_replace += block;
    bool running = false;
    int next = 1;
    for (int j = 0; j < k; ++j) {
      const CgScalars &x = e.host_sc[j];
      if (x.done && !x.verify) continue;
      running = true;
      if (x.fixed > 0) {
        next = std::max<int>(next, (int)std::min<int64_t>(4 * check, x.fixed - x.iters + (x.fresh ? 1 : 0)));
        continue;
      }
      int need = check;
      const int64_t di = x.iters - prev_it[j];
      if (!first_tick && di > 0 && x.rr > 0.0 && prev_rr[j] > x.rr && x.rr > x.tol2) {
        const double rate = std::pow(x.rr / prev_rr[j], 1.0 / (double)di);
        const double nd = std::log(x.tol2 / x.rr) / std::log(rate);
        if (std::isfinite(nd)) need = (int)std::max(1.0, std::min((double)(4 * check), std::ceil(nd)));
      }
      next = std::max(next, need);
      prev_rr[j] = x.rr;
      prev_it[j] = x.iters;
    }
    first_tick = false;
    if (!running) break;
    block = next;
    if (o.replace_every > 0 && since_replace >= o.replace_every) {
      // residual replacement on the iterating columns: r = f - K u
      launch_spmv(e, e.u.p, e.q.p, SEL_ALL, false, s);
      with_kc(e.kc, [&](auto K) {
        constexpr int KC = decltype(K)::value;
        hipLaunchKernelGGL(k_sub_dot<KC>, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, e.r.p, e.f.p, e.q.p,
                           (int)d.npad, e.sc.p, (int)SEL_FIRST, 0u, (double *)nullptr);
      });
      for (int j = 0; j < k; ++j)
        if (!e.host_sc[j].done && !e.host_sc[j].fresh) e.host_sc[j].replacements += 1;
      e.sc_dirty = true;
      since_replace = 0;
    }
  }
  store_block(e, u, e.u.p, k, dev, s);
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  bool all_conv = true;
  for (int j = 0; j < k; ++j) {
    const CgScalars &x = e.host_sc[j];
    const double fn = std::sqrt(x.f2);
    info[j].iters = x.iters;
    info[j].res_rec = fn > 0 ? std::sqrt(x.rr) / fn : std::sqrt(x.rr);
    info[j].res_true = fn > 0 ? std::sqrt(x.t2) / fn : std::sqrt(x.t2);
    info[j].converged = x.fixed > 0 ? 1 : column_converged(x.rr, x.t2, x.tol2);
    info[j].replacements = x.replacements;
    info[j].ms = ms;
    if (!info[j].converged) all_conv = false;
  }
  if (!all_conv)
    fail(SN_ENOCONV, "a column stopped before its true residual met the tolerance (max_iter reached, or the "
                     "attainable accuracy of the system in FP64 is above it)");
}

}  // namespace spnet
