// GPU hot path for gfx950 (MI355X): PCG on P = BK (Sec. 4.2) with the
// two-level additive Schwarz preconditioner B = P K_0^{-1} P^T +
// sum_j R_j^T K_j^{-1} R_j (Sec. 4.1).
//
// Per iteration:
//   spmv_dot    q = K p (sliced ELL, 64-row slices) and p.q        -> alpha
//   cg_update   u += alpha p, r -= alpha q, r.r, convergence flag
//   star sweeps z_j = K_j^{-1} r[S_j] for every star, one wavefront per star
//   coarse      r_H = P^T r, c = K_0^{-1} r_H (dense inverse)
//   reduce      z = P c + sum of the star slots of every dof, r.z   -> beta
//   p_update    p = z + beta p
// Dot products are reduced per block and then in a fixed order by the last
// block to finish, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.hpp"

namespace spnet {

#define HIPCHK(x)                                                                                \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) fail(SN_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));      \
  } while (0)

constexpr int kBlock = 256;   // threads of the vector kernels
constexpr int kSlice = 64;    // rows per ELL slice (one wavefront)
constexpr int kMaxGrid = 1024;  // blocks of the grid-stride vector kernels (= partial sums)

// ---------------------------------------------------------------------------
// device scalars of one PCG recurrence
// ---------------------------------------------------------------------------
struct CgScalars {
  double rho, alpha, beta, pq, rr, rz, f2, tol2;
  double tmp;  // scratch dot result
  int32_t iters, done, max_iter, fixed, first, pad0;
};

enum ScalarOp { OP_ALPHA = 0, OP_CONV = 1, OP_BETA = 2, OP_DOT = 3 };

// ---------------------------------------------------------------------------
// reductions: per-block partials in a fixed order, then one block combines
// them in a fixed order, so every result is independent of scheduling
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;  // lane 0
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

// one block: combine the partials of the previous kernel and update the scalars
__global__ __launch_bounds__(kBlock) void k_scalar(const double *__restrict__ partials, int nparts, CgScalars *sc,
                                                   int op) {
  __shared__ double sh[kBlock / 64];
  if (op != OP_DOT && sc->done) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) s += partials[i];
  const double tot = block_sum(s, sh);
  if (threadIdx.x != 0) return;
  switch (op) {
    case OP_ALPHA:
      sc->pq = tot;
      sc->alpha = sc->rho / tot;
      break;
    case OP_CONV: {
      sc->rr = tot;
      const int it = sc->iters + 1;
      sc->iters = it;
      const bool stop = sc->fixed > 0 ? it >= sc->fixed : (tot <= sc->tol2 || it >= sc->max_iter);
      if (stop) sc->done = 1;
      break;
    }
    case OP_BETA:
      sc->rz = tot;
      sc->beta = sc->first ? 0.0 : tot / sc->rho;
      sc->rho = tot;
      sc->first = 0;
      break;
    default:
      sc->tmp = tot;
  }
}

// ---------------------------------------------------------------------------
// sliced ELL SpMV: y = K x (optionally x.y partials)
// ---------------------------------------------------------------------------
struct Sell {
  const int32_t *sptr;  // slice start (elements)
  const int32_t *slen;  // slice width
  const int32_t *col;
  const double *val;
};

__global__ __launch_bounds__(kBlock) void k_spmv(Sell A, const double *__restrict__ x, double *__restrict__ y,
                                                 int nrows, const CgScalars *sc, double *partials) {
  __shared__ double sh[kBlock / 64];
  if (partials && sc->done) return;
  double dot = 0.0;
  for (int row = blockIdx.x * kBlock + threadIdx.x; row < nrows; row += gridDim.x * kBlock) {
    const int s = row >> 6, lane = row & 63;
    const int base = A.sptr[s], len = A.slen[s];
    double acc = 0.0;
    for (int c = 0; c < len; ++c) {
      const int e = base + c * kSlice + lane;
      acc += A.val[e] * x[A.col[e]];
    }
    y[row] = acc;
    dot += x[row] * acc;
  }
  if (!partials) return;
  const double part = block_sum(dot, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = part;
}

// u += alpha p, r -= alpha q, r.r partials
__global__ __launch_bounds__(kBlock) void k_cg_update(double *u, double *r, const double *p, const double *q, int n,
                                                      const CgScalars *sc, double *partials) {
  __shared__ double sh[kBlock / 64];
  if (sc->done) return;
  const double a = sc->alpha;
  double rr = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    u[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    rr += ri * ri;
  }
  const double part = block_sum(rr, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = part;
}

// z = P c + sum of the star slots of every dof (ascending star order), r.z partials
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_reduce(double *z, const double *r, const TS *__restrict__ slots,
                                                   const int32_t *__restrict__ slot_of,
                                                   const int32_t *__restrict__ Pc, const double *__restrict__ Pw,
                                                   const double *__restrict__ cvec, int n, int nv,
                                                   const CgScalars *sc, double *partials) {
  __shared__ double sh[kBlock / 64];
  if (partials && sc->done) return;
  double rz = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    double acc = 0.0;
    for (int b = 0; b < nv; ++b) {
      const int c = Pc[(size_t)i * nv + b];
      if (c >= 0) acc += Pw[(size_t)i * nv + b] * cvec[c];
    }
    for (int b = 0; b < nv; ++b) {
      const int s = slot_of[(size_t)i * nv + b];
      if (s >= 0) acc += (double)slots[s];
    }
    z[i] = acc;
    rz += r[i] * acc;
  }
  if (!partials) return;
  const double part = block_sum(rz, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = part;
}

__global__ __launch_bounds__(kBlock) void k_p_update(double *p, const double *z, int n, const CgScalars *sc) {
  if (sc->done) return;
  const double b = sc->beta;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = z[i] + b * p[i];
}

// r_H = P^T r: one block per coarse dof, fixed-order sums
__global__ __launch_bounds__(kBlock) void k_restrict(const int32_t *__restrict__ ptr, const int32_t *__restrict__ dof,
                                                     const double *__restrict__ w, const double *__restrict__ r,
                                                     double *rH, int m0, const CgScalars *sc, int check) {
  __shared__ double sh[kBlock / 64];
  if (check && sc->done) return;
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int q = ptr[c] + threadIdx.x; q < ptr[c + 1]; q += kBlock) acc += w[q] * r[dof[q]];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) rH[c] = acc;
}

// c = K_0^{-1} r_H, one wavefront per row of the dense inverse
__global__ __launch_bounds__(kBlock) void k_coarse_gemv(const double *__restrict__ Kinv, const double *__restrict__ rH,
                                                        double *cvec, int m0, const CgScalars *sc, int check) {
  if (check && sc->done) return;
  const int row = (blockIdx.x * kBlock + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (row >= m0) return;
  const double *a = Kinv + (size_t)row * m0;
  double acc = 0.0;
  for (int j = lane; j < m0; j += 64) acc += a[j] * rH[j];
  acc = wave_sum(acc);
  if (lane == 0) cvec[row] = acc;
}

__global__ __launch_bounds__(kBlock) void k_dot(const double *a, const double *b, int n, double *partials) {
  __shared__ double sh[kBlock / 64];
  double s = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) s += a[i] * b[i];
  const double part = block_sum(s, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = part;
}

// y = a - b
__global__ __launch_bounds__(kBlock) void k_sub(double *y, const double *a, const double *b, int n) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = a[i] - b[i];
}

// strided column gather / scatter between n x k blocks and a contiguous vector
__global__ __launch_bounds__(kBlock) void k_gather_col(double *dst, const double *src, int n, int k, int c) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[i] = src[(size_t)i * k + c];
}
__global__ __launch_bounds__(kBlock) void k_scatter_col(double *dst, const double *src, int n, int k, int c) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[(size_t)i * k + c] = src[i];
}

// ---------------------------------------------------------------------------
// Star sweeps. One wavefront solves L_j L_j^T z = r[S_j] for one star.
//
// The vector of the star lives in LDS in factor order. A sweep walks the
// steps of a stream: the forward stream holds the columns of L (step j: the
// entries L_{j+1..j+w, j}), the backward stream the rows of L from the last
// (step s = row i = n-1-s: the entries L_{i, i-1..i-w}); read in reverse
// order, the vector makes the backward sweep the same recurrence as the
// forward one. Stream values are divided by the step's pivot, so a step
// subtracts m_t g_j from row j+1+t with the raw running value g_j, and the
// pivot division is applied to 64 finished rows at once.
//
// Window: before step j, lane l of register g[q] holds the running value of
// row j + l + 64 q; lane 0 of g[0] is final. The window slides by one lane
// (DPP wave shift left), the next row enters at lane 63 of the last register.
// SG consecutive steps (4 in FP32, 2 in FP64) are packed lane-major, so one
// 16-byte load per lane and register fetches them all; groups are loaded RG
// groups ahead into a register ring, their offsets and widths arrive 64 at a
// time.
// ---------------------------------------------------------------------------
struct StarArgs {
  int32_t nstars;
  const int32_t *order;    // stars, longest first
  const int32_t *st_n;     // positions of the star
  const int32_t *st_vb;    // base in the per-position arrays
  const int32_t *st_q;     // window registers
  const int32_t *st_gb;    // base in the per-group arrays
  const int64_t *st_fb;    // forward stream value base
  const int64_t *st_bb;    // backward stream value base
  const int32_t *pos_dof;  // global dof of each position (factor order)
  const int32_t *f_go, *f_gw, *b_go, *b_gw;  // per group: value offset (from the star base), width
  const void *f_inv, *b_inv;                 // 1/pivot per step (T)
  const void *f_val, *b_val;                 // packed stream values (T)
  void *slots;                               // T, per position
  int32_t pad;                               // LDS zero padding each side (elements)
};

template <typename T>
struct Pack;
template <>
struct Pack<float> {
  using V = float4;
  static constexpr int SG = 4;
  static __device__ __forceinline__ float get(const V &v, int k) {
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
  }
  static __device__ __forceinline__ V masked(bool keep, const V &v) {
    return V{keep ? v.x : 0.f, keep ? v.y : 0.f, keep ? v.z : 0.f, keep ? v.w : 0.f};
  }
  static __device__ __forceinline__ float first(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
  }
  // lanes 0..62 take lane+1, lane 63 takes `in`
  static __device__ __forceinline__ float shl(float v, float in) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(in), __float_as_int(v), 0x130, 0xF, 0xF, false));
  }
  template <int L>
  static __device__ __forceinline__ float put(float vec, float s) {
    int r = __float_as_int(vec);
    asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(r) : "s"(__float_as_int(s)), "i"(L));
    return __int_as_float(r);
  }
};
template <>
struct Pack<double> {
  using V = double2;
  static constexpr int SG = 2;
  static __device__ __forceinline__ double get(const V &v, int k) { return k == 0 ? v.x : v.y; }
  static __device__ __forceinline__ V masked(bool keep, const V &v) {
    return V{keep ? v.x : 0.0, keep ? v.y : 0.0};
  }
  static __device__ __forceinline__ int lo(double v) { return (int)(uint32_t)(__double_as_longlong(v)); }
  static __device__ __forceinline__ int hi(double v) { return (int)(uint32_t)(__double_as_longlong(v) >> 32); }
  static __device__ __forceinline__ double mk(int l, int h) {
    return __longlong_as_double(((long long)(uint32_t)h << 32) | (long long)(uint32_t)l);
  }
  static __device__ __forceinline__ double first(double v) {
    return mk(__builtin_amdgcn_readfirstlane(lo(v)), __builtin_amdgcn_readfirstlane(hi(v)));
  }
  static __device__ __forceinline__ double shl(double v, double in) {
    return mk(__builtin_amdgcn_update_dpp(lo(in), lo(v), 0x130, 0xF, 0xF, false),
              __builtin_amdgcn_update_dpp(hi(in), hi(v), 0x130, 0xF, 0xF, false));
  }
  template <int L>
  static __device__ __forceinline__ double put(double vec, double s) {
    int l = lo(vec), h = hi(vec);
    asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(l) : "s"(lo(s)), "i"(L));
    asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(h) : "s"(hi(s)), "i"(L));
    return mk(l, h);
  }
};

template <int S, int E>
struct StaticFor {
  template <typename F>
  static __device__ __forceinline__ void run(F &&f) {
    f(std::integral_constant<int, S>{});
    StaticFor<S + 1, E>::run(f);
  }
};
template <int E>
struct StaticFor<E, E> {
  template <typename F>
  static __device__ __forceinline__ void run(F &&) {}
};

// One sweep over n steps. vec points at position 0 of the LDS vector (with
// `pad` zero elements on both sides); REV reads it in reverse.
template <typename T, int Q, int RG, bool REV>
__device__ __forceinline__ void sweep(T *vec, int n, const int32_t *__restrict__ go, const int32_t *__restrict__ gw,
                                      const T *__restrict__ inv, const T *__restrict__ vals) {
  using P = Pack<T>;
  using V = typename P::V;
  constexpr int SG = P::SG, GPB = 64 / SG;
  static_assert(GPB % RG == 0, "ring must divide the groups of a block");
  const int lane = threadIdx.x & 63;
  auto at = [&](int p) -> int { return REV ? (n - 1 - p) : p; };
  const int ngroups = (n + SG - 1) / SG;
  T g[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) g[q] = vec[at(lane + 64 * q)];
  // rows entering the window, read NP steps ahead: nxt[s % NP] is row j + 64 Q
  constexpr int NP = 8;
  T nxt[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) nxt[i] = vec[at(64 * Q + i)];
  // group headers of the 64 groups from the current block's first group
  int hoA = lane < ngroups ? go[lane] : 0, hwA = lane < ngroups ? gw[lane] : 0;
  T hinv = lane < n ? inv[lane] : T(0);
  V ring[RG][Q];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) {
    const int o = __builtin_amdgcn_readlane(hoA, rg), w = __builtin_amdgcn_readlane(hwA, rg);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const V v = *reinterpret_cast<const V *>(vals + o + (lane + 64 * q) * SG);
      ring[rg][q] = P::masked(lane + 64 * q < w, v);
    }
  }
  for (int jb = 0; jb < n; jb += 64) {
    const int gb = jb / SG;
    const int hoB = gb + GPB + lane < ngroups ? go[gb + GPB + lane] : 0;
    const int hwB = gb + GPB + lane < ngroups ? gw[gb + GPB + lane] : 0;
    const T hinvN = jb + 64 + lane < n ? inv[jb + 64 + lane] : T(0);
    T ybuf = T(0);
    StaticFor<0, 64>::run([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      constexpr int gi = s / SG, k = s % SG;
      const T gj = P::first(g[0]);
      T carry[Q];
#pragma unroll
      for (int q = 0; q + 1 < Q; ++q) carry[q] = P::first(g[q + 1]);
#pragma unroll
      for (int q = 0; q + 1 < Q; ++q) g[q] = P::shl(g[q], carry[q]);
      g[Q - 1] = P::shl(g[Q - 1], nxt[s % NP]);
      nxt[s % NP] = vec[at(jb + s + 64 * Q + NP)];
      ybuf = P::template put<s>(ybuf, gj);
#pragma unroll
      for (int q = 0; q < Q; ++q) g[q] = g[q] - P::get(ring[gi % RG][q], k) * gj;
      if constexpr (k == SG - 1) {
        // the group is consumed: fetch the group RG positions ahead
        constexpr int li = gi + RG;
        const int o = __builtin_amdgcn_readlane(hoA, li), w = __builtin_amdgcn_readlane(hwA, li);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const V v = *reinterpret_cast<const V *>(vals + o + (lane + 64 * q) * SG);
          ring[gi % RG][q] = P::masked(lane + 64 * q < w, v);
        }
      }
    });
    if (jb + lane < n) vec[at(jb + lane)] = ybuf * hinv;
    hinv = hinvN;
    hoA = hoB;
    hwA = hwB;
  }
}

template <typename T, int Q>
__device__ __forceinline__ void star_solve(const StarArgs &a, int st, int n, T *vec) {
  constexpr int GPB = 64 / Pack<T>::SG;
  constexpr int RG0 = 16 / Q;
  constexpr int RG = RG0 >= GPB ? GPB : (RG0 >= 8 ? 8 : (RG0 >= 4 ? 4 : (RG0 >= 2 ? 2 : 1)));
  const int vb = a.st_vb[st], gbase = a.st_gb[st];
  sweep<T, Q, RG, false>(vec, n, a.f_go + gbase, a.f_gw + gbase, static_cast<const T *>(a.f_inv) + vb,
                         static_cast<const T *>(a.f_val) + a.st_fb[st]);
  __syncthreads();
  sweep<T, Q, RG, true>(vec, n, a.b_go + gbase, a.b_gw + gbase, static_cast<const T *>(a.b_inv) + vb,
                        static_cast<const T *>(a.b_val) + a.st_bb[st]);
}

template <typename T>
__global__ __launch_bounds__(64) void k_star(StarArgs a, const double *__restrict__ r, const CgScalars *sc, int check) {
  if (check && sc->done) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);
  const int wv = blockIdx.x;
  if (wv >= a.nstars) return;
  const int st = a.order[wv];
  const int n = a.st_n[st], vb = a.st_vb[st], Q = a.st_q[st];
  const int lane = threadIdx.x;
  T *vec = lds + a.pad;
  for (int i = lane; i < a.pad; i += 64) {
    lds[i] = T(0);
    vec[n + i] = T(0);
  }
  const int32_t *dofs = a.pos_dof + vb;
  for (int p = lane; p < n; p += 64) vec[p] = (T)r[dofs[p]];
  __syncthreads();
  switch (Q) {
    case 1: star_solve<T, 1>(a, st, n, vec); break;
    case 2: star_solve<T, 2>(a, st, n, vec); break;
    case 4: star_solve<T, 4>(a, st, n, vec); break;
    case 8: star_solve<T, 8>(a, st, n, vec); break;
    default: star_solve<T, 16>(a, st, n, vec); break;
  }
  __syncthreads();
  T *out = static_cast<T *>(a.slots) + vb;
  for (int p = lane; p < n; p += 64) out[p] = vec[p];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  void alloc(size_t cnt) {
    release();
    n = cnt;
    if (cnt) HIPCHK(hipMalloc(&p, cnt * sizeof(T)));
  }
  void upload(const std::vector<T> &h) {
    alloc(h.size());
    if (n) HIPCHK(hipMemcpy(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice));
  }
  void zero() {
    if (n) HIPCHK(hipMemset(p, 0, n * sizeof(T)));
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
  ~DBuf() { release(); }
};

struct Workspace {
  int k = 0;
  DBuf<double> u, r, p, q, z, f, rH, c, partials;
  DBuf<CgScalars> sc;
};

struct DeviceState {
  int device = 0;
  int precision = 0;
  hipStream_t own = nullptr;
  int64_t n = 0, npad = 0, m0 = 0;
  int nv = 4;
  // matrix
  int nslices = 0;
  DBuf<int32_t> sptr, slen, col;
  DBuf<double> val;
  // stars
  int32_t nstars = 0, pad = 0, maxn = 0;
  DBuf<int32_t> order, st_n, st_vb, st_q, st_gb, pos_dof, f_go, f_gw, b_go, b_gw, slot_of;
  DBuf<int64_t> st_fb, st_bb;
  DBuf<float> f_inv32, b_inv32, f_val32, b_val32, slots32;
  DBuf<double> f_inv64, b_inv64, f_val64, b_val64, slots64;
  // coarse
  DBuf<double> Kinv, PTw, Pw;
  DBuf<int32_t> PTptr, PTdof, Pc;
  Workspace ws;
  int64_t bytes = 0;
  // captured iteration blocks: graphs[i] runs 2^i PCG iterations
  std::vector<hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_defs;
  // profiling
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
  int64_t prof_iters = 0;
  ~DeviceState() {
    for (auto &g : graphs)
      if (g) (void)hipGraphExecDestroy(g);
    for (auto &g : graph_defs)
      if (g) (void)hipGraphDestroy(g);
    for (auto &e : ev_used) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto &e : ev_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    if (own) (void)hipStreamDestroy(own);
  }
};

void device_release(DeviceState *d) { delete d; }
void DeviceDeleter::operator()(DeviceState *d) const { delete d; }

namespace {

int window_regs(int band) {
  const int q = (band + 63) / 64;
  for (int w = 1; w <= 16; w *= 2)
    if (q <= w) return w;
  return -1;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
inline unsigned grid_for(int64_t n) { return std::max(1u, std::min<unsigned>(kMaxGrid, nblk(n))); }

// Pack one sweep stream of a star: steps in groups of SG, each group padded
// to its widest step, lane-major (entry t of the SG steps adjacent), values
// divided by the step's pivot.
template <typename T>
void pack_stream(const std::vector<int32_t> &width, const std::vector<double> &vals, const std::vector<double> &inv,
                 int SG, std::vector<T> &out, std::vector<int32_t> &go, std::vector<int32_t> &gw, int64_t base) {
  const int n = (int)width.size();
  std::vector<int64_t> start((size_t)n + 1, 0);
  for (int j = 0; j < n; ++j) start[j + 1] = start[j] + width[j];
  for (int g0 = 0; g0 < n; g0 += SG) {
    int W = 0;
    for (int k = 0; k < SG && g0 + k < n; ++k) W = std::max(W, width[g0 + k]);
    go.push_back((int32_t)((int64_t)out.size() - base));
    gw.push_back(W);
    for (int t = 0; t < W; ++t)
      for (int k = 0; k < SG; ++k) {
        const int j = g0 + k;
        double v = 0.0;
        if (j < n && t < width[j]) v = vals[(size_t)(start[j] + t)] * inv[j];
        out.push_back((T)v);
      }
  }
}

template <typename T>
void upload_stars(DeviceState &d, const Precond &pre, const HostFactors &hf, sn_factor_info &fi) {
  constexpr int SG = 16 / (int)sizeof(T);
  const int64_t ns = (int64_t)hf.stars.size();
  std::vector<int32_t> st_n(ns), st_vb(ns), st_q(ns), st_gb(ns), pos_dof, f_go, f_gw, b_go, b_gw;
  std::vector<int64_t> st_fb(ns), st_bb(ns);
  std::vector<T> f_val, b_val, f_inv, b_inv;
  int64_t tot = 0, real_vals = 0;
  int maxband = 0, maxq = 1;
  for (int64_t s = 0; s < ns; ++s) {
    const StarFactor &F = hf.stars[s];
    const int q = window_regs(std::max(F.band, 1));
    if (q < 0) fail(SN_EINVAL, "star band " + std::to_string(F.band) + " exceeds the widest sweep window (1024)");
    st_n[s] = F.n;
    st_vb[s] = (int32_t)tot;
    st_q[s] = q;
    st_gb[s] = (int32_t)f_go.size();
    maxq = std::max(maxq, q);
    maxband = std::max(maxband, F.band);
    d.maxn = std::max(d.maxn, F.n);
    // forward: columns j; backward: rows n-1-s
    std::vector<double> finv(F.invdiag), binv((size_t)F.n);
    for (int p = 0; p < F.n; ++p) binv[p] = F.invdiag[F.n - 1 - p];
    st_fb[s] = (int64_t)f_val.size();
    pack_stream<T>(F.width_fwd, F.colvals, finv, SG, f_val, f_go, f_gw, st_fb[s]);
    st_bb[s] = (int64_t)b_val.size();
    pack_stream<T>(F.width_bwd, F.rowvals, binv, SG, b_val, b_go, b_gw, st_bb[s]);
    const int32_t *dofs = &pre.star_dofs[pre.star_ptr[s]];
    for (int p = 0; p < F.n; ++p) {
      pos_dof.push_back(dofs[F.perm[p]]);
      f_inv.push_back((T)finv[p]);
      b_inv.push_back((T)binv[p]);
    }
    tot += F.n;
    real_vals += (int64_t)(F.colvals.size() + F.rowvals.size());
  }
  if (tot >= (int64_t)1 << 31 || (int64_t)std::max(f_val.size(), b_val.size()) >= (int64_t)1 << 31)
    fail(SN_EINVAL, "star streams too large for 32-bit offsets");
  // over-read slack: a group load reads up to 64*Q lanes of SG values
  const size_t slack = (size_t)64 * 16 * SG + 64;
  f_val.resize(f_val.size() + slack, T(0));
  b_val.resize(b_val.size() + slack, T(0));
  d.pad = 64 * (maxq + 2);
  // schedule: longest chain first
  std::vector<int32_t> order((size_t)ns);
  for (int64_t s = 0; s < ns; ++s) order[s] = (int32_t)s;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return st_n[a] > st_n[b]; });
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
  d.order.upload(order);
  d.st_n.upload(st_n);
  d.st_vb.upload(st_vb);
  d.st_q.upload(st_q);
  d.st_gb.upload(st_gb);
  d.st_fb.upload(st_fb);
  d.st_bb.upload(st_bb);
  d.pos_dof.upload(pos_dof);
  d.f_go.upload(f_go);
  d.f_gw.upload(f_gw);
  d.b_go.upload(b_go);
  d.b_gw.upload(b_gw);
  d.slot_of.upload(slot_of);
  int64_t stream_bytes;
  if constexpr (sizeof(T) == 4) {
    d.f_inv32.upload(f_inv);
    d.b_inv32.upload(b_inv);
    d.f_val32.upload(f_val);
    d.b_val32.upload(b_val);
    d.slots32.alloc((size_t)tot);
    d.slots32.zero();
    stream_bytes = (int64_t)(d.f_val32.bytes() + d.b_val32.bytes());
  } else {
    d.f_inv64.upload(f_inv);
    d.b_inv64.upload(b_inv);
    d.f_val64.upload(f_val);
    d.b_val64.upload(b_val);
    d.slots64.alloc((size_t)tot);
    d.slots64.zero();
    stream_bytes = (int64_t)(d.f_val64.bytes() + d.b_val64.bytes());
  }
  const int64_t sT = sizeof(T);
  // algorithmic bytes of one application: every off-diagonal factor entry once
  // per sweep, the pivot of every step, the gather (dof id and r) and the slot
  // write of every position; the zero padding of the packed groups is not counted
  fi.sweep_bytes = real_vals * sT + tot * (2 * sT + 4 + 8 + sT);
  fi.sweep_flops = 2 * real_vals + 2 * tot;
  fi.star_stream_bytes = stream_bytes;
  fi.max_band = maxband;
  fi.max_star_dofs = d.maxn;
}

}  // namespace

void device_setup(Precond &pre, const HostFactors &hf, int precision) {
  double max_ratio = 1.0;
  for (const StarFactor &F : hf.stars) max_ratio = std::max(max_ratio, F.pivot_ratio);
  const int requested = precision;
  if (precision == SN_PREC_FP32_STARS && max_ratio * std::ldexp(1.0, -24) > 0.05) precision = SN_PREC_FP64;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(SN_EDEVICE, "no HIP device available");
  auto d = std::make_unique<DeviceState>();
  HIPCHK(hipGetDevice(&d->device));
  HIPCHK(hipStreamCreateWithFlags(&d->own, hipStreamNonBlocking));
  const System &sys = *pre.sys;
  d->precision = precision;
  d->n = sys.n;
  d->npad = (sys.n + kBlock - 1) / kBlock * kBlock;
  d->m0 = pre.m0;
  d->nv = pre.nvert_per_elem;
  const int64_t n = sys.n, npad = d->npad;
  if (n >= (int64_t)1 << 30) fail(SN_EINVAL, "system too large for 32-bit indices");
  sn_factor_info fi{};

  // sliced ELL
  {
    const int ns = (int)(npad / kSlice);
    d->nslices = ns;
    std::vector<int32_t> sptr(ns), slen(ns);
    int64_t tot = 0;
    for (int s = 0; s < ns; ++s) {
      int w = 0;
      for (int l = 0; l < kSlice; ++l) {
        const int64_t r = (int64_t)s * kSlice + l;
        if (r < n) w = std::max<int>(w, (int)(sys.rowptr[r + 1] - sys.rowptr[r]));
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
        const int64_t r = (int64_t)s * kSlice + l;
        const int64_t len = r < n ? sys.rowptr[r + 1] - sys.rowptr[r] : 0;
        for (int c = 0; c < slen[s]; ++c) {
          const size_t e = (size_t)sptr[s] + (size_t)c * kSlice + l;
          if (c < len) {
            col[e] = sys.col[sys.rowptr[r] + c];
            val[e] = sys.val[sys.rowptr[r] + c];
          } else {
            col[e] = (int32_t)std::min<int64_t>(r, n - 1);
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
  int64_t star_nnz = 0;
  for (const StarFactor &F : hf.stars) star_nnz += F.nnz;

  // coarse operator
  const int nc = sys.ncomp, nv = d->nv;
  if (d->m0 > 0) {
    d->Kinv.upload(hf.coarse_inv);
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
          const int64_t dof = f * nc + c;
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
  d->bytes = (int64_t)(d->sptr.bytes() + d->slen.bytes() + d->col.bytes() + d->val.bytes() + d->order.bytes() +
                       d->st_n.bytes() + d->st_vb.bytes() + d->st_q.bytes() + d->st_gb.bytes() + d->st_fb.bytes() +
                       d->st_bb.bytes() + d->pos_dof.bytes() + d->f_go.bytes() + d->f_gw.bytes() + d->b_go.bytes() +
                       d->b_gw.bytes() + d->slot_of.bytes() + d->Kinv.bytes() + d->Pc.bytes() + d->Pw.bytes() +
                       d->PTptr.bytes() + d->PTdof.bytes() + d->PTw.bytes() + d->f_inv32.bytes() +
                       d->b_inv32.bytes() + d->f_inv64.bytes() + d->b_inv64.bytes() + d->slots32.bytes() +
                       d->slots64.bytes()) +
             fi.star_stream_bytes;
  const int64_t nnz = (int64_t)sys.col.size();
  fi.spmv_bytes = nnz * (8 + 4 + 8) + n * 8;
  fi.max_pivot_ratio = max_ratio;
  fi.star_precision = precision;
  fi.star_factor_nnz = star_nnz;
  fi.coarse_bytes = (int64_t)d->Kinv.bytes();
  fi.device_bytes = d->bytes;
  fi.factor_seconds = hf.seconds;
  pre.finfo = fi;
  pre.precision = requested;
  pre.dev.reset(d.release());
}

namespace {

void ensure_ws(DeviceState &d, int k) {
  Workspace &w = d.ws;
  if (w.sc.p && w.k >= k) return;
  // captured graphs refer to the old buffers
  for (auto &g : d.graphs)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto &g : d.graph_defs)
    if (g) (void)hipGraphDestroy(g);
  d.graphs.clear();
  d.graph_defs.clear();
  const size_t np = (size_t)d.npad;
  for (auto *b : {&w.u, &w.r, &w.p, &w.q, &w.z, &w.f}) {
    b->alloc(np);
    b->zero();
  }
  w.rH.alloc((size_t)std::max<int64_t>(d.m0, 1));
  w.c.alloc((size_t)std::max<int64_t>(d.m0, 1));
  w.rH.zero();
  w.c.zero();
  w.partials.alloc(kMaxGrid);
  w.sc.alloc(1);
  w.sc.zero();
  w.k = k;
}

StarArgs star_args(DeviceState &d) {
  StarArgs a{};
  a.nstars = d.nstars;
  a.order = d.order.p;
  a.st_n = d.st_n.p;
  a.st_vb = d.st_vb.p;
  a.st_q = d.st_q.p;
  a.st_gb = d.st_gb.p;
  a.st_fb = d.st_fb.p;
  a.st_bb = d.st_bb.p;
  a.pos_dof = d.pos_dof.p;
  a.f_go = d.f_go.p;
  a.f_gw = d.f_gw.p;
  a.b_go = d.b_go.p;
  a.b_gw = d.b_gw.p;
  a.pad = d.pad;
  if (d.precision == SN_PREC_FP32_STARS) {
    a.f_inv = d.f_inv32.p;
    a.b_inv = d.b_inv32.p;
    a.f_val = d.f_val32.p;
    a.b_val = d.b_val32.p;
    a.slots = d.slots32.p;
  } else {
    a.f_inv = d.f_inv64.p;
    a.b_inv = d.b_inv64.p;
    a.f_val = d.f_val64.p;
    a.b_val = d.b_val64.p;
    a.slots = d.slots64.p;
  }
  return a;
}

template <typename T>
void launch_star(DeviceState &d, const double *r, const CgScalars *sc, int check, hipStream_t s) {
  const size_t lds = (size_t)(d.maxn + 2 * d.pad) * sizeof(T);
  if (lds > 65536)
    HIPCHK(hipFuncSetAttribute((const void *)k_star<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_star<T>, dim3(d.nstars), dim3(64), lds, s, star_args(d), r, sc, check);
}

// z = B r; with check = 1 the kernels skip work once the recurrence is done and
// r.z goes to the partials
void launch_B(DeviceState &d, const double *r, double *z, CgScalars *sc, int check, hipStream_t s) {
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
  if (d.nstars > 0) {
    if (d.precision == SN_PREC_FP32_STARS) launch_star<float>(d, r, sc, check, s);
    else launch_star<double>(d, r, sc, check, s);
  }
  if (d.profiling) {
    HIPCHK(hipEventRecord(ev.second, s));
    d.ev_used.push_back(ev);
  }
  Workspace &w = d.ws;
  if (d.m0 > 0) {
    hipLaunchKernelGGL(k_restrict, dim3((unsigned)d.m0), dim3(kBlock), 0, s, d.PTptr.p, d.PTdof.p, d.PTw.p, r, w.rH.p,
                       (int)d.m0, sc, check);
    hipLaunchKernelGGL(k_coarse_gemv, dim3(nblk(d.m0 * 64)), dim3(kBlock), 0, s, d.Kinv.p, w.rH.p, w.c.p, (int)d.m0,
                       sc, check);
  }
  const unsigned G = grid_for(d.npad);
  double *parts = check ? w.partials.p : nullptr;
  if (d.precision == SN_PREC_FP32_STARS)
    hipLaunchKernelGGL(k_reduce<float>, dim3(G), dim3(kBlock), 0, s, z, r, d.slots32.p, d.slot_of.p, d.Pc.p, d.Pw.p,
                       w.c.p, (int)d.npad, d.nv, sc, parts);
  else
    hipLaunchKernelGGL(k_reduce<double>, dim3(G), dim3(kBlock), 0, s, z, r, d.slots64.p, d.slot_of.p, d.Pc.p, d.Pw.p,
                       w.c.p, (int)d.npad, d.nv, sc, parts);
  if (check) hipLaunchKernelGGL(k_scalar, dim3(1), dim3(kBlock), 0, s, w.partials.p, (int)G, sc, (int)OP_BETA);
}

void launch_spmv(DeviceState &d, const double *x, double *y, CgScalars *sc, bool dot, hipStream_t s) {
  Sell A{d.sptr.p, d.slen.p, d.col.p, d.val.p};
  const unsigned G = grid_for(d.npad);
  hipLaunchKernelGGL(k_spmv, dim3(G), dim3(kBlock), 0, s, A, x, y, (int)d.npad, sc, dot ? d.ws.partials.p : nullptr);
  if (dot) hipLaunchKernelGGL(k_scalar, dim3(1), dim3(kBlock), 0, s, d.ws.partials.p, (int)G, sc, (int)OP_ALPHA);
}

void launch_iteration(DeviceState &d, hipStream_t s) {
  Workspace &w = d.ws;
  if (d.profiling) ++d.prof_iters;
  CgScalars *sc = w.sc.p;
  const unsigned G = grid_for(d.npad);
  launch_spmv(d, w.p.p, w.q.p, sc, true, s);
  hipLaunchKernelGGL(k_cg_update, dim3(G), dim3(kBlock), 0, s, w.u.p, w.r.p, w.p.p, w.q.p, (int)d.npad, sc,
                     w.partials.p);
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(kBlock), 0, s, w.partials.p, (int)G, sc, (int)OP_CONV);
  launch_B(d, w.r.p, w.z.p, sc, 1, s);
  hipLaunchKernelGGL(k_p_update, dim3(G), dim3(kBlock), 0, s, w.p.p, w.z.p, (int)d.npad, sc);
}

// run m iterations: as captured graphs of 2^i iterations, or launch by launch
void run_iterations(DeviceState &d, int m, bool use_graph, hipStream_t s) {
  if (!use_graph || d.profiling) {
    for (int it = 0; it < m; ++it) launch_iteration(d, s);
    return;
  }
  for (int i = 0; m > 0; ++i) {
    if (!(m & (1 << i))) continue;
    if ((int)d.graphs.size() <= i) {
      d.graphs.resize(i + 1, nullptr);
      d.graph_defs.resize(i + 1, nullptr);
    }
    if (!d.graphs[i]) {
      // capture on the library's own stream, replay on the caller's
      HIPCHK(hipStreamSynchronize(s));
      HIPCHK(hipStreamBeginCapture(d.own, hipStreamCaptureModeRelaxed));
      for (int it = 0; it < (1 << i); ++it) launch_iteration(d, d.own);
      HIPCHK(hipStreamEndCapture(d.own, &d.graph_defs[i]));
      HIPCHK(hipGraphInstantiate(&d.graphs[i], d.graph_defs[i], nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(d.graphs[i], s));
    m -= 1 << i;
  }
}

double device_dot(DeviceState &d, const double *a, const double *b, hipStream_t s) {
  Workspace &w = d.ws;
  const unsigned G = grid_for(d.npad);
  hipLaunchKernelGGL(k_dot, dim3(G), dim3(kBlock), 0, s, a, b, (int)d.npad, w.partials.p);
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(kBlock), 0, s, w.partials.p, (int)G, w.sc.p, (int)OP_DOT);
  double v = 0;
  HIPCHK(hipMemcpyAsync(&v, &w.sc.p->tmp, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return v;
}

// copy column c of an n x k block (host or device) into a padded device vector
void load_column(DeviceState &d, double *dst, const double *src, int k, int c, bool dev_ptrs, hipStream_t s) {
  const int64_t n = d.n;
  if (dev_ptrs) {
    hipLaunchKernelGGL(k_gather_col, dim3(grid_for(n)), dim3(kBlock), 0, s, dst, src, (int)n, k, c);
  } else {
    std::vector<double> tmp((size_t)n);
    for (int64_t i = 0; i < n; ++i) tmp[i] = src[(size_t)i * k + c];
    HIPCHK(hipMemcpyAsync(dst, tmp.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
}

void store_column(DeviceState &d, double *dst, const double *src, int k, int c, bool dev_ptrs, hipStream_t s) {
  const int64_t n = d.n;
  if (dev_ptrs) {
    hipLaunchKernelGGL(k_scatter_col, dim3(grid_for(n)), dim3(kBlock), 0, s, dst, src, (int)n, k, c);
  } else {
    std::vector<double> tmp((size_t)n);
    HIPCHK(hipMemcpyAsync(tmp.data(), src, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) dst[(size_t)i * k + c] = tmp[i];
  }
}

}  // namespace

void device_profile(Precond &pre, int enable) {
  DeviceState &d = *pre.dev;
  HIPCHK(hipDeviceSynchronize());
  for (auto &e : d.ev_used) d.ev_free.push_back(e);
  d.ev_used.clear();
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
}

void device_apply_K(Precond &pre, int k, const double *x, double *y, int device_ptrs, void *stream) {
  DeviceState &d = *pre.dev;
  hipStream_t s = stream ? (hipStream_t)stream : d.own;
  ensure_ws(d, k);
  Workspace &w = d.ws;
  for (int c = 0; c < k; ++c) {
    load_column(d, w.p.p, x, k, c, device_ptrs, s);
    launch_spmv(d, w.p.p, w.q.p, w.sc.p, false, s);
    store_column(d, y, w.q.p, k, c, device_ptrs, s);
  }
  HIPCHK(hipStreamSynchronize(s));
}

void device_apply_B(Precond &pre, int k, const double *r, double *z, int device_ptrs, void *stream) {
  DeviceState &d = *pre.dev;
  hipStream_t s = stream ? (hipStream_t)stream : d.own;
  ensure_ws(d, k);
  Workspace &w = d.ws;
  for (int c = 0; c < k; ++c) {
    load_column(d, w.r.p, r, k, c, device_ptrs, s);
    launch_B(d, w.r.p, w.z.p, w.sc.p, 0, s);
    store_column(d, z, w.z.p, k, c, device_ptrs, s);
  }
  HIPCHK(hipStreamSynchronize(s));
}

void device_solve(Precond &pre, int k, const double *f, double *u, const sn_solve_opts &o, sn_solve_info *info) {
  DeviceState &d = *pre.dev;
  hipStream_t s = o.stream ? (hipStream_t)o.stream : d.own;
  ensure_ws(d, k);
  Workspace &w = d.ws;
  const int check = o.check_every > 0 ? o.check_every : 8;
  bool all_conv = true;
  for (int c = 0; c < k; ++c) {
    const auto t0 = std::chrono::steady_clock::now();
    load_column(d, w.f.p, f, k, c, o.device_ptrs != 0, s);
    if (o.use_u0) load_column(d, w.u.p, u, k, c, o.device_ptrs != 0, s);
    else HIPCHK(hipMemsetAsync(w.u.p, 0, (size_t)d.npad * sizeof(double), s));
    // r = f - K u
    if (o.use_u0) {
      launch_spmv(d, w.u.p, w.q.p, w.sc.p, false, s);
      hipLaunchKernelGGL(k_sub, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, w.r.p, w.f.p, w.q.p, (int)d.npad);
    } else {
      HIPCHK(hipMemcpyAsync(w.r.p, w.f.p, (size_t)d.npad * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    const double f2 = device_dot(d, w.f.p, w.f.p, s);
    const double r2 = device_dot(d, w.r.p, w.r.p, s);
    CgScalars h{};
    h.f2 = f2;
    h.tol2 = o.rtol * o.rtol * f2;
    h.max_iter = (int32_t)std::min<int64_t>(o.max_iter > 0 ? o.max_iter : 1000, 1 << 30);
    h.fixed = (int32_t)std::max<int64_t>(o.fixed_iters, 0);
    h.first = 1;
    h.rr = r2;
    h.done = (h.fixed == 0 && r2 <= h.tol2) || (h.fixed == 0 && f2 == 0.0) ? 1 : 0;
    HIPCHK(hipMemcpyAsync(w.sc.p, &h, sizeof(h), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    int replacements = 0;
    if (!h.done) {
      // z = B r, rho = r.z, p = z
      launch_B(d, w.r.p, w.z.p, w.sc.p, 1, s);
      HIPCHK(hipMemcpyAsync(w.p.p, w.z.p, (size_t)d.npad * sizeof(double), hipMemcpyDeviceToDevice, s));
      int64_t since_replace = 0;
      // iterations queued between read-backs: first `check`, then the number the
      // observed contraction of ||r||^2 predicts is still needed (>= 1)
      int block = h.fixed > 0 ? std::min(check, h.fixed) : check;
      double prev_rr = h.rr;
      int prev_it = 0;
      for (;;) {
        run_iterations(d, block, o.use_graph != 0, s);
        HIPCHK(hipMemcpyAsync(&h, w.sc.p, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        since_replace += block;
        if (h.fixed > 0) {
          block = std::max(1, std::min(4 * check, h.fixed - h.iters));
        } else {
          const int di = h.iters - prev_it;
          block = check;
          if (di > 0 && h.rr > 0.0 && prev_rr > h.rr && h.rr > h.tol2) {
            const double rate = std::pow(h.rr / prev_rr, 1.0 / di);
            const double need = std::log(h.tol2 / h.rr) / std::log(rate);
            if (std::isfinite(need)) block = (int)std::max(1.0, std::min((double)(4 * check), std::ceil(need)));
          }
          prev_rr = h.rr;
          prev_it = h.iters;
        }
        if (h.done) {
          // confirm with the true residual. When it exceeds the tolerance by a
          // small factor the recurrence has drifted: restart from it. A true
          // residual far above the tolerance is the attainable accuracy of the
          // system in FP64, which a restart cannot improve.
          if (h.fixed == 0 && h.rr <= h.tol2 && h.iters < h.max_iter) {
            launch_spmv(d, w.u.p, w.q.p, w.sc.p, false, s);
            hipLaunchKernelGGL(k_sub, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, w.q.p, w.f.p, w.q.p, (int)d.npad);
            const double t2 = device_dot(d, w.q.p, w.q.p, s);
            if (t2 > h.tol2 * 1.0000001 && t2 < 100.0 * h.tol2 && replacements < 3) {
              // restart from the true residual: r = f - K u, z = B r, p = z
              HIPCHK(hipMemcpyAsync(w.r.p, w.q.p, (size_t)d.npad * sizeof(double), hipMemcpyDeviceToDevice, s));
              ++replacements;
              h.done = 0;
              h.rr = t2;
              h.first = 1;
              HIPCHK(hipMemcpyAsync(w.sc.p, &h, sizeof(h), hipMemcpyHostToDevice, s));
              HIPCHK(hipStreamSynchronize(s));
              launch_B(d, w.r.p, w.z.p, w.sc.p, 1, s);
              HIPCHK(hipMemcpyAsync(w.p.p, w.z.p, (size_t)d.npad * sizeof(double), hipMemcpyDeviceToDevice, s));
              since_replace = 0;
              block = check;
              prev_rr = t2;
              prev_it = h.iters;
              continue;
            }
          }
          break;
        }
        if (o.replace_every > 0 && since_replace >= o.replace_every) {
          launch_spmv(d, w.u.p, w.q.p, w.sc.p, false, s);
          hipLaunchKernelGGL(k_sub, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, w.r.p, w.f.p, w.q.p, (int)d.npad);
          ++replacements;
          since_replace = 0;
        }
      }
    }
    // true residual
    launch_spmv(d, w.u.p, w.q.p, w.sc.p, false, s);
    hipLaunchKernelGGL(k_sub, dim3(grid_for(d.npad)), dim3(kBlock), 0, s, w.q.p, w.f.p, w.q.p, (int)d.npad);
    const double t2 = device_dot(d, w.q.p, w.q.p, s);
    store_column(d, u, w.u.p, k, c, o.device_ptrs != 0, s);
    HIPCHK(hipStreamSynchronize(s));
    const double fn = std::sqrt(f2);
    info[c].iters = h.iters;
    info[c].res_rec = fn > 0 ? std::sqrt(h.rr) / fn : std::sqrt(h.rr);
    info[c].res_true = fn > 0 ? std::sqrt(t2) / fn : std::sqrt(t2);
    info[c].converged = (h.fixed > 0) ? 1 : (h.rr <= h.tol2 ? 1 : 0);
    info[c].replacements = replacements;
    info[c].ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (!info[c].converged) all_conv = false;
  }
  if (!all_conv) fail(SN_ENOCONV, "PCG reached max_iter before the tolerance");
}

}  // namespace spnet
