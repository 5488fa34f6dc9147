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

// ---------------------------------------------------------------------------
// device scalars of one PCG recurrence
// ---------------------------------------------------------------------------
struct CgScalars {
  double rho, alpha, beta, pq, rr, rz, f2, tol2;
  double tmp;          // scratch dot result
  int32_t iters, done, max_iter, fixed, first, pad0;
  uint32_t ticket[8];  // last-block counters, one per reduction site
};

enum { T_PQ = 0, T_RR = 1, T_RZ = 2, T_DOT = 3 };

// ---------------------------------------------------------------------------
// wavefront / block reductions with a fixed combination order
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

__device__ __forceinline__ double load_coherent(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish this block's partial; returns true in the block that finishes last,
// whose thread 0 then gets the fixed-order total in *total.
__device__ bool last_block_total(double part, double *partials, uint32_t *ticket, double *total, double *sh) {
  __shared__ bool amlast;
  if (threadIdx.x == 0) {
    __hip_atomic_store(&partials[blockIdx.x], part, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const uint32_t t = atomicAdd(ticket, 1u);
    amlast = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!amlast) return false;
  __threadfence();
  double s = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) s += load_coherent(&partials[i]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    *total = s;
    *ticket = 0u;
  }
  return true;
}

// ---------------------------------------------------------------------------
// sliced ELL SpMV: y = K x, optional x.y reduction
// ---------------------------------------------------------------------------
struct Sell {
  const int32_t *sptr;  // slice start (elements)
  const int32_t *slen;  // slice width
  const int32_t *col;
  const double *val;
};

__global__ __launch_bounds__(kBlock) void k_spmv(Sell A, const double *__restrict__ x, double *__restrict__ y,
                                                 int nslices, CgScalars *sc, double *partials, int mode) {
  __shared__ double sh[kBlock / 64];
  if (mode == 1 && sc->done) return;
  const int row = blockIdx.x * kBlock + threadIdx.x;
  const int s = row >> 6, lane = row & 63;
  double acc = 0.0;
  if (s < nslices) {
    const int base = A.sptr[s], len = A.slen[s];
    for (int c = 0; c < len; ++c) {
      const int e = base + c * kSlice + lane;
      acc += A.val[e] * x[A.col[e]];
    }
    y[row] = acc;
  }
  if (mode != 1) return;
  const double part = block_sum(s < nslices ? x[row] * acc : 0.0, sh);
  double tot;
  if (last_block_total(part, partials, &sc->ticket[T_PQ], &tot, sh) && threadIdx.x == 0) {
    sc->pq = tot;
    sc->alpha = sc->rho / tot;
  }
}

// u += alpha p, r -= alpha q, r.r, convergence test
__global__ __launch_bounds__(kBlock) void k_cg_update(double *u, double *r, const double *p, const double *q, int n,
                                                      CgScalars *sc, double *partials) {
  __shared__ double sh[kBlock / 64];
  if (sc->done) return;
  const double a = sc->alpha;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double rr = 0.0;
  if (i < n) {
    u[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    rr = ri * ri;
  }
  const double part = block_sum(rr, sh);
  double tot;
  if (last_block_total(part, partials, &sc->ticket[T_RR], &tot, sh) && threadIdx.x == 0) {
    sc->rr = tot;
    const int it = sc->iters + 1;
    sc->iters = it;
    bool stop;
    if (sc->fixed > 0) stop = it >= sc->fixed;
    else stop = (tot <= sc->tol2) || it >= sc->max_iter;
    if (stop) sc->done = 1;
  }
}

// z = P c + sum of star slots, r.z, beta
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_reduce(double *z, const double *r, const TS *__restrict__ slots,
                                                   const int32_t *__restrict__ slot_of,
                                                   const int32_t *__restrict__ Pc, const double *__restrict__ Pw,
                                                   const double *__restrict__ cvec, int n, int nv, CgScalars *sc,
                                                   double *partials, int mode) {
  __shared__ double sh[kBlock / 64];
  if (mode == 1 && sc->done) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double rz = 0.0;
  if (i < n) {
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
    rz = r[i] * acc;
  }
  if (mode != 1) return;
  const double part = block_sum(rz, sh);
  double tot;
  if (last_block_total(part, partials, &sc->ticket[T_RZ], &tot, sh) && threadIdx.x == 0) {
    sc->rz = tot;
    sc->beta = sc->first ? 0.0 : tot / sc->rho;
    sc->rho = tot;
    sc->first = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_p_update(double *p, const double *z, int n, CgScalars *sc) {
  if (sc->done) return;
  const double b = sc->beta;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = z[i] + b * p[i];
}

// r_H = P^T r: one wavefront per coarse dof, fixed-order lane sums
__global__ __launch_bounds__(kBlock) void k_restrict(const int32_t *__restrict__ ptr, const int32_t *__restrict__ dof,
                                                     const double *__restrict__ w, const double *__restrict__ r,
                                                     double *rH, int m0, CgScalars *sc, int mode) {
  if (mode == 1 && sc->done) return;
  const int c = (blockIdx.x * kBlock + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (c >= m0) return;
  double acc = 0.0;
  for (int q = ptr[c] + lane; q < ptr[c + 1]; q += 64) acc += w[q] * r[dof[q]];
  acc = wave_sum(acc);
  if (lane == 0) rH[c] = acc;
}

// c = K_0^{-1} r_H, one wavefront per row of the dense inverse
__global__ __launch_bounds__(kBlock) void k_coarse_gemv(const double *__restrict__ Kinv, const double *__restrict__ rH,
                                                        double *cvec, int m0, CgScalars *sc, int mode) {
  if (mode == 1 && sc->done) return;
  const int row = (blockIdx.x * kBlock + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (row >= m0) return;
  const double *a = Kinv + (size_t)row * m0;
  double acc = 0.0;
  for (int j = lane; j < m0; j += 64) acc += a[j] * rH[j];
  acc = wave_sum(acc);
  if (lane == 0) cvec[row] = acc;
}

__global__ __launch_bounds__(kBlock) void k_dot(const double *a, const double *b, int n, CgScalars *sc,
                                                double *partials) {
  __shared__ double sh[kBlock / 64];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const double part = block_sum(i < n ? a[i] * b[i] : 0.0, sh);
  double tot;
  if (last_block_total(part, partials, &sc->ticket[T_DOT], &tot, sh) && threadIdx.x == 0) sc->tmp = tot;
}

// y = a - b
__global__ __launch_bounds__(kBlock) void k_sub(double *y, const double *a, const double *b, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = a[i] - b[i];
}

// strided column gather / scatter between n x k blocks and a contiguous vector
__global__ __launch_bounds__(kBlock) void k_gather_col(double *dst, const double *src, int n, int k, int c) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[(size_t)i * k + c];
}
__global__ __launch_bounds__(kBlock) void k_scatter_col(double *dst, const double *src, int n, int k, int c) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[(size_t)i * k + c] = src[i];
}

// ---------------------------------------------------------------------------
// Star sweeps. One wavefront solves L_j L_j^T z = r[S_j] for one star.
//
// The vector of the star lives in LDS in factor order. A sweep walks the
// steps of a stream: the forward stream holds the columns of L (step j: the
// entries L_{j+1..j+w, j}), the backward stream the rows of L from the last
// (step s = row n-1-s: L_{i,i-1..i-w}); with the vector read in reverse order
// the backward sweep is the same recurrence as the forward one.
//
// Window: before step j, lane l of register g[q] holds the running value of
// row j + l + 64 q. Lane 0 of g[0] is then final: y_j = g * (1/L_jj). The
// window slides by one lane (DPP wave shift left), the next row enters at lane
// 63 of the last register, and every lane updates its row with the column
// entry t = lane + 64 q. Column values are loaded R steps ahead into a
// register ring; step headers (offset, width, 1/diag) arrive 64 at a time.
// ---------------------------------------------------------------------------
struct StarArgs {
  int32_t nstars;
  const int32_t *order;   // stars of this launch, largest first
  const int32_t *st_n;
  const int32_t *st_vb;   // base position of the star in all per-position arrays
  const int64_t *st_fb;   // forward stream value base
  const int64_t *st_bb;   // backward stream value base
  const int32_t *pos_dof; // global dof of each position (factor order)
  const int32_t *f_off, *f_w, *b_off, *b_w;  // per-step headers
  const void *f_inv, *b_inv;                 // 1/diag per step (T)
  const void *f_val, *b_val;                 // stream values (T)
  void *slots;                               // T, per position
  int32_t pad;                               // LDS zero padding each side (elements)
};

template <typename T>
struct Lanes;
template <>
struct Lanes<float> {
  static __device__ __forceinline__ float first(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
  }
  static __device__ __forceinline__ float lane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
  }
  static __device__ __forceinline__ float put(float old, float v, int l) {
    return (int)(threadIdx.x & 63) == l ? v : old;
  }
  // lanes 0..62 take lane+1, lane 63 takes `in`
  static __device__ __forceinline__ float shl(float v, float in) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(in), __float_as_int(v), 0x130, 0xF, 0xF, false));
  }
};
template <>
struct Lanes<double> {
  static __device__ __forceinline__ int lo(double v) { return (int)(uint32_t)(__double_as_longlong(v)); }
  static __device__ __forceinline__ int hi(double v) { return (int)(uint32_t)(__double_as_longlong(v) >> 32); }
  static __device__ __forceinline__ double mk(int l, int h) {
    return __longlong_as_double(((long long)(uint32_t)h << 32) | (long long)(uint32_t)l);
  }
  static __device__ __forceinline__ double first(double v) {
    return mk(__builtin_amdgcn_readfirstlane(lo(v)), __builtin_amdgcn_readfirstlane(hi(v)));
  }
  static __device__ __forceinline__ double lane(double v, int l) {
    return mk(__builtin_amdgcn_readlane(lo(v), l), __builtin_amdgcn_readlane(hi(v), l));
  }
  static __device__ __forceinline__ double put(double old, double v, int l) {
    return (int)(threadIdx.x & 63) == l ? v : old;
  }
  static __device__ __forceinline__ double shl(double v, double in) {
    return mk(__builtin_amdgcn_update_dpp(lo(in), lo(v), 0x130, 0xF, 0xF, false),
              __builtin_amdgcn_update_dpp(hi(in), hi(v), 0x130, 0xF, 0xF, false));
  }
};

// One sweep over n steps. vec points at position 0 of the LDS vector (with
// `pad` zero elements on both sides); rev selects reversed indexing.
template <typename T, int Q, int R, bool rev>
__device__ __forceinline__ void sweep(T *vec, int n, const int32_t *__restrict__ hoff,
                                      const int32_t *__restrict__ hw, const T *__restrict__ hinv,
                                      const T *__restrict__ vals) {
  const int lane = threadIdx.x & 63;
  auto at = [&](int p) -> int { return rev ? (n - 1 - p) : p; };
  T g[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) g[q] = vec[at(lane + 64 * q)];
  // header blocks: current, next, next-next
  int h_off0 = 0, h_w0 = 0, h_off1 = 0, h_w1 = 0, h_off2 = 0, h_w2 = 0;
  T h_inv0 = 0, h_inv1 = 0, h_inv2 = 0;
  if (lane < n) { h_off0 = hoff[lane]; h_w0 = hw[lane]; h_inv0 = hinv[lane]; }
  if (64 + lane < n) { h_off1 = hoff[64 + lane]; h_w1 = hw[64 + lane]; h_inv1 = hinv[64 + lane]; }
  if (128 + lane < n) { h_off2 = hoff[128 + lane]; h_w2 = hw[128 + lane]; h_inv2 = hinv[128 + lane]; }
  // value ring: ring[s % R] holds step (block base + s) values
  T ring[R][Q];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int o = __builtin_amdgcn_readlane(h_off0, s);
#pragma unroll
    for (int q = 0; q < Q; ++q) ring[s][q] = (s < n) ? vals[o + lane + 64 * q] : T(0);
  }
  T nxt0 = vec[at(64 * Q)], nxt1 = vec[at(64 * Q + 1)];
  // Steps past the end are harmless: their rows are zero padding, so y = 0.
  for (int jb = 0; jb < n; jb += 64) {
    T ybuf = 0;
#pragma unroll
    for (int s = 0; s < 64; ++s) {
      const int j = jb + s;
      const T inv = Lanes<T>::lane(h_inv0, s);
      const int w = __builtin_amdgcn_readlane(h_w0, s);
      const T y = Lanes<T>::first(g[0]) * inv;
      ybuf = Lanes<T>::shl(ybuf, y);  // after 64 steps lane l holds y of step jb + l
      T carry[Q];
#pragma unroll
      for (int q = 0; q + 1 < Q; ++q) carry[q] = Lanes<T>::first(g[q + 1]);
#pragma unroll
      for (int q = 0; q + 1 < Q; ++q) g[q] = Lanes<T>::shl(g[q], carry[q]);
      g[Q - 1] = Lanes<T>::shl(g[Q - 1], nxt0);
      nxt0 = nxt1;
      nxt1 = vec[at(j + 64 * Q + 2)];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const T lv = (lane + 64 * q < w) ? ring[s % R][q] : T(0);
        g[q] = g[q] - lv * y;
      }
      // loads of step j + R (offsets of steps past the end are 0: in bounds)
      const int o = (s + R < 64) ? __builtin_amdgcn_readlane(h_off0, (s + R) & 63)
                                 : __builtin_amdgcn_readlane(h_off1, (s + R) & 63);
#pragma unroll
      for (int q = 0; q < Q; ++q) ring[s % R][q] = vals[o + lane + 64 * q];
    }
    if (jb + lane < n) vec[at(jb + lane)] = ybuf;
    h_off0 = h_off1; h_w0 = h_w1; h_inv0 = h_inv1;
    h_off1 = h_off2; h_w1 = h_w2; h_inv1 = h_inv2;
    const int nb = jb + 192 + lane;
    h_off2 = 0; h_w2 = 0; h_inv2 = T(0);
    if (nb < n) { h_off2 = hoff[nb]; h_w2 = hw[nb]; h_inv2 = hinv[nb]; }
  }
}

template <typename T, int Q, int R>
__global__ __launch_bounds__(64) void k_star(StarArgs a, const double *__restrict__ r, const CgScalars *sc, int mode) {
  if (mode == 1 && sc->done) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);
  const int wv = blockIdx.x;
  if (wv >= a.nstars) return;
  const int st = a.order[wv];
  const int n = a.st_n[st], vb = a.st_vb[st];
  const int lane = threadIdx.x;
  T *vec = lds + a.pad;
  // zero the padding, gather r in factor order
  for (int i = lane; i < a.pad; i += 64) {
    lds[i] = T(0);
    vec[n + i] = T(0);
  }
  const int32_t *dofs = a.pos_dof + vb;
  for (int p = lane; p < n; p += 64) vec[p] = (T)r[dofs[p]];
  __syncthreads();
  sweep<T, Q, R, false>(vec, n, a.f_off + vb, a.f_w + vb, static_cast<const T *>(a.f_inv) + vb,
                 static_cast<const T *>(a.f_val) + a.st_fb[st]);
  __syncthreads();
  sweep<T, Q, R, true>(vec, n, a.b_off + vb, a.b_w + vb, static_cast<const T *>(a.b_inv) + vb,
                 static_cast<const T *>(a.b_val) + a.st_bb[st]);
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
};

struct StarBin {
  int Q = 1;
  int maxn = 0;
  DBuf<int32_t> order;
  int count = 0;
};

struct Workspace {
  int k = 0;
  DBuf<double> u, r, p, q, z, f, rH, c, partials, tmpk;
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
  int32_t nstars = 0, pad = 0;
  DBuf<int32_t> st_n, st_vb, pos_dof, f_off, f_w, b_off, b_w;
  DBuf<int64_t> st_fb, st_bb;
  DBuf<float> f_inv32, b_inv32, f_val32, b_val32, slots32;
  DBuf<double> f_inv64, b_inv64, f_val64, b_val64, slots64;
  std::vector<StarBin> bins;
  DBuf<int32_t> slot_of;
  // coarse
  DBuf<double> Kinv, PTw, Pw;
  DBuf<int32_t> PTptr, PTdof, Pc;
  Workspace ws;
  int64_t bytes = 0;
  ~DeviceState() {
    if (own) (void)hipStreamDestroy(own);
  }
};

void device_release(DeviceState *d) { delete d; }
void DeviceDeleter::operator()(DeviceState *d) const { delete d; }

namespace {

int pick_ring(int Q, bool dbl) {
  int regs = 64 / (dbl ? 2 : 1);  // ring registers budget (32-bit)
  int r = regs / Q;
  int p = 64;
  while (p > r && p > 4) p >>= 1;
  return p;
}

template <typename T, int Q, int R>
void launch_bin_t(const StarArgs &a, const StarBin &b, const double *r, const CgScalars *sc, int mode,
                  hipStream_t s, int pad) {
  StarArgs aa = a;
  aa.nstars = b.count;
  aa.order = b.order.p;
  const size_t lds = (size_t)(b.maxn + 2 * pad) * sizeof(T);
  if (lds > 65536) HIPCHK(hipFuncSetAttribute((const void *)k_star<T, Q, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)lds));
  hipLaunchKernelGGL((k_star<T, Q, R>), dim3(b.count), dim3(64), lds, s, aa, r, sc, mode);
}

template <typename T>
void launch_bin(const StarArgs &a, const StarBin &b, const double *r, const CgScalars *sc, int mode, hipStream_t s,
                int pad) {
  constexpr bool D = sizeof(T) == 8;
  switch (b.Q) {
    case 1: launch_bin_t<T, 1, D ? 16 : 32>(a, b, r, sc, mode, s, pad); break;
    case 2: launch_bin_t<T, 2, D ? 8 : 16>(a, b, r, sc, mode, s, pad); break;
    case 3: launch_bin_t<T, 3, D ? 4 : 8>(a, b, r, sc, mode, s, pad); break;
    case 4: launch_bin_t<T, 4, D ? 4 : 8>(a, b, r, sc, mode, s, pad); break;
    case 6: launch_bin_t<T, 6, D ? 2 : 4>(a, b, r, sc, mode, s, pad); break;
    case 8: launch_bin_t<T, 8, D ? 2 : 4>(a, b, r, sc, mode, s, pad); break;
    default: fail(SN_EINVAL, "unsupported star window");
  }
}

int bin_Q(int band) {
  const int q = (band + 63) / 64;
  if (q <= 4) return std::max(q, 1);
  if (q <= 6) return 6;
  if (q <= 8) return 8;
  return -1;
}

}  // namespace

void device_setup(Precond &pre, const HostFactors &hf, int precision) {
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
  const int64_t ns = (int64_t)hf.stars.size();
  d->nstars = (int32_t)ns;
  std::vector<int32_t> st_n(ns), st_vb(ns);
  std::vector<int64_t> st_fb(ns), st_bb(ns);
  int64_t tot = 0, fv = 0, bv = 0;
  int maxband = 0, maxn = 0;
  for (int64_t s = 0; s < ns; ++s) {
    const StarFactor &F = hf.stars[s];
    st_n[s] = F.n;
    st_vb[s] = (int32_t)tot;
    st_fb[s] = fv;
    st_bb[s] = bv;
    tot += F.n;
    fv += (int64_t)F.colvals.size();
    bv += (int64_t)F.rowvals.size();
    maxband = std::max(maxband, F.band);
    maxn = std::max(maxn, F.n);
  }
  if (tot >= (int64_t)1 << 31) fail(SN_EINVAL, "too many star positions");
  const int maxQ = std::max(1, bin_Q(maxband));
  if (bin_Q(maxband) < 0) fail(SN_EINVAL, "star band " + std::to_string(maxband) + " exceeds the widest sweep window (512)");
  d->pad = 64 * (maxQ + 3);
  const int64_t tailpad = 64 * 8 + 64;  // stream over-read slack
  std::vector<int32_t> pos_dof((size_t)tot), f_off((size_t)tot), f_w((size_t)tot), b_off((size_t)tot),
      b_w((size_t)tot);
  std::vector<double> f_inv((size_t)tot), b_inv((size_t)tot), f_val((size_t)(fv + tailpad), 0.0),
      b_val((size_t)(bv + tailpad), 0.0);
  std::vector<int32_t> slot_of((size_t)npad * d->nv, -1);
  int64_t star_nnz = 0;
  for (int64_t s = 0; s < ns; ++s) {
    const StarFactor &F = hf.stars[s];
    const int64_t vb = st_vb[s];
    const int32_t *dofs = &pre.star_dofs[pre.star_ptr[s]];
    int64_t of = 0, ob = 0;
    for (int p = 0; p < F.n; ++p) {
      const int32_t dof = dofs[F.perm[p]];
      pos_dof[vb + p] = dof;
      f_off[vb + p] = (int32_t)of;
      f_w[vb + p] = F.width_fwd[p];
      f_inv[vb + p] = F.invdiag[p];
      of += F.width_fwd[p];
      b_off[vb + p] = (int32_t)ob;
      b_w[vb + p] = F.width_bwd[p];
      b_inv[vb + p] = F.invdiag[F.n - 1 - p];
      ob += F.width_bwd[p];
    }
    std::copy(F.colvals.begin(), F.colvals.end(), f_val.begin() + st_fb[s]);
    std::copy(F.rowvals.begin(), F.rowvals.end(), b_val.begin() + st_bb[s]);
    star_nnz += F.nnz;
  }
  // dof -> slots in ascending star order
  {
    std::vector<int32_t> cnt((size_t)n, 0);
    for (int64_t s = 0; s < ns; ++s)
      for (int p = 0; p < st_n[s]; ++p) {
        const int32_t dof = pos_dof[st_vb[s] + p];
        if (cnt[dof] >= d->nv) fail(SN_EINVAL, "a dof lies in more stars than its element has mesh nodes");
        slot_of[(size_t)dof * d->nv + cnt[dof]++] = st_vb[s] + p;
      }
  }
  d->st_n.upload(st_n);
  d->st_vb.upload(st_vb);
  d->st_fb.upload(st_fb);
  d->st_bb.upload(st_bb);
  d->pos_dof.upload(pos_dof);
  d->f_off.upload(f_off);
  d->f_w.upload(f_w);
  d->b_off.upload(b_off);
  d->b_w.upload(b_w);
  d->slot_of.upload(slot_of);
  int64_t stream_bytes = 0;
  if (precision == SN_PREC_FP32_STARS) {
    auto cast = [](const std::vector<double> &v) {
      std::vector<float> o(v.size());
      for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
      return o;
    };
    d->f_inv32.upload(cast(f_inv));
    d->b_inv32.upload(cast(b_inv));
    d->f_val32.upload(cast(f_val));
    d->b_val32.upload(cast(b_val));
    d->slots32.alloc((size_t)tot);
    d->slots32.zero();
    stream_bytes = (int64_t)(d->f_val32.bytes() + d->b_val32.bytes() + d->f_inv32.bytes() + d->b_inv32.bytes());
  } else {
    d->f_inv64.upload(f_inv);
    d->b_inv64.upload(b_inv);
    d->f_val64.upload(f_val);
    d->b_val64.upload(b_val);
    d->slots64.alloc((size_t)tot);
    d->slots64.zero();
    stream_bytes = (int64_t)(d->f_val64.bytes() + d->b_val64.bytes() + d->f_inv64.bytes() + d->b_inv64.bytes());
  }
  // bins by window width, largest stars first
  {
    std::vector<std::vector<int32_t>> byq(9);
    for (int64_t s = 0; s < ns; ++s) byq[bin_Q(hf.stars[s].band < 1 ? 1 : hf.stars[s].band)].push_back((int32_t)s);
    for (int q = 1; q <= 8; ++q) {
      if (byq[q].empty()) continue;
      auto &v = byq[q];
      std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b) { return st_n[a] > st_n[b]; });
      StarBin b;
      b.Q = q;
      b.count = (int)v.size();
      b.maxn = st_n[v[0]];
      b.order.upload(v);
      d->bins.push_back(std::move(b));
    }
  }
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
  d->bytes = (int64_t)(d->sptr.bytes() + d->slen.bytes() + d->col.bytes() + d->val.bytes() + d->st_n.bytes() +
                       d->st_vb.bytes() + d->st_fb.bytes() + d->st_bb.bytes() + d->pos_dof.bytes() +
                       d->f_off.bytes() + d->f_w.bytes() + d->b_off.bytes() + d->b_w.bytes() + d->slot_of.bytes() +
                       d->Kinv.bytes() + d->Pc.bytes() + d->Pw.bytes() + d->PTptr.bytes() + d->PTdof.bytes() +
                       d->PTw.bytes()) +
             stream_bytes + (int64_t)(d->slots32.bytes() + d->slots64.bytes());
  pre.finfo.star_factor_nnz = star_nnz;
  pre.finfo.star_stream_bytes = stream_bytes;
  pre.finfo.coarse_bytes = (int64_t)d->Kinv.bytes();
  pre.finfo.device_bytes = d->bytes;
  pre.finfo.max_star_dofs = maxn;
  pre.finfo.max_band = maxband;
  pre.finfo.factor_seconds = hf.seconds;
  pre.precision = precision;
  pre.dev.reset(d.release());
}

namespace {

void ensure_ws(DeviceState &d, int k) {
  Workspace &w = d.ws;
  if (w.sc.p && w.k >= k) return;
  const size_t np = (size_t)d.npad;
  w.u.alloc(np);
  w.r.alloc(np);
  w.p.alloc(np);
  w.q.alloc(np);
  w.z.alloc(np);
  w.f.alloc(np);
  w.tmpk.alloc(np * (size_t)std::max(k, 1));
  w.rH.alloc((size_t)std::max<int64_t>(d.m0, 1));
  w.c.alloc((size_t)std::max<int64_t>(d.m0, 1));
  w.partials.alloc(np / kBlock + 64);
  w.sc.alloc(1);
  for (auto *b : {&w.u, &w.r, &w.p, &w.q, &w.z, &w.f, &w.rH, &w.c}) b->zero();
  w.sc.zero();
  w.k = k;
}

StarArgs star_args(DeviceState &d) {
  StarArgs a{};
  a.st_n = d.st_n.p;
  a.st_vb = d.st_vb.p;
  a.st_fb = d.st_fb.p;
  a.st_bb = d.st_bb.p;
  a.pos_dof = d.pos_dof.p;
  a.f_off = d.f_off.p;
  a.f_w = d.f_w.p;
  a.b_off = d.b_off.p;
  a.b_w = d.b_w.p;
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

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// z = B r (mode 1: part of a PCG iteration, also r.z and beta)
void launch_B(DeviceState &d, const double *r, double *z, CgScalars *sc, int mode, hipStream_t s) {
  const StarArgs a = star_args(d);
  for (const StarBin &b : d.bins) {
    if (d.precision == SN_PREC_FP32_STARS) launch_bin<float>(a, b, r, sc, mode, s, d.pad);
    else launch_bin<double>(a, b, r, sc, mode, s, d.pad);
  }
  Workspace &w = d.ws;
  if (d.m0 > 0) {
    hipLaunchKernelGGL(k_restrict, dim3(nblk(d.m0 * 64)), dim3(kBlock), 0, s, d.PTptr.p, d.PTdof.p, d.PTw.p, r, w.rH.p,
                       (int)d.m0, sc, mode);
    hipLaunchKernelGGL(k_coarse_gemv, dim3(nblk(d.m0 * 64)), dim3(kBlock), 0, s, d.Kinv.p, w.rH.p, w.c.p, (int)d.m0,
                       sc, mode);
  }
  if (d.precision == SN_PREC_FP32_STARS)
    hipLaunchKernelGGL(k_reduce<float>, dim3(nblk(d.npad)), dim3(kBlock), 0, s, z, r, d.slots32.p, d.slot_of.p,
                       d.Pc.p, d.Pw.p, w.c.p, (int)d.npad, d.nv, sc, w.partials.p, mode);
  else
    hipLaunchKernelGGL(k_reduce<double>, dim3(nblk(d.npad)), dim3(kBlock), 0, s, z, r, d.slots64.p, d.slot_of.p,
                       d.Pc.p, d.Pw.p, w.c.p, (int)d.npad, d.nv, sc, w.partials.p, mode);
}

void launch_spmv(DeviceState &d, const double *x, double *y, CgScalars *sc, int mode, hipStream_t s) {
  Sell A{d.sptr.p, d.slen.p, d.col.p, d.val.p};
  hipLaunchKernelGGL(k_spmv, dim3(nblk(d.npad)), dim3(kBlock), 0, s, A, x, y, d.nslices, sc, d.ws.partials.p, mode);
}

void launch_iteration(DeviceState &d, hipStream_t s) {
  Workspace &w = d.ws;
  CgScalars *sc = w.sc.p;
  launch_spmv(d, w.p.p, w.q.p, sc, 1, s);
  hipLaunchKernelGGL(k_cg_update, dim3(nblk(d.npad)), dim3(kBlock), 0, s, w.u.p, w.r.p, w.p.p, w.q.p, (int)d.npad, sc,
                     w.partials.p);
  launch_B(d, w.r.p, w.z.p, sc, 1, s);
  hipLaunchKernelGGL(k_p_update, dim3(nblk(d.npad)), dim3(kBlock), 0, s, w.p.p, w.z.p, (int)d.npad, sc);
}

double device_dot(DeviceState &d, const double *a, const double *b, hipStream_t s) {
  Workspace &w = d.ws;
  hipLaunchKernelGGL(k_dot, dim3(nblk(d.npad)), dim3(kBlock), 0, s, a, b, (int)d.npad, w.sc.p, w.partials.p);
  double v = 0;
  HIPCHK(hipMemcpyAsync(&v, &w.sc.p->tmp, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return v;
}

// copy column c of an n x k block (host or device) into a padded device vector
void load_column(DeviceState &d, double *dst, const double *src, int k, int c, bool dev_ptrs, hipStream_t s) {
  const int64_t n = d.n;
  if (dev_ptrs) {
    hipLaunchKernelGGL(k_gather_col, dim3(nblk(n)), dim3(kBlock), 0, s, dst, src, (int)n, k, c);
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
    hipLaunchKernelGGL(k_scatter_col, dim3(nblk(n)), dim3(kBlock), 0, s, dst, src, (int)n, k, c);
  } else {
    std::vector<double> tmp((size_t)n);
    HIPCHK(hipMemcpyAsync(tmp.data(), src, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) dst[(size_t)i * k + c] = tmp[i];
  }
}

}  // namespace

void device_apply_K(Precond &pre, int k, const double *x, double *y, int device_ptrs, void *stream) {
  DeviceState &d = *pre.dev;
  hipStream_t s = stream ? (hipStream_t)stream : d.own;
  ensure_ws(d, k);
  Workspace &w = d.ws;
  for (int c = 0; c < k; ++c) {
    load_column(d, w.p.p, x, k, c, device_ptrs, s);
    launch_spmv(d, w.p.p, w.q.p, w.sc.p, 0, s);
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
      launch_spmv(d, w.u.p, w.q.p, w.sc.p, 0, s);
      hipLaunchKernelGGL(k_sub, dim3(nblk(d.npad)), dim3(kBlock), 0, s, w.r.p, w.f.p, w.q.p, (int)d.npad);
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
      for (;;) {
        for (int it = 0; it < check; ++it) launch_iteration(d, s);
        HIPCHK(hipMemcpyAsync(&h, w.sc.p, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        since_replace += check;
        if (h.done) {
          // confirm with the true residual; continue from it if the recurrence drifted
          if (h.fixed == 0 && h.iters < h.max_iter) {
            launch_spmv(d, w.u.p, w.q.p, w.sc.p, 0, s);
            hipLaunchKernelGGL(k_sub, dim3(nblk(d.npad)), dim3(kBlock), 0, s, w.q.p, w.f.p, w.q.p, (int)d.npad);
            const double t2 = device_dot(d, w.q.p, w.q.p, s);
            if (t2 > h.tol2 * 1.0000001 && replacements < 20) {
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
              continue;
            }
          }
          break;
        }
        if (o.replace_every > 0 && since_replace >= o.replace_every) {
          launch_spmv(d, w.u.p, w.q.p, w.sc.p, 0, s);
          hipLaunchKernelGGL(k_sub, dim3(nblk(d.npad)), dim3(kBlock), 0, s, w.r.p, w.f.p, w.q.p, (int)d.npad);
          ++replacements;
          since_replace = 0;
        }
      }
    }
    // true residual
    launch_spmv(d, w.u.p, w.q.p, w.sc.p, 0, s);
    hipLaunchKernelGGL(k_sub, dim3(nblk(d.npad)), dim3(kBlock), 0, s, w.q.p, w.f.p, w.q.p, (int)d.npad);
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
