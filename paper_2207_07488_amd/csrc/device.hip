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
// Dot products are reduced per block in a fixed order and the partials are
// combined in a fixed order by a one-block kernel, so results do not depend on
// scheduling. The star sweeps live in star_kernel.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "device_common.hpp"

namespace spnet {


constexpr int kBlock = 256;   // threads of the vector kernels
constexpr int kSlice = 64;    // rows per ELL slice (one wavefront)
constexpr int kMaxGrid = 1024;  // blocks of the grid-stride vector kernels (= partial sums)

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
  int32_t n_narrow = 0, n_wide = 0, maxn_narrow = 0, maxn_wide = 0;
  hipStream_t aux = nullptr;       // wide stars run beside the narrow ones
  hipEvent_t fork = nullptr, join = nullptr;
  DBuf<int32_t> order_narrow, order_wide, st_n, st_vb, st_q, st_gb, pos_dof, slot_of;
  DBuf<uint32_t> f_hdr, b_hdr;
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
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (aux) (void)hipStreamDestroy(aux);
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

// Pack one sweep stream of a star: steps in groups of SG (the first step of
// every group a multiple of SG), values divided by the step's pivot. Lane l
// and window register q read slot u = ((l - j0 - 1) mod 64) + 64 q of the group
// with first step j0 (mod 64); slot u holds, for k = 0..SG-1, entry
// t = 64 q + ((u mod 64 - k) mod 64) of step j0 + k (zero past the step's width).
// The group stores slots 0..W-1, W one past the last non-zero slot.
template <typename T>
void pack_stream(const std::vector<int32_t> &width, const std::vector<double> &vals, const std::vector<double> &inv,
                 int SG, int Q, std::vector<T> &out, std::vector<uint32_t> &hdr, int64_t base) {
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
    const int64_t off = ((int64_t)out.size() - base) / SG;  // 16-byte units (groups are whole slots)
    if (off >= (1 << 21) || W >= (1 << 11)) fail(SN_EINVAL, "star stream too large for the packed group headers");
    hdr.push_back((uint32_t)W << 21 | (uint32_t)off);
    for (int slot = 0; slot < W; ++slot)
      for (int k = 0; k < SG; ++k) out.push_back((T)entry(j0, slot, k));
  }
  // zero headers past the end: the sweep reads whole blocks of headers ahead
  const int GPB = 64 / SG;
  const size_t ng = (size_t)(n + SG - 1) / SG;
  const size_t padded = (ng + GPB - 1) / GPB * GPB + 3 * GPB;
  hdr.resize(hdr.size() + (padded - ng), 0u);
}

template <typename T>
void upload_stars(DeviceState &d, const Precond &pre, const HostFactors &hf, sn_factor_info &fi) {
  constexpr int SG = 16 / (int)sizeof(T);
  const int64_t ns = (int64_t)hf.stars.size();
  std::vector<int32_t> st_n(ns), st_vb(ns), st_q(ns), st_gb(ns), pos_dof;
  std::vector<uint32_t> f_hdr, b_hdr;
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
    st_gb[s] = (int32_t)f_hdr.size();
    maxq = std::max(maxq, q);
    maxband = std::max(maxband, F.band);
    d.maxn = std::max(d.maxn, F.n);
    // forward: columns j; backward: rows n-1-s
    std::vector<double> finv(F.invdiag), binv((size_t)F.n);
    for (int p = 0; p < F.n; ++p) binv[p] = F.invdiag[F.n - 1 - p];
    st_fb[s] = (int64_t)f_val.size();
    pack_stream<T>(F.width_fwd, F.colvals, finv, SG, q, f_val, f_hdr, st_fb[s]);
    st_bb[s] = (int64_t)b_val.size();
    pack_stream<T>(F.width_bwd, F.rowvals, binv, SG, q, b_val, b_hdr, st_bb[s]);
    if (f_hdr.size() != b_hdr.size()) fail(SN_EINVAL, "internal: header arrays out of step");
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
  // schedule: longest chain first, narrow and wide windows in separate kernels
  std::vector<int32_t> narrow, wide;
  for (int64_t s = 0; s < ns; ++s) (st_q[s] <= 2 ? narrow : wide).push_back((int32_t)s);
  auto by_len = [&](int32_t a, int32_t b) { return st_n[a] > st_n[b]; };
  std::stable_sort(narrow.begin(), narrow.end(), by_len);
  std::stable_sort(wide.begin(), wide.end(), by_len);
  d.n_narrow = (int32_t)narrow.size();
  d.n_wide = (int32_t)wide.size();
  d.maxn_narrow = narrow.empty() ? 0 : st_n[narrow[0]];
  d.maxn_wide = wide.empty() ? 0 : st_n[wide[0]];
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
  d.order_narrow.upload(narrow);
  d.order_wide.upload(wide);
  d.st_n.upload(st_n);
  d.st_vb.upload(st_vb);
  d.st_q.upload(st_q);
  d.st_gb.upload(st_gb);
  d.st_fb.upload(st_fb);
  d.st_bb.upload(st_bb);
  d.pos_dof.upload(pos_dof);
  d.f_hdr.upload(f_hdr);
  d.b_hdr.upload(b_hdr);
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
  HIPCHK(hipStreamCreateWithFlags(&d->aux, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&d->fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&d->join, hipEventDisableTiming));
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
  d->bytes = (int64_t)(d->sptr.bytes() + d->slen.bytes() + d->col.bytes() + d->val.bytes() + d->order_narrow.bytes() +
                       d->order_wide.bytes() +
                       d->st_n.bytes() + d->st_vb.bytes() + d->st_q.bytes() + d->st_gb.bytes() + d->st_fb.bytes() +
                       d->st_bb.bytes() + d->pos_dof.bytes() + d->f_hdr.bytes() + d->b_hdr.bytes() +
                       d->slot_of.bytes() + d->Kinv.bytes() + d->Pc.bytes() + d->Pw.bytes() +
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
  a.nstars = d.n_narrow;
  a.order = d.order_narrow.p;
  a.st_n = d.st_n.p;
  a.st_vb = d.st_vb.p;
  a.st_q = d.st_q.p;
  a.st_gb = d.st_gb.p;
  a.st_fb = d.st_fb.p;
  a.st_bb = d.st_bb.p;
  a.pos_dof = d.pos_dof.p;
  a.f_hdr = d.f_hdr.p;
  a.b_hdr = d.b_hdr.p;
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
    StarArgs a = star_args(d);
    StarArgs aw = a;
    aw.nstars = d.n_wide;
    aw.order = d.order_wide.p;
    const bool f32 = d.precision == SN_PREC_FP32_STARS;
    if (d.n_wide > 0 && d.n_narrow > 0) {
      // fork: the wide stars run on the auxiliary stream beside the narrow ones
      HIPCHK(hipEventRecord(d.fork, s));
      HIPCHK(hipStreamWaitEvent(d.aux, d.fork, 0));
      if (f32) launch_star_fp32(aw, true, d.maxn_wide, r, sc, check, d.aux);
      else launch_star_fp64(aw, true, d.maxn_wide, r, sc, check, d.aux);
      HIPCHK(hipEventRecord(d.join, d.aux));
    } else if (d.n_wide > 0) {
      if (f32) launch_star_fp32(aw, true, d.maxn_wide, r, sc, check, s);
      else launch_star_fp64(aw, true, d.maxn_wide, r, sc, check, s);
    }
    if (d.n_narrow > 0) {
      if (f32) launch_star_fp32(a, false, d.maxn_narrow, r, sc, check, s);
      else launch_star_fp64(a, false, d.maxn_narrow, r, sc, check, s);
    }
    if (d.n_wide > 0 && d.n_narrow > 0) HIPCHK(hipStreamWaitEvent(s, d.join, 0));
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
