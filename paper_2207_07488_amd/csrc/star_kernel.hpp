// Star sweep kernel (templated on the factor precision): see the comment
// below. Included by star_fp32.hip and star_fp64.hip only.
#pragma once
#include "device_common.hpp"

namespace spnet {

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
  template <int L>
  static __device__ __forceinline__ float lane(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
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
  template <int L>
  static __device__ __forceinline__ double lane(double v) {
    return mk(__builtin_amdgcn_readlane(lo(v), L), __builtin_amdgcn_readlane(hi(v), L));
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
//
// Rows stay in their lanes: lane l, register q holds the row r = l (mod 64)
// that is the (q+1)-th such row after the current step j. Step j reads the
// finished row j from lane j mod 64 (a constant lane inside the unrolled
// block), that lane moves its later rows down one register and takes the
// next row from the incoming vector, and every lane subtracts its entry times
// g_j. Lane l of register q therefore needs entry t = ((l - j - 1) mod 64) + 64 q
// of step j; the host stores the SG steps of a group skewed so that lane l
// fetches all of them with one 16-byte load from slot ((l - j0 - 1) mod 64) + 64 q,
// j0 the group's first step.
// read-only data read through the constant address space (scalar loads)
typedef const __attribute__((address_space(4))) uint32_t *const_u32_ptr;

template <typename T, int Q, int RG, bool REV>
__device__ __forceinline__ void sweep(T *vec, int n, const uint32_t *__restrict__ hdr_g, const T *__restrict__ inv,
                                      const T *__restrict__ vals) {
  const const_u32_ptr hdr = (const_u32_ptr)hdr_g;
  using P = Pack<T>;
  using V = typename P::V;
  constexpr int SG = P::SG, GPB = 64 / SG;
  static_assert(GPB % RG == 0, "ring must divide the groups of a block");
  static_assert(GPB + RG <= 2 * GPB, "ring lookahead spans at most the next block");
  const int lane = threadIdx.x & 63;
  auto at = [&](int p) -> int { return REV ? (n - 1 - p) : p; };
  T g[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) g[q] = vec[at(lane + 64 * q)];
  T inc = vec[at(64 * Q + lane)];  // lane l: the row entering at step l of the block
  T hinv = lane < n ? inv[lane] : T(0);
  // group headers (uniform): width << 21 | offset in 16-byte units; hc: this
  // block, hn: the next (the header array is padded with zeros past the end)
  uint32_t hc[GPB], hn[GPB];
#pragma unroll
  for (int i = 0; i < GPB; ++i) {
    hc[i] = hdr[i];
    hn[i] = hdr[GPB + i];
  }
  auto fetch = [&](uint32_t h, int s0, V(&dst)[Q]) {
    const T *base = vals + (size_t)(h & 0x1FFFFFu) * SG;
    const int w = (int)(h >> 21);
    const int ub = (lane - s0 - 1) & 63;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const V v = *reinterpret_cast<const V *>(base + (ub + 64 * q) * SG);
      dst[q] = P::masked(ub + 64 * q < w, v);
    }
  };
  V ring[RG][Q];
#pragma unroll
  for (int rg = 0; rg < RG; ++rg) fetch(hc[rg], (rg * SG) & 63, ring[rg]);
  for (int jb = 0; jb < n; jb += 64) {
    const int gb = jb / SG;
    uint32_t hnn[GPB];
#pragma unroll
    for (int i = 0; i < GPB; ++i) hnn[i] = hdr[gb + 2 * GPB + i];
    const T hinvN = jb + 64 + lane < n ? inv[jb + 64 + lane] : T(0);
    const T incN = vec[at(jb + 64 + 64 * Q + lane)];
    T ybuf = T(0);
    StaticFor<0, 64>::run([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      constexpr int gi = s / SG, k = s % SG;
      const T gj = P::template lane<s>(g[0]);
      ybuf = P::template put<s>(ybuf, gj);
#pragma unroll
      for (int q = 0; q + 1 < Q; ++q) g[q] = P::template put<s>(g[q], P::template lane<s>(g[q + 1]));
      g[Q - 1] = P::template put<s>(g[Q - 1], P::template lane<s>(inc));
#pragma unroll
      for (int q = 0; q < Q; ++q) g[q] = g[q] - P::get(ring[gi % RG][q], k) * gj;
      if constexpr (k == SG - 1) {
        // the group is consumed: fetch the group RG positions ahead
        constexpr int li = gi + RG;
        fetch(li < GPB ? hc[li % GPB] : hn[li % GPB], (li * SG) & 63, ring[gi % RG]);
      }
    });
    if (jb + lane < n) vec[at(jb + lane)] = ybuf * hinv;
    hinv = hinvN;
    inc = incN;
#pragma unroll
    for (int i = 0; i < GPB; ++i) {
      hc[i] = hn[i];
      hn[i] = hnn[i];
    }
  }
}

template <typename T, int Q>
__device__ __forceinline__ void star_solve(const StarArgs &a, int st, int n, T *vec, int &sink) {
  constexpr int GPB = 64 / Pack<T>::SG;
  constexpr int RG0 = 16 / Q;
  constexpr int RG = RG0 >= GPB ? GPB : (RG0 >= 8 ? 8 : (RG0 >= 4 ? 4 : (RG0 >= 2 ? 2 : 1)));
  const int vb = a.st_vb[st], gbase = a.st_gb[st];
  const T *finv = static_cast<const T *>(a.f_inv) + vb, *binv = static_cast<const T *>(a.b_inv) + vb;
  const T *fval = static_cast<const T *>(a.f_val) + a.st_fb[st], *bval = static_cast<const T *>(a.b_val) + a.st_bb[st];
  sweep<T, Q, RG, false>(vec, n, a.f_hdr + gbase, finv, fval);
  __syncthreads();
  sweep<T, Q, RG, true>(vec, n, a.b_hdr + gbase, binv, bval);
  (void)sink;
}

// WIDE = false: stars with windows of 1-2 registers, true: 4-16 registers (kept
// in separate kernels so that each gets the registers its variants need)
template <typename T, bool WIDE>
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
  // gather r in factor order, 16 rows per lane in flight at a time
  const int32_t *dofs = a.pos_dof + vb;
  for (int p0 = 0; p0 < n; p0 += 64 * 16) {
    // unconditional loads at clamped positions keep all 16 in flight
    int idx[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) idx[u] = dofs[min(p0 + 64 * u + lane, n - 1)];
    double val[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) val[u] = r[idx[u]];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int p = p0 + 64 * u + lane;
      if (p < n) vec[p] = (T)val[u];
    }
  }
  __syncthreads();
  int sink = 0;
  if constexpr (!WIDE) {
    if (Q == 1) star_solve<T, 1>(a, st, n, vec, sink);
    else star_solve<T, 2>(a, st, n, vec, sink);
  } else {
    if (Q == 4) star_solve<T, 4>(a, st, n, vec, sink);
    else if (Q == 8) star_solve<T, 8>(a, st, n, vec, sink);
    else star_solve<T, 16>(a, st, n, vec, sink);
  }
  __syncthreads();
  T *out = static_cast<T *>(a.slots) + vb;
  for (int p = lane; p < n; p += 64) out[p] = vec[p];
}

// one launch over the stars of a.order (all narrow or all wide)
template <typename T>
void launch_star_t(const StarArgs &a, bool wide, int maxn, const double *r, const CgScalars *sc, int check,
                   hipStream_t s) {
  if (a.nstars <= 0) return;
  const size_t lds = (size_t)(maxn + 2 * a.pad) * sizeof(T);
  const void *fn = wide ? (const void *)k_star<T, true> : (const void *)k_star<T, false>;
  if (lds > 65536) HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (wide) hipLaunchKernelGGL((k_star<T, true>), dim3(a.nstars), dim3(64), lds, s, a, r, sc, check);
  else hipLaunchKernelGGL((k_star<T, false>), dim3(a.nstars), dim3(64), lds, s, a, r, sc, check);
}


}  // namespace spnet
