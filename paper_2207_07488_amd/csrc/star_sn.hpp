// Supernodal local solves z_j = K_j^{-1} r[S_j] (the direct solves
// behind the projections P_j, Sec. 4.1), templated on the factor precision T,
// the column count KC and the columns CW a wavefront carries. Included by
// star_inst.hip only.
//
// One workgroup per star; its wavefronts ("teams") take the star's column
// chunks of CW columns in turn and share the star's factor, which is staged in
// LDS once (the index part when it fits beside the vectors, the values when
// they fit too) and read from there by both solves; what is not staged is read
// from global memory.
//
// The factor of a star (see factor.cpp) is level-scheduled: its supernodes are
// grouped by height in the supernodal tree and positions are numbered level by
// level. Supernode k owns positions c0 .. c0+w-1 and has h rows below its
// diagonal block; S_k = [L_CC^{-1}; L_RC L_CC^{-1}] is stored lower
// trapezoidal, column c holding rows c .. w+h-1. With x the gathered r, per
// level l = 0, 1, ... (forward, L y = x):
//   A(l)  x_p -= sum of the u-slots aimed at p          (p in level l, l > 0)
//   B(l)  y_p  = sum_{c <= p-c0} S_k[p-c0][c] x_{c0+c}  (p in level l)
//         u_e  = sum_{c < w}     S_k[w+e-ub][c] x_{c0+c} (u-slots e of level l)
// and per level l = top .. 0 (backward, L^T z = y), z kept in x:
//   C(l)  z_p  = sum_{r >= j} S_k[r][j] y_{c0+r} - sum_i S_k[w+i][j] z_{R_i}  (j = p-c0)
// Every phase is a set of independent dot products between wavefront-ordered
// LDS accesses; each dot product adds its terms in a fixed order, so the
// result does not depend on scheduling. All arithmetic is in T (FP32 with FP32
// accumulation in the mixed form).
#pragma once
#include "device_common.hpp"

namespace spnet {

// LDS accesses of one wavefront complete in order; the fences keep the
// compiler from moving them across a phase boundary
__device__ __forceinline__ void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SnView {
  const uint32_t *lev;  // lev[l]: first position of level l (nlev + 1 entries)
  const SnPos *pos;     // per position: its supernode and the u-slots aimed at it
  const uint16_t *R, *alist, *bpos;
  // the level table held in registers (nlev < 64 and a wavefront team): lane
  // l has the first position of level l, read with readlane
  int lv_pos;
  bool lv_reg;
  __device__ __forceinline__ int level(int l) const {
    return lv_reg ? __builtin_amdgcn_readlane(lv_pos, l) : (int)lev[l];
  }
};

// offset of column c in a lower-trapezoidal block of leading dimension ld
// (column c holds rows c .. ld-1)
__device__ __forceinline__ uint32_t col_off(uint32_t c, uint32_t ld) { return c * ld - (c * (c - 1u)) / 2u; }

// a * b + c with one rounding, in the precision of T
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += s * v (CW columns), s taken as 0 when !on
template <typename T, int CW>
__device__ __forceinline__ void fma_row(T (&acc)[CW], bool on, T s, const Row<T, CW> &v) {
  const T f = on ? s : T(0);
#pragma unroll
  for (int c = 0; c < CW; ++c) acc[c] = fma_t(f, v.v[c], acc[c]);
}

// One team: CW columns of one star. G = false: the team is one wavefront and
// the vectors x, y (n x CW), u (nu x CW) and the index part are in LDS, S (the
// star's values) in LDS or global memory. G = true: the team is the whole
// workgroup and everything is in global memory (stars too large for LDS).
//
// Work per level: every position p of the level is one task (one lane).
//   forward A  x_p -= u-slots aimed at p (its u-slot list, ascending)
//   forward B  y_p = row r = p - c0 of L_CC^{-1} times x_C, and the update rows
//              i = r, r + w, r + 2w, ... < h of its supernode:
//              u_{ubase+i} = row i of L_RC L_CC^{-1} times x_C
//   backward   z_p = column j = p - c0 of S_k against (y_C, -z_R)
// Terms are added in ascending order (columns, rows, list entries); loads go
// in batches of eight with clamped indices (masked terms contribute zero), so
// that a task waits for few dependent memory round trips.
template <bool G>
__device__ __forceinline__ void phase_sync() {
  if constexpr (G) __syncthreads();
  else team_sync();
}

template <typename T, int CW, bool G>
__device__ __forceinline__ void team_solve(const SnView &B, const T *__restrict__ S, int nlev, T *x, T *y, T *u) {
  const int lane = G ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int NT = G ? (int)blockDim.x : 64;
  using RowT = Row<T, CW>;
  // forward
  for (int l = 0; l < nlev; ++l) {
    const int p0 = B.level(l), p1 = B.level(l + 1);
    if (l > 0) {
      for (int p = p0 + lane; p < p1; p += NT) {
        const SnPos P = B.pos[p];
        const int a0 = P.a0, a1 = P.a1;
        if (a0 == a1) continue;
        RowT a;
        a.load(x + (size_t)p * CW);
        for (int q0 = a0; q0 < a1; q0 += 8) {
          int idx[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) idx[i] = B.alist[min(q0 + i, a1 - 1)];
          RowT t[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) t[i].load(u + (size_t)idx[i] * CW);
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (q0 + i < a1) {
#pragma unroll
              for (int c = 0; c < CW; ++c) a.v[c] -= t[i].v[c];
            }
        }
        a.store(x + (size_t)p * CW);
      }
      phase_sync<G>();
    }
    for (int p = p0 + lane; p < p1; p += NT) {
      const SnPos P = B.pos[p];
      const int c0 = P.c0, w = P.w, h = P.h, r = p - c0;
      const uint32_t ld = (uint32_t)(w + h);
      const T *sk = S + P.sbase;
      T *ub = u + (size_t)P.ubase * CW;
      if (w <= 8) {
        // x_C in registers; row r of L_CC^{-1}, then the update rows
        RowT xc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) xc[c].load(x + (size_t)(c0 + min(c, w - 1)) * CW);
        T acc[CW];
#pragma unroll
        for (int c = 0; c < CW; ++c) acc[c] = T(0);
        T sv[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) sv[c] = sk[c <= r ? col_off((uint32_t)c, ld) + (uint32_t)(r - c) : 0u];
#pragma unroll
        for (int c = 0; c < 8; ++c) fma_row<T, CW>(acc, c <= r, sv[c], xc[c]);
        RowT o;
#pragma unroll
        for (int c = 0; c < CW; ++c) o.v[c] = acc[c];
        o.store(y + (size_t)p * CW);
        for (int i = r; i < h; i += w) {
          const uint32_t row = (uint32_t)(w + i);
#pragma unroll
          for (int c = 0; c < 8; ++c) sv[c] = sk[c < w ? col_off((uint32_t)c, ld) + row - (uint32_t)c : 0u];
#pragma unroll
          for (int c = 0; c < CW; ++c) acc[c] = T(0);
#pragma unroll
          for (int c = 0; c < 8; ++c) fma_row<T, CW>(acc, c < w, sv[c], xc[c]);
#pragma unroll
          for (int c = 0; c < CW; ++c) o.v[c] = acc[c];
          o.store(ub + (size_t)i * CW);
        }
      } else {
        // wide supernode: every row in chunks of eight columns
        for (int i = r - w; i < h; i = (i < 0 ? r : i + w)) {
          const bool tri = i < 0;
          const uint32_t row = tri ? (uint32_t)r : (uint32_t)(w + i);
          const int len = tri ? r + 1 : w;
          T acc[CW];
#pragma unroll
          for (int c = 0; c < CW; ++c) acc[c] = T(0);
          for (int q0 = 0; q0 < len; q0 += 8) {
            T sv[8];
            RowT xv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int c = min(q0 + q, len - 1);
              sv[q] = sk[col_off((uint32_t)c, ld) + row - (uint32_t)c];
              xv[q].load(x + (size_t)(c0 + c) * CW);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) fma_row<T, CW>(acc, q0 + q < len, sv[q], xv[q]);
          }
          RowT o;
#pragma unroll
          for (int c = 0; c < CW; ++c) o.v[c] = acc[c];
          o.store(tri ? y + (size_t)p * CW : ub + (size_t)i * CW);
        }
      }
    }
    phase_sync<G>();
  }
  // backward, z in x
  for (int l = nlev - 1; l >= 0; --l) {
    const int p0 = B.level(l), p1 = B.level(l + 1);
    for (int p = p0 + lane; p < p1; p += NT) {
      const SnPos P = B.pos[p];
      const int c0 = P.c0, w = P.w, h = P.h, j = p - c0;
      const T *col = S + P.sbase + col_off((uint32_t)j, (uint32_t)(w + h));
      T acc[CW];
#pragma unroll
      for (int c = 0; c < CW; ++c) acc[c] = T(0);
      // rows j .. w-1 of the column against y
      const int m1 = w - j;
      for (int q0 = 0; q0 < m1; q0 += 8) {
        T sv[8];
        RowT yv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int t = min(q0 + q, m1 - 1);
          sv[q] = col[t];
          yv[q].load(y + (size_t)(p + t) * CW);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) fma_row<T, CW>(acc, q0 + q < m1, sv[q], yv[q]);
      }
      // rows below the block against -z_R
      const T *mc = col + m1;
      const uint16_t *Rk = B.R + P.ubase;
      for (int q0 = 0; q0 < h; q0 += 8) {
        int ri[8];
        T sv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int t = min(q0 + q, h - 1);
          ri[q] = Rk[t];
          sv[q] = -mc[t];
        }
        RowT zv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) zv[q].load(x + (size_t)ri[q] * CW);
#pragma unroll
        for (int q = 0; q < 8; ++q) fma_row<T, CW>(acc, q0 + q < h, sv[q], zv[q]);
      }
      RowT o;
#pragma unroll
      for (int c = 0; c < CW; ++c) o.v[c] = acc[c];
      o.store(x + (size_t)p * CW);
    }
    phase_sync<G>();
  }
}

// gather r (CW of the KC adjacent columns, from col0) in factor order: the dof
// of position p is that of the star's slot bpos[p]; eight positions per
// thread in flight, NT threads from `lane`
template <typename T, int KC, int CW>
__device__ __forceinline__ void gather(T *x, const double *__restrict__ r, const int32_t *__restrict__ dofs,
                                       const uint16_t *bpos, int n, int col0, int lane, int NT) {
  for (int p0 = 0; p0 < n; p0 += NT * 8) {
    int idx[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) idx[q] = bpos[min(p0 + NT * q + lane, n - 1)];
#pragma unroll
    for (int q = 0; q < 8; ++q) idx[q] = dofs[idx[q]];
    Row<double, CW> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q].load(r + (size_t)idx[q] * KC + col0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      Row<T, CW> o;
#pragma unroll
      for (int c = 0; c < CW; ++c) o.v[c] = (T)v[q].v[c];
      o.store(x + (size_t)min(p0 + NT * q + lane, n - 1) * CW);
    }
  }
}

// One star per workgroup (see the header of this file); lds: the workgroup's
// dynamic LDS. k_sn runs up to four wavefronts, k_sn_wide up to sixteen (more
// wavefronts than column chunks solve the chunks together).
template <typename T, int KC, int CW>
__device__ __forceinline__ void sn_star(unsigned char *lds, const SnArgs &a, const double *__restrict__ r,
                                        const CgScalars *sc, int sel) {
  const int st = a.order[blockIdx.x];
  const unsigned char *gb = a.blob + a.st_blob[st];
  const SnHeader hd = *reinterpret_cast<const SnHeader *>(gb);
  const int n = (int)hd.n, nu = (int)hd.nu, nlev = (int)hd.nlev;
  const int nteam = (int)(blockDim.x >> 6), team = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  constexpr int NCH = KC / CW;
  // the column chunks this workgroup has to solve
  uint32_t chunks = 0;
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    bool on = false;
#pragma unroll
    for (int c = 0; c < CW; ++c) on |= sel == SEL_ALL || column_selected(sc[ch * CW + c], sel, 0u, ch * CW + c);
    if (on) chunks |= 1u << ch;
  }
  if (!chunks) return;
  const uint32_t xb = (uint32_t)((n * CW * (int)sizeof(T) + 15) & ~15);
  const uint32_t ub = (uint32_t)((nu * CW * (int)sizeof(T) + 15) & ~15);
  const uint32_t vec = 2 * xb + ub;
  // more wavefronts than column chunks: the whole workgroup solves one chunk
  // after the other (one set of vectors, workgroup barriers between phases)
  const bool coop = nteam > NCH;
  const uint32_t vsets = coop ? 1u : (uint32_t)nteam;
  // the index part is staged when it fits beside the vectors (else it is read
  // from global memory), the values when they fit too; the update slots stay
  // in global memory (a.vscratch) when x and y alone take the LDS
  const bool il = hd.idx_bytes + vsets * vec <= (uint32_t)a.lds_bytes;
  const bool ul = il || vsets * vec <= (uint32_t)a.lds_bytes;
  const bool vl = il && hd.idx_bytes + hd.val_bytes + vsets * vec <= (uint32_t)a.lds_bytes;
  const uint32_t staged = il ? hd.idx_bytes + (vl ? hd.val_bytes : 0u) : 0u;
  {
    // index part (and values) to LDS, 16 bytes per thread and load, sixteen
    // loads per thread in flight
    const float4 *src = reinterpret_cast<const float4 *>(gb);
    float4 *dst = reinterpret_cast<float4 *>(lds);
    const int n16 = (int)(staged >> 4);
    const int bs = (int)blockDim.x;
    // indices past the end are clamped for the loads and the stores alike (a
    // lane then rewrites the last chunk with its own value), so that no load
    // sits behind a branch and all of them are in flight together
    for (int i0 = (int)threadIdx.x; i0 < n16; i0 += 16 * bs) {
      float4 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = src[min(i0 + q * bs, n16 - 1)];
#pragma unroll
      for (int q = 0; q < 16; ++q) dst[min(i0 + q * bs, n16 - 1)] = v[q];
    }
  }
  const unsigned char *ib = il ? lds : gb;
  SnView B;
  B.lev = reinterpret_cast<const uint32_t *>(ib + hd.off_lev);
  B.lv_reg = nlev < 64;
  B.pos = reinterpret_cast<const SnPos *>(ib + hd.off_pos);
  B.R = reinterpret_cast<const uint16_t *>(ib + hd.off_R);
  B.alist = reinterpret_cast<const uint16_t *>(ib + hd.off_alist);
  B.bpos = reinterpret_cast<const uint16_t *>(ib + hd.off_bpos);
  unsigned char *tv = lds + staged + (coop ? 0u : (uint32_t)team * vec);
  T *x = reinterpret_cast<T *>(tv), *y = reinterpret_cast<T *>(tv + xb);
  T *u = ul ? reinterpret_cast<T *>(tv + 2 * xb) : reinterpret_cast<T *>(a.vscratch + a.st_vs[st]);
  const int32_t *dofs = a.pos_dof + a.st_pos[st];
  T *out = static_cast<T *>(a.slots) + (size_t)a.st_pos[st] * KC;
  __syncthreads();
  B.lv_pos = (int)B.lev[min(lane, nlev)];
  if (coop) {
    const int tid = (int)threadIdx.x, NT = (int)blockDim.x;
    for (int ch = 0; ch < NCH; ++ch) {
      if (!((chunks >> ch) & 1u)) continue;
      const int col0 = ch * CW;
      gather<T, KC, CW>(x, r, dofs, B.bpos, n, col0, tid, NT);
      __syncthreads();
      if (vl) team_solve<T, CW, true>(B, reinterpret_cast<const T *>(lds + hd.idx_bytes), nlev, x, y, u);
      else team_solve<T, CW, true>(B, reinterpret_cast<const T *>(gb + hd.idx_bytes), nlev, x, y, u);
      for (int p = tid; p < n; p += NT) {
        Row<T, CW> o;
        o.load(x + (size_t)p * CW);
        o.store(out + (size_t)B.bpos[p] * KC + col0);
      }
      __syncthreads();
    }
    return;
  }
  for (int ch = team; ch < NCH; ch += nteam) {
    if (!((chunks >> ch) & 1u)) continue;
    const int col0 = ch * CW;
    gather<T, KC, CW>(x, r, dofs, B.bpos, n, col0, lane, 64);
    team_sync();
    if (vl) team_solve<T, CW, false>(B, reinterpret_cast<const T *>(lds + hd.idx_bytes), nlev, x, y, u);
    else team_solve<T, CW, false>(B, reinterpret_cast<const T *>(gb + hd.idx_bytes), nlev, x, y, u);
    // z_j to the star's slots
    for (int p = lane; p < n; p += 64) {
      Row<T, CW> o;
      o.load(x + (size_t)p * CW);
      o.store(out + (size_t)B.bpos[p] * KC + col0);
    }
    team_sync();
  }
}

template <typename T, int KC, int CW>
__global__ __launch_bounds__(256) void k_sn(SnArgs a, const double *__restrict__ r, const CgScalars *sc, int sel) {
  extern __shared__ __align__(16) unsigned char lds[];
  sn_star<T, KC, CW>(lds, a, r, sc, sel);
}

template <typename T, int KC, int CW>
__global__ __launch_bounds__(1024) void k_sn_wide(SnArgs a, const double *__restrict__ r, const CgScalars *sc,
                                                  int sel) {
  extern __shared__ __align__(16) unsigned char lds[];
  sn_star<T, KC, CW>(lds, a, r, sc, sel);
}

// Stars too large for LDS: the whole workgroup (4 or 16 wavefronts) solves one
// column chunk after the other with the factor read from the blob and the
// vectors in the global scratch at a.vscratch + a.st_vs[star].
template <typename T, int KC, int CW>
__global__ __launch_bounds__(1024) void k_sn_global(SnArgs a, const double *__restrict__ r, const CgScalars *sc,
                                                     int sel) {
  const int st = a.order[blockIdx.x];
  const unsigned char *gb = a.blob + a.st_blob[st];
  const SnHeader hd = *reinterpret_cast<const SnHeader *>(gb);
  const int n = (int)hd.n, nlev = (int)hd.nlev;
  constexpr int NCH = KC / CW;
  SnView B;
  B.lev = reinterpret_cast<const uint32_t *>(gb + hd.off_lev);
  B.lv_reg = false;
  B.lv_pos = 0;
  B.pos = reinterpret_cast<const SnPos *>(gb + hd.off_pos);
  B.R = reinterpret_cast<const uint16_t *>(gb + hd.off_R);
  B.alist = reinterpret_cast<const uint16_t *>(gb + hd.off_alist);
  B.bpos = reinterpret_cast<const uint16_t *>(gb + hd.off_bpos);
  const uint32_t xb = (uint32_t)((n * CW * (int)sizeof(T) + 15) & ~15);
  unsigned char *tv = a.vscratch + a.st_vs[st];
  T *x = reinterpret_cast<T *>(tv), *y = reinterpret_cast<T *>(tv + xb), *u = reinterpret_cast<T *>(tv + 2 * xb);
  const int32_t *dofs = a.pos_dof + a.st_pos[st];
  T *out = static_cast<T *>(a.slots) + (size_t)a.st_pos[st] * KC;
  const int tid = (int)threadIdx.x, NT = (int)blockDim.x;
  for (int ch = 0; ch < NCH; ++ch) {
    bool on = false;
#pragma unroll
    for (int c = 0; c < CW; ++c) on |= sel == SEL_ALL || column_selected(sc[ch * CW + c], sel, 0u, ch * CW + c);
    if (!on) continue;
    const int col0 = ch * CW;
    gather<T, KC, CW>(x, r, dofs, B.bpos, n, col0, tid, NT);
    __syncthreads();
    team_solve<T, CW, true>(B, reinterpret_cast<const T *>(gb + hd.idx_bytes), nlev, x, y, u);
    for (int p = tid; p < n; p += NT) {
      Row<T, CW> o;
      o.load(x + (size_t)p * CW);
      o.store(out + (size_t)B.bpos[p] * KC + col0);
    }
    __syncthreads();
  }
}

template <typename T, int KC, int CW>
void launch_sn_t(const SnArgs &a, int nteam, bool global, const double *r, const CgScalars *sc, int sel,
                 hipStream_t s) {
  if (a.nstars <= 0) return;
  if (global) {
    if (nteam != 4 && nteam != 16) fail(SN_EINVAL, "4 or 16 wavefronts per star solved from global memory");
    hipLaunchKernelGGL((k_sn_global<T, KC, CW>), dim3(a.nstars), dim3(64 * nteam), 0, s, a, r, sc, sel);
    return;
  }
  // allow the kernels the whole LDS of a compute unit (once per instantiation)
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sn<T, KC, CW>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, kStarMaxLds);
  static const hipError_t attr_w = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sn_wide<T, KC, CW>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, kStarMaxLds);
  if (attr != hipSuccess || attr_w != hipSuccess)
    fail(SN_EDEVICE, std::string("star kernel LDS limit: ") + hipGetErrorString(attr != hipSuccess ? attr : attr_w));
  if (nteam < 1 || nteam > 16) fail(SN_EINVAL, "1 to 16 wavefronts per star");
  if (nteam <= 4)
    hipLaunchKernelGGL((k_sn<T, KC, CW>), dim3(a.nstars), dim3(64 * nteam), (size_t)a.lds_bytes, s, a, r, sc, sel);
  else
    hipLaunchKernelGGL((k_sn_wide<T, KC, CW>), dim3(a.nstars), dim3(64 * nteam), (size_t)a.lds_bytes, s, a, r, sc,
                       sel);
}

}  // namespace spnet
