// Band star sweep kernel (envelope factors in reverse Cuthill-McKee order),
// templated on the factor precision T and the number of right-hand-side
// columns KC. Included by star_inst.hip only.
#pragma once
#include "device_common.hpp"

namespace spnet {

// ---------------------------------------------------------------------------
// Star sweeps: z_j = K_j^{-1} r[S_j] = L_j^{-T} L_j^{-1} r[S_j] for every star j
// (the local solves behind the projections P_j, Sec. 4.1), for KC columns at
// once. One wavefront per star; the factor streams are read once for all
// columns.
//
// The star's working vector (position-major: the KC values of a position are
// adjacent) is in factor order; it lives in LDS during the sweeps when the
// launch asks for it and the largest star's fits in 32 KB, else in the star's
// slot segment in global memory; z_j ends in the slot segment either way. The forward sweep
// walks the columns of L (step j: entries L_{j+1..j+w, j}); the backward sweep
// walks the rows of L from the last one (step s = row n-1-s: entries
// L_{i, i-1..i-w}) on the vector read in reverse, which makes it the same
// recurrence. Stream values are divided by the pivot of their step, so step j
// subtracts m_t g_j from row j+1+t with the raw running value g_j; the pivot
// division is applied when a row is written back.
//
// Window: lane l holds the rows r = l (mod 64) in registers R[0..Q]: R[q] is
// the row 64(b+q) + l during block b. At step j = 64b + s the finished row j
// sits in lane s of R[0]; the rows still to be updated are, for lanes l > s,
// R[0..Q-1], for lanes l <= s, R[1..Q]. The q-th of them needs stream entry
// t = ((l - j - 1) mod 64) + 64 q, which the host stores so that lane l loads
// it for SG consecutive steps with one 16-byte load (lanes past the group's
// width load zeros from a zero region). A per-lane select routes
// the loaded multiplier q to R[q] or R[q+1]; no row moves between lanes. At
// the end of a block R[0] holds 64 finished rows, the registers shift by one
// and the next rows enter from memory (loaded one block ahead).
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
  template <int L>
  static __device__ __forceinline__ float lane(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
  }
  // v with lane L replaced by the wavefront-uniform value u
  template <int L>
  static __device__ __forceinline__ float put(float u, float v) {
    asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(u), "i"(L));
    return v;
  }
  static __device__ __forceinline__ float fnma(float m, float g, float x) { return __builtin_fmaf(-m, g, x); }
  // per-lane selects at a step: lanes whose bit is set in `up` (an SGPR pair)
  // take `hi`, the others `lo`
  static __device__ __forceinline__ float pick(float hi, float lo, uint64_t up) {
    float r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(lo), "v"(hi), "s"(up));
    return r;
  }
  static __device__ __forceinline__ float pick_or_zero(float hi, uint64_t up) {
    float r;
    asm("v_cndmask_b32_e64 %0, 0, %1, %2" : "=v"(r) : "v"(hi), "s"(up));
    return r;
  }
  static __device__ __forceinline__ float zero_or_pick(float lo, uint64_t up) {
    float r;
    asm("v_cndmask_b32_e64 %0, %1, 0, %2" : "=v"(r) : "v"(lo), "s"(up));
    return r;
  }
};
template <>
struct Pack<double> {
  using V = double2;
  static constexpr int SG = 2;
  static __device__ __forceinline__ double get(const V &v, int k) { return k == 0 ? v.x : v.y; }
  static __device__ __forceinline__ int lo(double v) { return (int)(uint32_t)(__double_as_longlong(v)); }
  static __device__ __forceinline__ int hi(double v) { return (int)(uint32_t)(__double_as_longlong(v) >> 32); }
  static __device__ __forceinline__ double mk(int l, int h) {
    return __longlong_as_double(((long long)(uint32_t)h << 32) | (long long)(uint32_t)l);
  }
  template <int L>
  static __device__ __forceinline__ double lane(double v) {
    return mk(__builtin_amdgcn_readlane(lo(v), L), __builtin_amdgcn_readlane(hi(v), L));
  }
  template <int L>
  static __device__ __forceinline__ double put(double u, double v) {
    int vl = lo(v), vh = hi(v);
    asm("v_writelane_b32 %0, %1, %2" : "+v"(vl) : "s"(lo(u)), "i"(L));
    asm("v_writelane_b32 %0, %1, %2" : "+v"(vh) : "s"(hi(u)), "i"(L));
    return mk(vl, vh);
  }
  static __device__ __forceinline__ double fnma(double m, double g, double x) { return __builtin_fma(-m, g, x); }
  // per-lane selects at a step: lanes whose bit is set in `up` take `hi`
  // (both 32-bit halves selected with the same SGPR-pair mask)
  static __device__ __forceinline__ int sel32(int hi, int lo, uint64_t up) {
    int r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(lo), "v"(hi), "s"(up));
    return r;
  }
  static __device__ __forceinline__ int sel32_or_zero(int hi, uint64_t up) {
    int r;
    asm("v_cndmask_b32_e64 %0, 0, %1, %2" : "=v"(r) : "v"(hi), "s"(up));
    return r;
  }
  static __device__ __forceinline__ int zero_or_sel32(int lo, uint64_t up) {
    int r;
    asm("v_cndmask_b32_e64 %0, %1, 0, %2" : "=v"(r) : "v"(lo), "s"(up));
    return r;
  }
  static __device__ __forceinline__ double pick(double hi, double lo, uint64_t up) {
    return mk(sel32(Pack::lo(hi), Pack::lo(lo), up), sel32(Pack::hi(hi), Pack::hi(lo), up));
  }
  static __device__ __forceinline__ double pick_or_zero(double hi, uint64_t up) {
    return mk(sel32_or_zero(lo(hi), up), sel32_or_zero(Pack::hi(hi), up));
  }
  static __device__ __forceinline__ double zero_or_pick(double lo_v, uint64_t up) {
    return mk(zero_or_sel32(lo(lo_v), up), zero_or_sel32(hi(lo_v), up));
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

// read-only data read through the constant address space (scalar loads)
typedef const __attribute__((address_space(4))) uint32_t *const_u32_ptr;

// One sweep over the n steps of a stream for CW columns c0..c0+CW-1 of the
// star's slot segment `sl` (KC values per position). REV reads and writes the
// vector in reverse position order.
// TW: the sweep is one chain of a two-chain star (k_star_twin): at the block
// starting at step twin_k the forward sweeps of both chains exchange their
// window through xbuf (LDS) and add the partner's partial sums of the
// separator rows (every row of the window from twin_k on is a separator row
// or past the end, and the other chain's are zero until then).
template <typename T, int KC, int CW, int Q, int RG, bool REV, bool TW = false>
__device__ __forceinline__ void sweep(T *sl, int c0, int n, const uint16_t *__restrict__ hdr_g,
                                      const T *__restrict__ inv, const T *__restrict__ vals, uint32_t sbase,
                                      uint32_t zbase, int twin_k = -1, T *xbuf = nullptr) {
  using P = Pack<T>;
  using V = typename P::V;
  constexpr int SG = P::SG, GPB = 64 / SG;
  const int lane = threadIdx.x & 63;
  // row p of the sweep (clamped into the star; rows past the end read as 0)
  auto load_row = [&](int p, T (&dst)[CW]) {
    const int pc = p < n ? p : n - 1;
    Row<T, CW> rw;
    rw.load(sl + (size_t)(REV ? n - 1 - pc : pc) * KC + c0);
#pragma unroll
    for (int c = 0; c < CW; ++c) dst[c] = p < n ? rw.v[c] : T(0);
  };
  // One column and a window of one register (rows 64 b + l, and 64 (b + 1) + l
  // in R[1]): lane l keeps only its open row in R[0] and swaps in its next row
  // at step l, so that every step applies one multiplier per lane; the same
  // updates as the general form, without the zero ones.
  constexpr bool ROT = Q == 1 && CW == 1;
  T R[Q + 1][CW];
  T done = T(0);  // ROT: the finished rows of the block, lane l at step l
#pragma unroll
  for (int q = 0; q <= Q; ++q) load_row(lane + 64 * q, R[q]);
  T inc[CW];
  load_row(64 * (Q + 1) + lane, inc);
  T hinv = lane < n ? inv[lane] : T(0);
  // Group widths (16-bit, two per word; zero past the end of the stream). A
  // group starts where the previous one ends, so the fetches, which come in
  // group order, keep a running offset. The ring reaches RG groups ahead, i.e.
  // into block b + HB - 1. Lane i of `wcur` holds width word i counted from the
  // current block's first group; `wnext` (the same from the next block on) is
  // loaded at the start of a block, a block before it is used. Vector loads
  // complete in order, so waiting for it does not wait for later loads. A ring
  // longer than a block repeats its slots every UB blocks, so the loop body
  // covers UB blocks.
  constexpr int HB = RG > GPB ? 3 : 2;
  constexpr int UB = RG > GPB ? RG / GPB : 1;
  constexpr int WPB = GPB / 2;  // width words per block
  static_assert(RG <= GPB ? GPB % RG == 0 : (RG % GPB == 0 && UB <= 2), "ring and block sizes do not fit");
  const uint32_t *hw = reinterpret_cast<const uint32_t *>(hdr_g);
  const int wl = lane < HB * WPB ? lane : HB * WPB - 1;
  uint32_t wcur = hw[wl];
  auto width_of = [&](auto gc) -> uint32_t {  // group index from the current block's first
    constexpr int g = decltype(gc)::value;
    const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)wcur, g / 2);
    return (w >> (16 * (g % 2))) & 0xFFFFu;
  };
  uint32_t foff = 0;  // 16-byte offset of the next group to fetch
  // ring of group loads RG groups ahead; lanes past a group's width read the
  // zero region instead, so a loaded group is used as it is
  V ring[RG][Q];
  auto fetch = [&](uint32_t w, int s0, int rg) {
    const uint32_t gbase = sbase + foff * SG;
    foff += w;
    // lane offsets computed at each fetch rather than kept for every group
    int l = lane;
    asm volatile("; fetch lane %0" : "+v"(l));
    const uint32_t ub = (uint32_t)((l - s0 - 1) & 63);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const uint32_t u = ub + 64u * q;
      const uint32_t off = (u < w ? gbase : zbase) + u * SG;
      ring[rg][q] = *reinterpret_cast<const V *>(vals + off);
    }
  };
  StaticFor<0, RG>::run([&](auto rc) {
    constexpr int rg = decltype(rc)::value;
    fetch(width_of(rc), (rg * SG) & 63, rg);
  });
  for (int jb0 = 0; jb0 < n; jb0 += 64 * UB) {
    StaticFor<0, UB>::run([&](auto hc_) {
      constexpr int H = decltype(hc_)::value;
      const int jb = jb0 + 64 * H;
      if (jb >= n) return;
      if constexpr (TW && !REV) {
        if (jb == twin_k) {
          constexpr int XW = (Q + 1) * CW * 64;
          T *mine = xbuf + (size_t)(threadIdx.x >> 6) * XW;
          const T *other = xbuf + (size_t)(1 - (threadIdx.x >> 6)) * XW;
#pragma unroll
          for (int q = 0; q <= Q; ++q)
#pragma unroll
            for (int c = 0; c < CW; ++c) mine[(q * CW + c) * 64 + lane] = R[q][c];
          __syncthreads();
#pragma unroll
          for (int q = 0; q <= Q; ++q)
#pragma unroll
            for (int c = 0; c < CW; ++c) R[q][c] += other[(q * CW + c) * 64 + lane];
        }
      }
      const uint32_t wnext = hw[(jb / 64 + 1) * WPB + wl];
      const T hinvN = jb + 64 + lane < n ? inv[jb + 64 + lane] : T(0);
      T incN[CW];
      load_row(jb + 64 * (Q + 2) + lane, incN);
      // lanes whose R[0] row is still open: bits s+1..63 at step s. The mask
      // is shifted once per step from an opaque start, so that the compiler
      // neither compares lane ids per step nor keeps 64 constant masks
      uint64_t up = ~1ull;
      asm volatile("; lane mask %0" : "+s"(up));
      StaticFor<0, 64>::run([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int gi = s / SG, k = s % SG;
        constexpr int slot = (H * GPB + gi) % RG;
        const V(&cur)[Q] = ring[slot];
        if constexpr (ROT) {
          // one open row per lane: lane s hands its finished row to `done`
          // and takes its next row; then every lane takes its multiplier
          const T g = P::template lane<s>(R[0][0]);
          done = P::template put<s>(g, done);
          R[0][0] = P::pick(R[1][0], R[0][0], 1ull << s);
          R[0][0] = P::fnma(P::get(cur[0], k), g, R[0][0]);
          asm volatile("" : "+v"(R[0][0]));
        } else {
          T g[CW];
#pragma unroll
          for (int c = 0; c < CW; ++c) g[c] = P::template lane<s>(R[0][c]);
          T M[Q + 1];
          M[0] = P::pick_or_zero(P::get(cur[0], k), up);
#pragma unroll
          for (int q = 1; q < Q; ++q) M[q] = P::pick(P::get(cur[q], k), P::get(cur[q - 1], k), up);
          M[Q] = P::zero_or_pick(P::get(cur[Q - 1], k), up);
          up <<= 1;
#pragma unroll
          for (int q = 0; q <= Q; ++q)
#pragma unroll
            for (int c = 0; c < CW; ++c) {
              R[q][c] = P::fnma(M[q], g[c], R[q][c]);
              // keep every update in its step: otherwise updates of registers
              // not read during the block sink to its end with their operands live
              asm volatile("" : "+v"(R[q][c]));
            }
        }
        if constexpr (k == SG - 1) {
          // the group is consumed: fetch the group RG positions ahead into its slot
          constexpr int li = gi + RG;
          fetch(width_of(std::integral_constant<int, li>{}), (li * SG) & 63, slot);
        }
      });
      if (jb + lane < n) {
        Row<T, CW> rw;
#pragma unroll
        for (int c = 0; c < CW; ++c) rw.v[c] = (ROT ? done : R[0][c]) * hinv;
        rw.store(sl + (size_t)(REV ? n - 1 - (jb + lane) : jb + lane) * KC + c0);
      }
      if constexpr (!ROT) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int c = 0; c < CW; ++c) R[q][c] = R[q + 1][c];
      }
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        R[Q][c] = inc[c];
        inc[c] = incN[c];
      }
      hinv = hinvN;
      wcur = wnext;
    });
  }
}

// columns per pass: keeps the window (Q+1 registers per column) within the
// register file next to the stream ring
template <typename T, int Q, int KC>
constexpr int pass_columns() {
  constexpr int words = (int)sizeof(T) / 4;
  constexpr int cap = (Q + 1) * words * 16 <= 96 ? 16
                      : (Q + 1) * words * 8 <= 96 ? 8
                      : (Q + 1) * words * 4 <= 96 ? 4
                      : (Q + 1) * words * 2 <= 96 ? 2 : 1;
  return KC < cap ? KC : cap;
}

template <typename T, int KC, int Q, bool TW = false>
__device__ __forceinline__ void star_solve(const StarArgs &a, int st, int n, T *sl, int twin_k = -1,
                                           T *xbuf = nullptr) {
  constexpr int GPB = 64 / Pack<T>::SG;
  constexpr int CW = pass_columns<T, Q, KC>();
  // ring of 16-byte group loads: 16 slots (64 registers; 32 at eight columns
  // in narrow windows), fewer when many columns share a step (a step then takes
  // longer, so fewer steps of lookahead hide the same latency). Measured: a
  // 32-slot ring at one column held the narrow kernel to three wavefronts per
  // SIMD and was slower; at eight columns the deeper ring wins.
  constexpr int SLOTS = (Q <= 2 && CW == 8 ? 32 : 16) / (CW >= 8 ? CW / 4 : 1);
  constexpr int RG0 = SLOTS / Q > 2 * GPB ? 2 * GPB : SLOTS / Q;
  constexpr int RG = RG0 >= 32 ? 32 : RG0 >= 16 ? 16 : RG0 >= 8 ? 8 : RG0 >= 4 ? 4 : RG0 >= 2 ? 2 : 1;
  const int vb = a.st_vb[st], gbase = a.st_gb[st];
  const T *finv = static_cast<const T *>(a.f_inv) + vb, *binv = static_cast<const T *>(a.b_inv) + vb;
  const T *fval = static_cast<const T *>(a.f_val), *bval = static_cast<const T *>(a.b_val);
  const uint32_t fb = (uint32_t)a.st_fb[st], bb = (uint32_t)a.st_bb[st];
  for (int c0 = 0; c0 < KC; c0 += CW) {
    sweep<T, KC, CW, Q, RG, false, TW>(sl, c0, n, a.f_hdr + gbase, finv, fval, fb, (uint32_t)a.f_zero, twin_k,
                                        xbuf);
    __syncthreads();
    sweep<T, KC, CW, Q, RG, true>(sl, c0, n, a.b_hdr + gbase, binv, bval, bb, (uint32_t)a.b_zero);
    __syncthreads();
  }
}

// WIDE = false: stars with windows of 1-2 registers, true: 4-16 registers (kept
// in separate kernels so that each gets the registers its variants need).
// LV: the star's working vector lives in LDS during the sweeps (gathered into
// it, swept in place, copied to the slots at the end) instead of in its slot
// segment.
// resident wavefronts per SIMD the register allocation must allow: four (at
// most 128 registers) for the narrow kernels that fit without spilling; the
// one-column FP64 kernel with the vector in LDS would otherwise take 129 and
// run three wavefronts per SIMD
template <typename T, bool WIDE, int KC, bool LV>
constexpr int star_min_waves() {
  return !WIDE && (sizeof(T) == 4 ? KC <= 2 : (KC == 1 && LV)) ? 4 : 1;
}

// one star on one wavefront: gather r[S_j] into its working vector, both
// sweeps, z_j to the star's slots
template <typename T, bool WIDE, int KC, bool LV>
__device__ __forceinline__ void band_star(const StarArgs &a, int st, const double *__restrict__ r,
                                          unsigned char *star_lds) {
  const int n = a.st_n[st], vb = a.st_vb[st], Q = a.st_q[st];
  const int lane = threadIdx.x;
  T *sl = static_cast<T *>(a.slots) + (size_t)vb * KC;
  T *vec = LV ? reinterpret_cast<T *>(star_lds) : sl;
  // gather r (KC adjacent values per dof) in factor order, U rows per lane in
  // flight; clamped unconditional loads keep them all in flight
  constexpr int U = KC <= 2 ? 16 : 32 / KC;
  const int32_t *dofs = a.pos_dof + vb;
  for (int p0 = 0; p0 < n; p0 += 64 * U) {
    int idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) idx[u] = dofs[min(p0 + 64 * u + lane, n - 1)];
    Row<double, KC> val[U];
#pragma unroll
    for (int u = 0; u < U; ++u) val[u].load(r + (size_t)idx[u] * KC);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + 64 * u + lane;
      if (p < n) {
        Row<T, KC> o;
#pragma unroll
        for (int c = 0; c < KC; ++c) o.v[c] = (T)val[u].v[c];
        o.store(vec + (size_t)p * KC);
      }
    }
  }
  __syncthreads();
  if constexpr (!WIDE) {
    if (Q == 1) star_solve<T, KC, 1>(a, st, n, vec);
    else star_solve<T, KC, 2>(a, st, n, vec);
  } else {
    if (Q == 4) star_solve<T, KC, 4>(a, st, n, vec);
    else if (Q == 8) star_solve<T, KC, 8>(a, st, n, vec);
    else star_solve<T, KC, 16>(a, st, n, vec);
  }
  if constexpr (LV) {
    // z_j to the star's slots
    for (int p = lane; p < n; p += 64) {
      Row<T, KC> o;
      o.load(vec + (size_t)p * KC);
      o.store(sl + (size_t)p * KC);
    }
  }
}

template <int KC>
__device__ __forceinline__ bool star_columns_idle(const CgScalars *sc, int sel) {
  if (sel == SEL_ALL) return false;
  bool any = false;
#pragma unroll
  for (int c = 0; c < KC; ++c) any |= column_selected(sc[c], sel, 0u, c);
  return !any;
}

// one workgroup (one wavefront) per star of a.order; the hardware dispatcher
// hands the next star to a SIMD as soon as one finishes
template <typename T, bool WIDE, int KC, bool LV>
__global__ __launch_bounds__(64, (star_min_waves<T, WIDE, KC, LV>())) void k_star(StarArgs a, const double *__restrict__ r,
                                                                              const CgScalars *sc, int sel) {
  extern __shared__ __align__(16) unsigned char star_lds[];
  if (star_columns_idle<KC>(sc, sel)) return;
  const int wv = blockIdx.x;
  if (wv >= a.nstars) return;
  // the wavefronts of the longest stars may win instruction issue over the
  // shorter stars sharing their SIMD (the engine measures whether it pays)
  if (wv < a.n_prio) __builtin_amdgcn_s_setprio(3);
  band_star<T, WIDE, KC, LV>(a, a.order[wv], r, star_lds);
}

// Persistent form of the narrow-window sweeps: gridDim.x resident wavefronts
// sweep the stars of a.order (sorted by length, longest first). Wavefront w
// takes star w first, then stars from one of Nq = min(8, gridDim.x) queues in
// global memory: queue g = w mod Nq hands out the entries g + Nq k of a.order,
// k counting on from the number of wavefronts of its group (every group has at
// least one), so that the draws of the wavefronts spread over Nq counters
// (a.queue[kQueueStride g], each in a line of its own) instead of serialising
// on one. a.queue[kQueueStride kQueues] counts the wavefronts that have left;
// every wavefront leaves once its queue is exhausted (no wait on another
// wavefront), and the last one to leave sets all counters back to zero for
// the next launch on the stream. Every star is swept exactly as in k_star, so
// both give the same bits.
template <typename T, int KC, bool LV>
__global__ __launch_bounds__(64, (star_min_waves<T, false, KC, LV>())) void k_star_queue(
    StarArgs a, const double *__restrict__ r, const CgScalars *sc, int sel) {
  extern __shared__ __align__(16) unsigned char star_lds[];
  if (star_columns_idle<KC>(sc, sel)) return;
  int32_t *q = a.queue;
  const int nqs = min(kQueues, (int)gridDim.x);
  const int lane = (int)threadIdx.x, w = (int)blockIdx.x, g = w % nqs;
  const int group = ((int)gridDim.x - g + nqs - 1) / nqs;  // wavefronts of queue g (at least one)
  int wv = w;
  while (wv < a.nstars) {
    if (wv < a.n_prio) __builtin_amdgcn_s_setprio(3);
    else __builtin_amdgcn_s_setprio(0);
    band_star<T, false, KC, LV>(a, a.order[wv], r, star_lds);
    __syncthreads();  // the next star's gather reuses the LDS vector
    int k = 0;
    if (lane == 0) k = atomicAdd(q + kQueueStride * g, 1);
    k = __builtin_amdgcn_readfirstlane(k);
    wv = g + nqs * (group + k);
  }
  if (lane == 0) {
    __threadfence();
    if (atomicAdd(q + kQueueStride * kQueues, 1) == (int)gridDim.x - 1) {
      for (int i = 0; i <= kQueues; ++i) atomicExch(q + kQueueStride * i, 0);
    }
  }
}

template <typename T, int KC>
void launch_star_t(const StarArgs &a, bool wide, const double *r, const CgScalars *sc, int sel, hipStream_t s) {
  if (a.nstars <= 0) return;
  // the working vector goes to LDS when asked for and the largest star's fits in
  // 32 KB (up to eight columns); the LDS reservation, if larger, limits how many
  // stars share a CU
  const size_t need = ((size_t)a.maxn * KC * sizeof(T) + 15) / 16 * 16;
  // the persistent form (narrow windows only): a.n_resident wavefronts, at
  // most one per star
  const bool queue = !wide && a.n_resident > 0 && a.queue != nullptr;
  const unsigned nq = (unsigned)std::min(a.n_resident, a.nstars);
  if constexpr (KC <= 8) {
    if (a.use_lds && need <= 32768) {
      const size_t lds = std::max<size_t>((size_t)a.lds_reserve, need);
      if (queue) hipLaunchKernelGGL((k_star_queue<T, KC, true>), dim3(nq), dim3(64), lds, s, a, r, sc, sel);
      else if (wide) hipLaunchKernelGGL((k_star<T, true, KC, true>), dim3(a.nstars), dim3(64), lds, s, a, r, sc, sel);
      else hipLaunchKernelGGL((k_star<T, false, KC, true>), dim3(a.nstars), dim3(64), lds, s, a, r, sc, sel);
      return;
    }
  }
  const size_t lds = (size_t)a.lds_reserve;
  if (queue) hipLaunchKernelGGL((k_star_queue<T, KC, false>), dim3(nq), dim3(64), lds, s, a, r, sc, sel);
  else if (wide) hipLaunchKernelGGL((k_star<T, true, KC, false>), dim3(a.nstars), dim3(64), lds, s, a, r, sc, sel);
  else hipLaunchKernelGGL((k_star<T, false, KC, false>), dim3(a.nstars), dim3(64), lds, s, a, r, sc, sel);
}

// Two-chain stars (see BandTwin in the host code): one workgroup of two
// wavefronts per star, wavefront w sweeping chain w (unit a.unit0 + 2 t + w of
// the per-star arrays) on its own vector in a.tw_scratch; the forward sweeps
// meet at step K (tw_K); at the end each chain writes the rows it owns to the
// star's slots in band order (pos_map, -1 for pads and the separator copy).
template <typename T, int KC>
__global__ __launch_bounds__(128, (star_min_waves<T, false, KC, false>())) void k_star_twin(
    StarArgs a, const double *__restrict__ r, const CgScalars *sc, int sel) {
  extern __shared__ __align__(16) unsigned char star_lds[];
  if (sel != SEL_ALL) {
    bool any = false;
#pragma unroll
    for (int c = 0; c < KC; ++c) any |= column_selected(sc[c], sel, 0u, c);
    if (!any) return;
  }
  if ((int)blockIdx.x >= a.nstars) return;
  const int t = a.order[blockIdx.x];
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int unit = a.unit0 + 2 * t + w;
  const int n = a.st_n[unit], vb = a.st_vb[unit], Q = a.st_q[unit];
  T *vec = static_cast<T *>(a.tw_scratch) + ((size_t)a.tw_vs[t] + (size_t)w * n) * KC;
  T *xbuf = reinterpret_cast<T *>(star_lds);
  // gather r in chain order; pads and the second chain's separator rows start at 0
  constexpr int U = KC <= 2 ? 16 : 32 / KC;
  const int32_t *dofs = a.pos_dof + vb;
  for (int p0 = 0; p0 < n; p0 += 64 * U) {
    int idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) idx[u] = dofs[min(p0 + 64 * u + lane, n - 1)];
    Row<double, KC> val[U];
#pragma unroll
    for (int u = 0; u < U; ++u) val[u].load(r + (size_t)max(idx[u], 0) * KC);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + 64 * u + lane;
      if (p < n) {
        Row<T, KC> o;
#pragma unroll
        for (int c = 0; c < KC; ++c) o.v[c] = idx[u] >= 0 ? (T)val[u].v[c] : T(0);
        o.store(vec + (size_t)p * KC);
      }
    }
  }
  __syncthreads();
  if (Q == 1) star_solve<T, KC, 1, true>(a, unit, n, vec, a.tw_K[t], xbuf);
  else star_solve<T, KC, 2, true>(a, unit, n, vec, a.tw_K[t], xbuf);
  T *sl = static_cast<T *>(a.slots) + (size_t)a.st_vb[a.tw_star[t]] * KC;
  for (int p = lane; p < n; p += 64) {
    const int m = a.pos_map[vb + p];
    if (m >= 0) {
      Row<T, KC> o;
      o.load(vec + (size_t)p * KC);
      o.store(sl + (size_t)m * KC);
    }
  }
}

template <typename T, int KC>
void launch_twin_t(const StarArgs &a, const double *r, const CgScalars *sc, int sel, hipStream_t s) {
  if (a.nstars <= 0) return;
  constexpr int c1 = pass_columns<T, 1, KC>(), c2 = pass_columns<T, 2, KC>();
  constexpr size_t lds = 2 * 3 * (size_t)(c1 > c2 ? c1 : c2) * 64 * sizeof(T);
  hipLaunchKernelGGL((k_star_twin<T, KC>), dim3(a.nstars), dim3(128), lds, s, a, r, sc, sel);
}

}  // namespace spnet
