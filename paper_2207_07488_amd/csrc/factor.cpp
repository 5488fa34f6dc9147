// Host-side ordering and FP64 numeric factorisation of the local matrices
// K_j = K[S_j, S_j] and of the coarse matrix K_0 = P^T K P: the direct solves
// behind the projections P_j of eq. 4.1 (Sec. 4.1).
//
// Local matrices: reverse Cuthill-McKee from a pseudo-peripheral vertex (George
// & Liu), a monotone variable-band (envelope) profile, right-looking Cholesky
// in column storage. The two GPU sweep streams are cut from the factor:
// columns of L for the forward sweep, rows of L (last first) for the backward
// sweep, each step listing its entries nearest the diagonal first.
// Coarse matrix: band Cholesky in lexicographic order and the dense inverse,
// applied on the GPU as one matrix-vector product.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

#include "internal.hpp"

namespace spnet {
namespace {

struct LocalGraph {
  int32_t n = 0;
  std::vector<int32_t> ptr, adj;  // off-diagonal adjacency
  std::vector<int32_t> dptr;      // CSR of the local matrix (incl. diagonal)
  std::vector<int32_t> dcol;
  std::vector<double> dval;
};

LocalGraph extract_local(const System &sys, const int32_t *dofs, int32_t m, std::vector<int32_t> &where) {
  LocalGraph g;
  g.n = m;
  g.ptr.assign((size_t)m + 1, 0);
  g.dptr.assign((size_t)m + 1, 0);
  for (int32_t a = 0; a < m; ++a) where[dofs[a]] = a;
  for (int32_t a = 0; a < m; ++a) {
    const int32_t d = dofs[a];
    for (int64_t q = sys.rowptr[d]; q < sys.rowptr[d + 1]; ++q) {
      const int32_t b = where[sys.col[q]];
      if (b < 0) continue;
      g.dcol.push_back(b);
      g.dval.push_back(sys.val[q]);
      if (b != a) g.adj.push_back(b);
    }
    g.ptr[a + 1] = (int32_t)g.adj.size();
    g.dptr[a + 1] = (int32_t)g.dcol.size();
  }
  for (int32_t a = 0; a < m; ++a) where[dofs[a]] = -1;
  return g;
}

// BFS level structure rooted at r restricted to unmarked vertices; returns
// the levels' vertex list and the start of the last level.
int32_t level_structure(const LocalGraph &g, int32_t r, const std::vector<uint8_t> &done,
                        std::vector<int32_t> &order, std::vector<int32_t> &level, int32_t &last_begin) {
  order.clear();
  order.push_back(r);
  level[r] = 0;
  size_t head = 0;
  int32_t depth = 0;
  last_begin = 0;
  while (head < order.size()) {
    const int32_t v = order[head++];
    for (int32_t q = g.ptr[v]; q < g.ptr[v + 1]; ++q) {
      const int32_t w = g.adj[q];
      if (done[w] || level[w] >= 0) continue;
      level[w] = level[v] + 1;
      if (level[w] > depth) {
        depth = level[w];
        last_begin = (int32_t)order.size();
      }
      order.push_back(w);
    }
  }
  for (int32_t v : order) level[v] = -1;
  return depth;
}

std::vector<int32_t> rcm(const LocalGraph &g) {
  const int32_t n = g.n;
  std::vector<int32_t> deg((size_t)n);
  for (int32_t v = 0; v < n; ++v) deg[v] = g.ptr[v + 1] - g.ptr[v];
  std::vector<uint8_t> done((size_t)n, 0);
  std::vector<int32_t> level((size_t)n, -1), order, cm;
  cm.reserve((size_t)n);
  std::vector<std::pair<int32_t, int32_t>> nb;
  for (int32_t seed = 0; seed < n; ++seed) {
    if (done[seed]) continue;
    // pseudo-peripheral start: walk to a least-degree vertex of the deepest
    // level while the eccentricity grows
    int32_t r = seed, lb = 0;
    int32_t ecc = level_structure(g, r, done, order, level, lb);
    for (int guard = 0; guard < 32; ++guard) {
      int32_t best = -1;
      for (size_t q = (size_t)lb; q < order.size(); ++q)
        if (best < 0 || deg[order[q]] < deg[best] || (deg[order[q]] == deg[best] && order[q] < best))
          best = order[q];
      int32_t lb2 = 0;
      const int32_t e2 = level_structure(g, best, done, order, level, lb2);
      if (e2 <= ecc) break;
      r = best;
      ecc = e2;
      lb = lb2;
    }
    // Cuthill-McKee from r
    const size_t base = cm.size();
    cm.push_back(r);
    done[r] = 1;
    for (size_t head = base; head < cm.size(); ++head) {
      const int32_t v = cm[head];
      nb.clear();
      for (int32_t q = g.ptr[v]; q < g.ptr[v + 1]; ++q) {
        const int32_t w = g.adj[q];
        if (!done[w]) {
          done[w] = 1;
          nb.push_back({deg[w], w});
        }
      }
      std::sort(nb.begin(), nb.end());
      for (auto &p : nb) cm.push_back(p.second);
    }
  }
  std::reverse(cm.begin(), cm.end());
  return cm;  // position -> local index
}

void factor_star(const System &sys, const int32_t *dofs, int32_t m, std::vector<int32_t> &where, StarFactor &F,
                 int64_t star_id) {
  LocalGraph g = extract_local(sys, dofs, m, where);
  F.n = m;
  F.perm = rcm(g);
  std::vector<int32_t> pos((size_t)m);
  for (int32_t p = 0; p < m; ++p) pos[F.perm[p]] = p;
  // monotone profile: first[i] = min over i' >= i of the lowest coupled column
  std::vector<int32_t> first((size_t)m);
  for (int32_t p = 0; p < m; ++p) first[p] = p;
  for (int32_t a = 0; a < m; ++a)
    for (int32_t q = g.ptr[a]; q < g.ptr[a + 1]; ++q) {
      const int32_t i = pos[a], j = pos[g.adj[q]];
      if (j < i) first[i] = std::min(first[i], j);
    }
  for (int32_t p = m - 2; p >= 0; --p) first[p] = std::min(first[p], first[p + 1]);
  // column storage: column j holds rows j..last[j]
  std::vector<int32_t> last((size_t)m);
  {
    int32_t i = m - 1;
    for (int32_t j = m - 1; j >= 0; --j) {
      while (i > j && first[i] > j) --i;
      last[j] = std::max(i, j);
    }
  }
  std::vector<int64_t> coff((size_t)m + 1, 0);
  for (int32_t j = 0; j < m; ++j) coff[j + 1] = coff[j] + (last[j] - j + 1);
  std::vector<double> A((size_t)coff[m], 0.0);
  for (int32_t a = 0; a < m; ++a)
    for (int32_t q = g.dptr[a]; q < g.dptr[a + 1]; ++q) {
      const int32_t i = pos[a], j = pos[g.dcol[q]];
      if (i >= j) A[coff[j] + (i - j)] += g.dval[q];
    }
  // right-looking Cholesky inside the profile
  for (int32_t j = 0; j < m; ++j) {
    double *cj = &A[coff[j]];
    const int32_t w = last[j] - j;
    if (!(cj[0] > 0.0))
      fail(SN_ENOTSPD, "local matrix of star " + std::to_string(star_id) + " is not positive definite");
    const double d = std::sqrt(cj[0]);
    cj[0] = d;
    const double inv = 1.0 / d;
    for (int32_t t = 1; t <= w; ++t) cj[t] *= inv;
    for (int32_t c = j + 1; c <= last[j]; ++c) {
      const double lcj = cj[c - j];
      if (lcj == 0.0) continue;
      double *cc = &A[coff[c]];
      for (int32_t i = c; i <= last[j]; ++i) cc[i - c] -= cj[i - j] * lcj;
    }
  }
  // streams
  F.width_fwd.resize((size_t)m);
  F.width_bwd.resize((size_t)m);
  F.invdiag.resize((size_t)m);
  F.colvals.clear();
  F.rowvals.clear();
  F.colvals.reserve((size_t)(coff[m] - m));
  F.rowvals.reserve((size_t)(coff[m] - m));
  int32_t band = 0;
  for (int32_t j = 0; j < m; ++j) {
    const int32_t w = last[j] - j;
    F.width_fwd[j] = w;
    F.invdiag[j] = 1.0 / A[coff[j]];
    for (int32_t t = 1; t <= w; ++t) F.colvals.push_back(A[coff[j] + t]);
    band = std::max(band, w);
  }
  for (int32_t s = 0; s < m; ++s) {
    const int32_t i = m - 1 - s;
    const int32_t w = i - first[i];
    F.width_bwd[s] = w;
    for (int32_t t = 0; t < w; ++t) {
      const int32_t c = i - 1 - t;
      F.rowvals.push_back(A[coff[c] + (i - c)]);
    }
    band = std::max(band, w);
  }
  F.band = band;
  F.nnz = coff[m];
  double dmin = 0.0, dmax = 0.0;
  for (int32_t j = 0; j < m; ++j) {
    const double dj = A[coff[j]] * A[coff[j]];
    if (j == 0 || dj < dmin) dmin = dj;
    if (j == 0 || dj > dmax) dmax = dj;
  }
  F.pivot_ratio = m > 0 ? dmax / dmin : 1.0;
}

template <typename Fn>
void parallel_for(int64_t n, Fn fn) {
  unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nt = (int)std::min<int64_t>(std::min<unsigned>(hw, 32u), std::max<int64_t>(n, 1));
  std::atomic<int64_t> next{0};
  std::mutex emu;
  std::unique_ptr<Error> err;
  auto work = [&]() {
    for (;;) {
      const int64_t i = next.fetch_add(1);
      if (i >= n) return;
      try {
        fn(i);
      } catch (const Error &e) {
        std::lock_guard<std::mutex> g(emu);
        if (!err) err = std::make_unique<Error>(e);
        next.store(n);
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto &t : th) t.join();
  if (err) throw *err;
}

}  // namespace

HostFactors factor_host(const Precond &pre) {
  const auto t0 = std::chrono::steady_clock::now();
  const System &sys = *pre.sys;
  HostFactors hf;
  const int64_t ns = (int64_t)pre.star_vertex.size();
  hf.stars.resize((size_t)ns);
  // one scratch map per thread slot (indexed by thread via thread_local)
  parallel_for(ns, [&](int64_t s) {
    thread_local std::vector<int32_t> where;
    if ((int64_t)where.size() < sys.n) where.assign((size_t)sys.n, -1);
    const int32_t m = (int32_t)(pre.star_ptr[s + 1] - pre.star_ptr[s]);
    factor_star(sys, &pre.star_dofs[pre.star_ptr[s]], m, where, hf.stars[s], s);
  });

  // coarse matrix K_0 = P^T K P in band storage, band Cholesky, explicit inverse
  const int64_t m0 = pre.m0;
  const int nc = sys.ncomp, nv = pre.nvert_per_elem;
  if (m0 > 16384) fail(SN_EINVAL, "coarse space too large for the dense coarse operator (m0 > 16384)");
  if (m0 > 0) {
    // every coupling of K_0: coarse dofs of the elements of the two ends of a
    // matrix entry; visit(A, B, value)
    auto couplings = [&](auto visit) {
      for (int64_t i = 0; i < sys.n; ++i) {
        const int64_t fi = i / nc;
        const int ci = (int)(i % nc);
        for (int64_t q = sys.rowptr[i]; q < sys.rowptr[i + 1]; ++q) {
          const int64_t j = sys.col[q], fj = j / nc;
          const int cj = (int)(j % nc);
          for (int a = 0; a < nv; ++a) {
            const int32_t ga = pre.vert_coarse[pre.Pvert[(size_t)fi * nv + a]];
            if (ga < 0) continue;
            const double wa = pre.Pphi[(size_t)fi * nv + a] * sys.val[q];
            const int64_t A_ = (int64_t)ga * nc + ci;
            for (int b = 0; b < nv; ++b) {
              const int32_t gb = pre.vert_coarse[pre.Pvert[(size_t)fj * nv + b]];
              if (gb < 0) continue;
              visit(A_, (int64_t)gb * nc + cj, wa * pre.Pphi[(size_t)fj * nv + b]);
            }
          }
        }
      }
    };
    int64_t bw = 0;
    couplings([&](int64_t A_, int64_t B_, double) { bw = std::max(bw, A_ - B_); });
    // lower band by columns: Lb[j * W + k] = K_0(j + k, j), k = 0..bw
    const int64_t W = bw + 1;
    std::vector<double> Lb((size_t)(m0 * W), 0.0);
    couplings([&](int64_t A_, int64_t B_, double v) {
      if (A_ >= B_) Lb[(size_t)(B_ * W + (A_ - B_))] += v;
    });
    // right-looking band Cholesky
    double dmin = HUGE_VAL, dmax = 0.0;
    for (int64_t j = 0; j < m0; ++j) {
      double *cj = &Lb[(size_t)(j * W)];
      const double d = cj[0];
      if (!(d > 0.0)) fail(SN_ENOTSPD, "coarse matrix P^T K P is not positive definite");
      dmin = std::min(dmin, d);
      dmax = std::max(dmax, d);
      const double sd = std::sqrt(d);
      cj[0] = sd;
      const int64_t len = std::min(W, m0 - j);
      for (int64_t k = 1; k < len; ++k) cj[k] /= sd;
      for (int64_t t = 1; t < len; ++t) {
        const double l = cj[t];
        if (l == 0.0) continue;
        double *cc = &Lb[(size_t)((j + t) * W)];  // column j + t, rows j + t ..
        for (int64_t k = t; k < len; ++k) cc[k - t] -= cj[k] * l;
      }
    }
    hf.coarse_pivot_ratio = dmax / dmin;
    // K_0^{-1}: columns solved with the band factor, eight at a time so that
    // one pass over the factor serves eight right-hand sides
    constexpr int RB = 8;
    hf.coarse_inv.assign((size_t)(m0 * m0), 0.0);
    const int64_t nblocks = (m0 + RB - 1) / RB;
    parallel_for(nblocks, [&](int64_t blk) {
      const int64_t c0 = blk * RB, nb = std::min<int64_t>(RB, m0 - c0);
      std::vector<double> y((size_t)(m0 * RB), 0.0);  // row-major: y[i * RB + r]
      for (int64_t r = 0; r < nb; ++r) y[(size_t)((c0 + r) * RB + r)] = 1.0;
      // forward: L y = e (column-oriented; rows above c0 stay zero)
      for (int64_t j = c0; j < m0; ++j) {
        const double *cj = &Lb[(size_t)(j * W)];
        double *yj = &y[(size_t)(j * RB)];
        for (int r = 0; r < RB; ++r) yj[r] /= cj[0];
        const int64_t len = std::min(W, m0 - j);
        for (int64_t k = 1; k < len; ++k) {
          double *yi = &y[(size_t)((j + k) * RB)];
          const double l = cj[k];
          for (int r = 0; r < RB; ++r) yi[r] -= l * yj[r];
        }
      }
      // backward: L^T x = y
      for (int64_t i = m0 - 1; i >= 0; --i) {
        const double *ci = &Lb[(size_t)(i * W)];
        double *yi = &y[(size_t)(i * RB)];
        const int64_t len = std::min(W, m0 - i);
        for (int64_t k = 1; k < len; ++k) {
          const double *yk = &y[(size_t)((i + k) * RB)];
          const double l = ci[k];
          for (int r = 0; r < RB; ++r) yi[r] -= l * yk[r];
        }
        for (int r = 0; r < RB; ++r) yi[r] /= ci[0];
      }
      for (int64_t r = 0; r < nb; ++r)
        for (int64_t i = 0; i < m0; ++i) hf.coarse_inv[(size_t)((c0 + r) * m0 + i)] = y[(size_t)(i * RB + r)];
    });
  }
  hf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return hf;
}

}  // namespace spnet
