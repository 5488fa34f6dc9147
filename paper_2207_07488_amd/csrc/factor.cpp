// Host-side ordering and FP64 numeric factorisation of the local matrices
// K_j = K[S_j, S_j] and of the coarse matrix K_0 = P^T K P: the direct solves
// behind the projections P_j of eq. 4.1 (Sec. 4.1).
//
// Local matrices, in the two layouts the GPU local solves read.
// Band layout: reverse Cuthill-McKee from a pseudo-peripheral vertex (George &
// Liu), a monotone variable-band (envelope) profile, right-looking Cholesky in
// column storage; the forward stream lists the columns of L, the backward
// stream the rows of L from the last, each step's entries nearest the
// diagonal first.
// Supernodal layout:
//   1. minimum degree ordering (Tinney-Walker / Rose: repeatedly eliminate a
//      vertex of least degree in the elimination graph; ties by smallest index);
//   2. elimination tree (Liu), postorder, column structures of L;
//   3. fundamental supernodes, then relaxed amalgamation: a supernode joins its
//      parent when the merged dense block holds at most a quarter explicit zeros;
//   4. level of a supernode = its height in the supernodal tree (leaves 0);
//      positions are renumbered level by level, which is a topological
//      reordering of the elimination tree and so leaves the filled graph, the
//      factor and its non-zero count unchanged;
//   5. left-looking supernodal Cholesky in FP64 on the dense panels;
//   6. per supernode k with columns C (w of them) and rows R (h of them) below
//      its diagonal block, the matrix S_k = [L_CC^{-1}; L_RC L_CC^{-1}]
//      (stored lower-trapezoidal, column-major). The forward solve of a level
//      is then y_C = L_CC^{-1} t_C with t = b minus the updates of lower levels,
//      and u_k = (L_RC L_CC^{-1}) t_C the update k sends to the rows R; the
//      backward solve is z_C = L_CC^{-T} y_C - (L_RC L_CC^{-1})^T z_R. Every
//      level of both solves is a set of independent dot products.
// Coarse matrix: band Cholesky in lexicographic order and the dense inverse,
// applied on the GPU as one matrix product.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <set>
#include <thread>

#include "internal.hpp"

namespace spnet {
namespace {

// local matrix K[S,S] (both triangles and the diagonal, columns ascending)
struct LocalMatrix {
  int32_t n = 0;
  std::vector<int32_t> ptr, col;
  std::vector<double> val;
};

LocalMatrix extract_local(const System &sys, const int32_t *dofs, int32_t m, std::vector<int32_t> &where) {
  LocalMatrix A;
  A.n = m;
  A.ptr.assign((size_t)m + 1, 0);
  for (int32_t a = 0; a < m; ++a) where[dofs[a]] = a;
  for (int32_t a = 0; a < m; ++a) {
    const int32_t d = dofs[a];
    for (int64_t q = sys.rowptr[d]; q < sys.rowptr[d + 1]; ++q) {
      const int32_t b = where[sys.col[q]];
      if (b < 0) continue;
      A.col.push_back(b);
      A.val.push_back(sys.val[q]);
    }
    A.ptr[a + 1] = (int32_t)A.col.size();
  }
  for (int32_t a = 0; a < m; ++a) where[dofs[a]] = -1;
  return A;
}

struct LocalGraph {
  int32_t n = 0;
  std::vector<int32_t> ptr, adj;  // off-diagonal adjacency
  std::vector<int32_t> dptr;      // CSR of the local matrix (incl. diagonal)
  std::vector<int32_t> dcol;
  std::vector<double> dval;
};

LocalGraph extract_local_graph(const System &sys, const int32_t *dofs, int32_t m, std::vector<int32_t> &where) {
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

void band_twin(const LocalGraph &g, const std::vector<int32_t> &pos, StarFactor &F);

void factor_star(const System &sys, const int32_t *dofs, int32_t m, std::vector<int32_t> &where, StarFactor &F,
                 int64_t star_id) {
  LocalGraph g = extract_local_graph(sys, dofs, m, where);
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
  F.env = coff[m];
  double dmin = 0.0, dmax = 0.0;
  for (int32_t j = 0; j < m; ++j) {
    const double dj = A[coff[j]] * A[coff[j]];
    if (j == 0 || dj < dmin) dmin = dj;
    if (j == 0 || dj > dmax) dmax = dj;
  }
  F.pivot_ratio = m > 0 ? dmax / dmin : 1.0;
  band_twin(g, pos, F);
}


// Stars from this many positions on also get the two-chain band factor
// (shorter stars are not helped by it: their launch is bound by how many
// chains a SIMD interleaves, not by the longest chain).
constexpr int32_t kTwinMin = 512;

// The envelope of one chain: first[i] = the lowest chain position coupled to
// row i or to a later row (a monotone profile), the separator rows (from K
// on) reaching back to K at least so that both chains hold all of L_ss.
void chain_profile(const LocalGraph &g, const std::vector<int32_t> &bpos, const std::vector<int32_t> &perm,
                   const std::vector<int32_t> &cpos, int32_t K, std::vector<int32_t> &first) {
  const int32_t n = (int32_t)bpos.size();
  first.resize((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    first[i] = i;
    if (bpos[i] < 0) continue;
    const int32_t a = perm[bpos[i]];
    for (int32_t q = g.ptr[a]; q < g.ptr[a + 1]; ++q) {
      const int32_t j = cpos[g.adj[q]];
      if (j >= 0 && j < i) first[i] = std::min(first[i], j);
    }
  }
  for (int32_t i = K; i < n; ++i) first[i] = std::min(first[i], K);
  for (int32_t i = n - 2; i >= 0; --i) first[i] = std::min(first[i], first[i + 1]);
}

// The two-chain form of the band factor (see BandTwin). Among the cuts k whose
// chains keep the star's window (envelope width within the same multiple of
// 64) the one with the shortest chain K + s is taken; no split when it saves
// less than a quarter of the steps.
void band_twin(const LocalGraph &g, const std::vector<int32_t> &pos, StarFactor &F) {
  const int32_t m = F.n;
  F.twin = BandTwin{};
  if (m < kTwinMin) return;
  // reach[k]: the last position coupled to a position before k
  std::vector<int32_t> reach((size_t)m + 1, -1);
  for (int32_t p = 0; p < m; ++p) {
    int32_t mx = p;
    const int32_t a = F.perm[p];
    for (int32_t q = g.ptr[a]; q < g.ptr[a + 1]; ++q) mx = std::max(mx, pos[g.adj[q]]);
    reach[p + 1] = std::max(reach[p], mx);
  }
  const int32_t wlim = std::max(64, (F.band + 63) / 64 * 64);
  std::vector<std::pair<int32_t, int32_t>> cand;  // (chain length, k)
  for (int32_t k = 1; k < m; ++k) {
    const int32_t s = std::max(0, reach[k] + 1 - k), nb = m - k - s;
    if (nb < 1 || s > wlim) continue;
    const int32_t K = (std::max(k, nb) + 63) / 64 * 64;
    if (4 * (K + s) > 3 * m) continue;
    cand.push_back({K + s, k});
  }
  std::sort(cand.begin(), cand.end());
  for (size_t ci = 0; ci < cand.size() && ci < 24; ++ci) {
    const int32_t k = cand[ci].second;
    const int32_t s = std::max(0, reach[k] + 1 - k), nb = m - k - s;
    const int32_t K = (std::max(k, nb) + 63) / 64 * 64, n = K + s;
    BandTwin T;
    T.K = K;
    T.s = s;
    std::vector<int32_t> first[2], last[2], cpos[2];
    std::vector<int64_t> coff[2];
    std::vector<double> A[2];
    bool ok = true;
    for (int c = 0; c < 2 && ok; ++c) {
      BandChain &C = T.c[c];
      C.bpos.assign((size_t)n, -1);
      const int32_t pad = c == 0 ? K - k : K - nb;
      if (c == 0)
        for (int32_t t = 0; t < k; ++t) C.bpos[pad + t] = t;
      else
        for (int32_t t = 0; t < nb; ++t) C.bpos[pad + t] = m - 1 - t;
      for (int32_t t = 0; t < s; ++t) C.bpos[K + t] = k + t;
      cpos[c].assign((size_t)m, -1);
      for (int32_t i = 0; i < n; ++i)
        if (C.bpos[i] >= 0) cpos[c][F.perm[C.bpos[i]]] = i;
      chain_profile(g, C.bpos, F.perm, cpos[c], K, first[c]);
      last[c].resize((size_t)n);
      int32_t i = n - 1;
      for (int32_t j = n - 1; j >= 0; --j) {
        while (i > j && first[c][i] > j) --i;
        last[c][j] = std::max(i, j);
      }
      C.band = 0;
      for (int32_t j = 0; j < n; ++j) C.band = std::max(C.band, std::max(last[c][j] - j, j - first[c][j]));
      if (C.band > wlim) ok = false;
    }
    if (!ok) continue;
    // values: chain 0 holds the top-top, top-separator and separator-separator
    // entries, chain 1 the bottom-bottom and bottom-separator ones; pads get 1
    for (int c = 0; c < 2 && ok; ++c) {
      BandChain &C = T.c[c];
      coff[c].assign((size_t)n + 1, 0);
      for (int32_t j = 0; j < n; ++j) coff[c][j + 1] = coff[c][j] + (last[c][j] - j + 1);
      A[c].assign((size_t)coff[c][n], 0.0);
      for (int32_t i = 0; i < n; ++i) {
        if (C.bpos[i] < 0) {
          A[c][coff[c][i]] = 1.0;
          continue;
        }
        const int32_t a = F.perm[C.bpos[i]];
        for (int32_t q = g.dptr[a]; q < g.dptr[a + 1]; ++q) {
          const int32_t j = cpos[c][g.dcol[q]];
          if (j < 0 || j > i) continue;
          if (c == 1 && i >= K && j >= K) continue;
          A[c][coff[c][j] + (i - j)] += g.dval[q];
        }
      }
      // right-looking Cholesky of the columns before the separator; the
      // separator block receives the chain's Schur complement update
      for (int32_t j = 0; j < K; ++j) {
        double *cj = &A[c][coff[c][j]];
        if (!(cj[0] > 0.0)) {
          ok = false;
          break;
        }
        const double d = std::sqrt(cj[0]);
        cj[0] = d;
        const double inv = 1.0 / d;
        for (int32_t t = 1; t <= last[c][j] - j; ++t) cj[t] *= inv;
        for (int32_t cc = j + 1; cc <= last[c][j]; ++cc) {
          const double l = cj[cc - j];
          if (l == 0.0) continue;
          double *col = &A[c][coff[c][cc]];
          for (int32_t r = cc; r <= last[c][j]; ++r) col[r - cc] -= cj[r - j] * l;
        }
      }
    }
    if (!ok) continue;
    // the separator block: A_ss minus both updates, factored once, copied to both chains
    for (int32_t j = K; j < n && ok; ++j) {
      double *c0 = &A[0][coff[0][j]];
      const double *c1 = &A[1][coff[1][j]];
      for (int32_t r = j; r < n; ++r) c0[r - j] += c1[r - j];
      if (!(c0[0] > 0.0)) {
        ok = false;
        break;
      }
      const double d = std::sqrt(c0[0]);
      c0[0] = d;
      const double inv = 1.0 / d;
      for (int32_t r = j + 1; r < n; ++r) c0[r - j] *= inv;
      for (int32_t cc = j + 1; cc < n; ++cc) {
        const double l = c0[cc - j];
        double *col = &A[0][coff[0][cc]];
        for (int32_t r = cc; r < n; ++r) col[r - cc] -= c0[r - j] * l;
      }
    }
    if (!ok) continue;
    for (int32_t j = K; j < n; ++j)
      for (int32_t r = j; r < n; ++r) A[1][coff[1][j] + (r - j)] = A[0][coff[0][j] + (r - j)];
    // streams, as for the single band factor
    for (int c = 0; c < 2; ++c) {
      BandChain &C = T.c[c];
      C.width_fwd.resize((size_t)n);
      C.width_bwd.resize((size_t)n);
      C.invdiag.resize((size_t)n);
      C.nnz = 0;
      for (int32_t j = 0; j < n; ++j) {
        const int32_t w = last[c][j] - j;
        C.width_fwd[j] = w;
        C.invdiag[j] = 1.0 / A[c][coff[c][j]];
        if (C.bpos[j] >= 0) ++C.nnz;
        for (int32_t t = 1; t <= w; ++t) {
          const double v = A[c][coff[c][j] + t];
          C.colvals.push_back(v);
          if (v != 0.0) ++C.nnz;
        }
      }
      for (int32_t st = 0; st < n; ++st) {
        const int32_t i = n - 1 - st;
        const int32_t w = i - first[c][i];
        C.width_bwd[st] = w;
        for (int32_t t = 0; t < w; ++t) {
          const int32_t cc = i - 1 - t;
          C.rowvals.push_back(A[c][coff[c][cc] + (i - cc)]);
        }
      }
    }
    F.twin = std::move(T);
    return;
  }
}

// Structural non-zeros of the Cholesky factor of A (incl. the diagonal) in
// the given order (order[p] = local index at position p): the elimination tree
// (Liu), then row i of L holds the tree paths from the neighbours j < i up to i.
int64_t structural_nnz(const LocalMatrix &A, const std::vector<int32_t> &order) {
  const int32_t n = A.n;
  std::vector<int32_t> pos((size_t)n), parent((size_t)n, -1), anc((size_t)n, -1), mark((size_t)n, -1);
  for (int32_t p = 0; p < n; ++p) pos[order[p]] = p;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t v = order[i];
    for (int32_t q = A.ptr[v]; q < A.ptr[v + 1]; ++q) {
      int32_t r = pos[A.col[q]];
      if (r >= i) continue;
      while (anc[r] != -1 && anc[r] != i) {
        const int32_t nx = anc[r];
        anc[r] = i;
        r = nx;
      }
      if (anc[r] == -1) {
        anc[r] = i;
        parent[r] = i;
      }
    }
  }
  int64_t nnz = n;
  for (int32_t i = 0; i < n; ++i) {
    mark[i] = i;
    const int32_t v = order[i];
    for (int32_t q = A.ptr[v]; q < A.ptr[v + 1]; ++q) {
      int32_t k = pos[A.col[q]];
      if (k >= i) continue;
      while (mark[k] != i) {
        mark[k] = i;
        ++nnz;
        k = parent[k];
      }
    }
  }
  return nnz;
}

// Minimum degree on the explicit elimination graph: the eliminated vertex's
// neighbours become a clique. Returns the elimination sequence (local indices).
std::vector<int32_t> min_degree(const LocalMatrix &A) {
  const int32_t n = A.n;
  std::vector<std::vector<int32_t>> adj((size_t)n);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
      if (A.col[q] != i) adj[i].push_back(A.col[q]);
  std::set<std::pair<int32_t, int32_t>> queue;
  for (int32_t i = 0; i < n; ++i) queue.insert({(int32_t)adj[i].size(), i});
  std::vector<int32_t> stamp((size_t)n, -1), order;
  order.reserve((size_t)n);
  int32_t tick = 0;
  std::vector<int32_t> merged;
  while (!queue.empty()) {
    const int32_t v = queue.begin()->second;
    queue.erase(queue.begin());
    order.push_back(v);
    const std::vector<int32_t> nb = std::move(adj[v]);
    adj[v].clear();
    for (const int32_t a : nb) {
      queue.erase({(int32_t)adj[a].size(), a});
      ++tick;
      merged.clear();
      for (const int32_t x : adj[a])
        if (x != v) {
          merged.push_back(x);
          stamp[x] = tick;
        }
      for (const int32_t x : nb)
        if (x != a && stamp[x] != tick) {
          merged.push_back(x);
          stamp[x] = tick;
        }
      adj[a].assign(merged.begin(), merged.end());
      queue.insert({(int32_t)adj[a].size(), a});
    }
  }
  return order;
}

// sorted union of two sorted lists, without the entries in [lo, hi)
void union_minus(const std::vector<int32_t> &a, const std::vector<int32_t> &b, int32_t lo, int32_t hi,
                 std::vector<int32_t> &out) {
  out.clear();
  size_t i = 0, j = 0;
  while (i < a.size() || j < b.size()) {
    int32_t v;
    if (j == b.size() || (i < a.size() && a[i] < b[j])) v = a[i++];
    else if (i == a.size() || b[j] < a[i]) v = b[j++];
    else {
      v = a[i++];
      ++j;
    }
    if (v >= lo && v < hi) continue;
    out.push_back(v);
  }
}

struct Super {
  std::vector<int32_t> cols;  // postorder column indices, in elimination order
  std::vector<int32_t> rows;  // rows below the block (postorder indices, ascending)
  int64_t true_nnz = 0;       // structural non-zeros of L in these columns
  int32_t lo = 0, hi = 0;     // its own columns before merges: postorder indices lo..hi-1
  int32_t parent = -1;
  bool alive = true;
  int64_t entries() const {
    const int64_t w = (int64_t)cols.size(), h = (int64_t)rows.size();
    return w * (w + 1) / 2 + w * h;
  }
};

// Symbolic analysis and numeric factorisation of one local matrix.
SnFactor factor_matrix(const LocalMatrix &A, int64_t id, const char *what) {
  const int32_t n = A.n;
  SnFactor F;
  F.n = n;
  if (n == 0) {
    F.lev_pos = {0};
    F.lev_u = {0};
    return F;
  }
  // 1. ordering
  const std::vector<int32_t> md = min_degree(A);
  std::vector<int32_t> mpos((size_t)n);
  for (int32_t p = 0; p < n; ++p) mpos[md[p]] = p;
  // 2. elimination tree in MD order (Liu, path compression)
  std::vector<int32_t> parent((size_t)n, -1), anc((size_t)n, -1);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t v = md[i];
    for (int32_t q = A.ptr[v]; q < A.ptr[v + 1]; ++q) {
      int32_t r = mpos[A.col[q]];
      if (r >= i) continue;
      while (anc[r] != -1 && anc[r] != i) {
        const int32_t nx = anc[r];
        anc[r] = i;
        r = nx;
      }
      if (anc[r] == -1) {
        anc[r] = i;
        parent[r] = i;
      }
    }
  }
  // postorder (children in increasing order)
  std::vector<int32_t> head((size_t)n, -1), next((size_t)n, -1);
  for (int32_t j = n - 1; j >= 0; --j)
    if (parent[j] >= 0) {
      next[j] = head[parent[j]];
      head[parent[j]] = j;
    }
  std::vector<int32_t> post;  // post[k] = MD index of the k-th column in postorder
  post.reserve((size_t)n);
  {
    std::vector<int32_t> stack;
    for (int32_t r = 0; r < n; ++r) {
      if (parent[r] != -1) continue;
      stack.push_back(r);
      while (!stack.empty()) {
        const int32_t v = stack.back();
        if (head[v] != -1) {
          const int32_t c = head[v];
          head[v] = next[c];
          stack.push_back(c);
        } else {
          stack.pop_back();
          post.push_back(v);
        }
      }
    }
  }
  std::vector<int32_t> ppos((size_t)n);  // MD index -> postorder index
  for (int32_t k = 0; k < n; ++k) ppos[post[k]] = k;
  std::vector<int32_t> pparent((size_t)n, -1), orig((size_t)n);  // in postorder indices
  for (int32_t k = 0; k < n; ++k) {
    pparent[k] = parent[post[k]] >= 0 ? ppos[parent[post[k]]] : -1;
    orig[k] = md[post[k]];
  }
  std::vector<int32_t> opos((size_t)n);  // local index -> postorder index
  for (int32_t k = 0; k < n; ++k) opos[orig[k]] = k;
  // column structures: row i of L holds the columns on the tree paths from
  // the neighbours j < i of i up to i
  std::vector<std::vector<int32_t>> colrows((size_t)n);
  {
    std::vector<int32_t> mark((size_t)n, -1);
    for (int32_t i = 0; i < n; ++i) {
      mark[i] = i;
      const int32_t v = orig[i];
      for (int32_t q = A.ptr[v]; q < A.ptr[v + 1]; ++q) {
        int32_t k = opos[A.col[q]];
        if (k >= i) continue;
        while (mark[k] != i) {
          mark[k] = i;
          colrows[k].push_back(i);
          k = pparent[k];
        }
      }
    }
  }
  int64_t true_nnz = 0;
  for (int32_t k = 0; k < n; ++k) true_nnz += 1 + (int64_t)colrows[k].size();
  F.nnz = true_nnz;
  // 3. fundamental supernodes
  std::vector<int32_t> nchild((size_t)n, 0);
  for (int32_t k = 0; k < n; ++k)
    if (pparent[k] >= 0) ++nchild[pparent[k]];
  std::vector<Super> sn;
  std::vector<int32_t> sn_of((size_t)n);
  for (int32_t k = 0; k < n; ++k) {
    const bool join = k > 0 && pparent[k - 1] == k && nchild[k] == 1 &&
                      colrows[k - 1].size() == colrows[k].size() + 1;
    if (!join) sn.emplace_back();
    sn.back().cols.push_back(k);
    sn.back().true_nnz += 1 + (int64_t)colrows[k].size();
    sn_of[k] = (int32_t)sn.size() - 1;
  }
  for (auto &s : sn) {
    s.rows = colrows[s.cols.back()];
    s.lo = s.cols.front();
    s.hi = s.cols.back() + 1;
    const int32_t pc = pparent[s.cols.back()];
    s.parent = pc >= 0 ? sn_of[pc] : -1;
  }
  // relaxed amalgamation, children before parents (supernodes are numbered in
  // postorder): merge a child into its parent when the merged block holds at
  // most a quarter explicit zeros (or at most 8 of them). A merged child's
  // columns go before its parent's. rep[k]: the supernode k was merged into.
  std::vector<int32_t> rep(sn.size());
  for (size_t k = 0; k < sn.size(); ++k) rep[k] = (int32_t)k;
  auto find = [&](int32_t k) {
    int32_t r = k;
    while (rep[r] != r) r = rep[r];
    while (rep[k] != r) {
      const int32_t nx = rep[k];
      rep[k] = r;
      k = nx;
    }
    return r;
  };
  {
    std::vector<int32_t> tmp;
    for (int32_t k = 0; k < (int32_t)sn.size(); ++k) {
      Super &c = sn[k];
      if (c.parent < 0) continue;
      c.parent = find(c.parent);
      Super &p = sn[c.parent];
      std::vector<int32_t> cols = c.cols;
      cols.insert(cols.end(), p.cols.begin(), p.cols.end());
      // c's rows are p's own columns and ancestors of p; p's earlier merged
      // children hold none of them
      union_minus(c.rows, p.rows, p.lo, p.hi, tmp);
      const int64_t w = (int64_t)cols.size(), h = (int64_t)tmp.size();
      const int64_t entries = w * (w + 1) / 2 + w * h, tn = c.true_nnz + p.true_nnz;
      if (4 * (entries - tn) <= entries || entries - tn <= 8) {
        p.cols = std::move(cols);
        p.rows = tmp;
        p.true_nnz = tn;
        c.alive = false;
        rep[k] = c.parent;
      }
    }
  }
  // 4. levels (height in the supernodal tree) and the final position order
  std::vector<int32_t> alive;
  for (int32_t k = 0; k < (int32_t)sn.size(); ++k)
    if (sn[k].alive) {
      alive.push_back(k);
      if (sn[k].parent >= 0) sn[k].parent = find(sn[k].parent);
    }
  std::vector<int32_t> level(sn.size(), 0);
  for (const int32_t k : alive)  // postorder: children first
    if (sn[k].parent >= 0) level[sn[k].parent] = std::max(level[sn[k].parent], level[k] + 1);
  int32_t nlev = 0;
  for (const int32_t k : alive) nlev = std::max(nlev, level[k] + 1);
  std::vector<int32_t> order = alive;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return level[a] < level[b]; });
  const int32_t nsn = (int32_t)order.size();
  std::vector<int32_t> fpos((size_t)n);  // postorder index -> final position
  F.perm.resize((size_t)n);
  F.c0.resize(nsn);
  F.w.resize(nsn);
  F.h.resize(nsn);
  F.lev_pos.assign((size_t)nlev + 1, 0);
  {
    int32_t p = 0;
    for (int32_t s = 0; s < nsn; ++s) {
      const Super &S = sn[order[s]];
      F.c0[s] = p;
      F.w[s] = (int32_t)S.cols.size();
      F.h[s] = (int32_t)S.rows.size();
      for (const int32_t c : S.cols) {
        fpos[c] = p;
        F.perm[p] = orig[c];
        ++p;
      }
      F.lev_pos[level[order[s]] + 1] = p;
    }
    for (int32_t l = 1; l <= nlev; ++l) F.lev_pos[l] = std::max(F.lev_pos[l], F.lev_pos[l - 1]);
  }
  F.snpos.resize((size_t)n);
  for (int32_t s = 0; s < nsn; ++s)
    for (int32_t c = 0; c < F.w[s]; ++c) F.snpos[F.c0[s] + c] = s;
  // rows below each block in final positions (ancestors: later levels)
  std::vector<std::vector<int32_t>> R((size_t)nsn);
  for (int32_t s = 0; s < nsn; ++s) {
    for (const int32_t r : sn[order[s]].rows) R[s].push_back(fpos[r]);
    std::sort(R[s].begin(), R[s].end());
    if (!R[s].empty() && R[s].front() < F.c0[s] + F.w[s])
      fail(SN_EINVAL, std::string("internal: ") + what + " supernode rows precede its block");
  }
  // u-slots: the update of supernode s to its rows, level by level
  F.ubase.resize(nsn);
  F.lev_u.assign((size_t)nlev + 1, 0);
  {
    int64_t u = 0;
    for (int32_t s = 0; s < nsn; ++s) {
      F.ubase[s] = u;
      u += F.h[s];
      F.lev_u[level[order[s]] + 1] = (int32_t)u;
    }
    for (int32_t l = 1; l <= nlev; ++l) F.lev_u[l] = std::max(F.lev_u[l], F.lev_u[l - 1]);
    F.nu = (int32_t)u;
  }
  F.nsn = nsn;
  F.nlev = nlev;
  F.snu.resize((size_t)F.nu);
  F.R.resize((size_t)F.nu);
  for (int32_t s = 0; s < nsn; ++s)
    for (int32_t i = 0; i < F.h[s]; ++i) {
      F.snu[(size_t)(F.ubase[s] + i)] = s;
      F.R[(size_t)(F.ubase[s] + i)] = R[s][i];
    }
  // u-slots aimed at each position, ascending
  F.aptr.assign((size_t)n + 1, 0);
  for (int32_t e = 0; e < F.nu; ++e) ++F.aptr[F.R[e] + 1];
  for (int32_t p = 0; p < n; ++p) F.aptr[p + 1] += F.aptr[p];
  F.alist.resize((size_t)F.nu);
  {
    std::vector<int32_t> fill(F.aptr.begin(), F.aptr.end() - 1);
    for (int32_t e = 0; e < F.nu; ++e) F.alist[fill[F.R[e]]++] = e;
  }
  // 5. numeric factorisation in final positions
  std::vector<int32_t> fin_of_local((size_t)n);
  for (int32_t p = 0; p < n; ++p) fin_of_local[F.perm[p]] = p;
  std::vector<std::vector<double>> panel((size_t)nsn);
  std::vector<std::vector<int32_t>> updaters((size_t)nsn);
  std::vector<int32_t> rowmap((size_t)n, -1);
  double dmin = HUGE_VAL, dmax = 0.0;
  for (int32_t s = 0; s < nsn; ++s) {
    const int32_t c0 = F.c0[s], w = F.w[s], h = F.h[s], ld = w + h;
    for (int32_t r = 0; r < w; ++r) rowmap[c0 + r] = r;
    for (int32_t i = 0; i < h; ++i) rowmap[R[s][i]] = w + i;
    std::vector<double> P((size_t)ld * w, 0.0);
    for (int32_t c = 0; c < w; ++c) {
      const int32_t v = F.perm[c0 + c];
      for (int32_t q = A.ptr[v]; q < A.ptr[v + 1]; ++q) {
        const int32_t j = fin_of_local[A.col[q]];
        if (j < c0 + c) continue;
        const int32_t rr = rowmap[j];
        if (rr < 0) fail(SN_EINVAL, std::string("internal: ") + what + " entry outside its supernode");
        P[(size_t)c * ld + rr] += A.val[q];
      }
    }
    for (const int32_t d : updaters[s]) {
      const std::vector<int32_t> &Rd = R[d];
      const int32_t wd = F.w[d], hd = F.h[d], ldd = wd + hd;
      const double *Ld = panel[d].data();
      const size_t i0 = (size_t)(std::lower_bound(Rd.begin(), Rd.end(), c0) - Rd.begin());
      for (size_t jj = i0; jj < Rd.size() && Rd[jj] < c0 + w; ++jj) {
        const int32_t cj = Rd[jj] - c0;
        for (size_t ii = jj; ii < Rd.size(); ++ii) {
          const int32_t rr = rowmap[Rd[ii]];
          if (rr < 0) fail(SN_EINVAL, std::string("internal: ") + what + " update outside its target");
          double dot = 0.0;
          for (int32_t c = 0; c < wd; ++c) dot += Ld[(size_t)c * ldd + wd + ii] * Ld[(size_t)c * ldd + wd + jj];
          P[(size_t)cj * ld + rr] -= dot;
        }
      }
    }
    for (int32_t c = 0; c < w; ++c) {
      double *pc = &P[(size_t)c * ld];
      const double dg = pc[c];
      if (!(dg > 0.0))
        fail(SN_ENOTSPD, std::string(what) + " " + std::to_string(id) + " is not positive definite");
      dmin = std::min(dmin, dg);
      dmax = std::max(dmax, dg);
      const double sd = std::sqrt(dg);
      pc[c] = sd;
      for (int32_t r = c + 1; r < ld; ++r) pc[r] /= sd;
      for (int32_t c2 = c + 1; c2 < w; ++c2) {
        const double l = pc[c2];
        if (l == 0.0) continue;
        double *p2 = &P[(size_t)c2 * ld];
        for (int32_t r = c2; r < ld; ++r) p2[r] -= pc[r] * l;
      }
    }
    panel[s] = std::move(P);
    for (int32_t r = 0; r < w; ++r) rowmap[c0 + r] = -1;
    for (int32_t i = 0; i < h; ++i) rowmap[R[s][i]] = -1;
    int32_t last = -1;
    for (int32_t i = 0; i < h; ++i) {
      const int32_t t = F.snpos[R[s][i]];
      if (t != last) updaters[t].push_back(s);
      last = t;
    }
  }
  F.pivot_ratio = dmax / dmin;
  // 6. S_k = [L_CC^{-1}; L_RC L_CC^{-1}], column c holding rows c..w+h-1
  F.sbase.resize(nsn);
  int64_t total = 0;
  for (int32_t s = 0; s < nsn; ++s) {
    F.sbase[s] = total;
    const int64_t w = F.w[s], h = F.h[s];
    total += w * (w + 1) / 2 + w * h;
  }
  F.S.assign((size_t)total, 0.0);
  for (int32_t s = 0; s < nsn; ++s) {
    const int32_t w = F.w[s], h = F.h[s], ld = w + h;
    const double *P = panel[s].data();
    // X = L_CC^{-1}, lower triangular, column by column (forward substitution)
    std::vector<double> X((size_t)w * w, 0.0);  // column-major
    for (int32_t c = 0; c < w; ++c) {
      double *xc = &X[(size_t)c * w];
      xc[c] = 1.0 / P[(size_t)c * ld + c];
      for (int32_t r = c + 1; r < w; ++r) {
        double acc = 0.0;
        for (int32_t k = c; k < r; ++k) acc += P[(size_t)k * ld + r] * xc[k];
        xc[r] = -acc / P[(size_t)r * ld + r];
      }
    }
    double *out = &F.S[(size_t)F.sbase[s]];
    for (int32_t c = 0; c < w; ++c) {
      for (int32_t r = c; r < w; ++r) *out++ = X[(size_t)c * w + r];
      for (int32_t i = 0; i < h; ++i) {  // (L_RC X)(i, c) = sum_{k >= c} L_RC(i, k) X(k, c)
        double acc = 0.0;
        for (int32_t k = c; k < w; ++k) acc += P[(size_t)k * ld + w + i] * X[(size_t)c * w + k];
        *out++ = acc;
      }
    }
  }
  return F;
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

SnFactor factor_csr_local(int32_t n, const int32_t *ptr, const int32_t *col, const double *val) {
  LocalMatrix A;
  A.n = n;
  A.ptr.assign(ptr, ptr + n + 1);
  A.col.assign(col, col + ptr[n]);
  A.val.assign(val, val + ptr[n]);
  return factor_matrix(A, 0, "matrix");
}

HostFactors factor_host(const Precond &pre) {
  const auto t0 = std::chrono::steady_clock::now();
  const System &sys = *pre.sys;
  HostFactors hf;
  const int64_t ns = (int64_t)pre.star_vertex.size();
  hf.stars.resize((size_t)ns);
  // the largest stars first, so that the threads finish together
  std::vector<int64_t> by_size((size_t)ns);
  for (int64_t s = 0; s < ns; ++s) by_size[s] = s;
  std::stable_sort(by_size.begin(), by_size.end(), [&](int64_t a, int64_t b) {
    return pre.star_ptr[a + 1] - pre.star_ptr[a] > pre.star_ptr[b + 1] - pre.star_ptr[b];
  });
  parallel_for(ns, [&](int64_t i) {
    const int64_t s = by_size[i];
    thread_local std::vector<int32_t> where;
    if ((int64_t)where.size() < sys.n) where.assign((size_t)sys.n, -1);
    const int32_t m = (int32_t)(pre.star_ptr[s + 1] - pre.star_ptr[s]);
    if (m >= 65536) fail(SN_EINVAL, "star " + std::to_string(s) + " has 65536 or more dofs");
    const int32_t *dofs = &pre.star_dofs[pre.star_ptr[s]];
    StarFactor &F = hf.stars[s];
    factor_star(sys, dofs, m, where, F, s);
    LocalMatrix A = extract_local(sys, dofs, m, where);
    F.sn = factor_matrix(A, s, "local matrix of star");
    F.nnz_rcm = structural_nnz(A, F.perm);
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
