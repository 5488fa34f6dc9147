// Network diagnostics of Assumption 3.4 (homogeneity, connectivity) and the
// Poincare constant of Lemma 3.5, as evaluated in Sec. 6.1 (Table 6.1) and
// Sec. 6.2.1 (Table 6.3). Host code: they describe a network, they are not
// part of an iteration.
//
// Boxes: [0,1]^d split into nb^d boxes of side h = 1/nb, lexicographic with
// axis 0 fastest.
//  * homogeneity: the lumped mass (M 1)(x) = 1/2 sum_{y~x} |x - y| (eq. 2.1)
//    summed over the nodes of each half-open box (Sec. 2.3), divided by h^d;
//    sigma = max / min;
//  * connectivity: per box, every edge with an endpoint in the closed box;
//    while that subgraph falls apart, a breadth-first search from the
//    component of its smallest node, through nodes within r0 of the box, adds
//    the edges of the first path that reaches another component. lambda_2 of
//    L u = lambda M u on the subgraph (L: the 1/|e| weighted Laplacian of eq.
//    2.2, M: the lumped mass of the subgraph's own edges, the Neumann case of
//    the proof of Lemma 3.5) gives mu_box = 1 / (h sqrt(lambda_2)); mu is the
//    largest. A box that cannot be joined within r0 has mu_box = inf, an
//    empty one 0.
// lambda_2 comes from shift-invert Lanczos on (L + s M)^{-1} M (the constant
// vector projected out in the M inner product), with the supernodal Cholesky
// factor of the local solves. Boxes run on all host threads.
#include <algorithm>
#include <cmath>
#include <deque>
#include <limits>
#include <thread>
#include <atomic>
#include <unordered_map>
#include <unordered_set>

#include "internal.hpp"

namespace spnet {
namespace {

inline uint32_t lower_col_off(uint32_t c, uint32_t ld) { return c * ld - (c * (c - 1u)) / 2u; }

// b := A^{-1} b for the factor F of A (canonical local order in and out)
void sn_factor_solve(const SnFactor &F, std::vector<double> &b) {
  const int n = F.n;
  std::vector<double> x((size_t)n), y((size_t)n), u((size_t)F.nu);
  for (int p = 0; p < n; ++p) x[(size_t)p] = b[(size_t)F.perm[p]];
  // forward: L y = x, level by level
  for (int l = 0; l < F.nlev; ++l) {
    const int p0 = F.lev_pos[l], p1 = F.lev_pos[l + 1];
    for (int p = p0; p < p1; ++p)
      for (int q = F.aptr[p]; q < F.aptr[p + 1]; ++q) x[(size_t)p] -= u[(size_t)F.alist[q]];
    for (int p = p0; p < p1; ++p) {
      const int k = F.snpos[p], c0 = F.c0[k], w = F.w[k], h = F.h[k], r = p - c0;
      const uint32_t ld = (uint32_t)(w + h);
      const double *S = F.S.data() + F.sbase[k];
      double acc = 0.0;
      for (int c = 0; c <= r; ++c) acc += S[lower_col_off((uint32_t)c, ld) + (uint32_t)(r - c)] * x[(size_t)(c0 + c)];
      y[(size_t)p] = acc;
      for (int i = r; i < h; i += w) {
        double a = 0.0;
        for (int c = 0; c < w; ++c)
          a += S[lower_col_off((uint32_t)c, ld) + (uint32_t)(w + i - c)] * x[(size_t)(c0 + c)];
        u[(size_t)(F.ubase[k] + i)] = a;
      }
    }
  }
  // backward: L^T z = y, from the top level down (z kept in x)
  for (int l = F.nlev - 1; l >= 0; --l) {
    const int p0 = F.lev_pos[l], p1 = F.lev_pos[l + 1];
    for (int p = p0; p < p1; ++p) {
      const int k = F.snpos[p], c0 = F.c0[k], w = F.w[k], h = F.h[k], j = p - c0;
      const uint32_t ld = (uint32_t)(w + h);
      const double *S = F.S.data() + F.sbase[k] + lower_col_off((uint32_t)j, ld);
      double acc = 0.0;
      for (int r = j; r < w; ++r) acc += S[r - j] * y[(size_t)(c0 + r)];
      for (int i = 0; i < h; ++i) acc -= S[w + i - j] * x[(size_t)F.R[(size_t)(F.ubase[k] + i)]];
      x[(size_t)p] = acc;
    }
  }
  for (int p = 0; p < n; ++p) b[(size_t)F.perm[p]] = x[(size_t)p];
}

// largest eigenvalue of the symmetric tridiagonal (a, b) by bisection
double tridiag_max(const std::vector<double> &a, const std::vector<double> &b) {
  const int k = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[(size_t)i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[(size_t)i]) : 0.0);
    lo = std::min(lo, a[(size_t)i] - r);
    hi = std::max(hi, a[(size_t)i] + r);
  }
  // count of eigenvalues below t (Sturm sequence)
  auto below = [&](double t) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
      const double bb = i > 0 ? b[(size_t)i - 1] * b[(size_t)i - 1] : 0.0;
      d = a[(size_t)i] - t - (i > 0 ? bb / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) >= k) hi = mid;
    else lo = mid;
  }
  return hi;
}

// lambda_2 of L u = lambda M u on a connected graph of m nodes (CSR of L with
// the diagonal, masses M). Lanczos in the M inner product on (L + s M)^{-1} M
// with the constant vector projected out: its largest Ritz value theta gives
// lambda_2 = 1 / theta - s. The shift s is a small fraction of the smallest
// L_ii / M_ii, so that the top of that spectrum is well separated.
double lambda2_of(int32_t m, const std::vector<int32_t> &ptr, const std::vector<int32_t> &col,
                  const std::vector<double> &lval, const std::vector<double> &mass) {
  if (m < 2) return 0.0;
  double dmin = std::numeric_limits<double>::infinity();
  for (int32_t i = 0; i < m; ++i)
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q)
      if (col[q] == i) dmin = std::min(dmin, lval[q] / mass[(size_t)i]);
  const double s = 1e-3 * dmin;
  std::vector<double> aval(lval);
  for (int32_t i = 0; i < m; ++i)
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q)
      if (col[q] == i) aval[q] += s * mass[(size_t)i];
  const SnFactor F = factor_csr_local(m, ptr.data(), col.data(), aval.data());
  double mtot = 0.0;
  for (double v : mass) mtot += v;
  auto mdot = [&](const std::vector<double> &a, const std::vector<double> &b) {
    double acc = 0.0;
    for (int32_t i = 0; i < m; ++i) acc += mass[(size_t)i] * a[(size_t)i] * b[(size_t)i];
    return acc;
  };
  auto deflate = [&](std::vector<double> &v) {
    double c = 0.0;
    for (int32_t i = 0; i < m; ++i) c += mass[(size_t)i] * v[(size_t)i];
    c /= mtot;
    for (auto &x : v) x -= c;
  };
  const int K = std::min<int>(m - 1, 160);
  std::vector<std::vector<double>> V;
  std::vector<double> v((size_t)m);
  for (int32_t i = 0; i < m; ++i) v[(size_t)i] = std::sin(1.0 + 0.7 * (double)i) + 0.3 * std::cos(0.37 * (double)i);
  deflate(v);
  const double nv = std::sqrt(mdot(v, v));
  for (auto &x : v) x /= nv;
  V.push_back(v);
  std::vector<double> alpha, beta;
  double theta = 0.0, last = -1.0;
  for (int k = 0; k < K; ++k) {
    std::vector<double> w((size_t)m);
    for (int32_t i = 0; i < m; ++i) w[(size_t)i] = mass[(size_t)i] * V[(size_t)k][(size_t)i];
    sn_factor_solve(F, w);
    deflate(w);
    const double ak = mdot(w, V[(size_t)k]);
    alpha.push_back(ak);
    // full reorthogonalisation (two passes) against the Lanczos basis
    for (int pass = 0; pass < 2; ++pass)
      for (const auto &q : V) {
        const double c = mdot(w, q);
        for (int32_t i = 0; i < m; ++i) w[(size_t)i] -= c * q[(size_t)i];
      }
    deflate(w);
    const double bk = std::sqrt(std::max(mdot(w, w), 0.0));
    const bool done = k + 1 == K || !(bk > 1e-13 * std::fabs(ak));
    if (done || (k + 1) % 8 == 0) {
      theta = tridiag_max(alpha, beta);
      if (done || std::fabs(theta - last) <= 1e-14 * theta) break;
      last = theta;
    }
    beta.push_back(bk);
    for (auto &x : w) x /= bk;
    V.push_back(std::move(w));
  }
  return 1.0 / theta - s;
}

}  // namespace

void network_diagnostics(const Network &net, int nb, double r0, double *sigma, double *mu, double *density,
                         double *mu_box) {
  if (nb < 1 || nb > 1024) fail(SN_EINVAL, "nb must be in 1..1024");
  const int d = net.dim;
  const int64_t N = net.n_nodes(), E = net.n_edges();
  int64_t nbox = 1;
  for (int k = 0; k < d; ++k) nbox *= nb;
  if (nbox > (int64_t)1 << 24) fail(SN_EINVAL, "too many boxes");
  auto len_of = [&](int64_t e) {
    const int32_t u = net.edges[2 * e], v = net.edges[2 * e + 1];
    double s2 = 0.0;
    for (int k = 0; k < d; ++k) {
      const double t = net.x[(size_t)u * d + k] - net.x[(size_t)v * d + k];
      s2 = s2 + t * t;
    }
    return std::sqrt(s2);
  };
  if (!(r0 > 0.0)) {
    r0 = 0.0;
    for (int64_t e = 0; e < E; ++e) r0 = std::max(r0, len_of(e));
  }
  const double h = 1.0 / nb;
  // node masses: first-end contributions in edge order, then second-end ones
  std::vector<double> mass((size_t)N, 0.0);
  for (int64_t e = 0; e < E; ++e) mass[(size_t)net.edges[2 * e]] += 0.5 * len_of(e);
  for (int64_t e = 0; e < E; ++e) mass[(size_t)net.edges[2 * e + 1]] += 0.5 * len_of(e);
  auto box_of = [&](int64_t i) {
    int64_t b = 0;
    for (int k = d - 1; k >= 0; --k) {
      int64_t c = (int64_t)std::floor(net.x[(size_t)i * d + k] * (double)nb);
      c = std::max<int64_t>(0, std::min<int64_t>(c, nb - 1));
      b = b * nb + c;
    }
    return b;
  };
  std::vector<double> dens((size_t)nbox, 0.0);
  std::vector<int64_t> bid((size_t)N);
  for (int64_t i = 0; i < N; ++i) {
    bid[(size_t)i] = box_of(i);
    dens[(size_t)bid[(size_t)i]] += mass[(size_t)i];
  }
  double area = 1.0;
  for (int k = 0; k < d; ++k) area *= (double)nb;
  double dmin = std::numeric_limits<double>::infinity(), dmax = 0.0;
  for (auto &v : dens) {
    v *= area;
    dmin = std::min(dmin, v);
    dmax = std::max(dmax, v);
  }
  *sigma = dmin > 0.0 ? dmax / dmin : std::numeric_limits<double>::infinity();
  if (density) std::copy(dens.begin(), dens.end(), density);

  // adjacency in edge order (both directions), nodes sorted by box
  std::vector<int64_t> astart((size_t)N + 1, 0);
  for (int64_t e = 0; e < E; ++e) {
    ++astart[(size_t)net.edges[2 * e] + 1];
    ++astart[(size_t)net.edges[2 * e + 1] + 1];
  }
  for (int64_t i = 0; i < N; ++i) astart[(size_t)i + 1] += astart[(size_t)i];
  std::vector<std::pair<int32_t, int64_t>> adj((size_t)astart[(size_t)N]);
  {
    std::vector<int64_t> pos(astart.begin(), astart.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
      const int32_t u = net.edges[2 * e], v = net.edges[2 * e + 1];
      adj[(size_t)pos[(size_t)u]++] = {v, e};
      adj[(size_t)pos[(size_t)v]++] = {u, e};
    }
  }
  std::vector<int64_t> order((size_t)N);
  for (int64_t i = 0; i < N; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return bid[(size_t)a] < bid[(size_t)b]; });
  std::vector<int64_t> bstart((size_t)nbox + 1, 0);
  for (int64_t i = 0; i < N; ++i) ++bstart[(size_t)bid[(size_t)i] + 1];
  for (int64_t b = 0; b < nbox; ++b) bstart[(size_t)b + 1] += bstart[(size_t)b];
  const int64_t span = (int64_t)std::ceil(r0 / h) + 1;

  std::vector<double> mus((size_t)nbox, 0.0);
  auto one_box = [&](int64_t b) {
    int64_t v[3] = {0, 0, 0}, rem = b;
    for (int k = 0; k < d; ++k) {
      v[k] = rem % nb;
      rem /= nb;
    }
    double lo[3], hi[3];
    for (int k = 0; k < d; ++k) {
      lo[k] = (double)v[k] / (double)nb;
      hi[k] = lo[k] + 1.0 / (double)nb;
    }
    // candidates: the nodes of the boxes within span of b
    std::vector<int64_t> cand;
    int64_t a0[3] = {0, 0, 0}, a1[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) {
      a0[k] = std::max<int64_t>(0, v[k] - span);
      a1[k] = std::min<int64_t>(nb - 1, v[k] + span);
    }
    for (int64_t z = a0[2]; z <= (d == 3 ? a1[2] : 0); ++z)
      for (int64_t y = a0[1]; y <= a1[1]; ++y)
        for (int64_t x = a0[0]; x <= a1[0]; ++x) {
          const int64_t q = (z * nb + y) * nb + x;
          for (int64_t t = bstart[(size_t)q]; t < bstart[(size_t)q + 1]; ++t) cand.push_back(order[(size_t)t]);
        }
    std::unordered_set<int64_t> near;
    std::vector<int64_t> inside;
    for (int64_t i : cand) {
      bool in = true, nr = true;
      for (int k = 0; k < d; ++k) {
        const double c = net.x[(size_t)i * d + k];
        in = in && c >= lo[k] && c <= hi[k];
        nr = nr && c >= lo[k] - r0 && c <= hi[k] + r0;
      }
      if (in) inside.push_back(i);
      if (nr) near.insert(i);
    }
    std::vector<int64_t> sel;
    for (int64_t i : inside)
      for (int64_t q = astart[(size_t)i]; q < astart[(size_t)i + 1]; ++q) sel.push_back(adj[(size_t)q].second);
    std::sort(sel.begin(), sel.end());
    sel.erase(std::unique(sel.begin(), sel.end()), sel.end());
    if (sel.empty()) {
      mus[(size_t)b] = 0.0;
      return;
    }
    for (;;) {
      std::vector<int32_t> nodes;
      for (int64_t e : sel) {
        nodes.push_back(net.edges[2 * e]);
        nodes.push_back(net.edges[2 * e + 1]);
      }
      std::sort(nodes.begin(), nodes.end());
      nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
      std::unordered_map<int32_t, int32_t> loc;
      for (size_t i = 0; i < nodes.size(); ++i) loc[nodes[i]] = (int32_t)i;
      std::vector<int32_t> parent(nodes.size());
      for (size_t i = 0; i < nodes.size(); ++i) parent[i] = (int32_t)i;
      auto find = [&](int32_t i) {
        while (parent[(size_t)i] != i) {
          parent[(size_t)i] = parent[(size_t)parent[(size_t)i]];
          i = parent[(size_t)i];
        }
        return i;
      };
      for (int64_t e : sel) {
        const int32_t ri = find(loc[net.edges[2 * e]]), rj = find(loc[net.edges[2 * e + 1]]);
        if (ri != rj) parent[(size_t)std::max(ri, rj)] = std::min(ri, rj);
      }
      std::vector<int32_t> comp(nodes.size());
      bool one = true;
      for (size_t i = 0; i < nodes.size(); ++i) {
        comp[i] = find((int32_t)i);
        one = one && comp[i] == comp[0];
      }
      if (one) break;
      std::unordered_map<int32_t, std::pair<int32_t, int64_t>> prev;
      std::unordered_set<int32_t> other;
      std::deque<int32_t> dq;
      for (size_t i = 0; i < nodes.size(); ++i) {
        if (comp[i] == comp[0]) {
          prev[nodes[i]] = {-1, -1};
          dq.push_back(nodes[i]);
        } else {
          other.insert(nodes[i]);
        }
      }
      int32_t hit = -1;
      while (!dq.empty() && hit < 0) {
        const int32_t u = dq.front();
        dq.pop_front();
        for (int64_t q = astart[(size_t)u]; q < astart[(size_t)u + 1]; ++q) {
          const int32_t w = adj[(size_t)q].first;
          if (prev.count(w) || !near.count(w)) continue;
          prev[w] = {u, adj[(size_t)q].second};
          if (other.count(w)) {
            hit = w;
            break;
          }
          dq.push_back(w);
        }
      }
      if (hit < 0) {
        mus[(size_t)b] = std::numeric_limits<double>::infinity();
        return;
      }
      for (int32_t w = hit; prev[w].first >= 0; w = prev[w].first) sel.push_back(prev[w].second);
      std::sort(sel.begin(), sel.end());
      sel.erase(std::unique(sel.begin(), sel.end()), sel.end());
    }
    // L and the subgraph's lumped mass
    std::vector<int32_t> nodes;
    for (int64_t e : sel) {
      nodes.push_back(net.edges[2 * e]);
      nodes.push_back(net.edges[2 * e + 1]);
    }
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    const int32_t m = (int32_t)nodes.size();
    std::unordered_map<int32_t, int32_t> loc;
    for (int32_t i = 0; i < m; ++i) loc[nodes[(size_t)i]] = i;
    std::vector<std::vector<std::pair<int32_t, double>>> rows((size_t)m);
    std::vector<double> ms((size_t)m, 0.0);
    for (int64_t e : sel) {
      const int32_t a = loc[net.edges[2 * e]], c = loc[net.edges[2 * e + 1]];
      const double ln = len_of(e), w = 1.0 / ln;
      rows[(size_t)a].push_back({a, w});
      rows[(size_t)a].push_back({c, -w});
      rows[(size_t)c].push_back({c, w});
      rows[(size_t)c].push_back({a, -w});
      ms[(size_t)a] += 0.5 * ln;
      ms[(size_t)c] += 0.5 * ln;
    }
    std::vector<int32_t> ptr((size_t)m + 1, 0), col;
    std::vector<double> val;
    for (int32_t i = 0; i < m; ++i) {
      auto &r = rows[(size_t)i];
      std::stable_sort(r.begin(), r.end(),
                       [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
                         return x.first < y.first;
                       });
      for (size_t q = 0; q < r.size(); ++q) {
        if (q > 0 && r[q].first == r[q - 1].first) {
          val.back() += r[q].second;
        } else {
          col.push_back(r[q].first);
          val.push_back(r[q].second);
        }
      }
      ptr[(size_t)i + 1] = (int32_t)col.size();
    }
    const double lam = lambda2_of(m, ptr, col, val, ms);
    mus[(size_t)b] = lam > 0.0 ? 1.0 / (h * std::sqrt(lam)) : std::numeric_limits<double>::infinity();
  };
  // boxes on all host threads
  std::atomic<int64_t> next{0};
  std::atomic<bool> failed{false};
  auto worker = [&]() {
    for (;;) {
      const int64_t b = next.fetch_add(1);
      if (b >= nbox || failed.load()) return;
      try {
        one_box(b);
      } catch (...) {
        failed.store(true);
      }
    }
  };
  const unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(worker);
  worker();
  for (auto &t : th) t.join();
  if (failed.load()) fail(SN_EINVAL, "connectivity: a box subgraph could not be factored");
  double mmax = 0.0;
  for (double v : mus) mmax = std::max(mmax, v);
  *mu = mmax;
  if (mu_box) std::copy(mus.begin(), mus.end(), mu_box);
}

}  // namespace spnet
