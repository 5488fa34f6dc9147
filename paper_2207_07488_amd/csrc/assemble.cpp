// Assembly of K on the free dofs (Sec. 2.2; heat model eq. 3.3, truss model eq. 3.4).
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace spnet {

std::shared_ptr<System> assemble(std::shared_ptr<const Network> net, int model, const double *gamma) {
  if (model != SN_MODEL_HEAT && model != SN_MODEL_TRUSS) fail(SN_EINVAL, "unknown model");
  if (model == SN_MODEL_TRUSS && net->dim != 3) fail(SN_EINVAL, "the truss model needs dim 3");
  auto sys = std::make_shared<System>();
  sys->net = net;
  sys->model = model;
  const int nc = model == SN_MODEL_HEAT ? 1 : 3;
  sys->ncomp = nc;
  const int dim = net->dim;
  const int64_t N = net->n_nodes(), E = net->n_edges();
  sys->node_free.assign((size_t)N, -1);
  for (int64_t i = 0; i < N; ++i)
    if (!net->dir[i]) {
      sys->node_free[i] = (int32_t)sys->free_node.size();
      sys->free_node.push_back((int32_t)i);
    }
  if ((int64_t)sys->free_node.size() == N) fail(SN_ESINGULAR, "no Dirichlet node: K is singular on V");
  const int64_t nf = (int64_t)sys->free_node.size();
  sys->n = nf * nc;

  // per free node, the edges touching it in edge order
  std::vector<int64_t> start((size_t)nf + 1, 0);
  for (int64_t e = 0; e < E; ++e)
    for (int s = 0; s < 2; ++s) {
      const int32_t f = sys->node_free[net->edges[2 * e + s]];
      if (f >= 0) ++start[f + 1];
    }
  for (int64_t f = 0; f < nf; ++f) start[f + 1] += start[f];
  std::vector<int64_t> inc((size_t)start[nf]);
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t e = 0; e < E; ++e)
      for (int s = 0; s < 2; ++s) {
        const int32_t f = sys->node_free[net->edges[2 * e + s]];
        if (f >= 0) inc[fill[f]++] = e;
      }
  }
  // 3x3 (or 1x1) edge block k_e
  auto edge_block = [&](int64_t e, double *blk) {
    const int32_t u = net->edges[2 * e], v = net->edges[2 * e + 1];
    const double *xu = &net->x[(size_t)u * dim], *xv = &net->x[(size_t)v * dim];
    double l2 = 0.0;
    for (int k = 0; k < dim; ++k) {
      const double t = xv[k] - xu[k];
      l2 = l2 + t * t;
    }
    const double len = std::sqrt(l2);
    const double g = gamma ? gamma[e] : 1.0;
    if (nc == 1) {
      blk[0] = g / len;
      return;
    }
    double t[3];
    for (int a = 0; a < 3; ++a) t[a] = (xv[a] - xu[a]) / len;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) blk[3 * a + b] = g * (t[a] * t[b]) / len + (a == b ? 1e-6 / len : 0.0);
  };

  sys->rowptr.assign((size_t)sys->n + 1, 0);
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t f = 0; f < nf; ++f) {
    for (int a = 0; a < nc; ++a) {
      row.clear();
      for (int64_t q = start[f]; q < start[f + 1]; ++q) {
        const int64_t e = inc[q];
        double blk[9];
        edge_block(e, blk);
        const int32_t u = net->edges[2 * e], v = net->edges[2 * e + 1];
        const int32_t other = sys->node_free[(sys->free_node[f] == u) ? v : u];
        for (int b = 0; b < nc; ++b) {
          row.push_back({(int32_t)(f * nc + b), blk[a * nc + b]});
          if (other >= 0) row.push_back({(int32_t)(other * nc + b), -blk[a * nc + b]});
        }
      }
      // diagonal-block terms first within an edge keeps the edge order per column
      std::stable_sort(row.begin(), row.end(),
                       [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
                         return x.first < y.first;
                       });
      const int64_t r = f * nc + a;
      for (size_t q = 0; q < row.size(); ++q) {
        if (q > 0 && row[q].first == row[q - 1].first) {
          sys->val.back() += row[q].second;
        } else {
          sys->col.push_back(row[q].first);
          sys->val.push_back(row[q].second);
          ++sys->rowptr[r + 1];
        }
      }
    }
  }
  for (int64_t i = 0; i < sys->n; ++i) sys->rowptr[i + 1] += sys->rowptr[i];
  return sys;
}

}  // namespace spnet
