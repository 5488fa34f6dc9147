// Assembly of K on the free dofs (Sec. 2.2): heat model (eq. 3.3), truss model
// (eq. 3.4 plus an isotropic 1e-6/|e| term) and beam model (eq. 3.4 plus the
// bending form of eq. 3.5, constants of Sec. 6.3). Each free row also keeps
// its entries against the dofs of Dirichlet nodes, which a non-zero Dirichlet
// lifting moves to the right-hand side, and each free node its lumped mass
// (M 1)(x) of eq. 2.1.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace spnet {

namespace {

// One row's contributions: (column as node * ncomp + component, value), kept
// in the order they are generated and summed per column in that order.
using RowTerms = std::vector<std::pair<int64_t, double>>;

// Node adjacency in edge order (both directions), over all nodes.
struct Adjacency {
  std::vector<int64_t> start;
  std::vector<int32_t> nbr;
  std::vector<int64_t> edge;
};

Adjacency adjacency(const Network &net) {
  const int64_t N = net.n_nodes(), E = net.n_edges();
  Adjacency a;
  a.start.assign((size_t)N + 1, 0);
  for (int64_t e = 0; e < E; ++e) {
    ++a.start[net.edges[2 * e] + 1];
    ++a.start[net.edges[2 * e + 1] + 1];
  }
  for (int64_t i = 0; i < N; ++i) a.start[i + 1] += a.start[i];
  a.nbr.resize((size_t)a.start[N]);
  a.edge.resize((size_t)a.start[N]);
  std::vector<int64_t> pos(a.start.begin(), a.start.end() - 1);
  for (int64_t e = 0; e < E; ++e) {
    const int32_t u = net.edges[2 * e], v = net.edges[2 * e + 1];
    a.nbr[(size_t)pos[u]] = v;
    a.edge[(size_t)pos[u]++] = e;
    a.nbr[(size_t)pos[v]] = u;
    a.edge[(size_t)pos[v]++] = e;
  }
  return a;
}

double edge_length(const Network &net, int32_t u, int32_t v) {
  const int dim = net.dim;
  double l2 = 0.0;
  for (int k = 0; k < dim; ++k) {
    const double t = net.x[(size_t)u * dim + k] - net.x[(size_t)v * dim + k];
    l2 = l2 + t * t;
  }
  return std::sqrt(l2);
}

void cross(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// The bending element of eq. 3.5 for centre x and ordered neighbour pair
// (y, z): weight w and, per term k, the vector c over the dofs of (x, y, z)
// with a_k = c . v. With unit vectors d_y = (x - y)/|x - y|, d_z likewise,
// n1 a unit normal of both edges (e_3 for a 2D network), the in-plane normals
// are d_y x n1 for y and n1 x d_z for z, so that a_2 is the change of the
// angle between the two edges (zero for a rigid motion; the curvature on a
// straight fiber); a_1 (three components only) uses n1 for both.
struct Bend {
  double w;
  int nk;
  double c[2][3][3];  // [term][x, y, z][component]
};

Bend bend_element(const Network &net, int nc, double g1, double rw, int32_t x, int32_t y, int32_t z) {
  const int dim = net.dim;
  const double ly = edge_length(net, x, y), lz = edge_length(net, x, z);
  double dy[3] = {0.0, 0.0, 0.0}, dz[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < dim; ++k) {
    dy[k] = (net.x[(size_t)x * dim + k] - net.x[(size_t)y * dim + k]) / ly;
    dz[k] = (net.x[(size_t)x * dim + k] - net.x[(size_t)z * dim + k]) / lz;
  }
  double n1[3] = {0.0, 0.0, 1.0};
  if (dim == 3) {
    cross(dy, dz, n1);
    double nn = std::sqrt(n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
    if (!(nn > 1e-12)) {
      // parallel edges: any unit normal of d_y (the two terms together do not
      // depend on which); take the axis least aligned with d_y
      int am = 0;
      for (int k = 1; k < 3; ++k)
        if (std::fabs(dy[k]) < std::fabs(dy[am])) am = k;
      double ax[3] = {0.0, 0.0, 0.0};
      ax[am] = 1.0;
      cross(dy, ax, n1);
      nn = std::sqrt(n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
    }
    for (int k = 0; k < 3; ++k) n1[k] /= nn;
  }
  double ny[3], nz[3];
  cross(dy, n1, ny);
  cross(n1, dz, nz);
  Bend b{};
  const double s = ly + lz;
  b.w = g1 * rw * rw / (4.0 * s * s) * s / 2.0;
  b.nk = 0;
  auto fill = [&](const double *ey, const double *ez) {
    double(*c)[3] = b.c[b.nk++];
    for (int a = 0; a < nc; ++a) {
      c[1][a] = ey[a] / ly;
      c[2][a] = ez[a] / lz;
      c[0][a] = -(c[1][a] + c[2][a]);
    }
  };
  if (nc == 3) fill(n1, n1);
  fill(ny, nz);
  return b;
}

}  // namespace

std::shared_ptr<System> assemble_model(std::shared_ptr<const Network> net, int model, const double *gamma,
                                       int ncomp, double g1, double rw) {
  const Network &nw = *net;
  auto sys = std::make_shared<System>();
  sys->net = net;
  sys->model = model;
  const int nc = ncomp;
  sys->ncomp = nc;
  const int dim = nw.dim;
  const int64_t N = nw.n_nodes();
  sys->node_free.assign((size_t)N, -1);
  for (int64_t i = 0; i < N; ++i)
    if (!nw.dir[i]) {
      sys->node_free[i] = (int32_t)sys->free_node.size();
      sys->free_node.push_back((int32_t)i);
    }
  if ((int64_t)sys->free_node.size() == N) fail(SN_ESINGULAR, "no Dirichlet node: K is singular on V");
  const int64_t nf = (int64_t)sys->free_node.size();
  sys->n = nf * nc;
  const Adjacency adj = adjacency(nw);

  // lumped mass of the constant one at the free nodes (eq. 2.1)
  sys->mass.assign((size_t)nf, 0.0);
  for (int64_t f = 0; f < nf; ++f) {
    const int32_t a = sys->free_node[f];
    double m = 0.0;
    for (int64_t q = adj.start[a]; q < adj.start[a + 1]; ++q) m += 0.5 * edge_length(nw, a, adj.nbr[q]);
    sys->mass[f] = m;
  }

  // 1x1 or 3x3 edge block of the heat / truss models
  auto edge_block = [&](int64_t e, double *blk) {
    const int32_t u = nw.edges[2 * e], v = nw.edges[2 * e + 1];
    const double len = edge_length(nw, u, v);
    const double g = gamma ? gamma[e] : 1.0;
    if (nc == 1) {
      blk[0] = g / len;
      return;
    }
    double t[3];
    for (int a = 0; a < 3; ++a) t[a] = (nw.x[(size_t)v * dim + a] - nw.x[(size_t)u * dim + a]) / len;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) blk[3 * a + b] = g * (t[a] * t[b]) / len + (a == b ? 1e-6 / len : 0.0);
  };

  sys->rowptr.assign((size_t)sys->n + 1, 0);
  sys->rowptr_d.assign((size_t)sys->n + 1, 0);
  std::vector<RowTerms> rows((size_t)nc);
  auto emit = [&](int64_t f) {
    for (int a = 0; a < nc; ++a) {
      RowTerms &row = rows[(size_t)a];
      std::stable_sort(row.begin(), row.end(), [](const std::pair<int64_t, double> &x,
                                                  const std::pair<int64_t, double> &y) { return x.first < y.first; });
      const int64_t r = f * nc + a;
      for (size_t q = 0; q < row.size(); ++q) {
        const int64_t node = row[q].first / nc, comp = row[q].first % nc;
        const int32_t fc = sys->node_free[(size_t)node];
        const bool same = q > 0 && row[q].first == row[q - 1].first;
        if (fc >= 0) {
          if (same) {
            sys->val.back() += row[q].second;
          } else {
            sys->col.push_back((int32_t)(fc * nc + comp));
            sys->val.push_back(row[q].second);
            ++sys->rowptr[(size_t)r + 1];
          }
        } else {
          if (same) {
            sys->val_d.back() += row[q].second;
          } else {
            sys->col_d.push_back((int32_t)row[q].first);
            sys->val_d.push_back(row[q].second);
            ++sys->rowptr_d[(size_t)r + 1];
          }
        }
      }
      row.clear();
    }
  };

  for (int64_t f = 0; f < nf; ++f) {
    const int32_t a = sys->free_node[f];
    if (model != SN_MODEL_BEAM) {
      for (int64_t q = adj.start[a]; q < adj.start[a + 1]; ++q) {
        const int64_t e = adj.edge[q];
        const int32_t other = adj.nbr[q];
        double blk[9];
        edge_block(e, blk);
        for (int i = 0; i < nc; ++i)
          for (int j = 0; j < nc; ++j) {
            rows[i].push_back({(int64_t)a * nc + j, blk[i * nc + j]});
            rows[i].push_back({(int64_t)other * nc + j, -blk[i * nc + j]});
          }
      }
      emit(f);
      continue;
    }
    // tensile part (eq. 3.4): g1/L d d^T against a, minus it against the other end
    for (int64_t q = adj.start[a]; q < adj.start[a + 1]; ++q) {
      const int32_t b = adj.nbr[q];
      const double len = edge_length(nw, a, b);
      double d[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < dim; ++k) d[k] = (nw.x[(size_t)a * dim + k] - nw.x[(size_t)b * dim + k]) / len;
      for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) {
          const double v = g1 * d[i] * d[j] / len;
          rows[i].push_back({(int64_t)a * nc + j, v});
          rows[i].push_back({(int64_t)b * nc + j, -v});
        }
    }
    // bending part (eq. 3.5): every element w c c^T whose nodes include a:
    // a as the centre, then a as the first and as the second of a pair
    auto add_element = [&](int32_t x, int32_t y, int32_t z, int pa) {
      const Bend be = bend_element(nw, nc, g1, rw, x, y, z);
      const int32_t nodes[3] = {x, y, z};
      for (int k = 0; k < be.nk; ++k)
        for (int i = 0; i < nc; ++i) {
          const double ci = be.w * be.c[k][pa][i];
          for (int p = 0; p < 3; ++p)
            for (int j = 0; j < nc; ++j) rows[i].push_back({(int64_t)nodes[p] * nc + j, ci * be.c[k][p][j]});
        }
    };
    for (int64_t qy = adj.start[a]; qy < adj.start[a + 1]; ++qy)
      for (int64_t qz = adj.start[a]; qz < adj.start[a + 1]; ++qz)
        if (adj.nbr[qy] != adj.nbr[qz]) add_element(a, adj.nbr[qy], adj.nbr[qz], 0);
    for (int64_t qx = adj.start[a]; qx < adj.start[a + 1]; ++qx) {
      const int32_t x = adj.nbr[qx];
      for (int64_t qo = adj.start[x]; qo < adj.start[x + 1]; ++qo) {
        const int32_t o = adj.nbr[qo];
        if (o == a) continue;
        add_element(x, a, o, 1);
        add_element(x, o, a, 2);
      }
    }
    emit(f);
  }
  for (int64_t i = 0; i < sys->n; ++i) {
    sys->rowptr[i + 1] += sys->rowptr[i];
    sys->rowptr_d[i + 1] += sys->rowptr_d[i];
  }
  return sys;
}

std::shared_ptr<System> assemble(std::shared_ptr<const Network> net, int model, const double *gamma) {
  if (model != SN_MODEL_HEAT && model != SN_MODEL_TRUSS) fail(SN_EINVAL, "unknown model");
  if (model == SN_MODEL_TRUSS && net->dim != 3) fail(SN_EINVAL, "the truss model needs dim 3");
  return assemble_model(net, model, gamma, model == SN_MODEL_HEAT ? 1 : 3, 1.0, 0.0);
}

std::shared_ptr<System> assemble_beam(std::shared_ptr<const Network> net, int ncomp, double g1, double rw) {
  if (ncomp != 2 && ncomp != 3) fail(SN_EINVAL, "the beam model has 2 or 3 components");
  if (ncomp == 2 && net->dim != 2) fail(SN_EINVAL, "two components need a 2D network");
  if (!(g1 > 0.0) || !(rw >= 0.0) || !std::isfinite(g1) || !std::isfinite(rw))
    fail(SN_EINVAL, "beam constants must be finite, gamma1 > 0 and r_w >= 0");
  return assemble_model(net, SN_MODEL_BEAM, nullptr, ncomp, g1, rw);
}

void apply_full(const System &sys, const double *g, double *y) {
  const int nc = sys.ncomp;
  for (int64_t i = 0; i < sys.n; ++i) {
    double acc = 0.0;
    for (int64_t q = sys.rowptr[i]; q < sys.rowptr[i + 1]; ++q) {
      const int64_t fc = sys.col[q] / nc, comp = sys.col[q] % nc;
      acc += sys.val[q] * g[(int64_t)sys.free_node[fc] * nc + comp];
    }
    for (int64_t q = sys.rowptr_d[i]; q < sys.rowptr_d[i + 1]; ++q) acc += sys.val_d[q] * g[sys.col_d[q]];
    y[i] = acc;
  }
}

}  // namespace spnet
