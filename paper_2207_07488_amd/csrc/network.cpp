// Network construction (Sec. 2.1) from raw fiber segments (generator of Sec. 6.1).
//
// The floating-point steps that decide the integer structure (clipping, the
// crossing and contact tests, merge distances, the Dirichlet band) evaluate the
// same expressions in the same order as the canonical description of the
// generator, so that the node and edge lists are reproducible bit for bit by
// any implementation of it. Built with -ffp-contract=off.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

#include "internal.hpp"

namespace spnet {
namespace {

inline double sq_dist(int dim, const double *p, const double *q) {
  double acc = 0.0;
  for (int k = 0; k < dim; ++k) {
    const double t = p[k] - q[k];
    acc = acc + t * t;
  }
  return acc;
}

inline double dotd(const double *u, const double *v) {
  double acc = 0.0;
  for (int k = 0; k < 3; ++k) acc = acc + u[k] * v[k];
  return acc;
}

inline double unit_clamp(double t) { return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t); }

struct Seg {
  double A[3], B[3];
};

// Liang-Barsky clipping to [0,1]^dim; the face that cuts an end snaps it.
bool clip_to_box(int dim, const double *a, const double *b, double tol, Seg &s) {
  double d[3];
  for (int k = 0; k < dim; ++k) d[k] = b[k] - a[k];
  double t_enter = 0.0, t_exit = 1.0;
  int face_enter = -1, face_exit = -1;
  for (int k = 0; k < dim; ++k) {
    if (d[k] == 0.0) {
      if (a[k] < 0.0 || a[k] > 1.0) return false;
      continue;
    }
    const double t_lo = (0.0 - a[k]) / d[k];
    const double t_hi = (1.0 - a[k]) / d[k];
    const bool up = d[k] > 0.0;
    const double tin = up ? t_lo : t_hi, tout = up ? t_hi : t_lo;
    const int fin = up ? 2 * k : 2 * k + 1, fout = up ? 2 * k + 1 : 2 * k;
    if (tin > t_enter) {
      t_enter = tin;
      face_enter = fin;
    }
    if (tout < t_exit) {
      t_exit = tout;
      face_exit = fout;
    }
  }
  if (!(t_enter < t_exit)) return false;
  for (int k = 0; k < dim; ++k) {
    s.A[k] = a[k] + t_enter * d[k];
    s.B[k] = a[k] + t_exit * d[k];
  }
  if (face_enter >= 0) s.A[face_enter >> 1] = (face_enter & 1) ? 1.0 : 0.0;
  if (face_exit >= 0) s.B[face_exit >> 1] = (face_exit & 1) ? 1.0 : 0.0;
  for (int k = 0; k < dim; ++k) {
    s.A[k] = unit_clamp(s.A[k]);
    s.B[k] = unit_clamp(s.B[k]);
  }
  return sq_dist(dim, s.A, s.B) >= tol * tol;
}

struct Hit {
  int64_t i, j;
  double ti, tj;
  double p[3];
  bool operator<(const Hit &o) const { return i != o.i ? i < o.i : j < o.j; }
};

bool crossing_2d(const Seg &u, const Seg &v, Hit &h) {
  const double du0 = u.B[0] - u.A[0], du1 = u.B[1] - u.A[1];
  const double dv0 = v.B[0] - v.A[0], dv1 = v.B[1] - v.A[1];
  const double det = du0 * dv1 - du1 * dv0;
  if (det == 0.0) return false;
  const double w0 = v.A[0] - u.A[0], w1 = v.A[1] - u.A[1];
  const double t = (w0 * dv1 - w1 * dv0) / det;
  const double s = (w0 * du1 - w1 * du0) / det;
  if (!(t >= 0.0 && t <= 1.0 && s >= 0.0 && s <= 1.0)) return false;
  h.ti = t;
  h.tj = s;
  h.p[0] = u.A[0] + t * du0;
  h.p[1] = u.A[1] + t * du1;
  h.p[2] = 0.0;
  return true;
}

// closest points of two segments with clamping of both parameters
bool contact_3d(const Seg &u, const Seg &v, double eps, Hit &h) {
  double d1[3], d2[3], r[3];
  for (int k = 0; k < 3; ++k) {
    d1[k] = u.B[k] - u.A[k];
    d2[k] = v.B[k] - v.A[k];
    r[k] = u.A[k] - v.A[k];
  }
  const double a = dotd(d1, d1), e = dotd(d2, d2), f = dotd(d2, r);
  const double c = dotd(d1, r), b = dotd(d1, d2);
  const double den = a * e - b * b;
  double s = den != 0.0 ? unit_clamp((b * f - c * e) / den) : 0.0;
  double t = (b * s + f) / e;
  if (t < 0.0) {
    t = 0.0;
    s = unit_clamp(-c / a);
  } else if (t > 1.0) {
    t = 1.0;
    s = unit_clamp((b - c) / a);
  }
  double pu[3], pv[3];
  for (int k = 0; k < 3; ++k) {
    pu[k] = u.A[k] + s * d1[k];
    pv[k] = v.A[k] + t * d2[k];
  }
  if (!(sq_dist(3, pu, pv) < eps * eps)) return false;
  h.ti = s;
  h.tj = t;
  for (int k = 0; k < 3; ++k) h.p[k] = 0.5 * (pu[k] + pv[k]);
  return true;
}

struct MinRootSets {
  std::vector<int64_t> up;
  explicit MinRootSets(int64_t n) : up(n) { std::iota(up.begin(), up.end(), 0); }
  int64_t root(int64_t i) {
    int64_t r = i;
    while (up[r] != r) r = up[r];
    while (up[i] != r) {
      const int64_t nx = up[i];
      up[i] = r;
      i = nx;
    }
    return r;
  }
  void join(int64_t a, int64_t b) {
    a = root(a);
    b = root(b);
    if (a == b) return;
    if (a < b) up[b] = a;
    else up[a] = b;
  }
};

}  // namespace

std::shared_ptr<Network> build_network_from_segments(int dim, int64_t nseg, const double *seg, double eps,
                                                     double merge_tol, int dir_lo, int dir_hi, double band) {
  if (dim != 2 && dim != 3) fail(SN_EINVAL, "dim must be 2 or 3");
  if (nseg < 0 || (nseg > 0 && !seg)) fail(SN_EINVAL, "segments missing");
  if (!(merge_tol > 0.0)) fail(SN_EINVAL, "merge_tol must be positive");
  if (dim == 3 && !(eps > 0.0)) fail(SN_EINVAL, "contact_eps must be positive in 3D");

  // clipped segments in input order
  std::vector<Seg> segs;
  segs.reserve((size_t)nseg);
  for (int64_t i = 0; i < nseg; ++i) {
    Seg s{};
    if (clip_to_box(dim, seg + (size_t)i * 2 * dim, seg + (size_t)i * 2 * dim + dim, merge_tol, s))
      segs.push_back(s);
  }
  const int64_t S = (int64_t)segs.size();

  // candidate pairs through a uniform grid over segment midpoints whose cell
  // side is at least (longest segment + contact distance)
  double longest = 0.0;
  for (const Seg &s : segs) longest = std::max(longest, std::sqrt(sq_dist(dim, s.A, s.B)));
  const double reach = longest + (dim == 3 ? eps : 0.0);
  // (the 1e-9 margin keeps the neighbour test exact under rounding of the cell index)
  int64_t cells = reach > 0.0 ? (int64_t)std::floor(1.0 / (reach * (1.0 + 1e-9))) : 1;
  cells = std::max<int64_t>(1, std::min<int64_t>(cells, dim == 2 ? 2048 : 160));
  std::vector<std::pair<int64_t, int64_t>> keyed((size_t)S);  // (cell key, segment)
  std::vector<int64_t> cell_of((size_t)S);
  for (int64_t i = 0; i < S; ++i) {
    int64_t key = 0;
    for (int k = dim - 1; k >= 0; --k) {
      const double mid = 0.5 * (segs[i].A[k] + segs[i].B[k]);
      int64_t c = (int64_t)std::floor(mid * (double)cells);
      c = std::min<int64_t>(std::max<int64_t>(c, 0), cells - 1);
      key = key * cells + c;
    }
    keyed[i] = {key, i};
    cell_of[i] = key;
  }
  std::sort(keyed.begin(), keyed.end());
  std::vector<Hit> hits;
  auto visit_cell = [&](int64_t i, int64_t key) {
    auto lo = std::lower_bound(keyed.begin(), keyed.end(), std::make_pair(key, (int64_t)-1));
    for (auto it = lo; it != keyed.end() && it->first == key; ++it) {
      const int64_t j = it->second;
      if (j <= i) continue;
      Hit h;
      const bool ok = dim == 2 ? crossing_2d(segs[i], segs[j], h) : contact_3d(segs[i], segs[j], eps, h);
      if (ok) {
        h.i = i;
        h.j = j;
        hits.push_back(h);
      }
    }
  };
  for (int64_t i = 0; i < S; ++i) {
    int64_t c[3] = {0, 0, 0};
    int64_t rem = cell_of[i];
    for (int k = 0; k < dim; ++k) {
      c[k] = rem % cells;
      rem /= cells;
    }
    const int64_t zlo = dim == 3 ? std::max<int64_t>(c[2] - 1, 0) : 0;
    const int64_t zhi = dim == 3 ? std::min<int64_t>(c[2] + 1, cells - 1) : 0;
    for (int64_t z = zlo; z <= zhi; ++z)
      for (int64_t y = std::max<int64_t>(c[1] - 1, 0); y <= std::min<int64_t>(c[1] + 1, cells - 1); ++y)
        for (int64_t xx = std::max<int64_t>(c[0] - 1, 0); xx <= std::min<int64_t>(c[0] + 1, cells - 1); ++xx)
          visit_cell(i, (z * cells + y) * cells + xx);
  }
  std::sort(hits.begin(), hits.end());

  // raw nodes: end points 2s, 2s+1, crossings after them in pair order
  const int64_t NR = 2 * S + (int64_t)hits.size();
  std::vector<double> X((size_t)NR * dim);
  for (int64_t s = 0; s < S; ++s)
    for (int k = 0; k < dim; ++k) {
      X[(size_t)(2 * s) * dim + k] = segs[s].A[k];
      X[(size_t)(2 * s + 1) * dim + k] = segs[s].B[k];
    }
  for (size_t h = 0; h < hits.size(); ++h)
    for (int k = 0; k < dim; ++k) X[(size_t)(2 * S + (int64_t)h) * dim + k] = hits[h].p[k];

  // nodes along each segment by (parameter, id); edges between neighbours
  std::vector<std::vector<std::pair<double, int64_t>>> along((size_t)S);
  for (int64_t s = 0; s < S; ++s) {
    along[s].push_back({0.0, 2 * s});
    along[s].push_back({1.0, 2 * s + 1});
  }
  for (size_t h = 0; h < hits.size(); ++h) {
    along[hits[h].i].push_back({hits[h].ti, 2 * S + (int64_t)h});
    along[hits[h].j].push_back({hits[h].tj, 2 * S + (int64_t)h});
  }
  std::vector<std::pair<int64_t, int64_t>> raw_edges;
  for (int64_t s = 0; s < S; ++s) {
    auto &v = along[s];
    std::sort(v.begin(), v.end());
    for (size_t q = 0; q + 1 < v.size(); ++q) raw_edges.push_back({v[q].second, v[q + 1].second});
    std::vector<std::pair<double, int64_t>>().swap(v);
  }

  // merge nodes closer than merge_tol: cells of side merge_tol, neighbours +-1
  MinRootSets merged(NR);
  {
    const double tol2 = merge_tol * merge_tol;
    const double cell_side = merge_tol * (1.0 + 1e-9);
    std::vector<std::pair<std::array<int64_t, 3>, int64_t>> bucket((size_t)NR);
    for (int64_t i = 0; i < NR; ++i) {
      std::array<int64_t, 3> c{0, 0, 0};
      for (int k = 0; k < dim; ++k) c[k] = (int64_t)std::floor(X[(size_t)i * dim + k] / cell_side);
      bucket[i] = {c, i};
    }
    std::sort(bucket.begin(), bucket.end());
    for (int64_t a = 0; a < NR; ++a) {
      const auto &ca = bucket[a].first;
      const int64_t i = bucket[a].second;
      const int64_t dz = dim == 3 ? 1 : 0;
      for (int64_t oz = -dz; oz <= dz; ++oz)
        for (int64_t oy = -1; oy <= 1; ++oy)
          for (int64_t ox = -1; ox <= 1; ++ox) {
            std::array<int64_t, 3> cb{ca[0] + ox, ca[1] + oy, ca[2] + oz};
            auto it = std::lower_bound(bucket.begin(), bucket.end(), std::make_pair(cb, (int64_t)-1));
            for (; it != bucket.end() && it->first == cb; ++it) {
              const int64_t j = it->second;
              if (j <= i) continue;
              if (sq_dist(dim, &X[(size_t)i * dim], &X[(size_t)j * dim]) < tol2) merged.join(i, j);
            }
          }
    }
  }
  std::vector<std::pair<int64_t, int64_t>> edges;
  edges.reserve(raw_edges.size());
  for (auto &e : raw_edges) {
    const int64_t a = merged.root(e.first), b = merged.root(e.second);
    if (a != b) edges.push_back({a, b});
  }
  std::vector<std::pair<int64_t, int64_t>>().swap(raw_edges);

  // largest connected component among the surviving (representative) nodes
  MinRootSets comp(NR);
  for (auto &e : edges) comp.join(e.first, e.second);
  std::vector<int64_t> count((size_t)NR, 0);
  for (int64_t i = 0; i < NR; ++i)
    if (merged.root(i) == i) ++count[comp.root(i)];
  int64_t best = -1;
  for (int64_t r = 0; r < NR; ++r)
    if (count[r] > 0 && (best < 0 || count[r] > count[best])) best = r;

  auto net = std::make_shared<Network>();
  net->dim = dim;
  std::vector<int64_t> renum((size_t)NR, -1);
  int64_t N = 0;
  for (int64_t i = 0; i < NR; ++i)
    if (best >= 0 && merged.root(i) == i && comp.root(i) == best) renum[i] = N++;
  net->x.resize((size_t)N * dim);
  net->dir.assign((size_t)N, 0);
  for (int64_t i = 0; i < NR; ++i)
    if (renum[i] >= 0)
      for (int k = 0; k < dim; ++k) net->x[(size_t)renum[i] * dim + k] = X[(size_t)i * dim + k];
  for (auto &e : edges)
    if (renum[e.first] >= 0) {
      net->edges.push_back((int32_t)renum[e.first]);
      net->edges.push_back((int32_t)renum[e.second]);
    }
  for (int64_t i = 0; i < N; ++i) {
    bool d = false;
    for (int k = 0; k < dim; ++k) {
      const double v = net->x[(size_t)i * dim + k];
      if (((dir_lo >> k) & 1) && v <= band) d = true;
      if (((dir_hi >> k) & 1) && v >= 1.0 - band) d = true;
    }
    net->dir[i] = d ? 1 : 0;
  }
  return net;
}

}  // namespace spnet
