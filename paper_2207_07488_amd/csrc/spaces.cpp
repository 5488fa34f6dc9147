// Coarse space V_H (Q1 on T_H restricted to the free nodes, Sec. 2.3) and the
// local spaces V_j = V(U(y_j)) on mesh stars (Sec. 4.1): the free nodes at which
// phi_j is positive (its support, which Sec. 5 identifies with U(y_j)).
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace spnet {

std::unique_ptr<Precond> build_spaces(std::shared_ptr<const System> sys, int nH, int policy, int dir_lo,
                                      int dir_hi) {
  if (nH < 1 || nH > 4096) fail(SN_EINVAL, "nH out of range");
  if (policy != SN_STARS_ALL && policy != SN_STARS_FREE) fail(SN_EINVAL, "unknown star policy");
  const Network &net = *sys->net;
  const int dim = net.dim, nc = sys->ncomp, nv = 1 << dim;
  auto pre = std::make_unique<Precond>();
  pre->sys = sys;
  pre->nH = nH;
  pre->policy = policy;
  pre->dir_lo = dir_lo;
  pre->dir_hi = dir_hi;
  pre->nvert_per_elem = nv;
  const int64_t side = nH + 1;
  int64_t nvert = 1;
  for (int k = 0; k < dim; ++k) nvert *= side;
  const int64_t nf = (int64_t)sys->free_node.size();

  // element of each free node and the Q1 basis values at it:
  // e_k = min(floor(x_k nH), nH - 1), xi_k = x_k nH - e_k,
  // phi_{e+b}(x) = prod_k (b_k ? xi_k : 1 - xi_k).
  // in_star[f, b]: every factor is positive, so x lies in the support of the
  // basis function of mesh node e + b (on a face of T_H some factors vanish)
  pre->Pvert.resize((size_t)nf * nv);
  pre->Pphi.resize((size_t)nf * nv);
  std::vector<uint8_t> in_star((size_t)nf * nv, 0);
  for (int64_t f = 0; f < nf; ++f) {
    const double *x = &net.x[(size_t)sys->free_node[f] * dim];
    int64_t e[3];
    double xi[3];
    for (int k = 0; k < dim; ++k) {
      int64_t ek = (int64_t)std::floor(x[k] * (double)nH);
      ek = std::max<int64_t>(0, std::min<int64_t>(ek, nH - 1));
      e[k] = ek;
      xi[k] = x[k] * (double)nH - (double)ek;
    }
    // per axis: is the lower (bit 0) / upper (bit 1) vertex's factor positive
    uint32_t pos_lo = 0, pos_hi = 0;
    for (int k = 0; k < dim; ++k) {
      if (xi[k] < 1.0) pos_lo |= 1u << k;
      if (xi[k] > 0.0) pos_hi |= 1u << k;
    }
    for (int b = 0; b < nv; ++b) {
      int64_t id = 0, stride = 1;
      double phi = 1.0;
      for (int k = 0; k < dim; ++k) {
        const int bit = (b >> k) & 1;
        id += (e[k] + bit) * stride;
        stride *= side;
        phi = phi * (bit ? xi[k] : 1.0 - xi[k]);
      }
      // an upper-vertex axis needs xi > 0, a lower-vertex axis xi < 1
      const uint32_t ub = (uint32_t)b, lower = ~ub & ((1u << dim) - 1);
      pre->Pvert[(size_t)f * nv + b] = (int32_t)id;
      pre->Pphi[(size_t)f * nv + b] = phi;
      in_star[(size_t)f * nv + b] = ((ub & ~pos_hi) | (lower & ~pos_lo)) == 0 ? 1 : 0;
    }
  }
  auto on_gamma = [&](int64_t id) {
    for (int k = 0; k < dim; ++k) {
      const int64_t c = id % side;
      id /= side;
      if (((dir_lo >> k) & 1) && c == 0) return true;
      if (((dir_hi >> k) & 1) && c == nH) return true;
    }
    return false;
  };
  // coarse dofs: mesh nodes off Gamma with a basis function that is non-zero
  // at some free node, lexicographic order
  std::vector<uint8_t> live((size_t)nvert, 0);
  for (size_t q = 0; q < in_star.size(); ++q)
    if (in_star[q]) live[pre->Pvert[q]] = 1;
  pre->vert_coarse.assign((size_t)nvert, -1);
  for (int64_t id = 0; id < nvert; ++id)
    if (live[id] && !on_gamma(id)) {
      pre->vert_coarse[id] = (int32_t)pre->coarse_vertex.size();
      pre->coarse_vertex.push_back((int32_t)id);
    }
  pre->m0 = (int64_t)pre->coarse_vertex.size() * nc;

  // stars: bucket the free nodes by the mesh nodes whose basis function is
  // positive at them (at most the 2^d of their element)
  std::vector<int64_t> cnt((size_t)nvert + 1, 0);
  for (size_t q = 0; q < pre->Pvert.size(); ++q)
    if (in_star[q]) ++cnt[pre->Pvert[q] + 1];
  for (int64_t id = 0; id < nvert; ++id) cnt[id + 1] += cnt[id];
  std::vector<int32_t> members((size_t)cnt[nvert]);
  {
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t f = 0; f < nf; ++f)
      for (int b = 0; b < nv; ++b)
        if (in_star[(size_t)f * nv + b]) members[pos[pre->Pvert[(size_t)f * nv + b]]++] = (int32_t)f;
  }
  pre->star_ptr.push_back(0);
  for (int64_t id = 0; id < nvert; ++id) {
    if (cnt[id + 1] == cnt[id]) continue;
    if (policy == SN_STARS_FREE && on_gamma(id)) continue;
    for (int64_t q = cnt[id]; q < cnt[id + 1]; ++q)
      for (int c = 0; c < nc; ++c) pre->star_dofs.push_back(members[q] * nc + c);
    pre->star_vertex.push_back((int32_t)id);
    pre->star_ptr.push_back((int64_t)pre->star_dofs.size());
  }
  return pre;
}

}  // namespace spnet
