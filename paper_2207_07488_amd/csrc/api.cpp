// C ABI of the spnet library: handles, status codes and thread-local errors.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "handles.hpp"

namespace {
thread_local std::string g_err;
}  // namespace

sn_status spnet::guarded_call(void (*fn)(void *), void *ctx) {
  try {
    fn(ctx);
    return SN_OK;
  } catch (const spnet::Error &e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return SN_ENOMEM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return SN_EINVAL;
  } catch (...) {
    g_err = "unknown error";
    return SN_EINVAL;
  }
}

namespace {
using spnet::guarded;

#define REQUIRE(c, msg) \
  do {                  \
    if (!(c)) spnet::fail(SN_EINVAL, msg); \
  } while (0)
}  // namespace

extern "C" {

const char *sn_last_error(void) { return g_err.c_str(); }
const char *sn_version(void) { return "spnet 0.1 gfx950"; }

sn_status sn_set_allocator(sn_alloc_fn alloc, sn_free_fn free_, void *ctx) {
  return guarded([&] { spnet::set_device_allocator(alloc, free_, ctx); });
}

sn_status sn_network_from_segments(int dim, int64_t n_segments, const double *segments, double contact_eps,
                                   double merge_tol, int dir_lo, int dir_hi, double band, sn_network *out) {
  return guarded([&] {
    REQUIRE(out, "out is NULL");
    auto net = spnet::build_network_from_segments(dim, n_segments, segments, contact_eps, merge_tol, dir_lo, dir_hi,
                                                  band);
    *out = new sn_network_s{net};
  });
}

sn_status sn_network_from_arrays(int dim, int64_t n_nodes, const double *coords, int64_t n_edges,
                                 const int32_t *edges, const uint8_t *dirichlet, sn_network *out) {
  return guarded([&] {
    REQUIRE(out, "out is NULL");
    REQUIRE(dim == 2 || dim == 3, "dim must be 2 or 3");
    REQUIRE(n_nodes >= 0 && n_edges >= 0, "negative size");
    REQUIRE((n_nodes == 0 || (coords && dirichlet)) && (n_edges == 0 || edges), "missing array");
    auto net = std::make_shared<spnet::Network>();
    net->dim = dim;
    net->x.assign(coords, coords + n_nodes * dim);
    net->edges.assign(edges, edges + 2 * n_edges);
    net->dir.assign(dirichlet, dirichlet + n_nodes);
    for (int64_t k = 0; k < 2 * n_edges; ++k)
      REQUIRE(edges[k] >= 0 && edges[k] < n_nodes, "edge end out of range");
    for (int64_t k = 0; k < n_edges; ++k) REQUIRE(edges[2 * k] != edges[2 * k + 1], "self loop");
    for (double v : net->x) REQUIRE(std::isfinite(v), "non-finite coordinate");
    *out = new sn_network_s{net};
  });
}

sn_status sn_network_info(sn_network net, int *dim, int64_t *n_nodes, int64_t *n_edges) {
  return guarded([&] {
    REQUIRE(net, "null network");
    if (dim) *dim = net->p->dim;
    if (n_nodes) *n_nodes = net->p->n_nodes();
    if (n_edges) *n_edges = net->p->n_edges();
  });
}

sn_status sn_network_export(sn_network net, double *coords, int32_t *edges, uint8_t *dirichlet) {
  return guarded([&] {
    REQUIRE(net, "null network");
    const auto &n = *net->p;
    if (coords) std::memcpy(coords, n.x.data(), n.x.size() * sizeof(double));
    if (edges) std::memcpy(edges, n.edges.data(), n.edges.size() * sizeof(int32_t));
    if (dirichlet) std::memcpy(dirichlet, n.dir.data(), n.dir.size());
  });
}

void sn_network_destroy(sn_network net) { delete net; }

sn_status sn_network_diagnostics(sn_network net, int nb, double r0, double *sigma, double *mu, double *density,
                                 double *mu_box) {
  return guarded([&] {
    REQUIRE(net, "null network");
    REQUIRE(sigma && mu, "null output");
    REQUIRE(std::isfinite(r0), "r0 must be finite");
    spnet::network_diagnostics(*net->p, nb, r0, sigma, mu, density, mu_box);
  });
}

sn_status sn_assemble(sn_network net, int model, const double *gamma, sn_system *out) {
  return guarded([&] {
    REQUIRE(net && out, "null argument");
    auto sys = spnet::assemble(net->p, model, gamma);
    *out = new sn_system_s{sys};
  });
}

sn_status sn_assemble_beam(sn_network net, int ncomp, double gamma1, double wire_radius, sn_system *out) {
  return guarded([&] {
    REQUIRE(net && out, "null argument");
    auto sys = spnet::assemble_beam(net->p, ncomp, gamma1, wire_radius);
    *out = new sn_system_s{sys};
  });
}

sn_status sn_system_apply_full(sn_system sys, const double *g, double *y) {
  return guarded([&] {
    REQUIRE(sys && g && y, "null argument");
    const int64_t nd = sys->p->net->n_nodes() * sys->p->ncomp;
    for (int64_t i = 0; i < nd; ++i) REQUIRE(std::isfinite(g[i]), "non-finite value in g");
    spnet::apply_full(*sys->p, g, y);
  });
}

sn_status sn_system_mass(sn_system sys, double *m) {
  return guarded([&] {
    REQUIRE(sys && m, "null argument");
    std::copy(sys->p->mass.begin(), sys->p->mass.end(), m);
  });
}

sn_status sn_system_info(sn_system sys, int64_t *n_dofs, int64_t *nnz, int *ncomp, int64_t *n_free_nodes) {
  return guarded([&] {
    REQUIRE(sys, "null system");
    if (n_dofs) *n_dofs = sys->p->n;
    if (nnz) *nnz = (int64_t)sys->p->col.size();
    if (ncomp) *ncomp = sys->p->ncomp;
    if (n_free_nodes) *n_free_nodes = (int64_t)sys->p->free_node.size();
  });
}

sn_status sn_system_export_csr(sn_system sys, int64_t *rowptr, int32_t *col, double *val) {
  return guarded([&] {
    REQUIRE(sys, "null system");
    const auto &s = *sys->p;
    if (rowptr) std::memcpy(rowptr, s.rowptr.data(), s.rowptr.size() * sizeof(int64_t));
    if (col) std::memcpy(col, s.col.data(), s.col.size() * sizeof(int32_t));
    if (val) std::memcpy(val, s.val.data(), s.val.size() * sizeof(double));
  });
}

sn_status sn_system_free_nodes(sn_system sys, int32_t *free_node) {
  return guarded([&] {
    REQUIRE(sys && free_node, "null argument");
    std::memcpy(free_node, sys->p->free_node.data(), sys->p->free_node.size() * sizeof(int32_t));
  });
}

void sn_system_destroy(sn_system sys) { delete sys; }

sn_status sn_precond_build(sn_system sys, int nH, int star_policy, int dir_lo, int dir_hi, sn_precond *out) {
  return guarded([&] {
    REQUIRE(sys && out, "null argument");
    std::unique_ptr<spnet::Precond> pre = spnet::build_spaces(sys->p, nH, star_policy, dir_lo, dir_hi);
    *out = new sn_precond_s{std::shared_ptr<spnet::Precond>(pre.release())};
  });
}

sn_status sn_precond_info(sn_precond pre, int64_t *m0, int64_t *n_stars, int64_t *star_total) {
  return guarded([&] {
    REQUIRE(pre, "null preconditioner");
    if (m0) *m0 = pre->p->m0;
    if (n_stars) *n_stars = (int64_t)pre->p->star_vertex.size();
    if (star_total) *star_total = (int64_t)pre->p->star_dofs.size();
  });
}

sn_status sn_precond_export_stars(sn_precond pre, int64_t *star_ptr, int32_t *star_dofs, int32_t *star_vertex) {
  return guarded([&] {
    REQUIRE(pre, "null preconditioner");
    const auto &p = *pre->p;
    if (star_ptr) std::memcpy(star_ptr, p.star_ptr.data(), p.star_ptr.size() * sizeof(int64_t));
    if (star_dofs) std::memcpy(star_dofs, p.star_dofs.data(), p.star_dofs.size() * sizeof(int32_t));
    if (star_vertex) std::memcpy(star_vertex, p.star_vertex.data(), p.star_vertex.size() * sizeof(int32_t));
  });
}

sn_status sn_precond_export_coarse(sn_precond pre, int32_t *coarse_vertex) {
  return guarded([&] {
    REQUIRE(pre && coarse_vertex, "null argument");
    const auto &p = *pre->p;
    std::memcpy(coarse_vertex, p.coarse_vertex.data(), p.coarse_vertex.size() * sizeof(int32_t));
  });
}

sn_status sn_precond_factor(sn_precond pre, int precision) {
  return guarded([&] {
    REQUIRE(pre, "null preconditioner");
    REQUIRE(precision == SN_PREC_FP64 || precision == SN_PREC_FP32_STARS ||
                precision == SN_PREC_FP32_STARS_COARSE,
            "unknown precision");
    spnet::Precond &p = *pre->p;
    if (p.dev) {
      spnet::device_release(p.dev.release());
      p.precision = -1;
    }
    spnet::HostFactors hf = spnet::factor_host(p);
    spnet::device_setup(p, hf, precision);
  });
}

sn_status sn_precond_factor_info(sn_precond pre, sn_factor_info *info) {
  return guarded([&] {
    REQUIRE(pre && info, "null argument");
    REQUIRE(pre->p->dev, "not factored");
    *info = pre->p->finfo;
  });
}

void sn_precond_destroy(sn_precond pre) { delete pre; }

void sn_solve_opts_default(sn_solve_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rtol = 1e-8;
  o->max_iter = 1000;
  o->check_every = 8;
}

sn_status sn_solve(sn_precond pre, int k, const double *f, double *u, const sn_solve_opts *opts,
                   sn_solve_info *info) {
  return guarded([&] {
    REQUIRE(pre && f && u && info, "null argument");
    REQUIRE(k >= 1 && k <= 16, "k must be in 1..16");
    REQUIRE(pre->p->dev, "preconditioner not factored");
    sn_solve_opts o;
    if (opts) o = *opts;
    else sn_solve_opts_default(&o);
    REQUIRE(o.rtol >= 0.0 && std::isfinite(o.rtol), "bad rtol");
    if (!o.device_ptrs) {
      const int64_t n = pre->p->sys->n;
      for (int64_t i = 0; i < n * k; ++i) REQUIRE(std::isfinite(f[i]), "non-finite right-hand side");
    }
    spnet::device_solve(*pre->p, k, f, u, o, info);
  });
}

sn_status sn_precond_profile(sn_precond pre, int enable) {
  return guarded([&] {
    REQUIRE(pre && pre->p->dev, "preconditioner not factored");
    spnet::device_profile(*pre->p, enable);
  });
}

sn_status sn_precond_kernel_stats(sn_precond pre, sn_kernel_stats *stats) {
  return guarded([&] {
    REQUIRE(pre && stats && pre->p->dev, "null argument or not factored");
    spnet::device_stats(*pre->p, stats);
  });
}

sn_status sn_precond_set_star_split(sn_precond pre, int64_t n_sn) {
  return guarded([&] {
    REQUIRE(pre && pre->p->dev, "null argument or not factored");
    spnet::device_set_star_split(*pre->p, n_sn);
  });
}

sn_status sn_precond_set_band_twins(sn_precond pre, int64_t min_positions) {
  return guarded([&] {
    REQUIRE(pre && pre->p->dev, "null argument or not factored");
    spnet::device_set_band_twins(*pre->p, min_positions);
  });
}

sn_status sn_precond_set_band_queue(sn_precond pre, int32_t waves) {
  return guarded([&] {
    REQUIRE(pre && pre->p->dev, "null argument or not factored");
    spnet::device_set_band_queue(*pre->p, waves);
  });
}

sn_status sn_precond_set_sn_beyond_lds(sn_precond pre, int mode) {
  return guarded([&] {
    REQUIRE(pre && pre->p->dev, "null argument or not factored");
    REQUIRE(mode >= -1 && mode <= 1, "mode must be in -1..1");
    spnet::device_set_sn_beyond_lds(*pre->p, mode);
  });
}

sn_status sn_precond_set_coarse_launch(sn_precond pre, int mode) {
  return guarded([&] {
    REQUIRE(pre && pre->p->dev, "null argument or not factored");
    REQUIRE(mode >= -1 && mode <= 8, "mode must be in -1..8");
    spnet::device_set_coarse_launch(*pre->p, mode);
  });
}

sn_status sn_precond_engine_info(sn_precond pre, int k, sn_engine_info *info) {
  return guarded([&] {
    REQUIRE(pre && info && pre->p->dev, "null argument or not factored");
    REQUIRE(k >= 1 && k <= 16, "k must be in 1..16");
    spnet::device_engine_info(*pre->p, k, info);
  });
}

sn_status sn_apply_K(sn_precond pre, int k, const double *x, double *y, int device_ptrs, void *stream) {
  return guarded([&] {
    REQUIRE(pre && x && y, "null argument");
    REQUIRE(k >= 1 && k <= 16, "k must be in 1..16");
    REQUIRE(pre->p->dev, "preconditioner not factored");
    spnet::device_apply_K(*pre->p, k, x, y, device_ptrs, stream);
  });
}

sn_status sn_apply_K_noalloc(sn_precond pre, int k, const double *x, double *y, void *stream) {
  return guarded([&] {
    REQUIRE(pre && x && y, "null argument");
    REQUIRE(k >= 1 && k <= 16, "k must be in 1..16");
    REQUIRE(pre->p->dev, "preconditioner not factored");
    spnet::device_apply_K_noalloc(*pre->p, k, x, y, stream);
  });
}

sn_status sn_apply_B(sn_precond pre, int k, const double *r, double *z, int device_ptrs, void *stream) {
  return guarded([&] {
    REQUIRE(pre && r && z, "null argument");
    REQUIRE(k >= 1 && k <= 16, "k must be in 1..16");
    REQUIRE(pre->p->dev, "preconditioner not factored");
    spnet::device_apply_B(*pre->p, k, r, z, device_ptrs, stream);
  });
}

}  // extern "C"
