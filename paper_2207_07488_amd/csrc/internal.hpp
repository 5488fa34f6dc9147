// Internal types of the spnet library (host side). Not part of the ABI.
#pragma once

#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/spnet.h"

namespace spnet {

// Error carried to the ABI boundary, where it becomes an sn_status.
struct Error : std::runtime_error {
  sn_status code;
  Error(sn_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(sn_status c, const std::string &m) { throw Error(c, m); }

struct Network {
  int dim = 2;
  std::vector<double> x;        // n_nodes * dim
  std::vector<int32_t> edges;   // 2 * n_edges
  std::vector<uint8_t> dir;     // Dirichlet flag per node
  int64_t n_nodes() const { return (int64_t)dir.size(); }
  int64_t n_edges() const { return (int64_t)edges.size() / 2; }
};

struct System {
  std::shared_ptr<const Network> net;
  int model = 0, ncomp = 1;
  int64_t n = 0;                     // free dofs
  std::vector<int32_t> free_node;    // free node index -> node id
  std::vector<int32_t> node_free;    // node id -> free node index or -1
  std::vector<int64_t> rowptr;       // CSR over dofs
  std::vector<int32_t> col;
  std::vector<double> val;
  // free rows against the dofs of Dirichlet nodes (columns node * ncomp + component)
  std::vector<int64_t> rowptr_d;
  std::vector<int32_t> col_d;
  std::vector<double> val_d;
  std::vector<double> mass;          // (M 1)(x) per free node, eq. 2.1
};

struct DeviceState;  // defined in device.hip
struct DeviceDeleter {
  void operator()(DeviceState *d) const;
};

struct Precond {
  std::shared_ptr<const System> sys;
  int nH = 1, policy = 0, dir_lo = 0, dir_hi = 0;
  int nvert_per_elem = 4;
  // coarse space: per free node, the 2^d mesh nodes of its element and phi values
  std::vector<int32_t> Pvert;  // n_free_nodes * 2^d (mesh node id)
  std::vector<double> Pphi;
  std::vector<int32_t> vert_coarse;  // mesh node -> coarse group index or -1
  std::vector<int32_t> coarse_vertex;
  int64_t m0 = 0;
  // local spaces (canonical: ascending mesh node, dofs ascending)
  std::vector<int64_t> star_ptr;
  std::vector<int32_t> star_dofs;
  std::vector<int32_t> star_vertex;
  // factorisation products (filled by factor())
  int precision = -1;
  sn_factor_info finfo{};
  std::unique_ptr<DeviceState, DeviceDeleter> dev;
};

// network.cpp
std::shared_ptr<Network> build_network_from_segments(int dim, int64_t nseg, const double *seg, double eps,
                                                     double merge_tol, int dir_lo, int dir_hi, double band);
// assemble.cpp
std::shared_ptr<System> assemble(std::shared_ptr<const Network> net, int model, const double *gamma);
std::shared_ptr<System> assemble_beam(std::shared_ptr<const Network> net, int ncomp, double g1, double rw);
void apply_full(const System &sys, const double *g, double *y);
// diagnostics.cpp: homogeneity and connectivity per box (Assumption 3.4)
void network_diagnostics(const Network &net, int nb, double r0, double *sigma, double *mu, double *density,
                         double *mu_box);
// spaces.cpp
std::unique_ptr<Precond> build_spaces(std::shared_ptr<const System> sys, int nH, int policy, int dir_lo,
                                      int dir_hi);

// factor.cpp: the factors of one local matrix in the two layouts of the GPU
// local solves.
//
// Supernodal (minimum degree order): positions are the local dofs in factor
// order, numbered level by level; a supernode s owns positions c0[s] ..
// c0[s]+w[s]-1 and sends updates to the h[s] positions R[ubase[s] ..] below
// its diagonal block (its u-slots).
struct SnFactor {
  int32_t n = 0;                    // positions
  int32_t nsn = 0, nu = 0, nlev = 0;  // supernodes, u-slots, levels
  std::vector<int32_t> perm;        // position -> canonical local index
  std::vector<int32_t> lev_pos;     // nlev + 1: first position of each level
  std::vector<int32_t> lev_u;       // nlev + 1: first u-slot of each level
  std::vector<int32_t> c0, w, h;    // per supernode
  std::vector<int64_t> sbase;       // per supernode: offset of S_s in S
  std::vector<int64_t> ubase;       // per supernode: its first u-slot
  std::vector<int32_t> snpos;       // per position: its supernode
  std::vector<int32_t> snu;         // per u-slot: its supernode
  std::vector<int32_t> R;           // per u-slot: the position it updates
  std::vector<int32_t> aptr, alist; // per position: the u-slots updating it, ascending (CSR)
  std::vector<double> S;            // per supernode [L_CC^{-1}; L_RC L_CC^{-1}], column c: rows c..w+h-1
  int64_t nnz = 0;                  // structural non-zeros of L (incl. diagonal)
  double pivot_ratio = 1.0;         // largest / smallest pivot L_jj^2
};

// The band factor split into two chains that a pair of wavefronts sweeps side
// by side. The reverse Cuthill-McKee positions are cut into a top part [0, k),
// a separator [k, k+s) (the positions coupled to the top part) and a bottom
// part [k+s, n). Chain 0 runs pads, the top part, the separator; chain 1 runs
// pads, the bottom part in reverse, the separator (each chain K + s steps, K
// a multiple of 64, the pads identity rows). L in the order (top, bottom,
// separator) has no entries between the top and the bottom part, so the two
// chains are the rows and columns (top, separator) and (bottom, separator) of
// one factor and share its separator block L_ss: the forward sweeps run apart
// until step K, where their partial sums of the separator rows are added,
// then both finish the separator identically; the backward sweeps start from
// the same separator values and run apart.
struct BandChain {
  int32_t band = 0;                 // max width of the envelope
  std::vector<int32_t> bpos;        // chain position -> band position of the star, -1: pad
  std::vector<int32_t> width_fwd, width_bwd;
  std::vector<double> invdiag, colvals, rowvals;
  int64_t nnz = 0;                  // non-zeros of the chain's factor (incl. diagonal, pads excluded)
};
struct BandTwin {
  int32_t K = 0, s = 0;             // K = 0: no split
  BandChain c[2];
};

// Both layouts of one local matrix. Band (reverse Cuthill-McKee order, the
// envelope factor): the forward stream walks the columns of L from the first,
// the backward stream walks the rows of L from the last, each listing the
// entries nearest the diagonal first. The slots of a star follow the band
// order whichever kernel solves it.
struct StarFactor {
  int32_t n = 0;
  int32_t band = 0;                 // max width of the envelope
  std::vector<int32_t> perm;        // band position -> canonical local index
  std::vector<int32_t> width_fwd;   // per step
  std::vector<int32_t> width_bwd;
  std::vector<double> invdiag;      // per position
  std::vector<double> colvals;      // forward stream values (no headers), column j entries j+1..j+w
  std::vector<double> rowvals;      // backward stream values, row i (from n-1 down) entries i-1..i-w
  int64_t env = 0;                  // stored envelope entries incl. diagonal
  int64_t nnz_rcm = 0;              // structural non-zeros of L in the band order (incl. diagonal)
  double pivot_ratio = 1.0;         // largest / smallest pivot L_jj^2 (envelope factor)
  SnFactor sn;                      // the supernodal factor of the same matrix
  BandTwin twin;                    // the band factor as two chains (long stars only)
};

struct HostFactors {
  std::vector<StarFactor> stars;
  std::vector<double> coarse_inv;   // m0 x m0 dense inverse of K_0 (symmetric)
  double coarse_pivot_ratio = 1.0;  // largest / smallest pivot of the band Cholesky of K_0
  double seconds = 0;
};

HostFactors factor_host(const Precond &pre);
// the supernodal factorisation of a symmetric positive definite matrix given
// in CSR (both triangles and the diagonal)
SnFactor factor_csr_local(int32_t n, const int32_t *ptr, const int32_t *col, const double *val);

// device.hip
void device_setup(Precond &pre, const HostFactors &hf, int precision);
void device_solve(Precond &pre, int k, const double *f, double *u, const sn_solve_opts &o, sn_solve_info *info);
void device_apply_K(Precond &pre, int k, const double *x, double *y, int device_ptrs, void *stream);
void device_apply_B(Precond &pre, int k, const double *r, double *z, int device_ptrs, void *stream);
void device_apply_K_noalloc(Precond &pre, int k, const double *x, double *y, void *stream);
void device_release(DeviceState *d);
void set_device_allocator(sn_alloc_fn alloc, sn_free_fn free_, void *ctx);
void device_profile(Precond &pre, int enable);
void device_stats(Precond &pre, sn_kernel_stats *st);
int64_t device_bytes(const Precond &pre);
void device_engine_info(Precond &pre, int k, sn_engine_info *info);
void device_set_star_split(Precond &pre, int64_t n_sn);
void device_set_coarse_launch(Precond &pre, int mode);
void device_set_sn_beyond_lds(Precond &pre, int mode);
void device_set_band_twins(Precond &pre, int64_t min_positions);
void device_set_band_queue(Precond &pre, int32_t waves);

// ---------------------------------------------------------------------------
// Engine: the device workspace of kc PCG columns (independent recurrences, one
// right-hand side each) on one factored preconditioner. Columns are admitted
// and retired between ticks; a tick queues iterations for every running
// column on the engine's own stream and reads the column states back
// asynchronously. sn_solve and the server both run on engines.
// ---------------------------------------------------------------------------
struct Engine;
struct ColumnStatus {
  int64_t iters;
  double rr, f2, tol2, t2;
  int32_t active, done, verify, replacements, fixed;
};
// a stopped column has converged when its recurrence residual and its FP64
// true residual (both squared) meet the squared tolerance (the true one up to
// rounding of its own sum)
inline int32_t column_converged(double rr, double t2, double tol2) {
  return rr <= tol2 && t2 <= tol2 * 1.0001 ? 1 : 0;
}
int engine_width_for(int k);                          // 1, 2, 4, 8 or 16 >= k
int64_t engine_footprint(const Precond &pre, int kc);  // device bytes of an engine
Engine *engine_create(Precond &pre, int kc);           // pre must be factored
void engine_destroy(Engine *e);
int engine_width(const Engine *e);
// Start columns cols[0..k-1] on f (host, n x k row-major): u = 0, r = f, p = 0,
// per-column tolerance and iteration limit. The engine must be idle.
void engine_admit(Engine *e, int k, const int32_t *cols, const double *f, const double *rtol,
                  const int64_t *max_iter);
// Queue `iters` iterations and the true-residual checks of stopped columns;
// the column states are read back when the tick completes.
void engine_tick(Engine *e, int iters, bool use_graph);
bool engine_query(Engine *e);  // the last tick has completed
void engine_wait(Engine *e);
// the calling host thread's current HIP device, and making `dev` current
int device_current();
void device_bind(int dev);
void engine_status(const Engine *e, ColumnStatus *out);  // kc entries, as of the last completed tick
// copy column c of u to host (stride ld) and free the column
void engine_retire(Engine *e, int c, double *u, int64_t ld);

}  // namespace spnet
