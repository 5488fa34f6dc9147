/*
 * spnet.h -- C ABI of the MI355X (gfx950) solver for spatial network models by
 * two-level additive Schwarz preconditioned conjugate gradients
 * (Goertz, Hellman, Malqvist, "Iterative solution of spatial network models by
 * subspace decomposition", arXiv 2207.07488).
 *
 * The calls follow the problem statement of the paper:
 *   1. build the network G = (N, E) in the box Omega, with a Dirichlet set
 *      N(Gamma) (Sec. 2.1; fiber generator of Sec. 6.1);
 *   2. assemble K on the free dofs, K u = f being the matrix form of
 *      (K u, v) = (f, v) for all v in V (eq. 3.1), for the heat model
 *      (Example 3.2, eq. 3.3) or the tensile truss model (Example 3.3, eq. 3.4);
 *   3. build the coarse space V_0 = V_H (Q1 on the mesh T_H restricted to the
 *      nodes, Sec. 2.3) and the local spaces V_j = V(U(y_j)) on mesh stars
 *      (Sec. 4.1);
 *   4. factor the local matrices and the coarse matrix P^T K P (the direct
 *      solves behind the projections P_j of eq. 4.1);
 *   5. solve K u = f with PCG on P = BK (Sec. 4.2) to a relative residual
 *      tolerance.
 *
 * Conventions
 *   - Every call returns an sn_status; SN_OK is 0, errors are negative. On error
 *     outputs are left untouched and sn_last_error() returns a message for the
 *     calling thread. No C++ exception crosses this boundary.
 *   - Handles are opaque and owned by the library; destroy them with the
 *     matching *_destroy call. A system keeps its network alive and a
 *     preconditioner keeps its system alive, so handles may be destroyed in any
 *     order.
 *   - Arrays passed in are copied. Export calls write into caller buffers whose
 *     sizes come from the matching *_info call.
 *   - Vectors of dofs are FP64, dof-major: dof d = free node index * ncomp +
 *     component; free nodes are numbered in ascending node id. With k
 *     right-hand sides a block is n x k row-major (the k values of a dof are
 *     adjacent).
 *   - Host or device pointers: solve-type calls take a flag; device pointers
 *     must be on the current HIP device and the work is queued on `stream`
 *     (a hipStream_t, NULL = the library's own stream). Calls are synchronous
 *     with respect to the host unless stated otherwise.
 *   - Device memory is allocated by the library with hipMalloc at factor time
 *     and at the first solve with a given k, and kept until destroy.
 */
#ifndef SPNET_H
#define SPNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SN_OK = 0,
  SN_EINVAL = -1,     /* bad argument or inconsistent sizes */
  SN_ENOMEM = -2,     /* host or device allocation failed */
  SN_EDEVICE = -3,    /* HIP runtime error or no usable gfx950 device */
  SN_ESINGULAR = -4,  /* no Dirichlet node: K is singular on V */
  SN_ENOTSPD = -5,    /* a local or the coarse matrix has a non-positive pivot */
  SN_ENOCONV = -6,    /* a column stopped before its true residual met the tolerance */
  SN_EBUSY = -7       /* serving: result not ready / no room */
} sn_status;

typedef struct sn_network_s *sn_network;
typedef struct sn_system_s *sn_system;
typedef struct sn_precond_s *sn_precond;
typedef struct sn_server_s *sn_server;

/*
 * Device allocator hook. Every device buffer the library keeps (matrix,
 * factors, coarse operator, engine vectors and slots, staging of host
 * arguments) is then taken from alloc(bytes, device, ctx) and given back
 * through free_(ptr, bytes, device, ctx), with `device` the HIP device that
 * is current during the call; this lets a caller put the library's memory in
 * its own pool (for example PyTorch's caching allocator). alloc must return
 * device memory on that device aligned to 256 bytes, or NULL, which the
 * calling function reports as SN_ENOMEM; a misaligned pointer is handed back
 * to free_ at once and reported as SN_EINVAL. Both callbacks may be called
 * from any thread that uses the library, the server's own thread included,
 * and must not call into the library. The hook is process-wide and applies to
 * allocations made after the call; every buffer is released through the pair
 * that allocated it, so the hook may change while handles live. alloc and
 * free_ both NULL restores hipMalloc / hipFree; exactly one NULL is SN_EINVAL.
 * Before free_ the library waits for the work queued on that device. Not
 * covered: pinned host staging, HIP graph and runtime internals, and the
 * fixed workspace of sn_apply_K_noalloc.
 */
typedef void *(*sn_alloc_fn)(size_t bytes, int device, void *ctx);
typedef void (*sn_free_fn)(void *ptr, size_t bytes, int device, void *ctx);
sn_status sn_set_allocator(sn_alloc_fn alloc, sn_free_fn free_, void *ctx);

/* Message of the last failing call on this thread (never NULL). */
const char *sn_last_error(void);
/* Library version string. */
const char *sn_version(void);

/* ------------------------------------------------------------------ */
/* 1. Network (Sec. 2.1; generator of Sec. 6.1)                        */
/* ------------------------------------------------------------------ */

/*
 * Build a fiber network in the unit box [0,1]^dim from raw straight segments.
 *   segments     n_segments x (2*dim) doubles: end points a then b.
 *   contact_eps  dim 3 only: two segments whose closest approach is below it
 *                are joined by one node at the midpoint of the closest points.
 *                In dim 2 nodes are placed at exact crossings.
 *   merge_tol    nodes closer than merge_tol are merged (Sec. 6.1 uses
 *                fiber length * 1e-4); segments clipped to less are dropped.
 *   dir_lo/hi    bit k: the face x_k = 0 (resp. 1) is part of Gamma.
 *   band         nodes within band of a Gamma face form N(Gamma).
 * The segments are clipped to the box, nodes are the clipped end points then the
 * crossings in lexicographic pair order, edges join consecutive nodes along each
 * segment, close nodes are merged (smallest id kept), and only the largest
 * connected component is kept (ties: the one with the smallest node id).
 * Errors: SN_EINVAL for dim not in {2,3}, non-positive merge_tol or contact_eps.
 */
sn_status sn_network_from_segments(int dim, int64_t n_segments, const double *segments,
                                   double contact_eps, double merge_tol, int dir_lo, int dir_hi,
                                   double band, sn_network *out);

/* A network given directly: coords n_nodes x dim, edges n_edges x 2 (int32
 * node ids), dirichlet n_nodes flags (1 = node in N(Gamma)). */
sn_status sn_network_from_arrays(int dim, int64_t n_nodes, const double *coords, int64_t n_edges,
                                 const int32_t *edges, const uint8_t *dirichlet, sn_network *out);

sn_status sn_network_info(sn_network net, int *dim, int64_t *n_nodes, int64_t *n_edges);
/* Any of the output pointers may be NULL. */
sn_status sn_network_export(sn_network net, double *coords, int32_t *edges, uint8_t *dirichlet);
void sn_network_destroy(sn_network net);

/*
 * Homogeneity and connectivity of the network (Assumption 3.4), the sigma and
 * mu of Tables 6.1 and 6.3 (Sec. 6.1, Sec. 6.2.1). Host computation.
 *   nb       [0,1]^dim is split into nb^dim boxes of side h = 1/nb (1..1024,
 *            at most 2^24 boxes), numbered lexicographically, axis 0 fastest.
 *   r0       the distance within which a disconnected box subgraph may be
 *            joined (Assumption 3.4.2); r0 <= 0 takes the longest edge.
 *   sigma    out: max / min over the boxes of the mass density, the lumped
 *            mass (M 1)(x) = 1/2 sum_{y~x} |x-y| (eq. 2.1) summed over the
 *            nodes of each half-open box (Sec. 2.3) and divided by h^dim
 *            (inf when a box holds no node).
 *   mu       out: max over the boxes of mu_box = 1 / (h sqrt(lambda_2)),
 *            lambda_2 the second eigenvalue of L u = lambda M u (L: the 1/|e|
 *            weighted Laplacian of eq. 2.2, M: the lumped mass of the
 *            subgraph's own edges) on the subgraph of every edge with an end
 *            point in the closed box; where that subgraph falls apart, a
 *            breadth-first search from the component of its smallest node id,
 *            through nodes within r0 of the box (adjacency in edge order),
 *            adds the edges of the first path that reaches another component,
 *            until it is connected. A box that cannot be joined gives inf, a box
 *            with no edge 0 (the bound of Lemma 3.5).
 *   density  optional (NULL), nb^dim doubles: the density of every box.
 *   mu_box   optional (NULL), nb^dim doubles: mu_box of every box.
 * Errors: SN_EINVAL for nb out of range or non-finite r0, SN_EINVAL when a
 * box's shifted Laplacian cannot be factored.
 */
sn_status sn_network_diagnostics(sn_network net, int nb, double r0, double *sigma, double *mu,
                                 double *density, double *mu_box);

/* ------------------------------------------------------------------ */
/* 2. Assembly (Examples 3.2 / 3.3)                                     */
/* ------------------------------------------------------------------ */
#define SN_MODEL_HEAT 0  /* scalar: each edge adds gamma/|e| (e_x-e_y)(e_x-e_y)^T, eq. 3.3 */
#define SN_MODEL_TRUSS 1 /* 3 dofs per node, dim 3: each edge adds (gamma/|e|) t t^T + (1e-6/|e|) I
                            in the xx, yy blocks and minus that in xy, yx (eq. 3.4) */
#define SN_MODEL_BEAM 2  /* tensile eq. 3.4 plus bending eq. 3.5: see sn_assemble_beam */

/* gamma: n_edges conductivities / stiffnesses, or NULL for all ones.
 * Errors: SN_ESINGULAR if the network has no Dirichlet node. */
sn_status sn_assemble(sn_network net, int model, const double *gamma, sn_system *out);

/*
 * Beam model (Example 3.3 with the constants of Sec. 6.3) with ncomp = 2
 * (in-plane displacements of a 2D network, Sec. 6.3.1) or 3 components (2D or
 * 3D network). With d_xy = (x - y)/|x - y|:
 *   tensile (eq. 3.4): each edge adds gamma1/|e| d d^T in the blocks xx, yy and
 *     minus it in xy, yx;
 *   bending (eq. 3.5): every centre x and ordered pair (y, z) of distinct
 *     neighbours adds w a_k^2 per term k, w = gamma1 r_w^2 / (4 (|x-y| +
 *     |x-z|)^2) * (|x-y| + |x-z|)/2, a_k = (v(y)-v(x)).eta_y^k/|x-y| +
 *     (v(z)-v(x)).eta_z^k/|x-z|; eta^1 (k = 1, three components only) is a unit
 *     normal of both edges (e_3 for a 2D network), eta_y^2 = d_xy x eta^1 and
 *     eta_z^2 = eta^1 x d_xz (the orientation for which a_2 is the change of the
 *     angle between the edges, so rigid motions carry no in-plane bending).
 * gamma1 = A E of the wire, wire_radius = r_w. A straight fiber then bends
 * like an Euler-Bernoulli beam of stiffness gamma1 r_w^2 / 8.
 * Errors: SN_EINVAL (ncomp, constants, ncomp = 2 on a 3D network),
 * SN_ESINGULAR if the network has no Dirichlet node.
 */
sn_status sn_assemble_beam(sn_network net, int ncomp, double gamma1, double wire_radius, sn_system *out);

/* y (n_dofs) = the free rows of K applied to g given on every node
 * (n_nodes x ncomp, node-major), Dirichlet nodes included: the term that a
 * non-zero Dirichlet lifting moves to the right-hand side (for u-hat = u + g
 * solve K u = f - y on V, Sec. 6.3). Host pointers. Errors: SN_EINVAL for a
 * non-finite g. */
sn_status sn_system_apply_full(sn_system sys, const double *g, double *y);
/* (M 1)(x) = 1/2 sum_{y~x} |x - y| at every free node (eq. 2.1), n_free_nodes entries */
sn_status sn_system_mass(sn_system sys, double *m);
sn_status sn_system_info(sn_system sys, int64_t *n_dofs, int64_t *nnz, int *ncomp, int64_t *n_free_nodes);
/* K in CSR over the free dofs: rowptr (n+1), col (nnz, ascending per row), val (nnz). */
sn_status sn_system_export_csr(sn_system sys, int64_t *rowptr, int32_t *col, double *val);
/* node id of every free node (n_free_nodes entries) */
sn_status sn_system_free_nodes(sn_system sys, int32_t *free_node);
void sn_system_destroy(sn_system sys);

/* ------------------------------------------------------------------ */
/* 3. Coarse and local spaces (Sec. 2.3, 4.1)                           */
/* ------------------------------------------------------------------ */
#define SN_STARS_ALL 0  /* one local space per mesh node y_j, j = 1..m (Sec. 4.1) */
#define SN_STARS_FREE 1 /* only mesh nodes off Gamma */

/*
 * nH = 1/H elements per axis. Element index of x: e_k = min(floor(x_k nH), nH-1)
 * (half-open boxes, closed at the upper face of Omega). Coarse dofs: mesh nodes
 * not on Gamma whose Q1 basis function is non-zero at some free node, in
 * lexicographic order (x fastest), times ncomp. Local space of mesh node v: the
 * free nodes at which its basis function is positive, |x_k nH - v_k| < 1 for all
 * k (the support of phi_v, which Sec. 5 identifies with the patch U(y_v); a node
 * on a face of T_H lies only in the stars of that face's mesh nodes), empty ones
 * dropped, in ascending mesh node order.
 * dir_lo/dir_hi give Gamma as in sn_network_from_segments.
 */
sn_status sn_precond_build(sn_system sys, int nH, int star_policy, int dir_lo, int dir_hi,
                           sn_precond *out);
sn_status sn_precond_info(sn_precond pre, int64_t *m0, int64_t *n_stars, int64_t *star_total);
/* star_ptr (n_stars+1), star_dofs (star_total, ascending per star), star_vertex (n_stars) */
sn_status sn_precond_export_stars(sn_precond pre, int64_t *star_ptr, int32_t *star_dofs,
                                  int32_t *star_vertex);
/* mesh node id of every coarse dof group (m0/ncomp entries) */
sn_status sn_precond_export_coarse(sn_precond pre, int32_t *coarse_vertex);

/* ------------------------------------------------------------------ */
/* 4. Factorisation (direct local and coarse solves, Sec. 4.1)          */
/* ------------------------------------------------------------------ */
#define SN_PREC_FP64 0              /* star factors, star solves and the coarse operator in FP64 */
#define SN_PREC_FP32_STARS 1        /* star factors stored and solved in FP32 with FP32 accumulation;
                                       the coarse operator, CG recurrences, residual replacement and
                                       dots stay FP64 (the mixed form) */
#define SN_PREC_FP32_STARS_COARSE 2 /* as SN_PREC_FP32_STARS, and the coarse inverse stored in FP32
                                       (its products accumulate in FP64) */

typedef struct {
  int64_t star_factor_nnz;   /* structural non-zeros of all local Cholesky factors (incl. the
                                diagonal) in minimum degree order (the supernodal layout) */
  int64_t star_rcm_nnz;      /* the same in reverse Cuthill-McKee order (the band layout) */
  int64_t star_envelope;     /* entries of the band layout's envelopes (incl. the diagonal) */
  int64_t star_stored;       /* entries the supernodal blocks store: the non-zeros plus the explicit
                                zeros of relaxed supernodes (L_CC^{-1} has the pattern of L_CC) */
  int64_t star_blob_bytes;   /* device bytes of the supernodal factors: index part and values */
  int64_t star_index_bytes;  /* of which the index part (headers, level tables, 16-bit lists) */
  int64_t star_stream_bytes; /* device bytes of the band layout's two sweep streams */
  int64_t coarse_bytes;      /* device bytes of the coarse operator */
  int64_t device_bytes;      /* all device memory held by the preconditioner */
  int32_t max_star_dofs;
  int32_t max_band;          /* widest envelope row/column of the band layout */
  int32_t max_levels;        /* most supernode levels of a star: a supernodal local solve runs
                                3 x levels - 1 dependent phases */
  int32_t pad0;
  double factor_seconds;     /* host time of ordering + numeric factorisation (both layouts) */
  int64_t sweep_bytes;       /* algorithmic bytes of one application of all local solves to one
                                column with every star on the band path (the supernodal path where
                                the band exceeds 1024): per star the structural non-zeros of its
                                factor in that path's order, twice for the band path (both sweeps
                                stream the factor) and once for the supernodal path (read once,
                                kept in LDS or cache), plus per position its dof index, the FP64
                                gather of r and the slot write; see sn_engine_info for the split
                                an engine runs */
  int64_t sweep_bytes_sn;    /* the same with every star the supernodal layout
                                holds on the supernodal path */
  int64_t spmv_bytes;        /* algorithmic bytes of one y = K x (values, columns, x, y) */
  int64_t sweep_flops;       /* 4 flops per structural non-zero of the minimum degree factors */
  double max_pivot_ratio;    /* max over stars and layouts of (largest / smallest Cholesky pivot),
                                a lower bound of cond(K_j) */
  int32_t star_precision;    /* precision the local solves run in: FP32 falls back to
                                SN_PREC_FP64 when max_pivot_ratio * 2^-24 > 0.05, i.e. when FP32
                                factors could not resolve the local solves */
  int32_t coarse_precision;  /* SN_PREC_FP64, or SN_PREC_FP32_STARS_COARSE when that was asked for,
                                the stars run in FP32 and coarse_pivot_ratio * 2^-24 <= 0.05 */
  double coarse_pivot_ratio; /* largest / smallest Cholesky pivot of K_0 */
} sn_factor_info;

/* Order, factor in FP64 on the host (threads over stars) and upload to the GPU.
 * precision is one of SN_PREC_* (the FP64 factor cast once). The local matrices are
 * ordered by minimum degree and factored in supernodes; see sn_factor_info.
 * Errors: SN_ENOTSPD naming the star, SN_EDEVICE, SN_ENOMEM. */
sn_status sn_precond_factor(sn_precond pre, int precision);
sn_status sn_precond_factor_info(sn_precond pre, sn_factor_info *info);
void sn_precond_destroy(sn_precond pre);

/* ------------------------------------------------------------------ */
/* 5. Solve (PCG on BK, Sec. 4.2)                                        */
/* ------------------------------------------------------------------ */
typedef struct {
  double rtol;           /* stop when ||r||_2 <= rtol ||f||_2 (per column, recurrence r) */
  int64_t max_iter;      /* default 1000 */
  int64_t fixed_iters;   /* > 0: run exactly this many iterations, ignore rtol */
  int64_t replace_every; /* > 0: r <- f - K u at the first convergence read-back
                            after every so many iterations (the queued blocks
                            between read-backs hold at most 4 check_every
                            iterations) */
  int32_t check_every;   /* iterations queued between convergence read-backs (default 8) */
  int32_t device_ptrs;   /* 1: f and u are device pointers */
  int32_t use_u0;        /* 1: u holds the initial guess u^(0), else u^(0) = 0 */
  int32_t use_graph;     /* 1: replay the iteration block as a captured HIP graph */
  void *stream;          /* hipStream_t or NULL */
} sn_solve_opts;

typedef struct {
  int64_t iters;   /* PCG iterations done */
  double res_rec;  /* ||r||_2 / ||f||_2 of the recurrence at exit */
  double res_true; /* ||f - K u||_2 / ||f||_2 recomputed in FP64 at exit */
  int32_t converged;  /* 1: res_rec and res_true both <= rtol (fixed_iters: the count was run) */
  int32_t replacements; /* residual replacements done */
  double ms;       /* wall time of the call */
} sn_solve_info;

/* Fill opts with defaults (rtol 1e-8, max_iter 1000, check_every 8). */
void sn_solve_opts_default(sn_solve_opts *opts);

/*
 * Solve K u = f for k right-hand sides (1 <= k <= 16): f and u are n x k
 * row-major. Each column runs its own PCG recurrence (alpha, beta per column);
 * columns share the matrix and factor reads. info has k entries.
 * Errors: SN_ENOCONV if some column stopped unconverged (max_iter reached, or its
 * FP64 true residual stays above rtol: the attainable accuracy of an
 * ill-conditioned system); u and info still hold the iterates and their state.
 */
sn_status sn_solve(sn_precond pre, int k, const double *f, double *u, const sn_solve_opts *opts,
                   sn_solve_info *info);

/* Kernel timing: while enabled, the local-solve launches of every B
 * application and the coarse product are bracketed by HIP events, and the
 * coarse solve runs before the local solves (not beside them) so that each is
 * timed alone. */
typedef struct {
  int64_t sweep_launches;  /* B applications timed */
  double sweep_ms;         /* summed device time of the local solves of those applications */
  int64_t iterations;      /* PCG iterations run while enabled */
  int64_t coarse_launches; /* coarse products timed */
  double coarse_ms;        /* their summed device time */
  int64_t coarse_flops;    /* flops of one coarse product per column (2 m0^2) */
} sn_kernel_stats;

/* enable = 1 starts (and resets) the recording, 0 stops it. */
sn_status sn_precond_profile(sn_precond pre, int enable);
/* Waits for recorded work and returns the totals since the last reset. */
sn_status sn_precond_kernel_stats(sn_precond pre, sn_kernel_stats *stats);

/*
 * Launch shape chosen for batches of k columns (measured on the device when
 * the preconditioner first solves with that batch width). The local solves
 * are split by size: the star_sn stars with the longest band sweeps (and any
 * star whose band exceeds 1024) run the supernodal kernel, the others the
 * band kernel, beside each other; every candidate split is timed.
 *   band path: at most star_waves_per_simd resident band wavefronts per SIMD
 *     (0 = no limit), working vectors in LDS (star_band_lds = 1) or in the
 *     slots;
 *   supernodal path: one star per workgroup of star_waves wavefronts, each
 *     carrying star_cols_per_wave of the k columns in turn; the workgroups of
 *     its main launch get star_lds_bytes of LDS, the star_big stars whose index
 *     part and vectors need more run with star_big_lds_bytes each, and the
 *     star_global stars that exceed the LDS of a compute unit are solved from
 *     global memory by workgroups of star_global_waves wavefronts;
 *   the band wavefronts of the longest stars may run at raised issue priority
 *     (star_band_prio).
 */
typedef struct {
  int32_t star_sn;
  int32_t star_waves_per_simd;
  int32_t star_band_lds;
  int32_t star_lds_bytes;
  int32_t star_cols_per_wave;
  int32_t star_waves;
  int32_t star_big;
  int32_t star_big_lds_bytes;
  int32_t star_global;
  int32_t star_band_prio; /* the band wavefronts of the star_band_prio longest stars of each band launch
                             run at raised instruction-issue priority (0: none) */
  int32_t star_global_waves; /* wavefronts per star of the star_global stars (4 or 16) */
  int32_t star_big_index_global; /* of the star_big stars, those whose vectors (or x and y alone) take the
                                    LDS, their index part, values (and update slots) read from global memory */
  int32_t star_twins;     /* band stars swept as two chains (sn_precond_set_band_twins) */
  int32_t coarse_first;  /* 1: the coarse solve runs before the local solves (and its restriction
                            also runs the convergence test), 0: beside them on a second stream */
  int32_t coarse_kernel; /* 0: the coarse product in 16-wavefront workgroups of 8 rows, 1: one
                            wavefront per 4 rows (the same results bit for bit), 2: the packed
                            symmetric kernel */
  int32_t coarse_late;   /* beside the local solves: 1 queued after them, 0 before */
  int32_t star_band_queue; /* > 0: the narrow band sweeps run as one persistent launch of that many
                              wavefronts taking the stars from a queue (sn_precond_set_band_queue) */
  int64_t sweep_bytes;   /* algorithmic bytes of one application of the local solves to one column
                            with this split (see sn_factor_info.sweep_bytes) */
  double star_sweep_us;  /* time of all local solves, microseconds per application of B */
  double b_apply_us;     /* time of the second half of an iteration (convergence test and B) */
} sn_engine_info;

sn_status sn_precond_engine_info(sn_precond pre, int k, sn_engine_info *info);

/*
 * The split of the local solves between the two kernels. By default it is
 * measured when the preconditioner first solves (the candidate that solves all
 * stars fastest) and then kept for every batch width, since the two kernels
 * round differently and a column's iterates must not depend on its batch.
 * n_sn >= 0 fixes it instead: of the n_sn stars with the most positions those
 * the supernodal layout holds (16-bit local indices: fewer than 65536
 * positions and update slots), and every star whose band exceeds 1024, run the
 * supernodal kernel, the others the band kernel; n_sn < 0 returns to
 * measuring. A star that fits neither layout fails the factorisation. Drops the preconditioner's
 * solve engines (the next solve creates them); engines a server already holds
 * keep their split until they are evicted. Errors: SN_EINVAL if not factored.
 */
sn_status sn_precond_set_star_split(sn_precond pre, int64_t n_sn);

/*
 * Where the supernodal stars whose index part and vectors together exceed the
 * LDS of a compute unit keep their data. mode = 0: everything in global memory
 * (star_global); mode = 1: the vectors in LDS and the index part and values
 * read from global memory wherever the vectors alone fit, else (workgroup
 * teams) x and y in LDS and the update slots in global memory
 * (star_big_index_global; the others stay in global memory); mode = -1 (default): both are measured
 * when an engine is created and the faster kept. Both give the same results
 * bit for bit. Drops the preconditioner's solve engines. Errors: SN_EINVAL if
 * not factored or mode outside -1..1.
 */
sn_status sn_precond_set_sn_beyond_lds(sn_precond pre, int mode);

/*
 * Persistent band sweeps: the band stars with windows of one or two registers
 * (the short ones) are swept by one launch of `waves` resident wavefronts,
 * each taking the next star of the length-sorted list (longest first) from a
 * queue in device memory until none is left, instead of one workgroup per
 * star. waves = 0: one workgroup per star; waves < 0 (default): measured when
 * an engine is created (one to six wavefronts per SIMD against one workgroup
 * per star, the fastest kept). Both forms sweep every star with the same
 * instructions, so the results are the same bit for bit. The queue belongs to
 * the engine, so launches of one engine must not overlap (as for all of its
 * buffers). Drops the preconditioner's solve engines. Errors: SN_EINVAL if not
 * factored.
 */
sn_status sn_precond_set_band_queue(sn_precond pre, int32_t waves);

/*
 * The two-chain form of the band sweeps for the longest stars. A star's RCM
 * order is cut into a top part, a separator (the positions coupled to the top
 * part) and a bottom part; one factor in the order (top, bottom, separator) is
 * swept as two chains by two wavefronts of one workgroup, (top, separator) and
 * (bottom reversed, separator), which meet at the separator, so a long star's
 * dependent chain is about half as long. Stars of at least 512 positions get
 * this factor when a cut saves a quarter of the steps without widening the
 * window. By default whether to use it, and from which star size on, is
 * measured when the preconditioner first solves and kept for every batch width
 * (it rounds differently); min_positions > 0 uses it for the stars of at least
 * that many positions, 0 never, -1 returns to measuring. Drops the
 * preconditioner's solve engines. Errors: SN_EINVAL if not factored.
 */
sn_status sn_precond_set_band_twins(sn_precond pre, int64_t min_positions);

/*
 * The coarse kernel and its placement beside the local solves (the product
 * c = K_0^-1 r_H, Sec. 4.1). By default the packed symmetric kernel runs and
 * its placement is measured when an engine is created. mode = kernel +
 * 2 placement fixes a dense kernel and its placement instead: kernel 0 runs
 * 16-wavefront workgroups of 8 rows, 1 one wavefront per 4 rows (every output
 * the same bit for bit); placement 0 runs the coarse solve before the local
 * solves, 1 beside them on a second stream queued before them, 2 queued after
 * them. mode = 6 + placement runs the packed symmetric kernel (the upper
 * triangle in 64 x 64 tiles, half the bytes; it rounds differently from the
 * dense kernels, so it is chosen per preconditioner, never per batch width).
 * mode = -1 returns to measuring. Drops the preconditioner's solve engines.
 * Errors: SN_EINVAL if not factored or mode outside -1..8.
 */
sn_status sn_precond_set_coarse_launch(sn_precond pre, int mode);

/* y = K x for k columns (n x k row-major). */
sn_status sn_apply_K(sn_precond pre, int k, const double *x, double *y, int device_ptrs, void *stream);
/*
 * y = K x as sn_apply_K with device pointers, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops): it calls
 * no allocation routine. Its staging vectors (x and y in the library's
 * internal dof order, 2 * npad * kc * 8 bytes, npad = n rounded up to 256,
 * kc = k rounded up to a power of two) live in a workspace of 64 MiB per GPU
 * that the library holds until the process ends; a larger need returns
 * SN_EINVAL. Every call on a GPU shares that workspace, so calls that overlap
 * on one GPU race. x and y are device pointers (n x k row-major) on the
 * preconditioner's device, which must be current; the work is queued on
 * `stream` (NULL: the default stream) and the call returns without waiting.
 */
sn_status sn_apply_K_noalloc(sn_precond pre, int k, const double *x, double *y, void *stream);
/* z = B r, B = P K_0^{-1} P^T + sum_j R_j^T K_j^{-1} R_j (so that BK = P_0 + ... + P_m). */
sn_status sn_apply_B(sn_precond pre, int k, const double *r, double *z, int device_ptrs, void *stream);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching of solves over device-resident factors  */
/* ------------------------------------------------------------------ */
/*
 * A server runs the PCG iterations of many requests together. Every
 * preconditioner with requests gets an engine: a batch of `max_columns` PCG
 * columns (one per right-hand side) whose iterations run as one launch
 * sequence on the engine's own stream, so that the engines of different
 * networks overlap on the device. A request occupies k columns of its
 * preconditioner's engine from admission until its last column converges;
 * columns are admitted and retired between ticks while the other columns keep
 * iterating (continuous batching). Every column runs its own recurrence with
 * the same arithmetic as sn_solve, so a result does not depend on the other
 * requests in the batch.
 *
 * Admission is by device-memory footprint: an engine costs its vectors and
 * star slots, a preconditioner the server factors costs its factors. When a
 * new engine does not fit in hbm_budget, idle engines are evicted (least
 * recently used first) together with the factors the server uploaded for
 * them. Unfactored preconditioners are factored on host worker threads while
 * other requests iterate. Either the caller steps the server (sn_server_step,
 * or sn_server_wait, which steps until a result is ready) or the server's own
 * host thread does (sn_server_run). Calls on one server are serialised by a
 * lock, so submit, poll and wait may come from several threads.
 */
typedef struct {
  int64_t hbm_budget;     /* bytes of device memory for engines and the factors the server uploads */
  int32_t max_columns;    /* engine width: 1, 2, 4, 8 or 16 (default 8); a request takes k <= this */
  int32_t iters_per_tick; /* PCG iterations queued per engine and tick (default 4) */
  int32_t precision;      /* precision of the factors the server computes (SN_PREC_*) */
  int32_t use_graph;      /* 1: replay iteration blocks as captured HIP graphs */
} sn_server_opts;

void sn_server_opts_default(sn_server_opts *opts);
sn_status sn_server_create(const sn_server_opts *opts, sn_server *out);
/*
 * Queue a solve of K u = f (k columns; f on the host, n x k row-major, copied)
 * with tolerance rtol and iteration limit max_iter per column. The
 * preconditioner may be factored or not (then the server factors it); the
 * server keeps it alive until the ticket is collected.
 * Errors: SN_EINVAL (k out of range, non-finite f), SN_EBUSY if the request
 * alone exceeds the budget.
 */
sn_status sn_server_submit(sn_server srv, sn_precond pre, int k, const double *f, double rtol,
                           int64_t max_iter, uint64_t *ticket);
/*
 * One scheduling step: retire the converged columns of every engine whose
 * last tick has completed (waiting for the first one if none has), admit
 * queued requests into idle engines that have room, and queue the next
 * iterations of every idle engine with running columns (asynchronously).
 * Engines advance independently. n_active: requests iterating, n_queued:
 * requests waiting.
 */
sn_status sn_server_step(sn_server srv, int32_t *n_active, int32_t *n_queued);
/* SN_EBUSY while pending; when done copies u (n x k) and k info entries and
 * forgets the ticket. With u and info both NULL it only reports the status
 * (SN_OK when done) and keeps the result. A request that failed returns its
 * error once. */
sn_status sn_server_poll(sn_server srv, uint64_t ticket, double *u, sn_solve_info *info);
/*
 * enable = 1: start the server's own host thread, which steps the server
 * (without blocking between steps) while requests are queued or iterating
 * and sleeps otherwise; the HIP device current in the calling thread is made
 * current in it. enable = 0: stop and join it (iterations already queued stay
 * queued; later steps continue them). While the thread runs, sn_server_step
 * returns SN_EBUSY. If the thread meets a device error it fails every pending
 * request with that error and stops; later submissions return it.
 */
sn_status sn_server_run(sn_server srv, int enable);
/*
 * Wait until request `ticket` is done or has failed (ticket = 0: until some
 * request is, whose result has not been collected yet), at most timeout_s
 * seconds; the result stays for sn_server_poll. Without the server's thread
 * the calling thread steps the server meanwhile. SN_OK when a result is
 * ready, SN_EBUSY on timeout (or when nothing is pending), SN_EINVAL for an
 * unknown ticket.
 */
sn_status sn_server_wait(sn_server srv, uint64_t ticket, double timeout_s);
/* Device bytes the server holds (engines and the factors it uploaded). */
sn_status sn_server_usage(sn_server srv, int64_t *device_bytes, int32_t *n_engines);
void sn_server_destroy(sn_server srv);

#ifdef __cplusplus
}
#endif
#endif /* SPNET_H */
