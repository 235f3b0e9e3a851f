/*
 * c0ip.h - C ABI of libc0ip: the C0 interior-penalty (C0IP) biharmonic
 * operator, the additive vertex-patch Schwarz smoother with fast-
 * diagonalisation local solvers, the geometric multigrid V-cycle and the
 * multigrid-preconditioned flexible GMRES solve, on one MI355X (gfx950).
 *
 * Problem (Sec. 2): Delta^2 u = f on [0,1]^d (d = 2, 3), clamped boundary
 * (u = d_n u = 0), continuous Q_k Lagrange elements (Gauss-Lobatto nodes)
 * on the uniform Cartesian mesh of N^d cells, discretised by the C0IP form
 * of eq. bfc0ip with penalty gamma / h on every face.
 *
 * Vectors.  Every vector argument is a caller-owned, contiguous DEVICE
 * buffer of num_dofs(level) = (k N_l + 1)^d entries in lexicographic node
 * order (x fastest), boundary nodes included.  Boundary entries of inputs
 * are ignored (treated as 0); boundary entries of outputs are written as 0.
 * Element type is given by the c0ip_dtype argument (double or float).
 *
 * Levels.  Level l = 0..L has N_l = 2^(l+1) cells per direction (level 0:
 * 2^d cells, one vertex patch); level L (= -1 in arguments) is the finest.
 *
 * Streams.  All device work of a handle is enqueued on the HIP stream given
 * at creation (NULL = the default stream).  c0ip_apply_A,
 * c0ip_apply_smoother and c0ip_vcycle are asynchronous; c0ip_solve
 * synchronises the stream.  A handle must not be used from two host
 * threads at once; calls on one handle are ordered by its stream.
 *
 * Errors.  Every call returns a c0ip_status; nothing aborts or throws
 * across the ABI.  c0ip_last_error() describes the last failure of the
 * calling thread.
 */
#ifndef C0IP_H
#define C0IP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  C0IP_OK = 0,
  C0IP_EINVAL = -1,          /* invalid argument (dimension, degree, size, pointer, level, option) */
  C0IP_ENOMEM = -2,          /* device or host allocation failed */
  C0IP_EHIP = -3,            /* a HIP runtime call or kernel launch failed (message in last_error) */
  C0IP_NOT_CONVERGED = -4,   /* solve stopped at max_iters; x holds the last iterate, info is filled */
  C0IP_ENAN = -5,            /* a non-finite value appeared in the Krylov iteration */
  C0IP_EUNSUPPORTED = -6     /* valid request this build does not provide */
} c0ip_status;

typedef enum { C0IP_F64 = 0, C0IP_F32 = 1 } c0ip_dtype;

typedef struct c0ip_problem c0ip_problem; /* opaque; owned by the library */

/* Mesh and discretisation (Sec. 2): dim in {2,3}; n_cells = N, a power of
 * two >= 2; degree = k in [2,7]; gamma = penalty constant (<= 0 selects
 * k(k+1)), applied as gamma / h on interior and boundary faces. */
typedef struct {
  int dim;
  int n_cells;
  int degree;
  double gamma;
} c0ip_mesh_desc;

/* Multigrid options (Sec. 3, Algorithm 1).
 * omega: damping of the additive smoother (> 0; the paper uses 1/4 in 2D
 *   and 0.1 in 3D; the overlap bounds it by 2^-d).
 * pre_steps, post_steps: smoothing steps per level (>= 0).
 * vcycle_dtype: precision of the V-cycle inside c0ip_solve (the coarse
 *   solve is always float64).
 * coarse_mode: 0 = exact level-0 solve (float64 dense inverse from a
 *   Cholesky factorisation); 1 = one smoothing step with omega = 1.
 * scatter_mode: how a smoothing step adds the overlapping patch corrections
 *   (Sec. 3; the paper compares coloured and atomic scatters).  0 = owner
 *   computes: each tile solves every patch touching it and writes each of
 *   its DoFs once (deterministic, no atomics).  1 = atomic: each patch is
 *   solved once and its correction added with floating-point atomics
 *   (results agree to rounding, not bit for bit; 2D only, else
 *   C0IP_EUNSUPPORTED; batched solves accept 0 only).  Other values:
 *   C0IP_EINVAL.
 * tail_levels: in 2D with degree <= 4, the lowest levels of the V-cycle can
 *   run as one launch of a single workgroup per system, all their vectors
 *   in LDS (same operations, fewer launches).  -1 = as many levels as fit
 *   in LDS; 0 = none (every level on the tiled kernels); m > 0 = at most
 *   levels 0..m-1.  Ignored in 3D and for degree > 4.
 * smoother: 0 = additive vertex-patch Schwarz (AVS); 1 = coloured
 *   multiplicative vertex-patch Schwarz (MVS, Sec. 3 and Fig. 2): the
 *   vertices are split into colours (2^d vertex-parity classes, each split
 *   red-black), patches of one colour share no node and no entry of A
 *   couples them; a step visits the colours in order c = 0, 1, ... and for
 *   each forms the residual of the current iterate and adds omega times the
 *   local solves of that colour's patches (the paper uses omega = 1 in 2D
 *   and 0.7 in 3D).  2^(d+1) colours: 8 in 2D, 16 in 3D.  Colour of vertex
 *   v: sum_m (v_m mod 2) 2^m + 2^d ((sum_m floor(v_m / 2)) mod 2).  MVS
 *   needs scatter_mode 0 (C0IP_EINVAL otherwise); batched solves use the
 *   additive smoother only (C0IP_EUNSUPPORTED).  Other values: C0IP_EINVAL.
 * local_solver: 0 = the separable local matrix A~_v of eq. localsolverbila
 *   inverted by fast diagonalisation (eq. inverse); 1 = the exact local
 *   matrix A_v = R_v A R_v^T (mixed second derivatives kept; the comparison
 *   of the paper's Tables 1 and 2), inverted densely at set-up (one inverse
 *   per patch boundary type, float64 Cholesky, rounded for float32) and
 *   applied as a dense product.  1 is built for 2D meshes with scatter_mode
 *   0 (C0IP_EUNSUPPORTED otherwise, and for batched solves).  Other values:
 *   C0IP_EINVAL.
 * mvs_residual: where a 2D multiplicative step forms each colour's
 *   residual b - A x.  1 = in the colour's own launch, on its patches'
 *   rows only (x staged in LDS around each patch); 2 = a full residual pass
 *   with the tiled operator before each colour's solves; 0 = automatic (1 on
 *   levels under 1.5 * 2^20 DoFs, where launches dominate, 2 on finer
 *   ones).  The modes form the same sums and agree to rounding.  Ignored
 *   in 3D (always 2) and by the additive smoother; batched solves take 0
 *   only.  Other values: C0IP_EINVAL. */
typedef struct {
  double omega;
  int pre_steps, post_steps;
  c0ip_dtype vcycle_dtype;
  int coarse_mode;
  int scatter_mode;
  int tail_levels;
  int smoother;
  int local_solver;
  int mvs_residual;
} c0ip_mg_opts;

/* Flexible GMRES options (Sec. 5.1: relative residual reduction 1e-8).
 * rtol: stop when the Arnoldi residual estimate <= rtol * ||b||_2.
 * max_iters: total iteration cap (>= 1).  restart: Krylov dimension m in
 * [1, 64].  x0_is_zero: 1 = start from 0 (x is output only), 0 = start
 * from the x passed in. */
typedef struct {
  double rtol;
  int max_iters;
  int restart;
  int x0_is_zero;
} c0ip_krylov_opts;

typedef struct {
  int iterations;      /* Arnoldi steps taken */
  int converged;       /* 1 if the estimate met rtol */
  double rel_res_est;  /* final Arnoldi estimate / ||b|| */
  double rel_res_true; /* ||b - A x|| / ||b|| recomputed in float64 */
  double frac_iters;   /* 8 n / (-log10(rel_res_est)) (Sec. 5.1) */
  /* wall time of the solve; time in the V-cycles (events on every 8th
   * iteration, scaled to all iterations); the rest (A z, the Krylov vector
   * passes and reductions, the host's Hessenberg work, restarts) */
  double seconds_total, seconds_vcycle, seconds_arnoldi;
} c0ip_solve_info;

/* Create a problem: level hierarchy, 1D matrices, patch eigenbases, coarse
 * inverse, device tables and work space (Sec. 3-4).  opts may be NULL
 * (omega 1/4 in 2D and 0.1 in 3D, 1 pre- and 1 post-step, float32
 * V-cycle, exact coarse solve, tail_levels -1, additive smoother with the
 * separable local solver).  hip_stream is a hipStream_t or NULL.
 * Meshes whose vectors would hold 2^31 or more DoFs ((k N + 1)^d) are
 * rejected with C0IP_EINVAL before any device call (the kernels index a
 * vector's entries with 32-bit integers in places; at that size a float64
 * Krylov basis would not fit in HBM anyway).
 * On success *out owns all device memory it allocated. */
c0ip_status c0ip_create(const c0ip_mesh_desc* mesh, const c0ip_mg_opts* opts, void* hip_stream,
                        c0ip_problem** out);
/* Free the problem and every device allocation it owns (NULL is a no-op). */
c0ip_status c0ip_destroy(c0ip_problem* p);

/* Number of levels L+1, and DoFs of a level (level -1 = finest). */
c0ip_status c0ip_num_levels(const c0ip_problem* p, int* n_levels);
c0ip_status c0ip_num_dofs(const c0ip_problem* p, int level, int64_t* n_total);

/* y = A_l x: the C0IP matrix of eq. bfc0ip on level l, applied matrix-free
 * through its Kronecker form (Sec. 4, eqs. c0iptensorvp / c0iptensorvp3D).
 * x and y must not overlap (no shared byte; else C0IP_EINVAL). */
c0ip_status c0ip_apply_A(c0ip_problem* p, int level, c0ip_dtype dtype, const void* x, void* y);

/* One step of the handle's vertex-patch smoother (Sec. 3).  Additive:
 *   x <- x + omega * sum_v R_v^T A~_v^{-1} R_v (b - A_l x),
 * with A~_v the separable local matrix of eq. localsolverbila inverted by
 * fast diagonalisation (eq. inverse); coloured multiplicative: the same
 * update restricted to one colour's patches, colour after colour, each
 * with the residual of the current iterate.  x_is_zero = 1 treats x as 0
 * on input (x is output only).  b and x must not overlap. */
c0ip_status c0ip_apply_smoother(c0ip_problem* p, int level, c0ip_dtype dtype, const void* b, void* x,
                                int x_is_zero);

/* Out-of-place form of one smoother step: x_out = S(x_in, b), or S(0, b)
 * when x_in is NULL.  x_out must not overlap b or x_in (in 2D the step
 * is one fused launch that reads x_in around every tile it writes). */
c0ip_status c0ip_smoother_step(c0ip_problem* p, int level, c0ip_dtype dtype, const void* b, const void* x_in,
                               void* x_out);

/* The step of c0ip_smoother_step for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, same kernels and result, and no
 * allocation of any kind during the call.  Where the step needs a residual
 * buffer (3D meshes, and scatter_mode 1, when x_in != NULL) it uses a fixed
 * work space of 64 MiB compiled into the library, one copy per GPU (held
 * until the process ends), instead of the handle's: a level whose residual
 * needs more (num_dofs x element size > 64 MiB) is rejected with
 * C0IP_EINVAL.  A float32 call needs the handle's float32 tables (created
 * with vcycle_dtype = C0IP_F32, or set up by an earlier float32 call of
 * another entry point), else C0IP_EINVAL.  All calls on one GPU share that
 * work space and it keeps the last call's contents: calls that overlap in
 * time on one GPU (several streams, handles or threads) race. */
c0ip_status c0ip_smoother_step_noalloc(c0ip_problem* p, int level, c0ip_dtype dtype, const void* b,
                                       const void* x_in, void* x_out);

/* Autotuner: for every level (and each precision the handle has set up),
 * time each compiled tile-size variant of the 2D fused smoother kernel
 * (reps launches after one warm-up, on the handle's stream and work space)
 * and keep the fastest for all later smoother steps of that level.
 * Synchronises the stream; no-op in 3D.  reps < 1 selects 3. */
c0ip_status c0ip_autotune(c0ip_problem* p, int reps);
/* The tile variant the autotuner chose for a level (0 = default), and a
 * manual override (EINVAL for a variant this degree was not compiled for). */
c0ip_status c0ip_tuned_variant(const c0ip_problem* p, int level, c0ip_dtype dtype, int* variant);
c0ip_status c0ip_set_variant(c0ip_problem* p, int level, c0ip_dtype dtype, int variant);

/* x = MG_L(0, b): one V-cycle of Algorithm 1 on the finest level in the
 * given precision (coarse solve in float64), with the options' pre/post
 * steps and damping. */
c0ip_status c0ip_vcycle(c0ip_problem* p, c0ip_dtype dtype, const void* b, void* x);

/* Solve A_L x = b by flexible GMRES in float64 right-preconditioned by one
 * V-cycle (precision opts.vcycle_dtype) per iteration (Sec. 5.1, 5.2).
 * b, x: float64 device vectors of the finest level.  info may be NULL.
 * Returns C0IP_NOT_CONVERGED (x = last iterate) if max_iters is reached. */
c0ip_status c0ip_solve(c0ip_problem* p, const c0ip_krylov_opts* opts, const double* b, double* x,
                       c0ip_solve_info* info);

/* Solve A_L x = b by flexible conjugate gradients in float64, preconditioned
 * by one V-cycle (precision opts.vcycle_dtype) per iteration: the paper's
 * Krylov method for the symmetric additive smoother (Sec. 5.1).  One
 * retained direction: z = MG(r), p = z - ((z . q_old) / (p_old . q_old))
 * p_old (p = z at the first iteration), q = A p, alpha = (r . p) / (p . q),
 * x += alpha p, r -= alpha q; the flexible form tolerates a preconditioner
 * that is symmetric only up to rounding (the float32 V-cycle).  Stops when
 * the recursive residual ||r||_2 <= rtol ||b||_2; opts->restart is not
 * used.  info (may be NULL): iterations, rel_res_est = ||r|| / ||b||,
 * rel_res_true = ||b - A x|| / ||b|| recomputed, frac_iters from the
 * reduction ||r_n|| / ||r_0||, seconds_arnoldi = time outside the V-cycles.
 * b, x: float64 device vectors of the finest level.  Returns
 * C0IP_NOT_CONVERGED (x = last iterate) if max_iters is reached, C0IP_ENAN
 * on a non-finite value (an indefinite preconditioner shows as one). */
c0ip_status c0ip_solve_fcg(c0ip_problem* p, const c0ip_krylov_opts* opts, const double* b, double* x,
                           c0ip_solve_info* info);

/* ---- batched solves (many independent 2D systems, one graph per round) ----
 * A batch holds n_problems 2D problems (meshes[i]: any n_cells and degree)
 * with n_rhs[i] right-hand sides each; every (problem, right-hand side) is
 * one system solved by its own float64 FGMRES with the V-cycle of opts
 * (shared damping, steps and precision).  Systems of equal degree and
 * penalty share every V-cycle launch of a level (all their meshes have
 * 2^(l+1) cells there), the Krylov kernels take per-system descriptors, and
 * each round -- one Arnoldi step of every active system, ending in its
 * Givens step on the device -- is a single replay of a captured HIP graph.
 * The device keeps every system's Krylov state: it advances a system, or
 * stops it (converged, basis full, max_iters) and masks it off; rounds are
 * queued back to back, and the host reads each round's state two rounds
 * later, queueing x += Z y and the restart of a stopped system behind the
 * rounds in flight.  dim must be 2 (C0IP_EUNSUPPORTED otherwise).
 * hip_stream: the caller's stream (NULL = default); the batch orders its
 * work after it. */
typedef struct c0ip_batch c0ip_batch; /* opaque; owned by the library */
c0ip_status c0ip_batch_create(const c0ip_mesh_desc* meshes, const int* n_rhs, int n_problems,
                              const c0ip_mg_opts* opts, void* hip_stream, c0ip_batch** out);
/* Number of systems (sum of n_rhs). */
c0ip_status c0ip_batch_num_systems(const c0ip_batch* batch, int* n_systems);
/* Solve every system.  b, x: HOST arrays of n_problems DEVICE pointers;
 * b[i] (x[i]) holds problem i's n_rhs[i] float64 vectors back to back, each
 * of num_dofs entries.  infos: NULL or an array of n_systems entries, in
 * problem order then right-hand-side order.  Synchronous.  Returns
 * C0IP_NOT_CONVERGED if any system reached max_iters (its x = last
 * iterate), C0IP_ENAN if any system met a non-finite value. */
c0ip_status c0ip_batch_solve(c0ip_batch* batch, const c0ip_krylov_opts* opts, const double* const* b,
                             double* const* x, c0ip_solve_info* infos);
c0ip_status c0ip_batch_destroy(c0ip_batch* batch);

/* Description of the last error on the calling thread ("" if none). */
const char* c0ip_last_error(void);

/* ---- host-only set-up inspection (no device needed) ----
 * The library's 1D factors of the level with n_cells = N (Sec. 4, eqs.
 * matrix1d, bulk1-bulk3, ev): dense (kN+1)^2 row-major host arrays M, L,
 * B, boundary rows and columns zero.  gamma <= 0 selects k(k+1). */
c0ip_status c0ip_host_matrices_1d(int degree, int n_cells, double gamma, double* M, double* L, double* B);
/* The fast-diagonalisation inverse (eq. inverse) of the separable patch
 * matrix of eq. localsolverbila for the vertex with multi-index
 * vertex[0..dim-1] in [1, N-1], as a dense host array of (2k-1)^(2 dim)
 * row-major entries (patch DoFs in lexicographic order, x fastest). */
c0ip_status c0ip_host_patch_inverse(int dim, int degree, int n_cells, double gamma, const int* vertex,
                                    double* Ainv);
/* The inverse of the exact local matrix A_v = R_v A R_v^T (the restriction
 * of the operator of eq. bfc0ip to the patch's interior nodes, by its
 * Kronecker form) used by local_solver 1: same layout as above. */
c0ip_status c0ip_host_patch_inverse_exact(int dim, int degree, int n_cells, double gamma, const int* vertex,
                                          double* Ainv);

#ifdef __cplusplus
}
#endif

#endif /* C0IP_H */
