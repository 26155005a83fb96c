/*
 * grouped.h - C ABI of the MI355X (gfx950) grouped Fourier transform library.
 *
 * The operation (Bartel, Potts, Schmischke, "Grouped Transformations and Regularization
 * in High-Dimensional Explainable ANOVA Approximation"):
 *
 *   forward  f_x   = sum_{u in U} sum_{k in I_{N_u}^{u,d}} fhat_k e^{2 pi i <k, x>}
 *                    (Sec. 3, Definition def:skatoons), computed per term as a
 *                    |u|-dimensional nonequispaced FFT of the projected nodes x_u
 *                    (eq. somafm and the sum after it);
 *   adjoint  fhat_u = F(X_u, I_{N_u}^{|u|})^H y, stacked over u (Sec. 3, adjoint display);
 *   LSQR     min 1/2 ||y - F fhat||^2 + lambda ||fhat||_W^2        (Sec. 4.1, eq. new_min_prob);
 *   FISTA    min 1/2 ||y - F fhat||^2 + lambda sum_u ||fhat_u||_W  (Sec. 4.2, eq. alligatoah,
 *            Algorithm algo:fista, Theorem theorem:projection).
 *
 * U = U_{d_s} = {u subset {0..d-1} : |u| <= d_s} (eq. pizmosch), N_u = N[|u|-1] (one even
 * bandwidth per order), I_N = {-N/2, ..., N/2-1} (eq. metallica).
 *
 * Coefficient order (the paper leaves it open, Sec. 3 before eq. bananarama): terms by order
 * |u|, then lexicographically by the sorted coordinate tuple, the empty set first; inside a
 * group the reduced frequency l = k_u runs row-major over (I_N minus {0})^{|u|}, last
 * coordinate fastest, each ascending -N/2..-1, 1..N/2-1.  gt_term_table() exports it.
 *
 * Conventions for every entry point:
 *  - Pointers named "device" are device memory of the current HIP device; "host" pointers are
 *    ordinary host memory.  The library never frees, retains or writes caller memory other
 *    than the documented outputs, and never keeps a caller pointer past the call (a plan keeps
 *    its own copy of the nodes).
 *  - Complex arrays are interleaved (re, im): float2 for GT_C64, double2 for GT_C128, which is
 *    the memory layout of torch.complex64 / torch.complex128.  Real arrays use the matching
 *    real type (float / double).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream) and is
 *    asynchronous unless stated otherwise.  Plan creation and the solvers synchronise the
 *    stream where documented.
 *  - Return value: GT_OK (0) or a negative gt_status.  Nothing aborts or throws across the
 *    ABI.  gt_last_error() returns a thread-local description of the last failure.
 *  - Nodes may be any finite reals; each coordinate is reduced modulo 1 into [-1/2, 1/2)
 *    (the torus T = R/Z, Sec. 2).  NaN or Inf nodes give GT_EINVAL.
 */
#ifndef GROUPED_H
#define GROUPED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GT_OK = 0,
  GT_EINVAL = -1,        /* invalid argument (message in gt_last_error) */
  GT_ENOMEM = -2,        /* device or host allocation failed */
  GT_EHIP = -3,          /* a HIP runtime call failed */
  GT_EUNSUPPORTED = -4   /* valid but outside what this library implements (e.g. d_s > 3) */
} gt_status;

enum { GT_C64 = 1, GT_C128 = 2 };   /* complex float (FP32 path) / complex double (FP64 path) */

/* Basis of the grouped transform (gt_problem.basis).
 *   GT_BASIS_EXP: e^{2 pi i <k, x>} on the torus, groups of k_j in I_N minus {0} (Sec. 2-3).
 *   GT_BASIS_COS: the half-period cosine basis on [0, 1]^d of the paper's non-periodic
 *     variant (Sec. 5; the extension remark after the adjoint display in Sec. 3):
 *     phi_k(x) = sqrt(2)^{|supp k|} prod_j cos(pi k_j x_j), groups {k : supp k = u,
 *     1 <= k_j <= N_u - 1}, the same sizes (N_u - 1)^{|u|} and the same order (k_j ascending
 *     1..N-1 inside a group, last coordinate fastest); the empty set holds k = 0 (phi_0 = 1).
 *     Nodes are meant in [0, 1]^d; any finite node is taken through the even, 2-periodic
 *     extension of the basis.  Bandwidths up to 2048.  Every entry point accepts either
 *     basis; the solvers and sensitivity indices apply unchanged (the basis is orthonormal). */
enum { GT_BASIS_EXP = 0, GT_BASIS_COS = 1 };
enum { GT_MAX_ORDER = 3 };          /* largest |u| the GPU path implements */

/* Problem description (Sec. 2-4).  Plain data; copied by every call. */
typedef struct gt_problem {
  int32_t d;                   /* spatial dimension, >= 1 */
  int32_t ds;                  /* superposition threshold, 0 <= ds <= min(d, 3) */
  int32_t N[GT_MAX_ORDER];     /* N[k-1]: even bandwidth >= 2 of every term with |u| = k; unused entries ignored */
  int64_t M;                   /* nodes (shared by all R right-hand sides), >= 1; ignored when offsets != NULL */
  int32_t R;                   /* batch: right-hand sides (lambda values) or ragged datasets, >= 1 */
  const int64_t *offsets;      /* host, NULL or R+1 non-decreasing prefix offsets starting at 0: dataset b owns
                                  nodes offsets[b]..offsets[b+1]-1 of the node array and has its own coefficients;
                                  a dataset may be empty, the total may not */
  int32_t dtype;               /* GT_C64 or GT_C128 */
  int32_t m;                   /* window half-width (Kaiser-Bessel support 2m grid points), 0 = chosen per order
                                  from the precision; otherwise 2..8 */
  double sigma;                /* oversampling factor n/N >= 1.5 of the FFT grids, 0 = 2.0 */
  const uint8_t *term_mask;    /* host, NULL (all of U_{d_s}) or gt_num_terms(d, ds) flags in the coefficient
                                  order of the unmasked index set: 0 drops the term, whose coefficients are then
                                  absent from every coefficient vector (an index set I_N(U) for a subset U, as the
                                  refit on an active set uses, eq. activeset); the empty set is always kept */
  int32_t basis;               /* GT_BASIS_EXP (0) or GT_BASIS_COS */
} gt_problem;

/* Solver report, one entry per right-hand side. */
typedef struct gt_solve_info {
  int32_t iters;               /* iterations done */
  int32_t flags;               /* GT_SOLVE_* bits */
  double resid;                /* LSQR: estimate of ||F^H(y - F fhat) - 2 lambda W fhat|| (normal equations);
                                  FISTA: relative change ||f_k - f_{k-1}|| / ||f_k|| of the last step */
  double t_k;                  /* FISTA momentum scalar t_{K+1} (resume); LSQR: phibar */
  double L;                    /* FISTA step constant used last (after backtracking); LSQR: 0 */
} gt_solve_info;

enum {
  GT_SOLVE_CONVERGED = 1,      /* tolerance reached */
  GT_SOLVE_MAX_ITER = 2,       /* stopped at max_iter */
  GT_SOLVE_BREAKDOWN = 4,      /* LSQR: alpha or beta became 0 (exact solution in the Krylov space) */
  GT_SOLVE_BACKTRACK_CAP = 8   /* FISTA: a step hit the backtracking cap (30 increases of L) */
};

typedef struct gt_plan gt_plan;   /* opaque */

/* ------------------------------------------------------------------ index set
 * |U_{d_s}| = sum_{t<=ds} C(d, t) (eq. pizmosch).  Returns -1 on invalid d, ds. */
int64_t gt_num_terms(int32_t d, int32_t ds);

/* |I_N(U_{d_s})| = 1 + sum_{t=1..ds} C(d,t) (N[t-1]-1)^t (Remark rem:cardinality, eq. groupedset).
 * N: host, ds entries.  Returns -1 on invalid arguments. */
int64_t gt_num_coeffs(int32_t d, int32_t ds, const int32_t *N);

/* Term table in coefficient order.  coords: host, |U| x 3 int32, coordinates of each term
 * ascending, -1 padded; offsets: host, |U|+1 coefficient offsets.  Either may be NULL.
 * With a term mask, only the kept terms (|U| = gt_problem_size's nterms). */
int gt_term_table(const gt_problem *p, int32_t *coords, int64_t *offsets);

/* Terms |U| and coefficients |I_N(U)| = 1 + sum over u != empty set of (N_{|u|} - 1)^{|u|}
 * (Remark rem:cardinality, eq. groupedset) of the problem's index set, its term mask
 * applied.  nterms, ncoeffs: host, either may be NULL.  Returns GT_EINVAL for invalid d, ds
 * or bandwidths. */
int gt_problem_size(const gt_problem *p, int64_t *nterms, int64_t *ncoeffs);

/* ------------------------------------------------------------------ one-shot transforms
 * Each call builds a plan for (p, x), runs it on `stream`, synchronises `stream` and
 * releases the plan before returning (so these calls are synchronous).
 *
 * grouped_trafo   (Definition def:skatoons via eq. somafm):  f = F fhat.
 *   x    device, real, Mtot x d row-major (Mtot = M, or offsets[R] when ragged)
 *   fhat device, complex, R x |I|
 *   f    device, complex, R x M (shared nodes) or Mtot (ragged, dataset b at offsets[b])
 * grouped_adjoint (Sec. 3, adjoint display):  fhat = F^H y, same layouts with roles swapped. */
int grouped_trafo(const gt_problem *p, const void *x, const void *fhat, void *f, void *stream);
int grouped_adjoint(const gt_problem *p, const void *x, const void *y, void *fhat, void *stream);

/* ------------------------------------------------------------------ plans
 * A plan holds the index set, FFT grid sizes, window and deconvolution tables, the wrapped
 * nodes (its own copy, transposed), the work lists and all scratch memory for (p, x).
 * Creation synchronises `stream` once (to validate the nodes).  A plan may be used from one
 * stream at a time; calls on the same plan must not overlap. */
int gt_plan_create(const gt_problem *p, const void *x, void *stream, gt_plan **out);
int gt_plan_destroy(gt_plan *plan);            /* synchronises the plan's last stream; NULL is a no-op;
                                                  a handle that is not a live plan gives GT_EINVAL */
int gt_plan_trafo(gt_plan *plan, const void *fhat, void *f, void *stream);
int gt_plan_adjoint(gt_plan *plan, const void *y, void *fhat, void *stream);

/* Node gradient for reverse-mode differentiation (not in the paper; derivative of
 * Definition def:skatoons).  With upstream gradient g = dL/d(conj f) (complex, layout of f)
 * it writes gx[v][j] = Re( conj(d f_v / d x_{v,j}) * g_v ), real, Mtot x d row-major
 * (per right-hand side summed over the R right-hand sides when nodes are shared). */
int gt_plan_node_grad(gt_plan *plan, const void *fhat, const void *g, void *gx, void *stream);

/* Window half-width m and FFT grid size n chosen for order t (1..ds); for reports. */
int gt_plan_order_info(const gt_plan *plan, int32_t t, int32_t *m, int32_t *n);

/* Which forward form the plan uses for order t (1..ds); for reports and tests.  The first
 * three compute the window sum of Definition def:skatoons via eq. somafm for every node of
 * every term of the order; the fourth the defining sum itself:
 *   GT_GATHER_SORTED  runs of cell-sorted nodes, the term's grid staged in LDS;
 *   GT_GATHER_CELL    one wavefront per run of <= 64 nodes of one grid cell, the grid block as
 *                     scalar operands (when the cells hold enough nodes);
 *   GT_GATHER_POLY    order 2, FP32: per-cell coefficients of the window polynomials (built by
 *                     the forward pack), evaluated per node by Horner sums;
 *   GT_GATHER_DIRECT  no window and no grid: sum_k fhat_k e^{2 pi i k.x_u} per node and term as
 *                     a dense contraction on the matrix cores (exact up to rounding), summed over
 *                     the order's terms in registers.  Shared nodes only, R <= 16, the group's
 *                     coefficients and the nodes' phases within the LDS. */
enum { GT_GATHER_SORTED = 0, GT_GATHER_CELL = 1, GT_GATHER_POLY = 2, GT_GATHER_DIRECT = 3 };
int gt_plan_gather_path(const gt_plan *plan, int32_t t, int32_t *path);

/* Selects the forward form of order t (1..ds) by hand (GT_GATHER_*), building what that form
 * needs; synchronises the plan's last stream first.  GT_EUNSUPPORTED when the form is not
 * available for this plan (GT_GATHER_POLY: order 2, FP32, coefficient buffer <= 1 GiB;
 * GT_GATHER_DIRECT: as stated above). */
int gt_plan_set_gather_path(gt_plan *plan, int32_t t, int32_t path);

/* The adjoint's form for order t (1..ds):
 *   GT_ADJ_WINDOW  spread onto the oversampled grid, adjoint FFT, deconvolution (Sec. 3, the
 *                  adjoint display);
 *   GT_ADJ_DIRECT  fhat_k = sum_v y_v e^{-2 pi i k.x_{v,u}} as a dense contraction on the matrix
 *                  cores over node slices, the slices summed in a fixed order (exact up to
 *                  rounding; shared nodes only, R <= 16, |I_u| <= 256).
 * gt_plan_set_adjoint_form synchronises the plan's last stream and allocates the slice
 * partials (at most 512 MiB); GT_EUNSUPPORTED when the form is not available. */
enum { GT_ADJ_WINDOW = 0, GT_ADJ_DIRECT = 1 };
int gt_plan_adjoint_form(const gt_plan *plan, int32_t t, int32_t *form);
int gt_plan_set_adjoint_form(gt_plan *plan, int32_t t, int32_t form);

/* New positions for a plan's nodes (not in the paper: for callers whose nodes move between
 * transforms, e.g. descent on the nodes with gt_plan_node_grad).  x: device, the layout and
 * count given at creation (Mtot x d, the plan's real type); datasets, bandwidths, forms and
 * everything else stay.  The plan keeps its memory and tables: the nodes are wrapped and
 * checked (one synchronisation of `stream`), re-binned on the device, and the order-2 tile
 * spread's work list is rebuilt on the device, with no further host round trip.  Orders whose
 * forward used GT_GATHER_CELL or GT_GATHER_POLY (work items built on the host from the node
 * positions) take GT_GATHER_SORTED; gt_plan_tune or gt_plan_set_gather_path may choose again.
 * The first update allocates the re-binning scratch (kept until the plan is destroyed) and
 * sizes the tile patches for any positions.  Captured graphs are dropped.  NaN or Inf nodes
 * give GT_EINVAL and leave the plan's nodes undefined until the next successful update. */
int gt_plan_update_nodes(gt_plan *plan, const void *x, void *stream);

/* ------------------------------------------------------------------ tuning and graphs
 * (not in the paper: launch choices among forms that compute the same product of
 * Definition def:skatoons and its adjoint, differing in rounding order only)
 *
 * gt_plan_tune times, on the plan's own nodes and with HIP events on `stream`, in this order:
 *   1. per order the forward forms the plan can take (GT_GATHER_SORTED / CELL / POLY /
 *      DIRECT), by the time of that order's kernels (launched one at a time with an event
 *      pair each), keeping the fastest;
 *   2. order 2: the resident wavefronts per compute unit of the tile spread (12, 20, 28, then
 *      4 either side of the best, as the staging LDS allows), by the time of the order-2
 *      adjoint kernels; then per order the adjoint forms (GT_ADJ_WINDOW / DIRECT), by the
 *      time of that order's adjoint kernels;
 *   3. whether order 1 runs on the plan's second stream (forward + adjoint), and, for plans
 *      of orders 1 and 2 that can take them, whether both orders run in shared launches
 *      (gt_plan_set_fused) instead;
 *   4. whether gt_plan_trafo / gt_plan_adjoint launch eagerly or replay a graph of their
 *      launches captured by the plan (forward + adjoint; not on the legacy default stream,
 *      where the plan never captures).
 * It allocates (and frees) one coefficient and one sample buffer for the timing runs, and
 * synchronises `stream`.  The choice is kept by the plan and cached per device and problem
 * signature (d, d_s, bandwidths, window widths, grid sizes, terms, R, node count, dtype,
 * basis, ragged or not): a plan created later with the same signature takes it without
 * timing.  gt_release_all clears the cache.
 *
 * gt_plan_tuning writes the JSON report of the plan's tuning (the candidates' milliseconds
 * and the choices; "cached": true when the plan took a cached choice; "{}" when none) into
 * buf (len bytes, NUL-terminated, truncated to fit) and returns the length it needs including
 * the NUL, or a negative GT_E* code for a handle that is not a live plan.
 *
 * gt_plan_set_graph(on) turns graph replay on or off by hand.  With it on, gt_plan_trafo and
 * gt_plan_adjoint capture their launch sequence on `stream` the first time they see an
 * (input, output) pair (up to 8 pairs per plan, the oldest dropped first) and replay it
 * afterwards; they launch eagerly on the legacy default stream, while `stream` is being
 * captured by the caller, and while per-launch profiling is on.  Only these two calls replay
 * graphs; the solvers and the node gradient launch eagerly.  Changing the plan's forms drops
 * its graphs (after a device synchronisation).
 *
 * gt_plan_set_fused(on) turns the shared launches on or off by hand (Sec. 3, eq. somafm: the
 * same steps for every group, here for the groups of orders 1 and 2 together).  With it on,
 * a forward is three launches (the K1 + K2 packs of both orders, the K3 gathers of both
 * orders, the sum over the groups) and an adjoint three (the K4 spreads of both orders with
 * the empty set's partial sums, the folds of both orders with the empty set's coefficient,
 * the K2 + K5 DFTs of both orders), all on `stream`; each part runs the kernel body and work
 * items of its own launch, so the results are bit for bit those of the separate launches.
 * Available (else GT_EUNSUPPORTED) for plans whose orders are exactly 1 and 2, both with
 * window forms (no GT_GATHER_DIRECT, GT_ADJ_WINDOW) and one window width m, whose gather
 * slots hold every term in one block, and whose order-2 fold takes its tile-sum form within
 * the LDS limit.  Changing a form of an order afterwards so that this no longer holds
 * returns the plan to the separate launches; switching drops the plan's graphs (after a
 * synchronisation of the plan's stream). */
int gt_plan_tune(gt_plan *plan, void *stream);
int64_t gt_plan_tuning(const gt_plan *plan, char *buf, int64_t len);
int gt_plan_set_graph(gt_plan *plan, int32_t on);
int gt_plan_set_fused(gt_plan *plan, int32_t on);

/* ------------------------------------------------------------------ solvers
 * lsqr_solve: R independent weighted Tikhonov problems (eq. new_min_prob), one per
 * right-hand side r with its own lambda[r] >= 0 (lambda = 0: eq. min_prob), solved by
 * LSQR (Paige & Saunders) on A = F W^{-1/2} with damping sqrt(2 lambda); fhat = W^{-1/2} x.
 *   y      device, complex, R x M (or ragged)
 *   lambda host, R doubles >= 0
 *   omega  device, double, |I| weights > 0 (W = diag(omega), Sec. 4.1) shared by all r, or
 *          NULL (omega = 1); FP64 on both precision paths
 *   max_iter >= 1; tol > 0: stop when every r has resid <= tol * resid_0 (checked every
 *   8 iterations with one stream synchronisation), tol <= 0: run exactly max_iter.
 *   fhat   device, complex, R x |I| (output)
 *   info   host, R entries (output); the call synchronises `stream` before returning.
 * Bulk vectors are in the dtype's precision; alpha, beta, norms and rotations are FP64.
 * A breakdown (alpha or beta exactly 0: the solution lies in the Krylov space) freezes that
 * right-hand side and sets GT_SOLVE_BREAKDOWN; it is not an error. */
int lsqr_solve(const gt_problem *p, const void *x, const void *y, const double *lambda,
               const double *omega, int32_t max_iter, double tol, void *fhat,
               gt_solve_info *info, void *stream);

/* lsqr_solve_path: eq. new_min_prob for nlambda values of lambda on each of the R right-hand
 * sides at once (the lambda sweep of the paper's experiments, Sec. 4.1).  The Golub-Kahan
 * bidiagonalisation of A = F W^{-1/2} started from y does not depend on lambda, which enters
 * LSQR only through one extra plane rotation per step, so all lambda values of a right-hand
 * side share one forward and one adjoint transform per iteration: the result for each
 * (lambda[j], r) is the iterate a separate lsqr_solve call with that lambda computes.
 *   lambda    host, nlambda doubles >= 0
 *   fhat_path device, complex, nlambda x R x |I| (output, lambda-major)
 *   info      host, nlambda x R entries (output)
 *   tol > 0: stop when every (lambda, r) has resid <= tol * resid_0 (checked every 8
 *   iterations); tol <= 0: exactly max_iter iterations.
 * Other arguments as for lsqr_solve.  Synchronises `stream`. */
int lsqr_solve_path(const gt_problem *p, const void *x, const void *y, int32_t nlambda,
                    const double *lambda, const double *omega, int32_t max_iter, double tol,
                    void *fhat_path, gt_solve_info *info, void *stream);

/* fista_group_lasso: R group-lasso problems (eq. alligatoah), lambda[r] > 0, every ANOVA
 * term (the empty set included) one group, Algorithm algo:fista from fhat (in: start
 * f_0, out: f_K).
 *   omega  device, double, |I| weights > 0 or NULL, as for lsqr_solve.
 *   L > 0: step constant (backtracking: L_0); L <= 0: 1.05 x a 50-step power-iteration
 *   estimate of ||F||_2^2.
 *   eta <= 1: constant step (the variant in the remark after the algorithm);
 *   eta > 1: backtracking with factor eta: a trial step is accepted when
 *   ||F(f - h)||^2 <= L ||f - h||^2 (the algorithm's test in an equivalent form), else L
 *   grows by eta and the step is retried; after 30 increases within one iteration the
 *   trial is taken and GT_SOLVE_BACKTRACK_CAP is set for that right-hand side.  The
 *   iteration state lives on the device; the host reads it once per batch of steps (not
 *   per trial).
 *   tol > 0: a right-hand side stops when its relative step ||f_k - f_{k-1}|| / ||f_k|| <=
 *   tol; tol <= 0: exactly max_iter accepted iterations.
 * Group norms, the proximal scale (closed form for omega = NULL, otherwise bisection +
 * Newton for xi as in the remark after Theorem theorem:projection), t_k, the momentum and
 * the test are FP64.  Synchronises `stream`. */
int fista_group_lasso(const gt_problem *p, const void *x, const void *y, const double *lambda,
                      const double *omega, int32_t max_iter, double L, double eta, double tol,
                      void *fhat, gt_solve_info *info, void *stream);

/* fista_group_lasso_path: the warm-started path of the paper's experiments (Sec. 4.2):
 * stage j = 0..nlambda-1 solves eq. alligatoah with lambda[j] for every right-hand side, as
 * fista_group_lasso does, starting from the previous stage's solution (stage 0 from fhat0,
 * device R x |I|, or zero when fhat0 is NULL); every stage restarts t_1 = 1 and L_0.  One
 * plan (node sort) serves the whole path.
 *   fhat_path device, complex, nlambda x R x |I| (output: every stage's solution)
 *   info      host, nlambda x R entries (output)
 * Other arguments as for fista_group_lasso.  Synchronises `stream`. */
int fista_group_lasso_path(const gt_problem *p, const void *x, const void *y, int32_t nlambda,
                           const double *lambda, const double *omega, int32_t max_iter, double L,
                           double eta, double tol, const void *fhat0, void *fhat_path,
                           gt_solve_info *info, void *stream);

/* The solvers on an existing plan (the plan's R right-hand sides; nodes sorted once and reused
 * by every call, so repeated solves on fixed nodes pay no plan creation).  Arguments and
 * results as for lsqr_solve and fista_group_lasso.  Work buffers are allocated per call. */
int gt_plan_lsqr(gt_plan *plan, const void *y, const double *lambda, const double *omega,
                 int32_t max_iter, double tol, void *fhat, gt_solve_info *info, void *stream);
int gt_plan_fista(gt_plan *plan, const void *y, const double *lambda, const double *omega,
                  int32_t max_iter, double L, double eta, double tol, void *fhat,
                  gt_solve_info *info, void *stream);
int gt_plan_lsqr_path(gt_plan *plan, const void *y, int32_t nlambda, const double *lambda,
                      const double *omega, int32_t max_iter, double tol, void *fhat_path,
                      gt_solve_info *info, void *stream);

/* ------------------------------------------------------------------ sensitivity analysis
 * gt_sensitivity: global sensitivity indices (eq. gsi) of the approximation with
 * coefficients fhat, by Parseval's identity: for every right-hand side r and term u of the
 * problem's index set, rho[r][u] = sum of |fhat_{u,k}|^2 over the term's coefficients
 * divided by the variance, the same sum over every term u != empty set (rho[r][0] = 0 for the
 * empty set; a zero variance gives rho = 0).  Sums in FP64, in a fixed order.
 *   fhat device, complex (dtype), R x |I|;  rho device, double, R x |U| (output).
 * Synchronises `stream`.
 * gt_active_set: the active set U* of eq. activeset from one right-hand side's indices:
 * the empty set and every term u of the problem with rho[u] > eps[|u| - 1].
 *   rho host, |U| doubles (the problem's terms);  eps host, ds thresholds;
 *   mask host, gt_num_terms(d, ds) flags (output), indexed like gt_problem.term_mask, so a
 *   problem with this mask (and new bandwidths N) gives the refit's index set I_N(U*);
 *   nactive host, terms in U* (output, may be NULL). */
int gt_sensitivity(const gt_problem *p, const void *fhat, double *rho, void *stream);
int gt_active_set(const gt_problem *p, const double *rho, const double *eps, uint8_t *mask, int64_t *nactive);

/* Power-iteration estimate of ||F||_2^2 (50 steps from the all-ones vector, FP64 scalars);
 * synchronises `stream`.  Uses right-hand side 0 of the plan. */
int gt_plan_norm_estimate(gt_plan *plan, int32_t iters, double *out, void *stream);

/* ------------------------------------------------------------------ lifetime
 * A destroyed plan's second stream (drained first) is kept per device and given to the
 * next plan created there (at most 64 kept).
 * gt_release_all: destroys every live plan (as gt_plan_destroy would), destroys the kept
 * streams and clears the process-wide window-table and tuning caches.  Handles of released
 * plans become invalid: later calls with them return GT_EINVAL (they are recognised, not
 * dereferenced), as do calls with a destroyed plan.  Synchronises the released plans'
 * streams. */
int gt_release_all(void);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid allocation): gt_plan_norm_estimate with every work buffer in a
 * fixed 16 MiB device array that the library holds per device for the life of the process,
 * instead of per-call allocations.  It allocates nothing, device or host.
 *   plan, iters, out, stream: as for gt_plan_norm_estimate (synchronises `stream`).
 *   The work buffers take 2 R |I| + R M complex values plus a few partial sums; a plan whose
 *   buffers exceed 16 MiB gives GT_EINVAL (the message states both sizes) without running.
 *   Every call on one device shares the array and leaves its contents behind (each call
 *   initialises what it reads); calls that overlap on one device, from any stream or thread,
 *   race and must not be made. */
int gt_plan_norm_estimate_noalloc(gt_plan *plan, int32_t iters, double *out, void *stream);

/* ------------------------------------------------------------------ diagnostics
 * gt_last_error: thread-local message of the last failing call ("" if none).
 * gt_prof_enable(1): record HIP events around every kernel launch (same stream);
 * gt_prof_report: synchronises, writes a JSON object {kernel: [launches, total_ms]} into
 * buf (truncated to len), clears the records and returns the needed length. */
const char *gt_last_error(void);
int gt_prof_enable(int32_t on);
int64_t gt_prof_report(char *buf, int64_t len);
const char *gt_version(void);

/* Allocation-failure hook for testing the error paths: gt_debug_fail_alloc(k), k >= 1, makes
 * the k-th device allocation from now on fail with GT_ENOMEM (k = 0 turns the hook off); it
 * also resets the count that gt_debug_alloc_count returns (device allocations since). */
int gt_debug_fail_alloc(int64_t k);
int64_t gt_debug_alloc_count(void);

#ifdef __cplusplus
}
#endif
#endif /* GROUPED_H */
