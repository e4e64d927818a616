/*
 * hopfpd -- primal-dual (Chambolle-Pock) solution of the generalized Hopf
 * formula for time-optimal control of linear systems, on AMD MI355X (gfx950).
 *
 * Method: Kirchner, Hewer, Darbon, Osher, "A Primal-Dual Method for Optimal
 * Control and Trajectory Generation in High-Dimensional Systems", arXiv
 * 1712.08226.  Problem statement:
 *   dynamics      dx/dt = A x + B u, u in U = Qu C            Sec. II-B eq. (8), Sec. III-A
 *   control set   C = unit l2 ball or unit box (|u_i| <= 1)    Sec. III-A eq. (16), Sec. VI-A
 *   target        Omega = {x : (x-c)^T W^{-1} (x-c) <= 1}      Sec. VI-A eq. (34)
 *   terminal cost J(x) = 1/2 ((x-c)^T W^{-1} (x-c) - 1)        Sec. IV (zero on the boundary)
 *   value         phi(x,T) from the quadrature form of the
 *                 generalized Hopf formula                     Sec. III-A eq. (18)
 *   minimum time  smallest T with phi(x,T) = 0                 Sec. IV
 *   control       from the optimal dual blocks                 Sec. IV eq. (27)
 *   trajectory    prefix sums over the quadrature nodes        Sec. V eq. (33)
 *
 * Discretisation.  Each system owns a table of N time-to-go nodes
 * tau_k = k h (h = t_max/(N-1) for the trapezoid rule, t_max/N for the left
 * rule of eq. (17)).  A solve at horizon T uses the nodes with tau_k <= T and,
 * for the trapezoid rule, one extra node at tau = T; at T = t_max this is the
 * paper's N-sample layout.
 *
 * Precision.  Tables and matrix exponentials are built in FP64; the
 * iterations run in FP64 (HOPF_FP64: the iterate stays in FP64 between
 * launches; the FP64 certificate evaluates its FP32 rounding, which bounds phi
 * as validly), FP32 (HOPF_FP32) or with K and the iterates split into bf16
 * hi + lo pairs, three bf16 MFMAs per product and FP32 accumulation
 * (HOPF_BF16X3); every
 * reported value, gap and sign decision is certified in FP64 from a primal
 * point lam and a dual-feasible point y:  -min(P(lam), 1/2) <= phi <= -D(y)
 * (P(0) = 1/2 because the terminal cost is at least -1/2).
 *
 * Conventions for every call:
 *   - arrays are row-major, float64 unless stated, owned by the caller;
 *     inputs are copied before the call returns and no pointer is retained;
 *   - "_dev" entry points take device pointers (memory the caller allocated
 *     on the context's device) and a hipStream_t passed as void*; they
 *     synchronise that stream before returning;
 *   - a failed call returns a non-zero hopf_status and leaves a message in
 *     hopf_last_error(ctx); no exception or abort crosses the interface;
 *   - per-point problems (unreachable, not converged, non-finite input) are
 *     reported per point and never fail the call;
 *   - a context is not thread-safe: use one per host thread.
 */
#ifndef HOPFPD_H
#define HOPFPD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hopf_ctx hopf_ctx;

typedef enum {
  HOPF_OK = 0,
  HOPF_EINVAL = 1,        /* bad argument (shape, range, W not SPD, NULL) */
  HOPF_ENOMEM = 2,        /* device or host allocation failed */
  HOPF_EDEVICE = 3,       /* HIP runtime error */
  HOPF_ESTATE = 4,        /* call out of order (e.g. solve before set_systems) */
  HOPF_EUNSUPPORTED = 5   /* valid request the library does not handle */
} hopf_status;

typedef enum { HOPF_U_L2 = 0, HOPF_U_BOX = 1 } hopf_uset;
typedef enum { HOPF_Q_TRAP = 0, HOPF_Q_LEFT = 1 } hopf_quad;
typedef enum { HOPF_FP64 = 0, HOPF_FP32 = 1, HOPF_BF16X3 = 2 } hopf_prec;
typedef enum {
  HOPF_WARM_COLD = 0, HOPF_WARM_CONT = 1, HOPF_WARM_MLP = 2, HOPF_WARM_MLP_LAM = 3, HOPF_WARM_MLP_FIRST = 4
} hopf_warm;
typedef enum { HOPF_ROOT_BISECT = 0, HOPF_ROOT_NEWTON = 1 } hopf_root;

/* per-point result status */
typedef enum {
  HOPF_PT_OK = 0,         /* certified to gap_tol */
  HOPF_PT_INSIDE = 1,     /* x already in the target: T = 0 */
  HOPF_PT_UNREACH = 2,    /* phi(x, t) > 0 certified at every scan horizon, t_max included: T = +inf */
  HOPF_PT_NOCONV = 3,     /* max_iter reached before a certified sign/gap */
  HOPF_PT_NONFINITE = 4   /* NaN/Inf in the input or the iterates */
} hopf_pt;

/* One system.  Sizes: A n*n, B n*m, Qu m*m (NULL = identity), W n*n
 * symmetric positive definite (HOPF_EINVAL otherwise; a W that is not
 * diagonal is diagonalised once, W = U diag(d) U^T, and the system is solved
 * in the rotated state U^T x: x, lam0 are rotated in and lam, x(s), p*
 * rotated back, so every call keeps the caller's coordinates), c n (NULL = 0).
 * Limits: 1 <= n <= 256, 1 <= m <= 64, 2 <= N <= 4096, t_max > 0.
 * c_tau: this system's primal step ratio (see hopf_opts.c_tau); 0 uses the
 * call's option.  Lets one call mix systems whose best ratio differs (the
 * box control set wants a much smaller one than the l2 ball). */
typedef struct {
  int n, m, N;
  double t_max;
  int quad;               /* hopf_quad */
  int uset;               /* hopf_uset */
  const double *A, *B, *Qu, *W, *c;
  double c_tau;
} hopf_system;

/* Solver options (hopf_default_opts fills the defaults in brackets).
 *   c_tau         primal step tau = c_tau / L, dual step sigma = 0.999/(tau L^2),
 *                 L >= ||K|| (Sec. III: tau sigma ||K||^2 < 1; Sec. VI: theta = 1)   [1.0]
 *   gap_tol       stop when (P - D) / max(1, |D|) <= gap_tol                         [1e-6]
 *   t_rel_tol     bisection stops when hi - lo <= max(t_rel_tol*hi,
 *   t_abs_frac                                    t_abs_frac*t_max)                 [0.5e-4, 1e-6]
 *   max_iter      iteration cap per solve (probe): a solve still undecided at a
 *                 certificate after max_iter or more iterations ends its query with
 *                 HOPF_PT_NOCONV (certificates come every check_every iterations) [200000]
 *   check_every   iterations between FP64 certificates                               [50]
 *   warm          HOPF_WARM_COLD: every probe starts at lam = 0, y = 0;
 *                 HOPF_WARM_CONT: every probe starts from the previous probe's iterate;
 *                 HOPF_WARM_MLP: as CONT, and the system's trained network's bracket
 *                 [T e^-d, T e^d] gives the probe hints (as hopf_min_time's t_bracket)
 *                 of points whose caller gave none;
 *                 HOPF_WARM_MLP_LAM: as MLP, and every probe starts from the
 *                 network's lam_0 (y from the previous probe);
 *                 HOPF_WARM_MLP_FIRST: as CONT, and the first probe (the only one
 *                 that CONT starts cold) starts from the network's lam_0 unless the
 *                 caller gave lam0.
 *                 The learned modes fall back to CONT where no trained network
 *                 exists.  The start changes only the iterations: the probe
 *                 horizons, hence T, are those of the search below (hints aside) [COLD]
 *   prec          hopf_prec of the iterations; with HOPF_BF16X3 a probe that is not
 *                 certified after 4000 iterations continues in FP32 (its iterates
 *                 carry over unchanged)                                              [FP32]
 *   scan          minimum time (Sec. IV: the smallest T with phi(x, T) = 0): the
 *                 horizons t_max (j / scan)^2, j = 1..scan, are probed in ascending
 *                 order until the first certified reach; the cell between the last
 *                 certified-unreachable horizon (0 for j = 1) and that reach is then
 *                 refined.  The spacing, about 2 sqrt(t t_max) / scan at horizon t, is
 *                 finest near 0, where reachable intervals are short.  A set of
 *                 reachable horizons that lies strictly between two neighbouring scan
 *                 horizons is not seen                                             [48]
 *   root          refinement of the cell [lo, hi] (after any hints):
 *                 HOPF_ROOT_BISECT: midpoint;  HOPF_ROOT_NEWTON: the hybrid of Sec. IV,
 *                 root estimate r = t - phi/(d phi/dt) with d phi/dt = -H_x(p*, x0) (the
 *                 Newton update with the Hamiltonian) and phi the midpoint of the
 *                 certified interval; the probe goes to r plus or minus (0.4 of the
 *                 stopping tolerance + half the interval's width / |slope|), towards the
 *                 bracket end farther from r; the midpoint where it would leave (lo, hi),
 *                 where the slope is not negative, and after a Newton probe that left
 *                 the bracket wider than half its width before the step            [BISECT]
 *   newton_after  hybrid only: probes of the cell before Newton steps start         [1]
 *   newton_rho    hybrid only: cell probes from newton_after on also run until
 *                 P - D <= newton_rho |P + D| / 2 so the Newton step sees an accurate
 *                 value                                                              [0.5]
 *   wide_min      FP32 and BF16 iterations run on 64-point workgroups that share one
 *                 LDS copy of the table's rows (each node block; for large m or n
 *                 each component pair of a block) while at least wide_min of a
 *                 system's points are active (then on 16-point tiles); 0: never  [16384]
 *   deep_max      FP32 16-point tiles: while at most deep_max of a system's points
 *                 are active, each tile's node blocks are spread over 8 waves
 *                 instead of 4; -1: 16 points per compute unit of the device,
 *                 0: never                                                           [-1]
 *   structure     value solves and minimum-time searches (those without a caller's
 *                 lam0) of a system made of k > 1 copies of one b-dimensional
 *                 system that share the control (A = I_k (x) A_b, B = 1_k (x) B_b,
 *                 W block-diagonal with blocks W_b / a_c, W_b diagonal, a_c > 0,
 *                 c = 1_k (x) c_b: the sampled-copy systems of Sec. VI-B/C, equal
 *                 or sigma-point weights) run on the b-dimensional system of the
 *                 copies' a-weighted mean with target matrix W_b / sum_c a_c; the
 *                 value adds the spread (1/2) sum_c a_c |e^{tA_b}(x_c - mean)|^2_{W_b^-1}
 *                 in FP64 (a search adds it to the certified bounds at every probe
 *                 horizon, and its points skip the tail solver) and lambda is
 *                 rebuilt per copy; iters and probes count the reduced solve's.
 *                 Exact (the copies share z(u) in x_c(t) = e^{tA_b} x_c + z(u));
 *                 0: solve the full system                                        [1]
 *   tail_max      FP32 iterations: once at most tail_max of a system's points are
 *                 still running, a per-point solver (one workgroup per point,
 *                 matrix-vector iterations, certificate and search step in one
 *                 launch) finishes them; 0 keeps every point on the 16-point tiles
 *                 (at most 8192; workgroups beyond two per compute unit wait
 *                 for a free slot)                                                  [2048]
 *   adapt         tail solver: adapt each point's step ratio at restarts (not in the
 *                 paper): when the certified gap has fallen to 0.2 of its value at the
 *                 last restart (or to 0.8 and rises again), the primal weight
 *                 omega = 1/c_tau moves to sqrt(omega * |dy| / |dlam|) (dy, dlam: the
 *                 change of the iterates since that restart), kept within 4x of the
 *                 probe's starting weight, and tau, sigma are rescaled with tau sigma
 *                 fixed; restarts are at least 4 certificates apart.  Results stay
 *                 certified; only the iteration path changes                          [1] */
typedef struct {
  double c_tau, gap_tol, t_rel_tol, t_abs_frac;
  int max_iter, check_every, warm, prec;
  int root, newton_after;
  double newton_rho;
  int tail_max, adapt;
  int scan;
  int wide_min;
  int deep_max;
  int structure;
} hopf_opts;

hopf_status hopf_default_opts(hopf_opts *out);

/* Create a context on HIP device `device` (owns a stream and all device
 * memory it allocates).  *out is NULL on failure. */
hopf_status hopf_create(int device, hopf_ctx **out);
void hopf_destroy(hopf_ctx *ctx);                      /* NULL is a no-op */
const char *hopf_strerror(hopf_status s);
const char *hopf_last_error(const hopf_ctx *ctx);      /* ctx-owned, valid until the next call */

/* Copy the systems and build their FP64 node tables e^{k h A} B Qu
 * (scaling-and-squaring matrix exponential, the setup step of Sec. III-A /
 * Sec. VI) and operator-norm prefix bounds; replaces earlier systems. */
hopf_status hopf_set_systems(hopf_ctx *ctx, int nsys, const hopf_system *sys);
hopf_status hopf_set_opts(hopf_ctx *ctx, const hopf_opts *opts);

/* Value phi(x_i, t_i) (eq. (18)), certified: phi_lo <= phi <= phi_hi with
 * (phi_hi - phi_lo)/max(1,|phi_hi|) <= gap_tol unless pt_status says otherwise.
 *   sys_id  npts ints or NULL (all system 0).  Points of different systems may
 *           be mixed in one call: each system's points run as their own job
 *           (own kernels and tiles) and the jobs run concurrently
 *   x       npts rows of stride n_max = the largest n among the systems the call
 *           uses; a row holds its system's n entries first (the rest is ignored)
 *   t       npts horizons in [0, t_max]
 *   lam     npts rows of stride n_max: terminal costates lam* = e^{-T A^T} p*
 *           (the system's n entries first; the rest is not written) or NULL
 *   iters   npts or NULL; pt_status npts (required). */
hopf_status hopf_value(hopf_ctx *ctx, long npts, const int *sys_id, const double *x,
                       const double *t, double *phi_lo, double *phi_hi, double *lam,
                       int *iters, int *pt_status);

/* Minimum time to reach the target (Sec. IV: the smallest T with
 * phi(x, T) = 0) by a certified search on (0, t_max]: the scan of opts.scan
 * horizons finds the first cell with a certified sign change, which is then
 * refined (bisection or the hybrid Newton step, opts.root) until
 * hi - lo <= max(t_rel_tol hi, t_abs_frac t_max); T = hi and the solve at hi
 * is continued to gap_tol.
 *   sys_id, x   as for hopf_value (systems may be mixed)
 *   lam0        NULL, or npts rows of stride n_max: the starting costate of
 *               each point's first probe (later probes start as opts.warm says)
 *   t_bracket   NULL, or npts pairs (a, b): probe hints; once the cell is found,
 *               b and then a are probed first, each only if it lies strictly
 *               inside the current bracket (non-finite values are skipped).
 *               Hints move probes, so where phi(x, .) has several zeros inside
 *               the cell they can change which one the refinement ends on
 * Outputs: T (npts; +inf where every scan horizon is certified unreachable, 0
 * inside the target, NaN for NOCONV / NONFINITE), gap (npts, normalised gap
 * of the final solve at T), lam (npts rows of stride n_max as for hopf_value,
 * or NULL), probes, iters (npts or NULL), pt_status (npts). */
hopf_status hopf_min_time(hopf_ctx *ctx, long npts, const int *sys_id, const double *x,
                          const double *lam0, const double *t_bracket, double *T, double *gap,
                          double *lam, int *probes, int *iters, int *pt_status);

/* Device-pointer twin of hopf_min_time: every array is device memory;
 * sys_id, lam0, t_bracket may be NULL; lam, probes, iters may be NULL. */
hopf_status hopf_min_time_dev(hopf_ctx *ctx, long npts, const int *sys_id, const double *x,
                              const double *lam0, const double *t_bracket, double *T, double *gap,
                              double *lam, int *probes, int *iters, int *pt_status, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): hopf_min_time_dev for the points
 * of one system `sys`, with the per-point solver state in a fixed device
 * scratch of 64 MiB that each GPU holds for the life of the process.  The
 * call makes no device, pinned-host or event allocation and creates no
 * stream; it checks the active count synchronously between rounds and
 * records no timing (hopf_last_timing reads zeros).  A call whose state does
 * not fit (about 43 KB per point for n = 100, m = 10, N = 300: some 1,500
 * points) returns HOPF_EINVAL with the size it needed.  Calls that overlap
 * on one GPU share the scratch and race: issue them one after another.
 * Arguments as for hopf_min_time_dev (lam0, t_bracket, lam, probes, iters
 * may be NULL; stream NULL: the context's). */
hopf_status hopf_min_time_dev_noalloc(hopf_ctx *ctx, long npts, int sys, const double *x, const double *lam0,
                                      const double *t_bracket, double *T, double *gap, double *lam, int *probes,
                                      int *iters, int *pt_status, void *stream);

/* Device-pointer twin of hopf_value: x, t, phi_lo, phi_hi, pt_status (and
 * sys_id, lam, iters when given) are device memory with the layouts of
 * hopf_value; the solve runs on `stream` (NULL: the context's stream).  The
 * call copies t (and sys_id) to the host and checks them before any kernel
 * runs (HOPF_EINVAL if a horizon lies outside [0, t_max] of its system), and
 * returns when the results are in place. */
hopf_status hopf_value_dev(hopf_ctx *ctx, long npts, const int *sys_id, const double *x,
                           const double *t, double *phi_lo, double *phi_hi, double *lam,
                           int *iters, int *pt_status, void *stream);

/* Optimal control and trajectory at horizon T from x0 (Sec. IV eq. (27),
 * Sec. V eq. (33)).  Solves phi(x0,T) to gap_tol first.  Outputs, with
 * n_nodes <= N+1 written to *n_nodes, rows sorted by increasing physical
 * time s in [0, T]:
 *   s       n_nodes   physical times of the nodes
 *   u       n_nodes*m control at each node (Qu y_k / w_k; 0 where w_k = 0)
 *   xs      n_nodes*n state after each node's contribution (last row = x(T))
 *   p_star  n         costate p* = e^{T A^T} lam*  (the paper's minimiser, eq. (24))
 * Arrays must hold N+1 rows. */
hopf_status hopf_trajectory(hopf_ctx *ctx, int sys_id, const double *x0, double T,
                            int *n_nodes, double *s, double *u, double *xs, double *p_star,
                            double *phi_lo, double *phi_hi);

/* Learned warm start (not in the paper): per system, an MLP (x, t) -> (lam_0,
 * log T_hat, bracket half-width) with three hidden layers of width 256 and
 * GELU, trained on the final costates of the solver's own probes.
 *   hopf_warm_init      (re)initialise the network of sys_id (He init, seed)
 *   hopf_warm_params    get (set=0) or set (set=1) the flat FP32 parameter
 *                       vector (count must equal the network's size) and
 *                       optionally the normalisation norm = [x_mean (n),
 *                       x_std (n), t_scale, lam_scale]; setting with norm
 *                       marks the network as trained
 *   hopf_warm_loss_grad loss and FP32 gradient of the current parameters on
 *                       rows Z (nrows x (n+1)), Y (nrows x (n+2)): targets
 *                       lam/lam_scale (n), log T*, reach flag (0/1)
 *   hopf_warm_train     solve min-time for the npts training points x (host,
 *                       npts x n), log every probe's (x, T, lam), then train
 *                       `epochs` epochs of Adam (batch rows, learning rate lr);
 *                       epoch_loss (epochs, may be NULL) gets the mean loss per
 *                       epoch and *pairs the number of training rows */
hopf_status hopf_warm_init(hopf_ctx *ctx, int sys_id, unsigned seed);
/* hopf_warm_save     write the trained network of sys_id to `path` (HOPF_ESTATE if
 *                    it has none)
 * hopf_warm_load     read a network written by hopf_warm_save into sys_id and mark
 *                    it trained; HOPF_EINVAL (nothing replaced) when the file is
 *                    missing, truncated, for another n or width, or non-finite
 * File format, little-endian: the 8 bytes "HOPFWARM", u32 version (1), u32 n,
 * u32 width H, u64 parameter count, f32 t_scale, f32 lam_scale, f32 x_mean[n],
 * f32 x_std[n], f32 parameters[count] (the flat vector of hopf_warm_params). */
hopf_status hopf_warm_save(hopf_ctx *ctx, int sys_id, const char *path);
hopf_status hopf_warm_load(hopf_ctx *ctx, int sys_id, const char *path);
hopf_status hopf_warm_params(hopf_ctx *ctx, int sys_id, int set, float *theta, long count, float *norm);
hopf_status hopf_warm_loss_grad(hopf_ctx *ctx, int sys_id, int nrows, const float *Z, const float *Y,
                                double *loss, float *grad);
hopf_status hopf_warm_train(hopf_ctx *ctx, int sys_id, long npts, const double *x, int epochs, int batch,
                            float lr, unsigned seed, double *epoch_loss, long *pairs);

/* Device time and work of the last solve call, for throughput and roofline
 * reporting.  A call runs rounds of tiled kernels (16 points per tile: probe
 * setup, fused iteration kernel, FP64 certificate) and, once at most
 * hopf_opts.tail_max of a system's points remain (FP32 iterations), a
 * per-point tail solver that finishes them in one launch.
 *   total_s          HIP events around the whole call
 *   iter_kernel_s    the tiled iteration kernels alone, summed over launches
 *                    (the launches of a multi-system call can overlap)
 *   iter_launches    their launch count
 *   iter_point_rows  point-rows they processed (one row = one quadrature node
 *                    of one point in one iteration)
 *   alg_flops        algorithmic flops of all iterations, 4 m n per point-row
 *                    (K lam and K^T y), summed over the systems of the call
 *   tail_kernel_s    the tail solver's launches (iterations, certificates and
 *                    probe setups of the points it finished)
 *   tail_point_rows  point-rows iterated by the tail solver
 *   tail_points      points handed to it
 *   wide_kernel_s, wide_launches, wide_point_rows
 *                    the share of iter_kernel_s, iter_launches and
 *                    iter_point_rows that ran on the 64-point iteration kernel
 *                    (rounds with at least hopf_opts.wide_min active points) */
typedef struct {
  double total_s, iter_kernel_s;
  long iter_launches;
  double iter_point_rows, alg_flops, tail_kernel_s, tail_point_rows;
  long tail_points;
  double wide_kernel_s;
  long wide_launches;
  double wide_point_rows;
} hopf_timing;

hopf_status hopf_last_timing(const hopf_ctx *ctx, hopf_timing *out);

#ifdef __cplusplus
}
#endif
#endif /* HOPFPD_H */
