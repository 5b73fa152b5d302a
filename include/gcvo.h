/*
 * gcvo.h - C ABI of the MI355X (gfx950) Generalized-CVO registration library.
 *
 * The library solves the registration problem of the paper's Sec. "Classical
 * RKHS loss functions" and Sec. "Generalized CVO": given a target cloud X and a
 * source cloud Z, find the pose T in SE(3) that maximises
 *
 *     f(T) = sum_{i,j} k(x_i, T^{-1} z_j)                        eq. (rkhs_loss)
 *     k(x, z) = sigma2 * exp(-1/2 (x - z)^T Sigma(x, z)^{-1} (x - z))   eq. (kernel)
 *     Sigma(x_i, z_j) = Sigma(x_i; X) + R^T Sigma(z_j; Z) R          eq. (covariance)
 *
 * with per-point covariances from the n nearest points (eq. (covariance)), an
 * eigenvalue bound per point (Remark 1), and Riemannian Gauss-Newton steps
 * T <- T exp([-H_GN^{-1} g]^) (Algorithm 1, eq. (gn_update)), where g is the
 * gradient of Lemma 1 and H_GN the approximate Hessian of eq. (hessian_gn) plus
 * the connection term of eq. (connection_se3).
 *
 * Readings of what the paper leaves open, used throughout:
 *   - Length scale: the per-point covariance is (ell^2 / 2) * S(p) where S(p)
 *     has its largest eigenvalue normalised to 1 and the other two floored at
 *     eig_ratio_min (rho); rho = 1 gives CVO's isotropic kernel (Remark 3).
 *   - Cutoff: only pairs with ||x_i - T^{-1} z_j||^2 <= (cutoff_scale * ell)^2
 *     enter the sums (the truncated double sum is the definition).
 *   - The covariances are frozen at the current rotation for each step
 *     (Remark 2); g is the gradient with the covariances frozen.
 *   - Annealing: ell_{s+1} = max(anneal_factor * ell_s, length_scale_min); a
 *     non-final stage ends when ||xi||_1 < stage_tol or after
 *     max_iters_per_stage iterations; the final stage runs to ||xi||_1 < tol.
 *   - Damping: if the Gauss-Newton step is not an ascent direction or H_GN is
 *     numerically singular, the connection term is dropped and
 *     (H_main - lambda * ||diag H_main||_2 * I) is used, lambda = 1e-6 * 10^m,
 *     m = 0..6.
 *
 * Conventions.  Poses are row-major 4x4 double, T p = R p + t; twists are
 * (omega, v), rotation first, with right perturbation T exp(xi^) (Notation
 * section).  The result satisfies x ~ T^{-1} z: if the target was generated as
 * x = G p from the source surface p, the expected answer is T = G^{-1}.
 *
 * Memory.  Point clouds are caller-owned DEVICE memory, float32, array of
 * structures [n][3].  Shapes are caller-owned DEVICE memory, float32, structure
 * of arrays [6][n] in the order (xx, xy, xz, yy, yz, zz).  Poses, parameters and
 * info structs are HOST memory unless stated otherwise.  Scratch memory is a
 * caller-provided DEVICE workspace of at least the size the matching
 * *_workspace_size function returns, aligned to 256 bytes; the library never
 * allocates device memory in these calls and never frees caller memory.
 * The one piece of state the library keeps across calls is a per-device pool
 * of small pinned host buffers (two ints per pair of a call, plus the pairs'
 * final states for calls that return them to the host) in which the device
 * reports completion to the polling host; a buffer returns to the pool when
 * the stream has passed the last work that writes it, and the pool is guarded
 * by a mutex, so calls from several threads are safe.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  All device
 * work is enqueued on it.  gcvo_register and gcvo_eval_fgh are complete when
 * the call returns (the call waits on the stream); gcvo_register_batch writes
 * its device outputs on the stream after it returns, and gcvo_point_shapes
 * returns without waiting.
 *
 * Errors.  Every function returns 0 (GCVO_OK) or a negative GCVO_ERR_* code;
 * no exception or abort crosses the ABI.  On error, pose outputs are left
 * untouched.  Not converging within max_iters is not an error: info.converged
 * is 0.  Calls are reentrant; two calls that share a workspace must not overlap.
 *
 * Determinism.  Reductions use a fixed order and no floating-point atomics, so
 * repeated calls on the same device and inputs give bitwise identical results.
 */
#ifndef GCVO_H
#define GCVO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCVO_OK 0
#define GCVO_ERR_INVALID (-1)        /* null pointer, bad size, non-finite input, T not in SE(3), bad parameter */
#define GCVO_ERR_TOO_FEW_POINTS (-2) /* a cloud has fewer points than knn                                        */
#define GCVO_ERR_NO_PAIRS (-3)       /* no (target, source) pair within the cutoff at some iteration            */
#define GCVO_ERR_SINGULAR (-4)       /* the damped Gauss-Newton system could not be solved                      */
#define GCVO_ERR_WORKSPACE (-5)      /* workspace NULL, too small or misaligned                                 */
#define GCVO_ERR_HIP (-6)            /* a HIP runtime call failed                                               */
#define GCVO_ERR_CAPACITY (-7)       /* a size exceeds the library's limits (see GCVO_MAX_*)                    */

#define GCVO_PRECISION_FP32 0 /* pair terms in FP32, FP32 per-block sums, compensated cross-block sums, FP64 solve */
#define GCVO_PRECISION_FP64 1 /* the same kernels instantiated in FP64 throughout                                  */

/* Solvers (Sec. "A first-order method", Sec. "A second-order method", the
 * exact-Hessian ablation).  All three stop on ||xi||_1 and anneal alike.
 *   GN           Gauss-Newton: H = H_main + C(g) (eq. (hessian_gn), eq. (connection_se3)).
 *   NEWTON       exact frozen-covariance Hessian: H = H_main + T1 + T2 + C(g),
 *                T1 = sum f (J^T u)(J^T u)^T (product rule on f_ij), T2 =
 *                -sum f [u^ J; 0] (derivative of J_j), u = Sigma^{-1} r
 *                (eq. (direction_derivative_gradf) with Sigma frozen).  Its
 *                step replaces the Gauss-Newton step where that system's
 *                symmetric part is negative definite (a concave model), the
 *                step ascends, and it is at most twice as long as the
 *                Gauss-Newton step (reading: far from a maximum, pure Newton
 *                steps leave the basin).  The damped fallback uses H_main as
 *                for GN.
 *   FIRST_ORDER  T <- T exp(mu g^) (eq. (fo_update)) with mu from the quartic
 *                expansion of f along g (eq. (linesearch), App. "Line search";
 *                coefficients re-derived by expanding the kernel exponent along
 *                exp(-t xi^) y, the printed ones being partly garbled): the
 *                smallest positive root of the expansion's derivative; where it
 *                has none, the maximiser of its quadratic part when that
 *                exists; mu is never below min_step.  Each iteration is a
 *                gradient pass and a line-search pass over the pairs. */
#define GCVO_SOLVER_GN 0
#define GCVO_SOLVER_NEWTON 1
#define GCVO_SOLVER_FIRST_ORDER 2

#define GCVO_MAX_KNN 16
#define GCVO_MAX_STAGES 16
#define GCVO_MAX_POINTS (1LL << 26) /* per cloud */
#define GCVO_MAX_LABEL_DIM 4        /* entries of a label vector (the *_labeled calls) */

/* Pair-kernel measurement of one call (caller-owned, zero it first; calls
 * that are given one add to it): over the launches of the per-iteration pair
 * kernel in which at least one pair was still iterating, their summed duration
 * (HIP events attached to each dispatch, on the caller's stream), their
 * number, the (target, source) pairs evaluated within the cutoff and the
 * source points processed.  A measured call waits on its stream. */
typedef struct gcvo_profile {
    double pair_kernel_ms;
    long long launches;
    long long pairs;
    long long source_points;
} gcvo_profile;

typedef struct gcvo_params {
    double length_scale;      /* ell of the first stage, metres (> 0)                                   */
    double length_scale_min;  /* ell of the final stage (0 < min <= length_scale); == length_scale: fixed */
    double anneal_factor;     /* alpha in (0, 1]; must be < 1 when min < length_scale                    */
    double cutoff_scale;      /* pair cutoff radius = cutoff_scale * ell (> 0; 3 in the paper's setups)  */
    int knn;                  /* n nearest points per covariance, self included, 2..GCVO_MAX_KNN (10)    */
    double eig_ratio_min;     /* rho in (0, 1]: floor of lambda / lambda_max per point (Remark 1); rho = 1:
                                 every shape is the identity (isotropic kernel, Remark 3), no neighbours
                                 are searched and Gauss-Newton uses the isotropic pair kernel            */
    double sigma2;            /* kernel amplitude sigma^2 (> 0; 1)                                       */
    int max_iters;            /* total Gauss-Newton iterations over all stages (>= 1)                    */
    int max_iters_per_stage;  /* iterations before a non-final stage is ended (>= 1)                     */
    double tol;               /* final-stage stop: ||xi||_1 < tol (> 0; 1e-6)                            */
    double stage_tol;         /* non-final stage stop: ||xi||_1 < stage_tol (> 0; 1e-4)                  */
    int precision;            /* GCVO_PRECISION_FP32 (default) or GCVO_PRECISION_FP64                    */
    int solver;               /* GCVO_SOLVER_GN (default), GCVO_SOLVER_NEWTON or GCVO_SOLVER_FIRST_ORDER */
    double min_step;          /* first-order solver: smallest step mu (> 0; 1e-10)                      */
    double cell_fraction;     /* pair-grid cell edge along y and z as a fraction of the cutoff radius,
                                 in [0.2, 1] (0.5)                                                       */
    double cell_fraction_x;   /* pair-grid cell edge along x (the direction of the cell rows a point
                                 walks), same unit, in [0.1, 1] (0.125).  Any cell shape gives the same
                                 pairs within the cutoff, so the same sums up to the order of FP32
                                 additions; smaller x cells clip each row closer to the cutoff ball
                                 without adding rows, smaller y-z cells add rows (see the autotuner
                                 of the Python binding).                                                */
    gcvo_profile *profile;    /* optional measurement of the call (NULL: none); a batch call uses the
                                 first parameter set's                                                   */
} gcvo_params;

typedef struct gcvo_info {
    int status;              /* mirrors the return value                                    */
    int converged;           /* 1 when the final stage reached ||xi||_1 < tol               */
    int iters;               /* solver iterations performed                                 */
    int stages;              /* length-scale stages entered                                 */
    long long pairs_last;    /* pairs within the cutoff at the last iteration               */
    double f;                /* objective at the last evaluated pose                        */
    double g[6];             /* gradient (omega, v) at the last evaluated pose              */
    double xi_l1;            /* ||xi||_1 of the last step                                   */
    int stage_iters[GCVO_MAX_STAGES]; /* iterations spent in each stage                     */
    int damped;              /* steps not taken with the plain system: damped Gauss-Newton steps
                                (Newton: also the steps taken with the Gauss-Newton system;
                                first order: steps not at a root of the line-search quartic) */
} gcvo_info;

/* Fills p with the defaults named above (ell = 0.3 fixed, cutoff 3, knn 10,
 * rho 0.01, sigma2 1, 30 iterations, tol 1e-6, stage_tol 1e-4, FP32, Gauss-Newton,
 * cell fractions 0.5 across and 0.125 along the rows, no profile). */
void gcvo_default_params(gcvo_params *p);

/* Bytes of device workspace gcvo_register needs for clouds of these sizes and
 * these parameters; 0 if the arguments are invalid. */
size_t gcvo_workspace_size(long long n_tgt, long long n_src, const gcvo_params *p);

/*
 * Registers one pair: Algorithm 1 with Gauss-Newton steps and length-scale
 * annealing, starting at T_init (host, 4x4; NULL = identity).  Computes the
 * per-point covariance shapes of both clouds (eq. (covariance), Remark 1) on
 * the device, builds the target cell lists for every stage, then iterates.
 * tgt_xyz / src_xyz: device float32 [n][3].  T_out (host, 4x4) receives the
 * pose; info (host, may be NULL) the run summary.  Waits on `stream`.
 */
int gcvo_register(const float *tgt_xyz, long long n_tgt, const float *src_xyz, long long n_src,
                  const double *T_init, const gcvo_params *p, double *T_out, gcvo_info *info,
                  void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of device workspace gcvo_register_batch needs for the same n_pairs,
 * offsets and parameters (see gcvo_register_batch); 0 if invalid. */
size_t gcvo_batch_workspace_size(int n_pairs, const long long *tgt_off, const long long *src_off,
                                 const gcvo_params *p, int shared_params);

/*
 * Registers n_pairs independent pairs in one pass over the device (Algorithm 1
 * for every pair, as gcvo_register does for one).  Pair k's target is
 * tgt_xyz[tgt_off[k] .. tgt_off[k+1]) and its source src_xyz[src_off[k] ..
 * src_off[k+1]) (device float32 [*][3]).
 *   tgt_off, src_off  HOST int64 [n_pairs + 1]: the host lays the workspace out
 *                     from the pair sizes, which the caller knows (taking them
 *                     from device memory would stall the stream on every call).
 *   T_init            DEVICE double [n_pairs][16] row-major start poses, or NULL
 *                     (identity).  A start pose that is not a rigid motion within
 *                     1e-6 fails its pair with GCVO_ERR_INVALID.
 *   p                 HOST: n_pairs parameter sets, or one set shared by all pairs
 *                     when shared_params != 0; all pairs must use the same knn,
 *                     precision and solver.
 *   T_out             DEVICE double [n_pairs][16]: the poses.
 *   info              DEVICE gcvo_info [n_pairs] or NULL: the run summaries.
 * A pair that fails (too few points, no pair in reach, a bad start pose, ...)
 * reports its status in info[k].status and gets T_out[k] = its start pose; the
 * call itself returns an error only for argument, workspace and HIP errors.
 * Asynchronous outputs: the call returns once every pair has stopped iterating
 * (the device reports completion through pinned host flags that the host
 * polls, so no iteration beyond the last useful chunk is enqueued); T_out and
 * info are then written by a kernel enqueued on `stream`, so they are ready
 * once the stream has reached it (synchronise the stream, or order later work
 * on it).  Until then the workspace, T_init, T_out and info must stay valid.
 * Two calls that share a workspace must not overlap on the device.
 */
int gcvo_register_batch(int n_pairs, const float *tgt_xyz, const long long *tgt_off, const float *src_xyz,
                        const long long *src_off, const double *T_init, const gcvo_params *p,
                        int shared_params, double *T_out, gcvo_info *info, void *workspace,
                        size_t workspace_bytes, void *stream);

/* Bytes of device workspace gcvo_eval_fgh needs; 0 if invalid. */
size_t gcvo_eval_workspace_size(long long n_tgt, long long n_src);

/*
 * One evaluation of Algorithm 1's body without the step: at pose T (host 4x4),
 * with the given shapes (device float32 SoA [6][n], covariance = (ell^2/2) *
 * shape), returns f (eq. (rkhs_loss)), the gradient g = (g_omega, g_v) of
 * Lemma 1 and the Gauss-Newton Hessian H (host, row-major 6x6) =
 * -sum f J^T Sigma^{-1} J + C(g) (eq. (hessian_gn), eq. (connection_se3)),
 * summed over pairs within `cutoff` metres; n_pairs (host, may be NULL)
 * receives their number.  precision selects the FP32 or FP64 kernels.
 * Waits on `stream`.
 */
int gcvo_eval_fgh(const float *tgt_xyz, const float *tgt_shape6, long long n_tgt, const float *src_xyz,
                  const float *src_shape6, long long n_src, const double *T, double length_scale,
                  double cutoff, double sigma2, int precision, double *f, double *g, double *H,
                  long long *n_pairs, void *workspace, size_t workspace_bytes, void *stream);

/*
 * gcvo_eval_fgh for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid allocation): the same
 * evaluation, the same kernels and bitwise the same results, with a library
 * scratch array of GCVO_NOALLOC_SCRATCH_BYTES per GPU in place of the
 * workspace, so the call allocates nothing (the array is part of the loaded
 * library; each GPU holds its own copy until the process ends).  Sizes whose
 * gcvo_eval_workspace_size exceeds the scratch (about 240k points per cloud
 * at equal sizes) return GCVO_ERR_CAPACITY before any device work.  Every call
 * on a GPU uses that GPU's one array: calls that overlap on a device (other
 * threads, other streams) race and must be serialised by the caller.  The call
 * waits on `stream`, so calls from one thread never overlap.
 */
#define GCVO_NOALLOC_SCRATCH_BYTES (64LL << 20)
int gcvo_eval_fgh_noalloc(const float *tgt_xyz, const float *tgt_shape6, long long n_tgt, const float *src_xyz,
                          const float *src_shape6, long long n_src, const double *T, double length_scale,
                          double cutoff, double sigma2, int precision, double *f, double *g, double *H,
                          long long *n_pairs, void *stream);

/*
 * Labelled pairs (eq. (rkhs_loss)): every point carries a label vector l in
 * R^label_dim (1 <= label_dim <= GCVO_MAX_LABEL_DIM: intensities, colours,
 * semantic class scores, one-hot classes), and each pair's kernel is weighted
 * by the label inner product c_ij = <l^X_i, l^Z_j>:
 *     f(T) = sum_{i,j} c_ij k(x_i, T^{-1} z_j).
 * The gradient and every Hessian carry the same weight (c_ij does not depend
 * on T).  Labels are caller-owned DEVICE memory, float32, [n][label_dim], in
 * the order of the points; they are used as given (negative weights allowed,
 * non-finite entries make the results non-finite).
 *
 * gcvo_register_batch_labeled: gcvo_register_batch with labels; pair k's labels
 * are tgt_label[tgt_off[k] .. tgt_off[k+1]) and src_label[src_off[k] ..
 * src_off[k+1]) (rows of label_dim floats).  Registering one labelled pair is a
 * batch of one.  gcvo_eval_fgh_labeled: gcvo_eval_fgh with labels.
 * The *_workspace_size_labeled functions size them (0 if invalid); other
 * arguments, outputs and errors are those of the unlabelled calls, and
 * label_dim outside 1..GCVO_MAX_LABEL_DIM is GCVO_ERR_INVALID.
 */
size_t gcvo_batch_workspace_size_labeled(int n_pairs, const long long *tgt_off, const long long *src_off,
                                         const gcvo_params *p, int shared_params, int label_dim);
int gcvo_register_batch_labeled(int n_pairs, const float *tgt_xyz, const float *tgt_label,
                                const long long *tgt_off, const float *src_xyz, const float *src_label,
                                const long long *src_off, int label_dim, const double *T_init,
                                const gcvo_params *p, int shared_params, double *T_out, gcvo_info *info,
                                void *workspace, size_t workspace_bytes, void *stream);
size_t gcvo_eval_workspace_size_labeled(long long n_tgt, long long n_src, int label_dim);
int gcvo_eval_fgh_labeled(const float *tgt_xyz, const float *tgt_shape6, const float *tgt_label, long long n_tgt,
                          const float *src_xyz, const float *src_shape6, const float *src_label, long long n_src,
                          int label_dim, const double *T, double length_scale, double cutoff, double sigma2,
                          int precision, double *f, double *g, double *H, long long *n_pairs, void *workspace,
                          size_t workspace_bytes, void *stream);

/* Bytes of device workspace gcvo_point_shapes needs; 0 if invalid. */
size_t gcvo_shapes_workspace_size(long long n);

/*
 * Per-point covariance shapes of one cloud (eq. (covariance) with Remark 1's
 * bound): for each point p, the knn nearest points of the cloud including p
 * (ties: smaller index first), M = 1/(knn-1) sum (q-p)(q-p)^T, eigenvalues
 * l1 >= l2 >= l3, S = U diag(1, max(l2/l1, rho), max(l3/l1, rho)) U^T, or S = I
 * when l1 is zero.  xyz: device float32 [n][3]; shape6_out: device float32
 * [6][n].  Does not wait on `stream`.
 */
int gcvo_point_shapes(const float *xyz, long long n, int knn, double rho, float *shape6_out,
                      void *workspace, size_t workspace_bytes, void *stream);

/*
 * Shapes of n_clouds clouds in one pass (gcvo_point_shapes for each): cloud k
 * is xyz[off[k] .. off[k+1]) (device float32 [*][3]; off HOST int64
 * [n_clouds + 1]), and its shapes go to shape6_out + 6 * off[k] as device
 * float32 [6][n_k] (the single-cloud layout, cloud after cloud).  Every cloud
 * needs at least knn points.  Does not wait on `stream`.
 */
size_t gcvo_shapes_batch_workspace_size(int n_clouds, const long long *off);
int gcvo_point_shapes_batch(int n_clouds, const float *xyz, const long long *off, int knn, double rho,
                            float *shape6_out, void *workspace, size_t workspace_bytes, void *stream);

/*
 * n_pairs evaluations (gcvo_eval_fgh for each) in one pass.  Pair k's clouds
 * are rows tgt_off[k] .. tgt_off[k+1] and src_off[k] .. src_off[k+1] of
 * tgt_xyz / src_xyz (device float32 [*][3]; offsets HOST int64 [n_pairs + 1]),
 * their shapes at tgt_shape6 + 6 * tgt_off[k] and src_shape6 + 6 * src_off[k]
 * (device float32 [6][n_k] each, the layout of gcvo_point_shapes_batch).
 * T: DEVICE double [n_pairs][16] poses, or NULL (identity); length_scale: HOST
 * double [n_pairs]; the cutoff of pair k is cutoff_scale * length_scale[k].
 * Outputs, DEVICE, each may be NULL: f [n_pairs], g [n_pairs][6], H [n_pairs][36]
 * (H_GN incl. the connection term, as gcvo_eval_fgh), n_pairs_out [n_pairs],
 * status [n_pairs] (GCVO_ERR_INVALID for a pose that is not a rigid motion,
 * whose sums are then 0).  A pair with an empty cloud has zero sums.  Written
 * on `stream` after the call returns.
 */
size_t gcvo_eval_batch_workspace_size(int n_pairs, const long long *tgt_off, const long long *src_off);
int gcvo_eval_fgh_batch(int n_pairs, const float *tgt_xyz, const float *tgt_shape6, const long long *tgt_off,
                        const float *src_xyz, const float *src_shape6, const long long *src_off, const double *T,
                        const double *length_scale, double cutoff_scale, double sigma2, int precision, double *f,
                        double *g, double *H, long long *n_pairs_out, int *status, void *workspace,
                        size_t workspace_bytes, void *stream);

/* Static text for a status code. */
const char *gcvo_strerror(int status);

/* ABI version of this header (major * 100 + minor): 200. */
int gcvo_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GCVO_H */
