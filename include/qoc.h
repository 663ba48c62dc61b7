/*
 * qoc.h - C ABI of the MI355X second-order adjoint quantum optimal-control library.
 *
 * Problem (paper Sec. II): given a real symmetric core Hamiltonian H0 and dipole matrix M
 * (n x n), an initial state psi0 and a target psi_target (complex n-vectors), a time grid
 * of nt steps of size dt and a control model f_j = (B theta)_j sampled at t_j = j dt
 * (eq. eom, eq. Zdef), the library evaluates the discretised objective
 *
 *     C(theta) = (gamma/2) sum_{j<nt} f_j^2 + (rho/2) || a_nt - psi_target ||^2,
 *     a_{j+1} = exp(-i dt (H0 + f_j M)) a_j,  a_0 = psi0          (eq. discTDSE, discretecost)
 *
 * together with its exact gradient (Alg. 1, eq. dLdf), exact Hessian (Alg. 2, eq. d2Ldf2)
 * and Hessian-vector products.  One control direction is supported (the paper's
 * experiments use the z dipole only, Sec. II).  All arithmetic is IEEE FP64 on the GPU.
 *
 * Conventions
 *  - Every call returns qoc_status; 0 is success, negative values are errors.  No C++
 *    exception crosses this boundary.  On error, output buffers are left untouched and
 *    qoc_last_error(handle) holds a message.
 *  - Matrices are row-major.  Complex vectors are interleaved (re, im) doubles.
 *  - Host-pointer entry points copy their inputs; no pointer is retained after return.
 *    They block until results are on the host.
 *  - *_dev entry points take device pointers valid on the handle's stream and only
 *    enqueue work on that stream; the caller keeps the buffers alive until the stream
 *    has passed them.  Device-side failures of a *_dev call (Jacobi non-convergence)
 *    are reported by qoc_sync(handle); every evaluation clears the handle's device status
 *    word when it starts, so qoc_sync reports the most recent evaluation enqueued.
 *  - A handle is not thread-safe; separate handles are independent.
 *  - psi0 and psi_target are used as given (not normalised).  The Hessian is returned
 *    symmetric by construction (the two-sweep form of the second-order adjoint).
 */
#ifndef QOC_H
#define QOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qoc_status;

#define QOC_OK                  0
#define QOC_ERR_INVALID_ARG    -1  /* NULL pointer, bad size, non-finite input, dt <= 0 ...  */
#define QOC_ERR_NOT_SYMMETRIC  -2  /* |X - X^T| > 1e-12 |X| for H0 or M                      */
#define QOC_ERR_STATE          -3  /* compute called before system and basis were set          */
#define QOC_ERR_UNSUPPORTED    -4  /* n above the build limit (288) or P above 4096          */
#define QOC_ERR_NOCONV         -5  /* Jacobi sweep cap reached on some step                   */
#define QOC_ERR_DEVICE         -6  /* HIP runtime failure (message in qoc_last_error)         */
#define QOC_ERR_OOM            -7  /* device allocation failed                                 */
#define QOC_ERR_NOT_CONVERGED  -8  /* trust-region solve hit max_iter (outputs still written)  */

typedef struct qoc_problem qoc_problem;
typedef struct qoc_batch qoc_batch;

typedef enum {
    QOC_BASIS_FOURIER = 0,   /* B[j,k-1] = cos(k pi t_j/T), B[j,K+k-1] = sin(k pi t_j/T), k=1..K; P=2K */
    QOC_BASIS_IDENTITY = 1,  /* maximal model f_j = theta_j (eq. maximal): P = nt                   */
    QOC_BASIS_DENSE = 2      /* caller-supplied nt x P row-major B                                 */
} qoc_basis_kind;

/* Create a handle on HIP device `device`.  hip_stream: a hipStream_t to run on, or NULL for a
 * library-owned stream.  *out receives the handle. */
qoc_status qoc_create(int device, void* hip_stream, qoc_problem** out);
/* Release the handle and all device memory it owns.  NULL-safe. */
void qoc_destroy(qoc_problem* p);
/* Switch the stream later calls are enqueued on; NULL selects the device's null (default)
 * stream, which is also what torch's default stream is.  Synchronises the previous stream. */
qoc_status qoc_set_stream(qoc_problem* p, void* hip_stream);

/* System of eq. matrixTDSE with one control (Sec. II): h0, m are n x n real symmetric
 * (symmetry checked to 1e-12 relative); psi0, psi_target are n complex (2n doubles). */
qoc_status qoc_set_system(qoc_problem* p, int32_t n, const double* h0, const double* m,
                          const double* psi0, const double* psi_target);
/* Complex Hermitian H0 and M (the random Hermitian dipole matrices of the paper's timing runs,
 * Sec. IV-A): n x n complex, row-major, interleaved (re, im), 2 n^2 doubles each, Hermitian to
 * 1e-12 relative (QOC_ERR_NOT_SYMMETRIC otherwise; the Hermitian part (X + X^H) / 2 is used);
 * psi0, psi_target: n complex.  n <= 144.  The system is evaluated exactly through its real
 * embedding E(X) = [[Re X, -Im X], [Im X, Re X]] of size 2n: the states phi(a) = [a; -i a] / sqrt(2)
 * span an invariant subspace on which E(H0 + f M) acts as H0 + f M, and |phi(a) - phi(b)| = |a - b|,
 * so cost, gradient and Hessian are those of the complex system (every eigenvalue of the embedding
 * is doubled, which the eigen-data path handles exactly).  Targets passed later (qoc_set_target,
 * per-theta targets) have n complex entries and are mapped the same way.  qoc_step_propagators
 * returns QOC_ERR_UNSUPPORTED for such a system. */
qoc_status qoc_set_system_hermitian(qoc_problem* p, int32_t n, const double* h0, const double* m,
                                    const double* psi0, const double* psi_target);
/* Several control directions (Sec. II, eq. matrixTDSE: H0 + sum_k f^k(t) M_k; the paper has
 * K = 3, the x, y, z dipole components): m holds ndir stacked n x n real symmetric matrices
 * (ndir x n x n doubles, ndir in 1..3); h0, psi0, psi_target as for qoc_set_system, which is this
 * call with ndir = 1.  The control model then has one nt x P matrix per direction, f^k = B_k theta
 * (qoc_set_control_basis: a dense b is ndir x nt x P; the Fourier and identity models give each
 * direction its own block of parameters, P = ndir x the one-direction count), and cost, gradient,
 * Hessian (with the mixed second derivatives of eq. d2Ldf2 between directions) and HVP come from
 * every evaluation entry point.  Changing ndir clears the control basis (set it again).  With
 * ndir > 1, checkpointing, batches, qoc_hess_many_dev_noalloc, qoc_eval_controls and
 * qoc_step_propagators return QOC_ERR_UNSUPPORTED.  Errors as qoc_set_system, and
 * QOC_ERR_INVALID_ARG for ndir outside 1..3. */
qoc_status qoc_set_system_multi(qoc_problem* p, int32_t n, int32_t ndir, const double* h0, const double* m,
                                const double* psi0, const double* psi_target);
/* Replace only the target state (2n doubles); cheap, keeps all other settings. */
qoc_status qoc_set_target(qoc_problem* p, const double* psi_target);

/* Control model f(j dt; theta) (Sec. II) on a grid of nt steps of size dt (T = nt dt).
 * FOURIER: k_or_p = K >= 1, b = NULL.  IDENTITY: k_or_p ignored, b = NULL.
 * DENSE: k_or_p = P >= 1, b = nt x P row-major (copied; ndir x nt x P with several control
 * directions, see qoc_set_system_multi). */
qoc_status qoc_set_control_basis(qoc_problem* p, qoc_basis_kind kind, int32_t nt, double dt,
                                 int32_t k_or_p, const double* b);
/* Weights of eq. discretecost: gamma on the field energy (paper: 1), rho on the terminal
 * error.  Default gamma = 2 dt, rho = 2, i.e. C = dt sum f_j^2 + |a_nt - psi_target|^2. */
qoc_status qoc_set_weights(qoc_problem* p, double gamma, double rho);
/* Number of control parameters P of the current basis. */
qoc_status qoc_get_num_params(const qoc_problem* p, int32_t* num_params);

/* Cost only: forward sweep of Alg. 1 and eq. discretecost. theta: P doubles. */
qoc_status qoc_cost(qoc_problem* p, const double* theta, double* cost);
/* Cost and gradient: Alg. 1 (first-order adjoint, eq. lambdasys, eq. dLdf). */
qoc_status qoc_grad(qoc_problem* p, const double* theta, double* cost, double* grad);
/* Cost, gradient and P x P Hessian (row-major): Alg. 2 up to its assembly (eq. musys, eq. gradatheta,
 * eq. d2Ldf2).  Any of cost / grad may be NULL. */
qoc_status qoc_hess(qoc_problem* p, const double* theta, double* cost, double* grad, double* hess);
/* Hessian-vector product H(theta) v (Alg. 2's tangent and second-adjoint sweeps for a single
 * direction).  v, hv: P doubles.  grad may be NULL; if not, receives the gradient too. */
qoc_status qoc_hvp(qoc_problem* p, const double* theta, const double* v, double* hv, double* grad);
/* `count` independent theta (count x P row-major) on the same system, evaluated together.
 * costs: count, grads: count x P, hess: count x P x P; any output may be NULL. */
qoc_status qoc_hess_many(qoc_problem* p, int32_t count, const double* thetas,
                         double* costs, double* grads, double* hess);
qoc_status qoc_grad_many(qoc_problem* p, int32_t count, const double* thetas,
                         double* costs, double* grads);
/* As qoc_hess_many with one target state per theta: targets is count x 2n doubles (complex). */
qoc_status qoc_hess_many_targets(qoc_problem* p, int32_t count, const double* thetas, const double* targets,
                                 double* costs, double* grads, double* hess);

/* Evaluation at given control samples, for control models that are not linear in theta (the
 * neural-network models the paper proposes, Sec. II's model f(t; theta) with any smoothness): the
 * caller evaluates its model at the current parameters, passes the samples f (nt doubles, host)
 * and sets the model's Jacobian df/dtheta as a DENSE control basis (nt x P).  Outputs (host, each
 * may be NULL): the cost at f; grad = J^T dC/df; hess = J^T (d2C/df2) J, the part of the Hessian
 * that the second-order adjoint sweeps give (eq. d2Ldf2 with the model's first derivatives); and
 * dcdf = dC/df (nt doubles: gamma f_j + q_j), with which the caller adds the model's own
 * second-order term sum_j dcdf_j d2f_j/dtheta2.  With hess == NULL only the first-order sweeps run.
 * QOC_ERR_INVALID_ARG if f is NULL or not finite. */
qoc_status qoc_eval_controls(qoc_problem* p, const double* f, double* cost, double* grad, double* hess,
                             double* dcdf);

/* Device-pointer twins (same kernels, enqueue only, no synchronisation). */
qoc_status qoc_cost_dev(qoc_problem* p, const double* theta, double* cost);
qoc_status qoc_grad_dev(qoc_problem* p, const double* theta, double* cost, double* grad);
qoc_status qoc_hess_dev(qoc_problem* p, const double* theta, double* cost, double* grad, double* hess);
qoc_status qoc_hvp_dev(qoc_problem* p, const double* theta, const double* v, double* hv, double* grad);
qoc_status qoc_hess_many_dev(qoc_problem* p, int32_t count, const double* thetas,
                             double* costs, double* grads, double* hess);
/* Allocation-free twin of qoc_hess_many_dev, for callers that cannot allocate device memory
 * (code under HIP stream/graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results; it allocates nothing (no hipMalloc, hipFree, event or
 * library allocation): its workspace is a static 256 MiB device array that each GPU the library
 * runs on holds from the first qoc_create on that device until the process ends.  The caller
 * still passes the device inputs and outputs.  Every step's eigen-data must fit: about
 * 24 n^2 nt bytes per theta plus lower-order terms (n = 36, nt = 4000: 135 MB for one theta);
 * a larger request returns QOC_ERR_UNSUPPORTED with nothing enqueued.  All handles on one GPU
 * share that array, so calls that overlap in time on one GPU (other streams, other threads)
 * race and must be serialised by the caller; each call fully rewrites what it reads, so no
 * state carries from one call to the next.  Device-side failures are reported by qoc_sync. */
qoc_status qoc_hess_many_dev_noalloc(qoc_problem* p, int32_t count, const double* thetas,
                                     double* costs, double* grads, double* hess);
/* Wait for the handle's stream and report device-side failures of earlier *_dev calls. */
qoc_status qoc_sync(qoc_problem* p);

/* Per-step propagator data from the device eigendecomposition at step j for parameters
 * theta (test and inspection aid): u, u1, u2 receive U_j, dU_j/df, d^2U_j/df^2 as n x n
 * complex row-major (2 n^2 doubles each; any may be NULL). */
qoc_status qoc_step_propagators(qoc_problem* p, const double* theta, int32_t j,
                                double* u, double* u1, double* u2);

/* Cap on the cyclic Jacobi sweeps per step's eigendecomposition (default 40; 0..1000).  A step
 * that is not diagonal to the stopping tolerance within the cap ends the kernel normally with its
 * current rotation and raises QOC_ERR_NOCONV for the call (host-pointer calls: returned, outputs
 * untouched; *_dev calls: reported by qoc_sync).  A low cap is a way to exercise that path. */
qoc_status qoc_set_jacobi_sweep_cap(qoc_problem* p, int32_t max_sweeps);
/* Stopping tolerance of the per-step Jacobi eigendecomposition: a step is converged when its
 * largest off-diagonal entry is at most tol_rel * ||H_j||_F (default 1e-15; 0 <= tol_rel <= 1e-6).
 * A tolerance of 0 runs the sweeps until the off-diagonal part is exactly zero or the cap. */
qoc_status qoc_set_jacobi_tolerance(qoc_problem* p, double tol_rel);

/* Length of the warm-started eigen-data chains: each chain of `steps` consecutive time steps is
 * one workgroup's work, its first step decomposed from scratch and every later one from the
 * previous step's basis.  0 (default) picks the length from the batch size (enough chains to fill
 * the device, at least 8 steps each); 1..32 fixes it.  Short chains pay off when the steps are
 * far apart anyway (large control jumps between steps, e.g. the maximal model with random
 * parameters), long ones when warm starts converge in few sweeps.  Results agree to rounding.
 * QOC_ERR_INVALID_ARG outside [0, 32]. */
qoc_status qoc_set_eig_chunk(qoc_problem* p, int32_t steps);
/* Checkpoint interval (steps) for the cost / gradient / HVP paths: 0 stores every step's
 * eigen-data; k > 0 keeps only states every k steps and recomputes one segment's
 * eigen-data at a time in the backward sweep (the memory reduction the paper names as
 * future work, Sec. V). */
qoc_status qoc_set_checkpoint_interval(qoc_problem* p, int32_t steps);
/* Device bytes currently held by the handle's workspaces, and the high-water mark. */
qoc_status qoc_memory_usage(const qoc_problem* p, int64_t* current_bytes, int64_t* peak_bytes);

/* Exact-Hessian trust-region solve (the second-order optimisation step that closes Alg. 2):
 * from theta0 iterate until the gradient is below gtol on the controllable subspace, or
 * max_iter.  The radius bounds ||B p|| (the change of the sampled control).  Directions of
 * the control matrix B with singular value below 1e-7 of the largest are numerically
 * unidentifiable in parameter space (their Hessian entries fall under rounding) and are not
 * moved; stationarity is ||V_r^T grad||_2 < gtol with V_r the kept right singular vectors
 * (equal to ||grad||_2 for a well-conditioned basis).  theta_out: P doubles; cost_out,
 * iters_out may be NULL.  Returns QOC_ERR_NOT_CONVERGED (outputs written) when max_iter is
 * reached or the iteration stalls at the rounding level of the cost. */
qoc_status qoc_tr_solve(qoc_problem* p, const double* theta0, double gtol, int32_t max_iter,
                        double* theta_out, double* cost_out, int32_t* iters_out);
/* `count` independent trust-region solves advanced in lockstep (one batched Hessian evaluation
 * and one batched P x P eigendecomposition per iteration).  theta0: count x P; targets: NULL
 * (handle's target for all) or count x 2n doubles; outputs count x P / count / count / count
 * (any may be NULL except theta_out).  converged_out[i] = 1 if the stationarity test above
 * was met.
 * Returns QOC_OK even if some solves did not converge (see converged_out). */
qoc_status qoc_tr_solve_many(qoc_problem* p, int32_t count, const double* theta0, const double* targets,
                             double gtol, int32_t max_iter, double* theta_out, double* cost_out,
                             int32_t* iters_out, int32_t* converged_out);

/* Subproblem solver of both trust-region solvers.  DEFAULT: the exact solver minimises the
 * model on the ball through an eigendecomposition of the (whitened) Hessian on the device, the
 * BFGS solver takes the dogleg step.  CG: both take the Steihaug-Toint truncated conjugate-
 * gradient step (Nocedal & Wright 2006, Alg. 7.2), which needs matrix-vector products only, so
 * the two solvers differ in nothing but the Hessian they are given. */
typedef enum {
  QOC_TR_SUBPROBLEM_DEFAULT = 0,
  QOC_TR_SUBPROBLEM_CG = 1,
} qoc_tr_subproblem;
qoc_status qoc_set_tr_subproblem(qoc_problem* p, int32_t kind);

/* Step tolerance of both trust-region solvers (the paper's delta test on the parameter change,
 * Alg. 1 and Alg. 2 stopping rules): a solve also stops, unconverged unless the gradient test
 * holds, once the step it just evaluated is shorter than xtol (theta 2-norm) or its radius has
 * shrunk below xtol.  Default 0 (off).  QOC_ERR_INVALID_ARG unless xtol is finite and >= 0. */
qoc_status qoc_set_tr_step_tolerance(qoc_problem* p, double xtol);

/* Quasi-Newton twin of qoc_tr_solve_many for the paper's comparison of Alg. 1 (gradient by the
 * first-order adjoint) with Alg. 2 (exact Hessian) (Sec. IV-B): the same trust region, ratio
 * test, radius rules and stopping test, with the Hessian replaced by a BFGS approximation
 * (first update scaled by y^T y / y^T s; updates without positive curvature skipped) and the
 * subproblem solved by the dogleg path.  Each iteration costs one gradient evaluation per active
 * solve.  Arguments, outputs and return value as qoc_tr_solve_many; iters_out counts evaluated
 * trial points (accepted or not). */
qoc_status qoc_tr_solve_bfgs_many(qoc_problem* p, int32_t count, const double* theta0, const double* targets,
                                  double gtol, int32_t max_iter, double* theta_out, double* cost_out,
                                  int32_t* iters_out, int32_t* converged_out);
/* The BFGS update used by qoc_tr_solve_bfgs_many (host arithmetic, no device): with s^T y > 0,
 * b <- b - (b s)(b s)^T / (s^T b s) + y y^T / (y^T s) and h <- its inverse update (r x r row-major,
 * h = b^{-1} on entry); rescale != 0 first resets b = (y^T y / y^T s) I and h = b^{-1}.
 * QOC_ERR_INVALID_ARG if s^T y <= 0 or a pointer is NULL. */
qoc_status qoc_bfgs_update(int32_t r, double* b, double* h, const double* s, const double* y, int32_t rescale);

/* Both stationarity measures of `count` gradients (count x P): gnorm_out[i] = ||g_i||_2 and
 * proj_out[i] = ||V_r^T g_i||_2, the measure the trust-region solve stops on (either output may
 * be NULL).  They agree for a well-conditioned control basis. */
qoc_status qoc_tr_gradient_norms(qoc_problem* p, int32_t count, const double* grads, double* gnorm_out,
                                 double* proj_out);

/* Coordinates of the trust-region metric: c = diag(sigma_r) V_r^T theta (count x P doubles
 * out; entries past the rank are 0), so that ||c|| = ||B theta|| on the kept subspace, and the
 * parameters theta = V_r diag(1/sigma_r) c that map back (the minimum-norm representative).
 * rank (may be NULL) receives the number of kept directions.  Used to give a learned warm
 * start well-conditioned regression targets. */
qoc_status qoc_control_coords(qoc_problem* p, int32_t count, const double* theta, double* coords, int32_t* rank);
qoc_status qoc_params_from_coords(qoc_problem* p, int32_t count, const double* coords, double* theta);

/* Batched evaluation of independent problems of uneven (n, nt, P): cost, gradient and Hessian
 * of every problem at its own theta.  Problems are grouped by n; each group runs as a chain of
 * persistent queue launches (one per phase of the evaluation: controls, eigen-data, chunk
 * joins, forward sweep, terminal, backward sweep, U'' contraction, assembly) whose workgroups
 * pull (problem, block) items longest first.  The chains run concurrently on their own streams
 * and the whole sequence is captured as one HIP graph on first use and replayed afterwards.
 * problems: `count` configured handles on `device`; the batch copies their systems, bases and
 * weights (later changes to the handles do not affect it) and owns one workspace per problem
 * (every step's eigen-data is stored: about 24 n^2 nt bytes per problem).
 * Errors: QOC_ERR_INVALID_ARG (NULL, count < 1, a handle on another device), QOC_ERR_STATE (a
 * handle without system or basis), QOC_ERR_UNSUPPORTED (a problem with n > 128, the batch's
 * size limit; single handles go to 288), QOC_ERR_OOM / QOC_ERR_DEVICE. */
qoc_status qoc_batch_create(int device, int32_t count, qoc_problem* const* problems, qoc_batch** out);
void       qoc_batch_destroy(qoc_batch* b);   /* NULL-safe */
/* thetas[i]: P_i doubles (host); costs[i] (1), grads[i] (P_i), hessians[i] (P_i x P_i row-major)
 * are host outputs, any may be NULL (hessians itself may be NULL).  Synchronous. */
qoc_status qoc_batch_hess(qoc_batch* b, const double* const* thetas, double* const* costs,
                          double* const* grads, double* const* hessians);
/* Same results through one launch sequence per problem (the reference point of the batched
 * launch; same kernels, same tuning). */
qoc_status qoc_batch_hess_unbatched(qoc_batch* b, const double* const* thetas, double* const* costs,
                                    double* const* grads, double* const* hessians);
/* Autotuner: on a sample of each (n, P) group (its 4 longest problems) it times the group's
 * eigen phase over candidate chunk lengths {8, 16, 32} and its sweeps over candidate tangent
 * columns per workgroup {2..32} at these thetas, keeps the fastest for the whole group, and
 * rebuilds the launch plan (the graph is recaptured on the next call). */
qoc_status qoc_batch_autotune(qoc_batch* b, const double* const* thetas);
/* Tuning in use for problem i (columns per sweep workgroup, eigen chunk length); set overrides
 * it (pg in [1, 32]; chunk in [8, 32], or [16, 32] for n > 64: the longest chain of warm-started
 * eigendecompositions is 32 steps, after which a chunk restarts cold). */
qoc_status qoc_batch_get_config(const qoc_batch* b, int32_t i, int32_t* pg, int32_t* chunk);
qoc_status qoc_batch_set_config(qoc_batch* b, int32_t i, int32_t pg, int32_t chunk);
/* Device time (HIP events) of the last qoc_batch_hess / _unbatched call's launches, in ms. */
qoc_status qoc_batch_last_ms(const qoc_batch* b, double* ms);
qoc_status qoc_batch_memory(const qoc_batch* b, int64_t* bytes);
const char* qoc_batch_last_error(const qoc_batch* b);

/* Per-kernel timing with HIP events recorded around every launch on the handle's stream.
 * qoc_profile_enable(p, 1) starts recording (and clears earlier totals), 0 stops.
 * qoc_profile_kernel_ms: total milliseconds and launch count since enabling, for one of
 * "controls", "eig", "boundary", "forward", "terminal", "backward", "sterm", "assemble"
 * (synchronises the stream).  Unknown names give 0 ms and 0 launches. */
qoc_status qoc_profile_enable(qoc_problem* p, int32_t on);
qoc_status qoc_profile_kernel_ms(qoc_problem* p, const char* kernel, double* total_ms, int32_t* launches);

/* Eigensolver statistics accumulated since the last reset (inspection aid): number of
 * per-step decompositions that converged and the Jacobi sweeps they took.  reset != 0
 * clears the counters after reading. */
qoc_status qoc_jacobi_stats(qoc_problem* p, int64_t* steps, int64_t* sweeps, int32_t reset);

/* ---- Learned warm start: 3-layer MLP n_in -> n_hidden -> n_hidden -> n_out with erf-GELU,
 * BF16 matrix-core products with FP32 accumulation, FP32 master weights and Adam.
 * Parameters are packed FP32 [W1 (hidden x in, row-major), b1, W2, b2, W3, b3].  All x / t / y
 * / loss pointers are device pointers of FP32 row-major batches on the handle's stream.
 * create: hip_stream is the stream every later call is enqueued on (NULL: the null stream);
 * max_batch bounds `batch` in the calls below (activation buffers are sized for it). */
typedef struct qoc_mlp qoc_mlp;
qoc_status qoc_mlp_create(int device, void* hip_stream, int32_t n_in, int32_t n_hidden, int32_t n_out,
                          int32_t max_batch, qoc_mlp** out);
void       qoc_mlp_destroy(qoc_mlp* h);
int64_t    qoc_mlp_num_params(const qoc_mlp* h);
qoc_status qoc_mlp_set_params(qoc_mlp* h, const float* params_host);   /* also resets Adam state */
qoc_status qoc_mlp_get_params(qoc_mlp* h, float* params_host);
qoc_status qoc_mlp_get_grads(qoc_mlp* h, float* grads_host);           /* of the last loss_grad / train_step */
/* y = MLP(x) for `batch` rows. */
qoc_status qoc_mlp_forward(qoc_mlp* h, int32_t batch, const float* x_dev, float* y_dev);
/* Mean-squared-error loss against t and its gradient with respect to every parameter. */
qoc_status qoc_mlp_loss_grad(qoc_mlp* h, int32_t batch, const float* x_dev, const float* t_dev, float* loss_dev);
/* loss_grad followed by one Adam step (bias-corrected) on the FP32 masters. */
qoc_status qoc_mlp_train_step(qoc_mlp* h, int32_t batch, const float* x_dev, const float* t_dev, float lr,
                              float beta1, float beta2, float eps, float* loss_dev);
qoc_status qoc_mlp_sync(qoc_mlp* h);
const char* qoc_mlp_last_error(const qoc_mlp* h);

/* Static strings; never NULL. */
const char* qoc_status_string(qoc_status s);
const char* qoc_last_error(const qoc_problem* p);

#ifdef __cplusplus
}
#endif
#endif /* QOC_H */
