/*
 * racmb.h -- C ABI of the MI355X (gfx950) RAC-MBADMM library.
 *
 * RAC-MBADMM is the randomly assembled cyclic multi-block ADMM of Zhu, Mihic and
 * Ye, "On a Randomized Multi-Block ADMM for Solving Selected Machine Learning
 * Problems" (arXiv 1907.01995).  The library solves the convex QP of Eq.(1) in
 * the split form used by the paper's machine-learning applications (Sec.3):
 *
 *     min_x  1/2 x'(F'F/Ns + diag h) x + c'x + P(z) + obj_const
 *     s.t.   a'x = b          (optional single equality row; Eq.(9)'s y'z = 0)
 *            x - z = 0        (the split of Eq.(7)/(8); z is solved as one block)
 *
 * with P = 0 (least squares), the elastic-net penalty of Eq.(6)
 * lambda*(alpha*|z|_1 + (1-alpha)/2*|z|^2), or the indicator of a box [lo, hi]
 * (the C-SVC dual of Eq.(9)).  For regression F = X (N x n) and Ns = N, so that
 * H = X'X/N and c = -X'y/N (Sec.3.1); for the linear-kernel SVM dual F = G'
 * with G = diag(y) X, Ns = 1, c = -e and a = y (Sec.3.2).
 *
 * One iteration (Eq.(3)): draw a random partition of the n variables into p
 * balanced blocks, minimise the augmented Lagrangian (Eq.(2), one penalty beta
 * on every constraint row) exactly over each block in the drawn order, then over
 * z, then take the dual step xi <- xi - beta(x - z), mu <- mu - beta(a'x - b).
 *
 * Conventions for every entry point:
 *  - Pointers documented as "device" are HIP device pointers owned by the
 *    caller; the library never frees them and reads them only during calls
 *    (a solver handle keeps borrowing the problem's pointers until destroyed).
 *  - Arrays are FP64 unless stated; F is column-major with leading dimension ldF.
 *  - Work is enqueued on the caller's stream; calls that return results
 *    synchronise that stream before returning.
 *  - Errors are returned as rac_status codes, never thrown across the ABI.
 *    A non-finite scalar argument, a non-positive beta, p < 1 or p > n, and
 *    a block larger than RAC_MAX_BLOCK give RAC_ERR_ARG.  rac_solver_create and
 *    rac_batch_create also read the problems' device arrays once (F or the sparse
 *    values or Hd, A, beq, and c, h, a) and give RAC_ERR_ARG if one holds a NaN or an
 *    infinity (on the null stream, before any other work).
 */
#ifndef RACMB_H
#define RACMB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RAC_MAX_BLOCK 128   /* largest block size ceil(n/p) the kernels accept */
#define RAC_MAX_EQ 16       /* largest number of equality rows of the dense form */
#define RAC_MLP_IN 8        /* controller features */
#define RAC_MLP_HIDDEN 64   /* controller hidden width */
#define RAC_MLP_NPARAM (RAC_MLP_HIDDEN * RAC_MLP_IN + RAC_MLP_HIDDEN + \
                        RAC_MLP_HIDDEN * RAC_MLP_HIDDEN + RAC_MLP_HIDDEN + RAC_MLP_HIDDEN + 1)

typedef enum {
  RAC_OK = 0,
  RAC_ERR_ARG = 1,         /* invalid argument (see conventions above) */
  RAC_ERR_NOT_PD = 2,      /* Assumption 2.1 violated: a block matrix H_BB + beta(I + a_B a_B')
                              had a non-positive Cholesky pivot; the failing (iteration, block)
                              is reported in rac_result */
  RAC_ERR_DEVICE = 3,      /* a HIP call failed, or a persistent kernel's bounded wait ran out */
  RAC_ERR_NOMEM = 4,       /* workspace allocation failed */
  RAC_ERR_UNSUPPORTED = 5  /* valid but not implemented (e.g. dtype/precision pair) */
} rac_status;

typedef enum { RAC_RUN_CONVERGED = 0, RAC_RUN_MAX_ITER = 1, RAC_RUN_DIVERGED = 2 } rac_run_status;
typedef enum { RAC_PROX_NONE = 0, RAC_PROX_ELASTIC_NET = 1, RAC_PROX_BOX = 2 } rac_prox;
typedef enum { RAC_DT_F64 = 0, RAC_DT_F32 = 1, RAC_DT_BF16 = 2 } rac_dtype;
/* FP64: block Grams formed in FP64.  MIXED: block Grams formed on the matrix cores
 * in the data's own precision (FP32 or BF16 inputs, FP32 accumulation), summed over
 * row chunks in FP64; gradients, residual maintenance, Cholesky pivots, duals and
 * norms stay FP64 in both modes, so the fixed point is the FP64 one. */
typedef enum { RAC_PREC_FP64 = 0, RAC_PREC_MIXED = 1 } rac_precision;
/* Penalty schedule: fixed; residual balancing (multiply by tau when r_p > mu_rb r_d,
 * divide when r_d > mu_rb r_p); the controller network (falls back to residual
 * balancing when its output is not finite); or a given per-iteration schedule. */
typedef enum { RAC_BETA_FIXED = 0, RAC_BETA_RESBAL = 1, RAC_BETA_MLP = 2, RAC_BETA_SCHEDULE = 3 } rac_beta_mode;
/* Which multi-block ADMM (Sec.1).  RAC: a fresh random partition of the variables every
 * iteration (RAC-MBADMM, Eq.(3)).  RP: the randomly permuted variant the paper compares
 * against -- the partition is fixed (block i = variables floor(i n/p) .. floor((i+1) n/p) - 1,
 * a predetermined contiguous split) and only the order in which the p blocks are solved is
 * drawn at random every iteration: the order of iteration k is the permutation of the p block
 * indices given by rac_permutation(seed, instance, k, p).  The block matrices of a fixed
 * partition change only with beta, so RP forms the block Grams once per solver and refactors
 * the blocks only when beta has changed (the saving the paper measures in Tables 1-3). */
typedef enum { RAC_VARIANT_RAC = 0, RAC_VARIANT_RP = 1 } rac_variant;

typedef struct {
  int64_t n;            /* number of variables (>= 1) */
  int64_t rows;         /* rows of F (>= 1) */
  const void* F;        /* device, column-major rows x n, element type F_dtype */
  int64_t ldF;          /* leading dimension of F (>= rows) */
  int32_t F_dtype;      /* rac_dtype */
  int32_t prox;         /* rac_prox */
  double Ns;            /* H = F'F/Ns + diag h (> 0) */
  const double* h;      /* device, n, or NULL */
  const double* c;      /* device, n */
  const double* a;      /* device, n, or NULL: the equality row a'x = b */
  double b;
  double lambda, alpha; /* elastic net: lambda >= 0, 0 <= alpha <= 1 */
  double lo, hi;        /* box bounds (lo <= hi) */
  double obj_const;     /* constant added to the reported objective */
  /* Dense form: the general QP of Eq.(1) with an explicit Hessian and several equality
   * rows (Eq.(4)).  When Hd is not NULL the quadratic is H = Hd + diag h, with Hd a
   * symmetric n x n matrix (device, column-major, leading dimension ldH >= n, element type
   * H_dtype: RAC_DT_F64 or RAC_DT_F32); F must then be NULL and rows 0, and Ns is not used.
   * The equality rows A x = beq are given as A (device, row-major meq x n, FP64) and beq
   * (device, meq) with 0 <= meq <= RAC_MAX_EQ, and a must be NULL.  In the factor form
   * (Hd NULL) meq must be 0 and the single row, if any, is a.  The Gaussian-kernel C-SVC
   * dual of Eq.(9) is this form with Hd = Q (rac_svm_kernel_matrix), meq = 1, A = y, beq = 0.
   * The dense form runs on one stream with the register-tile sweep (n up to 256 x 256 rows
   * per group); RAC_ERR_UNSUPPORTED beyond that and in a batch. */
  const void* Hd;
  int64_t ldH;
  int32_t H_dtype;
  int32_t meq;
  const double* A;
  const double* beq;
  /* Sparse factor form (the high-sparsity data of Sec.3.1, Tables 3-7): when colptr is
   * not NULL, F (rows x n) is given in compressed sparse columns: colptr (device, n + 1
   * int64, colptr[0] = 0), rowidx (device, colptr[n] int32 row indices, strictly increasing
   * within each column) and F holding the colptr[n] values (F_dtype RAC_DT_F64 or
   * RAC_DT_F32); ldF is not used.  The sparse form runs its sweep in one workgroup on one
   * stream; its residual update uses atomic additions, so iterates agree with
   * the dense computation to rounding but not bitwise from run to run. */
  const int64_t* colptr;
  const int32_t* rowidx;
} rac_problem;

typedef struct {
  int64_t num_blocks;   /* p (1 <= p <= n, ceil(n/p) <= RAC_MAX_BLOCK) */
  uint64_t seed;        /* partition seed */
  uint64_t instance;    /* instance id mixed into the partition keys */
  int32_t precision;    /* rac_precision */
  int32_t beta_mode;    /* rac_beta_mode */
  double beta0;         /* initial penalty (> 0) */
  double rb_mu, rb_tau; /* residual balancing thresholds (defaults 10, 2 when <= 0) */
  const double* beta_schedule;  /* host, max_iter entries, for RAC_BETA_SCHEDULE */
  const float* mlp_weights;     /* device, RAC_MLP_NPARAM floats, for RAC_BETA_MLP */
  double mlp_ymax;      /* bound of the controller's log multiplier (default ln 10) */
  int64_t check_every;  /* T: KKT check and penalty decision every T iterations (>= 1) */
  int64_t max_iter;     /* iteration budget of one rac_solver_run call; history capacity */
  double tol;           /* stop at the first check with KKT residual <= tol */
  int32_t sweep_groups; /* workgroups cooperating in the sweep (0 = automatic) */
  int32_t row_chunks;   /* row chunks of the block Gram contraction (0 = automatic) */
  int32_t overlap;      /* 0 (default): build the next iteration's block matrices on a second
                           stream during the sweep when all sweep groups fit on the device;
                           negative: one stream.  Overlapped solvers assume no other solver's
                           sweep runs on the device at the same time. */
  int32_t packed;       /* 0 (default): with the register-tile sweep, the Gram kernel also copies
                           each iteration's blocks into the sweep's register order (two copies of
                           about F's size, by iteration parity); negative: the sweep gathers the
                           block columns from F. */
  int32_t variant;      /* rac_variant: RAC_VARIANT_RAC (0, default) or RAC_VARIANT_RP */
  int32_t pad0;
} rac_opts;

typedef struct {
  int64_t iters;        /* iterations completed by the last run */
  int32_t status;       /* rac_run_status */
  int32_t pad0;
  double kkt;           /* KKT residual at the last check */
  double beta;          /* penalty after the last iteration */
  double objective;     /* objective at z after the run */
  int64_t fail_iter;    /* RAC_ERR_NOT_PD: failing iteration (global count) and block */
  int64_t fail_block;
} rac_result;

typedef struct rac_solver_s* rac_solver;

/* Create a solver for `prob` with options `opts` on the current HIP device.
 * Validates the arguments, allocates the workspace (partitions, block factors,
 * sweep partials, state, history) and zeroes the state (x = z = xi = 0, mu = 0).
 * The problem's device arrays are borrowed until rac_solver_destroy. */
rac_status rac_solver_create(const rac_problem* prob, const rac_opts* opts, rac_solver* out);
rac_status rac_solver_destroy(rac_solver s);

/* Run up to opts.max_iter iterations (Eq.(3)) from the current state, stopping at
 * the first KKT check <= tol, on `stream` (a hipStream_t; NULL = default stream).
 * Synchronises the stream and fills *res.  Returns RAC_ERR_NOT_PD when
 * Assumption 2.1 failed (res->fail_iter, res->fail_block name the block), and
 * RAC_ERR_DEVICE when a sweep's bounded wait for its other row groups ran out
 * (the state is then not usable; the limit can be lowered for tests through the
 * environment variable RACMB_SWEEP_MAX_SPIN, read at rac_solver_create). */
rac_status rac_solver_run(rac_solver s, void* stream, rac_result* res);

/* One call: solve `prob` with `opts` from the cold start x = z = xi = 0, mu = 0 (Eq.(3)
 * iterated until the first KKT check <= opts.tol or opts.max_iter iterations), on `stream`.
 * Creates a solver, runs it, copies the final x, z, xi (device, n doubles each; any may be
 * NULL) and mu (host, may be NULL), and destroys the solver.  *res (host) as for
 * rac_solver_run.  Errors as rac_solver_create / rac_solver_run; with RAC_ERR_NOT_PD the
 * state at the failure is still written. */
rac_status rac_solve(const rac_problem* prob, const rac_opts* opts, void* stream, double* x, double* z,
                     double* xi, double* mu, rac_result* res);

/* Copy the state in or out (device pointers, n doubles each; mu on the host).
 * Setting the state recomputes the maintained residuals u = Fx and t = a'x. */
rac_status rac_solver_set_state(rac_solver s, const double* x, const double* z, const double* xi,
                                double mu, double beta, int64_t iter, void* stream);
rac_status rac_solver_get_state(rac_solver s, double* x, double* z, double* xi, double* mu,
                                double* beta, int64_t* iter, void* stream);

/* Multipliers of the equality rows (host, count = meq in the dense form, 1 with a
 * factor-form row a, else 0; RAC_ERR_ARG for another count).  Setting them replaces the
 * multipliers of the current state (the dual variables of Eq.(3)'s last line). */
rac_status rac_solver_get_multipliers(rac_solver s, double* mu, int64_t count);
rac_status rac_solver_set_multipliers(rac_solver s, const double* mu, int64_t count);

/* Phase timing (HIP events on the run's stream, accumulated over runs until the
 * next rac_solver_set_timing call).  Phases, in order: partition draw, block Gram
 * (with the packed copy, when the solver keeps one), block factor, sweep, z/dual
 * step, KKT check + penalty rule. */
#define RAC_NUM_PHASES 6
enum { RAC_PHASE_PARTITION = 0, RAC_PHASE_GRAM = 1, RAC_PHASE_FACTOR = 2, RAC_PHASE_SWEEP = 3,
       RAC_PHASE_ZDUAL = 4, RAC_PHASE_CHECK = 5 };
rac_status rac_solver_set_timing(rac_solver s, int32_t enable);   /* also clears the totals */
/* Times only the phases whose bit (1 << RAC_PHASE_*) is set in mask (0: none); also
 * clears the totals.  Fewer events around the launches disturb the run less.
 * RAC_ERR_ARG for bits past RAC_NUM_PHASES. */
rac_status rac_solver_set_timing_mask(rac_solver s, uint32_t mask);
/* Times the per-iteration phases (Gram, factor, sweep, z/dual) only on iterations k
 * with k mod stride == 0 (stride >= 1; 1, the default, times every iteration); the
 * partition and check phases are timed at every occurrence.  Fewer event pairs
 * disturb a timed run less.  Also clears the totals.  RAC_ERR_ARG for stride < 1. */
rac_status rac_solver_set_timing_stride(rac_solver s, int64_t stride);
/* ms (host, RAC_NUM_PHASES) receives the summed milliseconds per phase, launches
 * (host, RAC_NUM_PHASES or NULL) the number of timed launches per phase. */
rac_status rac_solver_timing(rac_solver s, double* ms, int64_t* launches);
/* info (host, 8 int64): p, padded block size, sweep workgroups K, Gram row chunks R, T,
 * sweep register tile (rows per lane A, columns per wavefront B; 0 = streaming sweep),
 * and 1 if the assemble phase overlaps the sweep. */
rac_status rac_solver_info(rac_solver s, int64_t* info);

/* Controller interface for external policies and for generating training data.
 * rac_solver_features copies to host `out` (RAC_MLP_IN floats) the features that
 * the last KKT check formed from the residual history (the network's input):
 *   0.5 log10(r_p/r_d) now and at the window start, log10 of the window's change
 *   of r_p and of r_d, log10 of the KKT change since the previous check, the last
 *   log10 multiplier, (log10 KKT + 6)/3 and decisions/10, each clipped to [-4, 4].
 * rac_solver_scale_beta multiplies beta by mult (> 0) and records it as a decision,
 * exactly as the in-kernel controller does. */
rac_status rac_solver_features(rac_solver s, float* out);
rac_status rac_solver_scale_beta(rac_solver s, double mult, void* stream);

/* Per-iteration history of the last run: 4 doubles per iteration, (r_p, r_d,
 * beta, KKT or NaN), copied to host memory `out` (capacity max_iter*4). */
rac_status rac_solver_history(rac_solver s, double* out, int64_t capacity, int64_t* count);

/* Serialise / restore the complete solver state (x, z, xi, mu, t, beta, iteration
 * counter and controller memory) to / from a host buffer, for checkpoint/resume.
 * With buf == NULL, *bytes receives the size needed. */
rac_status rac_state_export(rac_solver s, void* buf, size_t* bytes);
rac_status rac_state_import(rac_solver s, const void* buf, size_t bytes);

/* The random partition of Eq.(3) for (seed, instance, iter): perm (device, n int32)
 * lists the variables sorted by their SplitMix64 key (ties by index); block i
 * holds perm[floor(i n/p) .. floor((i+1) n/p)).  Bit-identical to the oracle. */
rac_status rac_permutation(uint64_t seed, uint64_t instance, int64_t iter, int64_t n,
                           int32_t* perm, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): rac_permutation without any allocation
 * and without synchronising.  The sort's scratch is a fixed device array of this library,
 * RAC_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; n is limited to
 * RAC_NOALLOC_MAX_N (RAC_ERR_ARG beyond it, for n < 1, iter < 0 or perm == NULL).  perm
 * (device, n int32) receives the same permutation as rac_permutation gives, bit for bit,
 * once the work enqueued on `stream` has run.  Every call on a GPU uses that GPU's one
 * scratch array: calls that overlap on one GPU (concurrent streams, or host threads
 * enqueueing at once) race and must be serialised by the caller. */
#define RAC_NOALLOC_MAX_N 262144
#define RAC_NOALLOC_SCRATCH_BYTES 6291712
rac_status rac_permutation_noalloc(uint64_t seed, uint64_t instance, int64_t iter, int64_t n, int32_t* perm,
                                   void* stream);

/* Host form of rac_permutation: the same permutation, bit for bit, computed on the CPU
 * into perm (host, n int32).  No HIP call.  RAC_ERR_ARG for n < 1, n > INT32_MAX, iter < 0
 * or perm == NULL. */
rac_status rac_permutation_host(uint64_t seed, uint64_t instance, int64_t iter, int64_t n, int32_t* perm);

/* KKT residual of the split problem at (x, z, xi, mu) (device vectors, n each):
 * out[0] = max of the three parts, out[1] = primal feasibility, out[2] =
 * stationarity, out[3] = dual feasibility (host, 4 doubles).  Definitions:
 *   feas = |x-z|_inf/(1+max(|x|_inf,|z|_inf)), and |a'x-b|/(1+|b|+|a|_inf|x|_inf)
 *   stat = |F'Fx/Ns + h.x + c - xi - mu a|_inf / scale
 *   dual = dist(-xi, subdifferential of P at z) / scale
 *   scale = max(|F'Fx/Ns + h.x|_inf, |c|_inf, |xi|_inf, |mu||a|_inf, 1e-300). */
rac_status rac_kkt(const rac_problem* prob, const double* x, const double* z, const double* xi,
                   double mu, void* stream, double* out);

/* rac_kkt with every multiplier: mu (host, nmu doubles) holds one value per equality row
 * (nmu = meq in the dense form, 1 with a factor-form row a, else 0).  In the dense form the
 * equality feasibility is max_e |(A x - beq)_e| / (1 + |beq|_inf + |A|_inf |x|_inf) and the
 * multiplier term of the stationarity is A'mu. */
rac_status rac_kkt_mu(const rac_problem* prob, const double* x, const double* z, const double* xi,
                      const double* mu, int64_t nmu, void* stream, double* out);

/* Objective 1/2 z'Hz + c'z + P(z) + obj_const at device vector z (host result). */
rac_status rac_objective(const rac_problem* prob, const double* z, void* stream, double* out);

/* Regression set-up for sparse data: c = -F'y/Ns with F in compressed sparse columns
 * (colptr, rowidx, values as in rac_problem). */
rac_status rac_regression_c_csc(const int64_t* colptr, const int32_t* rowidx, const void* values, int32_t dtype,
                                int64_t rows, int64_t n, double Ns, const double* y, double* c, void* stream);

/* Regression set-up on the device: c = -F'y/Ns (y device, rows doubles). */
rac_status rac_regression_c(const void* F, int32_t F_dtype, int64_t rows, int64_t n, int64_t ldF,
                            double Ns, const double* y, double* c, void* stream);

/* Block matrices of one iteration, for inspection: writes, for each block i,
 * H_BB + beta(I + a_B a_B') (lower triangle valid, padded stride sp = the block
 * size rounded up to 16, 32, 64 or 128) to out (device, p*sp*sp doubles). */
rac_status rac_block_matrices(const rac_problem* prob, int64_t p, uint64_t seed, uint64_t instance,
                              int64_t iter, double beta, int32_t precision, double* out,
                              int64_t* sp_out, void* stream);

/* Gaussian-kernel C-SVC (Sec.3.2, Eq.(9)): the dual's Hessian
 *   Q_ij = y_i y_j exp(-gamma |x_i - x_j|^2)
 * of n training points X (device, row-major n x r: point i's r features contiguous,
 * X_dtype RAC_DT_F64 or RAC_DT_F32) with labels y (device, n, +-1), written to Q (device,
 * column-major n x n, leading dimension ldQ >= n).  Squared distances are summed in FP64
 * from the feature differences, so Q is exactly symmetric.  Pass Q as the dense form's Hd
 * (with meq = 1, A = y, beq = 0, c = -e and the box [0, C]). */
rac_status rac_svm_kernel_matrix(const void* X, int32_t X_dtype, int64_t n, int64_t r, const double* y, double gamma,
                                 double* Q, int64_t ldQ, void* stream);
/* Decision values f(v) = sum_j alpha_j y_j exp(-gamma |x_j - v|^2) + bias for m query points
 * V (device, row-major m x r, same element type as X) into f (device, m).  The bias of the
 * dual solution is minus the multiplier of y'alpha = 0 (b = -mu).  With labels (device, m)
 * and accuracy (host) non-NULL, *accuracy receives the fraction of query points whose label
 * has the sign of f (f = 0 counts as +1). */
rac_status rac_svm_decision(const void* X, int32_t X_dtype, int64_t n, int64_t r, const double* y,
                            const double* alpha, double gamma, double bias, const void* V, int64_t m, double* f,
                            const double* labels, double* accuracy, void* stream);

/* Controller network (8 -> 64 -> 64 -> 1, tanh hidden, y = ymax tanh(o)), FP32.
 * Parameters (device, RAC_MLP_NPARAM floats): W1[64][8], b1[64], W2[64][64], b2[64],
 * W3[64], b3.  Forward: feats (device, batch x 8) -> y (device, batch). */
rac_status rac_mlp_forward(const float* w, const float* feats, int64_t batch, float ymax, float* y,
                           void* stream);
/* Mean squared loss 1/(2B) sum (y - target)^2 and its gradient (device, NPARAM floats);
 * *loss (host) receives the loss. */
rac_status rac_mlp_loss_grad(const float* w, const float* feats, const float* target, int64_t batch,
                             float ymax, float* grad, double* loss, void* stream);
/* One Adam step (bias-corrected, step t >= 1) on w with moments m, v (device). */
rac_status rac_mlp_adam(float* w, const float* grad, float* m, float* v, int64_t t, float lr,
                        float b1, float b2, float eps, void* stream);

/* ------------------------------------------------------------------------
 * Batched solving: many instances of uneven size (each a rac_problem with its
 * own data) and lanes (independent solves on one instance's data, e.g. the
 * points of a lambda grid, each with its own penalty, iterate and controller),
 * advanced together with one launch per phase for the whole batch.  Lanes of an
 * instance share its partition of every iteration (drawn with the instance's
 * index as the instance id) and its block Grams F_B'F_B; block inverses, steps,
 * residuals and duals are per lane.  Each chunk of T iterations can be captured
 * once in a hipGraph and replayed.  Lanes retire individually at KKT <= tol.
 * Requirements: every instance has the same F_dtype, n_i <= 8192, block size
 * s <= 64, beta_mode FIXED, RESBAL or MLP. */
typedef struct rac_batch_s* rac_batch;
typedef struct {
  int32_t problem;      /* index of the instance this lane solves */
  int32_t prox;         /* rac_prox of this lane */
  double lambda, alpha; /* elastic-net parameters of this lane */
  double beta0;         /* initial penalty of this lane (> 0) */
} rac_lane;
typedef struct {
  int64_t block_size;   /* s (1..64): instance i has ceil(n_i/s) blocks */
  uint64_t seed;        /* partition seed */
  int32_t precision;    /* rac_precision */
  int32_t beta_mode;    /* RAC_BETA_FIXED, RAC_BETA_RESBAL or RAC_BETA_MLP */
  double rb_mu, rb_tau; /* residual balancing thresholds (defaults 10, 2 when <= 0) */
  const float* mlp_weights;     /* device, RAC_MLP_NPARAM floats, for RAC_BETA_MLP */
  double mlp_ymax;      /* default ln 10 when <= 0 */
  int64_t check_every;  /* T */
  int64_t max_iter;     /* iteration budget of one rac_batch_run call */
  double tol;           /* a lane retires at its first check with KKT <= tol */
  int32_t use_graph;    /* 1: capture a chunk of T iterations in a hipGraph and replay it */
  int32_t tune;         /* 1: time the sweep's launch layouts on this batch and keep the
                           fastest (cached per batch shape); 0: default layout.  Tuning
                           never changes results. */
  int32_t sweep;        /* sweep kernel: RAC_BSWEEP_AUTO, RAC_BSWEEP_LANE or RAC_BSWEEP_TEAM */
  int32_t pad0;
} rac_batch_opts;
/* Batched sweep kernels.  LANE: one workgroup per lane, which reads its instance's
 * data on its own.  TEAM: the lanes of an instance in groups of up to 16, advanced
 * together by a team of workgroups that split the instance's rows, so one read of
 * the data serves the whole group (FP64 matrix-core products).  A group runs on a
 * team of 16 workgroups when ceil(rows_i/16) + 15 <= 64 NT, else of 32; TEAM needs
 * ceil(rows_i/32) + 15 <= 64 NT for every instance (NT = 10 for BF16 data, 8 otherwise).
 * AUTO takes TEAM when the batch fits it, else LANE.  Requesting TEAM for a batch
 * that does not fit gives RAC_ERR_UNSUPPORTED.  The two kernels sum in different
 * orders, so their results agree to rounding, not bitwise. */
enum { RAC_BSWEEP_AUTO = 0, RAC_BSWEEP_LANE = 1, RAC_BSWEEP_TEAM = 2 };

/* ninst problems (device data borrowed until rac_batch_destroy), nlanes lanes (host). */
rac_status rac_batch_create(int32_t ninst, const rac_problem* inst, int32_t nlanes, const rac_lane* lanes,
                            const rac_batch_opts* opts, rac_batch* out);
rac_status rac_batch_destroy(rac_batch b);
/* Run up to max_iter iterations or until every lane has retired; *iters receives
 * the iterations run, *active the lanes still running (host pointers).  Lanes whose
 * block matrices violate Assumption 2.1 retire with the failing (iteration, block)
 * recorded (read it with rac_batch_lane).  Returns RAC_ERR_DEVICE when a team
 * sweep's bounded wait for another workgroup of its team ran out; the batch is then
 * not usable. */
rac_status rac_batch_run(rac_batch b, void* stream, int64_t* iters, int32_t* active);
/* Result and state of one lane: res (host) and x, z, xi (device, n_i doubles each,
 * any may be NULL).  res->status is the lane's rac_run_status (RAC_ERR_NOT_PD is
 * returned when one of its blocks violated Assumption 2.1). */
rac_status rac_batch_lane(rac_batch b, int32_t lane, rac_result* res, double* x, double* z, double* xi);
/* Warm start of one lane (a point of a regularisation path started from a neighbouring
 * point's solution, Sec.3.1): replaces the lane's x, z, xi (device, n doubles each, of its
 * instance), its multiplier mu and penalty beta (> 0), recomputes its residuals u = F x and
 * t = a'x, and restarts its controller memory and iteration count.  The lane must not have
 * retired (RAC_ERR_ARG otherwise); typically called between rac_batch_create and the first
 * rac_batch_run. */
rac_status rac_batch_set_lane_state(rac_batch b, int32_t lane, const double* x, const double* z, const double* xi,
                                    double mu, double beta);

/* Serialise / restore the state of every lane (x, z, xi, the previous z, u = F x, the
 * lanes' penalties, multipliers, controller memory and status) and the iteration counter to /
 * from a host buffer, for checkpoint/resume of a batch: a batch created with the same
 * instances, lanes and options that imports the buffer continues bit for bit as the exporting
 * batch would.  With buf == NULL, *bytes receives the size needed.  RAC_ERR_ARG for a buffer
 * that is too small or was written by a batch of another shape. */
rac_status rac_batch_state_export(rac_batch b, void* buf, size_t* bytes);
rac_status rac_batch_state_import(rac_batch b, const void* buf, size_t bytes);

/* One call: create a batch of ninst instances and nlanes lanes with opts, run it until every
 * lane has retired or opts.max_iter iterations, write each lane's result to res[u] (host,
 * nlanes) and its final x, z, xi to the device arrays x, z, xi (any may be NULL), which hold
 * the lanes' vectors one after another in lane order (lane u at offset sum_{v<u} n of lane v's
 * instance), and destroy the batch.  Returns RAC_ERR_NOT_PD when a lane retired on a failure
 * of Assumption 2.1 (its res entry names the iteration and block; the other lanes' results are
 * still written), else the errors of rac_batch_create / rac_batch_run. */
rac_status rac_solve_batch(int32_t ninst, const rac_problem* inst, int32_t nlanes, const rac_lane* lanes,
                           const rac_batch_opts* opts, void* stream, double* x, double* z, double* xi,
                           rac_result* res);

/* info (host, 10 int64): lanes, instances, block Gram tasks, inverse tasks, row
 * unroll of the LANE sweep, 1 if chunks are replayed from a hipGraph, workgroups of
 * the widest team of the TEAM sweep (0 when the LANE sweep runs), number of teams,
 * lane groups currently run solo (one workgroup each; they go to teams once few
 * lanes remain active, a decision taken from the lanes' status alone), and the block
 * Gram / inverse slots: check_every when the Grams and inverses of a whole chunk are
 * formed in one launch each at its start (the default while they fit an eighth of the
 * device memory; RACMB_ASSEMBLY_SLOTS=1 at creation disables it), else 1.  Both give
 * bit-identical results. */
rac_status rac_batch_info(rac_batch b, int64_t* info);
/* Per-phase device time of the batch's launches, as for rac_solver_set_timing /
 * rac_solver_timing (same phases; "factor" is the block inverses).  While timing is
 * enabled, chunks are launched directly rather than replayed from the hipGraph, with
 * events around every launch. */
rac_status rac_batch_set_timing(rac_batch b, int32_t enable);   /* also clears the totals */
rac_status rac_batch_timing(rac_batch b, double* ms, int64_t* launches);

const char* rac_status_str(rac_status s);

#ifdef __cplusplus
}
#endif
#endif /* RACMB_H */
