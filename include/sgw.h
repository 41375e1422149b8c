/*
 * sgw.h -- C-ABI of the MI355X stochastic Galerkin wave solver.
 *
 * The library advances the intrusive stochastic Galerkin (SG) discretisation
 * of the 2-D acoustic wave equation with a log-normal squared wave speed
 * (Sec. 4, Eq. acous_sto) in time with Newmark average acceleration
 * (Sec. 2, Eq. K_T, Kuf, fparts, UmCm).  Every time step solves the SG system
 * by conjugate gradients on the interface Schur complement (Eq. Sto_Schur)
 * preconditioned by the probabilistic two-level Neumann-Neumann
 * preconditioner with a corner coarse grid (Sec. 5, Eq. Fcc_2, NNCP2),
 * the per-step loop of Alg. 1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: 0 = OK, > 0 = warning (the requested work was done),
 *   < 0 = error (nothing usable was produced).  sgw_last_error() gives text.
 * - Mesh: the unit square cut into n x n square cells, each cell split along
 *   the diagonal (i,j)-(i+1,j+1); node (i,j) at (i/n, j/n) has mesh index
 *   i + (n+1) j; u = 0 on the whole boundary (Sec. 6 setup).
 * - PCE arrays at the boundary are mode-major ("PCE-major blocks", the
 *   layout of Eq. GAssembly_Sto): element (mode j, mesh node v) sits at
 *   [j * (n+1)^2 + v], j = 0..P-1.  Boundary nodes read back as 0 and are
 *   ignored on input.  The PCE basis is the normalised Hermite chaos of total
 *   degree <= p_out in L variables, graded then descending-lexicographic.
 * - where = SGW_HOST or SGW_DEVICE says whether a pointer is host memory or
 *   device memory of the context's GPU.  The caller owns all memory it
 *   passes; the library copies what it needs and never keeps a pointer.
 * - Device memory of a context is obtained from the allocator given at
 *   create time (PyTorch's caching allocator in the Python binding), or from
 *   hipMalloc when none is given; sgw_destroy releases it.
 * - A context is not thread-safe.  Calls that take a stream enqueue on it;
 *   sgw_step and sgw_factor synchronise that stream before returning (the
 *   iteration counts decide how much work is enqueued).
 */
#ifndef SGW_H
#define SGW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SGW_OK = 0,
  SGW_NOT_CONVERGED = 1,   /* warning: a PCG hit max_iter; state advanced */
  SGW_EINVAL = -1,         /* bad argument */
  SGW_ESTATE = -2,         /* call order (e.g. step before factor) */
  SGW_ENOMEM = -3,         /* allocation failed */
  SGW_ENOTSPD = -4,        /* non-positive pivot in a Cholesky factor */
  SGW_EBREAKDOWN = -5,     /* PCG breakdown (p'q <= 0) */
  SGW_ENAN = -6,           /* NaN or Inf in a residual */
  SGW_EHIP = -7            /* HIP runtime error */
};

enum { SGW_HOST = 0, SGW_DEVICE = 1 };
enum { SGW_FP64 = 0, SGW_FP32_IR64 = 1 };
enum { SGW_GUESS_PREV = 0, SGW_GUESS_NEWMARK = 1, SGW_GUESS_LEARNED = 2 };
enum { SGW_INNER_CHOLESKY = 0, SGW_INNER_CHEBYSHEV = 1 };
/* Interface preconditioner (Sec. 5; the one-level variants are those the
 * paper compares in Sec. 6.1, defined in the thesis it cites):
 * SGW_PRECOND_NN2: the two-level Neumann-Neumann preconditioner with the
 *   corner coarse grid (Eq. NNCP2);
 * SGW_PRECOND_NN1: one-level Neumann-Neumann, sum_s R_s^T D_s S_s^{-1} D_s R_s
 *   with each subdomain's whole local (Neumann) problem, corners included,
 *   and no coarse grid (the mass term keeps every local problem
 *   nonsingular, so no floating-subdomain treatment is needed);
 * SGW_PRECOND_LUMPED: one-level lumped, S_s^{-1} replaced by the inverse of
 *   the subdomain's interface block (K~^s_GG)^{-1}. */
enum { SGW_PRECOND_NN2 = 0, SGW_PRECOND_NN1 = 1, SGW_PRECOND_LUMPED = 2 };

/* Problem description.  Fields follow the paper's problem statement:
 * Eq. CovarKer2D_chapt2 (sigma, bx, by), Eq. KLEchapt2 (L), Eq. c0pce
 * (p_in: order of the input PCE of c_s), Eq. uPCE (p_out: order of the
 * output PCE), Eq. K_T (dt, zeta, gamma), Appendix Rayleigh damping
 * (alpha0, alpha1), Eq. initial_2Dwave (pulse x0, y0, amp, with
 * alpha = width^2).  The partition is rectilinear: nsx+1 increasing cut
 * positions in cells along x (first 0, last n), likewise along y. */
typedef struct sgw_problem_desc {
  int n;                 /* cells per side */
  int nsx, nsy;          /* number of subdomain strips along x and y */
  const int* xsplits;    /* host, nsx+1 cut positions in cells */
  const int* ysplits;    /* host, nsy+1 cut positions in cells */
  int L, p_in, p_out;    /* KLE terms, input PCE order, output PCE order */
  double sigma, bx, by;  /* std. dev. and correlation lengths of g = log c_s */
  double dt, zeta, gamma;
  double alpha0, alpha1;
  double x0, y0, width, amp;   /* initial pulse (used by sgw_set_state(NULL)) */
  double rtol;           /* outer PCG: ||r|| <= rtol ||G_Gamma||; IR: on the SG residual */
  int max_iter;          /* outer PCG iteration cap */
  double inner_rtol;     /* subdomain solves: ||r_s|| <= inner_rtol ||b_s|| */
  int inner_max_iter;
  int precision;         /* SGW_FP64 or SGW_FP32_IR64 */
  int guess;             /* initial interface guess, SGW_GUESS_* (LEARNED: see below) */
  double precond_rtol;   /* Neumann solves inside the preconditioner (<= 0: inner_rtol);
                            the interface PCG is the flexible (Polak-Ribiere) variant */
  int inner_prec;        /* preconditioner I_P (x) (K~_0^s)^-1 of the subdomain SG PCG:
                            SGW_INNER_CHOLESKY applies the mean-matrix inverse exactly
                            (supernodal Cholesky factors; every nested-dissection level
                            of a subdomain <= 2048 rows), SGW_INNER_CHEBYSHEV
                            approximates it by a Chebyshev polynomial in the
                            Jacobi-scaled mean matrix (blocks of <= 4096 rows) */
  int cheb_degree;       /* degree of that polynomial (<= 0: 4; at most 64) */
  double ir_outer_rtol;  /* refinement path (SGW_FP32_IR64): FP32 interface PCG per sweep */
  double ir_inner_rtol;  /*   FP32 Dirichlet solves */
  double ir_precond_rtol;/*   FP32 Neumann solves in the preconditioner
                            (each <= 0: 1e-5, 1e-6, 1e-3) */
  int graphs;            /* != 0: subdomain PCG iterations that need no host check run
                            as replays of captured HIP graphs (pairs of iterations);
                            results are identical, timing kernels (sgw_profile) off */
  int precond;           /* interface preconditioner, SGW_PRECOND_* (0: two-level NN) */
} sgw_problem_desc;

/* Optional device allocator.  alloc returns device memory of >= bytes
 * (256-byte aligned) or NULL; free releases it. */
typedef struct sgw_allocator {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} sgw_allocator;

/* Per-call statistics (host memory, filled by sgw_step). */
typedef struct sgw_step_stats {
  int steps;             /* steps advanced by the call */
  int outer_iters;       /* total outer PCG iterations */
  int outer_iters_max;   /* max outer iterations in one step */
  long long inner_iters; /* total inner iterations (summed over solves) */
  int inner_solves;      /* number of batched subdomain solves */
  int ir_sweeps;         /* iterative-refinement sweeps (mixed precision) */
  double last_rel_res;   /* outer ||r||/||G_Gamma|| of the last solve */
} sgw_step_stats;

typedef struct sgw_ctx sgw_ctx;

/* Build a context on the current HIP device: mesh, partition into
 * subdomains (interior, remaining and corner nodes, Sec. 3 and Eq.
 * uruc_sto), KLE (Eq. KLEchapt2), log-normal PCE coefficients
 * (Eq. c0pce, LNL0), Hermite triple products (Eq. galerproject_chap2),
 * SG transient matrices (Eq. K_T_Sto, K_T_Stosub) and the mean-matrix
 * factors of every subdomain.  Host inputs are copied.  alloc may be NULL.
 * Errors: SGW_EINVAL (bad sizes / splits), SGW_ENOMEM, SGW_ENOTSPD. */
int sgw_create(const sgw_problem_desc* d, const sgw_allocator* alloc,
               sgw_ctx** out);

/* Coarse-grid setup on the device: for every subdomain and every local
 * corner degree of freedom, the SG Neumann solve that gives the coarse
 * basis and the local coarse matrix; assembly of F_cc (Eq. Fcc_2) and its
 * Cholesky factor in FP64 (with FP32 copies of the factor's blocks and an
 * FP16 copy of the coarse basis for the FP32 solver's preconditioner).
 * Once per context.  stream may be 0.  Errors: SGW_ESTATE (already
 * factored), SGW_ENOTSPD, SGW_EHIP. */
int sgw_factor(sgw_ctx* ctx, void* stream);

/* Set the state (U, V, A), each mode-major [P][(n+1)^2] in memory `where`.
 * U == NULL: U_0 = pulse in mode 0, zero elsewhere (Eq. initial_2Dwave).
 * V == NULL: V_0 = 0.  A == NULL: A_0 solved from
 * (I (x) M) A_0 = -K U_0 - C V_0 (f = 0).  Also used to resume from a
 * checkpoint taken with sgw_get_state.  Resets the step counter to step. */
int sgw_set_state(sgw_ctx* ctx, const double* U, const double* V,
                  const double* A, int where, int step, void* stream);

/* Copy the state out (mode-major [P][(n+1)^2]); any pointer may be NULL. */
int sgw_get_state(sgw_ctx* ctx, double* U, double* V, double* A, int where,
                  void* stream);

/* Advance nsteps Newmark steps (Alg. 1 loop body): effective force,
 * static condensation, interface PCG with the two-level NN preconditioner,
 * interior recovery, Newmark update.  stats may be NULL.  Returns
 * SGW_NOT_CONVERGED if any PCG hit its cap (the state still advances), or an
 * error code. */
int sgw_step(sgw_ctx* ctx, int nsteps, void* stream, sgw_step_stats* stats);

/* Several independent problems (contexts, all distinct, on this device) in
 * one call: every context advances nsteps steps on its own stream --
 * streams[i], or when streams is NULL a non-blocking stream the context
 * creates and owns -- from its own host thread, so the problems' kernels
 * overlap on the GPU.  stats and status (may be NULL) receive each
 * context's statistics and return code.  Returns the first error, else
 * SGW_NOT_CONVERGED if any context reported it, else 0. */
int sgw_step_batch(sgw_ctx** ctx, int n, int nsteps, void** streams,
                   sgw_step_stats* stats, int* status);

/* Mean (mode 0) and variance (sum of squares of modes >= 1, normalised
 * basis) of U over all (n+1)^2 mesh nodes; either pointer may be NULL. */
int sgw_read_moments(sgw_ctx* ctx, double* mean, double* var, int where,
                     void* stream);

/* Apply the SG transient operator (Eq. K_T_Sto) to X, both mode-major
 * [P][(n+1)^2] device arrays: Y = K~ X on the free nodes, 0 on the boundary.
 * precision selects the FP64 or FP32 kernel (FP32 reads and writes double
 * arrays but computes in float). */
int sgw_apply_operator(sgw_ctx* ctx, const double* X, double* Y,
                       int precision, void* stream);

/* Solve one SG system K~ U = F (Eq. Kuf with the SG operator) with the
 * full DD-PCG of sgw_step, F and U mode-major [P][(n+1)^2] device arrays;
 * U holds the initial guess on entry. */
int sgw_solve(sgw_ctx* ctx, const double* F, double* U, void* stream,
              sgw_step_stats* stats);

/* Kernel timing (tracing).  enable = n > 0 records a HIP event pair on the
 * launch stream around every n-th launch of each kind: the SG operator
 * apply (kind 0), the batched subdomain triangular solves (kind 1) and the
 * Chebyshev preconditioner (kind 2) in FP64, kinds 3, 4, 5 the same in
 * FP32; it clears the counters.  enable == 0 stops recording.  Adds two
 * event records per timed launch (the Chebyshev launches have theirs
 * recorded with the kernel's dispatch, hipExtLaunchKernelGGL). */
int sgw_profile(sgw_ctx* ctx, int enable);

/* Timed launches, their total kernel milliseconds and total algorithmic
 * bytes for one kind (0..5) since the last sgw_profile call.  Bytes per SG-apply row:
 * 7 (M+1) values + 7 column indices + P inputs + P outputs (+ P when the
 * output is accumulated), 8-byte values (4-byte in FP32 launches); per
 * triangular-solve launch: the right-hand sides in and out plus the
 * factor's values and indices; per Chebyshev launch: the right-hand sides
 * in and out plus the mean matrix's values and column indices of the
 * blocks the launch actually processes (converged blocks are skipped; the
 * kernel counts them on the device). */
int sgw_profile_read(sgw_ctx* ctx, int kind, long long* launches, double* ms,
                     double* bytes);

/* Autotuner (tile shapes picked on the context's own data): times the
 * subdomain preconditioner kernels for every feasible mode tile Q = 1..8 on
 * the Dirichlet and the Neumann systems, and the SG apply with the unrolled
 * Galerkin tensor against the table-driven one, and keeps the fastest for
 * later calls.  report (may be NULL) receives up to nreport values, in
 * microseconds per launch (-1: not feasible or not used):
 *   [0..7]   FP64 Dirichlet triangular solve, Q = 1..8
 *   [8..15]  FP64 Neumann triangular solve
 *   [16]     FP64 unrolled SG apply     [17] FP64 table-driven SG apply
 *   [18..25] FP64 Dirichlet Chebyshev   [26..33] FP64 Neumann Chebyshev
 *   [34..41] FP32 Dirichlet triangular  [42..49] FP32 Neumann triangular
 *   [50..57] FP32 Dirichlet Chebyshev   [58..65] FP32 Neumann Chebyshev
 *   [66]     FP32 unrolled SG apply     [67] FP32 table-driven SG apply
 *   [68..71] Chebyshev launch shape kept for FP64 Dirichlet, FP64 Neumann,
 *            FP32 Dirichlet, FP32 Neumann (0, 1, 2: 1024, 512, 256 threads
 *            per workgroup; -1 when not tuned)
 * (the SG applies on the Dirichlet system; a Chebyshev entry is the fastest
 * launch shape for that Q).  Enqueues on stream and waits for it. */
int sgw_autotune(sgw_ctx* ctx, void* stream, double* report, int nreport);

/* Chebyshev preconditioner tile of one subdomain system, set by hand (as
 * sgw_autotune would keep it): precision = SGW_FP64 (the FP64 systems) or
 * SGW_FP32_IR64 (the FP32 systems of the refinement path), system = 0
 * Dirichlet, 1 Neumann; q = modes per workgroup (1..8); shape = 0, 1, 2 for
 * workgroups of 1024, 512, 256 threads (1, 2 or 4 rows per thread, the
 * fewest that cover the system's largest block).  Used by the parity tests
 * of every launch shape.  Returns SGW_EINVAL (context unchanged) when the
 * combination is not feasible for the system (too many modes for the
 * registers, LDS above 150 KiB, blocks larger than 4 x the workgroup) or
 * the FP32 systems do not exist. */
int sgw_set_cheb_tile(sgw_ctx* ctx, int precision, int system, int q, int shape);

/* Sizes and counters: what = 0 P, 1 number of input PCE terms, 2 free
 * nodes, 3 interface nodes (n_gamma), 4 corner nodes, 5 subdomains,
 * 6 (n+1)^2, 7 training samples recorded since sgw_guess_record,
 * 8 learned guesses replaced by the Newmark guess, 9 graph replays,
 * 10 samples in the store of sgw_guess_train. */
long long sgw_query(const sgw_ctx* ctx, int what);

/* ---- Learned initial guess of the interface PCG ----------------------
 * The paper starts each step's interface PCG from the previous solution
 * (Alg. 1).  SGW_GUESS_LEARNED starts it from the Newmark extrapolation
 * g_{n+1} = U_n + dt V_n + dt^2/2 A_n plus a correction predicted by a small
 * network; the PCG still runs to the same tolerance, so the guess only
 * changes the iteration count.  The network is shared by every interface
 * node i and PCE mode j: its input row is the history of the node's last
 * four converged interface values, taken as their deviations from the
 * Newmark extrapolations made at those steps, c_m = u_m - g_m for
 * m = n-3..n (oldest first), divided by s_j = max_i |c_n^j(i)|; its output
 * is the next deviation c_{n+1} / s_j.  One forward pass takes the
 * n_gamma x P rows of a step.  Layers 4 -> hidden (ReLU) -> hidden (ReLU) ->
 * 1; FP32 master parameters, BF16 weights in the matrix products (MFMA, FP32
 * accumulation), Adam.  Fallbacks to g: fewer than four past steps, no
 * model attached, a non-finite prediction, or an initial residual larger
 * than that of the zero guess. */
typedef struct sgw_mlp sgw_mlp;

/* New perceptron n_in -> hidden (ReLU) -> hidden (ReLU) -> n_out
 * (He-uniform weights from the counter-based generator splitmix64 seeded
 * with seed; the last layer is scaled by 0.1; zero biases).  The solver's
 * guess needs n_in = 4, n_out = 1.  Device memory from alloc (may be
 * NULL).  Errors: SGW_EINVAL, SGW_ENOMEM, SGW_EHIP. */
int sgw_mlp_create(int n_in, int n_out, int hidden, unsigned long long seed,
                   const sgw_allocator* alloc, sgw_mlp** out);
int sgw_mlp_destroy(sgw_mlp* m);
const char* sgw_mlp_last_error(const sgw_mlp* m);
/* Number of parameters: layout [W1 (hidden x n_in, row-major), b1,
 * W2 (hidden x hidden), b2, W3 (n_out x hidden), b3]. */
long long sgw_mlp_num_params(const sgw_mlp* m);
/* Copy the FP32 parameters out (set = 0) or in (set != 0; also refreshes
 * the BF16 copies and clears the Adam moments); w in memory `where`. */
int sgw_mlp_params(sgw_mlp* m, float* w, int set, int where, void* stream);
/* y[nb][n_out] = network(x[nb][n_in]), device arrays; waits for the
 * stream. */
int sgw_mlp_forward(sgw_mlp* m, const float* x, float* y, int nb, void* stream);
/* Allocation-free variant of sgw_mlp_forward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same kernels, with the two
 * hidden activations (BF16) in a static device scratch array of 16 MiB,
 * one per GPU, held until the process ends (nb x 2 x hidden at most 4 Mi,
 * else SGW_EINVAL).  Calls no allocator and does not wait: the work is
 * enqueued on the stream.  Calls that overlap on one GPU share that scratch
 * and race. */
int sgw_mlp_forward_noalloc(sgw_mlp* m, const float* x, float* y, int nb, void* stream);
/* Mean squared error of the network on (x[nb][n_in], t[nb][n_out])
 * (host *loss) and its gradient with respect to the parameters (device
 * grad[num_params], may be NULL); waits for the stream. */
int sgw_mlp_loss_grad(sgw_mlp* m, const float* x, const float* t, int nb,
                      float* grad, float* loss, void* stream);
/* Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the mean squared error
 * over nsamples device samples, `epochs` passes in minibatches of `batch`
 * (shuffled with splitmix64 seeded with seed; a trailing partial batch is
 * skipped).  *final_loss = mean minibatch loss of the last epoch. */
int sgw_mlp_train(sgw_mlp* m, const float* x, const float* t, int nsamples,
                  int epochs, int batch, double lr, unsigned long long seed,
                  void* stream, float* final_loss);

/* Record training samples from this context's trajectory: every later step
 * with four past steps appends n_gamma x P samples (mode-major, one per
 * (mode, interface node)) -- input rows to X[capacity][4], targets to
 * T[capacity], device FP32 -- while room is left.  X = T = NULL stops
 * recording.  The count is sgw_query(ctx, 7).  The caller keeps X and T
 * alive while recording. */
int sgw_guess_record(sgw_ctx* ctx, float* X, float* T, long long capacity);

/* Attach the network used by SGW_GUESS_LEARNED (NULL detaches); it must
 * have n_in = 4 and n_out = 1.  The context does not own it. */
int sgw_set_guess_model(sgw_ctx* ctx, sgw_mlp* m);

/* Initial interface guess of later steps, SGW_GUESS_* (replaces the one
 * given at create).  Errors: SGW_EINVAL. */
int sgw_set_guess(sgw_ctx* ctx, int mode);

/* Training of the attached network on the solver's own trajectories, in
 * one call: the context advances nsteps steps from its current state
 * (sgw_set_state chooses the trajectory; the steps use the context's guess
 * mode), recording every step's samples into a store the context owns
 * (device memory from its allocator; samples of earlier calls are kept
 * unless clear != 0), then, if epochs > 0, trains the attached network with
 * Adam on every stored sample (sgw_mlp_train with these parameters).
 * *final_loss (may be NULL) receives the mean loss of the last epoch.
 * Errors: SGW_ESTATE (no model attached, no state, not factored),
 * SGW_EINVAL, SGW_ENOMEM, and those of sgw_step. */
typedef struct sgw_train_desc {
  int nsteps;               /* steps to record (>= 0) */
  int clear;                /* != 0: drop the samples of earlier calls first */
  int epochs, batch;        /* training passes and minibatch size (epochs 0: record only) */
  double lr;                /* Adam step */
  unsigned long long seed;  /* minibatch shuffling */
} sgw_train_desc;
int sgw_guess_train(sgw_ctx* ctx, const sgw_train_desc* td, void* stream,
                    float* final_loss);

/* The chaos coefficients of the current displacement U (Eq. uPCE),
 * mode-major [P][(n+1)^2] in memory `where` (same as the U of
 * sgw_get_state). */
int sgw_read_pce(sgw_ctx* ctx, double* U, int where, void* stream);

const char* sgw_last_error(const sgw_ctx* ctx);
int sgw_destroy(sgw_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SGW_H */
