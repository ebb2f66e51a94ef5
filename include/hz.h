/*
 * hz.h -- C ABI of the MI355X twogrid-preconditioned FGMRES Helmholtz solver.
 *
 * Method (Drzisga, Koeppl, Wohlmuth, arXiv 2104.01439):
 *   * problem (Sec. 2, the impedance boundary value problem and its variational form):
 *       -Laplace u - k^2 u = f in the unit square,  du/dn - i k u = g on its boundary,
 *     discretised with P_p Lagrange elements (p = 1, 2, 3) on the uniform mesh whose square
 *     cells are split by their "/" diagonal; system matrix A(k, eps) = K - M(k, eps) - i B(k)
 *     (Sec. 2, definition of the system matrix).
 *   * preconditioner (Sec. 4, Algorithm 1 with two levels): one V(nu, nu)-cycle on the shifted
 *     operator A_eps with damped Jacobi smoothing, FE prolongation P, restriction P^T and an
 *     exact coarse solve on the 2h mesh. The shift is passed as a complex multiplier s of the
 *     k^2 mass term: A_eps = K - s k^2 M - i k B, i.e. eps = Im(s) k^2 when Re(s) = 1; the
 *     boundary term is not shifted (the shifted problem of Sec. 2 keeps the impedance
 *     condition). The fine level is matrix-free; the coarse operator is assembled as a
 *     block-tridiagonal matrix and factored on the device.
 *   * outer solver (Sec. 4, after Saad 1993): right-preconditioned flexible GMRES(restart)
 *     on A_0 = A(k, 0), zero initial guess, stopping on the relative residual (Sec. 5, the
 *     residual of the unpreconditioned system).
 *
 * Conventions shared by every entry point
 *   * Vectors are complex, interleaved (re, im), hz_c64 == std::complex<double> ==
 *     torch.complex128. A fine vector holds N = M*M values, M = p*n + 1, n = 1/h; the value of
 *     lattice point (a, b), located at (a h/p, b h/p), sits at index b*M + a. A coarse vector
 *     has the same layout with n/2 cells (Mc = p*n/2 + 1).
 *   * Pointers named d_* are DEVICE pointers owned by the caller; h_* are host pointers.
 *     The library owns everything inside hz_problem / hz_engine and frees it on destroy.
 *   * hip_stream is a hipStream_t (NULL = the default stream). Calls are asynchronous with
 *     respect to the host unless stated; hz_solve* synchronise the stream before returning.
 *   * No exception crosses the ABI. Every call returns a status; hz_last_error() gives a
 *     human-readable message for the calling thread. Non-convergence is not an error.
 *   * One problem must not be used by two threads at once; a concurrent call returns HZ_EBUSY.
 *     Different problems may be used from different threads and streams: the library orders
 *     its persistent coarse-solve launches on one device one after another (they must not be
 *     resident together), whatever streams they are issued on.
 */
#ifndef HZ_H
#define HZ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hz_problem hz_problem;
typedef struct hz_engine hz_engine;

typedef struct { double re, im; } hz_c64;

typedef enum {
  HZ_OK = 0,
  HZ_EINVAL = 1,      /* invalid argument (bad sizes, NaN input, Im(s) <= 0, ...) */
  HZ_ENOMEM = 2,      /* device allocation failed or a budget would be exceeded   */
  HZ_EDEVICE = 3,     /* HIP runtime error                                        */
  HZ_ESINGULAR = 4,   /* zero or non-finite pivot in the coarse factorisation     */
  HZ_EBUSY = 5        /* the object is in use by another call                     */
} hz_status;

typedef enum {
  HZ_FP64 = 0,        /* everything in complex FP64                                        */
  HZ_MIXED = 1        /* preconditioner (fine stencils, smoother, transfers, coarse
                         triangular solves) in complex FP32 with FP32 accumulation; outer
                         FGMRES, A_0, Arnoldi and Givens in FP64; coarse factor computed in
                         FP64 and stored in FP32 for the solves                              */
} hz_precision;

typedef struct {
  int nu;             /* pre- and post-smoothing sweeps (Algorithm 1); default 2          */
  double omega;       /* Jacobi damping; default 0.6                                      */
  int restart;        /* FGMRES restart length m (1..64); default 50                      */
  int maxit;          /* cap on the total number of preconditioner applications; 5000    */
  double tol;         /* relative residual tolerance; default 1e-8                        */
  int prec;           /* hz_precision; default HZ_FP64                                    */
  int timing;         /* nonzero at creation: record device time of the coarse solves   */
} hz_options;

typedef struct {
  int iterations;       /* preconditioner applications, summed over restart cycles          */
  int converged;        /* 1 if the true relative residual reached tol, else 0              */
  double rel_res_true;  /* ||F - A_0 u|| / ||F|| recomputed at exit                          */
  double rel_res_est;   /* last Givens estimate |g_{j+1}| / ||F||                            */
  double setup_s;       /* wall seconds spent in hz_create_problem (coarse factor included) */
  double solve_s;       /* wall seconds of this solve                                        */
} hz_result;

/* Counters of one problem (device times filled when created with timing != 0). A batched
 * solve books the coarse-solve launches of all its problems on its first problem. */
typedef struct {
  long vcycles;              /* V-cycles run by solves and by hz_apply(HZ_OP_VCYCLE)      */
  long coarse_solves;        /* kernel launches of the coarse direct solves                */
  double coarse_solve_ms;    /* their summed device time (HIP events around each solve)   */
  double factor_ms;          /* device time of the coarse assembly and factorisation       */
  double coarse_bytes;       /* algorithmic bytes of those solves: every stored factor
                                entry read once (multifrontal: S and G^T forward, G
                                backward; block-tridiagonal: each inverse twice, the last
                                once) plus 3 coarse vectors per right-hand side             */
  long graph_rounds;         /* FGMRES rounds replayed from a captured HIP graph           */
  long coarse_systems;       /* coarse systems solved (right-hand sides of those solves)   */
  double factor_flop;        /* algorithmic flops of the factorisation (complex
                                multiply-adds of the inverses and products, 8 flops each)  */
} hz_stats;

/* Operators exposed by hz_apply (parity hooks; all act on the problem's own data). Each is one
 * building block of the twogrid cycle of Sec. 4, Algorithm 1 (two levels) or of the system
 * matrix of Sec. 2. */
typedef enum {
  HZ_OP_A0 = 0,             /* y = A_0 x: the unshifted system matrix A(k, 0) of Sec. 2,
                               applied matrix-free                  (fine -> fine)     */
  HZ_OP_AEPS = 1,           /* y = A_eps x: the shifted matrix A(k, eps) of Sec. 2
                                                                    (fine -> fine)     */
  HZ_OP_JACOBI = 2,         /* y = x + omega D^-1 (f - A_eps x), D = diag(A_eps): one
                               damped Jacobi sweep, the smoother S of Algorithm 1       */
  HZ_OP_RESTRICT = 3,       /* y = P^T x: the restriction of Algorithm 1 (transpose of
                               the FE prolongation of nested spaces, Sec. 4)
                                                                    (fine -> coarse)   */
  HZ_OP_PROLONG = 4,        /* y = P x: the FE prolongation (coarse grid correction of
                               Algorithm 1)                         (coarse -> fine)   */
  HZ_OP_VCYCLE = 5,         /* y = V-cycle(x) from a zero initial guess: Algorithm 1 with
                               two levels, the preconditioner of Sec. 4 (fine -> fine) */
  HZ_OP_COARSE_SOLVE = 6,   /* y = (A_eps^{2h})^-1 x: the direct solve on the coarsest
                               level of Algorithm 1, with the factor computed once at
                               creation (Sec. 6 factors it once and reuses it)
                                                                    (coarse -> coarse) */
  HZ_OP_COARSE_A = 7,       /* y = A_eps^{2h} x: the shifted matrix of Sec. 2 rediscretised
                               on the 2h mesh (Sec. 4)              (coarse -> coarse) */
  HZ_OP_RESID_RESTRICT = 8  /* y = P^T (f - A_eps x): the "restrict residual" step of
                               Algorithm 1                          (fine -> coarse)   */
} hz_op;

/* Fills the defaults listed in hz_options. */
hz_status hz_default_options(hz_options* o);

/* Creates the discrete problem of Sec. 2 (the impedance boundary value problem, its
 * sesquilinear form and the system matrix A(k, eps) = K - M(k, eps) - i B(k)) together with
 * the twogrid preconditioner of Sec. 4, Algorithm 1 (coarse operator rediscretised on the
 * 2h mesh and factored once, as Sec. 6 does in the first FGMRES iteration).
 * Creates a problem for wavenumber k > 0 on n = 1/h cells per side (1/h must be an even
 * integer >= 2, up to 4096), element order p in {1,2,3} and shift multiplier s with
 * Im(s) > 0 (required: the coarse block LU runs without pivoting, which is safe because the
 * Hermitian part of i*A_eps is Im(s) k^2 M + k B, positive definite). Builds the stencil
 * tables, assembles and factors the coarse operator on the device and allocates the V-cycle
 * scratch (and keeps only an FP32 copy of the factor when o->prec == HZ_MIXED). o->restart
 * is the largest restart length later solves may use; the Krylov workspace of hz_solve is
 * allocated by the first hz_solve and kept until destruction. On success *out owns all of
 * it. Synchronises hip_stream. Errors: HZ_EINVAL, HZ_ENOMEM, HZ_ESINGULAR, HZ_EDEVICE; *out
 * is left NULL. */
hz_status hz_create_problem(double k, double h, int p, hz_c64 s, const hz_options* o,
                            void* hip_stream, hz_problem** out);

/* The heterogeneous-wavenumber problem of Sec. 6 (the setting of its numerical results:
 * k(x) = k_max mu(x), to be solved with a shift that follows the local k). k and the shift
 * multiplier are constant on every cell of the n x n fine mesh (n = 1/h):
 * k_cell[j * n + i] > 0 and s_cell[j * n + i] (Im > 0) for the cell [i h, (i+1) h] x
 * [j h, (j+1) h], host arrays read during the call. The system matrix becomes
 *   A_s = K - sum_c s_c k_c^2 M_c - i sum_{boundary edges e} k_e B_e
 * (M_c the mass matrix of cell c, k_e the k of the cell that edge e bounds); FGMRES runs on
 * A_0 (all s_c = 1), the twogrid cycle of Sec. 4, Algorithm 1 on A_s with the Galerkin coarse
 * operator P^T A_s P (the coarse form with the fine coefficient integrated exactly), factored
 * once as for hz_create_problem. Both levels store one stencil per lattice point, assembled
 * on the device. Every other entry point takes the returned problem as it takes one from
 * hz_create_problem (hz_solve_batched requires all problems of a batch to be of one kind);
 * hz_problem_info reports the largest k_cell as k. Errors as hz_create_problem (HZ_EINVAL
 * names the first invalid cell). Synchronises hip_stream. */
hz_status hz_create_problem_cells(const double* k_cell, const hz_c64* s_cell, double h, int p,
                                  const hz_options* o, void* hip_stream, hz_problem** out);

/* Load vector of the point source of Sec. 6, f(x) = amp exp(-width |x - (sx, sy)|^2) with
 * g = 0 (the paper takes amp = 2, width = 1000): F_i = integral of f phi_i, on every triangle
 * by the collapsed 6 x 6 Gauss-Legendre rule (Duffy). d_F: fine vector (device); any problem
 * (constant or per-cell k). Asynchronous on hip_stream. Errors: HZ_EINVAL for a null
 * argument or non-finite parameters (width must be >= 0). */
hz_status hz_gaussian_rhs(const hz_problem* pr, double sx, double sy, double amp, double width,
                          hz_c64* d_F, void* hip_stream);

/* Sizes of a created problem: fine dofs, coarse dofs, device bytes held. */
hz_status hz_problem_info(const hz_problem* pr, long* n_dofs, long* n_coarse,
                          size_t* footprint_bytes);

/* Device bytes a problem with these parameters holds after its first hz_solve (factor,
 * tables, scratch, Krylov workspace; no allocation); 0 for invalid parameters. Used for
 * admission by footprint. */
size_t hz_footprint_estimate(double k, double h, int p, const hz_options* o);

/* Writes the load vector of the plane-wave impedance data into d_F (fine vector):
 * F_i = integral over the boundary of g phi_i (Sec. 2, the linear form with f = 0),
 * g = du/dn - i k u for u = exp(i k (x cos(theta) + y sin(theta))); each boundary edge is
 * integrated with 10-point Gauss-Legendre. Asynchronous on hip_stream. */
hz_status hz_planewave_rhs(const hz_problem* pr, double theta, hz_c64* d_F, void* hip_stream);

/* The outer solve of Sec. 4: right-preconditioned flexible GMRES (after Saad 1993) on the
 * unshifted system, one twogrid V-cycle of Algorithm 1 on A_eps as the preconditioner, and the
 * stopping rule of Sec. 5 (relative residual of the unpreconditioned system).
 * Solves A_0 u = F by FGMRES(o->restart) preconditioned with the twogrid V-cycle; zero
 * initial guess; stops when the relative residual is <= o->tol (the rotation estimate inside
 * a cycle, confirmed by the recomputed true residual), or after o->maxit preconditioner
 * applications (then converged = 0, status HZ_OK). o->nu and o->omega are those given at
 * creation. d_F, d_u: fine vectors (d_u is overwritten). h_res_hist (nullable) receives one
 * relative residual estimate per iteration and must hold o->maxit doubles. A zero F gives
 * u = 0 after 0 iterations; a non-finite ||F|| returns HZ_EINVAL. Synchronises hip_stream. */
hz_status hz_solve(hz_problem* pr, const hz_c64* d_F, hz_c64* d_u, const hz_options* o,
                   hz_result* res, double* h_res_hist, void* hip_stream);

/* Applies one building block of Sec. 4, Algorithm 1 or of the system matrix of Sec. 2 (the
 * passage of each is named at its hz_op value). d_x, d_y: device vectors of the
 * op's input and output spaces; d_f: the second input of HZ_OP_JACOBI and
 * HZ_OP_RESID_RESTRICT (ignored otherwise, may be NULL). prec selects the FP64 or FP32
 * kernels; I/O is always complex FP64 (converted on the device for FP32). d_y must not alias
 * d_x or d_f. Asynchronous on hip_stream. */
hz_status hz_apply(const hz_problem* pr, int op, const hz_c64* d_x, const hz_c64* d_f,
                   hz_c64* d_y, int prec, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): hz_apply without any allocation. Same operators,
 * arguments, layouts, results (the same kernels with the same arithmetic) and errors as
 * hz_apply, plus:
 *   * the kernels' scratch (V-cycle iterates, residual, coarse vectors, the coarse solve's
 *     update vectors and timeout flag, FP32 staging) lives in one fixed device array
 *     of 64 MiB per GPU, held from the first call on that GPU until the process ends; a
 *     problem needing more (above about 0.96 M fine dofs in FP64, 0.86 M in HZ_MIXED for P1) is
 *     rejected with HZ_EINVAL and a message giving both sizes;
 *   * HZ_MIXED needs the problem's FP32 coarse factor to exist already (a problem created
 *     with HZ_MIXED, or one mixed hz_apply / hz_solve earlier), else HZ_EINVAL;
 *   * no timing is booked and the stencil autotuner times nothing (the cached choice, else
 *     the default tile; every tile gives the same result);
 *   * every call on one GPU shares that GPU's array: calls that overlap on one GPU (other
 *     streams or threads, before the previous call's kernels have completed) race and give
 *     undefined results. Serialise them, e.g. by issuing them all on one stream.
 * The first call on a device looks up the array's device address (no allocation). */
hz_status hz_apply_noalloc(const hz_problem* pr, int op, const hz_c64* d_x, const hz_c64* d_f,
                           hz_c64* d_y, int prec, void* hip_stream);

/* Many independent solves of the method at once: the sample generation of Sec. 5 runs one
 * FGMRES solve (Sec. 4) per (k, h, p, shift) sample and right-hand side.
 * Runs nprob * nrhs_per_prob independent FGMRES solves (the same method as hz_solve) in
 * lockstep: solve (i, r) uses problem probs[i] and right-hand side d_F[i*nrhs_per_prob + r],
 * writing d_u[i*nrhs_per_prob + r] and res[i*nrhs_per_prob + r]. Each round performs one
 * Arnoldi step of every unfinished solve: the V-cycles of one problem's right-hand sides run
 * as one batch whose coarse triangular solves read the factor once per group of up to 4
 * right-hand sides; A_0 and the Arnoldi kernels are launched once for all solves; the host
 * reads back once per round. Solves finish (or restart) independently. Every result is
 * bitwise what hz_solve gives for that solve alone (same kernels' arithmetic, same order).
 * Requirements: the problems are distinct, share (h, p) (the wavenumbers may differ), were
 * created with restart >= o->restart and, for HZ_FP64, with HZ_FP64; at most 4096 solves;
 * d_F and d_u are fine vectors (d_u may not alias any d_F). The call allocates a workspace of
 * hz_batch_workspace_bytes(...) device bytes and frees it before returning. Errors as
 * hz_solve, HZ_EBUSY if a problem is in use, HZ_ENOMEM if the workspace does not fit.
 * Synchronises hip_stream. */
hz_status hz_solve_batched(hz_problem* const* probs, int nprob, const hz_c64* const* d_F,
                           int nrhs_per_prob, hz_c64* const* d_u, const hz_options* o,
                           hz_result* res, void* hip_stream);

/* Device bytes of the workspace hz_solve_batched allocates for nprob problems of mesh size h
 * and order p with nrhs_per_prob right-hand sides each (restart and precision from o, NULL
 * = defaults); 0 for invalid parameters. */
size_t hz_batch_workspace_bytes(double h, int p, int nprob, int nrhs_per_prob,
                                const hz_options* o);

/* ---------------------------------------------------------------------------------------
 * Serving engine (the many-sample form of Sec. 5): requests of any (k, h, p, shift) are
 * queued, admitted in arrival order while a slot and the device-memory budget allow, set up
 * (tables, coarse factor) on setup threads with their own streams while the admitted
 * requests iterate, and solved by continuous batching: every round performs one FGMRES
 * iteration of each active request and synchronises once; finished requests leave between
 * rounds and free their memory, new ones join. Each request runs exactly the arithmetic of
 * hz_solve (its result is the same alone and in any mix). Options (restart, tol, maxit,
 * precision, nu, omega) are the engine's, fixed at creation.
 * --------------------------------------------------------------------------------------- */
typedef struct {
  size_t hbm_budget;   /* device bytes the engine may hold; 0 = 85 % of the free memory    */
  int max_active;      /* requests admitted at once (set up or iterating); default 64      */
  int setup_threads;   /* host threads preparing admitted requests; default 2              */
} hz_engine_config;

typedef struct {
  long id;              /* the req_id given to hz_engine_submit                            */
  int status;           /* HZ_OK, or the error that ended the request (then see message)   */
  hz_result result;     /* iterations, residuals; setup_s = creation, solve_s = iterations */
  double queue_s;       /* wall seconds from submission to admission                       */
  double latency_s;     /* wall seconds from submission to completion                      */
  char message[120];    /* error text when status != HZ_OK                                  */
} hz_engine_result;

typedef struct {
  int queued, admitted;        /* waiting for admission; admitted and not finished          */
  size_t bytes_in_use, hbm_budget;
  long submitted, completed;
} hz_engine_info_t;

hz_status hz_engine_default_config(hz_engine_config* c);

/* Starts an engine on the calling thread's current device (its own streams and threads).
 * o: solver options for every request (NULL = defaults). Errors: HZ_EINVAL, HZ_EDEVICE. */
hz_status hz_engine_create(const hz_engine_config* c, const hz_options* o, hz_engine** out);

/* Queues one solve of A_0(k, h, p) u = F preconditioned with shift s. F is the plane-wave
 * load for angle theta when d_F is NULL, else a copy of the fine vector d_F taken at setup
 * (d_F must stay valid until the request is reported). The solution is written to d_u (a
 * caller-owned fine vector that must stay valid and untouched until the request is
 * reported; it is complete when hz_engine_poll returns it); with d_u NULL only the result
 * (iterations, residuals) is reported. The engine reads d_F on its own
 * streams, which are not ordered after the caller's: the work that produces d_F must have
 * completed (e.g. its stream synchronised) before the call. Thread-safe, non-blocking.
 * Errors: HZ_EINVAL (bad parameters), HZ_ENOMEM (the request alone exceeds the budget),
 * HZ_EBUSY (the engine is being destroyed). */
hz_status hz_engine_submit(hz_engine* e, double k, double h, int p, hz_c64 s, double theta,
                           const hz_c64* d_F, hz_c64* d_u, long req_id);

/* Moves up to max finished requests into out (in completion order) and sets *ndone. Waits up
 * to wait_ms milliseconds for one when none is ready (0 = do not wait). Thread-safe. */
hz_status hz_engine_poll(hz_engine* e, hz_engine_result* out, int max, int* ndone, int wait_ms);

/* Queue and memory state. */
hz_status hz_engine_info(hz_engine* e, hz_engine_info_t* info);

/* Stops the engine: waits for the current round, drops queued and unfinished requests (they
 * are not reported) and frees everything. NULL is a no-op. */
void hz_engine_destroy(hz_engine* e);

/* ---------------------------------------------------------------------------------------
 * Shift search: the data generation of Sec. 5. For a sample (k, h, p) and a right-hand side
 * F (the paper draws its components uniformly from [-1, 1] and sets g = 0), the exponent
 * sigma of the shift eps = k^sigma (the multiplier s = 1 + i k^(sigma - 2)) that minimises
 * rho(sigma) = (r_end / r_0)^(1 / end), the average reduction of the true residual
 * ||F - A_0 u|| of an FGMRES solve stopped at the options' tolerance or iteration cap
 * (Sec. 5: 1e-8 and 50 iterations, no restarts), is located by golden-section search on
 * [sigma_lo, sigma_hi] until the bracket is at most tol wide (Sec. 5: [1, 2] and 1e-2).
 * --------------------------------------------------------------------------------------- */
typedef struct {
  double k;             /* wavenumber                                                  */
  double h;             /* fine mesh size (1/h an even integer)                         */
  int p;                /* element order                                               */
} hz_search_sample;

typedef struct {
  double sigma;         /* midpoint of the final bracket: the sample's near-optimal exponent */
  double rho;           /* smallest objective value evaluated                               */
  double sigma_best;    /* the exponent at which it was evaluated                           */
  int evaluations;      /* solves run for this sample                                        */
  int status;           /* HZ_OK, or the error of a failed solve                             */
} hz_search_result;

/* Runs the n searches concurrently on one serving engine (config cfg, solver options o; NULL
 * = defaults; the paper's setting is o->tol = 1e-8, o->maxit = 50, o->restart = 50): every
 * objective evaluation is an engine request that sets up and factors the problem with that
 * shift and solves A_0 u = F with d_F[i] (a caller-owned fine vector of sample i, read
 * while the call runs). In each step the bracket [a, b] with inner points c < d keeps [a, d]
 * if rho(c) < rho(d), else [c, b]; the new inner point is the golden section of the kept
 * bracket. Blocks until all searches are done; out[i] receives sample i's result. Errors:
 * HZ_EINVAL (arguments), the engine's errors; a failed solve ends its sample's search (its
 * status is set) and the call returns that error after all searches have ended. */
hz_status hz_shift_search(const hz_search_sample* samples, int n, const hz_c64* const* d_F,
                          double sigma_lo, double sigma_hi, double tol,
                          const hz_engine_config* cfg, const hz_options* o,
                          hz_search_result* out);

/* Copies the problem's counters into *out (waiting for pending timed launches) and, if
 * reset is nonzero, zeroes them. Without timing the device times stay 0. */
hz_status hz_problem_stats(hz_problem* pr, hz_stats* out, int reset);

/* Frees everything the problem owns (NULL is a no-op). */
void hz_destroy_problem(hz_problem* pr);

/* Message of the last failed call on this thread ("" if none). */
const char* hz_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HZ_H */
