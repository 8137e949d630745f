/*
 * fde.h -- C ABI of libfde, a GPU (MI355X, gfx950) solver for the linear
 * systems of the implicit time discretisation of the space-fractional
 * diffusion equation
 *     u_t = d+ D+^a u + d- D-^a u  (+ e+ D+^b u + e- D-^b u in 2D) + f,
 * alpha, beta in (1,2), homogeneous Dirichlet data, on a rectangle
 * (Section 1.1, eq. (1)), preconditioned by the symbol-based tau-algebra
 * preconditioner P_F (Section 3, eqs. prop_1D and 2D_preconditioner) of
 * Barakitis, Ekstrom and Vassalos.
 *
 * Conventions for every entry point
 *   - Vector arguments are DEVICE pointers to float64 arrays owned by the
 *     caller, of length N = n1 (1D) or N = n1*n2 (2D).  2D arrays are stored
 *     x-fastest, i.e. row-major with shape (n2, n1), the lexicographic order
 *     of Section 1.4.  Input and output vectors must not overlap.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  All calls are asynchronous on `stream`, except fde_assemble
 *     and fde_solve, which synchronise `stream` before returning.
 *   - A plan owns its device workspace and the copies it makes of the
 *     coefficient arrays; it is not thread-safe: use one plan per host
 *     thread/stream.  fde_destroy frees it.
 *   - Errors: a negative fde_status; nothing is launched when parameters are
 *     invalid.  fde_last_error() returns a thread-local message describing the
 *     last failure.  FDE_ENOTCONV (> 0) means the solver stopped at maxit:
 *     x then holds the last iterate and `info` is filled.
 *   - Transform sizes.  1D: any n <= 2^21 (chirp-z sine transforms when
 *     n + 1 is not a power of two), and n + 1 a power of two up to 2^22.
 *     2D: n_i + 1 a power of two up to 4096 (FFT line kernels), or any
 *     n_1, n_2 <= 1023 (the line operators as dense matrix products, whose
 *     cost grows as n^3: meant for the paper's small grids and for sizes the
 *     line kernels do not take).  Other sizes return FDE_EUNSUPPORTED.
 */
#ifndef FDE_H
#define FDE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fde_plan_s* fde_plan;

typedef enum {
  FDE_OK = 0,
  FDE_ENOTCONV = 1,        /* result returned, tolerance not reached within maxit */
  FDE_EINVAL = -1,         /* invalid parameter or argument                       */
  FDE_ENOMEM = -2,         /* device or host allocation failed                    */
  FDE_EHIP = -3,           /* a HIP runtime call failed                           */
  FDE_ENONFINITE = -4,     /* NaN/Inf met in the right-hand side or a residual    */
  FDE_EUNSUPPORTED = -5    /* a size or option this build does not handle        */
} fde_status;

/* Space discretisation (Sections 1.2 and 1.3). */
enum { FDE_W_SHIFTED = 0,   /* first-order shifted Grunwald weights g_k, matrix T (eq. grunwaldmatrix1) */
       FDE_W_WEIGHTED = 1   /* second-order weights w_k, matrix S (eq. grunwaldmatrix2)                 */ };
/* Time discretisation. */
enum { FDE_T_EULER = 0,     /* implicit Euler: M = nu I + A_x + kappa A_y, nu = h_x^a/dt (Section 1.2)     */
       FDE_T_CN = 1         /* Crank-Nicolson: M = (1/r) I + A_x + (s/r) A_y, 1/r = 2 h_x^a/dt (Section 1.4) */ };
/* Preconditioner. */
enum { FDE_P_NONE = 0,      /* identity                                                                      */
       FDE_P_TAU = 1,       /* P_F = D tau(F): D (S (x) S) diag(F) (S (x) S), F(i,j) = F_a(th_i) + kappa F_b(th_j)
                               + shift; D = (d+ + d-)/2 (1D), (d+ + d- + e+ + e-)/4 (2D)
                               (eq. prop_1D, eq. 2D_preconditioner)                                          */
       FDE_P_TAU_HAT = 2,   /* constant coefficients d+- = d, e+- = e: tau(nu + d F_a + kappa e F_b), no D
                               (Section 3.1 Case I, eq. 2D_preconditioner_proof_case)                       */
       FDE_P_TILDE = 3,     /* 1D: S diag(D_j p_a(theta_j)) S (Section 4, Table 2)                          */
       FDE_P_TRI = 4        /* 1D: the tridiagonal part of M, solved exactly (Table 2); requires a strictly
                               diagonally dominant tridiagonal part                                        */ };
/* Side of the diagonal factor D in P_F. */
enum { FDE_D_LEFT = 0,      /* P = D tau, as the text writes it: P^{-1} v = tau^{-1}(D^{-1} v) */
       FDE_D_RIGHT = 1      /* P = tau D: P^{-1} v = D^{-1} tau^{-1} v                          */ };
/* Krylov method. */
enum { FDE_S_GMRES = 0,     /* right-preconditioned flexible GMRES(restart), CGS2 orthogonalisation   */
       FDE_S_PCG = 1        /* preconditioned CG; needs a symmetric M (constant d+ = d-, e+ = e-)   */ };
/* Arithmetic. */
enum { FDE_FP64 = 0,        /* everything in float64                                                   */
       FDE_MIXED = 1        /* float64 outer FGMRES (Gram-Schmidt, Givens, true residual, update, outer
                               matvec) around a float32 inner GMRES(inner_steps) with float32 matvec
                               and float32 tau solve; inner_steps = 0 means a float32 tau solve only   */ };

typedef struct {
  int    dim;          /* 1 or 2                                                                  */
  int    n[2];         /* interior points n1 (x), n2 (y; ignored in 1D)                           */
  double alpha[2];     /* fractional orders alpha (x) and beta (y), each in (1, 2)                */
  double lo[2], hi[2]; /* domain (L1, R1) x (L2, R2); h_i = (hi - lo)/(n_i + 1)                   */
  double dt;           /* time step h_t > 0                                                        */
  int    weights;      /* FDE_W_*                                                                  */
  int    time;         /* FDE_T_*                                                                  */
  int    prec;         /* FDE_P_*                                                                  */
  int    dside;        /* FDE_D_*                                                                  */
  double shift;        /* added to every symbol sample of FDE_P_TAU; NaN selects the rule of
                          Section 3.1 Case I: nu/c when all coefficients equal one constant c,
                          0 otherwise                                                             */
  int    solver;       /* FDE_S_*                                                                  */
  int    restart;      /* GMRES cycle length m, 1..32                                              */
  int    maxit;        /* cap on the total number of (outer) iterations                           */
  double tol;          /* stop when ||b - M x||_2 <= tol ||b||_2                                   */
  int    precision;    /* FDE_FP64 | FDE_MIXED                                                     */
  int    inner_steps;  /* FDE_MIXED: float32 inner GMRES steps per outer step, 0..32              */
} fde_params;

typedef struct {
  int    iters;        /* outer iterations (preconditioner applications)                          */
  int    inner_iters;  /* float32 inner iterations (FDE_MIXED)                                    */
  int    restarts;     /* completed GMRES cycles that did not converge                            */
  int    converged;    /* 1 when the true relative residual is <= tol                             */
  double relres_true;  /* ||b - M x|| / ||b|| of the returned x, computed in float64             */
  double relres_est;   /* last Givens (GMRES) or recursive (PCG) residual estimate / ||b||       */
  double seconds;      /* wall time of the call                                                   */
} fde_info;

/* Fills `p` with: 1D, n = 1023, alpha = 1.5 on (0,2), dt = h, FDE_W_SHIFTED,
   FDE_T_EULER, FDE_P_TAU, FDE_D_LEFT, shift = NaN, FDE_S_GMRES, restart 30,
   maxit 10000, tol 1e-8, FDE_FP64, inner_steps 16. */
void fde_default_params(fde_params* p);

/* Builds a plan for M and P (setup row of the method: Grunwald weights
   (eq. grunwald1), circulant eigenvalues of T (T^T), symbol samples F at
   theta_j = j pi/(n+1) (eq. tau_preconditioner, Theorem 2), D^{-1}).
   dplus, dminus: device arrays of length N with d+ (x_i, y_j) >= 0, d- >= 0;
   eplus, eminus: the y-direction coefficients (2D) or NULL (1D).  The plan
   copies them.  Returns FDE_EINVAL when a parameter is out of range, when a
   coefficient is negative or not finite, or when D has a zero (d+ and d- share
   a zero, Section 3.1).  Synchronises `stream`. */
fde_status fde_assemble(const fde_params* p,
                        const double* dplus, const double* dminus,
                        const double* eplus, const double* eminus,
                        void* stream, fde_plan* out);

/* y = M x (eq. first_order_1d_coefficient_matrix / eq. coef:2d), computed with
   circulant-embedded FFT Toeplitz products.  x, y: device, length N. */
fde_status fde_matvec(fde_plan plan, const double* x, double* y, void* stream);

/* z = P^{-1} v for the plan's preconditioner: two (1D) or four (2D) DST-I
   passes around the division by the symbol samples, and the D^{-1} scaling
   (eqs. prop_1D, 2D_preconditioner); for FDE_P_TRI the tridiagonal solve.
   v, z: device, length N. */
fde_status fde_tau_apply(fde_plan plan, const double* v, double* z, void* stream);

/* The same two operators in float32 arithmetic, the arithmetic of the mixed
   form's inner solves: x (v) rounded to float32, the operator applied in
   float32, the result widened into y (z).  The plan must have been assembled
   with precision = FDE_MIXED (FDE_EINVAL otherwise).  Float64 device arrays of
   length N; asynchronous on `stream`. */
fde_status fde_matvec_f32(fde_plan plan, const double* x, double* y, void* stream);
fde_status fde_tau_apply_f32(fde_plan plan, const double* v, double* z, void* stream);

/* Solves M x = b (eq. linsystem).  b: device, length N.  x: device, length
   N, holds the starting vector on entry and the solution on return.  info:
   host pointer or NULL.  Synchronises `stream`.  b = 0 returns x = 0 with 0
   iterations.  FDE_ENONFINITE when b or a residual is not finite.
   Residual history: with the environment variable FDE_TRACE set to 1
   (standard error) or to a file name (appended to), the solve writes
     fde_trace solve=<k> solver=<gmres|pcg> kind=<est|true> iter=<i> relres=<v>
   per iteration (kind=est: the solver's estimate of ||b - M x|| / ||b||) and
   per true-residual check (kind=true); the one-workgroup 1D PCG solve writes
   its final values only.  Tracing reads the state back every cycle (PCG:
   every iteration) and is not meant for timing. */
fde_status fde_solve(fde_plan plan, const double* b, double* x, fde_info* info, void* stream);

/* Right-hand side of one time step (Section 1.2, eq. matrixform; Section 1.4
   for Crank-Nicolson): Euler b = nu u_prev + h_x^a f, Crank-Nicolson
   b = (nu I - A_x - kappa A_y) u_prev + 2 h_x^a f.  f may be NULL (f = 0). */
fde_status fde_rhs(fde_plan plan, const double* u_prev, const double* f, double* b, void* stream);

/* Device bytes a plan with these parameters allocates (for admission control). */
size_t fde_plan_bytes(const fde_params* p);

/* Releases the plan (synchronises the device first). NULL is ignored.  The
   plan's device buffers are kept by the library, per device and size, for
   the next plan of the same shape (at most 16 GiB in total). */
void fde_destroy(fde_plan plan);

/* Frees the device buffers the library keeps from destroyed plans
   (synchronises the current device first).  Plans in use are not affected. */
void fde_release_cache(void);

/* Kernel timing probe (benchmarking).  fde_probe(plan, cls) starts bracketing
   every 32nd launch of one kernel class issued by this plan with HIP events on
   the launch stream (a sample keeps the event overhead out of the timing),
   and accumulates those launches' algorithmic bytes (each vector operand read
   or written once); cls = FDE_PROBE_OFF stops.  fde_probe_read synchronises
   on the recorded events and returns the summed time of the bracketed
   launches in milliseconds, their number and their summed algorithmic bytes,
   then clears the record.  Either pointer argument may be NULL. */
enum { FDE_PROBE_OFF = 0,
       FDE_PROBE_MAXPY64 = 1,   /* float64 multi-vector update w -= sum c_i V_i (Gram-Schmidt) */
       FDE_PROBE_MDOT64 = 2,    /* float64 multi-dot V^T w                                       */
       FDE_PROBE_LINE64 = 3,    /* float64 line transforms (DST-I / Toeplitz passes)            */
       FDE_PROBE_LINE32 = 4,    /* float32 line transforms                                       */
       FDE_PROBE_MAXPY32 = 5,
       FDE_PROBE_MDOT32 = 6,
       FDE_PROBE_CGS64 = 7,     /* every float64 Gram-Schmidt pass (dot, update+dot, update+norm) */
       FDE_PROBE_CGS32 = 8,
       FDE_PROBE_LINE64_VARIANT = 64,   /* + line program flags (0..31): one float64 line kernel   */
       FDE_PROBE_LINE32_VARIANT = 96 }; /* + line program flags (0..31): one float32 line kernel   */
fde_status fde_probe(fde_plan plan, int cls);
fde_status fde_probe_read(fde_plan plan, double* ms, long long* launches, double* bytes);

/* ---------------------------------------------------------------------------
 * Batched 1D solves: many independent systems M_i u_i = b_i (Section 1.2,
 * eq. linsystem), each with its own n_i, alpha_i, coefficients and
 * parameters, solved together in one persistent launch.  Each instance is
 * solved by one workgroup with the right-preconditioned FGMRES of fde_solve
 * (float64, or the mixed form), so its result does not depend on the rest of
 * the batch.  Any n_i in 1..65535 is accepted: when n_i + 1 is not a power
 * of two the DST-I is evaluated by the chirp-z identity with power-of-two
 * FFTs.
 *
 * Packing: batch vectors are the instances' vectors concatenated in order;
 * instance i occupies elements [off_i, off_i + n_i) with
 * off_i = n_0 + ... + n_{i-1} (fde_batch_layout returns the offsets).
 * Restrictions: dim = 1, solver = FDE_S_GMRES, restart <= 32.
 * ------------------------------------------------------------------------- */
typedef struct fde_batch_s* fde_batch;

/* Launch configurations: variant selects the workgroup size and FFT radix
   (0: 512 threads, radix 8; 1: 512 threads, radix 4; 2 and 3, the
   256-thread forms, are disabled and rejected with FDE_EUNSUPPORTED); grid
   is the number of persistent workgroups; lpt = 1 hands out instances
   longest-estimated-work first, 0 in the given order; split = the number of
   instances with the largest estimated work (iterations of their last solve
   times n log n, or n log n before any) taken out of the persistent launch
   and solved on the plan path (fde_assemble + fde_solve, built on first use),
   by host worker threads on streams of their own, concurrently with the
   launch: a large, slow instance then runs on all CUs instead of one.  ms:
   the time of one step measured by the tuner. */
enum { FDE_BATCH_VARIANTS = 4 };
typedef struct {
  int    variant;
  int    grid;
  int    lpt;
  double ms;
  int    split;
} fde_batch_cfg;

/* Offsets of the packed layout (offsets: host array of count + 1 entries, or
   NULL); returns the total length, 0 when a parameter set is invalid. */
size_t fde_batch_layout(const fde_params* params, int count, long long* offsets);

/* Device bytes a batch with these parameters allocates. */
size_t fde_batch_bytes(const fde_params* params, int count);

/* Builds a batch from count parameter sets (host array) and the packed
   device arrays d+ and d- (length fde_batch_layout(...)).  Validation as in
   fde_assemble, per instance; FDE_EUNSUPPORTED for dim != 1, PCG or n > 65535.
   Synchronises `stream`. */
fde_status fde_batch_assemble(const fde_params* params, int count, const double* dplus,
                              const double* dminus, void* stream, fde_batch* out);

/* Solves every instance: b packed right-hand sides, x packed start vectors
   on entry and solutions on return (device).  info: host array of count
   entries or NULL.  FDE_ENOTCONV / FDE_ENONFINITE when any instance did not
   converge / met a non-finite value (the others are still solved).
   Synchronises `stream`. */
fde_status fde_batch_solve(fde_batch batch, const double* b, double* x, fde_info* info, void* stream);

/* Batched operators on packed vectors (device): y = M x and z = P^{-1} v for
   every instance, with its own operator and preconditioner (for FDE_P_TAU,
   the DST-I / symbol / DST-I solve and D^{-1}; for FDE_P_TRI the tridiagonal
   solve).  precision = FDE_FP64 computes in float64; FDE_MIXED in float32
   (the arithmetic of the mixed form's inner solves; the batch must have been
   assembled with FDE_MIXED).  Inputs and outputs are float64 and must not
   overlap.  Each instance's operator is applied with its own plan (built on
   first use: the first call allocates and synchronises `stream`), one launch
   sequence per instance; otherwise asynchronous on `stream`. */
fde_status fde_batch_matvec(fde_batch batch, int precision, const double* x, double* y, void* stream);
fde_status fde_batch_tau_apply(fde_batch batch, int precision, const double* v, double* z, void* stream);

/* Time stepping: `steps` implicit steps of every instance from the packed
   state u (device, advanced in place): b = rhs(u) with f = 0 (fde_rhs), then
   M u_new = b solved from u_new = u.  With use_graph != 0 one step (queue
   reset, solve launch, step counter) is captured once as a HIP graph and
   replayed per step.  info: host array of steps * count entries (step-major)
   or NULL.  Synchronises `stream`. */
fde_status fde_batch_run(fde_batch batch, double* u, int steps, int use_graph, fde_info* info,
                         void* stream);

/* Autotuner: times one time step from the packed state u (not modified) for
   every launch configuration (variant x grid x order, then split counts
   with the best of those) and keeps the fastest; `chosen` (may be NULL)
   receives it.  Synchronises `stream`. */
fde_status fde_batch_tune(fde_batch batch, const double* u, void* stream, fde_batch_cfg* chosen);
fde_status fde_batch_get_cfg(fde_batch batch, fde_batch_cfg* cfg);
fde_status fde_batch_set_cfg(fde_batch batch, const fde_batch_cfg* cfg);

/* Releases the batch (synchronises the device first). NULL is ignored. */
void fde_batch_destroy(fde_batch batch);

/* ---------------------------------------------------------------------------
 * Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  One call does what fde_assemble + fde_solve + fde_destroy do
 * for a 1D float64 PCG plan (dim = 1, solver = FDE_S_PCG, precision =
 * FDE_FP64, prec = FDE_P_TAU, FDE_P_TAU_HAT or FDE_P_TILDE) whose line fits
 * one workgroup: 8 <= n + 1 <= 4096, n + 1 a power of two.  It runs the same
 * set-up arithmetic and the same kernels, so its result equals that of the
 * plan path.  Every device table and work vector lives in one static device
 * array of 512 KiB that the library holds on each device it runs on until the
 * process ends; the call makes no hipMalloc/hipFree and no other device
 * allocation (its host-side set-up uses ordinary host memory).
 *   dplus, dminus, b: device, length n; read in place (not copied).
 *   x: device, length n: the starting vector on entry, the solution on return.
 *   info: host pointer or NULL.
 * Synchronises `stream`.  Errors as fde_assemble and fde_solve;
 * FDE_EUNSUPPORTED for any other configuration or size.  Calls that overlap
 * on one device share the static array and race: issue them one at a time
 * per device. */
fde_status fde_pcg1d_solve_noalloc(const fde_params* p, const double* dplus, const double* dminus,
                                   const double* b, double* x, fde_info* info, void* stream);

/* Thread-local description of the last error, "" when none. */
const char* fde_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDE_H */
