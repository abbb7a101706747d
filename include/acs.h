/*
 * acs.h - C ABI of the adaptively conditioned first-order conic solver for
 * MI355X (gfx950).
 *
 * Method: Algorithm 2 of "Rapid Convergence of First-Order Numerical
 * Algorithms via Adaptive Conditioning" (Adil, Tavakkol, Madani, arXiv
 * 2103.00736).  It solves the primal/dual pair of Sec. II
 *
 *     minimise   c^T x    s.t.  A x = b,            x in K        (eq. prob_primal)
 *     maximise   b^T y    s.t.  A^T y + z = c,      z in K        (eq. prob_dual)
 *
 * with K a product of Lorentz cones.  Every iteration reflects the iterate
 * through the cone (step 16), projects onto the scaled subspace
 * range((A O)^T) (step 17) and updates the Douglas-Rachford-type iterate s
 * (step 18); at the iterations of the set L (plus the first) it rescales the
 * columns of A by a diagonal O computed from the current x and z (steps 5-14).
 *
 * Conventions
 *   - All functions return int: ACS_OK (0) on success, a negative ACS_ERR_*
 *     code on failure.  acs_last_error() returns a message for the last
 *     failure on the calling thread.  No C++ exception crosses this ABI.
 *   - Matrices are CSR (row_ptr[m+1], col_idx[nnz], val[nnz]) with column
 *     indices strictly ascending inside each row; nnz < 2^31.
 *   - The cone list is [ n_orth orthant coordinates | soc_sizes[0] | ... ]:
 *     the first n_orth coordinates of x are R_+ (Lorentz cones of size one),
 *     followed by the second-order cones {w : w_1 >= ||w_{2:k}||_2} in list
 *     order; n_orth + sum(soc_sizes) must equal n.
 *   - Host pointers ("host") are read or written synchronously; the library
 *     never keeps them.  Device pointers ("device") must be HIP allocations
 *     on the current device.  Objects are not thread-safe unless stated.
 *   - `stream` is a hipStream_t (NULL = the library's own stream).  All GPU
 *     work of an object is ordered on that stream.
 */
#ifndef ACS_H_
#define ACS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------- */
#define ACS_OK 0
#define ACS_PENDING 1          /* server: request not finished yet            */
#define ACS_ERR_ARG (-1)       /* invalid argument or malformed problem        */
#define ACS_ERR_NOMEM (-2)     /* device or host allocation failed / too big   */
#define ACS_ERR_DEVICE (-3)    /* HIP runtime error, or no usable GPU          */
#define ACS_ERR_NUMERIC (-4)   /* NaN/Inf in the iterates                      */
#define ACS_ERR_STATE (-5)     /* call not valid in the object's state         */

/* ---- solve status (acs_info.status) -------------------------------------- */
#define ACS_SOLVED 0           /* KKT error <= eps_kkt at a check              */
#define ACS_MAX_ITER 1         /* iteration limit reached, best effort result  */
#define ACS_NUMERIC 2          /* NaN/Inf detected, iteration stopped          */
#define ACS_CANCELLED 3        /* server request cancelled                     */

/* ---- arithmetic ---------------------------------------------------------- */
#define ACS_PREC_MIXED 0  /* FP32 matrix values, iterate and CG vectors;
                             FP64 CG solution, residual accumulation,
                             reductions, scaling factors                   */
#define ACS_PREC_FP64 1   /* everything in FP64                            */

/* ---- projection of Alg. 2 step 17 (the paper does not say how (A O)^+ is
 * applied; Sec. II defines it as a pseudo-inverse) ------------------------ */
#define ACS_PROJ_CG 0      /* warm-started CG on (A_s A_s^T) w = rhs each iteration */
#define ACS_PROJ_FACTOR 1  /* M = A_s A_s^T formed and inverted in FP64 at every
                              conditioning event (M is fixed between events);
                              each iteration then sets w += M^{-1} r, exact up to
                              rounding.  Needs m <= 32768 and m * n <= 2^31;
                              extra device memory: acs_problem_factor_bytes.
                              Single-instance paths only (not the batch kernel). */
#define ACS_PROJ_AUTO 2    /* ACS_PROJ_FACTOR for m <= 2048, else ACS_PROJ_CG; the
                              batch kernel takes it as ACS_PROJ_CG.  Measured
                              whole solves on one MI355X: the 200 x 500 LP in
                              FP64 10 ms against 87 ms by CG; serving-trace LPs
                              with m = 1000 / 2000 10 / 16 ms against 27 / 34 ms,
                              with m = 4000 52 ms against 40 ms. */

/*
 * Settings (Alg. 2 Require line and Sec. V).  Call acs_settings_default()
 * first.  Conditioning set L = {l_first, l_first + l_every, ...} up to l_last
 * (inclusive; -1 = unbounded); l_first = 0 means L is empty (Algorithm 1),
 * l_every = 0 means L = {l_first}.  Iteration 1 always conditions.
 * With `auto_params` = 1 the library picks the paper's per-class values:
 * LP: t = 9.2, L = {300, 400, ...}; SOCP: t = 1.7, L = {200, 300, ...}; mu = 1.
 * Projection (Alg. 2 step 17) by warm-started CG, defaults cg_reduce = 0
 * (per class: 0.1 for LPs, 0.2 for SOCPs; a negative value is ACS_ERR_ARG),
 * cg_max = 500; obj_stop = 1.  The iteration just before a conditioning event
 * (its x, z set O) runs its CG to a 1e-6 reduction with up to 8 cg_max steps.
 * A cap that stops the CG short of cg_reduce leaves an error the outer
 * iteration may not recover from once O is spread; smaller cg_reduce trades
 * CG steps for outer iterations.  Measured whole solves: the row-scaled
 * 2M-variable LP runs fastest at 0.03 and takes 3x longer at 0.2, while the
 * 1M-variable SOCP, the small LPs of the batch recipe and the serving trace's
 * requests run fastest at 0.2-0.3.
 */
/*
 * Equilibration (settings.equilibrate = 1; sparse problems, one-instance
 * paths and the server's worker streams; the batch kernel refuses it).  Sec.
 * III preconditions the data as A_hat = D A E, b_hat = D b, c_hat = E c
 * (x_hat = E^{-1} x, z_hat = E z) and compares adaptive conditioning with the
 * D, E of an l2 Sinkhorn-Knopp balancing.  The library takes the plain
 * balancing of the squared entries: from E = 1, eq_sweeps sweeps of
 * D_i^2 = 1 / sum_j a_ij^2 E_j^2 (unit row norms), then
 * E_j^2 = (m/n) / sum_i a_ij^2 D_i^2 (column norms sqrt(m/n)), with one E per
 * Lorentz cone (its columns' mean square norm m/n) and 1 for empty rows and
 * columns; all in FP64 on the GPU.  Algorithm 2 then runs on the
 * preconditioned problem with its own O on top; in the original variables
 * that is the column scaling E O_hat, with the ratio of steps 5-10 taken from
 * x_hat, z_hat.  D drops out (neither range((D A E)^T) nor the affine set
 * depends on it), and results are returned in the original variables.  On
 * badly row-scaled problems E can span many decades (about 1e9 on a power-law
 * LP with row scales 1e+-3), where the FP32 CG of ACS_PREC_MIXED may stall
 * short of the tolerance; use ACS_PREC_FP64 with equilibration there.
 */
/*
 * Layout of the sparse products with A_s (a_slices).  With 8 slices each of
 * the MI355X's 8 XCDs multiplies one column slice of A_s, so the gathered
 * vector of one slice stays in that XCD's L2, and a second launch adds the
 * 8 partial sums of every row (and applies the CG update); the CG's own
 * vector is stored with each slice's columns in the order the layout first
 * reads them, on two more layouts (16 bytes per nonzero of device memory in
 * mixed precision, 20 in FP64; acs_problem_device_bytes counts them).  With 1 slice a
 * workgroup sums whole rows and applies the CG update itself: one launch
 * fewer per CG step and per outer iteration, for problems whose gathered
 * vector fits every L2.  0 picks 1 slice for n <= 262144, else 8.  The two
 * layouts add the products of a row in different orders, so their results
 * agree to rounding, not bit for bit; each is deterministic.
 */
typedef struct acs_settings {
  double mu;            /* proximal parameter mu > 0                            */
  double t;             /* cap on log(max O) - log(min O), t > 0 (step 11)      */
  int32_t l_first;      /* first conditioning iteration after l = 1             */
  int32_t l_every;      /* period of L                                          */
  int32_t l_last;       /* last member of L, -1 = none                          */
  int32_t auto_params;  /* 1: choose t and L from the problem class             */
  int32_t max_iter;     /* outer-iteration limit                                */
  int32_t check_every;  /* KKT evaluation period (iterations)                   */
  double eps_kkt;       /* stop when max(eps_p, eps_d, eps_gap, eps_cone) <= it */
  int32_t precision;    /* ACS_PREC_MIXED or ACS_PREC_FP64                      */
  int32_t cg_max;       /* CG steps per outer iteration, at most                */
  double cg_reduce;     /* stop CG once ||r|| <= cg_reduce * ||r_0|| (warm); 0 = per class */
  double cg_abs;        /* ... or once ||r|| <= cg_abs (scaled system)          */
  int32_t verbose;      /* 0 quiet, 1 one line per check on stderr              */
  int32_t projection;   /* ACS_PROJ_CG (default), ACS_PROJ_FACTOR or ACS_PROJ_AUTO */
  int32_t obj_stop;     /* k > 0: a check also needs k * eps_obj <= eps_kkt (default 1); 0: KKT only */
  int32_t equilibrate;  /* 1: Sinkhorn-Knopp column scaling E first (Sec. III, below); 0 (default): none */
  int32_t eq_sweeps;    /* sweeps of that equilibration (default 25)              */
  int32_t a_slices;     /* column slices of the sparse A_s products: 0 (default) by size, 1 or 8 (below) */
  int32_t reserved[2];
} acs_settings;

/* Per-solve report.  KKT errors follow the oracle's definition:
 *   eps_p = ||Ax-b||/(1+||b||), eps_d = ||A^T y+z-c||/(1+||c||),
 *   eps_gap = |c^T x - b^T y|/(1+|c^T x|+|b^T y|),
 *   eps_cone = max(dist(x,K), dist(z,K))/(1+max(||x||,||z||)).
 * Those are relative to the norms of b and c, so they do not bound the
 * relative error of the objective.  For an optimal pair (y*, z*) of the dual
 * (Sec. II), with r_p = Ax-b, c^T x - p* = z*^T x + y*^T r_p exactly; the
 * estimate takes the first term's bound at the current y, z, coordinate by
 * coordinate in absolute value on the orthant and summed with signs over the
 * Lorentz cones (each cone's term carries first-order errors of either sign):
 *   eps_obj = (sum_j |x_j z_j| + |sum_C x_C^T z_C| + |y^T r_p|)/(1+|c^T x|).
 * With settings.obj_stop = k (default 1) a solve stops only when
 * kkt <= eps_kkt and k * eps_obj <= eps_kkt.                              */
typedef struct acs_info {
  int32_t status;       /* ACS_SOLVED / ACS_MAX_ITER / ACS_NUMERIC / ACS_CANCELLED */
  int32_t iterations;   /* outer iterations run                                */
  int64_t cg_steps;     /* total CG steps                                      */
  int32_t conditionings;/* conditioning events run                             */
  int32_t reserved0;
  double eps_p, eps_d, eps_gap, eps_cone, kkt;
  double pobj, dobj;    /* c^T x and b^T y                                     */
  double solve_ms;      /* wall time of the iteration loop                     */
  double setup_ms;      /* upload + setup                                      */
  double alpha;         /* exponent of the last conditioning (step 11)         */
  double o_range;       /* log(max O) - log(min O) after the last conditioning */
  double queue_ms;      /* server: entry of submit -> admission                */
  double latency_ms;    /* server: entry of submit (layout build included) -> result ready */
  double eps_obj;       /* objective-error estimate of the last check (above)  */
  double reserved[3];
} acs_info;

typedef struct acs_problem acs_problem;
typedef struct acs_state acs_state;

/* Library and device. */
const char* acs_version(void);
const char* acs_last_error(void);
/* Initialise HIP on `device` (ordinal); returns ACS_ERR_DEVICE when no gfx950 GPU is usable. */
int acs_init(int32_t device);

void acs_settings_default(acs_settings* s);

/*
 * Problem (Sec. II).  Inputs are host arrays and are COPIED; the caller may
 * free them on return.  Validation: m, n >= 1; row_ptr[0] = 0, nondecreasing,
 * row_ptr[m] = nnz; 0 <= col < n, strictly ascending in a row; finite val,
 * b, c; n_orth >= 0, soc sizes >= 1, n_orth + sum(soc) = n.  Failure:
 * ACS_ERR_ARG and *out = NULL.  Pure host code: valid without a GPU.
 * A problem with m + nnz >= 2^18 is built, and later its device layouts, on
 * up to 16 host threads (fewer on smaller machines; the environment variable
 * ACS_HOST_THREADS, read once, caps them further).  The result does not
 * depend on the number of threads.
 */
int acs_problem_create(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                       const double* val, const double* b, const double* c, int32_t n_orth, int32_t n_soc,
                       const int32_t* soc_sizes, acs_problem** out);
/*
 * Dense problem (Sec. V: the paper's random LP and SOCP instances have dense
 * A with U[-1,1] entries).  a is row-major m x n (HOST, copied; the caller
 * may free it on return); b, c and the cone list as for acs_problem_create.
 * The products stream A in FP32 (plus the FP32 rounding error of each value
 * when some value is not an FP32 number, for the FP64 sweeps); the scalings
 * D and O of Alg. 2 step 12 are applied to vectors, so A is never rewritten.
 * Validation: m, n >= 1, finite values, m * round_up(n, 64) < 2^31.  Solved
 * by acs_solve and acs_state_*; the batch and the server pool take sparse
 * problems (a server runs dense requests on its worker streams).  Host code.
 */
int acs_problem_create_dense(int32_t m, int32_t n, const double* a, const double* b, const double* c, int32_t n_orth,
                             int32_t n_soc, const int32_t* soc_sizes, acs_problem** out);
void acs_problem_destroy(acs_problem* p);
/* Device bytes a one-instance solve of `p` in `precision` allocates (for
 * budgeting; includes the SELL layouts of the CG products).  Host code. */
int64_t acs_problem_device_bytes(const acs_problem* p, int32_t precision);
/* Device bytes the direct projection (ACS_PROJ_FACTOR) adds to that: M and
 * the FP64 copy of A_s (padded to mp = m rounded up to 128 rows), the sweep
 * panels.  -1 for a null problem.  Host code. */
int64_t acs_problem_factor_bytes(const acs_problem* p);
/* Device bytes `p` takes as one instance of a batch arena or a server pool
 * slot (the persistent kernel's layout); -1 for a dense problem, which the
 * batch does not take.  Host code. */
int64_t acs_batch_device_bytes(const acs_problem* p);

/*
 * One-shot solve (Alg. 2 until KKT <= eps_kkt or max_iter).  x, z (length n)
 * and y (length m) are caller-allocated HOST buffers (any may be NULL).
 * y is the multiplier -w/mu of the scaled dual (Sec. IV).  info may be NULL.
 */
int acs_solve(const acs_problem* p, const acs_settings* s, double* x, double* y, double* z, acs_info* info,
              void* stream);

/*
 * The same solve with DEVICE outputs: x, z (n doubles) and y (m doubles, the
 * caller's row order) are caller-owned device allocations (e.g. torch
 * tensors; any may be NULL), written by a kernel on `stream` (e.g. torch's
 * current stream; NULL = the library's own).  Results are bitwise those of
 * acs_solve.  Returns after they are written (synchronises with `stream`).
 * A pointer that is not a device allocation gives ACS_ERR_ARG before any
 * GPU work.
 */
int acs_solve_device(const acs_problem* p, const acs_settings* s, double* x, double* y, double* z, acs_info* info,
                     void* stream);

/*
 * acs_solve_device for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, bitwise the same results, with every device array of the
 * instance carved from a fixed 64 MiB array compiled into the library (one per
 * GPU, held until the process ends) and the progress record and fallback
 * stream (used when `stream` is NULL) set up once per device by acs_init or
 * by the first call.  The call itself makes no hipMalloc, hipFree, pinned or
 * other allocating HIP call.  Outputs as for acs_solve_device (device
 * buffers, written on `stream`, complete on return).
 * Limits and errors: ACS_ERR_NOMEM when acs_problem_device_bytes(p,
 * precision) exceeds 64 MiB (checked before any GPU work); ACS_ERR_ARG for
 * ACS_PROJ_FACTOR or a pointer that is not a device allocation.
 * Every call on a GPU uses that GPU's one array, which keeps the last call's
 * contents (the solve initialises everything it reads).  The library runs
 * such calls one at a time per process; calls from several processes, or
 * overlapping work by the caller on that memory, would race.
 */
int acs_solve_device_noalloc(const acs_problem* p, const acs_settings* s, double* x, double* y, double* z,
                             acs_info* info, void* stream);

/*
 * Solver state on the GPU (resident iterate and scalings; tests, benchmarks
 * and checkpoint/resume).  The state after l iterations is (l, s_prev, s, O, w):
 * s = s^{l+1}-to-be input of iteration l+1, s_prev the iterate before it, O the
 * current column scaling (positive, constant on every cone), w the unscaled
 * CG solution (y = -w/mu).  x and z of steps 19-20 are
 * x = O (abs_K(s_prev) + s) / 2 and z = (abs_K(s_prev) - s) / (2 mu O).
 * acs_state_create uploads the problem and sets the initial state l = 0,
 * x = z = e_K (s_prev = (1+mu) e_K, s = (1-mu) e_K, O = 1, w = 0).
 */
int acs_state_create(const acs_problem* p, const acs_settings* s, void* stream, acs_state** out);
void acs_state_destroy(acs_state* st);
/* Host arrays: s_prev, s, O (n), w (m).  O must be positive and constant per cone. */
int acs_state_set(acs_state* st, int32_t l, const double* s_prev, const double* s, const double* O, const double* w);
/* Runs exactly `iters` outer iterations (conditioning and checks per settings). */
int acs_state_step(acs_state* st, int32_t iters);
/* Runs until KKT <= eps_kkt at a check or `max_iter` total iterations. */
int acs_state_solve(acs_state* st, acs_info* info);
/* Host outputs, any may be NULL: s_prev, s, O, x, z (n); w, y (m).  Synchronises. */
int acs_state_get(acs_state* st, int32_t* l, double* s_prev, double* s, double* O, double* w, double* x,
                  double* y, double* z);
int acs_state_info(acs_state* st, acs_info* info);
/* KKT errors of the current state (runs the check kernels), fills info. */
int acs_state_check(acs_state* st, acs_info* info);

/*
 * Kernel-level entry points (device pointers, library stream of `st`), used
 * by tests and the benchmark's roofline measurement.
 *   which = 0: y = A_s x   (rows of the scaled matrix, FP32/FP64 per precision)
 *   which = 1: y = A_s^T x (rows of the scaled transpose)
 * where A_s = diag(d) A O is the state's current scaled matrix.  x and y are
 * device arrays of the state's value type (float in MIXED, double in FP64).
 * `reps` launches are timed with HIP events on the state's stream; *avg_ms
 * receives the mean duration per launch (may be NULL).
 */
int acs_state_spmv(acs_state* st, int32_t which, const void* x, void* y, int32_t reps, double* avg_ms);
/* Per-kernel-class event timing over subsequent acs_state_step calls.
 * `enable` is a bit mask of the classes to time (bit k = class k; 0 stops;
 * ACS_PROF_ALL times every class); each timed launch is bracketed by HIP
 * events on the state's stream, which costs a few microseconds per launch, so
 * timing only the class of interest keeps the overhead small.  A nonzero mask
 * resets the counts.  acs_state_timing reads {count, total_ms} for class k
 * (0 = update sweep k_update, 1 = residual sweep k_resid_part +
 * k_resid_comb, 2 = CG sweep k_cg_t, 3 = CG sliced sweep k_cg_a_part, 4 =
 * cone k_cone, 5 = check k_pres, 6 = conditioning, 7 = one-workgroup
 * finalizers, 8 = CG combine k_cg_a_comb; direct projection: 9 = M = A_s A_s^T
 * (k_fac_syrk), 10 = the inversion sweep's rank-64 updates (k_fac_update),
 * 11 = w += M^{-1} r (k_fac_apply), 12 = the sweep's pivot blocks and panels
 * (k_fac_pivot, k_fac_panel, k_fac_mirror)).  The direct projection's FP64
 * copy of A_s counts as conditioning (6). */
#define ACS_PROF_ALL 0x1fff
int acs_state_profile(acs_state* st, int32_t enable);
/* Direct projection only (ACS_PROJ_FACTOR): copies (A O^2 A^T)^+ as computed
 * by the last factorization (for the state's current O) into `out`, a
 * caller-owned host array of m * m doubles, row-major in the caller's row
 * order; rows and columns of dependent (e.g. empty) rows of A are zero.
 * ACS_ERR_STATE on a CG state or before the first factorization.  A test
 * entry point: it copies m rows one by one. */
int acs_state_normal_inverse(acs_state* st, double* out);
int acs_state_timing(acs_state* st, int32_t cls, int64_t* count, double* total_ms);

/*
 * Batched solving of many independent (small) problems in one persistent
 * kernel launch (captured in a HIP graph): each workgroup takes the next
 * instance from a device work queue, largest first, and runs Algorithm 2 for
 * it with workgroup-level sweeps and reductions until its KKT error meets
 * eps_kkt or the iteration budget runs out.  The same iteration as the
 * one-instance path (fused steps 16-20, conditioning steps 5-14, same
 * precision split); per-instance t and L follow the class when auto_params=1.
 * Device memory: one arena for all instances (acs_batch_device_bytes
 * summed); ACS_ERR_NOMEM if it does not fit.
 */
typedef struct acs_batch acs_batch;
int acs_batch_create(int32_t count, const acs_problem* const* probs, const acs_settings* s, void* stream,
                     acs_batch** out);
void acs_batch_destroy(acs_batch* b);
/* Timed choice of lanes-per-row (rows of A and of A^T) for each size class on
 * `sample` instances of the class, `iters` iterations per trial; results are
 * read from / merged into the text file cache_path (may be NULL).  Resets all
 * instances to their initial state. */
int acs_batch_autotune(acs_batch* b, int32_t sample, int32_t iters, const char* cache_path);
/* Advance every unfinished instance by up to iter_budget iterations in one
 * launch (use_graph = 1: replay of the captured graph; 0: eager launch);
 * *ms (may be NULL) gets the launch's GPU time.  Resumable: the state stays
 * resident between calls. */
int acs_batch_run(acs_batch* b, int32_t iter_budget, int32_t use_graph, double* ms);
/* Host outputs of instance i (any may be NULL); x, z length n_i, y length m_i. */
int acs_batch_result(acs_batch* b, int32_t i, double* x, double* y, double* z, acs_info* info);
/* Resident state of instance i (HOST outputs, any may be NULL): the
 * iterations run, s_prev and s (FP32 iterates widened to double), O (n), w
 * (unscaled, y = -w/mu) and the row norms sqrt(D_i) of the current scaling
 * (m, the caller's row order), as acs_state_get reports them for one
 * instance.  Synchronises with the batch's stream.  Tests and checkpoints. */
int acs_batch_state_get(acs_batch* b, int32_t i, int32_t* l, double* s_prev, double* s, double* O, double* w,
                        double* dsq);
/* Sweep schedule chosen for instance i (rows of A and of A^T): G > 0 lanes per
 * row reading the matrix directly, or -S for LDS-staged row blocks of at most
 * S nonzeros. */
int acs_batch_lanes(acs_batch* b, int32_t i, int32_t* g_a, int32_t* g_t);
/* One-shot: create, run to completion (max_iter), copy results, destroy.
 * x[i], y[i], z[i] are per-instance host buffers (the arrays may be NULL). */
int acs_batch_solve(int32_t count, const acs_problem* const* probs, const acs_settings* s, double* const* x,
                    double* const* y, double* const* z, acs_info* infos, void* stream);

/*
 * Serving loop (continuous batching), thread-safe.  Requests are admitted in
 * arrival order while fewer than max_slots are resident and their device
 * footprint fits hbm_budget bytes; each stays resident (iterates, scalings,
 * scaled matrix) until it finishes.  Requests with nnz <= small_nnz share a
 * slot pool advanced by one persistent batch-kernel launch per tick
 * (tick_iters iterations per tick; new requests join at the next tick);
 * larger ones run the one-instance kernels on `workers` streams (1..8)
 * concurrently.  A result does not depend on the other resident requests.
 * A request whose footprint exceeds the budget fails at submit with
 * ACS_ERR_NOMEM.  Choosing small_nnz: a pool request runs on one workgroup,
 * so its latency grows with its nonzeros (a 200k-nonzero LP took seconds,
 * against about 50 ms on the worker path).  Measured on a trace of 120
 * requests with m log-uniform in [1e3, 2e5] and small_nnz = 20000, served
 * over solved one at a time: 2 workers 2.0x, 3 2.0x, 4 2.1x, 6 2.6x, 8 2.5x;
 * small_nnz = 200000 served at 0.3x.
 */
typedef struct acs_server acs_server;
typedef struct acs_server_counters {
  int64_t queued;        /* waiting for admission                     */
  int64_t running;       /* resident                                  */
  int64_t completed;     /* finished (including cancelled)            */
  int64_t bytes_in_use;  /* device bytes reserved by resident requests */
  int64_t ticks;         /* pool launches so far                      */
  int64_t peak_running;
  int64_t reserved[2];
} acs_server_counters;
int acs_server_create(int64_t hbm_budget, int32_t max_slots, int64_t small_nnz, int32_t workers, int32_t tick_iters,
                      acs_server** out);
/* Stops the loop; unfinished requests are dropped. */
void acs_server_destroy(acs_server* srv);
/* Queue a solve of p (the problem handle may be destroyed afterwards).  A
 * request for the worker streams first has its device layouts built (on host
 * threads, once per problem handle) to size it against the budget, so on a
 * handle's first submit the call takes time that grows with nnz; the
 * request's latency_ms counts from the entry of this call. */
int acs_server_submit(acs_server* srv, const acs_problem* p, const acs_settings* s, uint64_t* ticket);
/* ACS_PENDING while unfinished; ACS_OK copies x, z (n), y (m) and info (any
 * may be NULL) and releases the ticket. */
int acs_server_poll(acs_server* srv, uint64_t ticket, double* x, double* y, double* z, acs_info* info);
/* As poll, blocking up to timeout_ms (< 0: no limit). */
int acs_server_wait(acs_server* srv, uint64_t ticket, int32_t timeout_ms, double* x, double* y, double* z,
                    acs_info* info);
/* Queued or pooled requests stop at once; a request on a worker stream is
 * marked and reported ACS_CANCELLED when it returns. */
int acs_server_cancel(acs_server* srv, uint64_t ticket);
int acs_server_stats(acs_server* srv, acs_server_counters* st);

#ifdef __cplusplus
}
#endif
#endif /* ACS_H_ */
