/*
 * fds.h -- C ABI of the MI355X FFT-preconditioned domain-decomposition solver
 * for the 2-D Helmholtz-Poisson equation  lap(p) + kappa p = f  on domains made
 * of concatenated rectangles (Jiang, Lian & Wang, arXiv 2509.23180).
 *
 * Method (paper Section 2):
 *   - each rectangle is discretised with the 5-point central-difference
 *     scheme (Section 2.1, uniform spacing h, delta = 1/h^2, kappa added on
 *     the diagonal as in the model equation of the Introduction);
 *   - the rectangles form a block system coupled through interface matrices
 *     R_ij = R_ji^T (Section 2.3); every rectangle touching only one other
 *     ("independent subdomain") is eliminated by a Schur complement, leaving
 *     L_c p_c = f'_c on the coupled centre rectangle;
 *   - L_c p_c = f'_c is solved by restarted GMRES preconditioned by A_c^{-1},
 *     the block operator without the Schur complement (Section 2.4), applied
 *     with a sine transform along one axis, one tridiagonal solve per mode
 *     along the other and the inverse sine transform (Section 2.1);
 *   - arms are back-substituted (Algorithm 1).
 *
 * Conventions shared by every entry point
 *   - All array arguments named "device" are device pointers of the current
 *     HIP device; they are never freed or retained by the library.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is ordered after everything already queued on `stream`; blocking calls
 *     return after it finished.
 *   - Return codes only; nothing throws across the ABI.  fds_last_error()
 *     gives a thread-local message for the last failing call.
 *
 * Geometry and layout (fds_plan_create)
 *   Rectangles are closed boxes of grid-node indices (i0, j0, i1, j1); node
 *   (i, j) sits at (i h, j h); interior nodes are i0 < i < i1, j0 < j < j1.
 *   Coupled subdomains are the rectangles that share an edge with two or
 *   more others; without one, the coupled "centre" is the rectangle that
 *   shares an edge with the most others (ties: first listed).  Several
 *   coupled rectangles (Section 2.4, closing remark: longer concatenations)
 *   must form a straight chain of equal width, each sharing a full side with
 *   the next; they and the lines between them are solved as ONE coupled
 *   block M (the union's interior).  Every other rectangle must share one
 *   FULL side of M (same extent) and no edge with any other rectangle.
 *   Nodes strictly inside a shared edge are unknowns: owned by the
 *   non-coupled rectangle on an edge of M ("arms own their interface line"),
 *   and by the rectangle listed first on an edge between two coupled ones.
 *   Corner nodes of shared edges and all other boundary nodes are Dirichlet
 *   nodes.  At most 64 rectangles.
 *
 *   Unknown vector (rhs, x): rectangle by rectangle in the given order, the
 *   owned nodes in row-major order (j ascending outer, i ascending inner).
 *   Dirichlet data (bc): rectangle by rectangle, values on the rectangle's
 *   whole closed box ((j1-j0+1) x (i1-i0+1), row-major); only entries at
 *   Dirichlet nodes are read.  bc may be NULL for homogeneous data.
 *   fds_plan_layout() returns the offsets of both layouts.
 */
#ifndef FDS_H
#define FDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FDS_OK = 0,
  FDS_PENDING = 1,            /* batch request not finished yet            */
  FDS_E_INVALID_ARG = -1,     /* bad pointer, size or option                */
  FDS_E_GEOMETRY = -2,        /* not a supported concatenation (see above)  */
  FDS_E_UNSUPPORTED = -3,     /* e.g. kappa making a mode oscillatory       */
  FDS_E_SINGULAR = -4,        /* a subdomain operator is singular           */
  FDS_E_NOMEM = -5,           /* device allocation failed / over budget     */
  FDS_E_NOT_CONVERGED = -6,   /* cycle cap or stagnation; best x returned   */
  FDS_E_NONFINITE = -7,       /* NaN/Inf in the right-hand side             */
  FDS_E_DEVICE = -8,          /* HIP runtime error                          */
  FDS_E_UNSUPPORTED_BC = -9   /* a boundary-condition kind this build does  */
                              /* not solve (see fds_bc)                     */
} fds_status;

typedef struct { int32_t i0, j0, i1, j1; } fds_rect;

/* Boundary-condition kinds of the paper's Section 2.2 (Dirichlet, Neumann,
 * periodic).  The kind selects the transform of each rectangle (sine
 * transform for Dirichlet), so it is fixed when the plan is made; the
 * Dirichlet VALUES are per-solve data and go to fds_solve / fds_batch_submit
 * with the right-hand side, so one plan serves any number of boundary data. */
typedef enum {
  FDS_BC_DIRICHLET = 0,
  FDS_BC_NEUMANN = 1,         /* reserved: FDS_E_UNSUPPORTED_BC             */
  FDS_BC_PERIODIC = 2         /* reserved: FDS_E_UNSUPPORTED_BC             */
} fds_bc_kind;

typedef struct {
  int32_t kind;               /* fds_bc_kind on every outer edge            */
  const int32_t* edge_kinds;  /* optional host array of 4 kinds per         */
                              /* rectangle (sides j=j0, i=i1, j=j1, i=i0),  */
                              /* overriding `kind`; entries on shared edges */
                              /* are ignored.  NULL: `kind` everywhere      */
} fds_bc;

typedef enum {
  FDS_FP64 = 0,               /* plain method: everything in FP64 (GMRES)   */
  FDS_FP32_PRECOND = 1,       /* FP32 sine transforms + tridiagonal solves  */
                              /* inside flexible GMRES; FP64 Gram-Schmidt,  */
                              /* Givens, operator, true residual, update    */
  FDS_NO_PRECOND = 2,         /* no preconditioner (P = I, Section 3.2's    */
                              /* baseline): flexible GMRES with z = v       */
                              /* stored in FP32; for convergence studies    */
  FDS_JACOBI = 3              /* Jacobi preconditioner P = diag(L_c), the   */
                              /* diagonal of the Schur-reduced operator     */
                              /* (Section 3.2's second baseline): flexible  */
                              /* GMRES with z = P^-1 v stored in FP32       */
} fds_precision;

typedef enum {
  FDS_STOP_NONE = 0,
  FDS_STOP_TOL = 1,           /* true relative residual <= tol              */
  FDS_STOP_AT_FLOOR = 2,      /* tol below the FP64 rounding floor; stopped */
                              /* at max(tol, 2*floor estimate), or a cycle  */
                              /* without 10% gain within twice that bound   */
  FDS_STOP_MAX_CYCLES = 3,
  FDS_STOP_STAGNATION = 4
} fds_stop_reason;

/* fds_options.flags */
enum {
  /* Interface Krylov iteration (FDS_FP64 only): the same right-preconditioned
   * GMRES(m), with its basis stored on the coupled rectangle's interface
   * lines.  The preconditioned operator I - S A_c^{-1} changes a vector only
   * on the lines that border an independent subdomain (S is zero elsewhere),
   * so every basis vector is a multiple of the cycle's interior residual plus
   * a vector on those lines; the Arnoldi step then costs O(line length)
   * memory traffic (plus O(nx ny) arithmetic for the coupling between the two
   * axes) instead of O(m nx ny), and the transforms and per-mode solves run
   * once per cycle.  Iterates equal those of the full-vector iteration up to
   * rounding.  Centres narrower than 2 nodes, or whose lines together exceed
   * 9215 nodes, use the full-vector iteration (the flag is then cleared in
   * the plan). */
  FDS_FLAG_INTERFACE_KRYLOV = 1u
};

typedef struct {
  int32_t restart_m;          /* Krylov dimension per cycle (default 30)    */
  int32_t max_cycles;         /* restart cap (default 200)                  */
  int32_t precision;          /* fds_precision                              */
  uint32_t flags;             /* FDS_FLAG_* (0: the full-vector iteration)  */
} fds_options;

typedef struct {
  int32_t status;             /* fds_status of this solve                   */
  int32_t iterations;         /* Arnoldi steps in total                     */
  int32_t cycles;             /* restarts + 1                               */
  int32_t stop_reason;        /* fds_stop_reason                            */
  double relres_schur;        /* ||f'_c - L_c x_c||_2/||f'_c||_2, FP64      */
  double relres_global;       /* ||b - A p||_2/||b||_2 on the composite grid */
  double seconds;             /* host wall time of the solve (blocking API) */
} fds_result;

typedef struct fds_plan fds_plan;
typedef struct fds_server fds_server;

/* ---------------------------------------------------------------- plans */

/* Validate the geometry, classify centre and arms (Section 2.4, last
 * paragraph: independent vs coupled subdomains), build the per-plan device
 * tables (sine-transform twiddles, per-mode tridiagonal coefficients, Schur
 * line coefficients) on the current device.  h > 0; kappa <= 0 is always
 * accepted; kappa > 0 is accepted only if every mode stays diagonally
 * dominant, else FDS_E_UNSUPPORTED (FDS_E_SINGULAR if a subdomain operator
 * has a zero eigenvalue).  bc (host struct) may be NULL (Dirichlet on every
 * outer edge); a Neumann or periodic edge gives FDS_E_UNSUPPORTED_BC, an
 * unknown kind FDS_E_INVALID_ARG.  opt may be NULL (defaults).  On success
 * *out owns the tables until fds_plan_destroy. */
fds_status fds_plan_create(const fds_rect* rects, int32_t nrect, double h, double kappa,
                           const fds_bc* bc, const fds_options* opt, fds_plan** out);
void fds_plan_destroy(fds_plan* plan);

/* Offsets (in doubles) of each rectangle's block in the unknown vector and in
 * the Dirichlet-data vector; both arrays have nrect+1 entries (last = total).
 * Either pointer may be NULL. */
fds_status fds_plan_layout(const fds_plan* plan, int64_t* unknown_offsets, int64_t* bc_offsets);

/* Device bytes one solve of this plan needs beyond rhs/bc/x (Krylov basis,
 * internal copies, scratch). */
fds_status fds_plan_footprint(const fds_plan* plan, size_t* bytes);

/* ---------------------------------------------------------------- solves */

/* Blocking solve of one problem (Algorithm 1): rhs (device, n_unknowns
 * doubles), bc (device, bc layout, or NULL), x (device, n_unknowns doubles,
 * written).  tol is the relative residual of the interface system
 * ||f'_c - L_c x_c||_2/||f'_c||_2 (x_0 = 0).  res may be NULL.  Returns the
 * solve's status (FDS_E_NOT_CONVERGED still writes the best x). */
fds_status fds_solve(fds_plan* plan, const double* rhs, const double* bc, double* x,
                     double tol, void* stream, fds_result* res);

/* Blocking solve of `count` independent problems in one batched engine: every
 * kernel of a GMRES iteration serves all unfinished problems in one launch.
 * plans[i] may repeat and may differ in size/shape/kappa; all plans must
 * share restart_m and precision.  rhs/bc/x/tol/res are arrays of length
 * count (bc entries may be NULL; res may be NULL).  The result of each
 * problem does not depend on the other members of the batch.  Returns
 * FDS_OK if every problem succeeded, else the first failing status. */
fds_status fds_solve_batch(fds_plan* const* plans, int32_t count, const double* const* rhs,
                           const double* const* bc, double* const* x, const double* tol,
                           void* stream, fds_result* res);

/* ---------------------------------------------------------------- serving */

/* A server runs a host thread that admits requests at GMRES-cycle
 * boundaries while earlier requests are still iterating (continuous
 * batching), as long as their footprint fits in hbm_budget_bytes and fewer
 * than max_slots are active.  Plans must outlive the server's use of them. */
fds_status fds_server_create(size_t hbm_budget_bytes, int32_t max_slots, fds_server** out);
void fds_server_destroy(fds_server* server);

/* Queue one solve; rhs/bc/x must stay valid until poll returns non-PENDING.
 * The solve reads rhs/bc only after all work queued on `stream` before this
 * call has completed (an event recorded on `stream`; NULL = the null stream),
 * so inputs produced asynchronously on the caller's stream are safe to
 * submit.  x is complete when poll returns non-PENDING.  FDS_E_NOMEM if the
 * request could never fit the budget. */
fds_status fds_batch_submit(fds_server* server, fds_plan* plan, const double* rhs,
                            const double* bc, double* x, double tol, void* stream,
                            uint64_t* ticket);

/* FDS_PENDING while the request is queued or running; otherwise its final
 * status, with *res filled (may be NULL).  res->seconds is the request's
 * latency: submission to publication of the result.  A finished ticket is
 * forgotten after the first non-PENDING poll. */
fds_status fds_batch_poll(fds_server* server, uint64_t ticket, fds_result* res);

/* Completion queue of a server: blocks until some request has finished and
 * has not been collected yet (by this call or fds_batch_poll), for at most
 * timeout_us microseconds (negative: no limit).  Sets *ticket and, when res
 * is not NULL, *res, forgets the ticket, and returns that request's final
 * status; returns FDS_PENDING (ticket untouched) on time-out.  Collects the
 * finished request with the smallest ticket first.  Thread-safe; the server
 * must not be destroyed while a call waits. */
fds_status fds_batch_wait_any(fds_server* server, int64_t timeout_us, uint64_t* ticket,
                              fds_result* res);

/* Counters of a server since it was created (a consistent snapshot). */
typedef struct {
  uint64_t submitted;         /* requests accepted by fds_batch_submit      */
  uint64_t admitted;          /* requests that started their set-up phase   */
  uint64_t completed;         /* results published                          */
  uint64_t admitted_mid_flight; /* admissions at a cycle boundary while     */
                              /* problems admitted earlier were still       */
                              /* iterating on the device                    */
  uint64_t cycles;            /* GMRES cycles stepped (all engine groups)   */
  int32_t queued;             /* waiting for a slot or for memory now       */
  int32_t running;            /* admitted and not yet retired now           */
  uint64_t bytes_in_use;      /* footprint of the running requests now      */
  uint64_t peak_bytes_in_use;
  double host_admit_s;        /* worker thread: admissions (set-up phases)  */
  double host_retire_s;       /*   retirements (back substitution, output)  */
  double host_tasks_s;        /*   task lists rebuilt after set changes     */
  double host_launch_s;       /*   queueing the cycles' kernels             */
  double host_wait_s;         /*   waiting for cycles to finish             */
} fds_server_stats;
fds_status fds_server_stats_get(fds_server* server, fds_server_stats* out);

/* ------------------------------------------------ kernel-level entry points
 * Single hot-path steps on raw device arrays, for verification and for
 * per-kernel measurement.  Layouts are row-major; `rows` x `n` arrays have
 * the transform axis contiguous. */

/* Unnormalised DST-I of every row (Section 2.1, sine eigenvectors; computed
 * through a complex FFT of length n+1):  out[r][k-1] = scale * sum_{j=1..n}
 * in[r][j-1] sin(pi j k/(n+1)).  in/out FP64 device arrays, may alias. */
fds_status fds_k_dst_rows(const double* in, double* out, int32_t rows, int32_t n, double scale,
                          void* stream);
/* Same in FP32. */
fds_status fds_k_dst_rows_f32(const float* in, float* out, int32_t rows, int32_t n, float scale,
                              void* stream);

/* Per-mode tridiagonal solves (Section 2.1, one independent system per sine
 * mode): for every column k (0 <= k < modes) solve, in place along the rows,
 *   delta y[i-1][k] + a_k y[i][k] + delta y[i+1][k] = scale * data[i][k],
 *   a_k = -4 delta + 2 delta cos((k+1) pi/(modes+1)) + kappa, delta = 1/h^2,
 * with zero data beyond the first and last row.  data: rows x modes FP64. */
fds_status fds_k_tridiag_modes(double* data, int32_t rows, int32_t modes, double h, double kappa,
                               double scale, void* stream);
fds_status fds_k_tridiag_modes_f32(float* data, int32_t rows, int32_t modes, double h,
                                   double kappa, double scale, void* stream);

/* Fast rectangle solve z = A^{-1} f for the rows x cols 5-point operator with
 * zero Dirichlet data (DST along the rows, tridiagonal solves along the
 * columns, inverse DST).  precision FDS_FP32_PRECOND runs the transforms and
 * solves in FP32 (f and z stay FP64). */
fds_status fds_k_rect_solve(const double* f, double* z, int32_t rows, int32_t cols, double h,
                            double kappa, int32_t precision, void* stream);

/* Interface operator of a plan's centre: w = L_c z = A_c z - sum_a S_ca z
 * (Section 2.3), z and w FP64 in the centre's row-major layout (n_y x n_x). */
fds_status fds_k_centre_operator(const fds_plan* plan, const double* z, double* w, void* stream);

/* One Arnoldi step with modified Gram-Schmidt (Section 2.4): V holds k
 * orthonormal rows of length len (device, FP64, row stride len) followed by a
 * row holding w; on return row k holds w orthogonalised and normalised and
 * h (device, k+1 doubles) holds <w_i, v_i> for i < k and the norm. */
fds_status fds_k_arnoldi_mgs(double* V, int32_t k, int64_t len, double* h, void* stream);

/* The same Arnoldi step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): its working memory (Hessenberg column, Gram matrix, block
 * partials and counters, state, task records) lives in a fixed array of 8 MiB
 * that each device holds from its first use until the process ends, and the
 * call allocates nothing.  V and h are as for fds_k_arnoldi_mgs and results
 * are identical.  Working memory grows with k and len (about
 * 8 (2k + 6) ceil(len / 2048) bytes of partials); a call that would need
 * more than the array holds fails with FDS_E_NOMEM before launching
 * anything.  All calls on one device share the array, which keeps the
 * previous call's contents (the call clears what must start at zero): calls
 * that overlap on one device race, so serialise them (one stream, or host
 * ordering). */
fds_status fds_k_arnoldi_mgs_noalloc(double* V, int32_t k, int64_t len, double* h, void* stream);

/* ---------------------------------------------------------------- misc */
const char* fds_status_str(fds_status s);
const char* fds_last_error(void);
/* Per-kernel-class timing with HIP events recorded on the launching stream
 * (off by default).  Classes: 0 sine transforms (k_dst_wave, k_dst_rows or
 * k_dst_gemm, whichever the tuner picked per length), 1 tridiagonal solves
 * (k_tridiag_seg or k_tridiag), 2 centre operator (k_operator, k_spec_op),
 * 3 Gram-Schmidt dot products (k_gram_dots, k_gram_bdots or k_ik_wdots),
 * 4 Schur line terms (k_lines_dense, the line transforms, or k_ik_cross),
 * 5 other small kernels, 6 Gram-Schmidt update (k_gram_update,
 * k_gram_update_lag or k_ik_update), 7 boundary columns (k_idst_cols).
 * `mask` selects the classes to time (bit c = class c; 0 = off).  Launches
 * from several threads (a server's groups) are each attributed to their own
 * thread's class.
 * fds_timing_read returns, per class, the launches timed, their summed
 * duration and the algorithmic bytes (minimal HBM traffic: every operand
 * read once and every result written once) the solver's work in those
 * launches required, all since the last reset.  fds_timing_read and
 * fds_timing_reset wait for the timed launches; call them when no timed
 * launch is being issued (e.g. between benchmark phases). */
fds_status fds_timing_enable(int32_t mask);
fds_status fds_timing_read(int32_t cls, int64_t* calls, double* total_ms);
fds_status fds_timing_bytes(int32_t cls, double* algorithmic_bytes);
fds_status fds_timing_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* FDS_H */
