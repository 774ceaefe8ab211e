/*
 * astrobdf: batched stiff astrochemistry on one AMD Instinct MI355X (gfx950).
 *
 * The library integrates the mass-action rate equations of a chemical
 * reaction network (paper Sec. 2: dn_i/dt is a sum of one-body terms k n_a and
 * two-body terms k n_a n_b with production and destruction signs) over many
 * independent gas cells at once.  Each cell has its own physical conditions
 * phi = (T, n_H, A_V, zeta, G0) (paper Sec. 2, the generalised system
 * n' = f(n, k(phi), phi)) and its own initial abundances and horizon.
 *
 * The state variable is the fractional abundance x_i = n_i / n_H.  Two-body
 * rate coefficients are therefore multiplied by n_H.  Rate laws:
 *   two-body   alpha (T/300)^beta exp(-gamma/T)        (paper Sec. 2, Kooij-Arrhenius)
 *   cosmic ray alpha zeta                              (paper Sec. 2, direct ionisation)
 *   photo      alpha G0 exp(-gamma A_V)                (paper App. B.1, photo-reactions)
 *
 * Integrator: variable-order (1..5), variable-step BDF in backward-difference
 * form (the family the paper names as the standard in Sec. 1), with modified
 * Newton on M = I - c J, c = h / gamma_q.
 *
 * Conventions for every entry point:
 *  - Array arguments are HIP DEVICE pointers unless stated otherwise, owned by
 *    the caller, and are not retained after the call returns.
 *  - Per-cell arrays are cell-major and contiguous: x[c * S + i] is species i
 *    of cell c; k[c * R + r] is reaction r of cell c.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue on
 *    it and return once their results are written (they synchronise it).
 *  - Return value: ABDF_OK or an abdf_status error code; the matching message
 *    is available from abdf_last_error() on the calling thread.  No C++
 *    exception crosses this interface.  Per-cell integration failures are not
 *    call errors: they are reported in the per-cell status array.
 */
#ifndef ASTROBDF_H
#define ASTROBDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum abdf_status {
    ABDF_OK = 0,
    ABDF_E_ARG = 1,            /* invalid argument: null pointer, bad size, bad option */
    ABDF_E_PARSE = 2,          /* malformed network text */
    ABDF_E_NONCONSERVING = 3,  /* a reaction does not conserve an element or the charge */
    ABDF_E_IO = 4,             /* network file cannot be read */
    ABDF_E_DEVICE = 5,         /* HIP runtime error, or no device */
    ABDF_E_BUDGET = 6,         /* not even one cell fits in hbm_budget_bytes */
    ABDF_E_NOMEM = 7,          /* device allocation failed */
    ABDF_E_BUSY = 8            /* server queue full */
} abdf_status;

/* Per-cell outcome codes written to cell_status arrays. */
enum {
    ABDF_CELL_OK = 0,              /* reached t_end */
    ABDF_CELL_STEP_TOO_SMALL = 1,  /* h fell below 10 u |t| */
    ABDF_CELL_MAX_STEPS = 2,       /* more than max_steps step attempts */
    ABDF_CELL_NONFINITE = 3,       /* a non-finite abundance or error norm */
    ABDF_CELL_BAD_INPUT = 4,       /* non-finite or non-physical phi, x0, t_end or tolerances */
    ABDF_CELL_TAPE_FULL = 5        /* reserved: recording solves integrate past a full tape (see
                                    * abdf_solve_record) and no longer end with it */
};

/* Precision of the Newton-matrix factorisation.  Residuals, error norms,
 * step control and Newton updates are FP64 in both forms.  In the FP32-LU
 * form a cell whose corrector fails with a fresh Jacobian retries the step
 * with each FP32 solve refined once against an FP64 residual of the linear
 * system, and after a second such failure continues with FP64 factors
 * (counted in n_lu_fp64). */
enum {
    ABDF_PREC_FP64 = 0,
    ABDF_PREC_FP32_LU = 1
};

/* Integration method (abdf_options.method).
 *   ABDF_METHOD_BDF: variable-order (1..5), variable-step BDF in the
 *     quasi-constant-step backward-difference form (the stiff integrator of
 *     the paper's Sec. 1).
 *   ABDF_METHOD_ESDIRK5: Kvaerno's seven-stage ESDIRK of order 5 with an
 *     embedded order-4 estimate (the integrator of the paper's Sec. 4;
 *     Kvaerno, BIT 44, 2004): explicit first stage, six implicit stages with
 *     the one Newton matrix I - 0.26 h J(x_n) per step attempt, each stage
 *     solved by the same modified Newton iteration as a BDF corrector from the
 *     previous stage's value; error Y_7 - Y_6; step factor
 *     min(10, max(0.2, 0.9 err^(-1/5))), no growth right after a rejection,
 *     h / 2 after a corrector failure.  abdf_solve and abdf_solve_noalloc
 *     only; max_order is ignored, lu_reuse must be 0 and phi_tc NULL.  Per-cell
 *     counters: n_attempts step attempts, n_lu one factorisation per attempt,
 *     order 5. */
enum {
    ABDF_METHOD_BDF = 0,
    ABDF_METHOD_ESDIRK5 = 1
};

typedef struct abdf_network abdf_network;

typedef struct abdf_options {
    double rtol;               /* relative tolerance, > 0 (default 1e-6) */
    double atol;               /* absolute tolerance in x units, >= 0 (default 1e-20) */
    int32_t max_steps;         /* step attempts per cell (default 100000) */
    int32_t precision;         /* ABDF_PREC_* (default FP64) */
    int32_t check_every;       /* step attempts between host polls of the running count (default 8) */
    int32_t max_order;         /* highest BDF order the order selection may reach, 1..5;
                                * 0 = 5 (default 5).  1 is the implicit Euler method
                                * with the same error control. */
    uint64_t hbm_budget_bytes; /* bound on the library's device workspace, 0 = no bound */
    double newton_tol;         /* 0 = max(10 u / rtol, min(0.03, sqrt(rtol))) */
    double lu_reuse;           /* keep a cell's Newton-matrix factorisation while
                                * |c / c_lu - 1| <= lu_reuse, c = h / gamma_q and
                                * c_lu the value it was formed at, scaling each
                                * correction by 2 / (1 + c / c_lu); 0 (default) =
                                * refactor whenever c changes.  In [0, 1). */
    double h0;                 /* first step size [s], > 0 replaces the starting-step
                                * heuristic (still capped by t_end and h_max); 0 (default) =
                                * heuristic */
    double h_max;              /* upper bound on every step size [s]; 0 (default) = none */
    const double *atol_species; /* DEVICE array of S absolute tolerances (one per species,
                                 * each finite and >= 0) used in place of atol, or NULL
                                 * (default).  Read when the call (or server) starts; the
                                 * caller keeps ownership. */
    const double *phi_tc;      /* DEVICE array [n_cells] of expansion times t_c [s] (each
                                * finite and >= 0; 0 = constant conditions), or NULL
                                * (default: every cell's conditions are constant).  A cell
                                * with t_c > 0 follows phi_j(t) = phi_j(0) (1 + t/t_c)^(-p_j)
                                * for phi = (T, n_H, A_V, zeta, G0), p = phi_exp (an
                                * expanding flow, the outflow setting of paper App. A);
                                * each step attempt from t to t + h takes the rate
                                * coefficients at t + h.  abdf_solve and abdf_solve_noalloc
                                * only (ABDF_E_ARG elsewhere). */
    double phi_exp[5];         /* the exponents p_j (finite; default 0) */
    int32_t method;            /* ABDF_METHOD_* (default BDF) */
    int32_t reserved;          /* 0 */
} abdf_options;

/* Per-cell counters (written to a DEVICE array of n_cells structs). */
typedef struct abdf_cell_stats {
    int32_t n_steps;        /* accepted steps */
    int32_t n_attempts;     /* step attempts */
    int32_t n_err_reject;   /* rejections by the local error test */
    int32_t n_newton_fail;  /* corrector failures */
    int32_t n_rhs;          /* right-hand-side evaluations */
    int32_t n_jac;          /* Jacobian evaluations */
    int32_t n_lu;           /* Newton-matrix factorisations */
    int32_t order;          /* BDF order at the end */
    double h;               /* step size at the end [s] */
    double t;               /* time reached [s] */
    int32_t n_lu_fp64;      /* factorisations in FP64 (FP32-LU form: those after a fallback) */
    int32_t reserved;
} abdf_cell_stats;

/* Fills `opt` with the defaults listed in abdf_options. */
void abdf_options_default(abdf_options *opt);

/* Thread-local message describing the last non-OK status on this thread. */
const char *abdf_last_error(void);

/* ---------------------------------------------------------------- network --
 * The uniform network record (paper Sec. 4: species and reactions in one
 * common format, from which the incidence matrix is built).  Text format:
 *   astrobdf-network 1
 *   name <word>
 *   [albedo <omega>]                                  (optional, in [0, 1), default 0)
 *   elements <E> <symbol>...
 *   species <S>
 *   <i> <name> <charge> <count of each element>      (S lines)
 *   reactions <R>
 *   <r> <type> <nr> <r1> <r2> <np> <p1> <p2> <p3> <alpha> <beta> <gamma>   (R lines)
 *   end
 * type: 0 two-body, 1 cosmic ray, 2 photo, 3 photoreaction by cosmic-ray-induced
 * photons, k = alpha (T/300)^beta gamma zeta / (1 - omega) with gamma the
 * reaction's efficiency (paper App. B.1); unused reactant/product slots are -1.
 * Every reaction must conserve each element and the charge exactly (integer
 * check); otherwise ABDF_E_NONCONSERVING names the reaction.  The handle is
 * owned by the library, immutable after loading and safe to share between
 * threads; free it with abdf_network_free.  Loading does not touch the GPU.
 */
abdf_status abdf_network_load(const char *path, abdf_network **out);
abdf_status abdf_network_load_mem(const char *text, size_t len, abdf_network **out);
void abdf_network_free(abdf_network *net);
int32_t abdf_network_num_species(const abdf_network *net);
int32_t abdf_network_num_reactions(const abdf_network *net);
int32_t abdf_network_num_elements(const abdf_network *net);
/* Species name (pointer valid while the network lives), NULL if out of range. */
const char *abdf_network_species_name(const abdf_network *net, int32_t i);

/* ------------------------------------------------------------------ solve --
 * Integrates every cell from t = 0 to its t_end (seconds).
 *   T, n_H, A_V, zeta, G0 : [n_cells] physical conditions
 *   x0                    : [n_cells][S] initial fractional abundances
 *   t_end                 : [n_cells] horizon in seconds (0 returns x0)
 *   x_out                 : [n_cells][S] abundances at t_end (may alias nothing)
 *   cell_status           : [n_cells] ABDF_CELL_* codes
 *   stats                 : [n_cells] counters, or NULL
 * Cells beyond the workspace budget are admitted as earlier cells finish.
 * Errors: ABDF_E_ARG (null pointers, n_cells < 0, rtol <= 0, atol < 0,
 * max_steps < 1, unknown precision), ABDF_E_BUDGET, ABDF_E_NOMEM, ABDF_E_DEVICE.
 */
abdf_status abdf_solve(const abdf_network *net, int64_t n_cells,
                       const double *T, const double *n_H, const double *A_V,
                       const double *zeta, const double *G0,
                       const double *x0, const double *t_end,
                       const abdf_options *opt,
                       double *x_out, int32_t *cell_status, abdf_cell_stats *stats,
                       void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid device allocation): abdf_solve with the
 * same arguments, results and errors, that calls no hipMalloc, hipFree or
 * other allocating routine.  Its workspace is a 64 MiB device array built into
 * the library (each device the library runs on holds its own copy until the
 * process ends) and static host buffers; it holds as many slots as fit there
 * (e.g. 24 cells of the 500-species network, ~100 of the 200-species one, at
 * most 4096), bounded further by opt->hbm_budget_bytes, and admits further
 * cells as slots free up.  Attempts run on `stream` alone.
 * Requirements and limits:
 *  - the network's device tables must already be on the current device (any
 *    other solving call with this network on this device uploads them);
 *    otherwise ABDF_E_ARG;
 *  - ABDF_E_BUDGET when not even one cell's workspace fits in 64 MiB (or in
 *    opt->hbm_budget_bytes when that is smaller);
 *  - every call on one device shares that device's array and host buffers,
 *    which keep the last call's contents (the call clears what must start at
 *    zero): calls that overlap on one device race and must be serialised by
 *    the caller. */
abdf_status abdf_solve_noalloc(const abdf_network *net, int64_t n_cells,
                               const double *T, const double *n_H, const double *A_V,
                               const double *zeta, const double *G0,
                               const double *x0, const double *t_end,
                               const abdf_options *opt,
                               double *x_out, int32_t *cell_status, abdf_cell_stats *stats,
                               void *stream);

/* ---------------------------------------------------------------- serving --
 * A request server with continuous batching (one per network and device).
 * Requests of any number of cells, each with its own horizon, are queued on
 * submission; a worker thread admits cells of the oldest requests into device
 * slots whenever slots are free (the slot pool is sized by hbm_budget_bytes),
 * keeps each cell's BDF history (difference table, step, order, Newton
 * factor) on the device between step attempts, and refills slots as cells
 * finish, so requests that arrive while others run share the step loop.
 * Each cell's arithmetic does not depend on which other cells run beside it:
 * a request's results are bitwise the same alone and in any mix, and equal
 * those of abdf_solve at the same tolerances.
 *
 * Inputs are HOST arrays copied at submission (the caller may reuse them at
 * once).  Outputs are written to the caller's HOST buffers named in the
 * request, which must stay valid until the request's completion has been
 * returned by abdf_server_poll (or the server is destroyed).  The network
 * must outlive the server.  All functions are safe to call from any thread.
 */
typedef struct abdf_server abdf_server;

typedef struct abdf_server_options {
    abdf_options solve;        /* default tolerances, max_steps, precision, check_every, hbm_budget_bytes */
    int64_t max_slots;         /* cells resident at once; 0 = as many as the budget and free memory allow */
    int64_t max_queued_cells;  /* submit returns ABDF_E_BUSY beyond this many waiting cells; 0 = no bound */
} abdf_server_options;

typedef struct abdf_request {
    int64_t n_cells;
    const double *T, *n_H, *A_V, *zeta, *G0;  /* HOST [n_cells] */
    const double *x0;                         /* HOST [n_cells][S] */
    const double *t_end;                      /* HOST [n_cells], seconds */
    double rtol;                              /* <= 0: the server's default */
    double atol;                              /* < 0: the server's default */
    double *x_out;                            /* HOST [n_cells][S] */
    int32_t *cell_status;                     /* HOST [n_cells] */
    abdf_cell_stats *stats;                   /* HOST [n_cells], or NULL */
} abdf_request;

typedef struct abdf_completion {
    uint64_t id;
    int64_t n_cells;
    int64_t n_failed;       /* cells whose status is not ABDF_CELL_OK */
    int32_t cancelled;      /* 1: cancelled; the output buffers hold no result */
    int32_t reserved;
    double t_submit;        /* seconds on the server clock (abdf_server_clock) */
    double t_first_admit;   /* first cell placed in a slot, -1 if none */
    double t_done;          /* last cell's result written to the caller's buffers */
} abdf_completion;

typedef struct abdf_server_info {
    int64_t slots;              /* size of the slot pool */
    int64_t occupied;           /* slots holding a cell */
    int64_t queued_cells;       /* submitted, not yet admitted */
    int64_t completed_requests;
    int64_t completed_cells;
    double busy_slot_seconds;   /* integral of occupied slots over time */
    double uptime;              /* seconds since creation */
} abdf_server_info;

void abdf_server_options_default(abdf_server_options *opt);
/* Creates a server on the current HIP device.  Errors: ABDF_E_ARG,
 * ABDF_E_BUDGET (not one slot fits), ABDF_E_NOMEM, ABDF_E_DEVICE. */
abdf_status abdf_server_create(const abdf_network *net, const abdf_server_options *opt, abdf_server **out);
/* Queues a request and returns its id (ids start at 1 and increase).
 * Errors: ABDF_E_ARG (null pointers, n_cells < 0, non-finite tolerances),
 * ABDF_E_BUSY (queue bound reached), ABDF_E_DEVICE (the worker stopped on a
 * device error; abdf_last_error names it). */
abdf_status abdf_server_submit(abdf_server *srv, const abdf_request *req, uint64_t *id);
/* Returns up to `max` completions in completion order.  timeout_ms = 0 does
 * not wait; > 0 waits up to that long for the first one; < 0 waits until one
 * is available.  *n_out may be 0.  After a device error in the worker the
 * completions already made are still returned, then ABDF_E_DEVICE. */
abdf_status abdf_server_poll(abdf_server *srv, abdf_completion *out, int32_t max, int32_t *n_out,
                             int32_t timeout_ms);
/* Cancels a request: its cells not yet admitted are dropped, running ones are
 * discarded when they finish, and a completion with cancelled = 1 follows.
 * ABDF_E_ARG if the id was never issued; a request already complete is not
 * affected. */
abdf_status abdf_server_cancel(abdf_server *srv, uint64_t id);
/* Seconds since the server was created (monotonic clock). */
double abdf_server_clock(const abdf_server *srv);
abdf_status abdf_server_info_get(abdf_server *srv, abdf_server_info *out);
/* Stops the worker after its current step attempt, drops queued and running
 * requests (their buffers are no longer written) and frees the server. */
void abdf_server_destroy(abdf_server *srv);

/* ---------------------------------------------------------------- adjoint --
 * Gradients of a loss L(x(t_end)) with respect to the log rate prefactors,
 * dL/dlog alpha_r for every reaction (the sensitivities to the chemical
 * parameters of paper Sec. 2 and its differentiable-solver motivation), and
 * with respect to the initial abundances.
 *
 * The gradient is that of the discrete map the forward solve followed: its
 * accepted (h, q) sequence held fixed and each corrector equation taken as
 * solved exactly.  A recording solve keeps, per cell, that sequence and the
 * abundances after every accepted step (the checkpoint); the reverse sweep
 * walks it backwards with one fresh factorisation of I - c J(x_{n+1}) and
 * one transposed solve per step.  Factorisations are FP64.
 *
 * The tape holds max_tape_steps steps per cell.  A cell that takes more is
 * swept in windows of max_tape_steps steps, the last window first: before each
 * window the forward solve of the cells that need it runs again from the
 * tape's copies of the inputs, records that window and stops at its end (the
 * solve is deterministic, so it repeats the recorded steps exactly), and the
 * sweep carries its adjoint state from one window to the next.  The gradient
 * is therefore the same as with a tape long enough for every step; a cell of
 * N steps costs about N^2 / (2 max_tape_steps) extra forward steps.
 */
typedef struct abdf_tape abdf_tape;

/* Solves like abdf_solve and records the step tape.
 *   alpha          : DEVICE [R] rate prefactors to use, or NULL for the network's
 *   max_tape_steps : accepted steps the tape holds per cell (0 = 2048); a cell
 *                    that takes more is integrated to t_end all the same and
 *                    swept in windows (see above)
 *   tape           : receives the tape, owned by the caller (abdf_tape_free);
 *                    it holds its own copies of the inputs and of alpha
 * Device memory: n_cells * (max_tape_steps * (S + 2) + S + 16) doubles for the
 * tape, counted against opt->hbm_budget_bytes before the solver's slots.
 * Errors: as abdf_solve; ABDF_E_ARG also for precision other than FP64 or
 * max_tape_steps < 0; ABDF_E_BUDGET when the tape alone exceeds the budget.
 * The network must outlive the tape. */
abdf_status abdf_solve_record(const abdf_network *net, int64_t n_cells,
                              const double *T, const double *n_H, const double *A_V,
                              const double *zeta, const double *G0,
                              const double *x0, const double *t_end, const double *alpha,
                              const abdf_options *opt, int32_t max_tape_steps,
                              double *x_out, int32_t *cell_status, abdf_cell_stats *stats,
                              abdf_tape **tape, void *stream);

/* Reverse sweep of a tape for dL_dx = dL/dx(t_end) (DEVICE [n_cells][S]).
 * The sweep accumulates dL/dk_r, the gradient with respect to each cell's rate
 * coefficients; since k_r is linear in alpha_r, dL/dlog alpha_r = k_r dL/dk_r.
 * Outputs (DEVICE, each may be NULL):
 *   dL_dlog_alpha      [R]          summed over cells, in cell order
 *   dL_dlog_alpha_cell [n_cells][R] per cell
 *   dL_dx0             [n_cells][S]
 *   dL_dphi            [n_cells][5] per cell, columns T, n_H, A_V, zeta, G0:
 *                      sum_r dL/dk_r dk_r/dphi with the derivatives of the
 *                      rate laws written out (no division by zeta or G0, so
 *                      the columns are exact where zeta = 0 or G0 = 0)
 * Cells whose forward status was not ABDF_CELL_OK contribute zeros.  A tape
 * may be swept any number of times.  The first sweep of a tape with a cell
 * longer than max_tape_steps allocates n_cells * (9 S + R) doubles of window
 * buffers, kept with the tape.  Errors: ABDF_E_ARG, ABDF_E_NOMEM,
 * ABDF_E_DEVICE. */
abdf_status abdf_tape_adjoint(abdf_tape *tape, const double *dL_dx, double *dL_dlog_alpha,
                              double *dL_dlog_alpha_cell, double *dL_dx0, double *dL_dphi, void *stream);

/* Device bytes held by the tape's checkpoint (inputs, alpha, steps). */
int64_t abdf_tape_bytes(const abdf_tape *tape);
void abdf_tape_free(abdf_tape *tape);

/* Record, sweep and free in one call. */
abdf_status abdf_solve_adjoint(const abdf_network *net, int64_t n_cells,
                               const double *T, const double *n_H, const double *A_V,
                               const double *zeta, const double *G0,
                               const double *x0, const double *t_end, const double *alpha,
                               const abdf_options *opt, const double *dL_dx,
                               double *x_out, int32_t *cell_status,
                               double *dL_dlog_alpha, double *dL_dlog_alpha_cell, double *dL_dx0,
                               double *dL_dphi, abdf_cell_stats *stats, void *stream);

/* Gradients with respect to each cell's physical parameters, from the per-cell
 * gradients with respect to log alpha (dL_dlog_alpha_cell of
 * abdf_tape_adjoint / abdf_solve_adjoint; DEVICE [n_cells][R]).  Every rate
 * coefficient is alpha_r times a function of the cell's parameters (paper
 * Sec. 2 two-body and cosmic-ray laws, App. B.1 photo law) and the parameters
 * enter the rate equations only through the coefficients, so per cell
 *   dL/dphi_j = sum_r dL/dlog alpha_r * d log k_r / d phi_j,
 * with d log k_r/dT = (beta + gamma/T)/T and d log k_r/dn_H = 1/n_H (two-body),
 * d log k_r/dzeta = 1/zeta (cosmic ray), d log k_r/dA_V = -gamma and
 * d log k_r/dG0 = 1/G0 (photo).  T, n_H, A_V, zeta, G0: DEVICE [n_cells], the
 * solve's inputs.  dL_dphi: DEVICE [n_cells][5], columns T, n_H, A_V, zeta,
 * G0; the sums over reactions run in reaction order per thread, then in a
 * fixed tree, so results are deterministic.  Asynchronous on the stream.
 * A cell with zeta = 0 (G0 = 0) has k_r = 0 for its cosmic-ray (photo)
 * reactions, so dL/dlog alpha_r carries nothing of their zeta (G0) derivative:
 * that column is then not finite.  The dL_dphi output of abdf_tape_adjoint,
 * formed from dL/dk, is exact there.
 * Errors: ABDF_E_ARG (null or non-device pointers, n_cells out of range),
 * ABDF_E_DEVICE. */
abdf_status abdf_phys_gradient(const abdf_network *net, int64_t n_cells,
                               const double *T, const double *n_H, const double *A_V,
                               const double *zeta, const double *G0,
                               const double *dL_dlog_alpha_cell, double *dL_dphi, void *stream);

/* -------------------------------------------------- component entry points --
 * The steps of one BDF step on their own, for kernel-level checks and timing.
 */

/* Rate coefficients k [n_cells][R] (formulas at the top of this file). */
abdf_status abdf_rates(const abdf_network *net, int64_t n_cells,
                       const double *T, const double *n_H, const double *A_V,
                       const double *zeta, const double *G0,
                       double *k_out, void *stream);

/* Right-hand side f = nu . rate(x), rate_r = k_r x_a (x_b): f_out [n_cells][S]
 * from k [n_cells][R] and x [n_cells][S] (paper Sec. 2 rate equation). */
abdf_status abdf_rhs(const abdf_network *net, int64_t n_cells,
                     const double *k, const double *x, double *f_out, void *stream);

/* Newton matrix M = I - c J(x), J = df/dx, dense row-major [n_cells][S][S],
 * from k [n_cells][R], x [n_cells][S] and c [n_cells]. */
abdf_status abdf_newton_matrix(const abdf_network *net, int64_t n_cells,
                               const double *k, const double *x, const double *c,
                               double *M_out, void *stream);

/* Batched LU with partial pivoting, P A = L U, of `batch` dense row-major n x n
 * FP64 matrices A [batch][n][n], overwritten by L (unit, strictly lower) and U.
 * perm [batch][n]: row i of P A is row perm[i] of A.  precision
 * ABDF_PREC_FP32_LU rounds A to FP32 before factoring (result returned
 * widened to FP64).  A zero pivot leaves the column unscaled; info [batch]
 * (device, or NULL) receives 0 or the 1-based index of the first zero pivot. */
abdf_status abdf_lu_factor(int32_t n, int64_t batch, double *A, int32_t *perm,
                           int32_t *info, int32_t precision, void *stream);

/* Solves A z = b for each matrix, given the factors and perm of
 * abdf_lu_factor; b [batch][n] is overwritten by z. */
abdf_status abdf_lu_solve(int32_t n, int64_t batch, const double *LU, const int32_t *perm,
                          double *b, void *stream);

/* ------------------------------------------------------------- profiling --
 * Process-wide kernel timers: while enabled, the solver brackets each of its
 * kernel launches with HIP events on the launch stream and accumulates the
 * durations per kernel family when it next synchronises.
 */
enum {
    ABDF_PROF_ADMIT = 0,    /* admission: rates, starting step, first attempt */
    ABDF_PROF_FACTOR = 1,   /* Newton-matrix assembly + LU factorisation */
    ABDF_PROF_NEWTON = 2,   /* Newton correction: triangular solves, norm, tests, update */
    ABDF_PROF_CONTROL = 3,  /* error test, step/order control, next predictor */
    ABDF_PROF_HARVEST = 4,  /* copy-out of finished cells */
    ABDF_PROF_RHS = 5,      /* Newton residual: rates times abundances, species sums */
    ABDF_PROF_ADJ_SOLVE = 6,  /* reverse sweep: transposed triangular solves */
    ABDF_PROF_ADJ_STEP = 7,   /* reverse sweep: adjoint step update and parameter gradient */
    /* Newton residual and correction of the cells that keep their factorisation,
     * launched on a second stream beside the factorisation kernel; their event
     * spans include the time spent waiting for compute units it holds. */
    ABDF_PROF_RHS_SIDE = 8,
    ABDF_PROF_NEWTON_SIDE = 9,
    ABDF_PROF_RHS_EVAL = 10,  /* abdf_rhs: the right-hand-side kernel on its own */
    ABDF_PROF_KINDS = 11
};

typedef struct abdf_profile {
    int64_t launches[11];   /* kernel launches per family */
    double ms[11];          /* summed launch durations [ms] per family */
} abdf_profile;

/* Turns the timers on (nonzero) or off. */
void abdf_profile_enable(int32_t on);
/* Copies the accumulated timers; clears them when reset is nonzero. */
void abdf_profile_read(abdf_profile *out, int32_t reset);

/* Checks on the device that the matrix-core lane layouts the kernels assume
 * hold (FP64 and FP32).  ABDF_OK if they do, ABDF_E_DEVICE otherwise. */
abdf_status abdf_selftest(void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ASTROBDF_H */
