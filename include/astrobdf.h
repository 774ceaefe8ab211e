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
    ABDF_CELL_BAD_INPUT = 4        /* non-finite or non-physical phi, x0, t_end or tolerances */
};

/* Precision of the Newton-matrix factorisation.  Residuals, error norms,
 * step control and Newton updates are FP64 in both forms. */
enum {
    ABDF_PREC_FP64 = 0,
    ABDF_PREC_FP32_LU = 1
};

typedef struct abdf_network abdf_network;

typedef struct abdf_options {
    double rtol;               /* relative tolerance, > 0 (default 1e-6) */
    double atol;               /* absolute tolerance in x units, >= 0 (default 1e-20) */
    int32_t max_steps;         /* step attempts per cell (default 100000) */
    int32_t precision;         /* ABDF_PREC_* (default FP64) */
    int32_t check_every;       /* step attempts between host polls of the running count (default 8) */
    int32_t reserved0;
    uint64_t hbm_budget_bytes; /* bound on the library's device workspace, 0 = no bound */
    double newton_tol;         /* 0 = max(10 u / rtol, min(0.03, sqrt(rtol))) */
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
 *   elements <E> <symbol>...
 *   species <S>
 *   <i> <name> <charge> <count of each element>      (S lines)
 *   reactions <R>
 *   <r> <type> <nr> <r1> <r2> <np> <p1> <p2> <p3> <alpha> <beta> <gamma>   (R lines)
 *   end
 * type: 0 two-body, 1 cosmic ray, 2 photo; unused reactant/product slots are -1.
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
    ABDF_PROF_KINDS = 6
};

typedef struct abdf_profile {
    int64_t launches[8];    /* kernel launches per family */
    double ms[8];           /* summed launch durations [ms] per family */
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
