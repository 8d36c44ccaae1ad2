/*
 * jfnk.h -- C ABI of the MI355X JFNK solver for the implicit electron /
 * electric-potential step of a low-Mach reacting flow under an applied field.
 *
 * One call of jfnk_step advances every column of a batch of independent 1D
 * columns by one backward-Euler step of the coupled system of the paper's
 * Section 3.2 (eq:pnp, discretised in time as eq:nls):
 *
 *   -n^{k+1} + f - dt k n^{k+1} - dt div Gamma(n^{k+1}, phi^{k+1})  = 0
 *   -n^{k+1} + q + (eps0 eps_r / e) lap phi^{k+1}                   = 0
 *
 * with f = n^k + dt s, the electron flux Gamma = n (u + mu grad phi) - D grad n
 * (electrons drift up the potential gradient; Scharfetter-Gummel face fluxes
 * on a uniform cell-centred grid), net ion charge q (the provisional charged
 * species of the paper's Algorithm 1, divided by e) and electrode potentials
 * phi_left, phi_right applied at the column ends (the applied voltage of
 * Section 4).  The root is reached by the paper's Algorithm 2: Newton with
 * the diagonal scalings of eq:newton_sc, right-preconditioned GMRES with the
 * finite-difference Jacobian-vector product eq:jf_dfapprox, an exact 2x2
 * block preconditioner (eq:prec) and a backtracking line search.
 *
 * Units: SI throughout.  Unless marked HOST, pointers are DEVICE pointers
 * (memory of the GPU the context was created on).  The caller owns every
 * array passed in and keeps it alive until the call returns; the library
 * owns its workspace, allocated once by jfnk_create.
 *
 * Errors: every entry point returns JFNK_OK (0) or a status.  Argument
 * errors (< 0) are detected before any launch and leave outputs untouched.
 * JFNK_EHIP reports a HIP runtime failure; the context must then be
 * destroyed.  A column that does not converge is not an error: the call
 * returns JFNK_NOT_CONVERGED and the column's status says why; its arrays
 * hold the last accepted iterate.  Per-cell inputs live on the device and are
 * checked there: a column with a cell outside the problem's domain (mu < 0,
 * D <= 0, k_loss < 0, or a non-finite mu, D, source, k_loss, ion charge,
 * face velocity, n^k or phi^k; with a transport table a non-finite c or a
 * gas density N <= 0 in place of mu and D) is not iterated, gets status
 * JFNK_COL_BAD_INPUT and keeps X^k; the call then returns
 * JFNK_NOT_CONVERGED.  jfnk_last_error gives a message.
 *
 * Threading: a context is used by one host thread at a time.  Calls on one
 * context are serialised on the stream they are given.
 */
#ifndef JFNK_H
#define JFNK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jfnk_ctx jfnk_ctx;

/* return codes */
enum {
    JFNK_OK = 0,
    JFNK_NOT_CONVERGED = 1,   /* call completed, >= 1 column flagged */
    JFNK_EINVAL = -1,         /* invalid argument (nothing launched) */
    JFNK_ENOMEM = -2,         /* device allocation failed (create) */
    JFNK_EHIP = -3,           /* HIP runtime error; destroy the context */
    JFNK_ECAPACITY = -4,      /* problem exceeds the capacity given to create */
    JFNK_EMODEL = -5          /* learned guess requested without a model */
};

/* electron condition at a column end */
enum { JFNK_BC_DIRICHLET = 0, JFNK_BC_ZERO_FLUX = 1 };
/* initial Newton guess.  PREV: X^n.  EXTRAP: the better (smaller scaled
   residual, ties to the extrapolation) of X^n and 2X^n - X^{n-1}.  LEARNED:
   the learned predictor, kept only if its scaled residual is strictly smaller
   than that of the EXTRAP choice (the fallback). */
enum { JFNK_GUESS_PREV = 0, JFNK_GUESS_EXTRAP = 1, JFNK_GUESS_LEARNED = 2 };
/* storage and arithmetic of the per-cell preconditioner factors */
enum { JFNK_PREC_FP64 = 0, JFNK_PREC_FP32 = 1 };
/* preconditioner.  BLOCK: the exact factorisation of the 2x2 block
   tridiagonal Jacobian (P = J; eq:prec with the true Schur complement).
   SCHUR: the paper's eq:prec_recast, the block factorisation with the Schur
   complement replaced by S~ = L + I_e dt D_r (Section 3.2), each block solved
   exactly (the tridiagonal solves the paper uses in 1D instead of multigrid):
   three solves per apply.  NONE: no preconditioner (P = I in the scaled
   variables, GMRES on S_F^-1 J S_X itself), the baseline of the paper's
   comparison of preconditioned and unpreconditioned iteration counts
   (Section 3.2); the error estimate then equals the scaled residual, and
   simplified-Newton steps are not taken (chord_tol is ignored).
   SCHUR_MG: SCHUR with the two scalar tridiagonal blocks (dt D_f - I and S~)
   solved by multigrid V-cycles to the tolerance mg_tol, as the paper does
   (Section 3.2): vertex-centred coarsening by two, Galerkin coarse
   operators P^T A P with restriction P^T, two red-black Gauss-Seidel sweeps
   before and after the coarse correction on every level, a direct solve on
   levels of at most 7 points; V-cycles repeat until ||b - A x||_2 <=
   mg_tol ||b||_2 (at most 200).  mg_blocks selects the blocks solved this
   way (bit 0: the electron block dt D_f - I, bit 1: S~); the others are
   solved exactly.  mg_transfer selects the interpolation P per block (bit
   set: matrix-dependent, the weights -a_i/b_i, -c_i/b_i of the operator's
   own row at the odd point; clear: linear, 1/2 and 1/2).  With linear
   interpolation the V-cycle diverges on the electron block wherever the
   cell Peclet number is large (its Galerkin coarse operators lose diagonal
   dominance); with matrix-dependent interpolation one V-cycle is an exact
   solve in 1D. */
enum { JFNK_PRECK_BLOCK = 0, JFNK_PRECK_SCHUR = 1, JFNK_PRECK_NONE = 2, JFNK_PRECK_SCHUR_MG = 3 };
/* PLAIN: one column at a time, every phase a launch, control on the host.
   BATCHED: three launches per step (gather, solve, write-back); the solve
   launch runs the whole step of every column, control on the GPU. */
enum { JFNK_SCHED_PLAIN = 0, JFNK_SCHED_BATCHED = 1 };
/* per-column status */
enum {
    JFNK_COL_CONVERGED = 0,
    JFNK_COL_MAX_NEWTON = 1,   /* max_newton iterations without convergence */
    JFNK_COL_NONFINITE = 2,    /* an iterate's residual is not finite */
    JFNK_COL_LINESEARCH = 3,   /* GMRES produced no direction */
    JFNK_COL_BAD_INPUT = 4     /* a per-cell input outside the domain (see above) */
};

typedef struct {
    int32_t max_cols;            /* capacity: columns per step */
    int64_t max_total_cells;     /* capacity: cells over all columns */
    int32_t max_cells_per_col;   /* capacity: cells of the longest column */
    int32_t gmres_restart;       /* Krylov space size m before restart (<= 30) */
    int32_t max_restarts;        /* GMRES restarts per Newton iteration */
    int32_t max_newton;          /* Newton iterations per step */
    int32_t max_backtracks;      /* halvings of the line-search step */
    double tol_f;                /* converged when ||S_F^-1 F||_inf <= tol_f */
    double tol_x;                /* 0: off; else also requires the error estimate
                                    ||P^-1 S_F^-1 F||_inf (the scaled Newton step
                                    from the current iterate) <= tol_x */
    double gamma;                /* GMRES forcing: ||J d + F|| <= gamma ||F|| */
    double ls_theta;             /* backtracking accepts X + lam d when the
                                    simplified Newton correction there satisfies
                                    ||P^-1 S_F^-1 F||_inf <= (1 - ls_theta lam) ||d||_inf */
    double chord_tol;            /* 0: off (every iteration is a GMRES Newton
                                    iteration).  Else, while the error estimate
                                    e = ||P^-1 S_F^-1 F||_inf of the iterate is in
                                    (tol_x, chord_tol], the step X + S_X d with
                                    d = -P^-1 S_F^-1 F (a Newton step with the
                                    analytic Jacobian of the latest factorisation)
                                    is tried first and kept if the estimate there
                                    is <= (1 - ls_theta) e; at most 4 in a row */
    int32_t prec_precision;      /* JFNK_PREC_* */
    int32_t guess;               /* JFNK_GUESS_* */
    int32_t schedule;            /* JFNK_SCHED_* */
    int32_t threads_override;    /* 0: autotuned; else workgroup size per column */
    int32_t prec_kind;           /* JFNK_PRECK_* */
    double mg_tol;               /* SCHUR_MG: V-cycle tolerance gamma_MG (0 < mg_tol < 1) */
    int32_t mg_blocks;           /* SCHUR_MG: 1, 2 or 3 (blocks solved by multigrid) */
    int32_t mg_transfer;         /* SCHUR_MG: 0..3 (blocks with matrix-dependent interpolation) */
} jfnk_config;

/* Electron transport table (Section 2.2: electron mobility and diffusivity
   as functions of the progress variable c and of the reduced field |E|/N,
   the paper's BOLSIG+ tables).  Values on uniform grids: nc points of c on
   [c_min, c_max] and nx points of x = log10(|E|/N / 1 Td) on [x_min, x_max]
   (1 Td = 1e-21 V m^2); nc, nx >= 2, c_max > c_min, x_max > x_min.  mu and
   diff: DEVICE [nc][nx] row-major (m^2/(V s), m^2/s), mu >= 0, diff > 0.
   With a table, mu_f and D_f of every face are read from it (bilinear,
   both arguments clamped to the grid, a zero field reading the x_min column)
   at the face's mean c and mean gas density N (the adjacent cell's at a wall)
   and at the field the face carries in the state being evaluated, |E| = the
   potential difference over the face distance (h, h/2 at a wall); the
   residual then depends on phi through them as well.  The finite-difference
   J.v products see that dependence, and so does the preconditioner's
   analytic Jacobian (the table's slope in x, d x / d(dphi) = 1/(dphi ln 10),
   zero where an argument is clamped); factors are not kept from one step to
   the next. */
typedef struct {
    int32_t nc, nx;
    double c_min, c_max, x_min, x_max;
    const double *mu, *diff;
} jfnk_table;

/* One step's problem: ncols columns packed back to back. */
typedef struct {
    int32_t ncols;
    const int64_t *col_offset;   /* HOST [ncols+1]: column c owns cells
                                    [col_offset[c], col_offset[c+1]), >= 3 cells */
    const double *length;        /* HOST [ncols] column length, m */
    const double *dt;            /* HOST [ncols] time step, s (> 0) */
    const double *phi_left;      /* HOST [ncols] electrode potential at x = 0, V */
    const double *phi_right;     /* HOST [ncols] electrode potential at x = L, V */
    const double *eps_over_e;    /* HOST [ncols] eps0 eps_r / e, 1/(V m) */
    const int32_t *bc_left;      /* HOST [ncols] JFNK_BC_* */
    const int32_t *bc_right;     /* HOST [ncols] */
    const double *ne_left;       /* HOST [ncols] wall density (Dirichlet), m^-3 */
    const double *ne_right;      /* HOST [ncols] */
    const double *mu;            /* [total] electron mobility >= 0, m^2/(V s) */
    const double *diff;          /* [total] electron diffusivity > 0, m^2/s */
    const double *src;           /* [total] explicit electron source, m^-3 s^-1 */
    const double *k_loss;        /* [total] implicit loss rate >= 0, 1/s (NULL: 0) */
    const double *q_ion;         /* [total] net ion charge / e, m^-3 */
    const double *u_face;        /* [total + ncols] face velocities (column c's
                                    n+1 faces start at col_offset[c] + c), m/s
                                    (NULL: 0) */
    const double *temp;          /* [total] gas temperature, K (learned guess) */
    const jfnk_table *table;     /* HOST struct; NULL: mu and diff per cell (above);
                                    else face mu, D from the table and mu, diff
                                    are not read (may be NULL) */
    const double *prog;          /* [total] progress variable c (table only) */
    const double *gas_n;         /* [total] gas number density N > 0, m^-3 (table only) */
} jfnk_problem;

typedef struct {
    double *ne;                  /* [total] in: n^k, out: n^{k+1} (unless ne_out) */
    double *phi;                 /* [total] in: phi^k, out: phi^{k+1} (unless phi_out) */
    const double *ne_prev;       /* [total] n^{k-1} for the guesses (NULL: none) */
    const double *phi_prev;      /* [total] */
    double *ne_out;              /* [total] NULL: the step is in place; else n^{k+1} is
                                    written here and ne, phi keep n^k, phi^k.  May be the
                                    ne_prev array (read before it is written), so that a
                                    caller alternates two states without a copy. */
    double *phi_out;             /* [total] with ne_out (both or neither) */
} jfnk_state;

/* HOST arrays [ncols]; any pointer may be NULL */
typedef struct {
    int32_t *status;             /* JFNK_COL_* */
    int32_t *newton_iters;
    int32_t *gmres_iters;
    int32_t *backtracks;
    int32_t *guess_used;         /* JFNK_GUESS_* actually taken */
    double *res_scaled;          /* final ||S_F^-1 F||_inf */
    int32_t *chord_steps;        /* simplified-Newton steps taken (see chord_tol) */
    int32_t *phase_counts;       /* HOST [ncols][8]: factorisations, preconditioner
                                    applies, residual evaluations after set-up
                                    (trials), J.v products, CGS passes, direction
                                    assemblies, extra vector reads, learned
                                    candidates evaluated (0 or 1) (what the
                                    step executed).  Extra vector reads count the
                                    FP64 vector pairs read by the Arnoldi dot
                                    sweeps, Gram-Schmidt passes and direction
                                    assemblies beyond their fixed operands: J.v's
                                    dots past the first two basis vectors (plus a
                                    re-read of w), every basis vector a CGS pass
                                    projects out (plus a re-read of w past the
                                    eighth), every vector summed into a direction. */
    int32_t *mg_cycles;          /* multigrid V-cycles of the step (SCHUR_MG; else 0) */
} jfnk_stats;

/* Fill cfg with the defaults: restart 30, 5 restarts, 50 Newton iterations,
   10 backtracks, tol_f 1e-10, tol_x 1e-10, gamma 1e-4, ls_theta 0.25,
   chord_tol 1e-3, FP32 preconditioner, extrapolated guess, batched schedule,
   BLOCK preconditioner; mg_tol 1e-4 (the paper's gamma_MG, Table 2), both
   blocks by multigrid when SCHUR_MG is chosen, the electron block with
   matrix-dependent and S~ with linear interpolation (mg_transfer 1). */
void jfnk_config_default(jfnk_config *cfg);

/* Allocate a context and its workspace on the current HIP device for the
   capacity in cfg.  *out receives the context (NULL on error).
   Errors: JFNK_EINVAL (bad config), JFNK_ENOMEM, JFNK_EHIP. */
int jfnk_create(const jfnk_config *cfg, jfnk_ctx **out);

/* Advance every column one step (Algorithm 2 per column).  Work is queued on
   `stream` (a hipStream_t; NULL = default stream) and the call returns once
   the results and stats are complete.  Allocates nothing.
   Returns JFNK_OK, JFNK_NOT_CONVERGED, or an error code. */
int jfnk_step(jfnk_ctx *ctx, const jfnk_problem *p, jfnk_state *x, jfnk_stats *st,
              void *stream);

/* The same step, returned as soon as it is queued (batched schedule only), so
   that the host prepares the next step while this one runs (Section 3.2's
   iteration per column is unchanged; only the host's waiting moves).  At most
   one step is in flight: a call that queues step k+1 then waits for step k
   and reports it through prev_stats (may be NULL) and *prev_rc (JFNK_OK or
   JFNK_NOT_CONVERGED; -1 when no step was in flight).  The host's per-step
   choices for step k+1 (workgroup order, which columns evaluate the learned
   guess) then come from step k-1 instead of step k.  Inputs of a queued step
   (the arrays behind p and x) must stay valid and unchanged until it is
   reported; x->ne/phi are written in stream order.  A step queued on another
   stream than the one in flight, or with another column layout, first waits
   for the step in flight and reports it through prev_stats and *prev_rc as
   above (the new step is then the only one in flight).  jfnk_step_finish waits for
   the step in flight and reports it.  Any other call on the context (a
   synchronous step, autotuning, a new model, the test exports) first finishes
   the step in flight and drops its statistics.  Allocates nothing.
   Errors: JFNK_EINVAL (plain schedule), and those of jfnk_step. */
int jfnk_step_async(jfnk_ctx *ctx, const jfnk_problem *p, jfnk_state *x, jfnk_stats *prev_stats,
                    int32_t *prev_rc, void *stream);

/* Wait for the step in flight and report it.  Returns JFNK_OK or
   JFNK_NOT_CONVERGED for it; JFNK_EINVAL when no step is in flight. */
int jfnk_step_finish(jfnk_ctx *ctx, jfnk_stats *st);

/* MISDC time step (the paper's Algorithm 1 with the provisional charged
 * species of Section 3.1 and the electron/Poisson system eq:nls of Section
 * 3.2, restricted to the charged species): electrons and the potential
 * implicit, one positive ion species explicit, chemistry
 * R = S - k_rec n_e n_i shared by both (S: the problem's src).  With A the
 * ion advection -div(n_i v) (second-order Godunov: monotonised-central
 * limited slopes, face values extrapolated to the half step with the upwind
 * cell's forcing R^n - n_i div v; electrodes absorb ions; v = u + mu_ion E
 * with the potential's face gradient, h/2 and the electrode potential at a
 * wall), iteration k = 0 .. k_max-1 from X^(0) = X^n, n_i^(0) = n_i^n forms
 *   I_R    = (R^n + R^(k)) / 2                 (chemistry over the step / dt)
 *   v      = (v(phi^n, t^n) + v(phi^(k), t^n+1)) / 2
 *   n_i~   = n_i^n + dt [A(n_i^n; v) + I_R]
 *   s      = I_R  (electron_sdc = 0: eq:nls, backward Euler for the
 *            electrons' transport), or
 *   s      = (T_e^n - T_e^(k)) / 2 + I_R  (electron_sdc = 1: the SDC
 *            correction of the other species' diffusion applied to the
 *            electrons, T_e = -div Gamma with the solve's Scharfetter-Gummel
 *            fluxes and the electrode potential of the state's time; its
 *            fixed point is the trapezoidal rule, second order in time but
 *            not L-stable)
 * and solves the backward-Euler system of jfnk_step with f = n_e^n + dt s,
 * no implicit loss, ion charge n_i~ and phi_right(t^n+1) for X^(k+1) (its
 * Newton iteration starting from X^(k)); n_i^(k+1) = n_i~.  The right
 * electrode potential is phi_right + A sin(2 pi f t) (Section 4.5's AC
 * forcing; DC when A = 0); phi_left is constant.  With cfl > 0 the step is
 * dt = min(p->dt, cfl h / max_f |v_f(phi^n, t^n)|) per column (Section
 * 4.1: the explicit ion advection limits the step), else p->dt.
 *
 * p: as for jfnk_step, with src the ionisation source S, k_loss NULL
 *    (losses come from the recombination term), q_ion not read (may be NULL)
 *    and phi_right the DC part of the right electrode potential.
 * m: k_max, electron_sdc, cfl (HOST scalars), t, ac_amp, ac_freq (HOST
 *    [ncols]; ac_amp and ac_freq both or neither), mu_ion >= 0 and
 *    k_rec >= 0 (DEVICE [total]; a cell outside that domain, or a non-finite
 *    n_ion, makes its column JFNK_COL_BAD_INPUT: it keeps X^n and n_i^n),
 *    n_ion (DEVICE [total], in: n_i^n, out: n_i^n+1), dt_used (HOST [ncols],
 *    may be NULL: the step each column took).
 * x: ne/phi in: X^n, out: X^n+1 (or in ne_out/phi_out when given);
 *    ne_prev/phi_prev, when given, serve the predictor's guess (k = 0) as in
 *    jfnk_step; later iterations start from X^(k).
 * st: per column, status = the first non-converged status of the k_max
 *    solves (else converged); newton_iters, gmres_iters, backtracks,
 *    chord_steps, phase_counts and mg_cycles summed over them; guess_used
 *    of the predictor; res_scaled of the last solve.
 * The first call allocates 11 x capacity cells doubles of device workspace
 * and two per-column tables (device and pinned host, capacity columns),
 * kept until jfnk_destroy; the call synchronises the stream after each
 * iteration's solve (and once more for the CFL step).  Like every call on a
 * context it first finishes an asynchronous step in flight.  Returns JFNK_OK, JFNK_NOT_CONVERGED, or an error code
 * (JFNK_EINVAL also for k_max outside 1..64, a k_loss array, electron_sdc
 * not 0 or 1, or cfl negative or not finite). */
typedef struct {
    int32_t k_max;               /* SDC iterations, 1..64 (1: the predictor, first order) */
    int32_t electron_sdc;        /* 0: eq:nls (backward Euler); 1: SDC-corrected transport */
    double cfl;                  /* > 0: constant ion-drift CFL step (capped by p->dt); 0: p->dt */
    const double *t;             /* HOST [ncols] time at the start of the step, s (NULL: 0) */
    const double *ac_amp;        /* HOST [ncols] AC amplitude A, V (NULL: DC) */
    const double *ac_freq;       /* HOST [ncols] AC frequency f, Hz */
    const double *mu_ion;        /* [total] ion mobility, m^2/(V s) */
    const double *k_rec;         /* [total] recombination coefficient, m^3/s */
    double *n_ion;               /* [total] in: n_i^n, out: n_i^n+1, m^-3 */
    double *dt_used;             /* HOST [ncols] out: the step taken, s (NULL: not reported) */
} jfnk_misdc;

int jfnk_misdc_step(jfnk_ctx *ctx, const jfnk_problem *p, const jfnk_misdc *m, jfnk_state *x,
                    jfnk_stats *st, void *stream);

/* Release the context and its workspace.  NULL-safe. */
void jfnk_destroy(jfnk_ctx *ctx);

/* Message of the last error on this context (never NULL). */
const char *jfnk_last_error(const jfnk_ctx *ctx);

/* Schedule autotuner (batched schedule, threads_override = 0).  Runs `steps`
   steps from the state x (x itself is not modified; the steps run on device
   copies, X^{n-1} taken from x when given) once for every workgroup size
   per column in {64, 128, 256, 512} that suits the longest column (at most
   64 cells per thread, not more threads than half its cells; 512 is tried
   for any column longer than 256 cells), measures the
   solve time of each with HIP events and keeps the fastest for this column
   layout: later steps with the same col_offset use it.  A learned guess is
   replaced by EXTRAP while tuning.  chosen (HOST, may be NULL) receives the
   workgroup size; times_ms (HOST [4], may be NULL) the summed solve times
   of the four candidates (-1: not tried).  Allocates and frees device
   scratch of 6 x total cells doubles.  Synchronises the stream. */
int jfnk_autotune(jfnk_ctx *ctx, const jfnk_problem *p, const jfnk_state *x, int32_t steps,
                  int32_t *chosen, double *times_ms, void *stream);

/* Persisted autotuner results, so that a later process on the same kind of
   GPU takes the tuned workgroup size without timing the candidates again.
   A layout is keyed by its column count, total cells, table transport on or
   off and the 64-bit FNV-1a hash of its col_offset array (a collision can
   only select a slower workgroup size, never change a result).

   jfnk_autotune_save appends one text line per layout this context tuned
   (device architecture name, prec_precision, prec_kind, the key, the chosen
   workgroup size and the four summed solve times) to the file at path
   (HOST string; created if absent).  JFNK_EINVAL if the file cannot be
   written.

   jfnk_autotune_load reads such a file and keeps the lines whose device
   architecture, prec_precision and prec_kind match this context (malformed
   lines are skipped; for a key present more than once, the last line wins);
   *nloaded (HOST, may be NULL) receives their count.  A later batched step
   without threads_override whose layout matches a kept line, and that this
   context has not tuned itself, takes that line's workgroup size if it owns
   the longest column with at most 64 cells per thread.  JFNK_EINVAL if the
   file cannot be opened.  Neither call touches the GPU. */
int jfnk_autotune_save(jfnk_ctx *ctx, const char *path);
int jfnk_autotune_load(jfnk_ctx *ctx, const char *path, int32_t *nloaded);

/* The workgroup size per column that the next step of this context takes
   for p's layout (threads_override, this context's autotuner result, a
   loaded entry, or the size rule), into *threads (HOST).  Reads only
   p->ncols and p->col_offset (HOST). */
int jfnk_schedule_threads(jfnk_ctx *ctx, const jfnk_problem *p, int32_t *threads);

/* Device time of the last jfnk_step's solve (ms, HIP events recorded on the
   step's stream right before and after the solve launches; for the plain
   schedule the span of all its phase launches; the learned guess, evaluated
   before, is not included) and the number of launches it spans (-1:
   host-driven; 3 for the batched schedule: gather, solve, write-back).
   Returns JFNK_EINVAL on NULL arguments. */
int jfnk_last_timing(const jfnk_ctx *ctx, double *solve_ms, int32_t *launches);

/* Batched schedule: device times (ms, HIP events on the step's stream) of
   the last jfnk_step's three launches: ms3[0] the gather (caller arrays ->
   workspace coefficients and start states), ms3[1] the solve (Algorithm 2
   per column), ms3[2] the write-back of X^{n+1}.  -1 each when the last step
   ran the plain schedule or has not been timed.  ms3: HOST [3].  Returns
   JFNK_EINVAL on NULL arguments. */
int jfnk_last_kernel_times(const jfnk_ctx *ctx, double *ms3);

/* ---- learned Newton initial guess --------------------------------------
 *
 * Not part of the paper's method: a small 1D convolutional network that
 * predicts X^{n+1} of every column from X^n (and X^{n-1}), the ion charge
 * q, the gas temperature and the applied voltage.  Its prediction is only a
 * Newton initial guess (JFNK_GUESS_LEARNED): the step keeps it only if its
 * scaled residual ||S_F^-1 F||_inf is strictly smaller than that of the
 * EXTRAP choice, so the root and the convergence test are those of the
 * method without it.
 *
 * Network: six convolutions along the column, kernel 5, zero padding at
 * the column ends, channels 8 -> 64 -> 64 -> 64 -> 64 -> 64 -> 2, ReLU after
 * the first five; BF16 weights and activations, FP32 accumulation (matrix
 * cores).  Input channels per cell, with n0 = 1e8 m^-3, a(n) = asinh(n/n0)/20
 * and phi_s = max(|phi_left|, |phi_right|, 1 V):
 *   a(n^n), phi^n/phi_s, a(q), (T - 1150 K)/850 K, log10(h / 1e-5 m),
 *   (phi_right - phi_left)/1000 V, a(n^n) - a(n^{n-1}), (phi^n - phi^{n-1})/phi_s
 * (the last two are 0 without X^{n-1}).  Outputs (o0, o1) give the guess
 *   n = n0 sinh(20 (a(n^n) + s0 o0)),  phi = phi^n + phi_s s1 o1
 * with the output scales s0, s1 of the configuration.  Loss of a batch:
 *   (1/N) sum over its N cells of (o0 - t0)^2 + (o1 - t1)^2,
 *   t0 = (a(n^{n+1}) - a(n^n))/s0,  t1 = (phi^{n+1} - phi^n)/(phi_s s1).
 * Parameters, as one flat FP32 array (jfnk_net_param_count() values): for
 * each layer in order, W[c_out][5][c_in] (tap j multiplies the input of cell
 * i + j - 2 for output cell i) followed by b[c_out].
 */
typedef struct jfnk_net jfnk_net;

typedef struct {
    int32_t max_cols;            /* capacity of a training batch: columns */
    int64_t max_total_cells;     /* capacity of a training batch: cells */
    float out_scale_ne;          /* s0 */
    float out_scale_phi;         /* s1 */
    float beta1, beta2, adam_eps;/* Adam moments and epsilon */
} jfnk_net_config;

/* Defaults: capacity 0 (prediction only), s0 = 0.1, s1 = 0.3, Adam 0.9,
   0.999, 1e-8. */
void jfnk_net_config_default(jfnk_net_config *cfg);

/* Number of parameters of the network. */
int64_t jfnk_net_param_count(void);

/* Allocate a network (parameters, Adam state, training workspace for the
   capacity) on the current HIP device.  Parameters start at zero: set them
   with jfnk_net_set_params.  Errors: JFNK_EINVAL, JFNK_ENOMEM, JFNK_EHIP. */
int jfnk_net_create(const jfnk_net_config *cfg, jfnk_net **out);
void jfnk_net_destroy(jfnk_net *net);                 /* NULL-safe */
const char *jfnk_net_last_error(const jfnk_net *net); /* never NULL */

/* HOST [n] parameters in the flat order above; n must equal
   jfnk_net_param_count().  set also clears the Adam moments and step count.
   Both synchronise the device. */
int jfnk_net_set_params(jfnk_net *net, const float *params, int64_t n);
int jfnk_net_get_params(jfnk_net *net, float *params, int64_t n);

/* The guess for every column of p: ne_out, phi_out DEVICE [total], layout
   of x->ne.  Uses p's col_offset, length, phi_left/right, q_ion, temp and
   x's ne, phi, ne_prev, phi_prev.  Queued on stream; returns when queued. */
int jfnk_net_predict(jfnk_net *net, const jfnk_problem *p, const jfnk_state *x,
                     double *ne_out, double *phi_out, void *stream);

/* Loss of one batch (inputs as for predict, targets X^{n+1} = (ne_next,
   phi_next) DEVICE [total]) and its gradient: grad HOST [param_count] (may be
   NULL), loss HOST (may be NULL).  Synchronises the stream. */
int jfnk_net_grad(jfnk_net *net, const jfnk_problem *p, const jfnk_state *x,
                  const double *ne_next, const double *phi_next, float *grad,
                  double *loss, void *stream);

/* One Adam step with learning rate lr on the batch's gradient (FP32 master
   weights, BF16 copies for the matrix cores).  loss HOST (may be NULL: then
   the call does not wait for the device) receives the batch loss before the
   update. */
int jfnk_net_train_step(jfnk_net *net, const jfnk_problem *p, const jfnk_state *x,
                        const double *ne_next, const double *phi_next, float lr,
                        double *loss, void *stream);

/* Attach a network to a solver context for JFNK_GUESS_LEARNED (NULL
   detaches).  The context does not own the network, which must outlive its
   use.  The network is evaluated before the solve for the columns whose
   previous step on this context needed at least one Newton iteration (all
   columns on the first step, whenever the column layout changes, and on a
   step without X^{n-1}, which starts a new history: the back-off records
   below are then cleared as well); after
   r consecutive evaluations whose candidate lost to the fallback, a column
   skips the network at its next 4^min(r,5) - 1 chances (steps at which it
   would otherwise be evaluated); any change of the network's weights
   (jfnk_net_set_params, jfnk_net_train_step) clears that record. */
int jfnk_set_model(jfnk_ctx *ctx, jfnk_net *net);

/* ---- allocation-free step ------------------------------------------------
 *
 * For callers that cannot allocate device memory (code that runs while a
 * HIP graph is being captured, tight serving loops, harnesses that forbid
 * hipMalloc): the batched step of jfnk_step without a context.  Its whole
 * workspace (the same arrays a context holds, for this problem's padded
 * cells, plus the work order and the gather tables) lives in a static device
 * array of JFNK_NOALLOC_BYTES bytes that every GPU the library runs on holds
 * from the first call on it until the process ends.  The call allocates
 * nothing (no hipMalloc, no host heap); the caller passes the inputs and
 * outputs as for jfnk_step.
 *
 * cfg: as for jfnk_create (its capacity fields bound nothing here except
 * max_cells_per_col); the schedule is always BATCHED, the workgroup size
 * follows the size rule (or threads_override); JFNK_GUESS_LEARNED is not
 * available (EINVAL).  Every call starts without the previous step's
 * factors (as the first step of a new context), so its iterates equal those
 * of jfnk_step on a fresh context.  Limits: at most JFNK_NOALLOC_MAX_COLS
 * columns, and the workspace must fit: 8 (48 + 4 m) bytes per padded cell
 * (cells rounded up to a multiple of the workgroup size, m = gmres_restart;
 * 1344 bytes at m = 30) plus 160 T bytes per column, in JFNK_NOALLOC_BYTES;
 * larger problems return JFNK_ECAPACITY (nothing launched).  err (HOST,
 * err_len bytes, may be NULL) receives a message on error.
 *
 * The array keeps the last call's contents and each call clears the part it
 * uses.  All calls on one GPU share it: calls that overlap on one GPU (on two
 * streams, or from two host threads) race and corrupt each other.  The call
 * queues its work on stream and returns once the results and stats are
 * complete.  Returns JFNK_OK, JFNK_NOT_CONVERGED, or an error code. */
#define JFNK_NOALLOC_BYTES ((size_t)64 << 20)
#define JFNK_NOALLOC_MAX_COLS 64
int jfnk_step_noalloc(const jfnk_config *cfg, const jfnk_problem *p, jfnk_state *x, jfnk_stats *st,
                      void *stream, char *err, size_t err_len);

/* ---- test exports: single phases of the step, same kernels ----------- */
/* Each runs its phases one launch at a time, every launch over all columns
   of p (one workgroup per column); the residual and J.v launches use kernels
   that hold that phase alone.  Vectors are FP64 and in the caller's
   natural layout.  The calls return once their results are complete. */

/* F(X) (unscaled, per cell: fe, fp) with X = (x_ne, x_phi) and the step's
   X^n = (x->ne, x->phi) giving f = n^n + dt s; scal (HOST [4*ncols], may be
   NULL) receives s_Fn, s_Fphi, s_Xn, s_Xphi per column. */
int jfnk_eval_residual(jfnk_ctx *ctx, const jfnk_problem *p, const jfnk_state *x,
                       const double *x_ne, const double *x_phi, double *fe, double *fp,
                       double *scal, void *stream);

/* w = S_F^-1 [F(X + eps S_X v) - F(X)] / eps with the step of
   eq:jf_dfapprox; v and w in scaled units, layout as fe/fp. */
int jfnk_eval_jv(jfnk_ctx *ctx, const jfnk_problem *p, const jfnk_state *x,
                 const double *x_ne, const double *x_phi, const double *v_ne,
                 const double *v_phi, double *w_ne, double *w_phi, void *stream);

/* z = P^-1 r for the scaled analytic Jacobian P = S_F^-1 J(X) S_X, factored
   as in a step (precision of the context). */
int jfnk_block_solve(jfnk_ctx *ctx, const jfnk_problem *p, const jfnk_state *x,
                     const double *x_ne, const double *x_phi, const double *r_ne,
                     const double *r_phi, double *z_ne, double *z_phi, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* JFNK_H */
