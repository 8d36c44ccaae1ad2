/*
 * CPU oracle for the implicit electron / electric-potential step.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product library.
 */
#ifndef JFNK_ORACLE_H
#define JFNK_ORACLE_H

#define ORC_BC_DIRICHLET 0
#define ORC_BC_ZERO_FLUX 1

/* band of the 2x2-block-tridiagonal Jacobian with unknowns interleaved
   (n_0, phi_0, n_1, ...): 2 sub-diagonals, 3 super-diagonals, plus KL
   columns of room for pivoting fill-in */
#define ORC_KL 2
#define ORC_KU 3
#define ORC_BAND_W (2 * ORC_KL + ORC_KU + 1)

enum { ORC_CONVERGED = 0, ORC_MAX_ITERS = 1, ORC_NONFINITE = 2, ORC_SINGULAR = 3 };

/* Electron transport table (Section 2.2): mobility and diffusivity on a
   uniform grid of the progress variable c (nc points on [c_min, c_max]) and
   of x = log10(|E|/N / 1 Td) (nx points on [x_min, x_max]), row-major
   [nc][nx]; bilinear interpolation, both arguments clamped to the grid. */
typedef struct {
    int nc, nx;
    double c_min, c_max, x_min, x_max;
    const double *mu, *diff;
} orc_table;

typedef struct {
    int n;                       /* cells */
    double length;               /* m */
    double dt;                   /* s */
    double phi_left, phi_right;  /* electrode potentials, V */
    double eps_over_e;           /* eps0 eps_r / e, (V m)^-1 */
    int bc_left, bc_right;       /* electron wall condition */
    double ne_left, ne_right;    /* wall density for Dirichlet walls, m^-3 */
    const double *mu;            /* [n] mobility, m^2/(V s) */
    const double *diff;          /* [n] diffusivity, m^2/s */
    const double *src;           /* [n] explicit source, m^-3 s^-1 */
    const double *kloss;         /* [n] implicit loss rate, 1/s (NULL = 0) */
    const double *q;             /* [n] net ion charge density / e, m^-3 */
    const double *uface;         /* [n+1] advective velocity at faces (NULL = 0) */
    const double *ne_old;        /* [n] n^n */
    const double *phi_old;       /* [n] phi^n */
    const orc_table *table;      /* NULL: per-cell mu, diff; else face mu, D from the table */
    const double *prog;          /* [n] progress variable (table only) */
    const double *gas_n;         /* [n] background gas number density, m^-3 (table only) */
} orc_column;

typedef struct {
    int max_iters;
    double tol;                  /* stop at ||S_F^-1 F||_inf <= tol (timed mode) */
    int reference_mode;          /* 1: iterate to the rounding floor and return
                                    the iterate with the smallest Newton correction */
    double floor_tol;            /* reference mode: stop once the scaled Newton
                                    correction ||S_X^-1 d||_inf is this small */
    double ls_theta;             /* restricted natural monotonicity factor */
    double lambda_min;
} orc_newton_opts;

typedef struct {
    int iters, backtracks, status;
    double res_scaled;
    double scal[4];
} orc_newton_stats;

double orc_bernoulli(double x);
void orc_table_lookup(const orc_table *t, double c, double en_td, double *mu, double *diff);
void orc_face_coeffs(const orc_column *c, const double *phi, double *mu, double *diff);
double orc_bernoulli_deriv(double x);
void orc_source_term(const orc_column *c, double *f);
void orc_face_fluxes(const orc_column *c, const double *ne, const double *phi, double *gamma);
void orc_residual(const orc_column *c, const double *f, const double *ne, const double *phi,
                  double *fe, double *fp);
void orc_scalings(const orc_column *c, double s[4]);
void orc_jacobian_dense(const orc_column *c, const double *ne, const double *phi, double *a);
void orc_jacobian_band(const orc_column *c, const double *ne, const double *phi, double *ab);
int orc_band_factor(int n, double *ab, int *piv);
void orc_band_factored_solve(int n, const double *ab, const int *piv, double *b);
int orc_band_solve(int n, double *ab, double *b);
int orc_dense_solve(int n, double *a, double *b);
int orc_newton(const orc_column *c, const orc_newton_opts *o, double *ne, double *phi,
               orc_newton_stats *st);

#endif
