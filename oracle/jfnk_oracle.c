/*
 * CPU oracle for the implicit electron / electric-potential step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU path.
 *
 * Plain, single-threaded, FP64.  It computes the root of the backward-Euler
 * system of the paper (Section 3.2, eq:pnp discretised in time as eq:nls) by
 * Newton's method with the analytic Jacobian and a banded direct solve (LU
 * with partial pivoting).  The paper reaches the same root with JFNK
 * (Algorithm 2); a direct Newton is the plain definition of that root.
 *
 * Discrete residual (where the paper is silent or garbled, the reading taken
 * is stated at the point it applies):
 *   cells i = 0..N-1 of width h = L/N; faces j = 0..N, face j left of cell j.
 *   interior face j (cells a=j-1, b=j): mu_f, D_f arithmetic means,
 *     Pe = (u_f h + mu_f (phi_b - phi_a)) / D_f,
 *     Gamma_j = (D_f/h) [ B(-Pe) n_a - B(Pe) n_b ],  B(x) = x/(e^x - 1)
 *     (Scharfetter-Gummel flux of Gamma = n (u + mu grad phi) - D grad n;
 *      electrons drift up the potential gradient).
 *   wall faces: distance h/2, the adjacent cell's mu and D, and the wall
 *     density in place of the missing cell (Dirichlet), or Gamma = 0.
 *   E_i = -n_i + f_i - dt k_i n_i - (dt/h)(Gamma_{i+1} - Gamma_i),
 *         f_i = n^n_i + dt s_i                         (eq:nls, first row)
 *   P_i = -n_i + q_i + (eps/e)(G_{i+1} - G_i)/h,
 *         G_j = potential difference across face j / face distance
 *                                                       (eq:nls, second row)
 * With a transport table (Section 2.2: electron mobility and diffusivity as
 * functions of the progress variable c and the reduced field |E|/N), mu_f and
 * D_f of face j come from the table at the face's mean c and mean N (the
 * adjacent cell's at a wall) and |E| = |G_j|, the field the face carries in
 * the state at hand; the residual then depends on phi through them too, and
 * Newton uses a finite-difference band Jacobian (central differences, six
 * colours of the three-cell stencil).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "jfnk_oracle.h"

/* ---------------------------------------------------------------------- */
/* Bernoulli function B(x) = x / (exp(x) - 1), B(0) = 1.                  */
/* ---------------------------------------------------------------------- */
double orc_bernoulli(double x)
{
    if (fabs(x) < 1e-3) {
        double x2 = x * x;
        return 1.0 - 0.5 * x + x2 / 12.0 - x2 * x2 / 720.0;
    }
    return x / expm1(x);
}

/* dB/dx = (B(x)/x) (1 - B(x) - x); series -1/2 + x/6 - x^3/180 near 0. */
double orc_bernoulli_deriv(double x)
{
    if (fabs(x) < 1e-3) {
        return -0.5 + x / 6.0 - x * x * x / 180.0;
    }
    double b = orc_bernoulli(x);
    return (b / x) * (1.0 - b - x);
}

/* ---------------------------------------------------------------------- */
/* Transport table (Section 2.2)                                          */
/* ---------------------------------------------------------------------- */

/* Bilinear interpolation of one table at (c, x), both clamped to the grid. */
static double table_interp(const orc_table *t, const double *v, double cv, double x)
{
    if (cv < t->c_min) cv = t->c_min;
    if (cv > t->c_max) cv = t->c_max;
    if (x < t->x_min) x = t->x_min;
    if (x > t->x_max) x = t->x_max;
    double fc = (cv - t->c_min) / (t->c_max - t->c_min) * (t->nc - 1);
    double fx = (x - t->x_min) / (t->x_max - t->x_min) * (t->nx - 1);
    int i = (int)floor(fc), k = (int)floor(fx);
    if (i > t->nc - 2) i = t->nc - 2;
    if (k > t->nx - 2) k = t->nx - 2;
    double wc = fc - i, wx = fx - k;
    const double *r0 = v + (size_t)i * t->nx, *r1 = r0 + t->nx;
    return (1.0 - wc) * ((1.0 - wx) * r0[k] + wx * r0[k + 1]) + wc * ((1.0 - wx) * r1[k] + wx * r1[k + 1]);
}

/* mu and D at progress variable c and reduced field en_td (in Townsend,
   1 Td = 1e-21 V m^2); a zero field takes the table's lowest column. */
void orc_table_lookup(const orc_table *t, double c, double en_td, double *mu, double *diff)
{
    double x = en_td > 0.0 ? log10(en_td) : t->x_min;
    *mu = table_interp(t, t->mu, c, x);
    *diff = table_interp(t, t->diff, c, x);
}

/* ---------------------------------------------------------------------- */
/* Face quantities                                                        */
/* ---------------------------------------------------------------------- */

/* Potential gradient across face j. */
static double face_grad(const orc_column *c, const double *phi, int j)
{
    const int N = c->n;
    const double h = c->length / N;
    if (j == 0) return (phi[0] - c->phi_left) / (0.5 * h);
    if (j == N) return (c->phi_right - phi[N - 1]) / (0.5 * h);
    return (phi[j] - phi[j - 1]) / h;
}

/* Mobility and diffusivity of face j in state phi: the arithmetic means of
   the two cells' values (a wall face: the adjacent cell's), or the table at
   the face's progress variable and reduced field |E| / N. */
static void face_mu_d(const orc_column *c, const double *phi, int j, double *mu, double *d)
{
    const int N = c->n;
    int a = j == 0 ? 0 : j - 1, b = j == N ? N - 1 : j;
    if (!c->table) {
        *mu = 0.5 * (c->mu[a] + c->mu[b]);
        *d = 0.5 * (c->diff[a] + c->diff[b]);
        return;
    }
    double cf = 0.5 * (c->prog[a] + c->prog[b]);
    double nf = 0.5 * (c->gas_n[a] + c->gas_n[b]);
    double e = fabs(face_grad(c, phi, j));
    orc_table_lookup(c->table, cf, e / nf / 1e-21, mu, d);
}

void orc_face_coeffs(const orc_column *c, const double *phi, double *mu, double *diff)
{
    for (int j = 0; j <= c->n; ++j) face_mu_d(c, phi, j, mu + j, diff + j);
}

/* Electron flux through face j at state (ne, phi). */
static double face_flux(const orc_column *c, const double *ne, const double *phi, int j)
{
    const int N = c->n;
    const double h = c->length / N;
    double u = c->uface ? c->uface[j] : 0.0;
    double muf, df;
    if ((j == 0 && c->bc_left == ORC_BC_ZERO_FLUX) || (j == N && c->bc_right == ORC_BC_ZERO_FLUX)) return 0.0;
    face_mu_d(c, phi, j, &muf, &df);
    if (j == 0) {
        double hb = 0.5 * h;
        double pe = (u * hb + muf * (phi[0] - c->phi_left)) / df;
        return (df / hb) * (orc_bernoulli(-pe) * c->ne_left - orc_bernoulli(pe) * ne[0]);
    }
    if (j == N) {
        double hb = 0.5 * h;
        double pe = (u * hb + muf * (c->phi_right - phi[N - 1])) / df;
        return (df / hb) * (orc_bernoulli(-pe) * ne[N - 1] - orc_bernoulli(pe) * c->ne_right);
    }
    double pe = (u * h + muf * (phi[j] - phi[j - 1])) / df;
    return (df / h) * (orc_bernoulli(-pe) * ne[j - 1] - orc_bernoulli(pe) * ne[j]);
}

void orc_face_fluxes(const orc_column *c, const double *ne, const double *phi, double *gamma)
{
    for (int j = 0; j <= c->n; ++j) gamma[j] = face_flux(c, ne, phi, j);
}

void orc_source_term(const orc_column *c, double *f)
{
    for (int i = 0; i < c->n; ++i) f[i] = c->ne_old[i] + c->dt * c->src[i];
}

/* ---------------------------------------------------------------------- */
/* Residual F(X) of eq:nls.                                               */
/* ---------------------------------------------------------------------- */
void orc_residual(const orc_column *c, const double *f, const double *ne,
                  const double *phi, double *fe, double *fp)
{
    const int N = c->n;
    const double h = c->length / N;
    const double dt = c->dt;
    double *gam = (double *)malloc(sizeof(double) * (N + 1));
    double *grd = (double *)malloc(sizeof(double) * (N + 1));
    for (int j = 0; j <= N; ++j) {
        gam[j] = face_flux(c, ne, phi, j);
        grd[j] = face_grad(c, phi, j);
    }
    for (int i = 0; i < N; ++i) {
        double k = c->kloss ? c->kloss[i] : 0.0;
        fe[i] = -ne[i] + f[i] - dt * k * ne[i] - (dt / h) * (gam[i + 1] - gam[i]);
        fp[i] = -ne[i] + c->q[i] + c->eps_over_e * (grd[i + 1] - grd[i]) / h;
    }
    free(gam);
    free(grd);
}

/* ---------------------------------------------------------------------- */
/* Diagonal scalings S_F, S_X (Section 3.2, eq:newton_sc): typical sizes  */
/* of F and X taken once, from the state X^n at the start of the step.    */
/* s[0] = s_Fn, s[1] = s_Fphi, s[2] = s_Xn, s[3] = s_Xphi.                */
/* s_Fn is the largest sum of magnitudes of the terms of an electron row, */
/* s_Fphi the same for a potential row; s_Xn, s_Xphi are the largest      */
/* magnitudes of n (or q) and phi (or the electrode potentials).          */
/* ---------------------------------------------------------------------- */
void orc_scalings(const orc_column *c, double s[4])
{
    const int N = c->n;
    const double h = c->length / N;
    const double dt = c->dt;
    const double *ne = c->ne_old, *phi = c->phi_old;
    /* magnitude of the two SG terms of each face */
    double *mag = (double *)malloc(sizeof(double) * (N + 1));
    for (int j = 0; j <= N; ++j) {
        double u = c->uface ? c->uface[j] : 0.0;
        double dfac, pe, na, nb, muf, df;
        if ((j == 0 && c->bc_left == ORC_BC_ZERO_FLUX) || (j == N && c->bc_right == ORC_BC_ZERO_FLUX)) {
            mag[j] = 0.0;
            continue;
        }
        face_mu_d(c, phi, j, &muf, &df);
        if (j == 0) {
            double hb = 0.5 * h;
            pe = (u * hb + muf * (phi[0] - c->phi_left)) / df;
            dfac = df / hb;
            na = c->ne_left; nb = ne[0];
        } else if (j == N) {
            double hb = 0.5 * h;
            pe = (u * hb + muf * (c->phi_right - phi[N - 1])) / df;
            dfac = df / hb;
            na = ne[N - 1]; nb = c->ne_right;
        } else {
            pe = (u * h + muf * (phi[j] - phi[j - 1])) / df;
            dfac = df / h;
            na = ne[j - 1]; nb = ne[j];
        }
        mag[j] = dfac * (orc_bernoulli(-pe) * fabs(na) + orc_bernoulli(pe) * fabs(nb));
    }
    double sfn = 0.0, sfp = 0.0, sxn = 1.0, sxp = 1.0;
    for (int i = 0; i < N; ++i) {
        double k = c->kloss ? c->kloss[i] : 0.0;
        double f = ne[i] + dt * c->src[i];
        double te = fabs(f) + dt * k * fabs(ne[i]) + (dt / h) * (mag[i] + mag[i + 1]);
        double tp = fabs(ne[i]) + fabs(c->q[i]) +
                    c->eps_over_e * (fabs(face_grad(c, phi, i)) + fabs(face_grad(c, phi, i + 1))) / h;
        if (te > sfn) sfn = te;
        if (tp > sfp) sfp = tp;
        if (fabs(ne[i]) > sxn) sxn = fabs(ne[i]);
        if (fabs(c->q[i]) > sxn) sxn = fabs(c->q[i]);
        if (fabs(phi[i]) > sxp) sxp = fabs(phi[i]);
    }
    if (fabs(c->phi_left) > sxp) sxp = fabs(c->phi_left);
    if (fabs(c->phi_right) > sxp) sxp = fabs(c->phi_right);
    free(mag);
    s[0] = sfn; s[1] = sfp; s[2] = sxn; s[3] = sxp;
}

/* ---------------------------------------------------------------------- */
/* Analytic Jacobian dF/dX (Section 3.2, linearisation eq:linear_nls),    */
/* unknowns ordered (n_0, phi_0, n_1, phi_1, ...), rows (E_0, P_0, ...).  */
/* Written into a caller-provided dense row-major matrix of size 2N x 2N  */
/* through a setter, so that the band and dense forms come from one code. */
/* ---------------------------------------------------------------------- */
typedef void (*setter_fn)(void *ctx, int row, int col, double v);

/* derivatives of the flux of face j w.r.t. the (n, phi) of its left cell (a)
   and right cell (b); absent cells (walls) report 0. */
static void face_flux_derivs(const orc_column *c, const double *ne, const double *phi, int j,
                             double *dna, double *dpa, double *dnb, double *dpb)
{
    const int N = c->n;
    const double h = c->length / N;
    double u = c->uface ? c->uface[j] : 0.0;
    *dna = *dpa = *dnb = *dpb = 0.0;
    if (j == 0) {
        if (c->bc_left == ORC_BC_ZERO_FLUX) return;
        double hb = 0.5 * h;
        double pe = (u * hb + c->mu[0] * (phi[0] - c->phi_left)) / c->diff[0];
        double dfac = c->diff[0] / hb;
        double dgdpe = dfac * (-orc_bernoulli_deriv(-pe) * c->ne_left - orc_bernoulli_deriv(pe) * ne[0]);
        *dnb = -dfac * orc_bernoulli(pe);
        *dpb = dgdpe * c->mu[0] / c->diff[0];
        return;
    }
    if (j == N) {
        if (c->bc_right == ORC_BC_ZERO_FLUX) return;
        double hb = 0.5 * h;
        double pe = (u * hb + c->mu[N - 1] * (c->phi_right - phi[N - 1])) / c->diff[N - 1];
        double dfac = c->diff[N - 1] / hb;
        double dgdpe = dfac * (-orc_bernoulli_deriv(-pe) * ne[N - 1] - orc_bernoulli_deriv(pe) * c->ne_right);
        *dna = dfac * orc_bernoulli(-pe);
        *dpa = -dgdpe * c->mu[N - 1] / c->diff[N - 1];
        return;
    }
    double muf = 0.5 * (c->mu[j - 1] + c->mu[j]);
    double df = 0.5 * (c->diff[j - 1] + c->diff[j]);
    double pe = (u * h + muf * (phi[j] - phi[j - 1])) / df;
    double dfac = df / h;
    double dgdpe = dfac * (-orc_bernoulli_deriv(-pe) * ne[j - 1] - orc_bernoulli_deriv(pe) * ne[j]);
    *dna = dfac * orc_bernoulli(-pe);
    *dnb = -dfac * orc_bernoulli(pe);
    *dpb = dgdpe * muf / df;
    *dpa = -*dpb;
}

static void jacobian_generic(const orc_column *c, const double *ne, const double *phi,
                             setter_fn set, void *ctx)
{
    const int N = c->n;
    const double h = c->length / N;
    const double dt = c->dt;
    const double eps = c->eps_over_e;
    for (int i = 0; i < N; ++i) {
        int rn = 2 * i, rp = 2 * i + 1;
        double k = c->kloss ? c->kloss[i] : 0.0;
        /* right face i+1: cell i is its left cell (a); left face i: cell i is b */
        double Rna, Rpa, Rnb, Rpb, Lna, Lpa, Lnb, Lpb;
        face_flux_derivs(c, ne, phi, i + 1, &Rna, &Rpa, &Rnb, &Rpb);
        face_flux_derivs(c, ne, phi, i, &Lna, &Lpa, &Lnb, &Lpb);
        double g = dt / h;
        /* electron row: -n - dt k n - g (Gamma_{i+1} - Gamma_i) */
        set(ctx, rn, 2 * i, -1.0 - dt * k - g * (Rna - Lnb));
        set(ctx, rn, 2 * i + 1, -g * (Rpa - Lpb));
        if (i > 0) {
            set(ctx, rn, 2 * (i - 1), g * Lna);
            set(ctx, rn, 2 * (i - 1) + 1, g * Lpa);
        }
        if (i < N - 1) {
            set(ctx, rn, 2 * (i + 1), -g * Rnb);
            set(ctx, rn, 2 * (i + 1) + 1, -g * Rpb);
        }
        /* potential row: -n + eps (G_{i+1} - G_i)/h */
        double hl = (i == 0) ? 0.5 * h : h;
        double hr = (i == N - 1) ? 0.5 * h : h;
        set(ctx, rp, 2 * i, -1.0);
        set(ctx, rp, 2 * i + 1, -eps * (1.0 / hr + 1.0 / hl) / h);
        if (i > 0) set(ctx, rp, 2 * (i - 1) + 1, eps / (hl * h));
        if (i < N - 1) set(ctx, rp, 2 * (i + 1) + 1, eps / (hr * h));
    }
}

/* Table mode: the Jacobian by central differences of the residual.  The
   residual of cell i depends on cells i-1, i, i+1 only, so perturbing every
   third cell in one component at once (six colours) gives every column of
   the band without overlap.  Step: 1e-6 of the component's magnitude at the
   cell (its scale s_X at least). */
static void jacobian_fd(const orc_column *c, const double *ne, const double *phi, setter_fn set, void *ctx)
{
    const int N = c->n;
    double s[4];
    orc_scalings(c, s);
    double *f = (double *)malloc(sizeof(double) * N);
    double *xn = (double *)malloc(sizeof(double) * N);
    double *xp = (double *)malloc(sizeof(double) * N);
    double *ep = (double *)malloc(sizeof(double) * 2 * N);
    double *em = (double *)malloc(sizeof(double) * 2 * N);
    double *del = (double *)malloc(sizeof(double) * N);
    orc_source_term(c, f);
    for (int comp = 0; comp < 2; ++comp) {
        for (int col = 0; col < 3; ++col) {
            for (int sgn = 0; sgn < 2; ++sgn) {
                memcpy(xn, ne, sizeof(double) * N);
                memcpy(xp, phi, sizeof(double) * N);
                for (int p = col; p < N; p += 3) {
                    double *x = comp == 0 ? xn : xp;
                    double scale = comp == 0 ? s[2] : s[3];
                    del[p] = 1e-6 * (fabs(x[p]) > scale ? fabs(x[p]) : scale);
                    x[p] += sgn == 0 ? del[p] : -del[p];
                }
                orc_residual(c, f, xn, xp, sgn == 0 ? ep : ep + N, sgn == 0 ? em : em + N);
            }
            /* ep[0..N): F_e(+), ep[N..2N): F_e(-); em likewise for F_phi */
            for (int p = col; p < N; p += 3) {
                for (int i = p - 1; i <= p + 1; ++i) {
                    if (i < 0 || i >= N) continue;
                    set(ctx, 2 * i, 2 * p + comp, (ep[i] - ep[N + i]) / (2.0 * del[p]));
                    set(ctx, 2 * i + 1, 2 * p + comp, (em[i] - em[N + i]) / (2.0 * del[p]));
                }
            }
        }
    }
    free(f); free(xn); free(xp); free(ep); free(em); free(del);
}

typedef struct { double *a; int n; } dense_ctx;
static void set_dense(void *p, int r, int col, double v)
{
    dense_ctx *d = (dense_ctx *)p;
    d->a[(size_t)r * d->n + col] = v;
}

void orc_jacobian_dense(const orc_column *c, const double *ne, const double *phi, double *a)
{
    int n2 = 2 * c->n;
    memset(a, 0, sizeof(double) * (size_t)n2 * n2);
    dense_ctx d = { a, n2 };
    if (c->table) jacobian_fd(c, ne, phi, set_dense, &d);
    else jacobian_generic(c, ne, phi, set_dense, &d);
}

/* Band storage by rows: A(i, j) at ab[i * ORC_BAND_W + (j - i + ORC_KL)],
   valid for j - i in [-KL, KL + KU] (the extra KL columns hold pivoting
   fill-in). */
typedef struct { double *ab; } band_ctx;
static void set_band(void *p, int r, int col, double v)
{
    band_ctx *b = (band_ctx *)p;
    b->ab[(size_t)r * ORC_BAND_W + (col - r + ORC_KL)] = v;
}

void orc_jacobian_band(const orc_column *c, const double *ne, const double *phi, double *ab)
{
    memset(ab, 0, sizeof(double) * (size_t)2 * c->n * ORC_BAND_W);
    band_ctx b = { ab };
    if (c->table) jacobian_fd(c, ne, phi, set_band, &b);
    else jacobian_generic(c, ne, phi, set_band, &b);
}

/* ---------------------------------------------------------------------- */
/* Direct solvers (textbook Gaussian elimination with partial pivoting).  */
/* ---------------------------------------------------------------------- */

/* Band LU with partial pivoting (row exchanges recorded in piv[n]).  ab is
   overwritten by the factors.  Returns 0, or k+1 if the k-th pivot is
   exactly zero. */
int orc_band_factor(int n, double *ab, int *piv)
{
    const int kl = ORC_KL, ku = ORC_KU, w = ORC_BAND_W;
#define AB(i, j) ab[(size_t)(i) * w + ((j) - (i) + kl)]
    int info = 0;
    for (int k = 0; k < n; ++k) {
        int last = k + kl < n - 1 ? k + kl : n - 1;
        int p = k;
        double best = fabs(AB(k, k));
        for (int i = k + 1; i <= last; ++i)
            if (fabs(AB(i, k)) > best) { best = fabs(AB(i, k)); p = i; }
        piv[k] = p;
        int jend = k + kl + ku < n - 1 ? k + kl + ku : n - 1;
        if (p != k) {
            for (int j = k; j <= jend; ++j) {
                double t = AB(k, j); AB(k, j) = AB(p, j); AB(p, j) = t;
            }
        }
        if (AB(k, k) == 0.0) { if (!info) info = k + 1; continue; }
        for (int i = k + 1; i <= last; ++i) {
            double l = AB(i, k) / AB(k, k);
            AB(i, k) = l;
            if (l != 0.0)
                for (int j = k + 1; j <= jend; ++j) AB(i, j) -= l * AB(k, j);
        }
    }
#undef AB
    return info;
}

/* Solve with the factors of orc_band_factor; b is overwritten. */
void orc_band_factored_solve(int n, const double *ab, const int *piv, double *b)
{
    const int kl = ORC_KL, ku = ORC_KU, w = ORC_BAND_W;
#define AB(i, j) ab[(size_t)(i) * w + ((j) - (i) + kl)]
    /* L y = P b */
    for (int k = 0; k < n; ++k) {
        int p = piv[k];
        if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
        int last = k + kl < n - 1 ? k + kl : n - 1;
        for (int i = k + 1; i <= last; ++i) b[i] -= AB(i, k) * b[k];
    }
    /* U x = y */
    for (int k = n - 1; k >= 0; --k) {
        int jend = k + kl + ku < n - 1 ? k + kl + ku : n - 1;
        double s = b[k];
        for (int j = k + 1; j <= jend; ++j) s -= AB(k, j) * b[j];
        b[k] = s / AB(k, k);
    }
#undef AB
}

/* Factor and solve one right-hand side (ab and b overwritten). */
int orc_band_solve(int n, double *ab, double *b)
{
    int *piv = (int *)malloc(sizeof(int) * n);
    int info = orc_band_factor(n, ab, piv);
    if (!info) orc_band_factored_solve(n, ab, piv, b);
    free(piv);
    return info;
}

/* Dense LU with partial pivoting; a (row-major n x n) and b overwritten. */
int orc_dense_solve(int n, double *a, double *b)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(a[(size_t)i * n + k]) > best) { best = fabs(a[(size_t)i * n + k]); p = i; }
        if (best == 0.0) return k + 1;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[(size_t)k * n + j]; a[(size_t)k * n + j] = a[(size_t)p * n + j]; a[(size_t)p * n + j] = t;
            }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double l = a[(size_t)i * n + k] / a[(size_t)k * n + k];
            for (int j = k; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int j = k + 1; j < n; ++j) s -= a[(size_t)k * n + j] * b[j];
        b[k] = s / a[(size_t)k * n + k];
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Newton's method with backtracking (Section 3.2: Newton step            */
/* eq:newton_ite, scaling eq:newton_sc, stopping tests on the scaled      */
/* residual, backtracking line search for globalisation).                 */
/* ---------------------------------------------------------------------- */
static void scaled_norms(int N, const double *fe, const double *fp, const double s[4],
                         double *ninf, double *n2)
{
    double mi = 0.0, s2 = 0.0;
    for (int i = 0; i < N; ++i) {
        double a = fe[i] / s[0], b = fp[i] / s[1];
        if (fabs(a) > mi) mi = fabs(a);
        if (fabs(b) > mi) mi = fabs(b);
        s2 += a * a + b * b;
    }
    if (ninf) *ninf = (isnan(mi) || isnan(s2)) ? NAN : mi;
    if (n2) *n2 = sqrt(s2);
}

/* ||S_X^-1 d||_inf of an interleaved (n, phi) vector */
static double scaled_step_inf(int N, const double *d, const double s[4])
{
    double m = 0.0;
    for (int i = 0; i < N; ++i) {
        double a = fabs(d[2 * i] / s[2]), b = fabs(d[2 * i + 1] / s[3]);
        if (a > m) m = a;
        if (b > m) m = b;
    }
    return m;
}

int orc_newton(const orc_column *c, const orc_newton_opts *o, double *ne, double *phi,
               orc_newton_stats *st)
{
    const int N = c->n, n2 = 2 * N;
    double s[4];
    orc_scalings(c, s);
    double *f = (double *)malloc(sizeof(double) * N);
    double *fe = (double *)malloc(sizeof(double) * N);
    double *fp = (double *)malloc(sizeof(double) * N);
    double *te = (double *)malloc(sizeof(double) * N);
    double *tp = (double *)malloc(sizeof(double) * N);
    double *xn = (double *)malloc(sizeof(double) * N);
    double *xp = (double *)malloc(sizeof(double) * N);
    double *rhs = (double *)malloc(sizeof(double) * n2);
    double *cor = (double *)malloc(sizeof(double) * n2);
    double *ab = (double *)malloc(sizeof(double) * (size_t)n2 * ORC_BAND_W);
    int *piv = (int *)malloc(sizeof(int) * n2);
    double *best_n = (double *)malloc(sizeof(double) * N);
    double *best_p = (double *)malloc(sizeof(double) * N);
    orc_source_term(c, f);

    int status = ORC_MAX_ITERS, it = 0, backtracks = 0, stagn = 0;
    double rinf, r2, best = INFINITY, best_r = INFINITY, prev_d = INFINITY;
    orc_residual(c, f, ne, phi, fe, fp);
    scaled_norms(N, fe, fp, s, &rinf, &r2);
    for (;;) {
        if (isnan(rinf)) { status = ORC_NONFINITE; break; }
        if (!o->reference_mode) {
            if (rinf < best) {
                best = rinf;
                best_r = rinf;
                memcpy(best_n, ne, sizeof(double) * N);
                memcpy(best_p, phi, sizeof(double) * N);
            }
            if (rinf <= o->tol) { status = ORC_CONVERGED; break; }
        }
        if (it >= o->max_iters && !o->reference_mode) break;
        /* Newton direction: J d = -F */
        orc_jacobian_band(c, ne, phi, ab);
        if (orc_band_factor(n2, ab, piv) != 0) { status = ORC_SINGULAR; break; }
        for (int i = 0; i < N; ++i) { rhs[2 * i] = -fe[i]; rhs[2 * i + 1] = -fp[i]; }
        orc_band_factored_solve(n2, ab, piv, rhs);
        const double dinf = scaled_step_inf(N, rhs, s);
        if (o->reference_mode) {
            /* Reference root: Newton runs on until its correction ||S_X^-1 d||_inf
               (the distance of the iterate to the root it converges to) reaches
               floor_tol or stops halving; the iterate with the smallest
               correction is returned.  In the stiff cases the residual reaches
               its FP64 rounding floor while the iterate is still measurably away
               from the root, so the residual cannot rank iterates there. */
            if (dinf < best) {
                best = dinf;
                best_r = rinf;
                memcpy(best_n, ne, sizeof(double) * N);
                memcpy(best_p, phi, sizeof(double) * N);
            }
            if (dinf <= o->floor_tol) { status = ORC_CONVERGED; break; }
            if (it > 0 && dinf > 0.5 * prev_d) {
                if (++stagn >= 2 && best_r <= o->tol) { status = ORC_CONVERGED; break; }
            } else {
                stagn = 0;
            }
            if (it >= o->max_iters) break;
            prev_d = dinf;
        }
        /* Backtracking (Section 3.2: line search for globalisation).  A trial
           step X + lam d is taken when the simplified Newton correction there,
           J(X)^-1 F(X + lam d), has shrunk against the step d in the scaled
           max norm: ||S_X^-1 J^-1 F(X + lam d)||_inf <= (1 - theta lam) ||S_X^-1 d||_inf
           with theta = ls_theta (the natural monotonicity test, invariant to
           the scaling of F).  If no halving passes, the full step is taken. */
        double lam = 1.0, rt2 = 0.0, rtinf = 0.0;
        int accepted = 0, finite_seen = 0;
        for (;;) {
            for (int i = 0; i < N; ++i) {
                xn[i] = ne[i] + lam * rhs[2 * i];
                xp[i] = phi[i] + lam * rhs[2 * i + 1];
            }
            orc_residual(c, f, xn, xp, te, tp);
            scaled_norms(N, te, tp, s, &rtinf, &rt2);
            if (!isnan(rt2)) {
                finite_seen = 1;
                for (int i = 0; i < N; ++i) { cor[2 * i] = -te[i]; cor[2 * i + 1] = -tp[i]; }
                orc_band_factored_solve(n2, ab, piv, cor);
                if (scaled_step_inf(N, cor, s) <= (1.0 - o->ls_theta * lam) * dinf) { accepted = 1; break; }
            }
            if (lam * 0.5 < o->lambda_min) break;
            lam *= 0.5;
            ++backtracks;
        }
        if (!accepted) {
            /* full step unless it is not finite (then the last finite trial) */
            for (int i = 0; i < N; ++i) { cor[2 * i] = ne[i] + rhs[2 * i]; cor[2 * i + 1] = phi[i] + rhs[2 * i + 1]; }
            for (int i = 0; i < N; ++i) { xn[i] = cor[2 * i]; xp[i] = cor[2 * i + 1]; }
            orc_residual(c, f, xn, xp, te, tp);
            scaled_norms(N, te, tp, s, &rtinf, &rt2);
            if (isnan(rt2) && finite_seen) {
                for (int i = 0; i < N; ++i) {
                    xn[i] = ne[i] + lam * rhs[2 * i];
                    xp[i] = phi[i] + lam * rhs[2 * i + 1];
                }
                orc_residual(c, f, xn, xp, te, tp);
                scaled_norms(N, te, tp, s, &rtinf, &rt2);
            }
        }
        memcpy(ne, xn, sizeof(double) * N);
        memcpy(phi, xp, sizeof(double) * N);
        memcpy(fe, te, sizeof(double) * N);
        memcpy(fp, tp, sizeof(double) * N);
        rinf = rtinf;
        r2 = rt2;
        ++it;
    }
    /* hand back the best iterate met on the way: smallest residual (timed
       mode) or smallest Newton correction (reference mode) */
    if (best_r < INFINITY && (o->reference_mode || best_r < rinf || isnan(rinf))) {
        memcpy(ne, best_n, sizeof(double) * N);
        memcpy(phi, best_p, sizeof(double) * N);
        rinf = best_r;
    }
    if (st) {
        st->iters = it;
        st->backtracks = backtracks;
        st->res_scaled = rinf;
        st->status = status;
        for (int k = 0; k < 4; ++k) st->scal[k] = s[k];
    }
    free(f); free(fe); free(fp); free(te); free(tp); free(xn); free(xp);
    free(rhs); free(cor); free(ab); free(piv); free(best_n); free(best_p);
    return status;
}
