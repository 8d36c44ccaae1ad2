// Newton-Krylov control logic of one column (paper Algorithm 2), written
// once over an executor.  Two executors run it:
//   * DevExec: the whole loop inside one workgroup (batched schedule: one
//     launch solves every column, each workgroup owning one column);
//   * the host-driven executor in jfnk_lib.hip (plain schedule: every phase
//     is a kernel launch and every decision reads scalars back to the host).
// Both call the same column phases, so both produce the same iterates.
#pragma once
#include <float.h>
#include <math.h>

#include "jfnk_column.h"

namespace jfnk {

struct ColOutcome {
    int status, newton, gmres, backtracks, guess, restarts, chords;
    int work[kWorkCounts];
    double rinf, r2;
    int cur;
};

// Givens-rotation update of column j of the Hessenberg matrix (paper:
// minimisation of the residual over the Krylov space).  h[0..j] and hn =
// h_{j+1,j}; H is (m+1) x m column major with leading dimension ld.
// Returns |g_{j+1}|, the norm of the GMRES residual after this column.
__host__ __device__ inline double givens_column(double* H, int ld, double* cs, double* sn,
                                                double* g, int j, const double* h, double hn,
                                                bool commit) {
    double col[kMaxRestart + 1];
    for (int i = 0; i <= j; ++i) col[i] = h[i];
    for (int i = 0; i < j; ++i) {
        const double a = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = a;
    }
    const double r = hypot(col[j], hn);
    double c = 1.0, s = 0.0;
    if (r > 0.0) { c = col[j] / r; s = hn / r; }
    col[j] = r;
    const double gj = g[j];
    const double gnext = -s * gj;
    if (commit) {
        for (int i = 0; i <= j; ++i) H[j * ld + i] = col[i];
        cs[j] = c; sn[j] = s;
        g[j] = c * gj;
        g[j + 1] = gnext;
    }
    return fabs(gnext);
}

// y = R^-1 g for the leading k x k upper triangle of H.
__host__ __device__ inline void givens_solve(const double* H, int ld, const double* g, int k,
                                             double* y) {
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int l = i + 1; l < k; ++l) s -= H[l * ld + i] * y[l];
        y[i] = s / H[i * ld + i];
    }
}

// Contraction ratio e_{k+1} / e_k of a simplified-Newton step above which
// the factors are rebuilt at the new iterate (the choice of stiff-integrator
// practice for modified Newton iterations, which re-evaluate the Jacobian once
// the observed rate exceeds a few tenths).
constexpr double kChordRefactorRate = 0.2;

template <class Ex>
__host__ __device__ void jfnk_solve(Ex& ex, const SolverParams& p, ColOutcome& out) {
    const double lam_fd = 6.0554544523933395e-06;   // cbrt(2^-52)
    int cur = 0, guess = 0;
    Norms nr = ex.setup(&cur, &guess);
    int it = 0, gtot = 0, btot = 0, rtot = 0;
    int status = COL_MAX_NEWTON;
    const bool bad_input = ex.bad_input();
    double hcol[kMaxRestart + 2];
    double y[kMaxRestart];
    // buffer whose state the current factorisation was built at; 3: the
    // previous step's factors (a lagged preconditioner: used for the error
    // estimate and simplified-Newton steps, replaced before any GMRES solve)
    int factored = ex.lagged_factors() ? 3 : -1;
    double est = -1.0;   // ||S_X^-1 P^-1 S_F^-1 F(X)||_inf of the current iterate (-1: unknown)
    int corr_at = -1;    // buffer whose correction -P^-1 S_F^-1 F sits in the last Krylov slot
    int chords = 0, chord_run = 0;
    int wk[kWorkCounts] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (;;) {
        if (bad_input) { status = COL_BAD_INPUT; break; }
        if (isnan(nr.r2)) { status = COL_NONFINITE; break; }
        if (nr.rinf <= p.tol_f) {
            if (p.tol_x <= 0.0) { status = COL_CONVERGED; break; }
            // stopping test on the Newton correction: the error estimate
            // ||S_X^-1 (X - X*)||_inf ~ ||P^-1 S_F^-1 F(X)||_inf with the latest factorisation
            if (est < 0.0) {
                if (factored < 0) { ex.factor(cur); factored = cur; ++wk[kWorkFactor]; }
                est = ex.correction(cur).y;
                ++wk[kWorkApply];
                corr_at = cur;
            }
            if (est <= p.tol_x) { status = COL_CONVERGED; break; }
        }
        if (it >= p.max_newton) break;
        // Near the root the correction already at hand is a Newton step with
        // the analytic Jacobian of the latest factorisation: take it as a
        // simplified-Newton step (no Krylov solve) while it passes the same
        // natural monotonicity test as the line search at lambda = 1.  The
        // convergence test above is unchanged.
        if (p.chord_tol > 0.0 && corr_at == cur && est > 0.0 && est <= p.chord_tol && chord_run < 4) {
            const int out = (cur + 1) % 3;
            const Norms tc = ex.chord_trial(cur, out);
            ++wk[kWorkResidual];
            double e2 = INFINITY;
            if (!isnan(tc.r2)) { e2 = ex.correction(out).y; ++wk[kWorkApply]; }
            if (e2 <= (1.0 - p.theta) * est) {
                const double rate = e2 / est;
                cur = out;
                nr = tc;
                est = e2;
                corr_at = out;
                ++chords;
                ++chord_run;
                // A slow contraction means the factors (built at an earlier
                // iterate, or in the previous time step) no longer describe the
                // Jacobian: refactor at the new iterate, so that the next
                // simplified-Newton step is a Newton step again.  Also when one
                // more step at the observed rate would not reach tol_x: the
                // refactorisation and one step cost about as much as two steps,
                // and a step after it converges quadratically.
                if (est > p.tol_x && (rate > kChordRefactorRate || est * rate > p.tol_x)) {
                    ex.factor(cur);
                    factored = cur;
                    ++wk[kWorkFactor];
                    est = ex.correction(cur).y;
                    ++wk[kWorkApply];
                }
                continue;
            }
            corr_at = -1;    // the slot now holds the rejected trial's correction
        }
        chord_run = 0;
        if (factored != cur) { ex.factor(cur); ++wk[kWorkFactor]; }
        factored = cur;
        // GMRES on S_F^-1 J S_X d = -S_F^-1 F, right preconditioned, d_0 = 0
        const double beta0 = nr.r2;
        const double xnorm = sqrt(nr.xn2);
        double beta = beta0;
        bool have_dx = false;
        bool lucky = false;
        for (int cyc = 0;; ++cyc) {
            if (cyc == 0) {
                ex.set_basis(0, ex.fref(cur, -1.0 / beta));
            } else {
                // restart from the true linear residual -F~ - J dX
                beta = ex.restart_residual(cur, xnorm);
                ++wk[kWorkJv];
                ++wk[kWorkLincomb];
                ++wk[kWorkVecReads];
                if (!(beta > 0.0)) break;
                ex.set_basis(0, ex.vslot(0, 1.0 / beta));
            }
            ex.gm_begin(beta);
            int j = 0;
            bool conv = false;
            for (j = 0; j < p.m; ++j) {
                const double zn2 = ex.apply(ex.basis(j), j).x;
                ++wk[kWorkApply];
                if (!(zn2 > 0.0)) { lucky = true; break; }
                const double eps = lam_fd * (lam_fd + xnorm / sqrt(zn2));
                // w = J Z_j into V slot j+1, with first-pass dots and ||w||^2
                ex.jv(cur, j, eps, j + 1, hcol);
                ++gtot;
                ++wk[kWorkJv];
                if (j + 1 > 2) wk[kWorkVecReads] += j;      // w and basis vectors 2..j
                double hsq = 0.0;
                for (int i = 0; i <= j; ++i) hsq += hcol[i] * hcol[i];
                const double hn_est = sqrt(fmax(hcol[j + 1] - hsq, 0.0));
                const double res_est = ex.gm_probe(j, hcol, hn_est);
                if (res_est <= p.gamma * beta0) {
                    ex.gm_commit(j, hcol, hn_est);
                    conv = true;
                    ++j;
                    break;
                }
                // not converged: orthogonalise properly (two classical passes)
                double h2[kMaxRestart + 2];
                ex.cgs(j + 1, j + 1, hcol, h2);        // w -= V h ; h2 = V^T w
                double h3[kMaxRestart + 2];
                ex.cgs(j + 1, j + 1, h2, h3);          // w -= V h2 ; ||w||^2
                wk[kWorkCgs] += 2;
                wk[kWorkVecReads] += 2 * (j + 1 + (j + 1 > 8 ? j - 6 : 0));
                for (int i = 0; i <= j; ++i) hcol[i] += h2[i];
                const double hn = sqrt(h3[j + 1]);
                const double res = ex.gm_commit(j, hcol, hn);
                if (!(hn > 0.0)) { conv = true; ++j; lucky = true; break; }
                ex.set_basis(j + 1, ex.vslot(j + 1, 1.0 / hn));
                if (res <= p.gamma * beta0) { conv = true; ++j; break; }
            }
            const int k = j;
            if (k > 0) {
                ex.gm_solve(k, y);
                ex.direction(k, y, have_dx);
                if (k > 1 || have_dx) {
                    ++wk[kWorkLincomb];
                    wk[kWorkVecReads] += k + (have_dx ? 1 : 0);
                }
                have_dx = true;
            }
            if (conv || lucky || cyc >= p.max_restarts) break;
            ++rtot;
        }
        if (!have_dx) { status = COL_LINESEARCH; break; }
        // Backtracking: the trial X + lam S_X d is taken when the simplified
        // Newton correction there, P^-1 S_F^-1 F(X + lam S_X d), has shrunk
        // against the step: ||.||_inf <= (1 - theta lam) ||d||_inf (natural
        // monotonicity test).  If no halving passes, the full step is taken.
        const int ba = (cur + 1) % 3, bb = (cur + 2) % 3;
        double lam = 1.0, dinf = 0.0, e_full = -1.0, e_acc = -1.0;
        int bt = 0, outb = ba;
        bool accepted = false;
        Norms tn, tfull;
        for (;;) {
            outb = (bt == 0) ? ba : bb;
            tn = ex.trial(cur, outb, lam);
            ++wk[kWorkResidual];
            if (bt == 0) { tfull = tn; dinf = tn.step; }
            if (!isnan(tn.r2)) {
                const double e = ex.correction(outb).y;
                ++wk[kWorkApply];
                if (bt == 0) e_full = e;
                if (e <= (1.0 - p.theta * lam) * dinf) { accepted = true; e_acc = e; break; }
            }
            if (bt >= p.max_backtracks) break;
            lam *= 0.5;
            ++bt;
        }
        btot += bt;
        if (!accepted) {
            if (!isnan(tfull.r2)) { outb = ba; tn = tfull; e_acc = e_full; }
            else if (isnan(tn.r2)) { status = COL_NONFINITE; break; }
        }
        est = e_acc;
        corr_at = accepted ? outb : -1;
        cur = outb;
        nr = tn;
        ++it;
    }
    out.status = status;
    out.newton = it;
    out.gmres = gtot;
    out.backtracks = btot;
    out.guess = guess;
    out.restarts = rtot;
    out.chords = chords;
    for (int i = 0; i < kWorkCounts; ++i) out.work[i] = wk[i];
    out.rinf = nr.rinf;
    out.r2 = nr.r2;
    out.cur = cur;
    ex.finalize(out);
}

// ---------------------------------------------------------------------------
// In-kernel executor: the workgroup runs the control logic redundantly on
// every thread; the small dense GMRES state lives in LDS and is written by
// thread 0 between barriers.
// ---------------------------------------------------------------------------
template <int T, class FT, bool TAB = false>
struct DevExec {
    Column<T, FT, TAB> col;
    UserArrays U;

    __device__ VecRef* basis_lds() { return (VecRef*)(double*)(col.lds + Lds<T>::kBasis); }
    // the small dense GMRES state (shared host/device routines take generic pointers)
    __device__ double* Hl() { return (double*)(col.lds + Lds<T>::kH); }
    __device__ double* lg(int off) { return (double*)(col.lds + off); }

    // the batched schedule runs the gather and the write-back as launches of their own
    static constexpr bool split = true;

    __device__ Norms setup(int* cur, int* guess) { return col.setup(U, cur, guess, split); }
    __device__ bool lagged_factors() const { return col.fac_reuse; }
    __device__ bool bad_input() const { return col.bad_input; }
    __device__ void factor(int cur) { col.factor(cur); }

    __device__ VecRef fref(int cur, double sc) {
        return VecRef{col.Fb(cur, 0), col.Fb(cur, 1), sc * col.isfn, sc * col.isfp};
    }
    __device__ VecRef vslot(int k, double sc) { return VecRef{col.Vb(k, 0), col.Vb(k, 1), sc, sc}; }
    __device__ void set_basis(int i, VecRef r) {
        __syncthreads();
        if (threadIdx.x == 0) basis_lds()[i] = r;
        __syncthreads();
    }
    __device__ VecRef basis(int i) { return basis_lds()[i]; }

    __device__ Vec2<double> apply(const VecRef& v, int zslot) {
        return col.apply(v, col.Zb(zslot, 0), col.Zb(zslot, 1));
    }
    // P^-1 (-S_F^-1 F) of buffer b, into the last Krylov slot (free after GMRES)
    __device__ Vec2<double> correction(int b) {
        return col.apply(fref(b, -1.0), col.Vb(col.prm.m, 0), col.Vb(col.prm.m, 1));
    }
    __device__ void jv(int cur, int zslot, double eps, int wslot, double* dots) {
        const VecRef z{col.Zb(zslot, 0), col.Zb(zslot, 1), 1.0, 1.0};
        col.jv(cur, z, eps, col.Vb(wslot, 0), col.Vb(wslot, 1), basis_lds(), wslot, dots);
    }
    __device__ void cgs(int wslot, int nb, const double* h, double* dots) {
        col.cgs_pass(col.Vb(wslot, 0), col.Vb(wslot, 1), basis_lds(), nb, h, dots);
        __syncthreads();
    }
    __device__ void gm_begin(double beta) {
        __syncthreads();
        if (threadIdx.x == 0) {
            ldbl* g = col.lds + Lds<T>::kG;
            g[0] = beta;
            for (int i = 1; i <= kMaxRestart; ++i) g[i] = 0.0;
        }
        __syncthreads();
    }
    __device__ double gm_probe(int j, const double* h, double hn) {
        return givens_column(Hl(), kMaxRestart + 1, lg(Lds<T>::kCs), lg(Lds<T>::kSn),
                             lg(Lds<T>::kG), j, h, hn, false);
    }
    __device__ double gm_commit(int j, const double* h, double hn) {
        double r = givens_column(Hl(), kMaxRestart + 1, lg(Lds<T>::kCs), lg(Lds<T>::kSn),
                                 lg(Lds<T>::kG), j, h, hn, false);
        __syncthreads();
        if (threadIdx.x == 0)
            givens_column(Hl(), kMaxRestart + 1, lg(Lds<T>::kCs), lg(Lds<T>::kSn),
                          lg(Lds<T>::kG), j, h, hn, true);
        __syncthreads();
        return r;
    }
    __device__ void gm_solve(int k, double* y) {
        givens_solve(Hl(), kMaxRestart + 1, lg(Lds<T>::kG), k, y);
    }
    // Newton direction d = (dX if have_dx) + sum_i y_i Z_i.  A first-cycle
    // direction made of a single Krylov vector stays implicit (y_0 Z_0, no
    // sweep); restart_residual materialises it before Z_0 is reused.
    __device__ int direction(int k, const double* y, bool have_dx) {
        ldbl* misc = col.lds + Lds<T>::kMisc;
        if (k == 1 && !have_dx) {
            __syncthreads();
            if (threadIdx.x == 0) { misc[8] = 1.0; misc[9] = y[0]; }
            __syncthreads();
            return k;
        }
        VecRef zs[kMaxRestart];
        for (int i = 0; i < k; ++i) zs[i] = VecRef{col.Zb(i, 0), col.Zb(i, 1), 1.0, 1.0};
        col.lincomb(col.dXb(0), col.dXb(1), zs, y, k, have_dx);
        if (threadIdx.x == 0) misc[8] = 0.0;
        __syncthreads();
        return k;
    }
    __device__ VecRef dir_ref() {
        const ldbl* misc = col.lds + Lds<T>::kMisc;
        if (misc[8] == 1.0) return VecRef{col.Zb(0, 0), col.Zb(0, 1), misc[9], misc[9]};
        return VecRef{col.dXb(0), col.dXb(1), 1.0, 1.0};
    }
    // r = -F~ - J dX into V slot 0; returns ||r||.  Materialises an implicit
    // single-vector direction into dX first.
    __device__ double restart_residual(int cur, double xnorm) {
        ldbl* misc = col.lds + Lds<T>::kMisc;
        if (misc[8] == 1.0) {
            const VecRef z0{col.Zb(0, 0), col.Zb(0, 1), 1.0, 1.0};
            const double c = misc[9];
            col.lincomb(col.dXb(0), col.dXb(1), &z0, &c, 1, false);
            __syncthreads();
            if (threadIdx.x == 0) misc[8] = 0.0;
            __syncthreads();
        }
        const VecRef d{col.dXb(0), col.dXb(1), 1.0, 1.0};
        // ||dX||^2 for the finite-difference step
        double dd[1] = {0.0};
        for (int j = 0; j < col.cd.M; ++j) {
            const int64_t s = col.sidx(col.t, j);
            dd[0] += d.p0[s] * d.p0[s] + d.p1[s] * d.p1[s];
        }
        wg_sum<T, 1>(dd, col.lds + Lds<T>::kScr);
        if (!(dd[0] > 0.0)) return 0.0;
        const double lam_fd = 6.0554544523933395e-06;
        const double eps = lam_fd * (lam_fd + xnorm / sqrt(dd[0]));
        double dots[2];
        col.jv(cur, d, eps, col.Vb(0, 0), col.Vb(0, 1), basis_lds(), 0, dots);
        // r = -F~ - w
        const CP v0 = col.Vb(0, 0);
        const CP v1 = col.Vb(0, 1);
        const CP F0 = col.Fb(cur, 0);
        const CP F1 = col.Fb(cur, 1);
        double acc[1] = {0.0};
        for (int j = 0; j < col.cd.M; ++j) {
            const int64_t s = col.sidx(col.t, j);
            const double a = -F0[s] * col.isfn - v0[s];
            const double b = -F1[s] * col.isfp - v1[s];
            v0[s] = a; v1[s] = b;
            acc[0] += a * a + b * b;
        }
        wg_sum<T, 1>(acc, col.lds + Lds<T>::kScr);
        return sqrt(acc[0]);
    }
    __device__ Norms trial(int cur, int out, double lam) {
        return col.trial(cur, out, dir_ref(), lam);
    }
    // X_out = X_cur + S_X d with d the correction in the last Krylov slot
    __device__ Norms chord_trial(int cur, int out) {
        return col.trial(cur, out, VecRef{col.Vb(col.prm.m, 0), col.Vb(col.prm.m, 1), 1.0, 1.0}, 1.0);
    }
    __device__ void finalize(const ColOutcome& o) {
        if (!split) col.write_back(col.xb(o.cur, 0), col.xb(o.cur, 1), U.ne_out, U.phi_out);
        if (threadIdx.x == 0) {
            ColState* cs = col.W.cst + col.cd.index;
            cs->cur = o.cur;
            cs->res_inf = o.rinf; cs->res2 = o.r2;
            cs->status = o.status; cs->newton = o.newton; cs->gmres = o.gmres;
            cs->backtracks = o.backtracks; cs->guess = o.guess; cs->restarts = o.restarts;
            cs->chords = o.chords;
            for (int i = 0; i < kWorkCounts; ++i) cs->work[i] = o.work[i];
        }
    }
};

}  // namespace jfnk
