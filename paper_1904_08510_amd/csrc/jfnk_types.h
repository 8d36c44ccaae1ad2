// Shared host/device types of the JFNK electron/potential solver.
//
// Data layout (HBM): every per-cell workspace field is a flat array over all
// columns, columns back to back, each padded to Np = T * M cells, where T is
// the workgroup size that solves the column and M = ceil(n / T) the chunk of
// consecutive cells one thread owns.  Inside a column, cell c = t * M + j
// (thread t, row j of its chunk) is stored at offset j * T + t, so that the
// threads of a workgroup sweeping their chunks in step touch consecutive
// addresses (coalesced 64-lane accesses) while each thread still walks its
// own contiguous run of cells, as the block-tridiagonal recursions require.
// Padding cells carry zero residuals and identity Jacobian rows.
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

namespace jfnk {

constexpr int kMaxRestart = 30;      // largest GMRES restart length supported
constexpr int kRedPerChunk = 20;     // doubles of reduced-system data per chunk: A0, C0, L, D, U
constexpr int kFactorSlots = 20;     // FT values per cell stored by the factorisation
                                     // (16 block factors + 4 coupling entries of the
                                     // approximate-Schur preconditioner)
constexpr int kMgFields = 9;         // multigrid arrays per column (see Column::mgf)
constexpr int kMgCoarse = 7;         // multigrid levels of at most this many points are solved directly
constexpr int kMgMaxCycles = 200;    // V-cycles per multigrid solve at most

// Per-column counts of the phases a step executed (order of jfnk_stats.phase_counts).
// kWorkVecReads counts the FP64 vector pairs (16 bytes per cell each) that the
// dot-product sweeps, Gram-Schmidt passes and direction assemblies read beyond
// the fixed operands of those phases: basis vectors past the first two in a
// J.v product's dots (plus one re-read of w), every basis vector of a
// Gram-Schmidt pass (plus w again past the eighth), and every vector summed
// into a direction.  kWorkLearned (1 when the learned candidate's residual was
// evaluated in the set-up) is filled in by the host, which chose the columns.
enum { kWorkFactor = 0, kWorkApply, kWorkResidual, kWorkJv, kWorkCgs, kWorkLincomb, kWorkVecReads,
       kWorkLearned, kWorkCounts = 8 };

// Column status codes (also in include/jfnk.h).
enum { COL_CONVERGED = 0, COL_MAX_NEWTON = 1, COL_NONFINITE = 2, COL_LINESEARCH = 3,
       COL_BAD_INPUT = 4 };

struct ColDesc {
    int32_t n;          // cells
    int32_t M;          // chunk length (cells per thread)
    int32_t bcl, bcr;   // 0 Dirichlet, 1 zero flux
    int32_t index;      // caller's column index
    int32_t T;          // workgroup size that owns this column
    int32_t g0, gn;     // batched schedule: first gather/write-back workgroup, their count
    int64_t uoff;       // first cell in the caller's packed arrays
    int64_t ws;         // first padded cell in the workspace
    int64_t red;        // first double of the per-chunk data
    double h, dt, phil, phir, eps, nel, ner;
};

// Per-column results and solver scalars (device resident).
struct ColState {
    double sfn, sfp, sxn, sxp;      // S_F and S_X block scalars
    double rR, gR, wR;              // right-wall face coefficients
    double res_inf, res2;
    int32_t status, newton, gmres, backtracks, guess, restarts, chords;
    int32_t fac_valid;              // the workspace holds factors of this column
    int32_t work[kWorkCounts];      // phases executed this step (see kWork*)
    double fsfn, fsfp, fsxn, fsxp;  // scalings those factors were built with
    double nrR, ngR, nwR;           // right-wall face coefficients of the coming step (gather launch)
    int32_t nchanged;               // gather launch: a face coefficient differs from the stored factors'
    int32_t cur;                    // workspace buffer holding the column's X^{n+1} after the step
    int32_t mg_cycles;              // multigrid V-cycles of the step (approximate Schur + MG)
};

// Electron transport table (device arrays [nc][nx] row-major) on uniform
// grids of the progress variable c and of x = log10(|E|/N / 1 Td); mu ==
// nullptr: per-cell coefficients instead.
struct TabRef {
    const double* mu;
    const double* diff;
    int32_t nc, nx;
    double c_min, c_max, x_min, x_max;
};

struct SolverParams {
    int32_t m;              // GMRES restart length
    int32_t max_restarts;
    int32_t max_newton;
    int32_t max_backtracks;
    int32_t guess;          // 0 prev, 1 extrap, 2 learned
    int32_t has_prev;       // X^{n-1} supplied
    int32_t has_learned;    // learned candidate supplied
    int32_t has_u;          // advective face velocities supplied
    int32_t fac_reuse;      // factors left by the previous step may serve this step
    int32_t prec_kind;      // 0 exact block factorisation, 1 approximate Schur (eq:prec_recast), 2 none,
                            // 3 approximate Schur with multigrid block solves
    int32_t mg_blocks;      // kind 3: bit 0 the electron block, bit 1 the S~ block by multigrid
    int32_t mg_transfer;    // kind 3: bit k set: block k uses matrix-dependent transfers, else linear
    int32_t dlds;           // the block solve keeps its intermediate d in LDS (the launch's dynamic
                            // LDS holds Lds<T>::bytes_d(M) for the longest column), else in W.tmp
    double tol_f, tol_x, gamma, theta;
    double chord_tol;       // simplified-Newton steps while the error estimate is below this (0: off)
    double mg_tol;          // kind 3: V-cycles until ||b - A x||_2 <= mg_tol ||b||_2
    TabRef tab;             // transport table (tab.mu == nullptr: none)
};

// Caller arrays (natural layout, device pointers).
struct UserArrays {
    const double *mu, *diff, *src, *kloss, *q, *uface;
    double *ne, *phi;             // X^n
    const double *ne_prev, *phi_prev;
    double *ne_out, *phi_out;     // where X^{n+1} goes (ne, phi for an in-place step)
    const double *ne_learn, *phi_learn;
    const double *prog, *gasn;    // table transport: progress variable, gas number density
};

// Workspace (device pointers).
struct Work {
    int64_t P;                       // padded cells over all columns
    double *fa, *fg, *fw;            // left-face mu_f/D_f, D_f/h_f, u_f h_f/D_f
    double *f, *kd, *q;              // n^n + dt s, dt k, q
    double *x;                       // 3 buffers x 2 components
    double *F;                       // unscaled residuals, 3 x 2
    double *V;                       // Krylov basis (m+1) x 2
    double *Z;                       // preconditioned basis m x 2
    double *dX;                      // Newton direction (scaled), 2
    void *fac;                       // kFactorSlots x P values of the factor type
    void *tmp;                       // 2 x P values of the factor type (apply)
    double *red;                     // per-chunk reduced-system data
    double *sch;                     // 4 x P doubles: approximate-Schur apply temporaries
    double *mg;                      // kMgFields x mgP doubles: multigrid arrays (kind 3 only)
    int64_t mgP;                     // doubles per multigrid field: 2 P + 64 max_cols
    ColDesc *cols;
    ColState *cst;
    double *scal;                    // per-column scalar exchange (host-driven mode)
    const int32_t *lmask;            // per column: learned candidate present (guess 2)
    int32_t *gflag;                  // per gather workgroup: a face coefficient changed
};

}  // namespace jfnk
