// Kernels of the MISDC time step around the electron/potential solve (paper
// Algorithm 1 restricted to the charged species, with the provisional
// charged-species update of Section 3.1 and the backward-Euler
// electron/Poisson system eq:nls of Section 3.2).  Per SDC iteration k the
// solve is preceded by one launch that forms, per cell,
//   R^(k)    = S - k_r n_e n_i                         (chemistry)
//   I_R^(k)  = (R^n + R^(k)) / 2                       (its integral over the step / dt)
//   n_i~     = n_i^n + dt [A(n_i^n; v) + I_R^(k)]
//              (provisional ions; A: second-order Godunov fluxes in the
//              drift velocity v = (v^n + v^(k)) / 2, v = u + mu_i E)
//   s        = I_R^(k), or with the electrons' SDC correction
//              s = (T_e^n - T_e^(k)) / 2 + I_R^(k), T_e = -div Gamma
//              (Scharfetter-Gummel fluxes, electrode potential at the
//              state's time)
// so that the backward-Euler solve with f = n_e^n + dt s and ion charge n_i~
// gives X^(k+1).  Natural (caller) layout, one thread per cell: the grid's
// first dimension runs over the columns, its second over 256-cell chunks.
// HBM-bound and small next to the solve: a cell reads its neighbours'
// fields and writes four values.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "jfnk_column.h"

namespace jfnk {

struct MisdcCol {
    int64_t off;              // first cell in the caller's arrays
    int64_t foff;             // first face in the face-velocity array (off + column index)
    int32_t n, bcl, bcr, pad;
    double h, dt, nel, ner, phil;
    double phir_n, phir_1;    // right electrode potential at t^n and t^n+1
};

struct MisdcArgs {
    const MisdcCol* cols;
    const double *mu, *diff, *src, *mu_i, *k_rec, *uface, *prog, *gasn;
    TabRef tab;
    const double *ne0, *phi0, *ni0;     // X^n, n_i^n
    const double *nek, *phik, *nik;     // X^(k), n_i^(k)
    double *Tn, *Rn;                    // T_e^n (electron_sdc only), R^n
    double *q, *s;                      // n_i~ and the solve's source
    double *pn, *pp;                    // 2 X^n - X^(k): the solve's extrapolated guess is then X^(k)
    double* vmax;                       // [ncols] max |v| over the faces at the start of the step
    int esdc;                           // the electrons' transport gets the SDC correction
};

// Electron flux through face j (0..n) of a column in the state (ne, phi):
// the solver's Scharfetter-Gummel flux, face mobility and diffusivity the
// arithmetic means of the two cells' (the adjacent cell's at a wall, at half
// a cell's distance), or read from the transport table at the face's mean
// progress variable, mean gas density and reduced field.
template <bool TAB>
__device__ __forceinline__ double misdc_gamma(const MisdcArgs& a, const MisdcCol& c, const double* ne,
                                              const double* phi, double phir, int j) {
    const int n = c.n;
    if ((j == 0 && c.bcl == 1) || (j == n && c.bcr == 1)) return 0.0;
    const int64_t o = c.off;
    const int64_t ia = o + (j == 0 ? 0 : j - 1), ib = o + (j == n ? n - 1 : j);
    const double hf = (j == 0 || j == n) ? 0.5 * c.h : c.h;
    const double ihf = 1.0 / hf;
    const double u = a.uface ? a.uface[c.foff + j] : 0.0;
    const double pa = j == 0 ? c.phil : phi[ia];
    const double pb = j == n ? phir : phi[ib];
    const double na = j == 0 ? c.nel : ne[ia];
    const double nb = j == n ? c.ner : ne[ib];
    double r, g, w;
    if constexpr (TAB) {
        face_rgw<true>(a.tab, 0.5 * (a.prog[ia] + a.prog[ib]), 0.5 * (a.gasn[ia] + a.gasn[ib]), u * hf, ihf,
                       pb - pa, r, g, w);
    } else {
        const double muf = 0.5 * (a.mu[ia] + a.mu[ib]), df = 0.5 * (a.diff[ia] + a.diff[ib]);
        r = muf / df; g = df * ihf; w = u * hf / df;
    }
    double bx, bmx;
    bernoulli_pair(w + r * (pb - pa), bx, bmx);
    return g * (bmx * na - bx * nb);
}

// Ion drift velocity at face j: u + mu_i,f (phi_a - phi_b) / h_f (positive
// ions move down the potential gradient; h/2 and the electrode potential at
// a wall).
__device__ __forceinline__ double misdc_vion(const MisdcArgs& a, const MisdcCol& c, const double* phi,
                                             double phir, int j) {
    const int64_t o = c.off;
    const int n = c.n;
    const double u = a.uface ? a.uface[c.foff + j] : 0.0;
    if (j == 0) return u + a.mu_i[o] * (c.phil - phi[o]) / (0.5 * c.h);
    if (j == n) return u + a.mu_i[o + n - 1] * (phi[o + n - 1] - phir) / (0.5 * c.h);
    return u + 0.5 * (a.mu_i[o + j - 1] + a.mu_i[o + j]) * (phi[o + j - 1] - phi[o + j]) / c.h;
}

// the time-centred drift velocity of face j (mean of the start of the step
// and the iterate)
__device__ __forceinline__ double misdc_vmid(const MisdcArgs& a, const MisdcCol& c, int j) {
    return 0.5 * (misdc_vion(a, c, a.phi0, c.phir_n, j) + misdc_vion(a, c, a.phik, c.phir_1, j));
}

// monotonised-central limited slope of the start-of-step ions in cell i
// (zero in the first and last cells)
__device__ __forceinline__ double misdc_slope(const MisdcArgs& a, const MisdcCol& c, int i) {
    if (i <= 0 || i >= c.n - 1) return 0.0;
    const double* x = a.ni0 + c.off;
    const double l = 2.0 * (x[i] - x[i - 1]), m = 0.5 * (x[i + 1] - x[i - 1]), r = 2.0 * (x[i + 1] - x[i]);
    if (l > 0.0 && m > 0.0 && r > 0.0) return fmin(fmin(l, m), r);
    if (l < 0.0 && m < 0.0 && r < 0.0) return -fmin(fmin(-l, -m), -r);
    return 0.0;
}

// Ion flux through face j: the upwind cell's value extrapolated to the face
// and to the half step with its forcing (R^n - n_i div v) (second-order
// Godunov); absorbing electrodes (ions only leave through a wall face, with
// the wall cell's value).
__device__ __forceinline__ double misdc_ion_flux(const MisdcArgs& a, const MisdcCol& c, int j) {
    const int n = c.n;
    const double v = misdc_vmid(a, c, j);
    const double* x = a.ni0 + c.off;
    if (j == 0) return v < 0.0 ? v * x[0] : 0.0;
    if (j == n) return v > 0.0 ? v * x[n - 1] : 0.0;
    const int up = v >= 0.0 ? j - 1 : j;
    const double div = (misdc_vmid(a, c, up + 1) - misdc_vmid(a, c, up)) / c.h;
    const double force = 0.5 * c.dt * (a.Rn[c.off + up] - x[up] * div);
    const double sg = misdc_slope(a, c, up);
    if (v >= 0.0) return v * (x[up] + 0.5 * (1.0 - v * c.dt / c.h) * sg + force);
    return v * (x[up] - 0.5 * (1.0 + v * c.dt / c.h) * sg + force);
}

// Largest ion drift speed over a column's faces at the start of the step
// (for the constant-CFL time step): one workgroup per column.
__global__ __launch_bounds__(256) void k_misdc_vmax(MisdcArgs a) {
    __shared__ double red[256];
    const MisdcCol c = a.cols[blockIdx.x];
    double m = 0.0;
    for (int j = threadIdx.x; j <= c.n; j += 256) m = fmax(m, fabs(misdc_vion(a, c, a.phi0, c.phir_n, j)));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) a.vmax[blockIdx.x] = red[0];
}

// Start of the step: R^n (and T_e^n with the electrons' SDC correction)
// from X^n, the electrode potential at t^n.
template <bool TAB>
__global__ __launch_bounds__(256) void k_misdc_start(MisdcArgs a) {
    const MisdcCol c = a.cols[blockIdx.x];
    const int i = blockIdx.y * blockDim.x + threadIdx.x;
    if (i >= c.n) return;
    const int64_t u = c.off + i;
    if (a.esdc) {
        const double gl = misdc_gamma<TAB>(a, c, a.ne0, a.phi0, c.phir_n, i);
        const double gr = misdc_gamma<TAB>(a, c, a.ne0, a.phi0, c.phir_n, i + 1);
        a.Tn[u] = -(gr - gl) / c.h;
    }
    a.Rn[u] = a.src[u] - a.k_rec[u] * a.ne0[u] * a.ni0[u];
}

// SDC iteration k: provisional ions, the correction source and the guess
// (first: the predictor, X^(0) = X^n, whose guess is the solve's own).  A
// cell whose ion mobility or recombination coefficient is negative or not
// finite gets a NaN source, so that the solve flags its column (bad input);
// non-finite ion densities reach the solve's checks through n_i~.
template <bool TAB>
__global__ __launch_bounds__(256) void k_misdc_iter(MisdcArgs a, int first) {
    const MisdcCol c = a.cols[blockIdx.x];
    const int i = blockIdx.y * blockDim.x + threadIdx.x;
    if (i >= c.n) return;
    const int64_t u = c.off + i;
    const double Rk = a.src[u] - a.k_rec[u] * a.nek[u] * a.nik[u];
    const double ir = 0.5 * (a.Rn[u] + Rk);
    const double Ai = -(misdc_ion_flux(a, c, i + 1) - misdc_ion_flux(a, c, i)) / c.h;
    double s = ir;
    if (a.esdc) {
        const double gl = misdc_gamma<TAB>(a, c, a.nek, a.phik, c.phir_1, i);
        const double gr = misdc_gamma<TAB>(a, c, a.nek, a.phik, c.phir_1, i + 1);
        s = 0.5 * (a.Tn[u] + (gr - gl) / c.h) + ir;
    }
    const bool dom = a.mu_i[u] >= 0.0 && a.mu_i[u] < INFINITY && a.k_rec[u] >= 0.0 && a.k_rec[u] < INFINITY;
    a.q[u] = a.ni0[u] + c.dt * (Ai + ir);
    a.s[u] = dom ? s : NAN;
    if (!first) {
        a.pn[u] = 2.0 * a.ne0[u] - a.nek[u];
        a.pp[u] = 2.0 * a.phi0[u] - a.phik[u];
    }
}

}  // namespace jfnk
