// Per-column phases of the JFNK electron/potential solve, executed by one
// workgroup of T threads that owns the column (layout in jfnk_types.h).
//
// Method (paper Section 3.2, Algorithm 2): Newton on the backward-Euler
// residual F(X) = 0 of the electron transport and Poisson equations
// (eq:nls), scaled by S_F, S_X (eq:newton_sc); each Newton system is solved
// by right-preconditioned GMRES from dX_0 = 0, with the finite-difference
// product J v ~ [F(X + eps v) - F(X)] / eps (eq:jf_dfapprox) and the
// step eps = lambda (lambda + |X| / |v|), lambda = eps_mach^(1/3); the
// preconditioner is the exact inverse of the 2x2 block Jacobian (the
// paper's eq:prec is exact too), obtained here by a direct block-tridiagonal
// factorisation instead of the paper's Schur complement + multigrid, since in
// 1D the Jacobian of the scheme is exactly 2x2 block tridiagonal.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "jfnk_types.h"

namespace jfnk {

// ---------------------------------------------------------------------------
// 2x2 blocks
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

template <class R>
struct Blk { R a, b, c, d; };   // [[a b] [c d]]
template <class R>
struct Vec2 { R x, y; };
// aligned records for vector loads and stores (one instruction per record)
template <class R>
struct alignas(4 * sizeof(R)) V4 { R a, b, c, d; };
template <class R>
struct alignas(2 * sizeof(R)) V2 { R x, y; };

template <class R> __device__ __forceinline__ Blk<R> bmul(const Blk<R>& p, const Blk<R>& q) {
    return {p.a * q.a + p.b * q.c, p.a * q.b + p.b * q.d, p.c * q.a + p.d * q.c, p.c * q.b + p.d * q.d};
}
template <class R> __device__ __forceinline__ Vec2<R> bmv(const Blk<R>& p, const Vec2<R>& v) {
    return {p.a * v.x + p.b * v.y, p.c * v.x + p.d * v.y};
}
template <class R> __device__ __forceinline__ Blk<R> bsub(const Blk<R>& p, const Blk<R>& q) {
    return {p.a - q.a, p.b - q.b, p.c - q.c, p.d - q.d};
}
template <class R> __device__ __forceinline__ Blk<R> bneg(const Blk<R>& p) { return {-p.a, -p.b, -p.c, -p.d}; }
template <class R> __device__ __forceinline__ Blk<R> binv(const Blk<R>& p) {
    const R id = R(1) / (p.a * p.d - p.b * p.c);
    return {p.d * id, -p.b * id, -p.c * id, p.a * id};
}
__device__ __forceinline__ Blk<double> bzero() { return {0.0, 0.0, 0.0, 0.0}; }

// Store through the global address space.  A store through a generic (flat)
// pointer also counts against the LDS wait counter, so the next barrier or
// LDS reduction would wait for it to reach memory; a global store does not.
template <class R>
__device__ __forceinline__ void gst(R* p, R v) { *(__attribute__((address_space(1))) R*)p = v; }
// Load through the global address space.  The wait counter of vector memory
// completes global accesses in order, so a sweep can wait for one group of
// loads while the next group is in flight; a generic (flat) access may also
// reach LDS, and every wait on one drains all outstanding memory operations.
template <class R>
__device__ __forceinline__ R gld(const R* p) { return *(const __attribute__((address_space(1))) R*)p; }
// The records go through vector types: an aggregate load is split into
// scalar loads that the optimiser may issue through the original generic
// pointer.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ V4<float> gld(const V4<float>* p) {
    const f32x4 r = *(const __attribute__((address_space(1))) f32x4*)p;
    return {r.x, r.y, r.z, r.w};
}
__device__ __forceinline__ V2<float> gld(const V2<float>* p) {
    const f32x2 r = *(const __attribute__((address_space(1))) f32x2*)p;
    return {r.x, r.y};
}
__device__ __forceinline__ V4<double> gld(const V4<double>* p) {
    const f64x4 r = *(const __attribute__((address_space(1))) f64x4*)p;
    return {r.x, r.y, r.z, r.w};
}
__device__ __forceinline__ V2<double> gld(const V2<double>* p) {
    const f64x2 r = *(const __attribute__((address_space(1))) f64x2*)p;
    return {r.x, r.y};
}
__device__ __forceinline__ void gst(V4<float>* p, V4<float> v) {
    *(__attribute__((address_space(1))) f32x4*)p = f32x4{v.a, v.b, v.c, v.d};
}
__device__ __forceinline__ void gst(V2<float>* p, V2<float> v) {
    *(__attribute__((address_space(1))) f32x2*)p = f32x2{v.x, v.y};
}
__device__ __forceinline__ void gst(V4<double>* p, V4<double> v) {
    *(__attribute__((address_space(1))) f64x4*)p = f64x4{v.a, v.b, v.c, v.d};
}
__device__ __forceinline__ void gst(V2<double>* p, V2<double> v) {
    *(__attribute__((address_space(1))) f64x2*)p = f64x2{v.x, v.y};
}
__device__ __forceinline__ Blk<double> beye() { return {1.0, 0.0, 0.0, 1.0}; }

// ---------------------------------------------------------------------------
// Bernoulli function B(x) = x / (e^x - 1) for the Scharfetter-Gummel flux.
// One expm1 per face gives both B(x) and B(-x): with a = |x|,
// B(-a) = B(a) + a, a sum of two non-negative terms (no cancellation).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bernoulli_pair(double x, double& bx, double& bmx) {
    const double a = fabs(x);
    double ba;
    if (a < 1e-3) {
        // 1 / (expm1(a)/a), Taylor series of expm1(a)/a to a^4
        ba = 1.0 / (1.0 + a * (0.5 + a * (1.0 / 6.0 + a * (1.0 / 24.0 + a * (1.0 / 120.0)))));
    } else {
        ba = a / expm1(a);
    }
    const double bna = ba + a;
    if (x >= 0.0) { bx = ba; bmx = bna; } else { bx = bna; bmx = ba; }
}

// dB/dx at x and at -x: B'(x) = (B(x)/x)(1 - B(-x)), -1/2 + x/6 - x^3/180 near 0.
__device__ __forceinline__ void bernoulli_dpair(double x, double bx, double bmx, double& dbx,
                                                double& dbmx) {
    if (fabs(x) < 1e-3) {
        const double x3 = x * x * x;
        dbx = -0.5 + x * (1.0 / 6.0) - x3 * (1.0 / 180.0);
        dbmx = -0.5 - x * (1.0 / 6.0) + x3 * (1.0 / 180.0);
    } else {
        dbx = (bx / x) * (1.0 - bmx);
        dbmx = -(bmx / x) * (1.0 - bx);
    }
}

// ---------------------------------------------------------------------------
// Face coefficients.  A face record holds (a, b, c); the Scharfetter-Gummel
// flux needs r = mu_f/D_f, g = D_f/h_f and w = u_f h_f/D_f.  Per-cell
// transport: the record is (r, g, w) itself.  Table transport (Section 2.2):
// the record is (mean progress variable, mean gas number density N (0 at a
// zero-flux wall), u_f h_f), and mu_f, D_f are read from the table at the
// face's reduced field |E|/N = |dphi| / (h_f N) (bilinear, clamped to the
// grid; a zero field reads the lowest column) in the state at hand.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double tab_interp(const TabRef& t, const double* v, int i, int k, double wc,
                                             double wx) {
    const double* r0 = v + (int64_t)i * t.nx;
    const double* r1 = r0 + t.nx;
    return (1.0 - wc) * ((1.0 - wx) * gld(r0 + k) + wx * gld(r0 + k + 1)) +
           wc * ((1.0 - wx) * gld(r1 + k) + wx * gld(r1 + k + 1));
}

template <bool TAB>
__device__ __forceinline__ void face_rgw(const TabRef& t, double a, double b, double c, double ihf, double dphi,
                                         double& r, double& g, double& w) {
    if constexpr (!TAB) {
        r = a; g = b; w = c;
    } else {
        if (!(b > 0.0)) { r = 0.0; g = 0.0; w = 0.0; return; }
        const double en = fabs(dphi) * ihf / b * 1e21;          // reduced field in Td
        double x = en > 0.0 ? log10(en) : t.x_min;
        x = fmin(fmax(x, t.x_min), t.x_max);
        const double cv = fmin(fmax(a, t.c_min), t.c_max);
        const double fc = (cv - t.c_min) / (t.c_max - t.c_min) * (t.nc - 1);
        const double fx = (x - t.x_min) / (t.x_max - t.x_min) * (t.nx - 1);
        const int i = min((int)floor(fc), t.nc - 2);
        const int k = min((int)floor(fx), t.nx - 2);
        const double wc = fc - i, wx = fx - k;
        const double mu = tab_interp(t, t.mu, i, k, wc, wx);
        const double d = tab_interp(t, t.diff, i, k, wc, wx);
        r = mu / d;
        g = d * ihf;
        w = c / d;
    }
}

// The same face coefficients and their derivatives with respect to the
// potential difference dphi across the face (zero without a table, where an
// argument is clamped to the grid, and at zero field): with x = log10(|E|/N)
// and E = |dphi| / h_f, dx/d(dphi) = 1 / (dphi ln 10), and the bilinear
// interpolant's slope in x gives dmu/dx and dD/dx.
template <bool TAB>
__device__ __forceinline__ void face_rgw_d(const TabRef& t, double a, double b, double c, double ihf, double dphi,
                                           double& r, double& g, double& w, double& dr, double& dg, double& dw) {
    dr = 0.0; dg = 0.0; dw = 0.0;
    if constexpr (!TAB) {
        r = a; g = b; w = c;
    } else {
        if (!(b > 0.0)) { r = 0.0; g = 0.0; w = 0.0; return; }
        const double en = fabs(dphi) * ihf / b * 1e21;
        const double x0 = en > 0.0 ? log10(en) : t.x_min;
        const bool inside = en > 0.0 && x0 > t.x_min && x0 < t.x_max;
        const double x = fmin(fmax(x0, t.x_min), t.x_max);
        const double cv = fmin(fmax(a, t.c_min), t.c_max);
        const double fc = (cv - t.c_min) / (t.c_max - t.c_min) * (t.nc - 1);
        const double fx = (x - t.x_min) / (t.x_max - t.x_min) * (t.nx - 1);
        const int i = min((int)floor(fc), t.nc - 2);
        const int k = min((int)floor(fx), t.nx - 2);
        const double wc = fc - i, wx = fx - k;
        const double mu = tab_interp(t, t.mu, i, k, wc, wx);
        const double d = tab_interp(t, t.diff, i, k, wc, wx);
        r = mu / d;
        g = d * ihf;
        w = c / d;
        if (inside) {
            const double sx = (t.nx - 1) / (t.x_max - t.x_min) / (dphi * 2.302585092994046);
            const double* m0 = t.mu + (int64_t)i * t.nx;
            const double* d0 = t.diff + (int64_t)i * t.nx;
            const double dmu = ((1.0 - wc) * (gld(m0 + k + 1) - gld(m0 + k)) +
                                wc * (gld(m0 + t.nx + k + 1) - gld(m0 + t.nx + k))) * sx;
            const double dd = ((1.0 - wc) * (gld(d0 + k + 1) - gld(d0 + k)) +
                               wc * (gld(d0 + t.nx + k + 1) - gld(d0 + t.nx + k))) * sx;
            dr = (dmu * d - mu * dd) / (d * d);
            dg = dd * ihf;
            dw = -c * dd / (d * d);
        }
    }
}

// ---------------------------------------------------------------------------
// Workgroup reductions (wave64 butterflies + LDS across waves).  Fixed order:
// bitwise reproducible from run to run.
// ---------------------------------------------------------------------------
// LDS-typed double: the solver keeps its workgroup scratch behind a pointer
// of this type, so accesses compile to LDS instructions even in phase
// functions the compiler keeps out of line (a generic pointer would compile
// to flat accesses, which also wait on the vector-memory counter).
typedef __attribute__((address_space(3))) double ldbl;

template <int T, int K, class SP>
__device__ __forceinline__ void wg_sum(double (&v)[K], SP scr) {
    constexpr int NW = T / 64;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) scr[k * NW + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) s += scr[k * NW + i];
        v[k] = s;
    }
    __syncthreads();
}

template <int T, int K, class SP>
__device__ __forceinline__ void wg_max(double (&v)[K], SP scr) {
    constexpr int NW = T / 64;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] = fmax(v[k], __shfl_xor(v[k], off, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) scr[k * NW + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = scr[k * NW];
#pragma unroll
        for (int i = 1; i < NW; ++i) s = fmax(s, scr[k * NW + i]);
        v[k] = s;
    }
    __syncthreads();
}

// A two-component vector of one column with a scale per component:
// value(s) = (p0[s] * s0, p1[s] * s1).
// One component of a two-component per-cell field (n_e, phi) stored as
// interleaved pairs: element s of component c sits at base[2 s + c].  The
// two components of a cell then sit in one 16-byte record, and a sweep that
// reads both issues one vector load for them.
struct CP {
    double* p;
    // device memory, accessed through the global address space
    __device__ __forceinline__ __attribute__((address_space(1))) double& operator[](int64_t s) const {
        return ((__attribute__((address_space(1))) double*)p)[2 * s];
    }
};

struct VecRef {
    CP p0;
    CP p1;
    double s0, s1;
};

// Both components of cell s of a vector whose components are the two halves
// of one pair array (p1 = p0 + 1: every Krylov vector, preconditioned
// vector, residual and direction), with one 16-byte load.
__device__ __forceinline__ Vec2<double> ld_pair(const VecRef& v, int64_t s) {
    const V2<double> r = gld((const V2<double>*)(v.p0.p + 2 * s));
    return {r.x, r.y};
}

struct Norms {
    double rinf;    // ||S_F^-1 F||_inf
    double r2;      // ||S_F^-1 F||_2
    double xn2;     // ||S_X^-1 X||_2^2
    double step;    // ||S_X^-1 dX||_inf of the step that produced X
};

// LDS layout of a column workgroup (doubles):
//   [0, 14T)            PCR rows / exchange buffers
//   [14T, 14T + 16*NW)  reduction scratch
//   then the GMRES small dense state.
template <int T>
struct Lds {
    static constexpr int NW = T / 64;
    static constexpr int kPcr = 0;
    static constexpr int kScr = 14 * T;
    static constexpr int kH = kScr + 16 * NW;                   // (m+1) x m, column major
    static constexpr int kCs = kH + (kMaxRestart + 1) * kMaxRestart;
    static constexpr int kSn = kCs + kMaxRestart;
    static constexpr int kG = kSn + kMaxRestart;
    static constexpr int kY = kG + kMaxRestart + 1;
    static constexpr int kMisc = kY + kMaxRestart;               // 16 scalar slots
    static constexpr int kBasis = kMisc + 16;                    // (m+1) VecRefs (4 words each)
    static constexpr int kTotal = kBasis + 4 * (kMaxRestart + 1);
    static constexpr size_t bytes() { return sizeof(double) * kTotal; }
    // with SolverParams::dlds: the block solve's intermediate d (2 factor
    // values per cell, rows j*T + t of up to m rows per thread) after the rest
    static constexpr int kDTmp = (kTotal + 1) & ~1;                // 16-byte aligned
    static constexpr size_t bytes_d(int m, size_t fts) { return sizeof(double) * kDTmp + (size_t)m * T * 2 * fts; }
};

// ---------------------------------------------------------------------------
// The column object: phases over the column owned by this workgroup.
// ---------------------------------------------------------------------------
template <int T, class FT, bool TAB = false>
struct Column {
    ColDesc cd;
    Work W;
    SolverParams prm;
    ldbl* lds;
    int t;
    double ih, dth, epsh;            // 1/h, dt/h, (eps/e)/h
    double rR, gR, wR;               // right-wall face coefficients
    double sfn, sfp, sxn, sxp, isfn, isfp;
    bool fac_reuse = false;          // setup found the previous step's factors usable
    bool bad_input = false;          // setup found an input outside the problem's domain

    __device__ void init(const ColDesc& d, const Work& w, const SolverParams& p, ldbl* l) {
        cd = d; W = w; prm = p; lds = l;
        t = threadIdx.x;
        ih = 1.0 / cd.h;
        dth = cd.dt / cd.h;
        epsh = cd.eps / cd.h;
    }

    __device__ __forceinline__ int64_t sidx(int tt, int j) const {
        return cd.ws + (int64_t)j * T + tt;
    }
    // two-component fields: buffer b is an array of P (n_e, phi) pairs
    __device__ __forceinline__ CP xb(int b, int comp) const { return CP{W.x + 2 * b * W.P + comp}; }
    __device__ __forceinline__ CP Fb(int b, int comp) const { return CP{W.F + 2 * b * W.P + comp}; }
    __device__ __forceinline__ CP Vb(int k, int comp) const { return CP{W.V + 2 * (int64_t)k * W.P + comp}; }
    __device__ __forceinline__ CP Zb(int k, int comp) const { return CP{W.Z + 2 * (int64_t)k * W.P + comp}; }
    __device__ __forceinline__ CP dXb(int comp) const { return CP{W.dX + comp}; }
    __device__ __forceinline__ CP schb(int k) const { return CP{W.sch + 2 * (k >> 1) * W.P + (k & 1)}; }
    // Per-cell factor values (FT), one record per cell for each group of
    // values a sweep reads together, so a sweep loads whole records with
    // vector instructions:
    //   [P][8]  slots 0..7:   m and m A      (apply down sweep)
    //   [P][4]  slots 8..11:  g = m C        (apply down and back sweeps)
    //   [P][4]  slots 12..15: a, the left-coupling spike recurrence (back sweep)
    //   [P][4]  slots 16..19: approximate-Schur couplings
    __device__ __forceinline__ FT* facp(int slot, int64_t s) const {
        FT* base = (FT*)W.fac;
        if (slot < 8) return base + s * 8 + slot;
        if (slot < 12) return base + 8 * W.P + s * 4 + (slot - 8);
        if (slot < 16) return base + 12 * W.P + s * 4 + (slot - 12);
        return base + 16 * W.P + s * 4 + (slot - 16);
    }
    // the apply's intermediate d (2 FT per cell), one record per cell
    __device__ __forceinline__ V2<FT>* tmpp(int64_t s) const { return (V2<FT>*)W.tmp + s; }
    // this thread's chunk entry of per-chunk slot k (SoA over the chunks)
    __device__ __forceinline__ double* red(int k) const { return W.red + cd.red + (int64_t)k * T + t; }

    // ------------------------------------------------------------------
    // Generic stencil sweep.  Thread t walks cells c = t*M + j, j = 0..M-1,
    // carrying the left face; faces see (left state, right state).  The cells
    // are taken in groups of U: all loads of a group (right-neighbour state,
    // face coefficients, and the cell's own operands from own(s)) are issued
    // before any cell of the group is computed, so the global-load latencies
    // of U cells overlap instead of serialising along the recursion.
    // getx(s, n, phi) returns the state at a storage index; cell(...) receives
    // both faces and the own operands of each real cell; pad(s) is called for
    // padding cells (always after the real cells of a chunk).
    // ------------------------------------------------------------------
    template <int U, class FaceRec, class GetX, class FaceFn, class OwnFn, class CellFn, class PadFn>
    __device__ __forceinline__ void sweep(GetX getx, FaceFn face, OwnFn own, CellFn cell, PadFn pad) {
        using Own = decltype(own(int64_t(0)));
        const int M = cd.M, n = cd.n;
        const int c0 = t * M;
        if (c0 >= n) {
            for (int j = 0; j < M; ++j) pad(sidx(t, j));
            return;
        }
        const int jr = (n - c0 < M) ? (n - c0) : M;   // real rows of this chunk
        const int64_t s0 = sidx(t, 0);
        double nC, pC, nL, pL, ihL;
        getx(s0, nC, pC);
        if (c0 == 0) { nL = cd.nel; pL = cd.phil; ihL = 2.0 * ih; }
        else { getx(sidx(t - 1, M - 1), nL, pL); ihL = ih; }
        FaceRec FL = face(gld(W.fa + s0), gld(W.fg + s0), prm.has_u ? gld(W.fw + s0) : 0.0, ihL, nL, pL, nC, pC);
        // Group of U rows' operands.  Loads carry no conditions, so a group's
        // loads issue back to back: rows past the chunk's end reload its last
        // real row, and the last cell of the column reloads itself in place of
        // its (absent) right neighbour; neither value is used.  Without flow
        // the u_f h_f/D_f loads read the mu_f/D_f array instead (the same
        // cache lines: no memory traffic) and the value is not used.
        const double* const fwa = prm.has_u ? W.fw : W.fa;
        struct Grp {
            double xn[U], xp[U], fa[U], fg[U], fw[U];
            Own ow[U];
        };
        auto load_grp = [&](int j0, Grp& g) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = min(j0 + u, jr - 1);
                const int64_t s = sidx(t, j);
                g.ow[u] = own(s);
                const int64_t sn = (c0 + j >= n - 1) ? s : ((j + 1 < M) ? s + T : sidx(t + 1, 0));
                getx(sn, g.xn[u], g.xp[u]);
                g.fa[u] = gld(W.fa + sn);
                g.fg[u] = gld(W.fg + sn);
                g.fw[u] = gld(fwa + sn);
            }
        };
        // Double buffer: the next group's loads issue before this group's
        // results are stored.  Loads and stores share one in-order counter, so
        // loads issued after the stores would also wait for the stores to
        // reach memory.
        Grp gc, gn;
        load_grp(0, gc);
        for (int j0 = 0; j0 < jr; j0 += U) {
            load_grp(j0 + U, gn);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 + u;
                if (j < jr) {
                    const int c = c0 + j;
                    const int64_t s = sidx(t, j);
                    double nR, pR;
                    FaceRec FR;
                    if (c == n - 1) {
                        nR = cd.ner; pR = cd.phir;
                        FR = face(rR, gR, wR, 2.0 * ih, nC, pC, nR, pR);
                    } else {
                        nR = gc.xn[u]; pR = gc.xp[u];
                        FR = face(gc.fa[u], gc.fg[u], prm.has_u ? gc.fw[u] : 0.0, ih, nC, pC, nR, pR);
                    }
                    cell(s, c, nC, pC, FL, FR, gc.ow[u]);
                    nC = nR; pC = pR; FL = FR;
                }
            }
            gc = gn;
        }
        for (int j = jr; j < M; ++j) pad(sidx(t, j));
    }

    // The same sweep over two states A and B at once (shared coefficient
    // loads and one pass): faceA/faceB build the face records of each state,
    // cell(s, c, nA, pA, nB, pB, LA, RA, LB, RB, own) sees both.
    template <int U, class RecA, class RecB, class GetXA, class GetXB, class FaceA, class FaceB, class OwnFn,
              class CellFn, class PadFn>
    __device__ __forceinline__ void sweep2(GetXA gxa, GetXB gxb, FaceA fA, FaceB fB, OwnFn own, CellFn cell,
                                           PadFn pad) {
        using Own = decltype(own(int64_t(0)));
        const int M = cd.M, n = cd.n;
        const int c0 = t * M;
        if (c0 >= n) {
            for (int j = 0; j < M; ++j) pad(sidx(t, j));
            return;
        }
        const int jr = (n - c0 < M) ? (n - c0) : M;
        const int64_t s0 = sidx(t, 0);
        double nA, pA, nB, pB, nAL, pAL, nBL, pBL, ihL;
        gxa(s0, nA, pA);
        gxb(s0, nB, pB);
        if (c0 == 0) {
            nAL = nBL = cd.nel; pAL = pBL = cd.phil; ihL = 2.0 * ih;
        } else {
            const int64_t sl = sidx(t - 1, M - 1);
            gxa(sl, nAL, pAL);
            gxb(sl, nBL, pBL);
            ihL = ih;
        }
        const double fw0 = prm.has_u ? gld(W.fw + s0) : 0.0;
        RecA FLA = fA(gld(W.fa + s0), gld(W.fg + s0), fw0, ihL, nAL, pAL, nA, pA);
        RecB FLB = fB(gld(W.fa + s0), gld(W.fg + s0), fw0, ihL, nBL, pBL, nB, pB);
        // double-buffered groups with unconditional loads, as in sweep
        const double* const fwa = prm.has_u ? W.fw : W.fa;
        struct Grp {
            double an[U], ap[U], bn[U], bp[U], fa[U], fg[U], fw[U];
            Own ow[U];
        };
        auto load_grp = [&](int j0, Grp& g) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = min(j0 + u, jr - 1);
                const int64_t s = sidx(t, j);
                g.ow[u] = own(s);
                const int64_t sn = (c0 + j >= n - 1) ? s : ((j + 1 < M) ? s + T : sidx(t + 1, 0));
                gxa(sn, g.an[u], g.ap[u]);
                gxb(sn, g.bn[u], g.bp[u]);
                g.fa[u] = gld(W.fa + sn);
                g.fg[u] = gld(W.fg + sn);
                g.fw[u] = gld(fwa + sn);
            }
        };
        Grp gc, gn;
        load_grp(0, gc);
        for (int j0 = 0; j0 < jr; j0 += U) {
            load_grp(j0 + U, gn);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 + u;
                if (j < jr) {
                    const int c = c0 + j;
                    const int64_t s = sidx(t, j);
                    RecA FRA;
                    RecB FRB;
                    double nAR, pAR, nBR, pBR;
                    if (c == n - 1) {
                        nAR = nBR = cd.ner; pAR = pBR = cd.phir;
                        FRA = fA(rR, gR, wR, 2.0 * ih, nA, pA, nAR, pAR);
                        FRB = fB(rR, gR, wR, 2.0 * ih, nB, pB, nBR, pBR);
                    } else {
                        nAR = gc.an[u]; pAR = gc.ap[u]; nBR = gc.bn[u]; pBR = gc.bp[u];
                        const double wu = prm.has_u ? gc.fw[u] : 0.0;
                        FRA = fA(gc.fa[u], gc.fg[u], wu, ih, nA, pA, nAR, pAR);
                        FRB = fB(gc.fa[u], gc.fg[u], wu, ih, nB, pB, nBR, pBR);
                    }
                    cell(s, c, nA, pA, nB, pB, FLA, FRA, FLB, FRB, gc.ow[u]);
                    nA = nAR; pA = pAR; nB = nBR; pB = pBR;
                    FLA = FRA; FLB = FRB;
                }
            }
            gc = gn;
        }
        for (int j = jr; j < M; ++j) pad(sidx(t, j));
    }

    struct FluxRec { double gam, grd; };

    // electron flux and potential gradient of one face
    struct FluxFace {
        TabRef tb;
        __device__ __forceinline__ FluxRec operator()(double fa, double fb, double fc, double ihf,
                                                      double nA, double pA, double nB, double pB) const {
            double r, g, w;
            face_rgw<TAB>(tb, fa, fb, fc, ihf, pB - pA, r, g, w);
            const double pe = w + r * (pB - pA);
            double bx, bmx;
            bernoulli_pair(pe, bx, bmx);
            return {g * (bmx * nA - bx * nB), (pB - pA) * ihf};
        }
    };

    // ------------------------------------------------------------------
    // The phases called out of line (the apply, the factorisation, trial and
    // residual evaluations, J.v, Gram-Schmidt passes, linear combinations)
    // run on a private copy of the column object.  In an out-of-line call
    // `this` is a generic pointer that a store through any vector pointer
    // might alias, so each field it reads would be loaded again (with a
    // generic load, which drains every outstanding memory operation) after
    // each store; the copy's fields stay in registers.
    // ------------------------------------------------------------------

    // ------------------------------------------------------------------
    // Residual F(X) at the state returned by getx; writes F (unscaled) and,
    // optionally, the state itself; returns the scaled norms.
    // ------------------------------------------------------------------
    template <class GetX>
    __device__ __forceinline__ Norms residual(GetX getx, CP oF0, CP oF1, CP oX0, CP oX1,
                              VecRef stepdir, double steplam) {
        double mx[3] = {0.0, 0.0, 0.0};       // max|Fe|, max|Fp|, max|step|
        double sm[4] = {0.0, 0.0, 0.0, 0.0};  // sum Fe^2, sum Fp^2, sum n^2, sum phi^2
        const double dt_h = dth, eps_h = epsh;
        const double* fv = W.f;
        const double* kv = W.kd;
        const double* qv = W.q;
        const bool wantstep = stepdir.p0.p != nullptr;
        // without a step direction the step loads read a valid array instead
        // (unconditional loads issue back to back) and are not used
        const CP dp0 = wantstep ? stepdir.p0 : xb(0, 0);
        const CP dp1 = wantstep ? stepdir.p1 : xb(0, 1);
        struct Own { double f, k, q, d0, d1; };
        sweep<2, FluxRec>(getx, FluxFace{prm.tab},
            [&](int64_t s) {
                Own o;
                o.f = gld(fv + s); o.k = gld(kv + s); o.q = gld(qv + s);
                o.d0 = dp0[s];
                o.d1 = dp1[s];
                return o;
            },
            [&](int64_t s, int c, double nC, double pC, const FluxRec& L, const FluxRec& R, const Own& o) {
                const double fe = -nC + o.f - o.k * nC - dt_h * (R.gam - L.gam);
                const double fp = -nC + o.q + eps_h * (R.grd - L.grd);
                oF0[s] = fe;
                oF1[s] = fp;
                if (oX0.p) { oX0[s] = nC; oX1[s] = pC; }
                mx[0] = fmax(mx[0], fabs(fe));
                mx[1] = fmax(mx[1], fabs(fp));
                sm[0] += fe * fe;
                sm[1] += fp * fp;
                sm[2] += nC * nC;
                sm[3] += pC * pC;
                if (wantstep) {
                    mx[2] = fmax(mx[2], fmax(fabs(steplam * o.d0 * stepdir.s0),
                                             fabs(steplam * o.d1 * stepdir.s1)));
                }
            },
            [&](int64_t s) {
                oF0[s] = 0.0; oF1[s] = 0.0;
                if (oX0.p) { oX0[s] = 0.0; oX1[s] = 0.0; }
            });
        ldbl* scr = lds + Lds<T>::kScr;
        wg_max<T, 3>(mx, scr);
        wg_sum<T, 4>(sm, scr);
        Norms r;
        r.rinf = fmax(mx[0] * isfn, mx[1] * isfp);
        r.r2 = sqrt(sm[0] * isfn * isfn + sm[1] * isfp * isfp);
        r.xn2 = sm[2] / (sxn * sxn) + sm[3] / (sxp * sxp);
        r.step = mx[2];
        if (isnan(sm[0]) || isnan(sm[1])) r.r2 = NAN;
        return r;
    }

    // ------------------------------------------------------------------
    // Step setup: caller arrays -> workspace, scalings from X^n, initial
    // guess candidates and the choice between them.  Returns the norms of
    // the chosen guess; *cur receives its buffer.
    // ------------------------------------------------------------------
    // ------------------------------------------------------------------
    // Gather pass: the caller's arrays (natural layout) -> the face and cell
    // coefficients and the start states X^n, the extrapolation 2 X^n - X^{n-1}
    // and the learned candidate (chunk-interleaved layout).  Tiles of 8 chunk
    // owners x 8 rows, one per wave: lane l takes owner 8g + l/8 and row
    // 8b + l%8 of tile (b, g), so 8 lanes read 8 consecutive cells of the
    // caller's arrays and 8 lanes write 8 consecutive chunk-interleaved slots
    // (64-byte pieces on both sides).  Wave w of nw takes tiles w, w + nw, ...
    // (the loads of UC tiles go first).  Tiles run through the row groups of
    // 8 owners first, so the UC * nw tiles a workgroup has in flight cover
    // whole chunks of adjacent owners: one contiguous range of the caller's
    // arrays, and whole (or half) cache lines of the interleaved rows.
    // Returns a mask: kGatherChanged when a face coefficient of the cells this
    // thread wrote differs from the one the stored factors were built with,
    // kGatherBad when one of its cells has an input outside the problem's
    // domain (mu < 0, D <= 0, k < 0, or a non-finite value); the thread of the
    // last cell writes the right-wall face coefficients to wall[0..2]
    // (global or LDS memory: stored through a generic pointer).
    // ------------------------------------------------------------------
    // tiles of 8 x 8 cells of this column's layout
    __device__ __forceinline__ int ntiles() const { return ((cd.M + 7) >> 3) * (T / 8); }

    static constexpr int kGatherChanged = 1, kGatherBad = 2;

    __device__ int gather(const UserArrays& U, int kb, int ke, int w, int nw, double* wall) {
        const int M = cd.M, n = cd.n;
        const double dt = cd.dt, hb = 0.5 * cd.h;
        const int64_t fo = cd.uoff + cd.index;   // faces of column: n + 1 per column
        const CP X00 = xb(0, 0); const CP X01 = xb(0, 1);
        const CP X10 = xb(1, 0); const CP X11 = xb(1, 1);
        const CP X20 = xb(2, 0); const CP X21 = xb(2, 1);
        const bool extrap = prm.guess >= 1 && prm.has_prev;
        const bool learn = prm.guess == 2 && prm.has_learned && W.lmask[cd.index] != 0;
        const bool may_reuse = prm.fac_reuse && W.cst[cd.index].fac_valid;
        bool changed = false, bad = false;
        constexpr int UC = 2;
        const int lane = threadIdx.x & 63;
        const int nrg = (M + 7) >> 3;            // row groups of 8
        auto tile_cell = [&](int k, int& tt, int& j) {
            tt = (k / nrg) * 8 + (lane >> 3);
            j = (k % nrg) * 8 + (lane & 7);
        };
        for (int k0 = kb + w; k0 < ke; k0 += UC * nw) {
            double mu[UC], D[UC], mum[UC], Dm[UC], ne[UC], ph[UC], sr[UC], kl[UC], qq[UC];
            double pn[UC], pp[UC], ln[UC], lp[UC], uf[UC];
            double ofa[UC], ofg[UC], ofw[UC], okd[UC];   // this column's coefficients of the last step
#pragma unroll
            for (int v = 0; v < UC; ++v) {
                const int k = k0 + v * nw;
                int tt, j;
                tile_cell(k, tt, j);
                const int c = tt * M + j;
                mu[v] = D[v] = mum[v] = Dm[v] = ne[v] = ph[v] = sr[v] = kl[v] = qq[v] = 0.0;
                pn[v] = pp[v] = ln[v] = lp[v] = uf[v] = 0.0;
                ofa[v] = ofg[v] = ofw[v] = okd[v] = 0.0;
                if (may_reuse && k < ke && j < M && c < n) {
                    const int64_t s = cd.ws + (int64_t)j * T + tt;
                    ofa[v] = gld(W.fa + s); ofg[v] = gld(W.fg + s); okd[v] = gld(W.kd + s);
                    if (prm.has_u) ofw[v] = gld(W.fw + s);
                }
                if (k < ke && j < M && c < n) {
                    const int64_t u = cd.uoff + c;
                    // table transport: (mu, D) slots carry (progress variable, gas density)
                    const double* A0 = TAB ? U.prog : U.mu;
                    const double* A1 = TAB ? U.gasn : U.diff;
                    mu[v] = gld(A0 + u); D[v] = gld(A1 + u);
                    if (c > 0) { mum[v] = gld(A0 + u - 1); Dm[v] = gld(A1 + u - 1); }
                    ne[v] = gld(U.ne + u); ph[v] = gld(U.phi + u); sr[v] = gld(U.src + u);
                    if (U.kloss) kl[v] = gld(U.kloss + u);
                    qq[v] = gld(U.q + u);
                    if (extrap) { pn[v] = gld(U.ne_prev + u); pp[v] = gld(U.phi_prev + u); }
                    if (learn) { ln[v] = gld(U.ne_learn + u); lp[v] = gld(U.phi_learn + u); }
                    if (prm.has_u) uf[v] = gld(U.uface + fo + c);
                }
            }
#pragma unroll
            for (int v = 0; v < UC; ++v) {
                const int k = k0 + v * nw;
                int tt, j;
                tile_cell(k, tt, j);
                const int c = tt * M + j;
                if (k >= ke || j >= M) continue;
                const int64_t s = cd.ws + (int64_t)j * T + tt;
                if (c >= n) {
                    gst(W.fa + s, (double)(0.0)); gst(W.fg + s, (double)(0.0));
                    if (prm.has_u) gst(W.fw + s, (double)(0.0));
                    gst(W.f + s, (double)(0.0)); gst(W.kd + s, (double)(0.0)); gst(W.q + s, (double)(0.0));
                    X00[s] = X01[s] = X10[s] = X11[s] = X20[s] = X21[s] = 0.0;
                    continue;
                }
                // the problem's domain: mu >= 0, D > 0 (table: c finite, N > 0),
                // k >= 0, all values finite (the comparisons are false for NaN)
                const bool ok = (TAB ? fabs(mu[v]) < INFINITY : mu[v] >= 0.0 && mu[v] < INFINITY) &&
                                D[v] > 0.0 && D[v] < INFINITY &&
                                kl[v] >= 0.0 && kl[v] < INFINITY && fabs(sr[v]) < INFINITY &&
                                fabs(qq[v]) < INFINITY && fabs(ne[v]) < INFINITY && fabs(ph[v]) < INFINITY &&
                                fabs(uf[v]) < INFINITY;
                bad = bad || !ok;
                double r, g, wf = 0.0;
                if constexpr (TAB) {
                    // the face record (mean c, mean N (0: zero-flux wall), u_f h_f)
                    if (c == 0) {
                        r = mu[v];
                        g = (cd.bcl == 1) ? 0.0 : D[v];
                        if (prm.has_u) wf = uf[v] * hb;
                    } else {
                        r = 0.5 * (mum[v] + mu[v]);
                        g = 0.5 * (Dm[v] + D[v]);
                        if (prm.has_u) wf = uf[v] * cd.h;
                    }
                } else if (c == 0) {
                    r = mu[v] / D[v];
                    g = (cd.bcl == 1) ? 0.0 : D[v] / hb;
                    if (prm.has_u) wf = uf[v] * hb / D[v];
                } else {
                    const double muf = 0.5 * (mum[v] + mu[v]);
                    const double Df = 0.5 * (Dm[v] + D[v]);
                    r = muf / Df;
                    g = Df / cd.h;
                    if (prm.has_u) wf = uf[v] * cd.h / Df;
                }
                // coefficients equal to the stored ones (bit for bit) are not
                // written again
                const bool same = may_reuse && ofa[v] == r && ofg[v] == g && okd[v] == dt * kl[v] &&
                                  (!prm.has_u || ofw[v] == wf);
                changed = changed || (may_reuse && !same);
                if (!same) {
                    gst(W.fa + s, (double)(r)); gst(W.fg + s, (double)(g));
                    if (prm.has_u) gst(W.fw + s, (double)(wf));
                    gst(W.kd + s, (double)(dt * kl[v]));
                }
                gst(W.f + s, (double)(ne[v] + dt * sr[v]));
                gst(W.q + s, (double)(qq[v]));
                X00[s] = ne[v]; X01[s] = ph[v];
                if (extrap) { X10[s] = 2.0 * ne[v] - pn[v]; X11[s] = 2.0 * ph[v] - pp[v]; }
                if (learn) { X20[s] = ln[v]; X21[s] = lp[v]; }
                if (c == n - 1) {
                    // right wall face: the last cell's mu and D at distance h/2
                    const double uR = prm.has_u ? gld(U.uface + fo + n) : 0.0;
                    bad = bad || !(fabs(uR) < INFINITY);
                    if constexpr (TAB) {
                        wall[0] = mu[v];
                        wall[1] = (cd.bcr == 1) ? 0.0 : D[v];
                        wall[2] = uR * hb;
                    } else {
                        wall[0] = mu[v] / D[v];
                        wall[1] = (cd.bcr == 1) ? 0.0 : D[v] / hb;
                        wall[2] = uR * hb / D[v];
                    }
                }
            }
        }
        return (changed ? kGatherChanged : 0) | (bad ? kGatherBad : 0);
    }

    // Workspace buffer -> caller arrays (natural layout), tiles [kb, ke) of
    // gather in the other direction.
    __device__ void scatter(CP s0p, CP s1p, double* o0, double* o1, int kb, int ke,
                            int w, int nw) {
        const int M = cd.M, n = cd.n;
        const int lane = threadIdx.x & 63;
        const int nrg = (M + 7) >> 3;
        constexpr int UC = 4;
        for (int k0 = kb + w; k0 < ke; k0 += UC * nw) {
            double a[UC], b[UC];
#pragma unroll
            for (int v = 0; v < UC; ++v) {
                const int k = k0 + v * nw;
                const int tt = (k / nrg) * 8 + (lane >> 3);
                const int j = (k % nrg) * 8 + (lane & 7);
                a[v] = b[v] = 0.0;
                if (k < ke && j < M && tt * M + j < n) {
                    const int64_t s = cd.ws + (int64_t)j * T + tt;
                    a[v] = s0p[s]; b[v] = s1p[s];
                }
            }
#pragma unroll
            for (int v = 0; v < UC; ++v) {
                const int k = k0 + v * nw;
                const int tt = (k / nrg) * 8 + (lane >> 3);
                const int j = (k % nrg) * 8 + (lane & 7);
                const int c = tt * M + j;
                if (k < ke && j < M && c < n) {
                    gst(o0 + cd.uoff + c, a[v]);
                    gst(o1 + cd.uoff + c, b[v]);
                }
            }
        }
    }

    // Start of a step: gather (unless separate launches already gathered
    // this column: then its wall coefficients sit in the column's ColState
    // and the change flags of its gather workgroups in W.gflag[g0, g0 + gn)),
    // scalings, residuals of the start candidates.
    __device__ Norms setup(const UserArrays& U, int* cur, int* guess_used, bool gathered = false) {
        const CP X00 = xb(0, 0); const CP X01 = xb(0, 1);
        const CP X10 = xb(1, 0); const CP X11 = xb(1, 1);
        const CP X20 = xb(2, 0); const CP X21 = xb(2, 1);
        const bool extrap = prm.guess >= 1 && prm.has_prev;
        const bool learn = prm.guess == 2 && prm.has_learned && W.lmask[cd.index] != 0;
        // the previous step's record of this column (read before it is rewritten)
        const ColState* csp = W.cst + cd.index;
        const bool may_reuse = prm.fac_reuse && csp->fac_valid;
        const double o_rR = csp->rR, o_gR = csp->gR, o_wR = csp->wR;
        const double o_sf[4] = {csp->fsfn, csp->fsfp, csp->fsxn, csp->fsxp};
        bool changed;    // a Jacobian coefficient of this thread's cells differs
        bool bad = false;
        if (gathered) {
            rR = csp->nrR; gR = csp->ngR; wR = csp->nwR;
            changed = false;
            for (int i = cd.g0; i < cd.g0 + cd.gn; ++i) {
                changed = changed || (W.gflag[i] & kGatherChanged) != 0;
                bad = bad || (W.gflag[i] & kGatherBad) != 0;
            }
        } else {
            const int gm = gather(U, 0, ntiles(), t >> 6, T / 64, (double*)(lds + Lds<T>::kMisc));
            changed = (gm & kGatherChanged) != 0;
            double bb[1] = {(gm & kGatherBad) ? 1.0 : 0.0};
            wg_max<T, 1>(bb, lds + Lds<T>::kScr);   // its barriers also publish the wall values
            bad = bb[0] != 0.0;
            const ldbl* misc = lds + Lds<T>::kMisc;
            rR = misc[0]; gR = misc[1]; wR = misc[2];
            __syncthreads();
        }
        if (bad) {
            // an input outside the problem's domain: no iteration; X^n stays
            bad_input = true;
            *cur = 0;
            *guess_used = 0;
            if (t == 0) {
                ColState* cs = W.cst + cd.index;
                cs->sfn = cs->sfp = cs->sxn = cs->sxp = 1.0;
                cs->fac_valid = 0;
                cs->mg_cycles = 0;
            }
            Norms r;
            r.rinf = NAN; r.r2 = NAN; r.xn2 = 0.0; r.step = INFINITY;
            return r;
        }

        // Sweep A: scalings from X^n (term magnitudes) + residual at X^n, and
        // in the same pass the residual of the extrapolated candidate.
        struct ScRec { double gam, grd, mag; };
        // te, tp, |n|, |q|, |phi|, then max|Fe|, max|Fp| of X^n and of the extrapolation
        double mx[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        // sums Fe^2, Fp^2, n^2, phi^2 of X^n, then of the extrapolation
        double sm[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        {
            const double dt_h = dth, eps_h = epsh;
            const CP F0 = Fb(0, 0); const CP F1 = Fb(0, 1);
            const CP E0 = Fb(1, 0); const CP E1 = Fb(1, 1);
            struct Own { double f, k, q; };
            const TabRef tb = prm.tab;
            const auto scface = [tb](double fa, double fb, double fc, double ihf, double nA, double pA, double nB,
                                     double pB) {
                double r, g, w;
                face_rgw<TAB>(tb, fa, fb, fc, ihf, pB - pA, r, g, w);
                const double pe = w + r * (pB - pA);
                double bx, bmx;
                bernoulli_pair(pe, bx, bmx);
                ScRec o;
                o.gam = g * (bmx * nA - bx * nB);
                o.grd = (pB - pA) * ihf;
                o.mag = g * (bmx * fabs(nA) + bx * fabs(nB));
                return o;
            };
            const auto own = [&](int64_t s) { return Own{gld(W.f + s), gld(W.kd + s), gld(W.q + s)}; };
            const auto cellA = [&](int64_t s, double nC, double pC, const ScRec& L, const ScRec& R, const Own& o) {
                const double fv = o.f, kv = o.k, qv = o.q;
                const double fe = -nC + fv - kv * nC - dt_h * (R.gam - L.gam);
                const double fp = -nC + qv + eps_h * (R.grd - L.grd);
                F0[s] = fe; F1[s] = fp;
                const double te = fabs(fv) + kv * fabs(nC) + dt_h * (L.mag + R.mag);
                const double tp = fabs(nC) + fabs(qv) + eps_h * (fabs(L.grd) + fabs(R.grd));
                mx[0] = fmax(mx[0], te);
                mx[1] = fmax(mx[1], tp);
                mx[2] = fmax(mx[2], fabs(nC));
                mx[3] = fmax(mx[3], fabs(qv));
                mx[4] = fmax(mx[4], fabs(pC));
                mx[5] = fmax(mx[5], fabs(fe));
                mx[6] = fmax(mx[6], fabs(fp));
                sm[0] += fe * fe; sm[1] += fp * fp;
                sm[2] += nC * nC; sm[3] += pC * pC;
            };
            if (extrap) {
                sweep2<4, ScRec, FluxRec>(
                    [&](int64_t s, double& a, double& b) { a = X00[s]; b = X01[s]; },
                    [&](int64_t s, double& a, double& b) { a = X10[s]; b = X11[s]; },
                    scface, FluxFace{prm.tab}, own,
                    [&](int64_t s, int c, double nC, double pC, double nE, double pE, const ScRec& L,
                        const ScRec& R, const FluxRec& LE, const FluxRec& RE, const Own& o) {
                        cellA(s, nC, pC, L, R, o);
                        const double fe = -nE + o.f - o.k * nE - dt_h * (RE.gam - LE.gam);
                        const double fp = -nE + o.q + eps_h * (RE.grd - LE.grd);
                        E0[s] = fe; E1[s] = fp;
                        mx[7] = fmax(mx[7], fabs(fe));
                        mx[8] = fmax(mx[8], fabs(fp));
                        sm[4] += fe * fe; sm[5] += fp * fp;
                        sm[6] += nE * nE; sm[7] += pE * pE;
                    },
                    [&](int64_t s) { F0[s] = 0.0; F1[s] = 0.0; E0[s] = 0.0; E1[s] = 0.0; });
            } else {
                sweep<2, ScRec>(
                    [&](int64_t s, double& a, double& b) { a = X00[s]; b = X01[s]; },
                    scface, own,
                    [&](int64_t s, int c, double nC, double pC, const ScRec& L, const ScRec& R, const Own& o) {
                        cellA(s, nC, pC, L, R, o);
                    },
                    [&](int64_t s) { F0[s] = 0.0; F1[s] = 0.0; });
            }
        }
        ldbl* scr = lds + Lds<T>::kScr;
        wg_max<T, 9>(mx, scr);
        wg_sum<T, 8>(sm, scr);
        const double mr[2] = {mx[5], mx[6]};
        sfn = mx[0];
        sfp = mx[1];
        sxn = fmax(1.0, fmax(mx[2], mx[3]));
        sxp = fmax(1.0, fmax(mx[4], fmax(fabs(cd.phil), fabs(cd.phir))));
        // an all-zero column (no terms at all) keeps unit scales
        if (!(sfn > 0.0)) sfn = 1.0;
        if (!(sfp > 0.0)) sfp = 1.0;
        isfn = 1.0 / sfn;
        isfp = 1.0 / sfp;
        Norms best;
        best.rinf = fmax(mr[0] * isfn, mr[1] * isfp);
        best.r2 = sqrt(sm[0] * isfn * isfn + sm[1] * isfp * isfp);
        best.xn2 = sm[2] / (sxn * sxn) + sm[3] / (sxp * sxp);
        best.step = INFINITY;
        if (isnan(sm[0]) || isnan(sm[1])) best.r2 = NAN;
        *cur = 0;
        *guess_used = 0;
        const VecRef none{CP{nullptr}, CP{nullptr}, 0.0, 0.0};
        if (extrap) {
            Norms e;
            e.rinf = fmax(mx[7] * isfn, mx[8] * isfp);
            e.r2 = sqrt(sm[4] * isfn * isfn + sm[5] * isfp * isfp);
            e.xn2 = sm[6] / (sxn * sxn) + sm[7] / (sxp * sxp);
            if (isnan(sm[4]) || isnan(sm[5])) e.r2 = NAN;
            e.step = INFINITY;
            // X^n or the extrapolation, whichever has the smaller scaled
            // residual (ties to the extrapolation): after a sharp transient the
            // extrapolated state can lie outside Newton's basin
            if (!isnan(e.r2) && (isnan(best.r2) || e.rinf <= best.rinf)) {
                best = e; *cur = 1; *guess_used = 1;
            }
        }
        // factors of the previous step stay usable (as a lagged preconditioner
        // and for the error estimate) when the Jacobian coefficients are the
        // same and the scalings moved by less than 1 %
        {
            double ch[1] = {changed ? 1.0 : 0.0};
            wg_max<T, 1>(ch, scr);
            const double nsf[4] = {sfn, sfp, sxn, sxp};
            bool ok = may_reuse && ch[0] == 0.0 && rR == o_rR && gR == o_gR && wR == o_wR;
            for (int k = 0; k < 4 && ok; ++k) ok = o_sf[k] > 0.0 && fabs(nsf[k] / o_sf[k] - 1.0) < 1e-2;
            fac_reuse = ok;
        }
        if (learn) {
            Norms l = residual([&](int64_t s, double& a, double& b) { a = X20[s]; b = X21[s]; },
                               Fb(2, 0), Fb(2, 1), CP{nullptr}, CP{nullptr}, none, 0.0);
            l.step = INFINITY;
            // fallback rule: the learned guess must beat the plain one strictly
            if (!isnan(l.r2) && (isnan(best.r2) || l.rinf < best.rinf)) {
                best = l; *cur = 2; *guess_used = 2;
            }
        }
        if (t == 0) {
            ColState* cs = W.cst + cd.index;
            cs->sfn = sfn; cs->sfp = sfp; cs->sxn = sxn; cs->sxp = sxp;
            cs->rR = rR; cs->gR = gR; cs->wR = wR;
            cs->mg_cycles = 0;
        }
        return best;
    }

    // restore scalars kept in ColState (host-driven mode re-enters per phase)
    __device__ void load_state() {
        const ColState* cs = W.cst + cd.index;
        sfn = cs->sfn; sfp = cs->sfp; sxn = cs->sxn; sxp = cs->sxp;
        isfn = 1.0 / sfn; isfp = 1.0 / sfp;
        rR = cs->rR; gR = cs->gR; wR = cs->wR;
    }

    // ------------------------------------------------------------------
    // Jacobian assembly + factorisation (FP64 arithmetic; per-cell factors
    // stored in FT; the reduced per-chunk system's rows kept in FP64, and
    // eliminated by each apply).
    // Rows of chunk t: row 0 is the chunk's interface unknown x0(t); rows
    // j >= 1 are eliminated by block LU of the chunk's interior with x0(t)
    // and x0(t+1) as boundary values:
    //   m_j = (B_j - A_j g_{j-1})^-1,  g_j = m_j C_j,
    //   a_1 = m_1 A_1,  a_j = -m_j A_j a_{j-1}     (response to x0(t)),
    //   d_j = m_j v_j - m_j A_j d_{j-1},
    //   x_j = d_j - a_j x0(t) - g_j x_{j+1}        (x_M = x0(t+1)).
    // The interface system needs only the chunk's end rows of the spikes
    // x_j = d''_j - a''_j x0(t) - g''_j x0(t+1): a''_{M-1} = a_{M-1},
    // g''_{M-1} = g_{M-1}, and at row 1, from the back substitution unrolled,
    //   a''_1 = sum_j Q_j a_j,  g''_1 = -Q_M,  d''_1 = sum_j Q_j d_j,
    //   Q_1 = I,  Q_{j+1} = -Q_j g_j,
    // which the forward sweeps accumulate as they go; so the factorisation is
    // one sweep and the apply two (down, then the back substitution).
    // ------------------------------------------------------------------
    struct JacRec { double dnA, dnB, dpB, ihf; };

    // derivatives of the face flux w.r.t. the left (A) and right (B) states
    // (with table transport including the coefficients' own dependence on
    // the face's field)
    struct JacFace {
        TabRef tb;
        __device__ __forceinline__ JacRec operator()(double fa, double fb, double fc, double ihf,
                                                     double nA, double pA, double nB, double pB) const {
            double r, g, w, dr, dg, dw;
            face_rgw_d<TAB>(tb, fa, fb, fc, ihf, pB - pA, r, g, w, dr, dg, dw);
            const double pe = w + r * (pB - pA);
            double bx, bmx, dbx, dbmx;
            bernoulli_pair(pe, bx, bmx);
            bernoulli_dpair(pe, bx, bmx, dbx, dbmx);
            JacRec o;
            o.dnA = g * bmx;
            o.dnB = -g * bx;
            if constexpr (TAB) {
                // the coefficients follow the face's field: d(Gamma)/d(dphi) =
                // dGamma/dpe (r + dphi dr + dw) + dGamma/dg dg
                o.dpB = g * (-dbmx * nA - dbx * nB) * (r + (pB - pA) * dr + dw) + (bmx * nA - bx * nB) * dg;
            } else {
                o.dpB = g * r * (-dbmx * nA - dbx * nB);
            }
            o.ihf = ihf;
            return o;
        }
    };

    __device__ __forceinline__ void store_blk(int slot, int64_t s, const Blk<double>& m) {
        gst((V4<FT>*)facp(slot, s), V4<FT>{(FT)m.a, (FT)m.b, (FT)m.c, (FT)m.d});
    }
    __device__ __forceinline__ Blk<FT> load_blk(int slot, int64_t s) const {
        const V4<FT> r = gld((const V4<FT>*)facp(slot, s));
        return {r.a, r.b, r.c, r.d};
    }

    __device__ void factor(int cur) {
        if (prm.prec_kind == 2) {
            // no preconditioner: nothing to factor
            if (t == 0) {
                ColState* cs = W.cst + cd.index;
                cs->fac_valid = 1;
                cs->fsfn = sfn; cs->fsfp = sfp; cs->fsxn = sxn; cs->fsxp = sxp;
            }
            __syncthreads();
            return;
        }
        {
            Column self(*this);
            self.factor_chunks(cur);
        }
        if (prm.prec_kind == 3) mg_build();
        __syncthreads();
    }

    // the factorisation proper (block preconditioners)
    __device__ __forceinline__ void factor_chunks(int cur) {
        const int M = cd.M, n = cd.n;
        const int c0 = t * M;
        const CP X0 = xb(cur, 0);
        const CP X1 = xb(cur, 1);
        const double dt_h = dth, eps_h = epsh;
        // scale factors of the four block entries
        const double s_en = isfn * sxn, s_ep = isfn * sxp, s_pn = isfp * sxn, s_pp = isfp * sxp;
        Blk<double> A0 = bzero(), B0 = beye(), C0 = bzero();
        Blk<double> gprev = bzero(), aprev = bzero();
        Blk<double> Q = beye(), a1 = bzero();     // Q_j and the partial sum of a''_1

        auto rowproc = [&](int j, int64_t s, const Blk<double>& A, const Blk<double>& B,
                           const Blk<double>& C) {
            if (j == 0) { A0 = A; B0 = B; C0 = C; return; }
            Blk<double> m, al;
            if (j == 1) {
                m = binv(B);
                al = bmul(m, A);
            } else {
                m = binv(bsub(B, bmul(A, gprev)));
                al = bneg(bmul(m, bmul(A, aprev)));
            }
            const Blk<double> ga = bmul(m, C);
            store_blk(0, s, m);
            store_blk(4, s, bmul(m, A));
            store_blk(8, s, ga);
            store_blk(12, s, al);
            const Blk<double> qa = bmul(Q, al);
            a1 = Blk<double>{a1.a + qa.a, a1.b + qa.b, a1.c + qa.c, a1.d + qa.d};
            Q = bneg(bmul(Q, ga));
            gprev = ga; aprev = al;
        };

        sweep<2, JacRec>(
            [&](int64_t s, double& a, double& b) { a = X0[s]; b = X1[s]; },
            JacFace{prm.tab},
            [&](int64_t s) { return gld(W.kd + s); },
            [&](int64_t s, int c, double nC, double pC, const JacRec& L, const JacRec& R, const double& kv) {
                const int j = c - c0;
                Blk<double> A, B, C;
                B.a = (-1.0 - kv - dt_h * (R.dnA - L.dnB)) * s_en;
                B.b = (dt_h * (R.dpB + L.dpB)) * s_ep;
                B.c = -1.0 * s_pn;
                B.d = (-eps_h * (R.ihf + L.ihf)) * s_pp;
                if (c > 0) {
                    A.a = dt_h * L.dnA * s_en;
                    A.b = -dt_h * L.dpB * s_ep;
                    A.c = 0.0;
                    A.d = eps_h * L.ihf * s_pp;
                } else {
                    A = bzero();
                }
                if (c < n - 1) {
                    C.a = -dt_h * R.dnB * s_en;
                    C.b = -dt_h * R.dpB * s_ep;
                    C.c = 0.0;
                    C.d = eps_h * R.ihf * s_pp;
                } else {
                    C = bzero();
                }
                if (prm.prec_kind == 1 || prm.prec_kind == 3) {
                    // eq:prec_recast: keep the couplings dt D_r (row of F_e in phi)
                    // and I_e (F_phi in n, diagonal) for the apply, and factor
                    // diag(dt D_f - I, S~) with S~ = L + I_e dt D_r, the Schur
                    // complement with (dt D_f - I)^-1 replaced by -I (scaled units:
                    // -(s_Fn / s_Xn) I)
                    gst((V4<FT>*)facp(16, s), V4<FT>{(FT)A.b, (FT)B.b, (FT)C.b, (FT)B.c});
                    const double kap = B.c / s_en;
                    A = Blk<double>{A.a, 0.0, 0.0, A.d + kap * A.b};
                    C = Blk<double>{C.a, 0.0, 0.0, C.d + kap * C.b};
                    B = Blk<double>{B.a, 0.0, 0.0, B.d + kap * B.b};
                    if (prm.prec_kind == 3) {
                        // the two scalar tridiagonal blocks on the multigrid's finest level
                        gst(mgf(0) + c, A.a); gst(mgf(1) + c, B.a); gst(mgf(2) + c, C.a);
                        gst(mgf(3) + c, A.d); gst(mgf(4) + c, B.d); gst(mgf(5) + c, C.d);
                    }
                }
                rowproc(j, s, A, B, C);
            },
            [&](int64_t s) {
                const int j = (int)((s - cd.ws) / T);
                if (prm.prec_kind == 1 || prm.prec_kind == 3) {
                    gst((V4<FT>*)facp(16, s), V4<FT>{FT(0), FT(0), FT(0), FT(0)});
                }
                rowproc(j, s, bzero(), beye(), bzero());
            });

        // the spikes' end rows (a chunk of one row has no interior: x_1 is
        // x0(t+1) itself)
        Blk<double> g1 = bneg(Q), aL = bneg(beye()), gL = bzero();
        if (M >= 2) {
            aL = aprev; gL = gprev;
        }
        // reduced system row of chunk t
        ldbl* P = lds + Lds<T>::kPcr;
        __syncthreads();
        P[8 * t + 0] = aL.a; P[8 * t + 1] = aL.b; P[8 * t + 2] = aL.c; P[8 * t + 3] = aL.d;
        P[8 * t + 4] = gL.a; P[8 * t + 5] = gL.b; P[8 * t + 6] = gL.c; P[8 * t + 7] = gL.d;
        __syncthreads();
        Blk<double> aLp = bzero(), gLp = bzero();
        if (t > 0) {
            aLp = {P[8 * (t - 1) + 0], P[8 * (t - 1) + 1], P[8 * (t - 1) + 2], P[8 * (t - 1) + 3]};
            gLp = {P[8 * (t - 1) + 4], P[8 * (t - 1) + 5], P[8 * (t - 1) + 6], P[8 * (t - 1) + 7]};
        }
        Blk<double> Lr = bneg(bmul(A0, aLp));
        Blk<double> Dr = bsub(bsub(B0, bmul(A0, gLp)), bmul(C0, a1));
        Blk<double> Ur = bneg(bmul(C0, g1));
        // red(k) = rb + k T: A0, C0 and the chunk's row (L, D, U) of the
        // interface system; each apply eliminates it by parallel cyclic
        // reduction together with its right-hand side
        double* const rb = W.red + cd.red + t;
        const double rv[20] = {A0.a, A0.b, A0.c, A0.d, C0.a, C0.b, C0.c, C0.d, Lr.a, Lr.b, Lr.c, Lr.d,
                               Dr.a, Dr.b, Dr.c, Dr.d, Ur.a, Ur.b, Ur.c, Ur.d};
#pragma unroll
        for (int k = 0; k < 20; ++k) gst(rb + (int64_t)k * T, rv[k]);
        if (t == 0) {
            ColState* cs = W.cst + cd.index;
            cs->fac_valid = 1;
            cs->fsfn = sfn; cs->fsfp = sfp; cs->fsxn = sxn; cs->fsxp = sxp;
        }
    }

    // ------------------------------------------------------------------
    // Multigrid V-cycles for the two scalar tridiagonal blocks of the
    // approximate Schur preconditioner (eq:prec_recast), as the paper solves
    // them (Section 3.2): vertex-centred coarsening by two (coarse point I is
    // fine point 2I), linear interpolation P, Galerkin coarse operators
    // P^T A P (tridiagonal again in 1D), restriction P^T, two red-black
    // Gauss-Seidel sweeps before and after each coarse correction, a direct
    // solve on a level of at most kMgCoarse points.  Natural-layout arrays of
    // this column (level l + 1 follows level l), field k of mgf(k): 0-2 the
    // electron block's sub-, main and super-diagonal, 3-5 those of S~, 6 the
    // iterate, 7 the right-hand side, 8 the residual.
    // ------------------------------------------------------------------
    static constexpr int kMgMaxLevels = 32;   // ceil(n / 2^31) <= kMgCoarse for any int n

    __device__ __forceinline__ double* mgf(int k) const {
        return W.mg + (int64_t)k * W.mgP + 2 * cd.ws + 64 * (int64_t)cd.index;
    }
    // level sizes and offsets; returns the number of levels
    __device__ int mg_shape(int* len, int* off) const {
        int L = 0, n = cd.n, o = 0;
        for (;;) {
            len[L] = n; off[L] = o; ++L;
            if (n <= kMgCoarse || L == kMgMaxLevels) break;
            o += n;
            n = (n + 1) >> 1;
        }
        return L;
    }
    // Interpolation weights of odd fine point i (between coarse points i/2
    // and i/2 + 1) on a level with rows (a, b, c) and nc coarse points:
    // linear (1/2, 1/2), or matrix-dependent (-a_i/b_i, -c_i/b_i: the value
    // row i of the operator gives from its two neighbours, de Zeeuw's
    // black-box transfer).  The right weight is 0 past the last coarse point.
    __device__ static __forceinline__ void mg_w(const double* a, const double* b, const double* c, int i, int nc,
                                                bool md, double& wl, double& wr) {
        if (md) { wl = -a[i] / b[i]; wr = -c[i] / b[i]; }
        else { wl = 0.5; wr = 0.5; }
        if ((i >> 1) + 1 >= nc) wr = 0.0;
    }
    // weight of coarse point J in the interpolated value at fine point k
    __device__ static __forceinline__ double mg_p(const double* a, const double* b, const double* c, int k, int J,
                                                  int nf, int nc, bool md) {
        if (k < 0 || k >= nf) return 0.0;
        if ((k & 1) == 0) return k == 2 * J ? 1.0 : 0.0;
        double wl, wr;
        mg_w(a, b, c, k, nc, md, wl, wr);
        return (k >> 1) == J ? wl : ((k >> 1) + 1 == J ? wr : 0.0);
    }
    __device__ void mg_build() {
        int len[kMgMaxLevels], off[kMgMaxLevels];
        const int L = mg_shape(len, off);
        for (int l = 0; l + 1 < L; ++l) {
            const int nf = len[l], nc = len[l + 1];
            __syncthreads();
            for (int blk = 0; blk < 2; ++blk) {
                const bool md = (prm.mg_transfer >> blk) & 1;
                const double* fa = mgf(3 * blk) + off[l];
                const double* fb = mgf(3 * blk + 1) + off[l];
                const double* fc = mgf(3 * blk + 2) + off[l];
                double* ca = mgf(3 * blk) + off[l + 1];
                double* cb = mgf(3 * blk + 1) + off[l + 1];
                double* cc = mgf(3 * blk + 2) + off[l + 1];
                // Galerkin: A_c[I][J] = sum_i P[i][I] (A P e_J)[i], rows i = 2I - 1 .. 2I + 1
                for (int I = t; I < nc; I += T) {
                    double e[3];
                    for (int d = -1; d <= 1; ++d) {
                        const int J = I + d;
                        double acc = 0.0;
                        if (J >= 0 && J < nc) {
                            for (int k = -1; k <= 1; ++k) {
                                const int i = 2 * I + k;
                                if (i < 0 || i >= nf) continue;
                                const double ap = (i > 0 ? fa[i] * mg_p(fa, fb, fc, i - 1, J, nf, nc, md) : 0.0) +
                                                  fb[i] * mg_p(fa, fb, fc, i, J, nf, nc, md) +
                                                  (i + 1 < nf ? fc[i] * mg_p(fa, fb, fc, i + 1, J, nf, nc, md) : 0.0);
                                acc += mg_p(fa, fb, fc, i, I, nf, nc, md) * ap;
                            }
                        }
                        e[d + 1] = acc;
                    }
                    ca[I] = e[0]; cb[I] = e[1]; cc[I] = e[2];
                }
            }
        }
        __syncthreads();
    }
    // nu red-black Gauss-Seidel sweeps on one level
    __device__ void mg_smooth(const double* a, const double* b, const double* c, double* x, const double* f,
                              int n, int nu) {
        for (int sw = 0; sw < nu; ++sw)
            for (int color = 0; color < 2; ++color) {
                for (int i = 2 * t + color; i < n; i += 2 * T) {
                    double r = f[i];
                    if (i > 0) r -= a[i] * x[i - 1];
                    if (i + 1 < n) r -= c[i] * x[i + 1];
                    x[i] = r / b[i];
                }
                __syncthreads();
            }
    }
    // one V-cycle for block blk from the iterate on level 0
    __device__ void mg_vcycle(int blk, const int* len, const int* off, int L) {
        double* X = mgf(6);
        double* Fr = mgf(7);
        double* R = mgf(8);
        const double* A = mgf(3 * blk);
        const double* B = mgf(3 * blk + 1);
        const double* C = mgf(3 * blk + 2);
        const bool md = (prm.mg_transfer >> blk) & 1;
        for (int l = 0; l + 1 < L; ++l) {
            const int n = len[l], o = off[l], nc = len[l + 1], oc = off[l + 1];
            mg_smooth(A + o, B + o, C + o, X + o, Fr + o, n, 2);
            for (int i = t; i < n; i += T) {
                double r = Fr[o + i] - B[o + i] * X[o + i];
                if (i > 0) r -= A[o + i] * X[o + i - 1];
                if (i + 1 < n) r -= C[o + i] * X[o + i + 1];
                R[o + i] = r;
            }
            __syncthreads();
            // restriction P^T: the coarse point and the odd neighbours' weights on it
            for (int I = t; I < nc; I += T) {
                double fcI = R[o + 2 * I];
                double wl, wr;
                if (2 * I - 1 >= 0) {
                    mg_w(A + o, B + o, C + o, 2 * I - 1, nc, md, wl, wr);
                    fcI += wr * R[o + 2 * I - 1];
                }
                if (2 * I + 1 < n) {
                    mg_w(A + o, B + o, C + o, 2 * I + 1, nc, md, wl, wr);
                    fcI += wl * R[o + 2 * I + 1];
                }
                Fr[oc + I] = fcI;
                X[oc + I] = 0.0;
            }
            __syncthreads();
        }
        {
            // direct solve on the coarsest level (Thomas; the blocks are
            // diagonally dominant M-matrices, no pivoting needed)
            const int n = len[L - 1], o = off[L - 1];
            if (t == 0) {
                double cp[kMgCoarse + 1], dp[kMgCoarse + 1];
                cp[0] = C[o] / B[o];
                dp[0] = Fr[o] / B[o];
                for (int i = 1; i < n; ++i) {
                    const double m = B[o + i] - A[o + i] * cp[i - 1];
                    cp[i] = C[o + i] / m;
                    dp[i] = (Fr[o + i] - A[o + i] * dp[i - 1]) / m;
                }
                X[o + n - 1] = dp[n - 1];
                for (int i = n - 2; i >= 0; --i) X[o + i] = dp[i] - cp[i] * X[o + i + 1];
            }
            __syncthreads();
        }
        for (int l = L - 2; l >= 0; --l) {
            const int n = len[l], o = off[l], nc = len[l + 1], oc = off[l + 1];
            for (int i = t; i < n; i += T) {
                double e;
                if ((i & 1) == 0) {
                    e = X[oc + (i >> 1)];
                } else {
                    double wl, wr;
                    mg_w(A + o, B + o, C + o, i, nc, md, wl, wr);
                    e = wl * X[oc + (i >> 1)] + (wr != 0.0 ? wr * X[oc + (i >> 1) + 1] : 0.0);
                }
                X[o + i] += e;
            }
            __syncthreads();
            mg_smooth(A + o, B + o, C + o, X + o, Fr + o, n, 2);
        }
    }
    // out = A_blk^-1 (rs * rhs) by V-cycles to ||b - A x||_2 <= mg_tol ||b||_2
    // (rhs and out: chunk layout; they may alias)
    __device__ void mg_solve(int blk, CP rhs, double rs, CP out) {
        int len[kMgMaxLevels], off[kMgMaxLevels];
        const int L = mg_shape(len, off);
        const int M = cd.M, n = cd.n;
        double* X = mgf(6);
        double* Fr = mgf(7);
        const double* A = mgf(3 * blk);
        const double* B = mgf(3 * blk + 1);
        const double* C = mgf(3 * blk + 2);
        double bb[1] = {0.0};
        for (int j = 0; j < M; ++j) {
            const int c = t * M + j;
            if (c >= n) break;
            const double v = rhs[sidx(t, j)] * rs;
            Fr[c] = v;
            X[c] = 0.0;
            bb[0] += v * v;
        }
        wg_sum<T, 1>(bb, lds + Lds<T>::kScr);
        int cyc = 0;
        if (bb[0] > 0.0) {
            const double lim = prm.mg_tol * prm.mg_tol * bb[0];
            while (cyc < kMgMaxCycles) {
                mg_vcycle(blk, len, off, L);
                ++cyc;
                double rr[1] = {0.0};
                for (int i = t; i < n; i += T) {
                    double r = Fr[i] - B[i] * X[i];
                    if (i > 0) r -= A[i] * X[i - 1];
                    if (i + 1 < n) r -= C[i] * X[i + 1];
                    rr[0] += r * r;
                }
                wg_sum<T, 1>(rr, lds + Lds<T>::kScr);
                if (rr[0] <= lim) break;
                if (!(rr[0] <= 1e20 * bb[0])) break;   // diverged (or not finite): stop cycling
            }
        }
        for (int j = 0; j < M; ++j) {
            const int c = t * M + j;
            out[sidx(t, j)] = (c < n && cyc > 0) ? X[c] : 0.0;
        }
        if (t == 0) W.cst[cd.index].mg_cycles += cyc;
        __syncthreads();
    }

    // ------------------------------------------------------------------
    // Preconditioner apply z = P^-1 v.  Returns (||z||_2^2, ||z||_inf).
    // v and z must not alias.
    // ------------------------------------------------------------------
    __device__ Vec2<double> apply(const VecRef& v, CP z0, CP z1) {
        if (prm.prec_kind == 2) return apply_identity(v, z0, z1);
        if (prm.prec_kind == 1 || prm.prec_kind == 3) return apply_schur(v, z0, z1);
        Column self(*this);
        const VecRef vl = v;    // by value: a reference would be re-read through a generic pointer
        if (prm.dlds) return self.template block_apply<true>(vl, z0, z1);
        return self.template block_apply<false>(vl, z0, z1);
    }

    // No preconditioner: z = v (with v's component scales), every row of the
    // chunk (padding rows of v hold zeros).
    __device__ Vec2<double> apply_identity(const VecRef& v, CP z0, CP z1) {
        const int M = cd.M;
        double zz = 0.0, zm = 0.0;
        for (int j = 0; j < M; ++j) {
            const int64_t s = sidx(t, j);
            const double a = v.p0[s] * v.s0, b = v.p1[s] * v.s1;
            z0[s] = a;
            z1[s] = b;
            zz += a * a + b * b;
            zm = fmax(zm, fmax(fabs(a), fabs(b)));
        }
        double sm[1] = {zz};
        double mm[1] = {zm};
        wg_sum<T, 1>(sm, lds + Lds<T>::kScr);
        wg_max<T, 1>(mm, lds + Lds<T>::kScr);
        return Vec2<double>{sm[0], mm[0]};
    }

    // Approximate Schur preconditioner, eq:prec_recast applied right to left:
    //   z_e' = (dt D_f - I)^-1 v_e,  z_phi = S~^-1 (v_phi - I_e z_e'),
    //   z_e  = z_e' - (dt D_f - I)^-1 dt D_r z_phi,
    // three solves with the factors of diag(dt D_f - I, S~) (each a pass of
    // the block solver with one component of the right-hand side zero).
    __device__ Vec2<double> apply_schur(const VecRef& v, CP z0, CP z1) {
        const int M = cd.M, n = cd.n;
        const CP Y0 = schb(0), Y1 = schb(1), Y2 = schb(2), Y3 = schb(3);
        // each block solve: exact (the block factorisation with the other
        // component of the right-hand side zero) or by multigrid V-cycles
        const bool mg_n = prm.prec_kind == 3 && (prm.mg_blocks & 1);
        const bool mg_p = prm.prec_kind == 3 && (prm.mg_blocks & 2);
        if (mg_n) mg_solve(0, v.p0, v.s0, Y0);
        else block_apply<false>(VecRef{v.p0, v.p1, v.s0, 0.0}, Y0, Y1);   // Y0 = z_e'
        for (int j = 0; j < M; ++j) {
            const int64_t s = sidx(t, j);
            Y2[s] = v.p1[s] * v.s1 - (double)gld(facp(19, s)) * Y0[s];        // v_phi - I_e z_e'
        }
        if (mg_p) mg_solve(1, Y2, 1.0, z1);
        else block_apply<false>(VecRef{Y2, Y2, 0.0, 1.0}, Y3, z1);         // z1 = z_phi
        // dt D_r z_phi (tridiagonal; neighbours across chunks are visible after
        // the solve's closing barriers)
        for (int j = 0; j < M; ++j) {
            const int64_t s = sidx(t, j);
            const int c = t * M + j;
            double w = 0.0;
            if (c < n) {
                const double zl = c > 0 ? z1[sidx((c - 1) / M, (c - 1) % M)] : 0.0;
                const double zr = c < n - 1 ? z1[sidx((c + 1) / M, (c + 1) % M)] : 0.0;
                w = (double)gld(facp(16, s)) * zl + (double)gld(facp(17, s)) * z1[s] + (double)gld(facp(18, s)) * zr;
            }
            Y2[s] = w;
        }
        if (mg_n) mg_solve(0, Y2, 1.0, Y3);
        else block_apply<false>(VecRef{Y2, Y2, 1.0, 0.0}, Y3, Y1);         // Y3 = (dt D_f - I)^-1 dt D_r z_phi
        double zz = 0.0, zm = 0.0;
        for (int j = 0; j < M; ++j) {
            const int64_t s = sidx(t, j);
            const double ze = Y0[s] - Y3[s];
            z0[s] = ze;
            zz += ze * ze + z1[s] * z1[s];
            zm = fmax(zm, fmax(fabs(ze), fabs(z1[s])));
        }
        double sm[1] = {zz};
        double mm[1] = {zm};
        wg_sum<T, 1>(sm, lds + Lds<T>::kScr);
        wg_max<T, 1>(mm, lds + Lds<T>::kScr);
        return Vec2<double>{sm[0], mm[0]};
    }

    // Block solve with the stored factors (chunk sweeps in FT, reduced
    // system in FP64).  Returns (||z||_2^2, ||z||_inf).  DL: the intermediate
    // d between the two sweeps lives in LDS (row j of this thread at j*T + t
    // past the GMRES state) instead of W.tmp in HBM.
    template <bool DL>
    __device__ __forceinline__ Vec2<double> block_apply(const VecRef& v, CP z0, CP z1) {
        typedef FT dv2 __attribute__((ext_vector_type(2)));
        typedef __attribute__((address_space(3))) dv2 lv2;
        lv2* const dl = (lv2*)(lds + Lds<T>::kDTmp);
        const int tl = t;   // a local: members are reloaded after every barrier
        constexpr int U = 4;
        constexpr int LG = ilog2(T);             // PCR stages of the interface system
        const int M = cd.M;
        // The interface system's row does not depend on v: its loads are
        // issued first, so that their latency overlaps the chunk sweeps.
        double pc[20];
#pragma unroll
        for (int i = 0; i < 20; ++i) pc[i] = gld(red(i));
        Vec2<double> d0{v.p0[sidx(tl, 0)] * v.s0, v.p1[sidx(tl, 0)] * v.s1};
        // down sweep: d_j = m_j v_j - At_j d_{j-1}, and with it d''_1 = sum Q_j d_j
        // (Q_1 = I, Q_{j+1} = -Q_j g_j); loads of U rows issued first.
        // Both sweeps double-buffer their U-row groups: the next group's
        // (unconditional) loads issue before this group's stores, which would
        // otherwise hold them up in the shared in-order memory counter.
        Vec2<FT> dprev{FT(0), FT(0)};
        Vec2<double> dLast{0.0, 0.0}, dFirst{0.0, 0.0};
        if (M >= 2) {
            Blk<FT> Q{FT(1), FT(0), FT(0), FT(1)};
            Vec2<FT> sq{FT(0), FT(0)};
            // 14 values per row: FP64 factors take groups of two rows
            constexpr int UD = sizeof(FT) == 4 ? U : 2;
            struct GD { Blk<FT> mm[UD], aa[UD], gg[UD]; Vec2<FT> vv[UD]; };
            auto load_d = [&](int j0, GD& g) {
#pragma unroll
                for (int u = 0; u < UD; ++u) {
                    const int64_t s = sidx(tl, min(j0 + u, M - 1));
                    g.mm[u] = load_blk(0, s);
                    g.aa[u] = load_blk(4, s);
                    g.gg[u] = load_blk(8, s);
                    g.vv[u] = Vec2<FT>{(FT)(v.p0[s] * v.s0), (FT)(v.p1[s] * v.s1)};
                }
            };
            GD gc, gn;
            load_d(1, gc);
            for (int j0 = 1; j0 < M; j0 += UD) {
                load_d(j0 + UD, gn);
#pragma unroll
                for (int u = 0; u < UD; ++u) {
                    const int j = j0 + u;
                    if (j < M) {
                        const int64_t s = sidx(tl, j);
                        Vec2<FT> de = bmv(gc.mm[u], gc.vv[u]);
                        if (j >= 2) {
                            const Vec2<FT> q = bmv(gc.aa[u], dprev);
                            de.x -= q.x; de.y -= q.y;
                        }
                        if (DL) dl[j * T + tl] = dv2{de.x, de.y};
                        else gst(tmpp(s), V2<FT>{de.x, de.y});
                        dprev = de;
                        const Vec2<FT> qd = bmv(Q, de);
                        sq.x += qd.x; sq.y += qd.y;
                        Q = bneg(bmul(Q, gc.gg[u]));
                    }
                }
                gc = gn;
            }
            dLast = {(double)dprev.x, (double)dprev.y};
            dFirst = {(double)sq.x, (double)sq.y};
        }
        ldbl* P = lds + Lds<T>::kPcr;
        __syncthreads();
        P[2 * tl] = dLast.x; P[2 * tl + 1] = dLast.y;
        __syncthreads();
        Vec2<double> dLp{0.0, 0.0};
        if (tl > 0) dLp = {P[2 * (tl - 1)], P[2 * (tl - 1) + 1]};
        const Blk<double> A0{pc[0], pc[1], pc[2], pc[3]};
        const Blk<double> C0{pc[4], pc[5], pc[6], pc[7]};
        const Vec2<double> qa = bmv(A0, dLp), qc = bmv(C0, dFirst);
        Vec2<double> r{d0.x - qa.x - qc.x, d0.y - qa.y - qc.y};
        // Parallel cyclic reduction (FP64) of the interface system: at stage
        // lv row t eliminates its couplings to rows t -+ 2^lv with
        // k1 = L_t D_{t-s}^-1, k2 = U_t D_{t+s}^-1, from the rows' (L, D, U, r)
        // exchanged through LDS (one array per value: no bank conflicts).
        Blk<double> Lr{pc[8], pc[9], pc[10], pc[11]};
        Blk<double> Dr{pc[12], pc[13], pc[14], pc[15]};
        Blk<double> Ur{pc[16], pc[17], pc[18], pc[19]};
#pragma unroll
        for (int lv = 0; lv < LG; ++lv) {
            const int st = 1 << lv;
            __syncthreads();
            const double w[14] = {Lr.a, Lr.b, Lr.c, Lr.d, Dr.a, Dr.b, Dr.c, Dr.d, Ur.a, Ur.b, Ur.c, Ur.d, r.x, r.y};
#pragma unroll
            for (int k = 0; k < 14; ++k) P[k * T + tl] = w[k];
            __syncthreads();
            Blk<double> k1 = bzero(), k2 = bzero(), Lm = bzero(), Um = bzero(), Lp = bzero(), Up = bzero();
            Vec2<double> rm{0.0, 0.0}, rp{0.0, 0.0};
            if (tl >= st) {
                const ldbl* o = P + (tl - st);
                Lm = {o[0 * T], o[1 * T], o[2 * T], o[3 * T]};
                const Blk<double> Dm{o[4 * T], o[5 * T], o[6 * T], o[7 * T]};
                Um = {o[8 * T], o[9 * T], o[10 * T], o[11 * T]};
                rm = {o[12 * T], o[13 * T]};
                k1 = bmul(Lr, binv(Dm));
            }
            if (tl + st < T) {
                const ldbl* o = P + (tl + st);
                Lp = {o[0 * T], o[1 * T], o[2 * T], o[3 * T]};
                const Blk<double> Dp{o[4 * T], o[5 * T], o[6 * T], o[7 * T]};
                Up = {o[8 * T], o[9 * T], o[10 * T], o[11 * T]};
                rp = {o[12 * T], o[13 * T]};
                k2 = bmul(Ur, binv(Dp));
            }
            Dr = bsub(bsub(Dr, bmul(k1, Um)), bmul(k2, Lp));
            Lr = bneg(bmul(k1, Lm));
            Ur = bneg(bmul(k2, Up));
            const Vec2<double> q1 = bmv(k1, rm), q2 = bmv(k2, rp);
            r.x -= q1.x; r.y -= q1.y;
            r.x -= q2.x; r.y -= q2.y;
        }
        const Vec2<double> x0 = bmv(binv(Dr), r);
        __syncthreads();
        P[2 * tl] = x0.x; P[2 * tl + 1] = x0.y;
        __syncthreads();
        Vec2<double> xn{0.0, 0.0};
        if (tl + 1 < T) xn = {P[2 * (tl + 1)], P[2 * (tl + 1) + 1]};
        double zz = 0.0, zm = 0.0;
        {
            const int64_t s = sidx(tl, 0);
            z0[s] = x0.x; z1[s] = x0.y;
            zz += x0.x * x0.x + x0.y * x0.y;
            zm = fmax(fabs(x0.x), fabs(x0.y));
        }
        // back substitution x_j = d_j - a_j x0(t) - g_j x_{j+1}, rows M-1 .. 1,
        // carried in FP64 from x_M = x0(t+1)
        if (M >= 2) {
            struct GF { Blk<FT> aa[U], gg[U]; Vec2<FT> dd[U]; };
            auto load_f = [&](int j0, GF& g) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int jj = max(j0 - u, 1);
                    const int64_t s = sidx(tl, jj);
                    g.aa[u] = load_blk(12, s);
                    g.gg[u] = load_blk(8, s);
                    if (DL) {
                        const dv2 r = dl[jj * T + tl];
                        g.dd[u] = Vec2<FT>{r.x, r.y};
                    } else {
                        const V2<FT> r = gld(tmpp(s));
                        g.dd[u] = Vec2<FT>{r.x, r.y};
                    }
                }
            };
            GF gc, gn;
            load_f(M - 1, gc);
            Vec2<double> xr = xn;
            for (int j0 = M - 1; j0 >= 1; j0 -= U) {
                load_f(j0 - U, gn);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int j = j0 - u;
                    if (j >= 1) {
                        const int64_t s = sidx(tl, j);
                        const Blk<FT> a = gc.aa[u], g = gc.gg[u];
                        const double zx = (double)gc.dd[u].x - ((double)a.a * x0.x + (double)a.b * x0.y) -
                                          ((double)g.a * xr.x + (double)g.b * xr.y);
                        const double zy = (double)gc.dd[u].y - ((double)a.c * x0.x + (double)a.d * x0.y) -
                                          ((double)g.c * xr.x + (double)g.d * xr.y);
                        z0[s] = zx; z1[s] = zy;
                        zz += zx * zx + zy * zy;
                        zm = fmax(zm, fmax(fabs(zx), fabs(zy)));
                        xr = {zx, zy};
                    }
                }
                gc = gn;
            }
        }
        double sm[1] = {zz};
        double mm[1] = {zm};
        wg_sum<T, 1>(sm, lds + Lds<T>::kScr);
        wg_max<T, 1>(mm, lds + Lds<T>::kScr);
        return Vec2<double>{sm[0], mm[0]};
    }

    // ------------------------------------------------------------------
    // Finite-difference product w = S_F^-1 [F(X + eps S_X z) - F(X)] / eps,
    // written to (w0, w1), fused with up to 8 dot products against basis
    // vectors and ||w||^2 (dots[nb] on return).
    // ------------------------------------------------------------------
    template <class BP>
    __device__ void jv(int cur, const VecRef& z, double eps, CP w0, CP w1,
                       BP basis, int nb, double* dots) {
        Column self(*this);
        const VecRef zl = z;
        self.jv_body(cur, zl, eps, w0, w1, basis, nb, dots);
    }
    template <class BP>
    __device__ __forceinline__ void jv_body(int cur, const VecRef& z, double eps, CP w0, CP w1,
                                            BP basis, int nb, double* dots) {
        const CP X0 = xb(cur, 0);
        const CP X1 = xb(cur, 1);
        const CP F0 = Fb(cur, 0);
        const CP F1 = Fb(cur, 1);
        const double e0 = eps * sxn * z.s0, e1 = eps * sxp * z.s1;
        const double c0 = isfn / eps, c1 = isfp / eps;
        const double dt_h = dth, eps_h = epsh;
        double acc[3] = {0.0, 0.0, 0.0};
        const int nbf = nb < 2 ? nb : 2;
        const VecRef b0 = nbf > 0 ? basis[0] : VecRef{F0, F1, 0.0, 0.0};
        const VecRef b1 = nbf > 1 ? basis[1] : VecRef{F0, F1, 0.0, 0.0};
        struct Own { double f, k, q, F0, F1, v00, v01, v10, v11; };
        sweep<2, FluxRec>(
            [&](int64_t s, double& a, double& b) { a = X0[s] + e0 * z.p0[s]; b = X1[s] + e1 * z.p1[s]; },
            FluxFace{prm.tab},
            [&](int64_t s) {
                Own o;
                o.f = gld(W.f + s); o.k = gld(W.kd + s); o.q = gld(W.q + s); o.F0 = F0[s]; o.F1 = F1[s];
                const Vec2<double> e0 = ld_pair(b0, s), e1 = ld_pair(b1, s);
                o.v00 = e0.x; o.v01 = e0.y;
                o.v10 = e1.x;                // b1 is a valid array for any nb; its dot
                o.v11 = e1.y;                // is used only when nb > 1
                return o;
            },
            [&](int64_t s, int c, double nC, double pC, const FluxRec& L, const FluxRec& R, const Own& o) {
                const double fe = -nC + o.f - o.k * nC - dt_h * (R.gam - L.gam);
                const double fp = -nC + o.q + eps_h * (R.grd - L.grd);
                const double a = (fe - o.F0) * c0;
                const double b = (fp - o.F1) * c1;
                w0[s] = a; w1[s] = b;
                acc[0] += o.v00 * b0.s0 * a + o.v01 * b0.s1 * b;
                acc[1] += o.v10 * b1.s0 * a + o.v11 * b1.s1 * b;
                acc[2] += a * a + b * b;
            },
            [&](int64_t s) { w0[s] = 0.0; w1[s] = 0.0; });
        wg_sum<T, 3>(acc, lds + Lds<T>::kScr);
        for (int i = 0; i < nbf; ++i) dots[i] = acc[i];
        if (nb > 2) dots_more(w0, w1, basis, 2, nb, dots);
        dots[nb] = acc[2];
    }

    // dots[i] = basis[i] . w for i in [i0, nb)
    template <class BP>
    __device__ __forceinline__ void dots_more(CP w0, CP w1, BP basis, int i0, int nb,
                                              double* dots) {
        constexpr int U = 2;
        const int M = cd.M;
        for (int g = i0; g < nb; g += 8) {
            double acc[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] = 0.0;
            VecRef bv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) bv[i] = basis[min(g + i, nb - 1)];
            for (int j0 = 0; j0 < M; j0 += U) {
                // every load of U rows x 8 vectors issues before any use: rows
                // past the chunk's end and vectors past nb reload valid ones,
                // and their terms are dropped by selects
                int64_t sl[U];
                double a[U], b[U], p[8][U], q[8][U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    sl[u] = sidx(t, min(j0 + u, M - 1));
                    a[u] = w0[sl[u]];
                    b[u] = w1[sl[u]];
                }
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const Vec2<double> e = ld_pair(bv[i], sl[u]);
                        p[i][u] = e.x;
                        q[i][u] = e.y;
                    }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const double term = p[i][u] * bv[i].s0 * a[u] + q[i][u] * bv[i].s1 * b[u];
                        acc[i] += (g + i < nb && j0 + u < M) ? term : 0.0;
                    }
            }
            wg_sum<T, 8>(acc, lds + Lds<T>::kScr);
            for (int i = 0; i < 8 && g + i < nb; ++i) dots[g + i] = acc[i];
        }
    }

    // One classical Gram-Schmidt pass: w -= sum_i h[i] basis[i]; then
    // dots[i] = basis[i] . w (i < nb) and dots[nb] = ||w||^2.
    template <class BP>
    __device__ void cgs_pass(CP w0, CP w1, BP basis, int nb, const double* h,
                             double* dots) {
        Column self(*this);
        self.cgs_pass_body(w0, w1, basis, nb, h, dots);
    }
    template <class BP>
    __device__ __forceinline__ void cgs_pass_body(CP w0, CP w1, BP basis, int nb, const double* h,
                                                  double* dots) {
        if (nb <= 0) cgs_pass_any(w0, w1, basis, nb, h, dots);
        else if (nb == 1) cgs_pass_n<1>(w0, w1, basis, nb, h, dots);
        else if (nb == 2) cgs_pass_n<2>(w0, w1, basis, nb, h, dots);
        else if (nb == 3) cgs_pass_n<3>(w0, w1, basis, nb, h, dots);
        else if (nb == 4) cgs_pass_n<4>(w0, w1, basis, nb, h, dots);
        else if (nb <= 8) cgs_pass_n<8>(w0, w1, basis, nb, h, dots);
        else cgs_pass_any(w0, w1, basis, nb, h, dots);
    }

    // The pass for nb <= NB basis vectors.  Their references and coefficients
    // are read once, ahead of the row loop: read inside it, each would wait
    // behind the rows' loads in the in-order memory counter, one round trip
    // per vector.  Slots past nb repeat the last vector with weight 0.
    template <int NB, class BP>
    __device__ __forceinline__ void cgs_pass_n(CP w0, CP w1, BP basis, int nb, const double* h,
                                               double* dots) {
        constexpr int U = NB <= 4 ? 4 : 2;
        const int M = cd.M;
        VecRef bv[NB];
        double hs0[NB], hs1[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            bv[i] = basis[min(i, nb - 1)];
            const double hi = i < nb ? h[min(i, nb - 1)] : 0.0;
            hs0[i] = hi * bv[i].s0;
            hs1[i] = hi * bv[i].s1;
        }
        double acc[NB + 1];
#pragma unroll
        for (int i = 0; i <= NB; ++i) acc[i] = 0.0;
        for (int j0 = 0; j0 < M; j0 += U) {
            // unconditional loads (rows past the chunk's end reload its last
            // row; their results are neither stored nor summed)
            double a[U], b[U], p[NB][U], q[NB][U];
            int64_t sl[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                sl[u] = sidx(t, min(j0 + u, M - 1));
                a[u] = w0[sl[u]];
                b[u] = w1[sl[u]];
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const Vec2<double> e = ld_pair(bv[i], sl[u]);
                    p[i][u] = e.x;
                    q[i][u] = e.y;
                }
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    a[u] -= hs0[i] * p[i][u];
                    b[u] -= hs1[i] * q[i][u];
                }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = j0 + u < M;
                if (ok) { w0[sl[u]] = a[u]; w1[sl[u]] = b[u]; }
                acc[NB] += ok ? a[u] * a[u] + b[u] * b[u] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                double sacc = 0.0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double term = p[i][u] * bv[i].s0 * a[u] + q[i][u] * bv[i].s1 * b[u];
                    sacc += (j0 + u < M) ? term : 0.0;
                }
                acc[i] += sacc;
            }
        }
        wg_sum<T, NB + 1>(acc, lds + Lds<T>::kScr);
        for (int i = 0; i < nb; ++i) dots[i] = acc[i];
        dots[nb] = acc[NB];
    }

    // The pass for any nb (references read per vector inside the row loop).
    template <class BP>
    __device__ __forceinline__ void cgs_pass_any(CP w0, CP w1, BP basis, int nb, const double* h,
                                 double* dots) {
        constexpr int U = 4;
        const int M = cd.M;
        double acc[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) acc[i] = 0.0;
        const int nbf = nb < 8 ? nb : 8;
        for (int j0 = 0; j0 < M; j0 += U) {
            // unconditional loads (rows past the chunk's end reload its last
            // row; their results are neither stored nor summed)
            double a[U], b[U];
            int64_t sl[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                sl[u] = sidx(t, min(j0 + u, M - 1));
                a[u] = w0[sl[u]];
                b[u] = w1[sl[u]];
            }
#pragma unroll 4
            for (int i = 0; i < nb; ++i) {
                const VecRef bi = basis[i];
                const double hi = h[i];
                double p[U], q[U];
#pragma unroll
                for (int u = 0; u < U; ++u) { const Vec2<double> e = ld_pair(bi, sl[u]); p[u] = e.x; q[u] = e.y; }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    a[u] -= hi * p[u] * bi.s0;
                    b[u] -= hi * q[u] * bi.s1;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = j0 + u < M;
                if (ok) { w0[sl[u]] = a[u]; w1[sl[u]] = b[u]; }
                acc[8] += ok ? a[u] * a[u] + b[u] * b[u] : 0.0;
            }
#pragma unroll 4
            for (int i = 0; i < nbf; ++i) {
                const VecRef bi = basis[i];
                double p[U], q[U];
#pragma unroll
                for (int u = 0; u < U; ++u) { const Vec2<double> e = ld_pair(bi, sl[u]); p[u] = e.x; q[u] = e.y; }
                double sacc = 0.0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double term = p[u] * bi.s0 * a[u] + q[u] * bi.s1 * b[u];
                    sacc += (j0 + u < M) ? term : 0.0;
                }
                acc[i] += sacc;
            }
        }
        wg_sum<T, 9>(acc, lds + Lds<T>::kScr);
        for (int i = 0; i < nbf; ++i) dots[i] = acc[i];
        if (nb > 8) dots_more(w0, w1, basis, 8, nb, dots);
        dots[nb] = acc[8];
    }

    // out = (accumulate ? out : 0) + sum_i c[i] vecs[i]
    __device__ void lincomb(CP o0, CP o1, const VecRef* vecs, const double* c, int nv,
                            bool accumulate) {
        Column self(*this);
        self.lincomb_body(o0, o1, vecs, c, nv, accumulate);
    }
    __device__ __forceinline__ void lincomb_body(CP o0, CP o1, const VecRef* vecs, const double* c, int nv,
                                                 bool accumulate) {
        if (nv <= 0) {
            if (accumulate) lincomb_t<true>(o0, o1, vecs, c, nv);
            else lincomb_t<false>(o0, o1, vecs, c, nv);
        } else if (accumulate) {
            if (nv <= 4) lincomb_n<4, true>(o0, o1, vecs, c, nv);
            else if (nv <= 8) lincomb_n<8, true>(o0, o1, vecs, c, nv);
            else lincomb_t<true>(o0, o1, vecs, c, nv);
        } else {
            if (nv == 1) lincomb_n<1, false>(o0, o1, vecs, c, nv);
            else if (nv == 2) lincomb_n<2, false>(o0, o1, vecs, c, nv);
            else if (nv <= 4) lincomb_n<4, false>(o0, o1, vecs, c, nv);
            else if (nv <= 8) lincomb_n<8, false>(o0, o1, vecs, c, nv);
            else lincomb_t<false>(o0, o1, vecs, c, nv);
        }
        __syncthreads();
    }
    // nv <= NV vectors, references and weights read ahead of the row loop
    // (as in cgs_pass_n); slots past nv repeat the last vector with weight 0
    template <int NV, bool ACC>
    __device__ __forceinline__ void lincomb_n(CP o0, CP o1, const VecRef* vecs, const double* c, int nv) {
        constexpr int U = NV <= 4 ? 4 : 2;
        const int M = cd.M;
        VecRef vv[NV];
        double cs0[NV], cs1[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            vv[i] = vecs[min(i, nv - 1)];
            const double ci = i < nv ? c[min(i, nv - 1)] : 0.0;
            cs0[i] = ci * vv[i].s0;
            cs1[i] = ci * vv[i].s1;
        }
        for (int j0 = 0; j0 < M; j0 += U) {
            double a[U], b[U], p[NV][U], q[NV][U];
            int64_t sl[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                sl[u] = sidx(t, min(j0 + u, M - 1));
                a[u] = ACC ? o0[sl[u]] : 0.0;
                b[u] = ACC ? o1[sl[u]] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < NV; ++i)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const Vec2<double> e = ld_pair(vv[i], sl[u]);
                    p[i][u] = e.x;
                    q[i][u] = e.y;
                }
#pragma unroll
            for (int i = 0; i < NV; ++i)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    a[u] += cs0[i] * p[i][u];
                    b[u] += cs1[i] * q[i][u];
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (j0 + u < M) { o0[sl[u]] = a[u]; o1[sl[u]] = b[u]; }
        }
    }
    template <bool ACC>
    __device__ __forceinline__ void lincomb_t(CP o0, CP o1, const VecRef* vecs, const double* c, int nv) {
        constexpr int U = 4;
        const int M = cd.M;
        for (int j0 = 0; j0 < M; j0 += U) {
            // unconditional loads, as in cgs_pass
            double a[U], b[U];
            int64_t sl[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                sl[u] = sidx(t, min(j0 + u, M - 1));
                a[u] = ACC ? o0[sl[u]] : 0.0;
                b[u] = ACC ? o1[sl[u]] : 0.0;
            }
#pragma unroll 4
            for (int i = 0; i < nv; ++i) {
                const VecRef vi = vecs[i];
                const double ci = c[i];
                double p[U], q[U];
#pragma unroll
                for (int u = 0; u < U; ++u) { const Vec2<double> e = ld_pair(vi, sl[u]); p[u] = e.x; q[u] = e.y; }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    a[u] += ci * p[u] * vi.s0;
                    b[u] += ci * q[u] * vi.s1;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (j0 + u < M) { o0[sl[u]] = a[u]; o1[sl[u]] = b[u]; }
        }
    }

    // Line-search trial X_t = X + lam S_X d, its residual and norms.
    __device__ Norms trial(int cur, int out, const VecRef& d, double lam) {
        Column self(*this);
        const VecRef dl = d;
        return self.trial_body(cur, out, dl, lam);
    }
    __device__ __forceinline__ Norms trial_body(int cur, int out, const VecRef& d, double lam) {
        const CP X0 = xb(cur, 0);
        const CP X1 = xb(cur, 1);
        const double a0 = lam * sxn * d.s0, a1 = lam * sxp * d.s1;
        return residual(
            [&](int64_t s, double& a, double& b) { a = X0[s] + a0 * d.p0[s]; b = X1[s] + a1 * d.p1[s]; },
            Fb(out, 0), Fb(out, 1), xb(out, 0), xb(out, 1), d, lam);
    }

    // Residual of buffer b (test export / re-evaluation)
    __device__ Norms eval(int b) {
        Column self(*this);
        return self.eval_body(b);
    }
    __device__ __forceinline__ Norms eval_body(int b) {
        const CP X0 = xb(b, 0);
        const CP X1 = xb(b, 1);
        const VecRef none{CP{nullptr}, CP{nullptr}, 0.0, 0.0};
        return residual([&](int64_t s, double& a, double& c) { a = X0[s]; c = X1[s]; },
                        Fb(b, 0), Fb(b, 1), CP{nullptr}, CP{nullptr}, none, 0.0);
    }

    // Workspace buffer -> caller arrays (natural layout)
    __device__ void write_back(CP s0p, CP s1p, double* o0, double* o1) {
        const int M = cd.M, n = cd.n;
        for (int j = 0; j < M; ++j) {
            const int c = t * M + j;
            if (c >= n) break;
            const int64_t s = sidx(t, j);
            o0[cd.uoff + c] = s0p[s];
            o1[cd.uoff + c] = s1p[s];
        }
    }
};

}  // namespace jfnk
