// libjfnk: kernels and host runtime of the C ABI declared in include/jfnk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "jfnk.h"
#include "jfnk_misdc.h"
#include "jfnk_net.h"
#include "jfnk_solver.h"

using namespace jfnk;

namespace {

constexpr int kTmax = 512;          // largest workgroup that owns a column
constexpr int kScalSlots = 64;      // doubles of scalar exchange per column
constexpr int kMaxBackoff = 5;      // a losing learned guess is skipped at up to 4^5 - 1 chances
constexpr int kMoveTiles = 32;      // 8 x 8-cell tiles per gather / write-back workgroup
constexpr int kMisdcArrays = 11;    // T_e^n, R^n, s, n_i~ (2), 2X^n - X^(k) (2), X^(k) (2 x 2)
constexpr int kMisdcMaxK = 64;      // SDC iterations per step

// ---------------------------------------------------------------------------
// Batched schedule: one workgroup per column, whole step in one launch.
// ---------------------------------------------------------------------------
struct SolveArgs {
    Work W;
    SolverParams prm;
    UserArrays U;
    const int* order;   // blockIdx -> column
    const int* mcol;    // gather / write-back workgroup -> column
    int ncols;
};

template <int T, class FT, bool TAB>
__global__ __launch_bounds__(T) void k_solve(SolveArgs a) {
    extern __shared__ double lds[];
    const int ci = a.order[blockIdx.x];
    if (ci < 0 || ci >= a.ncols) return;   // the order is a permutation; never taken
    DevExec<T, FT, TAB> ex;
    ex.col.init(a.W.cols[ci], a.W, a.prm, (ldbl*)lds);
    ex.U = a.U;
    ColOutcome o;
    jfnk_solve(ex, a.prm, o);
}

// Workgroup order of the next solve launch, by expected work, largest first
// (longest-processing-time): a column's work is taken as its cells times the
// bytes per cell its step just moved (from the phase counts).  A counting sort
// on the key's binary exponent and top three mantissa bits (eighths of an
// octave, keys 1..2^64); the order within a bucket is free.  One workgroup.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 8 * 64;

__device__ __forceinline__ int order_bucket(const ColState& s, int n) {
    const int32_t* w = s.work;
    const double cost = 104.0 + 120.0 * w[kWorkFactor] + 112.0 * w[kWorkApply] + 104.0 * w[kWorkResidual] +
                        120.0 * w[kWorkJv] + 32.0 * w[kWorkCgs] + 16.0 * w[kWorkLincomb] + 16.0 * w[kWorkVecReads];
    const double key = fmax(1.0, (double)n * cost);
    const uint64_t u = (uint64_t)__double_as_longlong(key);
    const int b = min(kOrderBuckets - 1, (int)((u >> 49) - (uint64_t)1023 * 8));
    return kOrderBuckets - 1 - b;
}

__global__ __launch_bounds__(kOrderThreads) void k_order(const ColState* cst, const ColDesc* cols, int ncols,
                                                         int* order) {
    __shared__ int start[kOrderBuckets];
    const int t = threadIdx.x;
    for (int b = t; b < kOrderBuckets; b += kOrderThreads) start[b] = 0;
    __syncthreads();
    for (int c = t; c < ncols; c += kOrderThreads) atomicAdd(&start[order_bucket(cst[c], cols[c].n)], 1);
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int b = 0; b < kOrderBuckets; ++b) {
            const int n = start[b];
            start[b] = acc;
            acc += n;
        }
    }
    __syncthreads();
    for (int c = t; c < ncols; c += kOrderThreads) {
        const int pos = atomicAdd(&start[order_bucket(cst[c], cols[c].n)], 1);
        if (pos < ncols) order[pos] = c;
    }
}

// The data-movement ends of a batched step as launches of their own: they
// need few registers, so many waves per SIMD hide the memory latency that
// the solve's single wave per SIMD cannot, and they split every column into
// workgroups of at most kMoveTiles tiles so that long columns do not leave a
// tail.  Workgroup g serves column mcol[g], tiles [(g - g0) kMoveTiles, ...).
constexpr int kMoveThreads = 256;

template <int T, bool TAB>
__global__ __launch_bounds__(kMoveThreads) void k_gather(SolveArgs a) {
    const int ci = a.mcol[blockIdx.x];
    using Col = Column<T, float, TAB>;
    Col col;
    col.init(a.W.cols[ci], a.W, a.prm, nullptr);
    ColState* cs = a.W.cst + col.cd.index;
    const int kb = ((int)blockIdx.x - col.cd.g0) * kMoveTiles;
    const int ke = min(kb + kMoveTiles, col.ntiles());
    const int gm = col.gather(a.U, kb, ke, threadIdx.x >> 6, kMoveThreads / 64, &cs->nrR);
    const int any_changed = __syncthreads_or(gm & Col::kGatherChanged);
    const int any_bad = __syncthreads_or(gm & Col::kGatherBad);
    if (threadIdx.x == 0)
        a.W.gflag[blockIdx.x] = (any_changed ? Col::kGatherChanged : 0) | (any_bad ? Col::kGatherBad : 0);
}

template <int T>
__global__ __launch_bounds__(kMoveThreads) void k_scatter(SolveArgs a) {
    const int ci = a.mcol[blockIdx.x];
    Column<T, float> col;
    col.init(a.W.cols[ci], a.W, a.prm, nullptr);
    const int b = a.W.cst[col.cd.index].cur;
    const int kb = ((int)blockIdx.x - col.cd.g0) * kMoveTiles;
    const int ke = min(kb + kMoveTiles, col.ntiles());
    col.scatter(col.xb(b, 0), col.xb(b, 1), a.U.ne_out, a.U.phi_out, kb, ke, threadIdx.x >> 6, kMoveThreads / 64);
}

// ---------------------------------------------------------------------------
// Plain schedule: one kernel per phase of one column; scalars go back to the
// host through W.scal.
// ---------------------------------------------------------------------------
enum Phase {
    PH_SETUP, PH_FACTOR, PH_APPLY, PH_CORR, PH_JV, PH_CGS, PH_LINCOMB, PH_NORM_DX, PH_RES0, PH_TRIAL,
    PH_FINAL, PH_EVAL, PH_LOAD_X, PH_LOAD_V, PH_STORE_V, PH_STORE_W, PH_STORE_F
};

struct PhaseArgs {
    Work W;
    SolverParams prm;
    UserArrays U;
    int ci;
    int phase;
    int cur, out, zslot, wslot, nb, acc;
    double eps, lam;
    VecRef v;
    VecRef basis[kMaxRestart + 1];
    double h[kMaxRestart + 2];
    ColOutcome o;
    const double* in0;
    const double* in1;
    double* out0;
    double* out1;
    int32_t all;        // one workgroup per column (column order[blockIdx.x]) instead of column ci alone
    int32_t ncols;      // columns of a launch over all of them
    const int* order;   // longest columns first (the dispatcher then balances the tail)
    int32_t eps_dev;    // PH_JV: the finite-difference step from the column's scalars (see below)
};

// PH >= 0: a kernel holding that phase alone (its registers are that
// phase's, not the largest over all phases); -1: the phase from the arguments.
template <int T, class FT, bool TAB, int PH = -1>
__global__ __launch_bounds__(T) void k_phase(PhaseArgs a) {
    extern __shared__ double lds[];
    const int phase = PH >= 0 ? PH : a.phase;
    const int ci = a.all ? a.order[blockIdx.x] : a.ci;
    Column<T, FT, TAB> col;
    col.init(a.W.cols[ci], a.W, a.prm, (ldbl*)lds);
    double* scal = a.W.scal + (int64_t)ci * kScalSlots;
    VecRef* bl = (VecRef*)(lds + Lds<T>::kBasis);
    if (phase != PH_SETUP) col.load_state();
    if (phase == PH_JV || phase == PH_CGS) {
        if (threadIdx.x == 0)
            for (int i = 0; i < a.nb; ++i) bl[i] = a.basis[i];
        __syncthreads();
    }
    switch (phase) {
    case PH_SETUP: {
        int cur, g;
        const Norms n = col.setup(a.U, &cur, &g);
        if (threadIdx.x == 0) {
            scal[0] = cur; scal[1] = g; scal[2] = n.rinf; scal[3] = n.r2; scal[4] = n.xn2;
            scal[5] = n.step; scal[6] = col.sfn; scal[7] = col.sfp; scal[8] = col.sxn; scal[9] = col.sxp;
            scal[10] = col.fac_reuse ? 1.0 : 0.0;
            scal[11] = col.bad_input ? 1.0 : 0.0;
        }
        break;
    }
    case PH_FACTOR:
        col.factor(a.cur);
        break;
    case PH_APPLY: {
        const Vec2<double> z = col.apply(a.v, col.Zb(a.zslot, 0), col.Zb(a.zslot, 1));
        if (threadIdx.x == 0) { scal[0] = z.x; scal[1] = z.y; }
        break;
    }
    case PH_CORR: {
        const Vec2<double> z = col.apply(a.v, col.Vb(a.prm.m, 0), col.Vb(a.prm.m, 1));
        if (threadIdx.x == 0) { scal[0] = z.x; scal[1] = z.y; }
        break;
    }
    case PH_JV: {
        double dots[kMaxRestart + 2];
        double eps = a.eps;
        if (a.eps_dev) {
            // eq:jf_dfapprox's step for z = Z[zslot] from ||S_X^-1 X||^2 (left in
            // scal[2] by PH_EVAL) and ||z||^2 (left in scal[0] by PH_NORM_DX);
            // every thread reads them before thread 0 overwrites scal below
            const double xn2 = scal[2], vn2 = scal[0];
            const double lam_fd = 6.0554544523933395e-06;
            eps = vn2 > 0.0 ? lam_fd * (lam_fd + sqrt(xn2) / sqrt(vn2)) : 1.0;
        }
        const VecRef z = (a.zslot >= 0) ? VecRef{col.Zb(a.zslot, 0), col.Zb(a.zslot, 1), 1.0, 1.0}
                                        : a.v;
        col.jv(a.cur, z, eps, col.Vb(a.wslot, 0), col.Vb(a.wslot, 1), bl, a.nb, dots);
        if (threadIdx.x == 0)
            for (int i = 0; i <= a.nb; ++i) scal[i] = dots[i];
        break;
    }
    case PH_CGS: {
        double dots[kMaxRestart + 2];
        col.cgs_pass(col.Vb(a.wslot, 0), col.Vb(a.wslot, 1), bl, a.nb, a.h, dots);
        if (threadIdx.x == 0)
            for (int i = 0; i <= a.nb; ++i) scal[i] = dots[i];
        break;
    }
    case PH_LINCOMB: {
        VecRef zs[kMaxRestart];
        for (int i = 0; i < a.nb; ++i) zs[i] = VecRef{col.Zb(i, 0), col.Zb(i, 1), 1.0, 1.0};
        col.lincomb(col.dXb(0), col.dXb(1), zs, a.h, a.nb, a.acc != 0);
        break;
    }
    case PH_NORM_DX: {
        double dd[1] = {0.0};
        const CP d0 = col.dXb(0);
        const CP d1 = col.dXb(1);
        for (int j = 0; j < col.cd.M; ++j) {
            const int64_t s = col.sidx(col.t, j);
            dd[0] += d0[s] * d0[s] + d1[s] * d1[s];
        }
        wg_sum<T, 1>(dd, lds + Lds<T>::kScr);
        if (threadIdx.x == 0) scal[0] = dd[0];
        break;
    }
    case PH_RES0: {
        const CP v0 = col.Vb(0, 0);
        const CP v1 = col.Vb(0, 1);
        const CP F0 = col.Fb(a.cur, 0);
        const CP F1 = col.Fb(a.cur, 1);
        double acc[1] = {0.0};
        for (int j = 0; j < col.cd.M; ++j) {
            const int64_t s = col.sidx(col.t, j);
            const double x = -F0[s] * col.isfn - v0[s];
            const double y = -F1[s] * col.isfp - v1[s];
            v0[s] = x; v1[s] = y;
            acc[0] += x * x + y * y;
        }
        wg_sum<T, 1>(acc, lds + Lds<T>::kScr);
        if (threadIdx.x == 0) scal[0] = acc[0];
        break;
    }
    case PH_TRIAL: {
        const Norms n = col.trial(a.cur, a.out, a.v, a.lam);
        if (threadIdx.x == 0) { scal[0] = n.rinf; scal[1] = n.r2; scal[2] = n.xn2; scal[3] = n.step; }
        break;
    }
    case PH_FINAL: {
        col.write_back(col.xb(a.o.cur, 0), col.xb(a.o.cur, 1), a.U.ne_out, a.U.phi_out);
        if (threadIdx.x == 0) {
            ColState* cs = a.W.cst + col.cd.index;
            cs->res_inf = a.o.rinf; cs->res2 = a.o.r2; cs->status = a.o.status;
            cs->newton = a.o.newton; cs->gmres = a.o.gmres; cs->backtracks = a.o.backtracks;
            cs->guess = a.o.guess; cs->restarts = a.o.restarts; cs->chords = a.o.chords;
            for (int i = 0; i < kWorkCounts; ++i) cs->work[i] = a.o.work[i];
        }
        break;
    }
    case PH_EVAL: {
        const Norms n = col.eval(a.cur);
        if (threadIdx.x == 0) { scal[0] = n.rinf; scal[1] = n.r2; scal[2] = n.xn2; }
        break;
    }
    case PH_LOAD_X:
    case PH_LOAD_V: {
        // natural-layout caller arrays -> buffer (x[cur] or Z[zslot])
        const CP o0 = (a.phase == PH_LOAD_X) ? col.xb(a.cur, 0) : col.Zb(a.zslot, 0);
        const CP o1 = (a.phase == PH_LOAD_X) ? col.xb(a.cur, 1) : col.Zb(a.zslot, 1);
        for (int j = 0; j < col.cd.M; ++j) {
            const int c = col.t * col.cd.M + j;
            const int64_t s = col.sidx(col.t, j);
            if (c < col.cd.n) { o0[s] = a.in0[col.cd.uoff + c]; o1[s] = a.in1[col.cd.uoff + c]; }
            else { o0[s] = 0.0; o1[s] = 0.0; }
        }
        __syncthreads();
        break;
    }
    case PH_STORE_V:
        col.write_back(col.Zb(a.zslot, 0), col.Zb(a.zslot, 1), a.out0, a.out1);
        break;
    case PH_STORE_W:
        col.write_back(col.Vb(a.wslot, 0), col.Vb(a.wslot, 1), a.out0, a.out1);
        break;
    case PH_STORE_F:
        col.write_back(col.Fb(a.cur, 0), col.Fb(a.cur, 1), a.out0, a.out1);
        break;
    default:
        break;
    }
}

// ---------------------------------------------------------------------------
// Host context
// ---------------------------------------------------------------------------
}  // namespace

struct jfnk_ctx {
    jfnk_config cfg{};
    int device = 0;
    int64_t capP = 0;
    int64_t capRed = 0;
    char* base = nullptr;        // single workspace allocation
    Work W{};
    int* d_order = nullptr;
    ColDesc* h_cols = nullptr;   // pinned
    ColState* h_cst = nullptr;   // pinned
    double* h_scal = nullptr;    // pinned
    int* h_order = nullptr;      // pinned
    std::string err;
    bool poisoned = false;
    int Tsel = 0;                // workgroup size of the last schedule
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // around the solve launches
    hipEvent_t evg = nullptr, evs = nullptr;   // batched: after the gather and after the solve launch
    int64_t capMove = 0;                       // gather / write-back workgroups the tables hold
    int32_t* d_mcol = nullptr;                 // [capMove] workgroup -> column
    int32_t* h_mcol = nullptr;                 // pinned
    int32_t* d_gflag = nullptr;                // [capMove] coefficient-change flag per gather workgroup
    int nmove = 0;                             // gather / write-back workgroups of the current schedule
    bool timed3 = false;                       // the last step recorded evg and evs
    double last_kms[3] = {0.0, 0.0, 0.0};      // gather, solve, write-back (ms)
    // schedule cache: the per-column inputs the last uploaded schedule was built from
    std::vector<int64_t> last_off;
    std::vector<double> last_scal;
    std::vector<int32_t> last_bc;
    bool sched_valid = false;
    bool timed = false;
    double last_ms = 0.0;
    int last_launches = 0;
    // learned guess
    jfnk_net* model = nullptr;
    uint64_t model_version = 0;  // weight version the back-off records below were judged with
    double* d_learn = nullptr;   // [2][max_total_cells]: guess n, phi
    int32_t* d_lmask = nullptr;  // [max_cols]
    int32_t* h_lmask = nullptr;  // pinned
    bool learn_active = false;
    bool fac_reuse_ok = false;   // the workspace holds factors of the current layout from the last step
    bool hist_valid = false;     // the per-column records below describe the current layout
    std::vector<int32_t> last_newton, last_status;
    // schedule autotuner: workgroup size measured best for a column layout
    int force_T = 0;                      // set while the tuner tries a candidate
    int tuned_T = 0;
    std::vector<int64_t> tuned_off;
    // tuned workgroup sizes by layout: this context's autotuner results and
    // those read by jfnk_autotune_load (matched by the layout's hash)
    struct TuneEntry {
        uint64_t hash;
        int32_t ncols, table, T;
        int64_t total;
        double ms[4];
        bool mine;      // tuned by this context (saved by jfnk_autotune_save)
    };
    std::vector<TuneEntry> tune_table;
    std::vector<uint8_t> evaluated;       // network evaluated for the column this step
    std::vector<int32_t> reject_streak;   // consecutive evaluations its candidate lost
    std::vector<int32_t> skip_left;       // chances to skip before evaluating it again
    // Steps in flight (jfnk_step_async).  The per-step host resources above
    // (statistics buffer, events, staging of the work order and of the learned
    // mask, the evaluated set) are swapped with this slot after every
    // asynchronous enqueue, so the step in flight keeps its own while the next
    // one is prepared.
    struct Slot {
        ColState* h_cst = nullptr;
        int* h_order = nullptr;
        int32_t* h_lmask = nullptr;
        hipEvent_t ev0 = nullptr, evg = nullptr, evs = nullptr, ev1 = nullptr, done = nullptr;
        std::vector<uint8_t> evaluated;
        bool timed = false, timed3 = false, learned_ran = false;
        int launches = 0;
    } alt;
    hipEvent_t evdone = nullptr;   // recorded after the statistics copy of the step
    bool learned_ran = false;      // the step's set-up evaluated learned candidates
    bool pending = false;          // an asynchronous step is in flight (its resources in alt)
    int pending_ncols = 0;
    hipStream_t pending_stream = nullptr;
    // MISDC step: workspace allocated by its first call
    double* mis = nullptr;         // [kMisdcArrays][capP]
    MisdcCol* d_mis = nullptr;     // [max_cols]
    MisdcCol* h_mis = nullptr;     // pinned
    double* d_vmax = nullptr;      // [max_cols] largest ion drift speed per column
    double* h_vmax = nullptr;      // pinned
};

namespace {

int drain(jfnk_ctx* ctx, jfnk_stats* stt = nullptr, int32_t* rc_out = nullptr);

int fail(jfnk_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIP_OK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ctx->poisoned = true;                                                        \
            return fail(ctx, JFNK_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
        }                                                                                \
    } while (0)

// 64-bit FNV-1a over the column offsets: the key of a tuned layout
uint64_t layout_hash(const int64_t* off, int n1) {
    uint64_t h = 1469598103934665603ull;
    const unsigned char* b = (const unsigned char*)off;
    for (size_t i = 0; i < sizeof(int64_t) * (size_t)n1; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

// the current device's architecture name (a tuned entry's device)
std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t pr;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string a = pr.gcnArchName;
    for (char& ch : a)
        if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
    return a.empty() ? "unknown" : a;
}

// A workgroup size is used for a layout when it owns its longest column with
// at most 64 cells per thread (any size for columns beyond 64 kTmax cells,
// which only the largest can take at 64) -- the autotuner's rule.
bool threads_fit(int T, int nmax) {
    if (T != 64 && T != 128 && T != 256 && T != 512) return false;
    return T == kTmax || (nmax + T - 1) / T <= 64;
}

int choose_T(const jfnk_config& cfg, int nmax) {
    if (cfg.threads_override > 0) return cfg.threads_override;
    // chunk of <= 16 cells per thread where possible
    int T = 64;
    while (T < kTmax && (nmax + T - 1) / T > 16) T <<= 1;
    return T;
}

// The workspace arrays for P padded cells (a multiple of 64), GMRES restart
// m, red doubles of per-chunk data and max_cols columns (and the multigrid
// arrays when mg), carved from base in this order; returns the doubles they
// span.  With base == nullptr only the size is computed (W untouched).
int64_t carve_work(double* base, int64_t P, int m, int64_t red, int max_cols, Work* W, bool mg) {
    int64_t off = 0;
    auto take = [&](int64_t n) { double* r = base ? base + off : nullptr; off += n; return r; };
    Work w{};
    w.P = P;
    w.fa = take(P); w.fg = take(P); w.fw = take(P);
    w.f = take(P); w.kd = take(P); w.q = take(P);
    w.x = take(6 * P); w.F = take(6 * P);
    w.V = take(2 * (int64_t)(m + 1) * P);
    w.Z = take(2 * (int64_t)m * P);
    w.dX = take(2 * P);
    w.fac = (void*)take((int64_t)kFactorSlots * P);
    w.tmp = (void*)take(2 * P);
    w.sch = take(4 * P);
    w.red = take(red);
    w.cols = (ColDesc*)take((max_cols * (int64_t)sizeof(ColDesc) + 7) / 8);
    w.cst = (ColState*)take((max_cols * (int64_t)sizeof(ColState) + 7) / 8);
    w.scal = take((int64_t)max_cols * kScalSlots);
    w.mgP = mg ? 2 * P + 64 * (int64_t)max_cols : 0;
    w.mg = mg ? take(kMgFields * w.mgP) : nullptr;
    if (base && W) {
        w.lmask = W->lmask;
        w.gflag = W->gflag;
        *W = w;
    }
    return off;
}

void carve(jfnk_ctx* c) {
    carve_work((double*)c->base, c->capP, c->cfg.gmres_restart, c->capRed, c->cfg.max_cols, &c->W,
               c->cfg.prec_kind == JFNK_PRECK_SCHUR_MG);
}

// The configuration's own checks (those of jfnk_create).
bool config_valid(const jfnk_config* cfg) {
    if (cfg->max_cols < 1 || cfg->max_total_cells < 3 || cfg->max_cells_per_col < 3 ||
        cfg->gmres_restart < 1 || cfg->gmres_restart > kMaxRestart || cfg->max_restarts < 0 ||
        cfg->max_newton < 0 || cfg->max_backtracks < 0 || !(cfg->tol_f > 0.0) || !(cfg->tol_x >= 0.0) ||
        !(cfg->gamma > 0.0 && cfg->gamma < 1.0) || !(cfg->ls_theta >= 0.0 && cfg->ls_theta < 1.0) ||
        !(cfg->chord_tol >= 0.0 && cfg->chord_tol < 1.0) ||
        (cfg->prec_precision != JFNK_PREC_FP64 && cfg->prec_precision != JFNK_PREC_FP32) ||
        (cfg->prec_kind != JFNK_PRECK_BLOCK && cfg->prec_kind != JFNK_PRECK_SCHUR &&
         cfg->prec_kind != JFNK_PRECK_NONE && cfg->prec_kind != JFNK_PRECK_SCHUR_MG) ||
        (cfg->prec_kind == JFNK_PRECK_SCHUR_MG &&
         (!(cfg->mg_tol > 0.0 && cfg->mg_tol < 1.0) || cfg->mg_blocks < 1 || cfg->mg_blocks > 3 ||
          cfg->mg_transfer < 0 || cfg->mg_transfer > 3)) ||
        cfg->guess < 0 || cfg->guess > 2 ||
        (cfg->schedule != JFNK_SCHED_PLAIN && cfg->schedule != JFNK_SCHED_BATCHED))
        return false;
    const int t = cfg->threads_override;
    return t == 0 || t == 64 || t == 128 || t == 256 || t == 512;
}

// The per-cell arrays and the transport table: nullptr when usable, else why not.
const char* check_cells(const jfnk_problem* p, const jfnk_state* x) {
    if (!p->src || !p->q_ion || !x->ne || !x->phi) return "null per-cell array";
    if (p->table) {
        const jfnk_table* t = p->table;
        if (!p->prog || !p->gas_n) return "table transport needs prog and gas_n";
        if (t->nc < 2 || t->nx < 2 || !t->mu || !t->diff) return "transport table: bad size or null array";
        if (!(t->c_max > t->c_min) || !(t->x_max > t->x_min) || !std::isfinite(t->c_min) ||
            !std::isfinite(t->c_max) || !std::isfinite(t->x_min) || !std::isfinite(t->x_max))
            return "transport table: bad grid range";
    } else if (!p->mu || !p->diff) {
        return "null per-cell array";
    }
    if ((x->ne_prev == nullptr) != (x->phi_prev == nullptr))
        return "ne_prev and phi_prev must both be given or both NULL";
    if ((x->ne_out == nullptr) != (x->phi_out == nullptr))
        return "ne_out and phi_out must both be given or both NULL";
    return nullptr;
}

TabRef tab_of(const jfnk_problem* p) {
    TabRef t{};
    if (p->table) {
        t.mu = p->table->mu; t.diff = p->table->diff;
        t.nc = p->table->nc; t.nx = p->table->nx;
        t.c_min = p->table->c_min; t.c_max = p->table->c_max;
        t.x_min = p->table->x_min; t.x_max = p->table->x_max;
    }
    return t;
}

// validation of the problem; fills the schedule on success
// the workgroup size of a tuned entry for this layout (0: none)
int tuned_lookup(const jfnk_ctx* ctx, const jfnk_problem* p, int nmax) {
    if (ctx->tune_table.empty()) return 0;
    const uint64_t h = layout_hash(p->col_offset, p->ncols + 1);
    const int tab = p->table ? 1 : 0;
    for (auto it = ctx->tune_table.rbegin(); it != ctx->tune_table.rend(); ++it)
        if (it->hash == h && it->ncols == p->ncols && it->total == p->col_offset[p->ncols] && it->table == tab &&
            threads_fit(it->T, nmax))
            return it->T;
    return 0;
}

// the workgroup size a step of this context takes for p's layout
int step_threads(const jfnk_ctx* ctx, const jfnk_problem* p, int nmax) {
    if (ctx->force_T > 0) return ctx->force_T;
    if (ctx->cfg.threads_override == 0 && ctx->tuned_T > 0 && (int)ctx->tuned_off.size() == p->ncols + 1 &&
        memcmp(ctx->tuned_off.data(), p->col_offset, sizeof(int64_t) * (p->ncols + 1)) == 0)
        return ctx->tuned_T;
    if (ctx->cfg.threads_override == 0 && ctx->cfg.schedule == JFNK_SCHED_BATCHED) {
        const int tt = tuned_lookup(ctx, p, nmax);
        if (tt > 0) return tt;
    }
    return choose_T(ctx->cfg, nmax);
}

int validate(jfnk_ctx* ctx, const jfnk_problem* p, const jfnk_state* x) {
    if (!p || !x) return fail(ctx, JFNK_EINVAL, "null problem or state");
    if (p->ncols < 1) return fail(ctx, JFNK_EINVAL, "ncols < 1");
    if (p->ncols > ctx->cfg.max_cols) return fail(ctx, JFNK_ECAPACITY, "ncols exceeds capacity");
    if (!p->col_offset || !p->length || !p->dt || !p->phi_left || !p->phi_right || !p->eps_over_e ||
        !p->bc_left || !p->bc_right || !p->ne_left || !p->ne_right)
        return fail(ctx, JFNK_EINVAL, "null per-column array");
    if (const char* why = check_cells(p, x)) return fail(ctx, JFNK_EINVAL, why);
    if (p->col_offset[0] != 0) return fail(ctx, JFNK_EINVAL, "col_offset[0] != 0");
    int nmax = 0;
    for (int c = 0; c < p->ncols; ++c) {
        const int64_t n = p->col_offset[c + 1] - p->col_offset[c];
        if (n < 3) return fail(ctx, JFNK_EINVAL, "column with fewer than 3 cells");
        if (n > ctx->cfg.max_cells_per_col) return fail(ctx, JFNK_ECAPACITY, "column longer than capacity");
        nmax = std::max<int>(nmax, (int)n);
        const double v[7] = {p->length[c], p->dt[c], p->phi_left[c], p->phi_right[c], p->eps_over_e[c],
                             p->ne_left[c], p->ne_right[c]};
        for (double d : v)
            if (!std::isfinite(d)) return fail(ctx, JFNK_EINVAL, "non-finite per-column scalar");
        if (!(p->length[c] > 0.0) || !(p->dt[c] > 0.0) || !(p->eps_over_e[c] > 0.0))
            return fail(ctx, JFNK_EINVAL, "length, dt and eps_over_e must be > 0");
        if ((p->bc_left[c] != 0 && p->bc_left[c] != 1) || (p->bc_right[c] != 0 && p->bc_right[c] != 1))
            return fail(ctx, JFNK_EINVAL, "bad boundary condition code");
    }
    if (p->col_offset[p->ncols] > ctx->cfg.max_total_cells)
        return fail(ctx, JFNK_ECAPACITY, "total cells exceed capacity");
    const int T = step_threads(ctx, p, nmax);
    int64_t ws = 0, red = 0;
    for (int c = 0; c < p->ncols; ++c) {
        const int n = (int)(p->col_offset[c + 1] - p->col_offset[c]);
        const int M = (n + T - 1) / T;
        ColDesc& d = ctx->h_cols[c];
        d.n = n; d.M = M; d.bcl = p->bc_left[c]; d.bcr = p->bc_right[c];
        d.index = c; d.T = T;
        d.uoff = p->col_offset[c]; d.ws = ws; d.red = red;
        d.h = p->length[c] / n; d.dt = p->dt[c];
        d.phil = p->phi_left[c]; d.phir = p->phi_right[c];
        d.eps = p->eps_over_e[c]; d.nel = p->ne_left[c]; d.ner = p->ne_right[c];
        ws += (int64_t)T * M;
        red += (int64_t)T * kRedPerChunk;
    }
    if (ws > ctx->capP || red > ctx->capRed) return fail(ctx, JFNK_ECAPACITY, "padded workspace exceeds capacity");
    // longest columns first: the dispatcher then balances the tail (LPT)
    std::vector<int> ord(p->ncols);
    for (int c = 0; c < p->ncols; ++c) ord[c] = c;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return ctx->h_cols[a].n > ctx->h_cols[b].n; });
    for (int c = 0; c < p->ncols; ++c) ctx->h_order[c] = ord[c];
    // gather / write-back workgroups: up to kMoveTiles tiles of one column each
    int64_t g = 0;
    for (int i = 0; i < p->ncols; ++i) {
        ColDesc& d = ctx->h_cols[ord[i]];
        const int64_t tiles = (int64_t)((d.M + 7) / 8) * (T / 8);
        const int64_t gn = (tiles + kMoveTiles - 1) / kMoveTiles;
        if (g + gn > ctx->capMove) return fail(ctx, JFNK_ECAPACITY, "gather workgroups exceed capacity");
        d.g0 = (int32_t)g; d.gn = (int32_t)gn;
        for (int64_t k = 0; k < gn; ++k) ctx->h_mcol[g + k] = ord[i];
        g += gn;
    }
    ctx->nmove = (int)g;
    ctx->Tsel = T;
    return JFNK_OK;
}

SolverParams params_of(const jfnk_config& cfg, const jfnk_problem* p, const jfnk_state* x, bool learned,
                       bool fac_reuse) {
    SolverParams s{};
    s.m = cfg.gmres_restart;
    s.max_restarts = cfg.max_restarts;
    s.max_newton = cfg.max_newton;
    s.max_backtracks = cfg.max_backtracks;
    s.guess = cfg.guess;
    s.has_prev = x->ne_prev != nullptr;
    s.has_learned = learned ? 1 : 0;
    s.has_u = p->u_face != nullptr;
    s.fac_reuse = fac_reuse ? 1 : 0;
    s.prec_kind = cfg.prec_kind;
    s.tol_f = cfg.tol_f;
    s.tol_x = cfg.tol_x;
    s.gamma = cfg.gamma;
    s.theta = cfg.ls_theta;
    // without a preconditioner a simplified-Newton step would be a unit
    // Richardson step on the scaled system: none is taken
    s.chord_tol = cfg.prec_kind == JFNK_PRECK_NONE ? 0.0 : cfg.chord_tol;
    s.mg_tol = cfg.mg_tol;
    s.mg_blocks = cfg.mg_blocks;
    s.mg_transfer = cfg.mg_transfer;
    s.tab = tab_of(p);
    // with table transport the Jacobian changes with the field even when the
    // face records do not: no factors are kept from the step before
    if (p->table) s.fac_reuse = 0;
    return s;
}

SolverParams make_params(const jfnk_ctx* ctx, const jfnk_problem* p, const jfnk_state* x) {
    return params_of(ctx->cfg, p, x, ctx->learn_active, ctx->fac_reuse_ok);
}

UserArrays make_user(const jfnk_ctx* ctx, const jfnk_problem* p, jfnk_state* x) {
    UserArrays U{};
    U.mu = p->mu; U.diff = p->diff; U.src = p->src; U.kloss = p->k_loss; U.q = p->q_ion;
    U.uface = p->u_face;
    U.ne = x->ne; U.phi = x->phi;
    U.ne_out = x->ne_out ? x->ne_out : x->ne;
    U.phi_out = x->phi_out ? x->phi_out : x->phi;
    U.ne_prev = x->ne_prev; U.phi_prev = x->phi_prev;
    U.ne_learn = nullptr; U.phi_learn = nullptr;
    U.prog = p->prog; U.gasn = p->gas_n;
    if (ctx->learn_active) {
        U.ne_learn = ctx->d_learn;
        U.phi_learn = ctx->d_learn + ctx->cfg.max_total_cells;
    }
    return U;
}

// Dynamic LDS of a solve launch.  The solve runs one wave per SIMD (its
// registers), so T / 64 waves share a CU's 160 KiB with 256 / T - 1 other
// workgroups (one at T >= 256); when the block solve's intermediate d for the
// longest column (mmax rows per thread) fits in that share beside the GMRES
// state, it stays in LDS (*dlds = 1) instead of making a round trip to HBM.
template <int T, class FT>
size_t solve_lds(int prec_kind, int mmax, int32_t* dlds) {
    constexpr size_t kCU = 160 * 1024;
    constexpr size_t share = T >= 256 ? kCU : kCU * T / 256;
    const size_t with_d = Lds<T>::bytes_d(mmax, sizeof(FT));
    *dlds = (prec_kind == JFNK_PRECK_BLOCK && with_d <= share) ? 1 : 0;
    return *dlds ? with_d : Lds<T>::bytes();
}

// ---------------------------------------------------------------------------
// Host-driven executor of the control logic (plain schedule).
// ---------------------------------------------------------------------------
template <int T, class FT, bool TAB>
struct HostExecT {
    jfnk_ctx* ctx;
    hipStream_t st;
    PhaseArgs a;
    hipError_t herr = hipSuccess;
    size_t lds_bytes = Lds<T>::bytes();   // the phases' dynamic LDS (solve_lds)
    double sfn = 1, sfp = 1, isfn = 1, isfp = 1;
    VecRef bas[kMaxRestart + 1];
    double H[(kMaxRestart + 1) * kMaxRestart];
    double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1];
    bool implicit_dir = false;
    double implicit_y = 0.0;

    const ColDesc& cd() const { return ctx->h_cols[a.ci]; }
    // device addresses of the two-component fields (interleaved pairs, as Column)
    CP xb(int b, int comp) const { return CP{ctx->W.x + 2 * b * ctx->W.P + comp}; }
    CP Fb(int b, int comp) const { return CP{ctx->W.F + 2 * b * ctx->W.P + comp}; }
    CP Vb(int k, int comp) const { return CP{ctx->W.V + 2 * (int64_t)k * ctx->W.P + comp}; }
    CP Zb(int k, int comp) const { return CP{ctx->W.Z + 2 * (int64_t)k * ctx->W.P + comp}; }
    CP dXb(int comp) const { return CP{ctx->W.dX + comp}; }

    void launch(int phase) {
        a.phase = phase;
        if (herr != hipSuccess) return;
        hipLaunchKernelGGL((k_phase<T, FT, TAB>), dim3(1), dim3(T), lds_bytes, st, a);
        herr = hipGetLastError();
    }
    const double* fetch(int n) {
        double* hs = ctx->h_scal;
        if (herr != hipSuccess) { for (int i = 0; i < n; ++i) hs[i] = NAN; return hs; }
        herr = hipMemcpyAsync(hs, ctx->W.scal + (int64_t)a.ci * kScalSlots, sizeof(double) * n,
                              hipMemcpyDeviceToHost, st);
        if (herr == hipSuccess) herr = hipStreamSynchronize(st);
        if (herr != hipSuccess) for (int i = 0; i < n; ++i) hs[i] = NAN;
        return hs;
    }

    bool lagged = false, bad = false;
    bool lagged_factors() const { return lagged; }
    bool bad_input() const { return bad; }
    Norms setup(int* cur, int* guess) {
        launch(PH_SETUP);
        const double* s = fetch(12);
        *cur = (int)s[0]; *guess = (int)s[1];
        Norms n{s[2], s[3], s[4], s[5]};
        lagged = s[10] == 1.0;
        bad = s[11] == 1.0;
        sfn = s[6]; sfp = s[7];
        isfn = 1.0 / sfn; isfp = 1.0 / sfp;
        if (herr != hipSuccess) n.r2 = NAN;
        return n;
    }
    void factor(int cur) { a.cur = cur; launch(PH_FACTOR); }
    Vec2<double> correction(int b) {
        a.v = fref(b, -1.0);
        launch(PH_CORR);
        const double* s = fetch(2);
        return Vec2<double>{s[0], s[1]};
    }
    VecRef fref(int cur, double sc) { return VecRef{Fb(cur, 0), Fb(cur, 1), sc * isfn, sc * isfp}; }
    VecRef vslot(int k, double sc) { return VecRef{Vb(k, 0), Vb(k, 1), sc, sc}; }
    void set_basis(int i, VecRef r) { bas[i] = r; }
    VecRef basis(int i) { return bas[i]; }
    Vec2<double> apply(const VecRef& v, int zslot) {
        a.v = v; a.zslot = zslot;
        launch(PH_APPLY);
        const double* s = fetch(2);
        return Vec2<double>{s[0], s[1]};
    }
    void jv(int cur, int zslot, double eps, int wslot, double* dots) {
        a.cur = cur; a.zslot = zslot; a.eps = eps; a.wslot = wslot; a.nb = wslot;
        for (int i = 0; i < wslot; ++i) a.basis[i] = bas[i];
        launch(PH_JV);
        const double* s = fetch(wslot + 1);
        for (int i = 0; i <= wslot; ++i) dots[i] = s[i];
    }
    void cgs(int wslot, int nb, const double* h, double* dots) {
        a.wslot = wslot; a.nb = nb;
        for (int i = 0; i < nb; ++i) { a.basis[i] = bas[i]; a.h[i] = h[i]; }
        launch(PH_CGS);
        const double* s = fetch(nb + 1);
        for (int i = 0; i <= nb; ++i) dots[i] = s[i];
    }
    void gm_begin(double beta) {
        g[0] = beta;
        for (int i = 1; i <= kMaxRestart; ++i) g[i] = 0.0;
    }
    double gm_probe(int j, const double* h, double hn) {
        return givens_column(H, kMaxRestart + 1, cs, sn, g, j, h, hn, false);
    }
    double gm_commit(int j, const double* h, double hn) {
        return givens_column(H, kMaxRestart + 1, cs, sn, g, j, h, hn, true);
    }
    void gm_solve(int k, double* y) { givens_solve(H, kMaxRestart + 1, g, k, y); }
    int direction(int k, const double* y, bool have_dx) {
        if (k == 1 && !have_dx) { implicit_dir = true; implicit_y = y[0]; return k; }
        a.nb = k; a.acc = have_dx ? 1 : 0;
        for (int i = 0; i < k; ++i) a.h[i] = y[i];
        launch(PH_LINCOMB);
        implicit_dir = false;
        return k;
    }
    VecRef dir_ref() {
        if (implicit_dir) return VecRef{Zb(0, 0), Zb(0, 1), implicit_y, implicit_y};
        return VecRef{dXb(0), dXb(1), 1.0, 1.0};
    }
    double restart_residual(int cur, double xnorm) {
        if (implicit_dir) {
            a.nb = 1; a.acc = 0; a.h[0] = implicit_y;
            launch(PH_LINCOMB);
            implicit_dir = false;
        }
        launch(PH_NORM_DX);
        const double dd = fetch(1)[0];
        if (!(dd > 0.0)) return 0.0;
        const double lam_fd = 6.0554544523933395e-06;
        a.cur = cur; a.zslot = -1; a.v = VecRef{dXb(0), dXb(1), 1.0, 1.0};
        a.eps = lam_fd * (lam_fd + xnorm / std::sqrt(dd));
        a.wslot = 0; a.nb = 0;
        launch(PH_JV);
        fetch(1);
        a.cur = cur;
        launch(PH_RES0);
        return std::sqrt(fetch(1)[0]);
    }
    Norms trial(int cur, int out, double lam) {
        a.cur = cur; a.out = out; a.lam = lam; a.v = dir_ref();
        launch(PH_TRIAL);
        const double* s = fetch(4);
        return Norms{s[0], s[1], s[2], s[3]};
    }
    Norms chord_trial(int cur, int out) {
        const int m = a.prm.m;
        a.cur = cur; a.out = out; a.lam = 1.0; a.v = VecRef{Vb(m, 0), Vb(m, 1), 1.0, 1.0};
        launch(PH_TRIAL);
        const double* s = fetch(4);
        return Norms{s[0], s[1], s[2], s[3]};
    }
    void finalize(const ColOutcome& o) {
        a.o = o;
        launch(PH_FINAL);
    }
};

template <int T, class FT, bool TAB>
int run_plain(jfnk_ctx* ctx, const jfnk_problem* p, jfnk_state* x, hipStream_t st) {
    SolverParams prm = make_params(ctx, p, x);
    // the batched schedule's placement of the block solve's intermediate, so
    // that both schedules run the same arithmetic
    int mmax = 1;
    for (int c = 0; c < p->ncols; ++c) mmax = std::max(mmax, (int)ctx->h_cols[c].M);
    const size_t lds_bytes = solve_lds<T, FT>(prm.prec_kind, mmax, &prm.dlds);
    const UserArrays U = make_user(ctx, p, x);
    HIP_OK(hipEventRecord(ctx->ev0, st));
    for (int c = 0; c < p->ncols; ++c) {
        HostExecT<T, FT, TAB> ex;
        ex.ctx = ctx;
        ex.st = st;
        ex.lds_bytes = lds_bytes;
        memset(&ex.a, 0, sizeof(ex.a));
        ex.a.W = ctx->W;
        ex.a.prm = prm;
        ex.a.U = U;
        ex.a.ci = c;
        ColOutcome o;
        jfnk_solve(ex, prm, o);
        if (ex.herr != hipSuccess) {
            ctx->poisoned = true;
            return fail(ctx, JFNK_EHIP, std::string("plain schedule: ") + hipGetErrorString(ex.herr));
        }
    }
    HIP_OK(hipEventRecord(ctx->ev1, st));
    ctx->timed = true;
    ctx->last_launches = -1;   // host-driven: many launches, span measured
    return JFNK_OK;
}

template <int T, class FT, bool TAB>
int run_batched(jfnk_ctx* ctx, const jfnk_problem* p, jfnk_state* x, hipStream_t st) {
    SolveArgs a;
    a.W = ctx->W;
    a.prm = make_params(ctx, p, x);
    int mmax = 1;
    for (int c = 0; c < p->ncols; ++c) mmax = std::max(mmax, (int)ctx->h_cols[c].M);
    const size_t lds_bytes = solve_lds<T, FT>(a.prm.prec_kind, mmax, &a.prm.dlds);
    a.U = make_user(ctx, p, x);
    a.order = ctx->d_order;
    a.mcol = ctx->d_mcol;
    a.ncols = p->ncols;
    HIP_OK(hipEventRecord(ctx->ev0, st));
    hipLaunchKernelGGL((k_gather<T, TAB>), dim3(ctx->nmove), dim3(kMoveThreads), 0, st, a);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(ctx->evg, st));
    hipLaunchKernelGGL((k_solve<T, FT, TAB>), dim3(p->ncols), dim3(T), lds_bytes, st, a);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(ctx->evs, st));
    hipLaunchKernelGGL((k_scatter<T>), dim3(ctx->nmove), dim3(kMoveThreads), 0, st, a);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(ctx->ev1, st));
    // the next step's workgroup order from this step's work
    hipLaunchKernelGGL(k_order, dim3(1), dim3(kOrderThreads), 0, st, (const ColState*)ctx->W.cst,
                       (const ColDesc*)ctx->W.cols, p->ncols, ctx->d_order);
    HIP_OK(hipGetLastError());
    ctx->timed = true;
    ctx->timed3 = true;
    ctx->last_launches = 3;
    return JFNK_OK;
}

template <class FT, bool TAB>
int dispatch_run_t(jfnk_ctx* ctx, const jfnk_problem* p, jfnk_state* x, hipStream_t st) {
    const bool plain = ctx->cfg.schedule == JFNK_SCHED_PLAIN;
    switch (ctx->Tsel) {
#define CASE_T(TT) \
    case TT: return plain ? run_plain<TT, FT, TAB>(ctx, p, x, st) : run_batched<TT, FT, TAB>(ctx, p, x, st);
        CASE_T(64) CASE_T(128) CASE_T(256) CASE_T(512)
#undef CASE_T
    default:
        return fail(ctx, JFNK_EINVAL, "unsupported workgroup size");
    }
}

template <class FT>
int dispatch_run(jfnk_ctx* ctx, const jfnk_problem* p, jfnk_state* x, hipStream_t st) {
    return p->table ? dispatch_run_t<FT, true>(ctx, p, x, st) : dispatch_run_t<FT, false>(ctx, p, x, st);
}

// phase runner for the test exports: column a.ci, or every column (a.all)
// with one workgroup each; the residual and J v phases run in kernels of
// their own
template <int T, class FT, bool TAB>
int run_phases(jfnk_ctx* ctx, hipStream_t st, PhaseArgs& a, const std::vector<int>& phases) {
    const dim3 grid(a.all ? (unsigned)a.ncols : 1u);
    for (int ph : phases) {
        a.phase = ph;
        if (ph == PH_EVAL)
            hipLaunchKernelGGL((k_phase<T, FT, TAB, PH_EVAL>), grid, dim3(T), Lds<T>::bytes(), st, a);
        else if (ph == PH_JV)
            hipLaunchKernelGGL((k_phase<T, FT, TAB, PH_JV>), grid, dim3(T), Lds<T>::bytes(), st, a);
        else
            hipLaunchKernelGGL((k_phase<T, FT, TAB>), grid, dim3(T), Lds<T>::bytes(), st, a);
        HIP_OK(hipGetLastError());
    }
    return JFNK_OK;
}

template <class FT>
int dispatch_phases(jfnk_ctx* ctx, hipStream_t st, PhaseArgs& a, const std::vector<int>& ph) {
    const bool tab = a.prm.tab.mu != nullptr;
    switch (ctx->Tsel) {
#define CASE_T(TT) \
    case TT: return tab ? run_phases<TT, FT, true>(ctx, st, a, ph) : run_phases<TT, FT, false>(ctx, st, a, ph);
        CASE_T(64) CASE_T(128) CASE_T(256) CASE_T(512)
#undef CASE_T
    default:
        return fail(ctx, JFNK_EINVAL, "unsupported workgroup size");
    }
}

int upload_schedule(jfnk_ctx* ctx, int ncols, hipStream_t st) {
    HIP_OK(hipMemcpyAsync(ctx->W.cols, ctx->h_cols, sizeof(ColDesc) * ncols, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->d_order, ctx->h_order, sizeof(int) * ncols, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->d_mcol, ctx->h_mcol, sizeof(int32_t) * ctx->nmove, hipMemcpyHostToDevice, st));
    return JFNK_OK;
}

// Validate and upload the schedule, unless the per-column inputs are the
// ones the resident schedule was built from (then only the pointers are checked).
// The per-column inputs are the ones the resident schedule was built from.
bool schedule_matches(const jfnk_ctx* ctx, const jfnk_problem* p) {
    if (!(p && ctx->sched_valid && p->ncols >= 1 && p->col_offset && p->length && p->dt && p->phi_left &&
          p->phi_right && p->eps_over_e && p->ne_left && p->ne_right && p->bc_left && p->bc_right &&
          (int)ctx->last_off.size() == p->ncols + 1 &&
          memcmp(ctx->last_off.data(), p->col_offset, sizeof(int64_t) * (p->ncols + 1)) == 0))
        return false;
    const double* srcs[7] = {p->length, p->dt, p->phi_left, p->phi_right, p->eps_over_e, p->ne_left,
                             p->ne_right};
    for (int k = 0; k < 7; ++k)
        if (memcmp(ctx->last_scal.data() + (size_t)k * p->ncols, srcs[k], sizeof(double) * p->ncols) != 0)
            return false;
    return memcmp(ctx->last_bc.data(), p->bc_left, sizeof(int32_t) * p->ncols) == 0 &&
           memcmp(ctx->last_bc.data() + p->ncols, p->bc_right, sizeof(int32_t) * p->ncols) == 0;
}

int schedule_cached(jfnk_ctx* ctx, const jfnk_problem* p, const jfnk_state* x, hipStream_t st) {
    if (!p || !x) return fail(ctx, JFNK_EINVAL, "null problem or state");
    {
        if (schedule_matches(ctx, p)) {
            if (const char* why = check_cells(p, x)) return fail(ctx, JFNK_EINVAL, why);
            return JFNK_OK;
        }
    }
    ctx->sched_valid = false;
    ctx->hist_valid = false;
    ctx->fac_reuse_ok = false;
    int rc = validate(ctx, p, x);
    if (rc) return rc;
    rc = upload_schedule(ctx, p->ncols, st);
    if (rc) return rc;
    ctx->last_off.assign(p->col_offset, p->col_offset + p->ncols + 1);
    ctx->last_scal.resize((size_t)7 * p->ncols);
    const double* srcs[7] = {p->length, p->dt, p->phi_left, p->phi_right, p->eps_over_e, p->ne_left, p->ne_right};
    for (int k = 0; k < 7; ++k) memcpy(ctx->last_scal.data() + (size_t)k * p->ncols, srcs[k], sizeof(double) * p->ncols);
    ctx->last_bc.assign(p->bc_left, p->bc_left + p->ncols);
    ctx->last_bc.insert(ctx->last_bc.end(), p->bc_right, p->bc_right + p->ncols);
    ctx->sched_valid = true;
    return JFNK_OK;
}

// Statistics of the step whose copy to h_cst was enqueued before evdone.
int gather_stats(jfnk_ctx* ctx, int ncols, jfnk_stats* stt, int* nfail) {
    HIP_OK(hipEventSynchronize(ctx->evdone));
    if (ctx->timed) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->last_ms = ms;
        ctx->timed = false;
        if (ctx->timed3) {
            float k0 = 0.0f, k1 = 0.0f, k2 = 0.0f;
            HIP_OK(hipEventElapsedTime(&k0, ctx->ev0, ctx->evg));
            HIP_OK(hipEventElapsedTime(&k1, ctx->evg, ctx->evs));
            HIP_OK(hipEventElapsedTime(&k2, ctx->evs, ctx->ev1));
            ctx->last_kms[0] = k0; ctx->last_kms[1] = k1; ctx->last_kms[2] = k2;
        } else {
            ctx->last_kms[0] = ctx->last_kms[1] = ctx->last_kms[2] = -1.0;
        }
        ctx->timed3 = false;
    }
    int bad = 0;
    for (int c = 0; c < ncols; ++c) {
        const ColState& s = ctx->h_cst[c];
        if (s.status != COL_CONVERGED) ++bad;
        if (stt) {
            if (stt->status) stt->status[c] = s.status;
            if (stt->newton_iters) stt->newton_iters[c] = s.newton;
            if (stt->gmres_iters) stt->gmres_iters[c] = s.gmres;
            if (stt->backtracks) stt->backtracks[c] = s.backtracks;
            if (stt->guess_used) stt->guess_used[c] = s.guess;
            if (stt->chord_steps) stt->chord_steps[c] = s.chords;
            if (stt->phase_counts)
                for (int i = 0; i < kWorkCounts; ++i) stt->phase_counts[(int64_t)c * kWorkCounts + i] = s.work[i];
            if (stt->res_scaled) stt->res_scaled[c] = s.res_inf;
            if (stt->mg_cycles) stt->mg_cycles[c] = s.mg_cycles;
        }
    }
    *nfail = bad;
    return JFNK_OK;
}

int check_ctx(jfnk_ctx* ctx) {
    if (!ctx) return JFNK_EINVAL;
    if (ctx->poisoned) return fail(ctx, JFNK_EHIP, "context poisoned by an earlier HIP error");
    return JFNK_OK;
}

// common set-up of the single-phase test exports
int prepare_test(jfnk_ctx* ctx, const jfnk_problem* p, const jfnk_state* x, hipStream_t st,
                 PhaseArgs& a) {
    if (int rc = drain(ctx)) return rc;
    ctx->sched_valid = false;
    ctx->hist_valid = false;
    ctx->learn_active = false;
    ctx->fac_reuse_ok = false;
    int rc = validate(ctx, p, x);
    if (rc) return rc;
    rc = upload_schedule(ctx, p->ncols, st);
    if (rc) return rc;
    memset(&a, 0, sizeof(a));
    a.W = ctx->W;
    jfnk_state xs = *x;
    xs.ne_prev = nullptr; xs.phi_prev = nullptr;
    a.prm = make_params(ctx, p, &xs);
    a.prm.guess = JFNK_GUESS_PREV;
    a.U = make_user(ctx, p, &xs);
    return JFNK_OK;
}

// phases in the context's precision (over every column when a.all)
int run_all(jfnk_ctx* ctx, hipStream_t st, PhaseArgs& a, const std::vector<int>& ph) {
    return ctx->cfg.prec_precision == JFNK_PREC_FP32 ? dispatch_phases<float>(ctx, st, a, ph)
                                                    : dispatch_phases<double>(ctx, st, a, ph);
}

// Learned candidate for the columns whose previous step on this layout
// needed Newton iterations (all columns without such a record).
int learned_guess(jfnk_ctx* ctx, const jfnk_problem* p, jfnk_state* x, hipStream_t st) {
    if (!p->temp) return fail(ctx, JFNK_EINVAL, "the learned guess needs the temperature field");
    const int nc = p->ncols;
    std::vector<uint8_t>& use = ctx->evaluated;
    use.assign(nc, 1);
    int nuse = nc;
    const uint64_t ver = net_version(ctx->model);
    // A step without X^{n-1} starts a new history of the columns (a new
    // episode from its start state): the records of earlier steps, and the
    // judgement of the network made on them, do not describe it.
    const bool fresh = x->ne_prev == nullptr;
    const bool have_hist = ctx->hist_valid && !fresh && (int)ctx->last_newton.size() == nc;
    if (have_hist && ctx->model_version != ver) {
        ctx->reject_streak.assign(nc, 0);
        ctx->skip_left.assign(nc, 0);
    }
    ctx->model_version = ver;
    if (have_hist) {
        // skip columns that converged at their initial guess last step, and
        // back off exponentially from columns whose learned candidate keeps
        // losing: after r losses in a row, the next 4^r - 1 chances (steps at
        // which the column would be evaluated) are skipped.  New weights
        // restart the judgement.
        nuse = 0;
        for (int c = 0; c < nc; ++c) {
            const bool settled = ctx->last_status[c] == COL_CONVERGED && ctx->last_newton[c] == 0;
            if (settled) {
                use[c] = 0;
            } else if (ctx->skip_left[c] > 0) {
                --ctx->skip_left[c];
                use[c] = 0;
            } else {
                use[c] = 1;
            }
            nuse += use[c];
        }
    } else {
        ctx->reject_streak.assign(nc, 0);
        ctx->skip_left.assign(nc, 0);
    }
    if (nuse == 0) return JFNK_OK;
    for (int c = 0; c < nc; ++c) ctx->h_lmask[c] = use[c];
    HIP_OK(hipMemcpyAsync(ctx->d_lmask, ctx->h_lmask, sizeof(int32_t) * nc, hipMemcpyHostToDevice, st));
    const int rc = net_predict_masked(ctx->model, p, x, use.data(), ctx->d_learn,
                                      ctx->d_learn + ctx->cfg.max_total_cells, st);
    if (rc) return fail(ctx, rc, std::string("learned guess: ") + jfnk_net_last_error(ctx->model));
    ctx->learn_active = true;
    return JFNK_OK;
}

void swap_slot(jfnk_ctx* ctx) {
    jfnk_ctx::Slot& a = ctx->alt;
    std::swap(ctx->h_cst, a.h_cst);
    std::swap(ctx->h_order, a.h_order);
    std::swap(ctx->h_lmask, a.h_lmask);
    std::swap(ctx->ev0, a.ev0);
    std::swap(ctx->evg, a.evg);
    std::swap(ctx->evs, a.evs);
    std::swap(ctx->ev1, a.ev1);
    std::swap(ctx->evdone, a.done);
    std::swap(ctx->evaluated, a.evaluated);
    std::swap(ctx->timed, a.timed);
    std::swap(ctx->timed3, a.timed3);
    std::swap(ctx->learned_ran, a.learned_ran);
    std::swap(ctx->last_launches, a.launches);
}

// Enqueue one step and the copy of its column statistics (evdone after it).
int step_enqueue(jfnk_ctx* ctx, const jfnk_problem* p, jfnk_state* x, hipStream_t st) {
    int rc = schedule_cached(ctx, p, x, st);
    if (rc) return rc;
    ctx->learn_active = false;
    if (ctx->cfg.guess == JFNK_GUESS_LEARNED) {
        rc = learned_guess(ctx, p, x, st);
        if (rc) return rc;
    }
    rc = ctx->cfg.prec_precision == JFNK_PREC_FP32 ? dispatch_run<float>(ctx, p, x, st)
                                                   : dispatch_run<double>(ctx, p, x, st);
    ctx->learned_ran = ctx->learn_active && (int)ctx->evaluated.size() == p->ncols;
    ctx->learn_active = false;
    if (rc) return rc;
    HIP_OK(hipMemcpyAsync(ctx->h_cst, ctx->W.cst, sizeof(ColState) * p->ncols, hipMemcpyDeviceToHost, st));
    HIP_OK(hipEventRecord(ctx->evdone, st));
    return JFNK_OK;
}

// Wait for the step whose resources are current, report its statistics and
// update the per-column history the next steps' decisions use.
int step_process(jfnk_ctx* ctx, int ncols, jfnk_stats* stt) {
    int nfail = 0;
    int rc = gather_stats(ctx, ncols, stt, &nfail);
    if (rc) return rc;
    const bool learned_ran = ctx->learned_ran && (int)ctx->evaluated.size() == ncols;
    if (stt && stt->phase_counts)
        for (int c = 0; c < ncols; ++c)
            stt->phase_counts[(int64_t)c * kWorkCounts + kWorkLearned] = learned_ran && ctx->evaluated[c] ? 1 : 0;
    // which columns needed Newton iterations (the learned guess is evaluated for those)
    ctx->last_newton.resize(ncols);
    ctx->last_status.resize(ncols);
    const bool learned = ctx->cfg.guess == JFNK_GUESS_LEARNED && (int)ctx->evaluated.size() == ncols &&
                         (int)ctx->reject_streak.size() == ncols;
    for (int c = 0; c < ncols; ++c) {
        ctx->last_newton[c] = ctx->h_cst[c].newton;
        ctx->last_status[c] = ctx->h_cst[c].status;
        if (learned && ctx->evaluated[c]) {
            if (ctx->h_cst[c].guess == JFNK_GUESS_LEARNED) {
                ctx->reject_streak[c] = 0;
            } else {
                ctx->reject_streak[c] = std::min(ctx->reject_streak[c] + 1, kMaxBackoff);
                ctx->skip_left[c] = (1 << (2 * ctx->reject_streak[c])) - 1;
            }
        }
    }
    ctx->hist_valid = true;
    ctx->fac_reuse_ok = true;
    return nfail ? JFNK_NOT_CONVERGED : JFNK_OK;
}

// Finish an asynchronous step still in flight.  Its statistics go to stt and
// its code (JFNK_OK or JFNK_NOT_CONVERGED) to *rc_out, each when not NULL;
// callers that pass neither drop them.
int drain(jfnk_ctx* ctx, jfnk_stats* stt, int32_t* rc_out) {
    if (!ctx->pending) return JFNK_OK;
    swap_slot(ctx);
    ctx->pending = false;
    const int rc = step_process(ctx, ctx->pending_ncols, stt);
    if (rc_out && (rc == JFNK_OK || rc == JFNK_NOT_CONVERGED)) *rc_out = rc;
    return rc == JFNK_NOT_CONVERGED ? JFNK_OK : rc;
}

}  // namespace

// ===========================================================================
// Allocation-free step: the whole workspace of one batched step lives in a
// file-scope device array, which every GPU the library runs on holds (at its
// own address) until the process ends.  Host code never passes the array's
// name to a kernel: it is a host-side stand-in there.  Its device address is
// taken once per device with hipGetSymbolAddress, that device current, and
// kept in g_scratch_ptr.
// ===========================================================================
static __device__ __align__(256) unsigned char scratch[JFNK_NOALLOC_BYTES];

namespace {

constexpr int kStaticMaxDevices = 64;
constexpr int kStaticMoveCap = 1024;    // gather / write-back workgroups of one step
void* g_scratch_ptr[kStaticMaxDevices];
std::mutex g_scratch_mu;

// Device address of this device's array (device current); nullptr on error.
void* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kStaticMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

__global__ __launch_bounds__(256) void k_clear(uint4* p, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

template <int T, class FT, bool TAB>
hipError_t static_launch(const SolveArgs& a0, int nmove, int ncols, int mmax, hipStream_t st) {
    SolveArgs a = a0;
    const size_t lds_bytes = solve_lds<T, FT>(a.prm.prec_kind, mmax, &a.prm.dlds);
    hipLaunchKernelGGL((k_gather<T, TAB>), dim3(nmove), dim3(kMoveThreads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_solve<T, FT, TAB>), dim3(ncols), dim3(T), lds_bytes, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_scatter<T>), dim3(nmove), dim3(kMoveThreads), 0, st, a);
    return hipGetLastError();
}

template <class FT, bool TAB>
hipError_t static_dispatch_t(int T, const SolveArgs& a, int nmove, int ncols, int mmax, hipStream_t st) {
    switch (T) {
    case 64: return static_launch<64, FT, TAB>(a, nmove, ncols, mmax, st);
    case 128: return static_launch<128, FT, TAB>(a, nmove, ncols, mmax, st);
    case 256: return static_launch<256, FT, TAB>(a, nmove, ncols, mmax, st);
    case 512: return static_launch<512, FT, TAB>(a, nmove, ncols, mmax, st);
    default: return hipErrorInvalidValue;
    }
}

template <class FT>
hipError_t static_dispatch(int T, const SolveArgs& a, int nmove, int ncols, int mmax, hipStream_t st) {
    return a.prm.tab.mu ? static_dispatch_t<FT, true>(T, a, nmove, ncols, mmax, st)
                        : static_dispatch_t<FT, false>(T, a, nmove, ncols, mmax, st);
}

int static_fail(char* err, size_t len, int code, const char* msg) {
    if (err && len > 0) snprintf(err, len, "%s", msg);
    return code;
}

}  // namespace

// ---------------------------------------------------------------------------
// MISDC step (Algorithm 1 and the SDC update of Section 3.1 around the
// electron/potential solve): one launch of the SDC terms per iteration, then
// the batched (or plain) JFNK step on the corrected problem.  Iteration k
// solves from X^n with f = n_e^n + dt s^(k) and ion charge n_i~; its Newton
// iteration starts from X^(k) by way of the extrapolated guess with
// X^{n-1} := 2 X^n - X^(k).
// ---------------------------------------------------------------------------
namespace {

template <bool TAB>
int misdc_launch(jfnk_ctx* ctx, const MisdcArgs& a, int ncols, int nmax, int k, hipStream_t st) {
    const dim3 grid(ncols, (nmax + 255) / 256);
    if (k < 0)
        hipLaunchKernelGGL(k_misdc_start<TAB>, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_misdc_iter<TAB>, grid, dim3(256), 0, st, a, k == 0 ? 1 : 0);
    HIP_OK(hipGetLastError());
    return JFNK_OK;
}

int misdc_alloc(jfnk_ctx* ctx) {
    if (ctx->mis) return JFNK_OK;
    hipError_t e = hipMalloc((void**)&ctx->mis, sizeof(double) * kMisdcArrays * ctx->capP);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_mis, sizeof(MisdcCol) * ctx->cfg.max_cols);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_mis, sizeof(MisdcCol) * ctx->cfg.max_cols, 0);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_vmax, sizeof(double) * ctx->cfg.max_cols);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_vmax, sizeof(double) * ctx->cfg.max_cols, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->mis) (void)hipFree(ctx->mis);
        if (ctx->d_mis) (void)hipFree(ctx->d_mis);
        if (ctx->h_mis) (void)hipHostFree(ctx->h_mis);
        if (ctx->d_vmax) (void)hipFree(ctx->d_vmax);
        ctx->mis = nullptr;
        ctx->d_mis = nullptr;
        ctx->h_mis = nullptr;
        ctx->d_vmax = nullptr;
        return fail(ctx, JFNK_ENOMEM, "MISDC workspace allocation failed");
    }
    return JFNK_OK;
}

// per-column statistics of one SDC iteration, summed into the step's
struct IterStats {
    std::vector<int32_t> status, newton, gmres, backtracks, guess, chords, phases, mg;
    std::vector<double> res;
    jfnk_stats view{};
    explicit IterStats(int n)
        : status(n), newton(n), gmres(n), backtracks(n), guess(n), chords(n), phases((size_t)n * kWorkCounts), mg(n),
          res(n) {
        view = {status.data(), newton.data(), gmres.data(), backtracks.data(), guess.data(), res.data(),
                chords.data(), phases.data(), mg.data()};
    }
};

void misdc_accumulate(const IterStats& it, int ncols, bool first, jfnk_stats* st) {
    if (!st) return;
    for (int c = 0; c < ncols; ++c) {
        if (st->status && (first || st->status[c] == JFNK_COL_CONVERGED)) st->status[c] = it.status[c];
        auto add = [&](int32_t* dst, int32_t v) { if (dst) dst[c] = first ? v : dst[c] + v; };
        add(st->newton_iters, it.newton[c]);
        add(st->gmres_iters, it.gmres[c]);
        add(st->backtracks, it.backtracks[c]);
        add(st->chord_steps, it.chords[c]);
        add(st->mg_cycles, it.mg[c]);
        if (st->phase_counts)
            for (int i = 0; i < kWorkCounts; ++i) {
                int32_t& d = st->phase_counts[(int64_t)c * kWorkCounts + i];
                d = (first ? 0 : d) + it.phases[(size_t)c * kWorkCounts + i];
            }
        if (st->guess_used && first) st->guess_used[c] = it.guess[c];
        if (st->res_scaled) st->res_scaled[c] = it.res[c];
    }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void jfnk_config_default(jfnk_config* cfg) {
    if (!cfg) return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->max_cols = 1;
    cfg->max_total_cells = 4096;
    cfg->max_cells_per_col = 4096;
    cfg->gmres_restart = 30;
    cfg->max_restarts = 5;
    cfg->max_newton = 50;
    cfg->max_backtracks = 10;
    cfg->tol_f = 1e-10;
    cfg->tol_x = 1e-10;
    cfg->gamma = 1e-4;
    cfg->ls_theta = 0.25;
    cfg->chord_tol = 1e-3;
    cfg->prec_precision = JFNK_PREC_FP32;
    cfg->guess = JFNK_GUESS_EXTRAP;
    cfg->schedule = JFNK_SCHED_BATCHED;
    cfg->threads_override = 0;
    cfg->prec_kind = JFNK_PRECK_BLOCK;
    cfg->mg_tol = 1e-4;
    cfg->mg_blocks = 3;
    cfg->mg_transfer = 1;
}

int jfnk_create(const jfnk_config* cfg, jfnk_ctx** out) {
    if (!out) return JFNK_EINVAL;
    *out = nullptr;
    if (!cfg) return JFNK_EINVAL;
    if (!config_valid(cfg)) return JFNK_EINVAL;
    jfnk_ctx* ctx = new (std::nothrow) jfnk_ctx();
    if (!ctx) return JFNK_ENOMEM;
    ctx->cfg = *cfg;
    if (hipGetDevice(&ctx->device) != hipSuccess) { delete ctx; return JFNK_EHIP; }
    const int Tcap = cfg->threads_override > 0 ? cfg->threads_override : kTmax;
    // a multiple of 64 cells: every workspace array then starts 512-byte aligned
    ctx->capP = (cfg->max_total_cells + (int64_t)cfg->max_cols * Tcap + 63) / 64 * 64;
    ctx->capRed = (int64_t)cfg->max_cols * Tcap * kRedPerChunk;
    const int64_t words = carve_work(nullptr, ctx->capP, cfg->gmres_restart, ctx->capRed, cfg->max_cols, nullptr,
                                     cfg->prec_kind == JFNK_PRECK_SCHUR_MG);
    hipError_t e = hipMalloc((void**)&ctx->base, sizeof(double) * words);
    if (e != hipSuccess) { (void)hipGetLastError(); delete ctx; return JFNK_ENOMEM; }
    carve(ctx);
    e = hipMalloc((void**)&ctx->d_order, sizeof(int) * cfg->max_cols);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_cols, sizeof(ColDesc) * cfg->max_cols, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_cst, sizeof(ColState) * cfg->max_cols, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_scal, sizeof(double) * kScalSlots * 2, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_order, sizeof(int) * cfg->max_cols, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->alt.h_cst, sizeof(ColState) * cfg->max_cols, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->alt.h_order, sizeof(int) * cfg->max_cols, 0);
    // gather / write-back tables: a column of M rows and T owners has ceil(M/8) T/8 tiles
    ctx->capMove = (ctx->capP + 8 * (int64_t)Tcap * cfg->max_cols) / (64 * kMoveTiles) + cfg->max_cols + 1;
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_mcol, sizeof(int32_t) * ctx->capMove);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_gflag, sizeof(int32_t) * ctx->capMove);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_mcol, sizeof(int32_t) * ctx->capMove, 0);
    if (e == hipSuccess) ctx->W.gflag = ctx->d_gflag;
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev0);
    if (e == hipSuccess) e = hipEventCreate(&ctx->ev1);
    if (e == hipSuccess) e = hipEventCreate(&ctx->evg);
    if (e == hipSuccess) e = hipEventCreate(&ctx->evs);
    if (e == hipSuccess) e = hipEventCreate(&ctx->evdone);
    if (e == hipSuccess) e = hipEventCreate(&ctx->alt.ev0);
    if (e == hipSuccess) e = hipEventCreate(&ctx->alt.ev1);
    if (e == hipSuccess) e = hipEventCreate(&ctx->alt.evg);
    if (e == hipSuccess) e = hipEventCreate(&ctx->alt.evs);
    if (e == hipSuccess) e = hipEventCreate(&ctx->alt.done);
    if (e != hipSuccess) { (void)hipGetLastError(); jfnk_destroy(ctx); return JFNK_ENOMEM; }
    // zero the whole workspace once: padding cells must read as zero
    e = hipMemset(ctx->base, 0, sizeof(double) * words);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { jfnk_destroy(ctx); return JFNK_EHIP; }
    *out = ctx;
    return JFNK_OK;
}

void jfnk_destroy(jfnk_ctx* ctx) {
    if (!ctx) return;
    if (ctx->pending && ctx->alt.done) (void)hipEventSynchronize(ctx->alt.done);   // step in flight
    if (ctx->base) (void)hipFree(ctx->base);
    if (ctx->d_order) (void)hipFree(ctx->d_order);
    if (ctx->d_mcol) (void)hipFree(ctx->d_mcol);
    if (ctx->d_gflag) (void)hipFree(ctx->d_gflag);
    if (ctx->h_mcol) (void)hipHostFree(ctx->h_mcol);
    if (ctx->h_cols) (void)hipHostFree(ctx->h_cols);
    if (ctx->h_cst) (void)hipHostFree(ctx->h_cst);
    if (ctx->h_scal) (void)hipHostFree(ctx->h_scal);
    if (ctx->h_order) (void)hipHostFree(ctx->h_order);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->evg) (void)hipEventDestroy(ctx->evg);
    if (ctx->evs) (void)hipEventDestroy(ctx->evs);
    if (ctx->d_learn) (void)hipFree(ctx->d_learn);
    if (ctx->d_lmask) (void)hipFree(ctx->d_lmask);
    if (ctx->h_lmask) (void)hipHostFree(ctx->h_lmask);
    if (ctx->evdone) (void)hipEventDestroy(ctx->evdone);
    if (ctx->mis) (void)hipFree(ctx->mis);
    if (ctx->d_mis) (void)hipFree(ctx->d_mis);
    if (ctx->h_mis) (void)hipHostFree(ctx->h_mis);
    if (ctx->d_vmax) (void)hipFree(ctx->d_vmax);
    if (ctx->h_vmax) (void)hipHostFree(ctx->h_vmax);
    jfnk_ctx::Slot& a = ctx->alt;
    if (a.h_cst) (void)hipHostFree(a.h_cst);
    if (a.h_order) (void)hipHostFree(a.h_order);
    if (a.h_lmask) (void)hipHostFree(a.h_lmask);
    for (hipEvent_t ev : {a.ev0, a.ev1, a.evg, a.evs, a.done})
        if (ev) (void)hipEventDestroy(ev);
    delete ctx;
}

int jfnk_last_timing(const jfnk_ctx* ctx, double* solve_ms, int32_t* launches) {
    if (!ctx || !solve_ms) return JFNK_EINVAL;
    *solve_ms = ctx->last_ms;
    if (launches) *launches = ctx->last_launches;
    return JFNK_OK;
}

int jfnk_last_kernel_times(const jfnk_ctx* ctx, double* ms3) {
    if (!ctx || !ms3) return JFNK_EINVAL;
    for (int k = 0; k < 3; ++k) ms3[k] = ctx->last_kms[k];
    return JFNK_OK;
}

const char* jfnk_last_error(const jfnk_ctx* ctx) {
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

int jfnk_step(jfnk_ctx* ctx, const jfnk_problem* p, jfnk_state* x, jfnk_stats* stt, void* stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (ctx->cfg.guess == JFNK_GUESS_LEARNED && !ctx->model)
        return fail(ctx, JFNK_EMODEL, "learned guess requested but no model is loaded");
    rc = drain(ctx);
    if (rc) return rc;
    rc = step_enqueue(ctx, p, x, (hipStream_t)stream);
    if (rc) return rc;
    return step_process(ctx, p->ncols, stt);
}

int jfnk_step_async(jfnk_ctx* ctx, const jfnk_problem* p, jfnk_state* x, jfnk_stats* prev_stats,
                    int32_t* prev_rc, void* stream) {
    if (prev_rc) *prev_rc = -1;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (ctx->cfg.guess == JFNK_GUESS_LEARNED && !ctx->model)
        return fail(ctx, JFNK_EMODEL, "learned guess requested but no model is loaded");
    if (ctx->cfg.schedule != JFNK_SCHED_BATCHED)
        return fail(ctx, JFNK_EINVAL, "asynchronous steps need the batched schedule");
    // a new layout rewrites the staged schedule, and a step on another stream
    // would not be ordered after it: finish the step in flight first (and
    // report it, as the enqueue below would have)
    if (ctx->pending && (!schedule_matches(ctx, p) || ctx->pending_stream != (hipStream_t)stream)) {
        rc = drain(ctx, prev_stats, prev_rc);
        if (rc) return rc;
    }
    rc = step_enqueue(ctx, p, x, (hipStream_t)stream);
    if (rc) return rc;
    ctx->fac_reuse_ok = true;      // the next step runs after this one on the stream
    // this step's resources move to the in-flight slot; those of the previous
    // step in flight (if any) come back to the current one
    swap_slot(ctx);
    if (ctx->pending) {
        // finish the previous step while this one runs
        const int n = ctx->pending_ncols;
        ctx->pending_ncols = p->ncols;
        ctx->pending_stream = (hipStream_t)stream;
        const int prc = step_process(ctx, n, prev_stats);
        if (prc != JFNK_OK && prc != JFNK_NOT_CONVERGED) return prc;
        if (prev_rc) *prev_rc = prc;
    } else {
        ctx->pending = true;
        ctx->pending_ncols = p->ncols;
        ctx->pending_stream = (hipStream_t)stream;
    }
    return JFNK_OK;
}

int jfnk_step_finish(jfnk_ctx* ctx, jfnk_stats* stt) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!ctx->pending) return fail(ctx, JFNK_EINVAL, "no asynchronous step in flight");
    swap_slot(ctx);
    ctx->pending = false;
    return step_process(ctx, ctx->pending_ncols, stt);
}

int jfnk_misdc_step(jfnk_ctx* ctx, const jfnk_problem* p, const jfnk_misdc* m, jfnk_state* x, jfnk_stats* stt,
                    void* stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!p || !m || !x) return fail(ctx, JFNK_EINVAL, "null problem, MISDC data or state");
    if (m->k_max < 1 || m->k_max > kMisdcMaxK) return fail(ctx, JFNK_EINVAL, "k_max must be in 1..64");
    if (!m->mu_ion || !m->k_rec || !m->n_ion) return fail(ctx, JFNK_EINVAL, "null ion array");
    if ((m->ac_amp == nullptr) != (m->ac_freq == nullptr))
        return fail(ctx, JFNK_EINVAL, "ac_amp and ac_freq must both be given or both NULL");
    if (p->k_loss) return fail(ctx, JFNK_EINVAL, "the MISDC step takes losses from its chemistry: k_loss must be NULL");
    if (m->electron_sdc != 0 && m->electron_sdc != 1) return fail(ctx, JFNK_EINVAL, "electron_sdc must be 0 or 1");
    if (!(m->cfl >= 0.0) || !std::isfinite(m->cfl)) return fail(ctx, JFNK_EINVAL, "cfl must be finite and >= 0");
    if (ctx->cfg.guess == JFNK_GUESS_LEARNED && !ctx->model)
        return fail(ctx, JFNK_EMODEL, "learned guess requested but no model is loaded");
    rc = drain(ctx);
    if (rc) return rc;
    rc = misdc_alloc(ctx);
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const int64_t P = ctx->capP;
    double* A = ctx->mis;
    double *Tn = A, *Rn = A + P, *S = A + 2 * P, *Q[2] = {A + 3 * P, A + 4 * P}, *PN = A + 5 * P, *PP = A + 6 * P;
    double *BN[2] = {A + 7 * P, A + 9 * P}, *BP[2] = {A + 8 * P, A + 10 * P};
    if (p->ncols < 1) return fail(ctx, JFNK_EINVAL, "ncols < 1");
    if (p->ncols > ctx->cfg.max_cols) return fail(ctx, JFNK_ECAPACITY, "ncols exceeds capacity");
    if (!p->src || !p->phi_right) return fail(ctx, JFNK_EINVAL, "null per-cell or per-column array");
    const int ncols = p->ncols;
    // the problem as every iteration passes it to the solve: validated before
    // the first launch unless it is the one the resident schedule was built from
    std::vector<double> phir1(p->phi_right, p->phi_right + ncols);
    jfnk_problem p2 = *p;
    p2.src = S;
    p2.q_ion = Q[0];
    p2.k_loss = nullptr;
    p2.phi_right = phir1.data();
    {
        jfnk_state xv = *x;
        if (schedule_matches(ctx, &p2)) {
            if (const char* why = check_cells(&p2, &xv)) return fail(ctx, JFNK_EINVAL, why);
        } else {
            ctx->sched_valid = false;
            rc = validate(ctx, &p2, &xv);
            if (rc) return rc;
        }
    }
    int nmax = 0;
    std::vector<double> dtv(p->dt, p->dt + ncols);
    for (int c = 0; c < ncols; ++c) {
        MisdcCol& mc = ctx->h_mis[c];
        mc.off = p->col_offset[c];
        mc.foff = p->col_offset[c] + c;
        mc.n = (int32_t)(p->col_offset[c + 1] - p->col_offset[c]);
        mc.bcl = p->bc_left[c];
        mc.bcr = p->bc_right[c];
        mc.pad = 0;
        mc.h = p->length[c] / mc.n;
        mc.dt = p->dt[c];
        mc.nel = p->ne_left[c];
        mc.ner = p->ne_right[c];
        mc.phil = p->phi_left[c];
        const double amp = m->ac_amp ? m->ac_amp[c] : 0.0, fr = m->ac_freq ? m->ac_freq[c] : 0.0;
        const double t0 = m->t ? m->t[c] : 0.0;
        if (!std::isfinite(amp) || !std::isfinite(fr) || !std::isfinite(t0))
            return fail(ctx, JFNK_EINVAL, "non-finite start time, AC amplitude or frequency");
        mc.phir_n = p->phi_right[c] + amp * std::sin(2.0 * M_PI * fr * t0);
        nmax = std::max(nmax, mc.n);
    }
    if ((nmax + 255) / 256 > 65535) return fail(ctx, JFNK_ECAPACITY, "column too long for the MISDC launch");
    MisdcArgs a{};
    a.cols = ctx->d_mis;
    a.mu = p->mu; a.diff = p->diff; a.src = p->src; a.mu_i = m->mu_ion; a.k_rec = m->k_rec;
    a.uface = p->u_face; a.prog = p->prog; a.gasn = p->gas_n; a.tab = tab_of(p);
    a.ne0 = x->ne; a.phi0 = x->phi; a.ni0 = m->n_ion;
    a.Tn = Tn; a.Rn = Rn; a.s = S; a.pn = PN; a.pp = PP;
    a.vmax = ctx->d_vmax;
    a.esdc = m->electron_sdc;
    if (m->cfl > 0.0) {
        // the step from the start-of-step drift speeds (NaN speeds keep p->dt;
        // the solve then flags the column's non-finite inputs)
        HIP_OK(hipMemcpyAsync(ctx->d_mis, ctx->h_mis, sizeof(MisdcCol) * ncols, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_misdc_vmax, dim3(ncols), dim3(256), 0, st, a);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(ctx->h_vmax, ctx->d_vmax, sizeof(double) * ncols, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        for (int c = 0; c < ncols; ++c) {
            const double h = p->length[c] / (double)(p->col_offset[c + 1] - p->col_offset[c]);
            const double vm = ctx->h_vmax[c];
            if (vm > 0.0 && std::isfinite(vm)) dtv[c] = std::min(p->dt[c], m->cfl * h / vm);
        }
    }
    for (int c = 0; c < ncols; ++c) {
        MisdcCol& mc = ctx->h_mis[c];
        const double amp = m->ac_amp ? m->ac_amp[c] : 0.0, fr = m->ac_freq ? m->ac_freq[c] : 0.0;
        const double t0 = m->t ? m->t[c] : 0.0;
        mc.dt = dtv[c];
        mc.phir_1 = p->phi_right[c] + amp * std::sin(2.0 * M_PI * fr * (t0 + mc.dt));
        phir1[c] = mc.phir_1;
        if (m->dt_used) m->dt_used[c] = dtv[c];
    }
    p2.dt = dtv.data();
    // (h_mis is not rewritten before the call's final synchronisation)
    HIP_OK(hipMemcpyAsync(ctx->d_mis, ctx->h_mis, sizeof(MisdcCol) * ncols, hipMemcpyHostToDevice, st));
    const bool tab = p->table != nullptr;
    rc = tab ? misdc_launch<true>(ctx, a, ncols, nmax, -1, st) : misdc_launch<false>(ctx, a, ncols, nmax, -1, st);
    if (rc) return rc;
    const int32_t guess0 = ctx->cfg.guess;
    IterStats it(ncols);
    std::vector<uint8_t> bad(ncols, 0);    // flagged bad input by some iteration's solve
    int worst = JFNK_OK;
    for (int k = 0; k < m->k_max; ++k) {
        const int cur = k & 1, nxt = (k + 1) & 1;
        a.nek = k == 0 ? x->ne : BN[cur];
        a.phik = k == 0 ? x->phi : BP[cur];
        a.nik = k == 0 ? m->n_ion : Q[nxt];
        a.q = Q[cur];
        rc = tab ? misdc_launch<true>(ctx, a, ncols, nmax, k, st) : misdc_launch<false>(ctx, a, ncols, nmax, k, st);
        if (rc) return rc;
        p2.q_ion = Q[cur];
        jfnk_state x2{};
        x2.ne = x->ne;
        x2.phi = x->phi;
        x2.ne_prev = k == 0 ? x->ne_prev : PN;
        x2.phi_prev = k == 0 ? x->phi_prev : PP;
        const bool last = k == m->k_max - 1;
        x2.ne_out = last ? x->ne_out : BN[nxt];
        x2.phi_out = last ? x->phi_out : BP[nxt];
        ctx->cfg.guess = k == 0 ? guess0 : JFNK_GUESS_EXTRAP;
        rc = step_enqueue(ctx, &p2, &x2, st);
        if (rc == JFNK_OK) rc = step_process(ctx, ncols, &it.view);
        ctx->cfg.guess = guess0;
        if (rc < 0) return rc;
        if (rc == JFNK_NOT_CONVERGED) worst = JFNK_NOT_CONVERGED;
        for (int c = 0; c < ncols; ++c) bad[c] |= it.status[c] == JFNK_COL_BAD_INPUT;
        misdc_accumulate(it, ncols, k == 0, stt);
    }
    // n_i^n+1 = the last n_i~, except in columns flagged bad input (runs of
    // the other columns copied at once)
    const double* qf = Q[(m->k_max - 1) & 1];
    for (int c = 0; c < ncols;) {
        const bool keep = bad[c] != 0;
        int e = c + 1;
        while (e < ncols && (bad[e] != 0) == keep) ++e;
        if (!keep)
            HIP_OK(hipMemcpyAsync(m->n_ion + p->col_offset[c], qf + p->col_offset[c],
                                  sizeof(double) * (p->col_offset[e] - p->col_offset[c]), hipMemcpyDeviceToDevice, st));
        c = e;
    }
    HIP_OK(hipStreamSynchronize(st));
    return worst;
}

int jfnk_autotune(jfnk_ctx* ctx, const jfnk_problem* p, const jfnk_state* x, int32_t steps,
                  int32_t* chosen, double* times_ms, void* stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!p || !x || !x->ne || !x->phi || !p->col_offset || p->ncols < 1 || steps < 1)
        return fail(ctx, JFNK_EINVAL, "autotune: bad arguments");
    if (ctx->cfg.schedule != JFNK_SCHED_BATCHED || ctx->cfg.threads_override != 0)
        return fail(ctx, JFNK_EINVAL, "autotune: needs the batched schedule and no threads_override");
    rc = drain(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t total = p->col_offset[p->ncols];
    if (total < 1 || total > ctx->cfg.max_total_cells) return fail(ctx, JFNK_ECAPACITY, "autotune: capacity");
    int nmax = 0;
    for (int c = 0; c < p->ncols; ++c) nmax = std::max(nmax, (int)(p->col_offset[c + 1] - p->col_offset[c]));
    // scratch state: current, previous and a save slot (ne, phi each)
    double* buf = nullptr;
    HIP_OK(hipMalloc((void**)&buf, sizeof(double) * 6 * total));
    double *cn = buf, *cp = buf + total, *pn = buf + 2 * total, *pp = buf + 3 * total;
    double *sn = buf + 4 * total, *sp = buf + 5 * total;
    const int saved_guess = ctx->cfg.guess;
    if (ctx->cfg.guess == JFNK_GUESS_LEARNED) ctx->cfg.guess = JFNK_GUESS_EXTRAP;
    const int cand[4] = {64, 128, 256, 512};
    double best_ms = INFINITY;
    int best = 0;
    for (int k = 0; k < 4 && rc == JFNK_OK; ++k) {
        const int T = cand[k];
        if (times_ms) times_ms[k] = -1.0;
        // at most 64 cells per thread (the largest size is always tried: it
        // is the only one for columns longer than 64 kTmax cells)
        if (T > kTmax || (T < kTmax && (nmax + T - 1) / T > 64) || (T > 64 && nmax <= T / 2)) continue;
        ctx->force_T = T;
        ctx->sched_valid = false;
        const size_t nb = sizeof(double) * total;
        if (hipMemcpyAsync(cn, x->ne, nb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(cp, x->phi, nb, hipMemcpyDeviceToDevice, st) != hipSuccess) { rc = JFNK_EHIP; break; }
        bool have_prev = x->ne_prev && x->phi_prev;
        if (have_prev && (hipMemcpyAsync(pn, x->ne_prev, nb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                          hipMemcpyAsync(pp, x->phi_prev, nb, hipMemcpyDeviceToDevice, st) != hipSuccess)) {
            rc = JFNK_EHIP;
            break;
        }
        double ms = 0.0;
        for (int s = 0; s < steps && rc == JFNK_OK; ++s) {
            if (hipMemcpyAsync(sn, cn, nb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(sp, cp, nb, hipMemcpyDeviceToDevice, st) != hipSuccess) { rc = JFNK_EHIP; break; }
            jfnk_state xs{cn, cp, have_prev ? pn : nullptr, have_prev ? pp : nullptr};
            rc = jfnk_step(ctx, p, &xs, nullptr, stream);
            if (rc == JFNK_NOT_CONVERGED) rc = JFNK_OK;
            if (rc) break;
            ms += ctx->last_ms;
            std::swap(pn, sn);
            std::swap(pp, sp);
            have_prev = true;
        }
        if (rc) break;
        if (times_ms) times_ms[k] = ms;
        if (ms < best_ms) { best_ms = ms; best = T; }
    }
    ctx->force_T = 0;
    ctx->cfg.guess = saved_guess;
    ctx->sched_valid = false;
    ctx->hist_valid = false;
    ctx->fac_reuse_ok = false;
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (rc) return rc == JFNK_EHIP ? fail(ctx, rc, "autotune: HIP copy failed") : rc;
    ctx->tuned_T = best;
    ctx->tuned_off.assign(p->col_offset, p->col_offset + p->ncols + 1);
    jfnk_ctx::TuneEntry te{};
    te.hash = layout_hash(p->col_offset, p->ncols + 1);
    te.ncols = p->ncols;
    te.table = p->table ? 1 : 0;
    te.T = best;
    te.total = total;
    te.mine = true;
    for (int k = 0; k < 4; ++k) te.ms[k] = times_ms ? times_ms[k] : -1.0;
    ctx->tune_table.push_back(te);
    if (chosen) *chosen = best;
    return JFNK_OK;
}

int jfnk_autotune_save(jfnk_ctx* ctx, const char* path) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!path) return fail(ctx, JFNK_EINVAL, "autotune_save: null path");
    FILE* f = fopen(path, "a");
    if (!f) return fail(ctx, JFNK_EINVAL, std::string("autotune_save: cannot open ") + path);
    const std::string arch = device_arch();
    for (const auto& e : ctx->tune_table) {
        if (!e.mine) continue;
        fprintf(f, "jfnk-autotune v1 %s %d %d %d %d %lld %016llx %d %.6g %.6g %.6g %.6g\n", arch.c_str(),
                ctx->cfg.prec_precision, ctx->cfg.prec_kind, e.table, e.ncols, (long long)e.total,
                (unsigned long long)e.hash, e.T, e.ms[0], e.ms[1], e.ms[2], e.ms[3]);
    }
    const bool ok = fclose(f) == 0;
    if (!ok) return fail(ctx, JFNK_EINVAL, std::string("autotune_save: write failed: ") + path);
    return JFNK_OK;
}

int jfnk_autotune_load(jfnk_ctx* ctx, const char* path, int32_t* nloaded) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!path) return fail(ctx, JFNK_EINVAL, "autotune_load: null path");
    FILE* f = fopen(path, "r");
    if (!f) return fail(ctx, JFNK_EINVAL, std::string("autotune_load: cannot open ") + path);
    const std::string arch = device_arch();
    char line[512];
    int n = 0;
    while (fgets(line, sizeof(line), f)) {
        char a[160];
        int prec, kind, table, ncols, T;
        long long total;
        unsigned long long hash;
        double ms[4];
        if (sscanf(line, "jfnk-autotune v1 %159s %d %d %d %d %lld %llx %d %lf %lf %lf %lf", a, &prec, &kind, &table,
                   &ncols, &total, &hash, &T, &ms[0], &ms[1], &ms[2], &ms[3]) != 12)
            continue;
        if (arch != a || prec != ctx->cfg.prec_precision || kind != ctx->cfg.prec_kind) continue;
        if (ncols < 1 || total < 1 || (table != 0 && table != 1) || (T != 64 && T != 128 && T != 256 && T != 512))
            continue;
        jfnk_ctx::TuneEntry e{};
        e.hash = (uint64_t)hash;
        e.ncols = ncols;
        e.table = table;
        e.T = T;
        e.total = total;
        e.mine = false;
        for (int k = 0; k < 4; ++k) e.ms[k] = ms[k];
        ctx->tune_table.push_back(e);
        ++n;
    }
    fclose(f);
    ctx->sched_valid = false;
    if (nloaded) *nloaded = n;
    return JFNK_OK;
}

int jfnk_schedule_threads(jfnk_ctx* ctx, const jfnk_problem* p, int32_t* threads) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!p || !p->col_offset || p->ncols < 1 || !threads) return fail(ctx, JFNK_EINVAL, "schedule_threads: bad arguments");
    int nmax = 0;
    for (int c = 0; c < p->ncols; ++c) nmax = std::max(nmax, (int)(p->col_offset[c + 1] - p->col_offset[c]));
    *threads = ctx->cfg.threads_override > 0 ? ctx->cfg.threads_override : step_threads(ctx, p, nmax);
    return JFNK_OK;
}

int jfnk_set_model(jfnk_ctx* ctx, jfnk_net* net) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    rc = drain(ctx);
    if (rc) return rc;
    if (!net) {
        ctx->model = nullptr;
        return JFNK_OK;
    }
    HIP_OK(hipSetDevice(ctx->device));
    rc = net_ensure_predict_capacity(net, ctx->cfg.max_cols, ctx->cfg.max_total_cells);
    if (rc) return fail(ctx, rc, std::string("model: ") + jfnk_net_last_error(net));
    if (!ctx->d_learn) {
        HIP_OK(hipMalloc((void**)&ctx->d_learn, sizeof(double) * 2 * ctx->cfg.max_total_cells));
        HIP_OK(hipMalloc((void**)&ctx->d_lmask, sizeof(int32_t) * ctx->cfg.max_cols));
        HIP_OK(hipHostMalloc((void**)&ctx->h_lmask, sizeof(int32_t) * ctx->cfg.max_cols, 0));
        HIP_OK(hipHostMalloc((void**)&ctx->alt.h_lmask, sizeof(int32_t) * ctx->cfg.max_cols, 0));
        HIP_OK(hipMemset(ctx->d_lmask, 0, sizeof(int32_t) * ctx->cfg.max_cols));
        HIP_OK(hipDeviceSynchronize());
        ctx->W.lmask = ctx->d_lmask;
    }
    ctx->model = net;
    ctx->hist_valid = false;
    return JFNK_OK;
}

int jfnk_eval_residual(jfnk_ctx* ctx, const jfnk_problem* p, const jfnk_state* x, const double* x_ne,
                       const double* x_phi, double* fe, double* fp, double* scal, void* stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!x_ne || !x_phi || !fe || !fp) return fail(ctx, JFNK_EINVAL, "null array");
    hipStream_t st = (hipStream_t)stream;
    PhaseArgs a;
    rc = prepare_test(ctx, p, x, st, a);
    if (rc) return rc;
    a.in0 = x_ne; a.in1 = x_phi; a.out0 = fe; a.out1 = fp; a.cur = 1;
    a.all = 1; a.ncols = p->ncols; a.order = ctx->d_order;
    rc = run_all(ctx, st, a, {PH_SETUP, PH_LOAD_X, PH_EVAL, PH_STORE_F});
    if (rc) return rc;
    if (scal) {
        HIP_OK(hipMemcpyAsync(ctx->h_cst, ctx->W.cst, sizeof(ColState) * p->ncols, hipMemcpyDeviceToHost, st));
    }
    HIP_OK(hipStreamSynchronize(st));
    if (scal)
        for (int c = 0; c < p->ncols; ++c) {
            scal[4 * c + 0] = ctx->h_cst[c].sfn; scal[4 * c + 1] = ctx->h_cst[c].sfp;
            scal[4 * c + 2] = ctx->h_cst[c].sxn; scal[4 * c + 3] = ctx->h_cst[c].sxp;
        }
    return JFNK_OK;
}

int jfnk_eval_jv(jfnk_ctx* ctx, const jfnk_problem* p, const jfnk_state* x, const double* x_ne,
                 const double* x_phi, const double* v_ne, const double* v_phi, double* w_ne,
                 double* w_phi, void* stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!x_ne || !x_phi || !v_ne || !v_phi || !w_ne || !w_phi) return fail(ctx, JFNK_EINVAL, "null array");
    hipStream_t st = (hipStream_t)stream;
    PhaseArgs a;
    rc = prepare_test(ctx, p, x, st, a);
    if (rc) return rc;
    // every column at once: set up, X into buffer 1 and F(X) (||S_X^-1 X||^2
    // left in scal[2]), v into Z[0], ||v||^2 into scal[0] through the dX norm
    // phase (v copied into dX by a one-term lincomb), then w = J v with the
    // step formed from the two norms on the device
    a.all = 1; a.ncols = p->ncols; a.order = ctx->d_order;
    a.cur = 1; a.in0 = x_ne; a.in1 = x_phi;
    rc = run_all(ctx, st, a, {PH_SETUP, PH_LOAD_X, PH_EVAL});
    if (rc) return rc;
    a.zslot = 0; a.in0 = v_ne; a.in1 = v_phi;
    a.nb = 1; a.acc = 0; a.h[0] = 1.0;
    rc = run_all(ctx, st, a, {PH_LOAD_V, PH_LINCOMB, PH_NORM_DX});
    if (rc) return rc;
    a.cur = 1; a.zslot = 0; a.wslot = 1; a.nb = 0; a.eps_dev = 1;
    a.out0 = w_ne; a.out1 = w_phi;
    rc = run_all(ctx, st, a, {PH_JV, PH_STORE_W});
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(st));
    return JFNK_OK;
}

int jfnk_block_solve(jfnk_ctx* ctx, const jfnk_problem* p, const jfnk_state* x, const double* x_ne,
                     const double* x_phi, const double* r_ne, const double* r_phi, double* z_ne,
                     double* z_phi, void* stream) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!x_ne || !x_phi || !r_ne || !r_phi || !z_ne || !z_phi) return fail(ctx, JFNK_EINVAL, "null array");
    hipStream_t st = (hipStream_t)stream;
    PhaseArgs a;
    rc = prepare_test(ctx, p, x, st, a);
    if (rc) return rc;
    // every column at once: set up, X into buffer 1, factor; r into Z[0];
    // z = P^-1 r into Z[1]; z back to the caller
    a.all = 1; a.ncols = p->ncols; a.order = ctx->d_order;
    a.cur = 1; a.in0 = x_ne; a.in1 = x_phi;
    rc = run_all(ctx, st, a, {PH_SETUP, PH_LOAD_X, PH_FACTOR});
    if (rc) return rc;
    a.zslot = 0; a.in0 = r_ne; a.in1 = r_phi;
    rc = run_all(ctx, st, a, {PH_LOAD_V});
    if (rc) return rc;
    a.v = VecRef{CP{ctx->W.Z}, CP{ctx->W.Z + 1}, 1.0, 1.0};
    a.zslot = 1; a.out0 = z_ne; a.out1 = z_phi;
    rc = run_all(ctx, st, a, {PH_APPLY, PH_STORE_V});
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(st));
    return JFNK_OK;
}

int jfnk_step_noalloc(const jfnk_config* cfg, const jfnk_problem* p, jfnk_state* x, jfnk_stats* stt,
                      void* stream, char* err, size_t err_len) {
    if (err && err_len > 0) err[0] = '\0';
    if (!cfg || !p || !x) return static_fail(err, err_len, JFNK_EINVAL, "null config, problem or state");
    if (!config_valid(cfg)) return static_fail(err, err_len, JFNK_EINVAL, "invalid configuration");
    if (cfg->guess == JFNK_GUESS_LEARNED)
        return static_fail(err, err_len, JFNK_EINVAL, "the learned guess needs a context (jfnk_set_model)");
    if (p->ncols < 1) return static_fail(err, err_len, JFNK_EINVAL, "ncols < 1");
    if (p->ncols > JFNK_NOALLOC_MAX_COLS)
        return static_fail(err, err_len, JFNK_ECAPACITY, "more columns than JFNK_NOALLOC_MAX_COLS");
    if (!p->col_offset || !p->length || !p->dt || !p->phi_left || !p->phi_right || !p->eps_over_e ||
        !p->bc_left || !p->bc_right || !p->ne_left || !p->ne_right)
        return static_fail(err, err_len, JFNK_EINVAL, "null per-column array");
    if (const char* why = check_cells(p, x)) return static_fail(err, err_len, JFNK_EINVAL, why);
    if (p->col_offset[0] != 0) return static_fail(err, err_len, JFNK_EINVAL, "col_offset[0] != 0");
    const int nc = p->ncols;
    int nmax = 0;
    for (int c = 0; c < nc; ++c) {
        const int64_t n = p->col_offset[c + 1] - p->col_offset[c];
        if (n < 3) return static_fail(err, err_len, JFNK_EINVAL, "column with fewer than 3 cells");
        if (n > cfg->max_cells_per_col) return static_fail(err, err_len, JFNK_ECAPACITY, "column longer than max_cells_per_col");
        nmax = std::max<int>(nmax, (int)n);
        const double v[7] = {p->length[c], p->dt[c], p->phi_left[c], p->phi_right[c], p->eps_over_e[c],
                             p->ne_left[c], p->ne_right[c]};
        for (double d : v)
            if (!std::isfinite(d)) return static_fail(err, err_len, JFNK_EINVAL, "non-finite per-column scalar");
        if (!(p->length[c] > 0.0) || !(p->dt[c] > 0.0) || !(p->eps_over_e[c] > 0.0))
            return static_fail(err, err_len, JFNK_EINVAL, "length, dt and eps_over_e must be > 0");
        if ((p->bc_left[c] != 0 && p->bc_left[c] != 1) || (p->bc_right[c] != 0 && p->bc_right[c] != 1))
            return static_fail(err, err_len, JFNK_EINVAL, "bad boundary condition code");
    }
    // the schedule of jfnk_step's batched path (workgroup size by the size
    // rule or threads_override; longest columns first), in host stack arrays
    const int T = choose_T(*cfg, nmax);
    ColDesc cols[JFNK_NOALLOC_MAX_COLS];
    int order[JFNK_NOALLOC_MAX_COLS];
    int32_t mcol[kStaticMoveCap];
    int64_t ws = 0, red = 0;
    for (int c = 0; c < nc; ++c) {
        const int n = (int)(p->col_offset[c + 1] - p->col_offset[c]);
        const int M = (n + T - 1) / T;
        ColDesc& d = cols[c];
        memset(&d, 0, sizeof(d));
        d.n = n; d.M = M; d.bcl = p->bc_left[c]; d.bcr = p->bc_right[c];
        d.index = c; d.T = T;
        d.uoff = p->col_offset[c]; d.ws = ws; d.red = red;
        d.h = p->length[c] / n; d.dt = p->dt[c];
        d.phil = p->phi_left[c]; d.phir = p->phi_right[c];
        d.eps = p->eps_over_e[c]; d.nel = p->ne_left[c]; d.ner = p->ne_right[c];
        ws += (int64_t)T * M;
        red += (int64_t)T * kRedPerChunk;
        // insertion into the order by cells, longest first (stable)
        int k = c;
        while (k > 0 && cols[order[k - 1]].n < n) { order[k] = order[k - 1]; --k; }
        order[k] = c;
    }
    int nmove = 0;
    for (int i = 0; i < nc; ++i) {
        ColDesc& d = cols[order[i]];
        const int tiles = ((d.M + 7) / 8) * (T / 8);
        const int gn = (tiles + kMoveTiles - 1) / kMoveTiles;
        if (nmove + gn > kStaticMoveCap)
            return static_fail(err, err_len, JFNK_ECAPACITY, "problem exceeds the allocation-free step's capacity");
        d.g0 = nmove; d.gn = gn;
        for (int k = 0; k < gn; ++k) mcol[nmove + k] = order[i];
        nmove += gn;
    }
    // bytes: the workspace (as jfnk_create lays it out), then the work order,
    // the write-back table and the gather flags, each 256-byte aligned
    auto up256 = [](int64_t b) { return (b + 255) / 256 * 256; };
    const bool mg = cfg->prec_kind == JFNK_PRECK_SCHUR_MG;
    const int64_t wbytes = up256(8 * carve_work(nullptr, ws, cfg->gmres_restart, red, nc, nullptr, mg));
    const int64_t obytes = up256(sizeof(int) * (int64_t)nc);
    const int64_t mbytes = up256(sizeof(int32_t) * (int64_t)nmove);
    const int64_t total = wbytes + obytes + 2 * mbytes;
    if (total > (int64_t)JFNK_NOALLOC_BYTES)
        return static_fail(err, err_len, JFNK_ECAPACITY,
                           "problem exceeds the allocation-free step's capacity (JFNK_NOALLOC_BYTES)");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return static_fail(err, err_len, JFNK_EHIP, "hipGetDevice failed");
    unsigned char* base = (unsigned char*)scratch_ptr(dev);
    if (!base) return static_fail(err, err_len, JFNK_EHIP, "hipGetSymbolAddress of the scratch array failed");
    hipStream_t st = (hipStream_t)stream;
    Work W{};
    carve_work((double*)base, ws, cfg->gmres_restart, red, nc, &W, mg);
    int* d_order = (int*)(base + wbytes);
    int32_t* d_mcol = (int32_t*)(base + wbytes + obytes);
    W.gflag = (int32_t*)(base + wbytes + obytes + mbytes);
    W.lmask = nullptr;
    // the array keeps the last call's contents: clear what this step uses
    // (padding cells must read as zero), with a kernel, not a memset node
    const int64_t n16 = total / 16;
    const int nb = (int)std::min<int64_t>((n16 + 255) / 256, 2048);
    hipLaunchKernelGGL(k_clear, dim3(nb), dim3(256), 0, st, (uint4*)base, n16);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(W.cols, cols, sizeof(ColDesc) * nc, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_order, order, sizeof(int) * nc, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_mcol, mcol, sizeof(int32_t) * nmove, hipMemcpyHostToDevice, st);
    SolveArgs a;
    a.W = W;
    a.prm = params_of(*cfg, p, x, false, false);
    a.U = UserArrays{};
    a.U.mu = p->mu; a.U.diff = p->diff; a.U.src = p->src; a.U.kloss = p->k_loss; a.U.q = p->q_ion;
    a.U.uface = p->u_face;
    a.U.ne = x->ne; a.U.phi = x->phi;
    a.U.ne_out = x->ne_out ? x->ne_out : x->ne;
    a.U.phi_out = x->phi_out ? x->phi_out : x->phi;
    a.U.ne_prev = x->ne_prev; a.U.phi_prev = x->phi_prev;
    a.U.prog = p->prog; a.U.gasn = p->gas_n;
    a.order = d_order;
    a.mcol = d_mcol;
    a.ncols = nc;
    int mmax = 1;
    for (int c = 0; c < nc; ++c) mmax = std::max(mmax, (int)cols[c].M);
    if (e == hipSuccess)
        e = cfg->prec_precision == JFNK_PREC_FP32 ? static_dispatch<float>(T, a, nmove, nc, mmax, st)
                                                  : static_dispatch<double>(T, a, nmove, nc, mmax, st);
    ColState hcst[JFNK_NOALLOC_MAX_COLS];
    if (e == hipSuccess) e = hipMemcpyAsync(hcst, W.cst, sizeof(ColState) * nc, hipMemcpyDeviceToHost, st);
    // the host arrays above live on this call's stack: wait before returning
    const hipError_t es = hipStreamSynchronize(st);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return static_fail(err, err_len, JFNK_EHIP, hipGetErrorString(e));
    int bad = 0;
    for (int c = 0; c < nc; ++c) {
        const ColState& s = hcst[c];
        if (s.status != COL_CONVERGED) ++bad;
        if (!stt) continue;
        if (stt->status) stt->status[c] = s.status;
        if (stt->newton_iters) stt->newton_iters[c] = s.newton;
        if (stt->gmres_iters) stt->gmres_iters[c] = s.gmres;
        if (stt->backtracks) stt->backtracks[c] = s.backtracks;
        if (stt->guess_used) stt->guess_used[c] = s.guess;
        if (stt->chord_steps) stt->chord_steps[c] = s.chords;
        if (stt->phase_counts)
            for (int i = 0; i < kWorkCounts; ++i)
                stt->phase_counts[(int64_t)c * kWorkCounts + i] = i == kWorkLearned ? 0 : s.work[i];
        if (stt->res_scaled) stt->res_scaled[c] = s.res_inf;
        if (stt->mg_cycles) stt->mg_cycles[c] = s.mg_cycles;
    }
    return bad ? JFNK_NOT_CONVERGED : JFNK_OK;
}

}  // extern "C"
