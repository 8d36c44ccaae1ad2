// Learned Newton initial guess: a 1D convolutional network over the cells of
// each column (six layers of kernel 5, 8 -> 64 x 5 -> 2 channels), evaluated
// and trained with BF16 x BF16 -> FP32 matrix-core (MFMA 16x16x32) kernels.
//
// Matrix formulation.  A layer is, per tap j, a product of the activations
// of cells i + j - 2 (rows: cells, columns: input channels) with the tap's
// weights (input x output channels).  The MFMA reduction index runs over
// (tap, group of 8 input channels) pairs; lane l of a wave supplies the 8
// channels of pair 4s + l/16 at k-step s, for the row (cell) l%16 of the A
// tile and the column (output channel) l%16 of the B tile.  Because A and B
// use the same pair for the same lane and slot, the result does not depend
// on how the instruction orders the reduction internally.  Only the row and
// column lane mapping and the accumulator layout (lane l holds rows
// 4 (l/16) + i, column l % 16) are assumed.
//
// Inference fuses all six layers per tile of 128 cells: the tile reads 12
// cells of context on each side (2 per layer), keeps the activations in LDS
// (two ping-pong buffers of [cell][channel] rows), zeroes cells outside the
// column at every layer (the zero padding of each convolution), and writes
// only the guess.  Training runs the same fused kernel, which in addition
// stores every hidden activation, the output gradient and the loss; the
// backward pass is one kernel per layer for the input gradient (the forward
// kernel's tiling with flipped, transposed weights, times the ReLU mask) and
// one for the weight gradient (a reduction over cells; MFMA with cells as
// the reduction index, operands read from [channel][cell] copies of the
// activations and output gradients, fixed-order partial sums per chunk of
// cells).  Training cells live in a gapped layout: column c's cell i sits at
// position kFront + offset(c) + 2c + i, so two zero cells separate columns
// and the weight-gradient reduction needs no column bookkeeping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "jfnk.h"
#include "jfnk_net.h"

using namespace jfnk;
using namespace jfnk::net;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;             // 4 waves per tile
constexpr int kRS = 72;                   // LDS row stride (bf16): 64 channels + 8 of skew
constexpr int kRows = 168;                // LDS rows: kWin rounded up for the last 16-row tile
constexpr int64_t kFront = 16;            // leading zero positions of the gapped layout
constexpr int kPW = 2048;                 // cells per weight-gradient chunk
constexpr int64_t kTMargin = 8;           // zero elements before each [channel][cell] array

struct NetTile { int32_t col, s0; };      // column (index into the column table), first cell
struct NetCol {
    int64_t off;      // first cell in the caller's packed arrays
    int64_t goff;     // first cell in the gapped training layout
    int32_t n, pad;
    float logh, dv;   // log10(h / 1e-5 m), (phi_R - phi_L) / 1000 V
    double ps;        // phi_s
};

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *(const u32x4*)p);
}

__device__ __forceinline__ bf16x8 zero8() {
    u32x4 z = {0u, 0u, 0u, 0u};
    return __builtin_bit_cast(bf16x8, z);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Features of one cell (the input channels documented with the C ABI).
// ---------------------------------------------------------------------------
struct CellIn {
    const double *ne, *phi, *ne_prev, *phi_prev, *q, *temp;
};

__device__ __forceinline__ double a_of(double n) { return asinh(n / kN0) / 20.0; }

__device__ __forceinline__ void features(const CellIn& in, const NetCol& cc, int64_t u, float f[8]) {
    const double ne = in.ne[u], ph = in.phi[u];
    const double an = a_of(ne);
    f[0] = (float)an;
    f[1] = (float)(ph / cc.ps);
    f[2] = (float)a_of(in.q[u]);
    f[3] = (float)((in.temp[u] - 1150.0) / 850.0);
    f[4] = cc.logh;
    f[5] = cc.dv;
    if (in.ne_prev) {
        f[6] = (float)(an - a_of(in.ne_prev[u]));
        f[7] = (float)((ph - in.phi_prev[u]) / cc.ps);
    } else {
        f[6] = 0.0f;
        f[7] = 0.0f;
    }
}

__device__ __forceinline__ u32x4 pack8(const float f[8]) {
    u32x4 v;
    v[0] = (uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16);
    v[1] = (uint32_t)f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16);
    v[2] = (uint32_t)f2bf(f[4]) | ((uint32_t)f2bf(f[5]) << 16);
    v[3] = (uint32_t)f2bf(f[6]) | ((uint32_t)f2bf(f[7]) << 16);
    return v;
}

// ---------------------------------------------------------------------------
// One convolution over the rows of an LDS buffer.  Rows [row0, row0 + 16 nmt)
// of the output are computed from input rows r - 2 .. r + 2 (tap j reads row
// r + j - 2).  G groups of 8 input channels, COP output channels (64: the
// four waves take two 16-channel tiles each and alternate over the row
// tiles; 16: every wave takes the one channel tile and a quarter of the row
// tiles).  w: [tap][COP][8G] BF16 weights.  epi(m0, co, acc) receives the
// lane's accumulators: rows m0 + 4 (lane/16) + i, output channel co.
// ---------------------------------------------------------------------------
template <int G, int COP, int RS, class Epi>
__device__ __forceinline__ void conv_rows(const uint16_t* in, int row0, int nmt,
                                          const uint16_t* __restrict__ w, Epi epi) {
    constexpr int NT = COP / 16;
    constexpr int NTW = NT == 4 ? 2 : 1;
    constexpr int MSTR = NT == 4 ? 2 : 4;
    constexpr int KS = (kTaps * G + 3) / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, rl = lane & 15;
    const int nt0 = NT == 4 ? 2 * (wave & 1) : 0;
    const int moff = NT == 4 ? (wave >> 1) : wave;
    bf16x8 b[KS][NTW];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int q = 4 * s + g, tap = q / G, grp = q % G;
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
            const int co = (nt0 + j) * 16 + rl;
            b[s][j] = tap < kTaps ? ld8(w + (int64_t)(tap * COP + co) * (8 * G) + grp * 8) : zero8();
        }
    }
    for (int mt = moff; mt < nmt; mt += MSTR) {
        const int m0 = row0 + 16 * mt;
        f32x4 acc[NTW];
#pragma unroll
        for (int j = 0; j < NTW; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int q = 4 * s + g, tap = q / G, grp = q % G;
            const bf16x8 av = tap < kTaps ? ld8(in + (m0 + rl + tap - 2) * RS + grp * 8) : zero8();
#pragma unroll
            for (int j = 0; j < NTW; ++j) acc[j] = mfma(av, b[s][j], acc[j]);
        }
#pragma unroll
        for (int j = 0; j < NTW; ++j) epi(m0, (nt0 + j) * 16 + rl, acc[j]);
    }
}

// ---------------------------------------------------------------------------
// Fused forward over tiles of 128 cells.
// ---------------------------------------------------------------------------
enum { MODE_INFER = 0, MODE_TRAIN = 1 };

struct Weights {
    const uint16_t* wf[kLayers];   // [tap][coutp][cin] BF16
    const uint16_t* wt[kLayers];   // [tap][cin][coutp] BF16, taps reversed (input gradient)
    const float* b[kLayers];       // [coutp]
};

struct FusedArgs {
    const NetTile* tiles;
    const NetCol* cols;
    CellIn in;
    Weights W;
    float s0, s1;
    // inference
    double *ne_out, *phi_out;
    // training
    const uint16_t* x0;            // [pos][8]
    const float* tgt;              // [pos][2]
    uint16_t* act[kLayers - 1];    // [pos][64]
    uint16_t* actT[kLayers - 1];   // [64][pcap]
    uint16_t *dy5, *dy5T;          // [pos][16], [16][pcap]
    double* loss_part;             // [tiles]
    int64_t pcap;
    float inv_n;
};

template <int MODE, int l>
__device__ __forceinline__ void fused_hidden(const FusedArgs& a, const NetTile& tl, const NetCol& cc,
                                             const uint16_t* in, uint16_t* out) {
    constexpr int G = cin(l) / 8;
    constexpr int row0 = 2 * (l + 1);
    constexpr int rend = kWin - 2 * (l + 1);
    constexpr int nmt = (rend - row0 + 15) / 16;
    const float* bias = a.W.b[l];
    const int g = (threadIdx.x & 63) >> 4;
    conv_rows<G, 64, kRS>(in, row0, nmt, a.W.wf[l], [&](int m0, int co, f32x4 acc) {
        const float bv = bias[co];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = m0 + 4 * g + i;
            const int cell = tl.s0 + r - kHalo;
            const bool ok = r < rend && cell >= 0 && cell < cc.n;
            const uint16_t hv = f2bf(ok ? fmaxf(acc[i] + bv, 0.0f) : 0.0f);
            out[r * kRS + co] = hv;
            if (MODE == MODE_TRAIN && ok && r >= kHalo && r < kHalo + kTile) {
                const int64_t gp = cc.goff + cell;
                a.act[l][gp * 64 + co] = hv;
                a.actT[l][co * a.pcap + gp] = hv;
            }
        }
    });
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_fused(FusedArgs a) {
    __shared__ __align__(16) uint16_t bufA[kRows * kRS];
    __shared__ __align__(16) uint16_t bufB[kRows * kRS];
    __shared__ double red[kThreads / 64];
    const NetTile tl = a.tiles[blockIdx.x];
    const NetCol cc = a.cols[tl.col];
    const int tid = threadIdx.x;
    {
        u32x4 z = {0u, 0u, 0u, 0u};
        for (int i = tid; i < kRows * kRS / 8; i += kThreads) {
            ((u32x4*)bufA)[i] = z;
            ((u32x4*)bufB)[i] = z;
        }
    }
    __syncthreads();
    // input rows (8 channels) into bufB
    for (int r = tid; r < kWin; r += kThreads) {
        const int cell = tl.s0 + r - kHalo;
        if (cell < 0 || cell >= cc.n) continue;
        u32x4 v;
        if (MODE == MODE_INFER) {
            float f[8];
            features(a.in, cc, cc.off + cell, f);
            v = pack8(f);
        } else {
            v = *(const u32x4*)(a.x0 + (cc.goff + cell) * 8);
        }
        *(u32x4*)(bufB + r * kRS) = v;
    }
    __syncthreads();
    fused_hidden<MODE, 0>(a, tl, cc, bufB, bufA);
    __syncthreads();
    fused_hidden<MODE, 1>(a, tl, cc, bufA, bufB);
    __syncthreads();
    fused_hidden<MODE, 2>(a, tl, cc, bufB, bufA);
    __syncthreads();
    fused_hidden<MODE, 3>(a, tl, cc, bufA, bufB);
    __syncthreads();
    fused_hidden<MODE, 4>(a, tl, cc, bufB, bufA);
    __syncthreads();
    // output layer: rows [kHalo, kHalo + kTile), 2 real channels of 16
    constexpr int l = kLayers - 1;
    const int lane = tid & 63, g = lane >> 4;
    double lsum = 0.0;
    conv_rows<8, 16, kRS>(bufA, kHalo, kTile / 16, a.W.wf[l], [&](int m0, int co, f32x4 acc) {
        if (co >= 2) return;
        const float bv = a.W.b[l][co];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = m0 + 4 * g + i;
            const int cell = tl.s0 + r - kHalo;
            if (cell < 0 || cell >= cc.n) continue;
            const float o = acc[i] + bv;
            if (MODE == MODE_INFER) {
                const int64_t u = cc.off + cell;
                if (co == 0) {
                    const double an = a_of(a.in.ne[u]) + (double)a.s0 * (double)o;
                    a.ne_out[u] = kN0 * sinh(20.0 * an);
                } else {
                    a.phi_out[u] = a.in.phi[u] + cc.ps * (double)a.s1 * (double)o;
                }
            } else {
                const int64_t gp = cc.goff + cell;
                const float d = o - a.tgt[gp * 2 + co];
                lsum += (double)d * (double)d;
                const uint16_t hv = f2bf(2.0f * d * a.inv_n);
                a.dy5[gp * 16 + co] = hv;
                a.dy5T[co * a.pcap + gp] = hv;
            }
        }
    });
    if (MODE == MODE_TRAIN) {
        for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
        if (lane == 0) red[tid >> 6] = lsum;
        __syncthreads();
        if (tid == 0) a.loss_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// ---------------------------------------------------------------------------
// Training: features and targets, gap clearing, input gradient, weight
// gradient, reductions, Adam, BF16 packing.
// ---------------------------------------------------------------------------
struct FeatArgs {
    const NetTile* tiles;
    const NetCol* cols;
    CellIn in;
    const double *ne_next, *phi_next;
    uint16_t* x0;
    uint16_t* x0T;
    float* tgt;
    int64_t pcap;
    float s0, s1;
};

__global__ __launch_bounds__(kTile) void k_features(FeatArgs a) {
    const NetTile tl = a.tiles[blockIdx.x];
    const NetCol cc = a.cols[tl.col];
    const int cell = tl.s0 + threadIdx.x;
    if (cell >= cc.n) return;
    const int64_t u = cc.off + cell, gp = cc.goff + cell;
    float f[8];
    features(a.in, cc, u, f);
    const u32x4 v = pack8(f);
    *(u32x4*)(a.x0 + gp * 8) = v;
#pragma unroll
    for (int j = 0; j < 8; ++j) a.x0T[j * a.pcap + gp] = f2bf(f[j]);
    const double an = a_of(a.in.ne[u]);
    a.tgt[gp * 2 + 0] = (float)((a_of(a.ne_next[u]) - an) / (double)a.s0);
    a.tgt[gp * 2 + 1] = (float)((a.phi_next[u] - a.in.phi[u]) / (cc.ps * (double)a.s1));
}

struct GapArgs {
    const NetCol* cols;
    int ncols;
    int64_t pend;
    int64_t pcap;
    uint16_t* arr[16];   // [channel][cell] arrays
    int rows[16];
    int narr;
};

// zero every [channel][cell] entry at positions in [0, pend) that are not cells
__global__ void k_zero_gaps(GapArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.pend) return;
    int lo = 0, hi = a.ncols - 1;   // last column with goff <= p
    if (p < a.cols[0].goff) {
        lo = -1;
    } else {
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.cols[mid].goff <= p) lo = mid; else hi = mid - 1;
        }
    }
    if (lo >= 0 && p < a.cols[lo].goff + a.cols[lo].n) return;
    for (int k = 0; k < a.narr; ++k)
        for (int r = 0; r < a.rows[k]; ++r) a.arr[k][r * a.pcap + p] = 0;
}

struct DgradArgs {
    const NetTile* tiles;
    const NetCol* cols;
    const uint16_t* dy;        // [pos][8G]: gradient at the layer's output
    const uint16_t* w;         // [tap][64][8G]
    const uint16_t* act;       // [pos][64]: the layer's input (post-ReLU)
    uint16_t* out;             // [pos][64]
    uint16_t* outT;            // [64][pcap]
    int64_t pcap;
};

template <int G>
__global__ __launch_bounds__(kThreads) void k_dgrad(DgradArgs a) {
    constexpr int CI = 8 * G, RS = CI + 8, ROWS = kTile + 4 + 16;
    __shared__ __align__(16) uint16_t buf[ROWS * RS];
    const NetTile tl = a.tiles[blockIdx.x];
    const NetCol cc = a.cols[tl.col];
    const int tid = threadIdx.x;
    {
        u32x4 z = {0u, 0u, 0u, 0u};
        for (int i = tid; i < ROWS * RS / 8; i += kThreads) ((u32x4*)buf)[i] = z;
    }
    __syncthreads();
    for (int idx = tid; idx < (kTile + 4) * G; idx += kThreads) {
        const int r = idx / G, gi = idx % G;
        const int cell = tl.s0 + r - 2;
        if (cell < 0 || cell >= cc.n) continue;
        *(u32x4*)(buf + r * RS + gi * 8) = *(const u32x4*)(a.dy + (cc.goff + cell) * CI + gi * 8);
    }
    __syncthreads();
    const int g = (tid & 63) >> 4;
    conv_rows<G, 64, RS>(buf, 2, kTile / 16, a.w, [&](int m0, int co, f32x4 acc) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = m0 + 4 * g + i;
            const int cell = tl.s0 + r - 2;
            if (cell < 0 || cell >= cc.n) continue;
            const int64_t gp = cc.goff + cell;
            const uint16_t av = a.act[gp * 64 + co];
            const bool pos = av != 0 && (av & 0x8000u) == 0;
            const uint16_t hv = f2bf(pos ? acc[i] : 0.0f);
            a.out[gp * 64 + co] = hv;
            a.outT[co * a.pcap + gp] = hv;
        }
    });
}

struct WgradArgs {
    const uint16_t* xT;        // [CIP][pcap] layer input
    const uint16_t* dyT;       // [COP][pcap] gradient at the layer output
    float* part;               // [chunks][block]
    int64_t pcap;
    int block;                 // parameters of the layer
};

// chunk of kPW cells: dW[co][j][ci] += sum_p dy[co][p] x[ci][p + j - 2]; db[co] += sum_p dy[co][p]
template <int CIP, int COP, int CIN, int COUT>
__global__ __launch_bounds__(kThreads) void k_wgrad(WgradArgs a) {
    constexpr int NCO = COP / 16, NCI = (CIP + 15) / 16, NP = NCO * NCI, PPW = NP / 4;
    static_assert(NP % 4 == 0, "pairs per wave");
    static_assert(NCI == 1 || NCI == 4, "input tile per wave");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, rl = lane & 15;
    const int cit = NCI == 4 ? wave : 0;
    const int ci = cit * 16 + rl;
    f32x4 acc[PPW][kTaps];
    f32x4 accb[PPW];
#pragma unroll
    for (int j = 0; j < PPW; ++j) {
        accb[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < kTaps; ++k) acc[j][k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    u32x4 onesw;
    onesw[0] = onesw[1] = onesw[2] = onesw[3] = 0x3f803f80u;   // BF16 1.0 pairs
    const bf16x8 ones = __builtin_bit_cast(bf16x8, onesw);
    const int64_t pb = (int64_t)blockIdx.x * kPW;
    for (int ks = 0; ks < kPW / 32; ++ks) {
        const int64_t p0 = pb + 32 * ks + 8 * g;
        // elements p0 - 2 .. p0 + 9 of input channel ci (words 0..5)
        uint32_t wv[6] = {0u, 0u, 0u, 0u, 0u, 0u};
        if (ci < CIP) {
            const uint16_t* xr = a.xT + ci * a.pcap;
            wv[0] = *(const uint32_t*)(xr + p0 - 2);
            const u32x4 mid = *(const u32x4*)(xr + p0);
            wv[1] = mid[0]; wv[2] = mid[1]; wv[3] = mid[2]; wv[4] = mid[3];
            wv[5] = *(const uint32_t*)(xr + p0 + 8);
        }
        bf16x8 bt[kTaps];
#pragma unroll
        for (int k = 0; k < kTaps; ++k) {
            // tap k covers elements p0 + k - 2 .. p0 + k + 5, i.e. starting at half-word k of wv
            u32x4 o;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if ((k & 1) == 0) o[m] = wv[k / 2 + m];
                else o[m] = (wv[k / 2 + m] >> 16) | (wv[k / 2 + m + 1] << 16);
            }
            bt[k] = __builtin_bit_cast(bf16x8, o);
        }
#pragma unroll
        for (int j = 0; j < PPW; ++j) {
            const int p = wave + 4 * j;
            const int cot = p / NCI;
            const bf16x8 av = ld8(a.dyT + (cot * 16 + rl) * a.pcap + p0);
#pragma unroll
            for (int k = 0; k < kTaps; ++k) acc[j][k] = mfma(av, bt[k], acc[j][k]);
            if (cit == 0) accb[j] = mfma(av, ones, accb[j]);
        }
    }
    float* part = a.part + (int64_t)blockIdx.x * a.block;
#pragma unroll
    for (int j = 0; j < PPW; ++j) {
        const int p = wave + 4 * j;
        const int cot = p / NCI;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = cot * 16 + 4 * g + i;
            if (co >= COUT) continue;
            if (ci < CIN) {
#pragma unroll
                for (int k = 0; k < kTaps; ++k) part[(co * kTaps + k) * CIN + ci] = acc[j][k][i];
            }
            if (cit == 0 && rl == 0) part[COUT * kTaps * CIN + co] = accb[j][i];
        }
    }
}

__global__ void k_reduce(const float* __restrict__ part, int nchunks, int block, float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= block) return;
    float s = 0.0f;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * block + j];
    out[j] = s;
}

__global__ __launch_bounds__(256) void k_loss_sum(const double* __restrict__ part, int n, double scale,
                                                  double* __restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] * scale;
}

struct AdamArgs {
    float *p, *m, *v;
    const float* g;
    int64_t n;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t)
};

__global__ void k_adam(AdamArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float g = a.g[i];
    const float m = a.b1 * a.m[i] + (1.0f - a.b1) * g;
    const float v = a.b2 * a.v[i] + (1.0f - a.b2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    a.p[i] -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
}

struct PackArgs {
    const float* p;
    uint16_t* wf[kLayers];
    uint16_t* wt[kLayers];
    float* b[kLayers];
};

template <int l>
__device__ void pack_layer(const PackArgs& a, int64_t i0, int64_t stride) {
    constexpr int CI = cin(l), CO = cout(l), COP = coutp(l);
    const float* W = a.p + poffset(l);
    const float* B = W + wcount(l);
    const int64_t nf = (int64_t)kTaps * COP * CI;
    for (int64_t i = i0; i < nf; i += stride) {
        const int ci = (int)(i % CI), co = (int)((i / CI) % COP), k = (int)(i / (CI * COP));
        a.wf[l][i] = f2bf(co < CO ? W[(co * kTaps + k) * CI + ci] : 0.0f);
        if (l > 0) {
            // transposed, taps reversed: wt[k][ci][co] = W[co][4 - k][ci]
            const int co2 = (int)(i % COP), ci2 = (int)((i / COP) % CI), k2 = (int)(i / (COP * CI));
            a.wt[l][i] = f2bf(co2 < CO ? W[(co2 * kTaps + (kTaps - 1 - k2)) * CI + ci2] : 0.0f);
        }
    }
    for (int64_t i = i0; i < COP; i += stride) a.b[l][i] = i < CO ? B[i] : 0.0f;
}

__global__ void k_pack(PackArgs a) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    switch (blockIdx.y) {
        case 0: pack_layer<0>(a, i0, st); break;
        case 1: pack_layer<1>(a, i0, st); break;
        case 2: pack_layer<2>(a, i0, st); break;
        case 3: pack_layer<3>(a, i0, st); break;
        case 4: pack_layer<4>(a, i0, st); break;
        default: pack_layer<5>(a, i0, st); break;
    }
}

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct jfnk_net {
    jfnk_net_config cfg{};
    std::string err;
    int device = 0;
    void* base = nullptr;            // parameters, packed weights, training workspace
    float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    int64_t step = 0;
    uint64_t version = 0;            // weight changes so far
    uint16_t* wf[kLayers] = {};
    uint16_t* wt[kLayers] = {};
    float* bias[kLayers] = {};
    // training workspace (gapped layout)
    int64_t pcap = 0;
    int64_t tcap = 0;                // tiles
    uint16_t *x0 = nullptr, *x0T = nullptr;
    float* tgt = nullptr;
    uint16_t* act[kLayers - 1] = {};
    uint16_t* actT[kLayers - 1] = {};
    uint16_t *dya = nullptr, *dyaT = nullptr, *dyb = nullptr, *dybT = nullptr;
    uint16_t *dy5 = nullptr, *dy5T = nullptr;
    float* part = nullptr;
    double* loss_part = nullptr;
    double* loss_dev = nullptr;
    NetTile* d_tiles = nullptr;
    NetCol* d_cols = nullptr;
    // prediction tables
    void* pbase = nullptr;
    int64_t p_tcap = 0;
    int32_t p_ccap = 0;
    NetTile* p_tiles = nullptr;
    NetCol* p_cols = nullptr;
    // pinned staging and its reuse fence
    NetTile* h_tiles = nullptr;
    NetCol* h_cols = nullptr;
    int64_t h_tcap = 0;
    int32_t h_ccap = 0;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
};

namespace {

int nfail(jfnk_net* n, int code, const std::string& msg) {
    if (n) n->err = msg;
    return code;
}

#define NET_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return nfail(net, JFNK_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

Weights weights_of(const jfnk_net* net) {
    Weights w;
    for (int l = 0; l < kLayers; ++l) {
        w.wf[l] = net->wf[l];
        w.wt[l] = net->wt[l];
        w.b[l] = net->bias[l];
    }
    return w;
}

int launch_pack(jfnk_net* net, hipStream_t st) {
    PackArgs a;
    a.p = net->params;
    for (int l = 0; l < kLayers; ++l) {
        a.wf[l] = net->wf[l];
        a.wt[l] = net->wt[l];
        a.b[l] = net->bias[l];
    }
    hipLaunchKernelGGL(k_pack, dim3(40, kLayers), dim3(256), 0, st, a);
    NET_HIP(hipGetLastError());
    return JFNK_OK;
}

// pinned staging tables, grown on demand (the previous upload must be done)
int stage_reserve(jfnk_net* net, int64_t ntiles, int32_t ncols) {
    if (net->staged_pending) {
        NET_HIP(hipEventSynchronize(net->staged));
        net->staged_pending = false;
    }
    if (ntiles > net->h_tcap) {
        if (net->h_tiles) NET_HIP(hipHostFree(net->h_tiles));
        net->h_tiles = nullptr;
        NET_HIP(hipHostMalloc((void**)&net->h_tiles, sizeof(NetTile) * ntiles));
        net->h_tcap = ntiles;
    }
    if (ncols > net->h_ccap) {
        if (net->h_cols) NET_HIP(hipHostFree(net->h_cols));
        net->h_cols = nullptr;
        NET_HIP(hipHostMalloc((void**)&net->h_cols, sizeof(NetCol) * ncols));
        net->h_ccap = ncols;
    }
    return JFNK_OK;
}

int check_problem(jfnk_net* net, const jfnk_problem* p, const jfnk_state* x) {
    if (!p || !x) return nfail(net, JFNK_EINVAL, "null problem or state");
    if (p->ncols < 1) return nfail(net, JFNK_EINVAL, "ncols < 1");
    if (!p->col_offset || !p->length || !p->phi_left || !p->phi_right)
        return nfail(net, JFNK_EINVAL, "null per-column array");
    if (!p->q_ion || !p->temp || !x->ne || !x->phi)
        return nfail(net, JFNK_EINVAL, "null per-cell array (q_ion, temp, ne and phi are required)");
    if ((x->ne_prev == nullptr) != (x->phi_prev == nullptr))
        return nfail(net, JFNK_EINVAL, "ne_prev and phi_prev must both be given or both NULL");
    if (p->col_offset[0] != 0) return nfail(net, JFNK_EINVAL, "col_offset[0] != 0");
    for (int c = 0; c < p->ncols; ++c) {
        const int64_t n = p->col_offset[c + 1] - p->col_offset[c];
        if (n < 1 || n > INT32_MAX) return nfail(net, JFNK_EINVAL, "bad column size");
        if (!(p->length[c] > 0.0) || !std::isfinite(p->length[c]) || !std::isfinite(p->phi_left[c]) ||
            !std::isfinite(p->phi_right[c]))
            return nfail(net, JFNK_EINVAL, "bad per-column scalar");
    }
    return JFNK_OK;
}

NetCol make_col(const jfnk_problem* p, int c) {
    NetCol k;
    k.off = p->col_offset[c];
    k.goff = kFront + p->col_offset[c] + 2 * (int64_t)c;
    k.n = (int32_t)(p->col_offset[c + 1] - p->col_offset[c]);
    k.pad = 0;
    const double h = p->length[c] / k.n;
    k.logh = (float)std::log10(h / 1e-5);
    k.dv = (float)((p->phi_right[c] - p->phi_left[c]) / 1000.0);
    k.ps = std::max(std::max(std::fabs(p->phi_left[c]), std::fabs(p->phi_right[c])), 1.0);
    return k;
}

// tiles of the columns with use[c] != 0 (all when use is NULL) into the staging tables
int64_t build_tiles(jfnk_net* net, const jfnk_problem* p, const uint8_t* use) {
    int64_t nt = 0;
    for (int c = 0; c < p->ncols; ++c) {
        net->h_cols[c] = make_col(p, c);
        if (use && !use[c]) continue;
        for (int s = 0; s < net->h_cols[c].n; s += kTile) net->h_tiles[nt++] = NetTile{c, s};
    }
    return nt;
}

int64_t count_tiles(const jfnk_problem* p) {
    int64_t nt = 0;
    for (int c = 0; c < p->ncols; ++c) {
        const int64_t n = p->col_offset[c + 1] - p->col_offset[c];
        nt += (n + kTile - 1) / kTile;
    }
    return nt;
}

int upload_tables(jfnk_net* net, NetTile* dt, NetCol* dc, int64_t nt, int ncols, hipStream_t st) {
    if (nt > 0) NET_HIP(hipMemcpyAsync(dt, net->h_tiles, sizeof(NetTile) * nt, hipMemcpyHostToDevice, st));
    NET_HIP(hipMemcpyAsync(dc, net->h_cols, sizeof(NetCol) * ncols, hipMemcpyHostToDevice, st));
    NET_HIP(hipEventRecord(net->staged, st));
    net->staged_pending = true;
    return JFNK_OK;
}

FusedArgs fused_args(const jfnk_net* net, const jfnk_problem* p, const jfnk_state* x, const NetTile* tiles,
                     const NetCol* cols) {
    FusedArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tiles = tiles;
    a.cols = cols;
    a.in = CellIn{x->ne, x->phi, x->ne_prev, x->phi_prev, p->q_ion, p->temp};
    a.W = weights_of(net);
    a.s0 = net->cfg.out_scale_ne;
    a.s1 = net->cfg.out_scale_phi;
    return a;
}

// forward (saving activations), loss and gradient of one training batch
int forward_backward(jfnk_net* net, const jfnk_problem* p, const jfnk_state* x, const double* ne_next,
                     const double* phi_next, hipStream_t st) {
    if (int rc = check_problem(net, p, x)) return rc;
    if (!ne_next || !phi_next) return nfail(net, JFNK_EINVAL, "null target array");
    if (net->pcap == 0) return nfail(net, JFNK_ECAPACITY, "network created without training capacity");
    const int ncols = p->ncols;
    const int64_t total = p->col_offset[ncols];
    if (ncols > net->cfg.max_cols || total > net->cfg.max_total_cells)
        return nfail(net, JFNK_ECAPACITY, "batch exceeds the training capacity");
    const int64_t ntiles = count_tiles(p);
    if (ntiles > net->tcap) return nfail(net, JFNK_ECAPACITY, "batch exceeds the tile capacity");
    const int64_t pos_end = kFront + total + 2 * (int64_t)ncols;
    const int64_t pend = align_up(pos_end, kPW);
    if (pend + 16 > net->pcap) return nfail(net, JFNK_ECAPACITY, "batch exceeds the position capacity");
    if (int rc = stage_reserve(net, ntiles, ncols)) return rc;
    build_tiles(net, p, nullptr);
    if (int rc = upload_tables(net, net->d_tiles, net->d_cols, ntiles, ncols, st)) return rc;

    FeatArgs fa;
    fa.tiles = net->d_tiles;
    fa.cols = net->d_cols;
    fa.in = CellIn{x->ne, x->phi, x->ne_prev, x->phi_prev, p->q_ion, p->temp};
    fa.ne_next = ne_next;
    fa.phi_next = phi_next;
    fa.x0 = net->x0;
    fa.x0T = net->x0T;
    fa.tgt = net->tgt;
    fa.pcap = net->pcap;
    fa.s0 = net->cfg.out_scale_ne;
    fa.s1 = net->cfg.out_scale_phi;
    hipLaunchKernelGGL(k_features, dim3((unsigned)ntiles), dim3(kTile), 0, st, fa);
    NET_HIP(hipGetLastError());

    GapArgs ga;
    std::memset(&ga, 0, sizeof(ga));
    ga.cols = net->d_cols;
    ga.ncols = ncols;
    ga.pend = pend + 16;
    ga.pcap = net->pcap;
    int k = 0;
    ga.arr[k] = net->x0T; ga.rows[k++] = 8;
    for (int l = 0; l < kLayers - 1; ++l) { ga.arr[k] = net->actT[l]; ga.rows[k++] = 64; }
    ga.arr[k] = net->dyaT; ga.rows[k++] = 64;
    ga.arr[k] = net->dybT; ga.rows[k++] = 64;
    ga.arr[k] = net->dy5T; ga.rows[k++] = 16;
    ga.narr = k;
    hipLaunchKernelGGL(k_zero_gaps, dim3((unsigned)((ga.pend + 255) / 256)), dim3(256), 0, st, ga);
    NET_HIP(hipGetLastError());

    FusedArgs a = fused_args(net, p, x, net->d_tiles, net->d_cols);
    a.x0 = net->x0;
    a.tgt = net->tgt;
    for (int l = 0; l < kLayers - 1; ++l) {
        a.act[l] = net->act[l];
        a.actT[l] = net->actT[l];
    }
    a.dy5 = net->dy5;
    a.dy5T = net->dy5T;
    a.loss_part = net->loss_part;
    a.pcap = net->pcap;
    a.inv_n = (float)(1.0 / (double)total);
    hipLaunchKernelGGL(k_fused<MODE_TRAIN>, dim3((unsigned)ntiles), dim3(kThreads), 0, st, a);
    NET_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, st, (const double*)net->loss_part, (int)ntiles,
                       1.0 / (double)total, net->loss_dev);
    NET_HIP(hipGetLastError());

    // backward, output layer first
    const int nchunks = (int)(pend / kPW);
    const uint16_t* dyT_of[kLayers] = {net->dyaT, net->dybT, net->dyaT, net->dybT, net->dyaT, net->dy5T};
    const uint16_t* dy_of[kLayers] = {net->dya, net->dyb, net->dya, net->dyb, net->dya, net->dy5};
    uint16_t* out_of[kLayers] = {nullptr, net->dya, net->dyb, net->dya, net->dyb, net->dya};
    uint16_t* outT_of[kLayers] = {nullptr, net->dyaT, net->dybT, net->dyaT, net->dybT, net->dyaT};
    for (int l = kLayers - 1; l >= 0; --l) {
        WgradArgs wa;
        wa.xT = l == 0 ? net->x0T : net->actT[l - 1];
        wa.dyT = dyT_of[l];
        wa.part = net->part;
        wa.pcap = net->pcap;
        wa.block = (int)pcount(l);
        if (l == 0)
            hipLaunchKernelGGL((k_wgrad<8, 64, 8, 64>), dim3(nchunks), dim3(kThreads), 0, st, wa);
        else if (l == kLayers - 1)
            hipLaunchKernelGGL((k_wgrad<64, 16, 64, 2>), dim3(nchunks), dim3(kThreads), 0, st, wa);
        else
            hipLaunchKernelGGL((k_wgrad<64, 64, 64, 64>), dim3(nchunks), dim3(kThreads), 0, st, wa);
        NET_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_reduce, dim3((unsigned)((pcount(l) + 255) / 256)), dim3(256), 0, st,
                           (const float*)net->part, nchunks, (int)pcount(l), net->grad + poffset(l));
        NET_HIP(hipGetLastError());
        if (l == 0) break;
        DgradArgs da;
        da.tiles = net->d_tiles;
        da.cols = net->d_cols;
        da.dy = dy_of[l];
        da.w = net->wt[l];
        da.act = net->act[l - 1];
        da.out = out_of[l];
        da.outT = outT_of[l];
        da.pcap = net->pcap;
        if (l == kLayers - 1)
            hipLaunchKernelGGL(k_dgrad<2>, dim3((unsigned)ntiles), dim3(kThreads), 0, st, da);
        else
            hipLaunchKernelGGL(k_dgrad<8>, dim3((unsigned)ntiles), dim3(kThreads), 0, st, da);
        NET_HIP(hipGetLastError());
    }
    return JFNK_OK;
}

}  // namespace

namespace jfnk {

int net_ensure_predict_capacity(jfnk_net* net, int32_t max_cols, int64_t max_total_cells) {
    if (!net) return JFNK_EINVAL;
    const int64_t tiles = max_total_cells / kTile + max_cols + 1;
    if (tiles <= net->p_tcap && max_cols <= net->p_ccap) return JFNK_OK;
    NET_HIP(hipSetDevice(net->device));
    NET_HIP(hipDeviceSynchronize());
    if (net->pbase) NET_HIP(hipFree(net->pbase));
    net->pbase = nullptr;
    net->p_tcap = net->p_ccap = 0;
    const int64_t tb = align_up(sizeof(NetTile) * tiles, 256);
    const int64_t cb = align_up(sizeof(NetCol) * (int64_t)max_cols, 256);
    if (hipMalloc(&net->pbase, tb + cb) != hipSuccess) {
        net->pbase = nullptr;
        return nfail(net, JFNK_ENOMEM, "prediction tables");
    }
    net->p_tiles = (NetTile*)net->pbase;
    net->p_cols = (NetCol*)((char*)net->pbase + tb);
    net->p_tcap = tiles;
    net->p_ccap = max_cols;
    return stage_reserve(net, tiles, max_cols);
}

uint64_t net_version(const jfnk_net* net) { return net->version; }

int net_predict_masked(jfnk_net* net, const jfnk_problem* p, const jfnk_state* x, const uint8_t* use_col,
                       double* ne_out, double* phi_out, void* stream) {
    if (!net) return JFNK_EINVAL;
    if (int rc = check_problem(net, p, x)) return rc;
    if (!ne_out || !phi_out) return nfail(net, JFNK_EINVAL, "null output array");
    const int64_t need = count_tiles(p);
    if (need > net->p_tcap || p->ncols > net->p_ccap)
        return nfail(net, JFNK_ECAPACITY, "prediction tables too small");
    hipStream_t st = (hipStream_t)stream;
    if (int rc = stage_reserve(net, need, p->ncols)) return rc;
    const int64_t nt = build_tiles(net, p, use_col);
    if (int rc = upload_tables(net, net->p_tiles, net->p_cols, nt, p->ncols, st)) return rc;
    if (nt == 0) return JFNK_OK;
    FusedArgs a = fused_args(net, p, x, net->p_tiles, net->p_cols);
    a.ne_out = ne_out;
    a.phi_out = phi_out;
    hipLaunchKernelGGL(k_fused<MODE_INFER>, dim3((unsigned)nt), dim3(kThreads), 0, st, a);
    NET_HIP(hipGetLastError());
    return JFNK_OK;
}

}  // namespace jfnk

extern "C" {

void jfnk_net_config_default(jfnk_net_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->max_cols = 0;
    cfg->max_total_cells = 0;
    cfg->out_scale_ne = 0.1f;
    cfg->out_scale_phi = 0.3f;
    cfg->beta1 = 0.9f;
    cfg->beta2 = 0.999f;
    cfg->adam_eps = 1e-8f;
}

int64_t jfnk_net_param_count(void) { return kParams; }

int jfnk_net_create(const jfnk_net_config* cfg, jfnk_net** out) {
    if (!out) return JFNK_EINVAL;
    *out = nullptr;
    if (!cfg) return JFNK_EINVAL;
    if (cfg->max_cols < 0 || cfg->max_total_cells < 0 || (cfg->max_cols == 0) != (cfg->max_total_cells == 0))
        return JFNK_EINVAL;
    if (!(cfg->out_scale_ne > 0.0f) || !(cfg->out_scale_phi > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->adam_eps > 0.0f))
        return JFNK_EINVAL;
    jfnk_net* net = new (std::nothrow) jfnk_net;
    if (!net) return JFNK_ENOMEM;
    net->cfg = *cfg;
    if (hipGetDevice(&net->device) != hipSuccess || hipEventCreateWithFlags(&net->staged, hipEventDisableTiming) != hipSuccess) {
        delete net;
        return JFNK_EHIP;
    }
    // one allocation: parameters (4 x FP32), packed weights, then the training workspace
    std::vector<std::pair<void**, int64_t>> plan;
    plan.push_back({(void**)&net->params, 4 * kParams});
    plan.push_back({(void**)&net->grad, 4 * kParams});
    plan.push_back({(void**)&net->m, 4 * kParams});
    plan.push_back({(void**)&net->v, 4 * kParams});
    for (int l = 0; l < kLayers; ++l) {
        plan.push_back({(void**)&net->wf[l], 2LL * kTaps * coutp(l) * cin(l)});
        plan.push_back({(void**)&net->wt[l], 2LL * kTaps * coutp(l) * cin(l)});
        plan.push_back({(void**)&net->bias[l], 4LL * coutp(l)});
    }
    int64_t tmargin_bytes = 0;
    if (cfg->max_cols > 0) {
        net->pcap = align_up(kFront + cfg->max_total_cells + 2 * (int64_t)cfg->max_cols, kPW) + 64;
        net->tcap = cfg->max_total_cells / kTile + cfg->max_cols + 1;
        const int64_t P = net->pcap;
        const int64_t tb = 2 * (P + 2 * kTMargin);   // bytes per [channel][cell] row incl. margins
        (void)tb;
        plan.push_back({(void**)&net->x0, 2 * 8 * P});
        plan.push_back({(void**)&net->x0T, 2 * (8 * P + 2 * kTMargin)});
        plan.push_back({(void**)&net->tgt, 4 * 2 * P});
        for (int l = 0; l < kLayers - 1; ++l) {
            plan.push_back({(void**)&net->act[l], 2 * 64 * P});
            plan.push_back({(void**)&net->actT[l], 2 * (64 * P + 2 * kTMargin)});
        }
        plan.push_back({(void**)&net->dya, 2 * 64 * P});
        plan.push_back({(void**)&net->dyaT, 2 * (64 * P + 2 * kTMargin)});
        plan.push_back({(void**)&net->dyb, 2 * 64 * P});
        plan.push_back({(void**)&net->dybT, 2 * (64 * P + 2 * kTMargin)});
        plan.push_back({(void**)&net->dy5, 2 * 16 * P});
        plan.push_back({(void**)&net->dy5T, 2 * (16 * P + 2 * kTMargin)});
        plan.push_back({(void**)&net->part, 4 * (P / kPW) * pcount(1)});
        plan.push_back({(void**)&net->loss_part, 8 * net->tcap});
        plan.push_back({(void**)&net->loss_dev, 8});
        plan.push_back({(void**)&net->d_tiles, (int64_t)sizeof(NetTile) * net->tcap});
        plan.push_back({(void**)&net->d_cols, (int64_t)sizeof(NetCol) * cfg->max_cols});
        tmargin_bytes = 2 * kTMargin;
    }
    int64_t total = 0;
    for (auto& e : plan) total += align_up(e.second, 256);
    if (hipMalloc(&net->base, total) != hipSuccess) {
        net->base = nullptr;
        (void)hipEventDestroy(net->staged);
        delete net;
        return JFNK_ENOMEM;
    }
    if (hipMemset(net->base, 0, total) != hipSuccess) {
        (void)hipFree(net->base);
        (void)hipEventDestroy(net->staged);
        delete net;
        return JFNK_EHIP;
    }
    int64_t o = 0;
    for (auto& e : plan) {
        *e.first = (char*)net->base + o;
        o += align_up(e.second, 256);
    }
    if (cfg->max_cols > 0) {
        // [channel][cell] arrays start after a zero margin: the weight-gradient
        // reads reach two cells before position 0
        net->x0T = (uint16_t*)((char*)net->x0T + tmargin_bytes);
        for (int l = 0; l < kLayers - 1; ++l) net->actT[l] = (uint16_t*)((char*)net->actT[l] + tmargin_bytes);
        net->dyaT = (uint16_t*)((char*)net->dyaT + tmargin_bytes);
        net->dybT = (uint16_t*)((char*)net->dybT + tmargin_bytes);
        net->dy5T = (uint16_t*)((char*)net->dy5T + tmargin_bytes);
        if (net_ensure_predict_capacity(net, cfg->max_cols, cfg->max_total_cells) != JFNK_OK) {
            jfnk_net_destroy(net);
            return JFNK_ENOMEM;
        }
    }
    *out = net;
    return JFNK_OK;
}

void jfnk_net_destroy(jfnk_net* net) {
    if (!net) return;
    (void)hipSetDevice(net->device);
    (void)hipDeviceSynchronize();
    if (net->base) (void)hipFree(net->base);
    if (net->pbase) (void)hipFree(net->pbase);
    if (net->h_tiles) (void)hipHostFree(net->h_tiles);
    if (net->h_cols) (void)hipHostFree(net->h_cols);
    if (net->staged) (void)hipEventDestroy(net->staged);
    delete net;
}

const char* jfnk_net_last_error(const jfnk_net* net) {
    if (!net) return "null network";
    return net->err.c_str();
}

int jfnk_net_set_params(jfnk_net* net, const float* params, int64_t n) {
    if (!net) return JFNK_EINVAL;
    if (!params || n != kParams) return nfail(net, JFNK_EINVAL, "parameter count mismatch");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return nfail(net, JFNK_EINVAL, "non-finite parameter");
    NET_HIP(hipSetDevice(net->device));
    NET_HIP(hipDeviceSynchronize());
    NET_HIP(hipMemcpy(net->params, params, 4 * kParams, hipMemcpyHostToDevice));
    NET_HIP(hipMemset(net->m, 0, 4 * kParams));
    NET_HIP(hipMemset(net->v, 0, 4 * kParams));
    net->step = 0;
    ++net->version;
    if (int rc = launch_pack(net, nullptr)) return rc;
    NET_HIP(hipDeviceSynchronize());
    return JFNK_OK;
}

int jfnk_net_get_params(jfnk_net* net, float* params, int64_t n) {
    if (!net) return JFNK_EINVAL;
    if (!params || n != kParams) return nfail(net, JFNK_EINVAL, "parameter count mismatch");
    NET_HIP(hipSetDevice(net->device));
    NET_HIP(hipDeviceSynchronize());
    NET_HIP(hipMemcpy(params, net->params, 4 * kParams, hipMemcpyDeviceToHost));
    return JFNK_OK;
}

int jfnk_net_predict(jfnk_net* net, const jfnk_problem* p, const jfnk_state* x, double* ne_out, double* phi_out,
                     void* stream) {
    if (!net) return JFNK_EINVAL;
    if (int rc = check_problem(net, p, x)) return rc;
    if (int rc = net_ensure_predict_capacity(net, p->ncols, p->col_offset[p->ncols])) return rc;
    return net_predict_masked(net, p, x, nullptr, ne_out, phi_out, stream);
}

int jfnk_net_grad(jfnk_net* net, const jfnk_problem* p, const jfnk_state* x, const double* ne_next,
                  const double* phi_next, float* grad, double* loss, void* stream) {
    if (!net) return JFNK_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (int rc = forward_backward(net, p, x, ne_next, phi_next, st)) return rc;
    if (grad) NET_HIP(hipMemcpyAsync(grad, net->grad, 4 * kParams, hipMemcpyDeviceToHost, st));
    if (loss) NET_HIP(hipMemcpyAsync(loss, net->loss_dev, 8, hipMemcpyDeviceToHost, st));
    NET_HIP(hipStreamSynchronize(st));
    return JFNK_OK;
}

int jfnk_net_train_step(jfnk_net* net, const jfnk_problem* p, const jfnk_state* x, const double* ne_next,
                        const double* phi_next, float lr, double* loss, void* stream) {
    if (!net) return JFNK_EINVAL;
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return nfail(net, JFNK_EINVAL, "bad learning rate");
    hipStream_t st = (hipStream_t)stream;
    if (int rc = forward_backward(net, p, x, ne_next, phi_next, st)) return rc;
    net->step += 1;
    AdamArgs a;
    a.p = net->params;
    a.m = net->m;
    a.v = net->v;
    a.g = net->grad;
    a.n = kParams;
    a.lr = lr;
    a.b1 = net->cfg.beta1;
    a.b2 = net->cfg.beta2;
    a.eps = net->cfg.adam_eps;
    a.c1 = (float)(1.0 / (1.0 - std::pow((double)net->cfg.beta1, (double)net->step)));
    a.c2 = (float)(1.0 / (1.0 - std::pow((double)net->cfg.beta2, (double)net->step)));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, st, a);
    NET_HIP(hipGetLastError());
    ++net->version;
    if (int rc = launch_pack(net, st)) return rc;
    if (loss) {
        NET_HIP(hipMemcpyAsync(loss, net->loss_dev, 8, hipMemcpyDeviceToHost, st));
        NET_HIP(hipStreamSynchronize(st));
    }
    return JFNK_OK;
}

}  // extern "C"
