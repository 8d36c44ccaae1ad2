// Learned Newton initial guess: shapes of the network and the internal entry
// point the solver context uses.  The network is described with its C ABI in
// include/jfnk.h.
#pragma once
#include <stdint.h>

#include "jfnk.h"

namespace jfnk {
namespace net {

constexpr int kLayers = 6;
constexpr int kTaps = 5;
constexpr int kHalo = 2 * kLayers;        // cells of context per side for 6 layers of kernel 5
constexpr int kTile = 128;                // output cells per inference / training tile
constexpr int kWin = kTile + 2 * kHalo;   // cells a fused tile reads
constexpr double kN0 = 1e8;               // density unit of the a(n) transform, m^-3

__host__ __device__ constexpr int cin(int l) { return l == 0 ? 8 : 64; }
__host__ __device__ constexpr int cout(int l) { return l == kLayers - 1 ? 2 : 64; }
// output channels padded to whole 16-wide matrix tiles
__host__ __device__ constexpr int coutp(int l) { return l == kLayers - 1 ? 16 : 64; }
__host__ __device__ constexpr int64_t wcount(int l) { return (int64_t)cout(l) * kTaps * cin(l); }
__host__ __device__ constexpr int64_t pcount(int l) { return wcount(l) + cout(l); }
__host__ __device__ constexpr int64_t poffset(int l) {
    return l == 0 ? 0 : poffset(l - 1) + pcount(l - 1);
}
constexpr int64_t kParams = poffset(kLayers);

}  // namespace net

// Guess of the learned network for the columns of p whose flag in
// use_col (HOST [ncols]) is nonzero; other columns' outputs are left as they
// are.  Requires the network's prediction capacity (ensure_predict_capacity)
// to cover p.  Returns a JFNK_* code; the message goes to the network.
int net_predict_masked(jfnk_net* net, const jfnk_problem* p, const jfnk_state* x,
                       const uint8_t* use_col, double* ne_out, double* phi_out, void* stream);
int net_ensure_predict_capacity(jfnk_net* net, int32_t max_cols, int64_t max_total_cells);
// Counter of weight changes (set_params, train_step): a context that judged
// the network's candidates re-judges them after the weights change.
uint64_t net_version(const jfnk_net* net);

}  // namespace jfnk
