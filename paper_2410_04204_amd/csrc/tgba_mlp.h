// Internal interface of the learned truncation (tgba_mlp.hip).
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "tgba_internal.h"

namespace tgba {

constexpr int kMlpIn = 32, kMlpHidden = 256;
constexpr int64_t kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + 2 * (kMlpHidden * kMlpHidden + kMlpHidden) +
                               kMlpHidden + 1;

// Mode tables of both sectors and the energy reference, passed by value to the
// feature kernel.
struct MlpTab {
    double k[2][kMaxN];
    double eps[2][kMaxN];
    double h, e0;
    int N;
};

inline void mlp_tab_from_basis(const Basis &b, MlpTab &t) {
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < kMaxN; ++i) {
            t.k[s][i] = (i < b.N) ? b.k[s][i] : 0.0;
            t.eps[s][i] = (i < b.N) ? b.eps[s][i] : 0.0;
        }
    t.h = b.h_perp;
    t.e0 = b.e0;
    t.N = b.N;
}

// Features of n states (device arrays); sector[a] (0 NS, 1 R) or, with
// sector == NULL, NS for a < n_ns and R otherwise.  F: n x 32 row-major, ldf.
int mlp_features(const MlpTab &tab, int64_t n, const uint64_t *masks, const double *e, const uint8_t *sector,
                 int64_t n_ns, float *F, int64_t ldf, hipStream_t st);
// BF16 scores of n feature rows.
int mlp_score_bf16(int64_t n, const float *X, int64_t ldx, const float *params, float *y, hipStream_t st);
// Positions (ascending) of the `keep` largest scores; equal scores are taken
// in position order.  Synchronises the stream.
int mlp_select_top(int64_t n, const float *scores, int64_t keep, std::vector<int64_t> &sel, hipStream_t st);

}  // namespace tgba
