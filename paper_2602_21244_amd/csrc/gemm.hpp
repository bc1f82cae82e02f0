// Tiled BF16 MFMA GEMM with fused bias / activation / activation-derivative
// epilogues (used by the angle network and its training).
#pragma once
#include "common.hpp"

namespace dsmc {

enum { GEMM_ACT_NONE = 0, GEMM_ACT_SILU = 1, GEMM_ACT_SOFTPLUS = 2 };

struct GemmArgs {
    const __bf16* a;
    const __bf16* b;
    int64_t lda, ldb;
    int ta, tb;            // A(m,k) = ta ? a[k lda + m] : a[m lda + k]; B(k,n) = tb ? b[n ldb + k] : b[k ldb + n]
    int64_t M, N, K;
    const float* bias;     // [N] or null
    float* z_out;          // pre-activation (after bias) [M][ldz] or null
    const float* dact_z;   // if set: v *= act'(dact_z[m][n]) instead of applying act
    int64_t ldz;
    int act;
    int accumulate;        // out_f32 += v
    float* out_f32;        // [M][ldo] or null
    __bf16* out_bf16;      // [M][ldo] or null
    int64_t ldo;
    float* partial;        // split-K partials [splits][M][N] (splits > 1)
};

// Launch on stream s; splits > 1 divides K over workgroups (FP32 partials
// summed in a fixed order).
int gemm_bf16(const GemmArgs& g, int splits, hipStream_t s);

}  // namespace dsmc
