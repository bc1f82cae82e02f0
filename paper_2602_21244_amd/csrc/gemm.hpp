// Tiled BF16 MFMA GEMM with fused bias / activation / activation-derivative
// epilogues (used by the angle network and its training).
#pragma once
#include "common.hpp"

namespace dsmc {

enum { GEMM_ACT_NONE = 0, GEMM_ACT_SILU = 1, GEMM_ACT_SOFTPLUS = 2, GEMM_ACT_RELU = 3 };

constexpr int GEMM_RB = 128;   // rows per block of a row-blocked operand

// Offset of element (i, j) of a matrix with leading dimension ld, or, with
// block stride bs != 0, of the row-blocked layout described in GemmArgs.
__host__ __device__ inline int64_t gemm_off(int64_t i, int64_t j, int64_t ld, int64_t bs)
{
    return bs ? i * GEMM_RB + (j / GEMM_RB) * bs + (j % GEMM_RB) : i * ld + j;
}

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
    // Row blocking: an operand, z or the outputs with bs* != 0 store element
    // (i, j) of the layouts above (i the index multiplied by ld, j the one
    // added) at i * ld + (j / GEMM_RB) * bs + j % GEMM_RB, with ld = GEMM_RB:
    // a [units][rows] matrix kept as blocks of GEMM_RB rows, units-major
    // inside each block (a tile's rows then lie in one contiguous block).
    int64_t bsa, bsb, bsz, bso;
    // Row sums of A over K (sum_k A(m, k), e.g. a bias gradient), when
    // asum_out is set: FP32, fixed order, += when accumulate; with a K split
    // the per-split sums go to asum_part [splits][M] and the reduce kernel
    // adds them in split order.
    float* asum_out;
    float* asum_part;
    float* partial;        // split-K partials [splits][M][N] (splits > 1)
    int ksplits;           // set by gemm_bf16: K splits (one 1-D grid of tiles x splits)
};

// Launch on stream s; splits > 1 divides K over workgroups (FP32 partials
// summed in a fixed order).
int gemm_bf16(const GemmArgs& g, int splits, hipStream_t s);

// Column sums of a[R][n] (FP32) in a fixed order: out[c] = sum_r a[r][c]
// (+= when accumulate); with x2 != null also out2[2c + q] = sum_r a[r][c] x2[r][q].
// red: colsum_ws_floats(R, n) floats of workspace.
constexpr int COLSUM_ROWS = 256;
inline size_t colsum_ws_floats(int64_t R, int n)
{
    const int64_t chunks = (R + COLSUM_ROWS - 1) / COLSUM_ROWS;
    return (size_t)(chunks > 0 ? chunks : 1) * (size_t)n * 3;
}
int colsum_f32(const float* a, int64_t R, int n, const float* x2, float* red, float* out,
               float* out2, int accumulate, hipStream_t s);

}  // namespace dsmc
