// Tiled BF16 matrix-core GEMM with fused epilogues, for networks whose layers
// do not fit the fused in-LDS MLP kernel (the angle network of section
// "Neural Network Architecture": 2 -> 512 -> 512 -> 512 -> 256 -> 128 -> 1).
//
//   C[m][n] = epilogue( sum_k A(m, k) B(k, n) ),   A, B bf16, FP32 accumulate
//   A(m, k) = TA ? a[k lda + m] : a[m lda + k]
//   B(k, n) = TB ? b[n ldb + k] : b[k ldb + n]
//
// A 256-thread workgroup computes a 128 x 128 tile: each wave a 64 x 64 block
// as 2 x 2 v_mfma_f32_32x32x16_bf16 accumulators.  Operand tiles (128 x 32)
// are staged in LDS with k contiguous (row stride 40 bf16 to spread banks),
// double-buffered: the next tile is loaded into registers during the MFMAs;
// operands that are k-contiguous in memory are copied with 16-byte loads, the
// transposed ones are scattered into that layout element by element.  A
// split of K (the split index fastest in the 1-D grid) writes FP32 partials
// that a second kernel sums in a fixed order, so results do not depend on
// timing.
#include "gemm.hpp"

namespace dsmc {

typedef __bf16 bf16x8g __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float floatx16g __attribute__((__vector_size__(16 * sizeof(float))));

constexpr int GM = 128, GN = 128, GK = 32, GLD = GK + 8;
constexpr int G_CHUNKS = GM * GK / 8 / 256;   // 8-element chunks per thread and operand
constexpr int G_THREADS = 256;

// Activations of the epilogue with the hardware exp2 / log2 / reciprocal
// (the results are rounded to bf16 for the next layer; the pre-activations
// are kept in FP32 separately).
__device__ __forceinline__ float sigm(float z)
{
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

__device__ __forceinline__ float act_apply(int act, float z)
{
    switch (act) {
    case GEMM_ACT_SILU: return z * sigm(z);
    case GEMM_ACT_SOFTPLUS:
        // ln(1 + e^z) = max(z, 0) + ln(1 + e^-|z|)
        return fmaxf(z, 0.0f) + 0.69314718055994531f *
                                    __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(
                                                                     -1.4426950408889634f *
                                                                     fabsf(z)));
    case GEMM_ACT_RELU: return z > 0.0f ? z : 0.0f;
    default: return z;
    }
}

__device__ __forceinline__ float act_deriv(int act, float z)
{
    switch (act) {
    case GEMM_ACT_SILU: {
        const float s = sigm(z);
        return s * (1.0f + z * (1.0f - s));
    }
    case GEMM_ACT_SOFTPLUS: return sigm(z);
    case GEMM_ACT_RELU: return z > 0.0f ? 1.0f : 0.0f;
    default: return 1.0f;
    }
}

// zd: dact_z at (m, n) when dact_z is set (loaded by the caller).
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, int64_t m, int64_t n, float v,
                                              float zd)
{
    const int64_t oz = gemm_off(m, n, g.ldz, g.bsz), oo = gemm_off(m, n, g.ldo, g.bso);
    if (g.bias) v += g.bias[n];
    if (g.z_out) g.z_out[oz] = v;
    if (g.dact_z) v *= act_deriv(g.act, zd);
    else v = act_apply(g.act, v);
    if (g.accumulate && g.out_f32) v += g.out_f32[oo];
    if (g.out_f32) g.out_f32[oo] = v;
    if (g.out_bf16) g.out_bf16[oo] = (__bf16)v;
}

// One operand tile (rows [r0, r0 + 128) x k [k0, k0 + GK)) in flight: each
// thread holds G_CHUNKS 8-element chunks.  kcontig: element (row, k) at
// p[row * ld + k], chunks run along k; otherwise at p[k * ld + row], chunks
// run along rows and are scattered into the k-contiguous LDS layout.
// Out-of-range elements are zero.
struct TileRegs {
    bf16x8g v[G_CHUNKS];
};

__device__ __forceinline__ void load_tile(const __bf16* __restrict__ p, int64_t ld, int64_t bs,
                                          int64_t rows, int64_t K, int64_t r0, int64_t k0,
                                          bool kcontig, TileRegs& R)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < G_CHUNKS; ++q) {
        const int c = t + G_THREADS * q;
        int64_t gr, gk;
        const __bf16* src;
        bool full;
        if (kcontig) {
            gr = r0 + c / (GK / 8);
            gk = k0 + (c % (GK / 8)) * 8;
            src = p + gemm_off(gr, gk, ld, bs);
            full = gr < rows && gk + 8 <= K;
        } else {
            gk = k0 + (c >> 4);
            gr = r0 + (c & 15) * 8;
            src = p + gemm_off(gk, gr, ld, bs);
            full = gk < K && gr + 8 <= rows;
        }
        if (full && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
            R.v[q] = *reinterpret_cast<const bf16x8g*>(src);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool ok = kcontig ? (gr < rows && gk + e < K) : (gk < K && gr + e < rows);
                R.v[q][e] = ok ? src[e] : (__bf16)0.0f;
            }
        }
    }
}

__device__ __forceinline__ void store_tile(const TileRegs& R, bool kcontig, __bf16* tile)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < G_CHUNKS; ++q) {
        const int c = t + G_THREADS * q;
        if (kcontig) {
            *reinterpret_cast<bf16x8g*>(tile + (c / (GK / 8)) * GLD + (c % (GK / 8)) * 8) = R.v[q];
        } else {
            const int kk = c >> 4, rc = (c & 15) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) tile[(rc + e) * GLD + kk] = R.v[q][e];
        }
    }
}

// Double-buffered main loop: the next k tile is loaded into registers while
// the current one is multiplied from LDS, then stored into the other buffer;
// one barrier per k tile.
__global__ void __launch_bounds__(G_THREADS, 3)
k_gemm_bf16(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[2][GM * GLD];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][GN * GLD];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int h = lane >> 5, col = lane & 31;
    // XCD-aware tile order: workgroups are dealt to the 8 XCDs in turn, so
    // workgroup w runs on XCD w % 8; the n tiles of one m tile are given to
    // consecutive workgroups of the same XCD and share its L2 copy of the A
    // rows.
    // With a K split the grid is tiles x splits in one dimension, split
    // fastest, so a few output tiles with many splits still spread over
    // every XCD.  With fewer than eight m tiles (a short, wide C) the tiles
    // are dealt m fastest: the few A rows are shared by every XCD anyway.
    const int64_t m_tiles = (g.M + GM - 1) / GM, n_tiles = (g.N + GN - 1) / GN;
    const int64_t wid = blockIdx.x;
    int64_t mt, nt, split = 0;
    const int64_t splits = g.ksplits > 1 ? g.ksplits : 1;
    if (splits > 1) {
        split = wid % splits;
        const int64_t tile = wid / splits;
        mt = tile / n_tiles;
        nt = tile % n_tiles;
    } else if (m_tiles >= 8) {
        const int64_t r8 = wid >> 3;
        mt = (r8 / n_tiles) * 8 + (wid & 7);
        nt = r8 % n_tiles;
    } else {
        mt = wid % m_tiles;
        nt = wid / m_tiles;
    }
    if (mt >= m_tiles) return;
    const int64_t m0 = mt * GM, n0 = nt * GN;
    // split length a whole number of k tiles, so every k tile (and every
    // 8-element chunk of it) starts on a multiple of GK and never straddles a
    // GEMM_RB block of a row-blocked operand; trailing splits may be empty
    const int64_t kc = ((g.K + splits - 1) / splits + GK - 1) / GK * GK;
    const int64_t kbeg = split * kc;
    const int64_t kend = kbeg + kc < g.K ? kbeg + kc : g.K;
    const bool a_kc = !g.ta, b_kc = g.tb;

    floatx16g acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    TileRegs ra, rb;
    if (kbeg < kend) {
        load_tile(g.a, g.lda, g.bsa, g.M, kend, m0, kbeg, a_kc, ra);
        load_tile(g.b, g.ldb, g.bsb, g.N, kend, n0, kbeg, b_kc, rb);
        store_tile(ra, a_kc, As[0]);
        store_tile(rb, b_kc, Bs[0]);
    }
    __syncthreads();
    int cur = 0;
    // row sums of A: thread t adds k half (t & 1) of tile row t >> 1
    const bool asum = g.asum_out != nullptr && nt == 0;
    float arow = 0.0f;
    for (int64_t k0 = kbeg; k0 < kend; k0 += GK) {
        const bool more = k0 + GK < kend;
        if (more) {
            load_tile(g.a, g.lda, g.bsa, g.M, kend, m0, k0 + GK, a_kc, ra);
            load_tile(g.b, g.ldb, g.bsb, g.N, kend, n0, k0 + GK, b_kc, rb);
        }
        const __bf16* A_ = As[cur];
        const __bf16* B_ = Bs[cur];
        if (asum) {
            const __bf16* ar = A_ + (threadIdx.x >> 1) * GLD + (threadIdx.x & 1) * (GK / 2);
            const bf16x8g a0 = *reinterpret_cast<const bf16x8g*>(ar);
            const bf16x8g a1 = *reinterpret_cast<const bf16x8g*>(ar + 8);
#pragma unroll
            for (int e = 0; e < 8; ++e) arow += (float)a0[e];
#pragma unroll
            for (int e = 0; e < 8; ++e) arow += (float)a1[e];
        }
#pragma unroll
        for (int ks = 0; ks < GK / 16; ++ks) {
            bf16x8g fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                fa[i] = *reinterpret_cast<const bf16x8g*>(
                    A_ + (wm * 64 + i * 32 + col) * GLD + ks * 16 + 8 * h);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                fb[j] = *reinterpret_cast<const bf16x8g*>(
                    B_ + (wn * 64 + j * 32 + col) * GLD + ks * 16 + 8 * h);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j],
                                                                        0, 0, 0);
        }
        if (more) {
            store_tile(ra, a_kc, As[cur ^ 1]);
            store_tile(rb, b_kc, Bs[cur ^ 1]);
        }
        __syncthreads();
        cur ^= 1;
    }

    if (asum) {
        const float tot = arow + __shfl_xor(arow, 1, 64);   // halves in a fixed order
        const int64_t m = m0 + (threadIdx.x >> 1);
        if ((threadIdx.x & 1) == 0 && m < g.M) {
            if (splits > 1) g.asum_part[split * g.M + m] = tot;
            else g.asum_out[m] = g.accumulate ? g.asum_out[m] + tot : tot;
        }
    }

    // epilogue: register r of lane (h, col) holds row 8 (r / 4) + 4 h + r % 4, column col
    float* part = g.partial ? g.partial + split * g.M * g.N : nullptr;
    // The derivative epilogue's z values of each half of the wave's block
    // are loaded before its first store: the stores may alias them as far as
    // the compiler knows, so loads interleaved with stores would each wait a
    // full round trip.
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        float zd[2][16];
        if (!part && g.dact_z) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t m = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                    const int64_t n = n0 + wn * 64 + j * 32 + col;
                    zd[j][r] = (m < g.M && n < g.N) ? g.dact_z[gemm_off(m, n, g.ldz, g.bsz)]
                                                    : 0.0f;
                }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t m = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int64_t n = n0 + wn * 64 + j * 32 + col;
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                if (part) {
                    part[m * g.N + n] = v;
                    continue;
                }
                gemm_epilogue(g, m, n, v, g.dact_z ? zd[j][r] : 0.0f);
            }
    }
}

// Sum of the K-split partials, then the epilogue.  A workgroup takes 64
// outputs; its four waves sum interleaved quarters of the splits (split
// s to wave s % 4, in split order), and the four sums are added in wave
// order: a fixed order whatever the launch.
__global__ void __launch_bounds__(256)
k_gemm_reduce(GemmArgs g, int splits)
{
    __shared__ float part[4][64];
    const int64_t total = g.M * g.N;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t q0 = (int64_t)blockIdx.x * 64; q0 < total; q0 += (int64_t)gridDim.x * 64) {
        const int64_t q = q0 + lane;
        float v = 0.0f;
        if (q < total) {
            int s = w;
            for (; s + 12 < splits; s += 16) {
                const float a0 = g.partial[(int64_t)s * total + q];
                const float a1 = g.partial[(int64_t)(s + 4) * total + q];
                const float a2 = g.partial[(int64_t)(s + 8) * total + q];
                const float a3 = g.partial[(int64_t)(s + 12) * total + q];
                v += a0; v += a1; v += a2; v += a3;
            }
            for (; s < splits; s += 4) v += g.partial[(int64_t)s * total + q];
        }
        part[w][lane] = v;
        __syncthreads();
        if (w == 0 && q < total) {
            const float r = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
            const int64_t m = q / g.N, n = q % g.N;
            gemm_epilogue(g, m, n, r,
                          g.dact_z ? g.dact_z[gemm_off(m, n, g.ldz, g.bsz)] : 0.0f);
        }
        __syncthreads();
    }
    // row sums of A from the per-split sums, in the same fixed order (split
    // s to wave s % 4, the four wave sums in wave order), by the last
    // workgroups of the grid
    if (g.asum_out) {
        const int64_t nb = (g.M + 63) / 64;
        const int64_t b = (int64_t)gridDim.x - 1 - blockIdx.x;
        for (int64_t mb = b; mb < nb; mb += gridDim.x) {
            const int64_t m = mb * 64 + lane;
            float v = 0.0f;
            if (m < g.M) {
                int s = w;
                for (; s + 12 < splits; s += 16) {
                    const float a0 = g.asum_part[(int64_t)s * g.M + m];
                    const float a1 = g.asum_part[(int64_t)(s + 4) * g.M + m];
                    const float a2 = g.asum_part[(int64_t)(s + 8) * g.M + m];
                    const float a3 = g.asum_part[(int64_t)(s + 12) * g.M + m];
                    v += a0; v += a1; v += a2; v += a3;
                }
                for (; s < splits; s += 4) v += g.asum_part[(int64_t)s * g.M + m];
            }
            part[w][lane] = v;
            __syncthreads();
            if (w == 0 && m < g.M) {
                const float r = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
                g.asum_out[m] = g.accumulate ? g.asum_out[m] + r : r;
            }
            __syncthreads();
        }
    }
}

// Column sums in two fixed-order stages.  Partial: a workgroup takes
// COLSUM_ROWS rows and 64 columns; wave w sums rows w, w + 4, ... of the
// chunk and the four wave sums are added in wave order.  Final: a workgroup
// takes 64 columns; its 16 waves sum chunks g, g + 16, ... and the sums are
// added in wave order.
__global__ void __launch_bounds__(256)
k_col_partial(const float* __restrict__ a, int64_t R, int n, const float* __restrict__ x,
              float* __restrict__ red)
{
    __shared__ float ps[4][3][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.y * 64 + lane;
    const int64_t r0 = (int64_t)blockIdx.x * COLSUM_ROWS;
    const int64_t r1 = r0 + COLSUM_ROWS < R ? r0 + COLSUM_ROWS : R;
    float s = 0.f, s0 = 0.f, s1 = 0.f;
    if (c < n) {
        int64_t r = r0 + w;
        for (; r + 28 < r1; r += 32) {
            float d[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) d[u] = a[(r + 4 * u) * n + c];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                s += d[u];
                if (x) {
                    s0 += d[u] * x[2 * (r + 4 * u)];
                    s1 += d[u] * x[2 * (r + 4 * u) + 1];
                }
            }
        }
        for (; r < r1; r += 4) {
            const float d = a[r * n + c];
            s += d;
            if (x) {
                s0 += d * x[2 * r];
                s1 += d * x[2 * r + 1];
            }
        }
    }
    ps[w][0][lane] = s;
    ps[w][1][lane] = s0;
    ps[w][2][lane] = s1;
    __syncthreads();
    if (w == 0 && c < n) {
        float* o = red + ((int64_t)blockIdx.x * n + c) * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            o[k] = ((ps[0][k][lane] + ps[1][k][lane]) + ps[2][k][lane]) + ps[3][k][lane];
    }
}

constexpr int COLSUM_FINAL_WAVES = 16;

__global__ void __launch_bounds__(64 * COLSUM_FINAL_WAVES)
k_col_final(const float* __restrict__ red, int64_t chunks, int n, float* __restrict__ out,
            float* __restrict__ out2, int accumulate)
{
    __shared__ float ps[COLSUM_FINAL_WAVES][3][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    float s = 0.f, s0 = 0.f, s1 = 0.f;
    if (c < n) {
        for (int64_t q = w; q < chunks; q += COLSUM_FINAL_WAVES) {
            const float* o = red + (q * n + c) * 3;
            s += o[0];
            s0 += o[1];
            s1 += o[2];
        }
    }
    ps[w][0][lane] = s;
    ps[w][1][lane] = s0;
    ps[w][2][lane] = s1;
    __syncthreads();
    if (w == 0 && c < n) {
        float t[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < COLSUM_FINAL_WAVES; ++q)
#pragma unroll
            for (int k = 0; k < 3; ++k) t[k] += ps[q][k][lane];
        out[c] = accumulate ? out[c] + t[0] : t[0];
        if (out2) {
            out2[2 * c] = accumulate ? out2[2 * c] + t[1] : t[1];
            out2[2 * c + 1] = accumulate ? out2[2 * c + 1] + t[2] : t[2];
        }
    }
}

int colsum_f32(const float* a, int64_t R, int n, const float* x2, float* red, float* out,
               float* out2, int accumulate, hipStream_t s)
{
    if (R <= 0 || n <= 0) return DSMC_OK;
    const int64_t chunks = (R + COLSUM_ROWS - 1) / COLSUM_ROWS;
    if (chunks > 2147483647) return arg_error("colsum: too many rows");
    dim3 pg((unsigned)chunks, (unsigned)((n + 63) / 64));
    k_col_partial<<<pg, 256, 0, s>>>(a, R, n, x2, red);
    DSMC_LAUNCH_CHECK("colsum:partial");
    k_col_final<<<(n + 63) / 64, 64 * COLSUM_FINAL_WAVES, 0, s>>>(red, chunks, n, out, out2,
                                                                  accumulate);
    DSMC_LAUNCH_CHECK("colsum:final");
    return DSMC_OK;
}

int gemm_bf16(const GemmArgs& g0, int splits, hipStream_t s)
{
    GemmArgs g = g0;
    if (g.M <= 0 || g.N <= 0) return DSMC_OK;
    if (splits < 1) splits = 1;
    const int64_t gx = (g.M + GM - 1) / GM, gy = (g.N + GN - 1) / GN;
    const int64_t tiles = splits > 1 ? gx * gy * splits : (gx >= 8 ? (gx + 7) / 8 * 8 * gy : gx * gy);
    if (tiles > 2147483647 || splits > 65535) return arg_error("gemm: grid too large");
    if (splits > 1 && !g.partial) return arg_error("gemm: split-K needs a partial buffer");
    if (splits > 1 && g.asum_out && !g.asum_part)
        return arg_error("gemm: split-K row sums need a partial buffer");
    if (splits == 1) g.partial = nullptr;
    g.ksplits = splits;
    dim3 grid((unsigned)tiles, 1u, 1u);
    k_gemm_bf16<<<grid, G_THREADS, 0, s>>>(g);
    DSMC_LAUNCH_CHECK("gemm_bf16");
    if (splits > 1) {
        const int64_t total = g.M * g.N;
        int64_t blocks = (total + 63) / 64;
        const int pb = persistent_blocks(256);
        if (blocks > pb) blocks = pb;
        k_gemm_reduce<<<(int)blocks, 256, 0, s>>>(g, splits);
        DSMC_LAUNCH_CHECK("gemm_reduce");
    }
    return DSMC_OK;
}

}  // namespace dsmc
