// Neural collision operator (sections "Cell-Based Neural Collision Operator"
// and "Hard Conservation via Projection and Pair Update").
//
// BF16 path: one fused kernel evaluates the whole MLP on the matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation) for 32-row tiles per wave.
// Weights are bf16; every activation (and the network input) enters the
// matrix cores as a bf16 pair hi + lo (hi = bf16(h), lo = bf16(h - hi), 16
// significant bits), two MFMAs on the same weight fragment.  A trained
// network's output y can be much shorter than its terms (|y| ~ 0.01 against
// O(1) contributions), and u = y/|y| then turns single-bf16 rounding of the
// activations into direction errors of ~0.03 rad; with the pair the result
// is that of the bf16 weights to ~1e-4 rad.
// Each layer is computed transposed, D = W * H^T, so a wave's accumulators
// hold, for its 32 rows, the layer's outputs in the MFMA result layout; after
// the activation they are converted to bf16 and used directly as the B operand
// of the next layer.  The weights are staged once per workgroup in LDS in
// "fragment-major" order (the 64 lanes' 16-byte A fragments contiguous) with
// the columns permuted to match the register layout of the previous layer's
// outputs, so no LDS round trip of activations is needed.
//
// FP64 (and FP32) reference path: plain per-element kernels, used for parity
// with the FP64 oracle and for finite-difference gradient checks.
#include <math.h>
#include <stdlib.h>

#include "collide.hpp"
#include "gemm.hpp"

namespace dsmc {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float floatx16 __attribute__((__vector_size__(16 * sizeof(float))));

constexpr int MLP_MAX_LAYERS = 6;

struct MlpDev {
    int L;
    int dims[MLP_MAX_LAYERS + 1];
    int act;
    const void* W[MLP_MAX_LAYERS];
    const void* b[MLP_MAX_LAYERS];
    double inv_sigma_v;
    int split;
};

static int check_mlp(const dsmc_mlp* net, MlpDev* d)
{
    if (!net) return arg_error("dsmc_mlp: null");
    if (net->n_layers < 1 || net->n_layers > MLP_MAX_LAYERS)
        return arg_error("dsmc_mlp: n_layers %d not in [1, %d]", net->n_layers, MLP_MAX_LAYERS);
    if (net->act != DSMC_ACT_SILU && net->act != DSMC_ACT_RELU)
        return arg_error("dsmc_mlp: act %d", net->act);
    if (net->wdtype != DSMC_BF16 && net->wdtype != DSMC_F64 && net->wdtype != DSMC_F32)
        return arg_error("dsmc_mlp: wdtype %d", net->wdtype);
    d->L = net->n_layers;
    for (int l = 0; l <= net->n_layers; ++l) {
        if (net->dims[l] < 1 || net->dims[l] > 256)
            return arg_error("dsmc_mlp: dims[%d] = %d not in [1, 256]", l, net->dims[l]);
        d->dims[l] = net->dims[l];
    }
    for (int l = 0; l < net->n_layers; ++l) {
        if (!net->W[l] || !net->b[l]) return arg_error("dsmc_mlp: null W/b of layer %d", l);
        d->W[l] = net->W[l];
        d->b[l] = net->b[l];
    }
    if (!(net->sigma_v > 0)) return arg_error("dsmc_mlp: sigma_v must be > 0");
    d->inv_sigma_v = 1.0 / net->sigma_v;
    d->act = net->act;
    if (net->split != DSMC_SPLIT_ALL && net->split != DSMC_SPLIT_FRONT &&
        net->split != DSMC_SPLIT_FIRST)
        return arg_error("dsmc_mlp: split %d", net->split);
    d->split = net->split;
    return DSMC_OK;
}

// Shape the fused MFMA kernel supports.
static bool mfma_shape_ok(const MlpDev& d, int* H)
{
    if (d.L < 2) return false;
    const int h = d.dims[1];
    if (h != 64 && h != 128 && h != 256) return false;
    for (int l = 1; l < d.L; ++l)
        if (d.dims[l] != h) return false;
    if (d.dims[0] > 30 || d.dims[d.L] > 32) return false;
    *H = h;
    return true;
}

template <typename T>
__device__ __forceinline__ T act_t(T z, int act)
{
    if (act == DSMC_ACT_RELU) return z > T(0) ? z : T(0);
    return z / (T(1) + exp(-z));
}
template <typename T>
__device__ __forceinline__ T act_grad_t(T z, int act)
{
    if (act == DSMC_ACT_RELU) return z > T(0) ? T(1) : T(0);
    const T s = T(1) / (T(1) + exp(-z));
    return s * (T(1) + z * (T(1) - s));
}

// ------------------------------------------------------------------------
// Fused BF16 MFMA forward
// ------------------------------------------------------------------------
// The matrix cores compute s = c z instead of the pre-activation z, with
// c = -log2(e) for SiLU (then exp2(s) = exp(-z) needs no multiply) and c = 1
// for ReLU.  The network input and every bias are scaled by c; the hidden
// weights stay as they are, because every hidden layer's input (the scaled
// activation c act(z)) carries the same factor; the outputs are divided by c.
// Biases enter the MFMAs as an extra k step against a constant-one input, as
// a bf16 (hi, lo) split of c b, so no accumulator is initialised on the VALU.
template <int ACT> struct ActScale;
template <> struct ActScale<DSMC_ACT_SILU> {
    static constexpr float c = -1.4426950408889634f;
    static constexpr float inv = -0.69314718055994531f;
};
template <> struct ActScale<DSMC_ACT_RELU> {
    static constexpr float c = 1.0f;
    static constexpr float inv = 1.0f;
};

// c act(z) from s = c z.  SiLU: c z sigma(z) = s / (1 + 2^s).
template <int ACT>
__device__ __forceinline__ float act_scaled(float s)
{
    if (ACT == DSMC_ACT_RELU) return s > 0.f ? s : 0.f;
    return s * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(s));
}

struct FragLayout {
    int off[MLP_MAX_LAYERS];   // element offset of each layer's fragments in LDS
    int nb[MLP_MAX_LAYERS];    // 32-row output blocks
    int ks[MLP_MAX_LAYERS];    // 16-wide k steps, the bias step included
    int total_bf16;
    size_t bytes;
};

// LDS of one CU, which holds the whole bf16 network in fragment order.
constexpr size_t MLP_LDS_BYTES = 160 * 1024;

static FragLayout frag_layout(const MlpDev& d)
{
    FragLayout f{};
    int o = 0;
    for (int l = 0; l < d.L; ++l) {
        f.nb[l] = (d.dims[l + 1] + 31) / 32;
        f.ks[l] = (l == 0) ? ((d.dims[0] + 2 + 15) / 16) : (d.dims[l] / 16 + 1);
        f.off[l] = o;
        o += f.nb[l] * f.ks[l] * 64 * 8;
    }
    f.total_bf16 = o;
    f.bytes = (size_t)o * 2;
    return f;
}

// Input slot k (0..15) of the first k step in pairs mode.  Lane-half 0
// supplies xi, lane-half 1 supplies v_r / sigma_v, z and the two constant-one
// bias inputs, so that each half computes its own latents.  Returns the
// column of W, or -1 (hi bias), -2 (lo bias), -3 (unused).
__device__ __forceinline__ int pairs_slot_col(int k)
{
    switch (k) {
    case 0: return 3;
    case 1: return 4;
    case 2: return 5;
    case 8: return 0;
    case 9: return 1;
    case 10: return 2;
    case 11: return 6;
    case 12: return 7;
    case 13: return -1;
    case 14: return -2;
    default: return -3;
    }
}

// Column of W (or bias code, as above) feeding element e of lane-half h in
// k step ks of layer l (in = input width of the layer).
template <bool PAIRS>
__device__ __forceinline__ int frag_col(int layer, int in, int ks, int h, int e)
{
    if (layer == 0) {
        const int k = 16 * ks + 8 * h + e;
        if (PAIRS) return pairs_slot_col(k);
        return k < in ? k : (k == in ? -1 : (k == in + 1 ? -2 : -3));
    }
    if (ks == in / 16) return (h == 0 && e < 2) ? -1 - e : -3;
    const int pb = ks >> 1, jp = ks & 1;
    return pb * 32 + 16 * jp + 8 * (e >> 2) + 4 * h + (e & 3);
}

template <bool PAIRS, int ACT>
__device__ void stage_weights(const MlpDev& d, const FragLayout& f, __bf16* wl)
{
    constexpr float C = ActScale<ACT>::c;
    for (int l = 0; l < d.L; ++l) {
        const __bf16* W = static_cast<const __bf16*>(d.W[l]);
        const float* B = static_cast<const float*>(d.b[l]);
        const int out = d.dims[l + 1], in = d.dims[l];
        const int n_el = f.nb[l] * f.ks[l] * 64 * 8;
        for (int q = threadIdx.x; q < n_el; q += blockDim.x) {
            const int e = q & 7, lane = (q >> 3) & 63, frag = q >> 9;
            const int nb = frag / f.ks[l], ks = frag % f.ks[l];
            const int row = nb * 32 + (lane & 31);
            const int col = frag_col<PAIRS>(l, in, ks, lane >> 5, e);
            __bf16 w = (__bf16)0.0f;
            if (row < out) {
                if (col >= 0) {
                    w = W[(size_t)row * in + col];
                } else if (col >= -2) {
                    const float cb = C * B[row];
                    const __bf16 hi = (__bf16)cb;
                    w = (col == -1) ? hi : (__bf16)(cb - (float)hi);
                }
            }
            wl[f.off[l] + q] = w;
        }
    }
}

__device__ __forceinline__ bf16x8 lds_frag(const __bf16* wl, int off, int frag, int lane)
{
    return *reinterpret_cast<const bf16x8*>(wl + off + (frag * 64 + lane) * 8);
}

// Row mapping of accumulator register r for lane-half h.
__device__ __forceinline__ int acc_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

typedef __bf16 bf16x2 __attribute__((__vector_size__(2 * sizeof(__bf16))));

// Activation of 8 accumulator values as bf16 fragments.  PAIR: hi = bf16(v)
// and lo = bf16(v - hi); two values are rounded by one conversion and hi is
// read back as floats by shifting/masking the packed halves.  Otherwise hi
// only (lo is left untouched).
template <int ACT, bool PAIR>
__device__ __forceinline__ void to_frag(const floatx16& a, int jp, bf16x8& hi, bf16x8& lo)
{
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        const float v0 = act_scaled<ACT>(a[8 * jp + e]);
        const float v1 = act_scaled<ACT>(a[8 * jp + e + 1]);
        bf16x2 hp;
        hp[0] = (__bf16)v0;
        hp[1] = (__bf16)v1;
        hi[e] = hp[0];
        hi[e + 1] = hp[1];
        if (PAIR) {
            const uint32_t u = __builtin_bit_cast(uint32_t, hp);
            const float h0 = __builtin_bit_cast(float, u << 16);
            const float h1 = __builtin_bit_cast(float, u & 0xffff0000u);
            lo[e] = (__bf16)(v0 - h0);
            lo[e + 1] = (__bf16)(v1 - h1);
        }
    }
}

// Number of GEMM_RB-row blocks of a B-row batch (the row-blocked layout of
// the saved activations and of the backward's delta^T).
__host__ __device__ inline int64_t row_blocks(int64_t B) { return (B + GEMM_RB - 1) / GEMM_RB; }

struct RowsIO {
    const float* x;   // [B][dims0]
    const float* g;   // [B]
    float* y_raw;     // [B][dout]
    float* vr_out;    // [B][3]
    float* zsave;     // pre-activations of each hidden layer, row-blocked (below), or null
    __bf16* hsave;    // their bf16 activations, same layout, with zsave
    __bf16* xsave;    // the inputs in bf16, same layout, with zsave
    int64_t B;
};

template <typename VT> struct PairsIO {
    PairsView pr;
    int32_t n_cells;
    V3<const VT> v;
    dsmc_rng rng;
    PairBuf<VT> out;
};

// Box-Muller on the hardware transcendentals (v_log_f32 is log2, v_sin_f32
// and v_cos_f32 take revolutions, so sin(2 pi u) needs no scaling): used for
// the latents of the bf16 network only, whose inputs carry 16 significant
// bits (a bf16 pair), far above the ~1 ulp of these FP32 instructions.
__device__ __forceinline__ void box_muller_hw(float ua, float ub, float& n1, float& n2)
{
    const float R = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(1.0f - ua));
    n1 = R * __builtin_amdgcn_cosf(ub);
    n2 = R * __builtin_amdgcn_sinf(ub);
}

// The same on 53-bit uniforms: 1 - ua is formed in FP64 (it never rounds to
// zero) and both arguments are then rounded to FP32.
__device__ __forceinline__ void box_muller_hw53(double ua, double ub, float& n1, float& n2)
{
    const float w = (float)(1.0 - ua), b = (float)ub;
    const float R = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(w));
    n1 = R * __builtin_amdgcn_cosf(b);
    n2 = R * __builtin_amdgcn_sinf(b);
}

// One layer on NT tiles: acc holds s of the previous layer (NB blocks),
// nxt receives s of this layer (NBO blocks).  The activation of block nb
// produces the inputs of k steps 2 nb and 2 nb + 1, whose MFMAs are issued
// right away, so the matrix cores run while the next block is activated.
// PAIR: each input as a bf16 pair (two MFMAs per k step), else one bf16.
// SAVE_H (one tile, NT == 1): the activations are also stored in bf16 at
// hp[unit * GEMM_RB] (the row-blocked layout of the saved activations; hp
// null for rows past the end).
template <int NB, int NBO, int NT, int ACT, bool PAIR, bool SAVE_H = false>
__device__ __forceinline__ void layer_step(const __bf16* wl, int off, int ksl,
                                           const floatx16 (&acc)[NT][NB],
                                           floatx16 (&nxt)[NT][NBO], const bf16x8& bone,
                                           int lane, __bf16* hp = nullptr)
{
    static_assert(!SAVE_H || NT == 1, "activation save takes one tile per wave");
    const floatx16 zero = {};
#pragma unroll
    for (int nb2 = 0; nb2 < NBO; ++nb2) {
        const bf16x8 a = lds_frag(wl, off, nb2 * ksl + (ksl - 1), lane);
#pragma unroll
        for (int t = 0; t < NT; ++t)
            nxt[t][nb2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bone, zero, 0, 0, 0);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        bf16x8 b0[NT], b1[NT], c0[NT], c1[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            to_frag<ACT, PAIR>(acc[t][nb], 0, b0[t], c0[t]);
            to_frag<ACT, PAIR>(acc[t][nb], 1, b1[t], c1[t]);
        }
        if (SAVE_H && hp) {
            // h = hi / c: the bf16 activation the next layer used, unscaled
            const int hh = lane >> 5;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                hp[(nb * 32 + acc_row(e, hh)) * GEMM_RB] =
                    (__bf16)((float)b0[0][e] * ActScale<ACT>::inv);
                hp[(nb * 32 + acc_row(8 + e, hh)) * GEMM_RB] =
                    (__bf16)((float)b1[0][e] * ActScale<ACT>::inv);
            }
        }
#pragma unroll
        for (int nb2 = 0; nb2 < NBO; ++nb2) {
            const bf16x8 a0 = lds_frag(wl, off, nb2 * ksl + 2 * nb, lane);
            const bf16x8 a1 = lds_frag(wl, off, nb2 * ksl + 2 * nb + 1, lane);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                nxt[t][nb2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0[t], nxt[t][nb2], 0, 0, 0);
                if (PAIR)
                    nxt[t][nb2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, c0[t], nxt[t][nb2], 0, 0, 0);
                nxt[t][nb2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1[t], nxt[t][nb2], 0, 0, 0);
                if (PAIR)
                    nxt[t][nb2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, c1[t], nxt[t][nb2], 0, 0, 0);
            }
        }
    }
}

template <int H, int NT, bool SAVE, int ACT>
__device__ __forceinline__ void save_pre(const RowsIO& rio, int l, const int64_t (&row)[NT],
                                         const bool (&valid)[NT], const floatx16 (&acc)[NT][H / 32],
                                         int h)
{
    if (!SAVE) return;
    // Row-blocked transposed layout (blocks of GEMM_RB rows, [unit][row]
    // inside a block): the 32 lanes of a lane-half hold 32 consecutive rows
    // of one unit, so each store is one contiguous run, and a tile's stores
    // stay inside one block.  The activations are stored by layer_step,
    // where they are formed.
    constexpr float IC = ActScale<ACT>::inv;
    const size_t Bp = (size_t)row_blocks(rio.B) * GEMM_RB;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (!valid[t]) continue;
        const size_t base = (size_t)(l - 1) * H * Bp + (size_t)(row[t] / GEMM_RB) * H * GEMM_RB +
                            (size_t)(row[t] % GEMM_RB);
#pragma unroll
        for (int nb = 0; nb < H / 32; ++nb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const size_t q = base + (size_t)(nb * 32 + acc_row(r, h)) * GEMM_RB;
                rio.zsave[q] = acc[t][nb][r] * IC;
            }
    }
}

// Each wave processes NT tiles of 32 rows; every A fragment read from LDS
// feeds NT MFMAs.  Pairs mode: the lane of row r in lane-half 0 computes the
// pair's xi, the lane in lane-half 1 its z and v_r (dims[0] == 8).
template <int H, bool PAIRS, typename VT, int ACT, bool SAVE, int NT, int TPB, int SPLIT>
__global__ void __launch_bounds__(TPB)
k_mlp_bf16(MlpDev d, FragLayout f, RowsIO rio, PairsIO<VT> pio)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __bf16* wl = reinterpret_cast<__bf16*>(smem);
    stage_weights<PAIRS, ACT>(d, f, wl);
    __syncthreads();

    constexpr float C = ActScale<ACT>::c, IC = ActScale<ACT>::inv;
    const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
    const int waves = blockDim.x >> 6;
    const int64_t nrows = PAIRS ? pio.pr.total(pio.n_cells) : rio.B;
    const int L = d.L, dout = d.dims[L];
    constexpr int NB = H / 32;
    bf16x8 bone;
#pragma unroll
    for (int e = 0; e < 8; ++e) bone[e] = (__bf16)((h == 0 && e < 2) ? 1.0f : 0.0f);
    const floatx16 zero = {};

    // pairs mode: the next tile's pair record (cell, i, j) is loaded while the
    // current tile runs through the network, so a tile's first loads wait on
    // one round trip (offsets and velocities) instead of two
    const int64_t gstride = (int64_t)gridDim.x * waves;
    int32_t pf_k[NT], pf_i[NT], pf_j[NT];
    auto prefetch = [&](int64_t g) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t r = (g * NT + t) * 32 + col;
            pf_k[t] = 0;
            pf_i[t] = 0;
            pf_j[t] = 0;
            if (PAIRS && r < nrows) {
                pf_k[t] = pio.pr.cell[r];
                if (h == 1) {
                    pf_i[t] = pio.pr.i[r];
                    pf_j[t] = pio.pr.j[r];
                }
            }
        }
    };
    if (PAIRS) prefetch((int64_t)blockIdx.x * waves + (threadIdx.x >> 6));
    for (int64_t grp = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); grp * 32 * NT < nrows;
         grp += gstride) {
        int64_t row[NT];
        bool valid[NT];
        float xin[NT][2][8];  // c x of the first two k steps (1 in the bias slots)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            row[t] = (grp * NT + t) * 32 + col;
            valid[t] = row[t] < nrows;
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 8; ++e) xin[t][q][e] = 0.0f;
            if (PAIRS) {
                if (h == 1) {
                    xin[t][0][5] = 1.0f;
                    xin[t][0][6] = 1.0f;
                }
                if (valid[t] && sizeof(VT) == 4) {
                    // FP32 latents: the xi draw (slot 2) and the z draw
                    // (slot 3) take the same instructions, so each lane-half
                    // runs one Philox call and the same Box-Muller transforms
                    // on its own slot without divergence (half 1 discards the
                    // second transform).
                    const int64_t r = row[t];
                    const int32_t k = pf_k[t];
                    const uint32_t a = (uint32_t)(r - pio.pr.off[k]);
                    const U4 rr = draw(pio.rng, a, (uint32_t)k, SLOT_LAT0 + (uint32_t)h);
                    float n0, n1, n2, spare;
                    box_muller_hw(unif24(rr.a), unif24(rr.b), n0, n1);
                    box_muller_hw(unif24(rr.c), unif24(rr.d), n2, spare);
                    if (h == 0) {
                        xin[t][0][0] = C * n0;
                        xin[t][0][1] = C * n1;
                        xin[t][0][2] = C * n2;
                    } else {
                        const int32_t i = pf_i[t], j = pf_j[t];
                        const VT isv = (VT)d.inv_sigma_v;
                        xin[t][0][0] = C * (float)((pio.v.x[i] - pio.v.x[j]) * isv);
                        xin[t][0][1] = C * (float)((pio.v.y[i] - pio.v.y[j]) * isv);
                        xin[t][0][2] = C * (float)((pio.v.z[i] - pio.v.z[j]) * isv);
                        xin[t][0][3] = C * n0;
                        xin[t][0][4] = C * n1;
                    }
                } else if (valid[t]) {
                    // FP64 velocities: the 53-bit uniforms of the FP64
                    // contract, transformed on the FP32 hardware units
                    const int64_t r = row[t];
                    const int32_t k = pf_k[t];
                    const uint32_t a = (uint32_t)(r - pio.pr.off[k]);
                    if (h == 0) {
                        double U[4];
                        uniforms_xi(pio.rng, a, (uint32_t)k, U);
                        float xi[3], spare;
                        box_muller_hw53(U[0], U[1], xi[0], xi[1]);
                        box_muller_hw53(U[2], U[3], xi[2], spare);
                        xin[t][0][0] = C * xi[0];
                        xin[t][0][1] = C * xi[1];
                        xin[t][0][2] = C * xi[2];
                    } else {
                        double U[2];
                        uniforms_z(pio.rng, a, (uint32_t)k, U);
                        float z[2];
                        box_muller_hw53(U[0], U[1], z[0], z[1]);
                        const int32_t i = pf_i[t], j = pf_j[t];
                        const VT isv = (VT)d.inv_sigma_v;
                        xin[t][0][0] = C * (float)((pio.v.x[i] - pio.v.x[j]) * isv);
                        xin[t][0][1] = C * (float)((pio.v.y[i] - pio.v.y[j]) * isv);
                        xin[t][0][2] = C * (float)((pio.v.z[i] - pio.v.z[j]) * isv);
                        xin[t][0][3] = C * (float)z[0];
                        xin[t][0][4] = C * (float)z[1];
                    }
                }
            } else {
                const int din = d.dims[0];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int c = 16 * q + 8 * h + e;
                        if (c < din) {
                            if (valid[t]) {
                                const float xv = rio.x[row[t] * din + c];
                                xin[t][q][e] = C * xv;
                                if (SAVE)
                                    rio.xsave[gemm_off(c, row[t], 0, (int64_t)din * GEMM_RB)] =
                                        (__bf16)xv;
                            }
                        } else if (c < din + 2) {
                            xin[t][q][e] = 1.0f;
                        }
                    }
            }
        }

        if (PAIRS) prefetch(grp + gstride);

        // input layer: s = W (c x) + c b, each input as a bf16 pair
        bf16x8 bin[NT][2], blo[NT][2];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 hb = (__bf16)xin[t][q][e];
                    bin[t][q][e] = hb;
                    blo[t][q][e] = (__bf16)(xin[t][q][e] - (float)hb);
                }
        floatx16 acc[NT][NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const bf16x8 a = lds_frag(wl, f.off[0], nb * f.ks[0], lane);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                acc[t][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bin[t][0], zero, 0, 0, 0);
                acc[t][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, blo[t][0], acc[t][nb], 0, 0, 0);
            }
        }
        if (f.ks[0] > 1) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const bf16x8 a = lds_frag(wl, f.off[0], nb * f.ks[0] + 1, lane);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    acc[t][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bin[t][1], acc[t][nb], 0, 0, 0);
                    acc[t][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, blo[t][1], acc[t][nb], 0, 0, 0);
                }
            }
        }
        // hidden layers, two at a time so the accumulators alternate
        // between two register sets without copies.  With SPLIT == FRONT
        // only layers 1 and 2 take pair inputs: they form the first pass
        // of the loop, and the tail (layers l and l + 1) is paired when
        // l < 3.
        constexpr bool LATE = SPLIT == DSMC_SPLIT_ALL;
        constexpr bool SECOND = SPLIT != DSMC_SPLIT_FIRST;   // h2 as a pair
        const int ks = H / 16 + 1;
        // saved activations of hidden layer ll (rows mode, NT == 1)
        auto hptr = [&](int ll) -> __bf16* {
            if (!SAVE || !valid[0]) return nullptr;
            const size_t Bp = (size_t)row_blocks(rio.B) * GEMM_RB;
            return rio.hsave + (size_t)(ll - 1) * H * Bp +
                   (size_t)(row[0] / GEMM_RB) * H * GEMM_RB + (size_t)(row[0] % GEMM_RB);
        };
        floatx16 alt[NT][NB];
        floatx16 ao[NT][1];
        int l = 1;
        if (l + 1 < L - 1) {
            save_pre<H, NT, SAVE, ACT>(rio, l, row, valid, acc, h);
            layer_step<NB, NB, NT, ACT, true, SAVE>(wl, f.off[l], ks, acc, alt, bone, lane, hptr(l));
            save_pre<H, NT, SAVE, ACT>(rio, l + 1, row, valid, alt, h);
            layer_step<NB, NB, NT, ACT, SECOND, SAVE && SECOND>(wl, f.off[l + 1], ks, alt, acc, bone, lane, hptr(l + 1));
            l += 2;
        }
        for (; l + 1 < L - 1; l += 2) {
            save_pre<H, NT, SAVE, ACT>(rio, l, row, valid, acc, h);
            layer_step<NB, NB, NT, ACT, LATE, SAVE && LATE>(wl, f.off[l], ks, acc, alt, bone, lane, hptr(l));
            save_pre<H, NT, SAVE, ACT>(rio, l + 1, row, valid, alt, h);
            layer_step<NB, NB, NT, ACT, LATE, SAVE && LATE>(wl, f.off[l + 1], ks, alt, acc, bone, lane, hptr(l + 1));
        }
        if (LATE || l < 3) {
            if (l < L - 1) {
                save_pre<H, NT, SAVE, ACT>(rio, l, row, valid, acc, h);
                layer_step<NB, NB, NT, ACT, true, SAVE>(wl, f.off[l], ks, acc, alt, bone, lane, hptr(l));
                save_pre<H, NT, SAVE, ACT>(rio, l + 1, row, valid, alt, h);
                layer_step<NB, 1, NT, ACT, SECOND, SAVE && SECOND>(wl, f.off[L - 1], ks, alt, ao, bone, lane, hptr(l + 1));
            } else {
                save_pre<H, NT, SAVE, ACT>(rio, l, row, valid, acc, h);
                layer_step<NB, 1, NT, ACT, true, SAVE>(wl, f.off[L - 1], ks, acc, ao, bone, lane, hptr(l));
            }
        } else {
            if (l < L - 1) {
                layer_step<NB, NB, NT, ACT, false>(wl, f.off[l], ks, acc, alt, bone, lane);
                layer_step<NB, 1, NT, ACT, false>(wl, f.off[L - 1], ks, alt, ao, bone, lane);
            } else {
                layer_step<NB, 1, NT, ACT, false>(wl, f.off[L - 1], ks, acc, ao, bone, lane);
            }
        }
        // output layer result: y = s / c, <= 32 outputs in one block
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (!valid[t]) continue;
            const int64_t r0 = row[t];
            if (!PAIRS) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int n = acc_row(r, h);
                    if (n < dout) rio.y_raw[r0 * dout + n] = ao[t][0][r] * IC;
                }
            }
            if (h != 0) continue;
            // outputs 0..2 sit in registers 0..2 of lane-half 0
            const float y0 = ao[t][0][0] * IC, y1 = ao[t][0][1] * IC, y2 = ao[t][0][2] * IC;
            const float nrm = sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
            if (PAIRS) {
                VT u[3];
                if (nrm > 1e-30f) {
                    const float inv = 1.0f / nrm;
                    u[0] = (VT)(y0 * inv); u[1] = (VT)(y1 * inv); u[2] = (VT)(y2 * inv);
                } else {
                    // degenerate output: the isotropic direction of this pair
                    const int32_t k = pio.pr.cell[r0];
                    const uint32_t a = (uint32_t)(r0 - pio.pr.off[k]);
                    VT xi[3], z[2], u4, vh[3], e[3];
                    pair_latents(pio.rng, a, (uint32_t)k, xi, z, u4);
                    const int32_t i = pio.pr.i[r0], j = pio.pr.j[r0];
                    unit3<VT>(pio.v.x[i] - pio.v.x[j], pio.v.y[i] - pio.v.y[j],
                              pio.v.z[i] - pio.v.z[j], vh);
                    const VT cc = VT(2) * u4 - VT(1);
                    const VT sc = VT(2) * dev_sqrt<VT>(u4 * (VT(1) - u4));
                    perp_dir<VT>(xi, vh, e);
                    for (int q = 0; q < 3; ++q) u[q] = cc * vh[q] + sc * e[q];
                }
                pio.out.a[r0] = u[0];
                pio.out.b[r0] = u[1];
                pio.out.c[r0] = u[2];
            } else if (rio.vr_out && dout == 3) {
                const float gg = rio.g[r0];
                const float sg = nrm > 1e-30f ? gg / nrm : 0.0f;
                rio.vr_out[3 * r0 + 0] = y0 * sg;
                rio.vr_out[3 * r0 + 1] = y1 * sg;
                rio.vr_out[3 * r0 + 2] = y2 * sg;
            }
        }
    }
}

// Launch shape of the fused kernel: one 32-row tile per wave; 512-thread
// workgroups (two waves per SIMD share the LDS copy of the weights) for
// hidden width 64 and 128, 256 threads (one wave per SIMD with the whole
// register file) for width 256.  A persistent grid of one workgroup per CU.
template <int H, bool PAIRS, typename VT, int ACT, bool SAVE, int SPLIT>
static int launch_one(const MlpDev& d, const FragLayout& f, RowsIO rio, PairsIO<VT> pio,
                      int64_t max_rows, hipStream_t s)
{
    constexpr int NT = 1, TPB = H == 256 ? 256 : 512;
    auto kern = k_mlp_bf16<H, PAIRS, VT, ACT, SAVE, NT, TPB, SPLIT>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return hip_check(e, "mlp: set LDS attribute");
        attr_set = true;
    }
    const int cus = device_cus();
    const int64_t groups = (max_rows + 32 * NT - 1) / (32 * NT);
    int64_t blocks = (groups + TPB / 64 - 1) / (TPB / 64);
    if (blocks > cus) blocks = cus;
    if (blocks < 1) blocks = 1;
    kern<<<(int)blocks, TPB, f.bytes, s>>>(d, f, rio, pio);
    DSMC_LAUNCH_CHECK("mlp_bf16");
    return DSMC_OK;
}

// The row entry points (PAIRS false) save pre-activations on request and
// always carry every activation as a pair; the in-step entry point never
// saves and follows the network's split setting.
template <int H, bool PAIRS, typename VT, int ACT>
static int launch_act(const MlpDev& d, const FragLayout& f, RowsIO rio, PairsIO<VT> pio,
                      int64_t max_rows, hipStream_t s)
{
    if constexpr (PAIRS) {
        if (d.split == DSMC_SPLIT_FRONT)
            return launch_one<H, PAIRS, VT, ACT, false, DSMC_SPLIT_FRONT>(d, f, rio, pio, max_rows, s);
        if (d.split == DSMC_SPLIT_FIRST)
            return launch_one<H, PAIRS, VT, ACT, false, DSMC_SPLIT_FIRST>(d, f, rio, pio, max_rows, s);
        return launch_one<H, PAIRS, VT, ACT, false, DSMC_SPLIT_ALL>(d, f, rio, pio, max_rows, s);
    } else {
        if (rio.zsave != nullptr)
            return launch_one<H, PAIRS, VT, ACT, true, DSMC_SPLIT_ALL>(d, f, rio, pio, max_rows, s);
        return launch_one<H, PAIRS, VT, ACT, false, DSMC_SPLIT_ALL>(d, f, rio, pio, max_rows, s);
    }
}

template <int H, bool PAIRS, typename VT>
static int launch_mlp_bf16(const MlpDev& d, const FragLayout& f, RowsIO rio, PairsIO<VT> pio,
                           int64_t max_rows, hipStream_t s)
{
    if (d.act == DSMC_ACT_SILU)
        return launch_act<H, PAIRS, VT, DSMC_ACT_SILU>(d, f, rio, pio, max_rows, s);
    return launch_act<H, PAIRS, VT, DSMC_ACT_RELU>(d, f, rio, pio, max_rows, s);
}

// ------------------------------------------------------------------------
// Reference path (FP64 / FP32): per-element layer kernels
// ------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_x_from_pairs(int32_t n_cells, PairsView pr, dsmc_rng rng, V3<const T> v, T inv_sv, T* X)
{
    const int64_t np = pr.total(n_cells);
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = pr.cell[p];
        const uint32_t a = (uint32_t)(p - pr.off[k]);
        T xi[3], z[2], u4;
        pair_latents(rng, a, (uint32_t)k, xi, z, u4);
        const int32_t i = pr.i[p], j = pr.j[p];
        T* x = X + 8 * p;
        x[0] = (v.x[i] - v.x[j]) * inv_sv;
        x[1] = (v.y[i] - v.y[j]) * inv_sv;
        x[2] = (v.z[i] - v.z[j]) * inv_sv;
        x[3] = xi[0]; x[4] = xi[1]; x[5] = xi[2];
        x[6] = z[0]; x[7] = z[1];
    }
}

// z = h W^T + b (one thread per output element); h_out = act(z) if hidden.
template <typename T, typename WT>
__global__ void __launch_bounds__(256)
k_layer(const T* __restrict__ hin, int64_t B, const int64_t* nrows_dev, int in, int out,
        const WT* __restrict__ W, const WT* __restrict__ bias, int act, int hidden,
        T* __restrict__ z, T* __restrict__ hout)
{
    const int64_t nrows = nrows_dev ? *nrows_dev : B;
    const int64_t n_el = nrows * out;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n_el;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / out;
        const int n = (int)(q % out);
        T acc = (T)bias[n];
        const T* hr = hin + r * in;
        const WT* wr = W + (size_t)n * in;
        for (int k = 0; k < in; ++k) acc += (T)wr[k] * hr[k];
        if (z) z[q] = acc;
        if (hidden) hout[q] = act_t<T>(acc, act);
        else hout[q] = acc;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_project_pairs(int32_t n_cells, PairsView pr, dsmc_rng rng, V3<const T> v, const T* Y, int dout,
                PairBuf<T> out)
{
    const int64_t np = pr.total(n_cells);
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        const T y0 = Y[p * dout], y1 = Y[p * dout + 1], y2 = Y[p * dout + 2];
        const T n = dev_sqrt<T>(y0 * y0 + y1 * y1 + y2 * y2);
        T u[3];
        if (n > T(1e-30)) {
            u[0] = y0 / n; u[1] = y1 / n; u[2] = y2 / n;
        } else {
            const int32_t k = pr.cell[p];
            const uint32_t a = (uint32_t)(p - pr.off[k]);
            T xi[3], z[2], u4, vh[3], e[3];
            pair_latents(rng, a, (uint32_t)k, xi, z, u4);
            const int32_t i = pr.i[p], j = pr.j[p];
            unit3<T>(v.x[i] - v.x[j], v.y[i] - v.y[j], v.z[i] - v.z[j], vh);
            const T cc = T(2) * u4 - T(1);
            const T sc = T(2) * dev_sqrt<T>(u4 * (T(1) - u4));
            perp_dir<T>(xi, vh, e);
            for (int q = 0; q < 3; ++q) u[q] = cc * vh[q] + sc * e[q];
        }
        out.a[p] = u[0]; out.b[p] = u[1]; out.c[p] = u[2];
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_project_rows(int64_t B, const T* __restrict__ Y, int dout, const T* __restrict__ g,
               T* __restrict__ vr)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < B;
         r += (int64_t)gridDim.x * blockDim.x) {
        const T y0 = Y[r * dout], y1 = Y[r * dout + 1], y2 = Y[r * dout + 2];
        const T n = dev_sqrt<T>(y0 * y0 + y1 * y1 + y2 * y2);
        const T s = n > T(1e-30) ? g[r] / n : T(0);
        vr[3 * r] = y0 * s; vr[3 * r + 1] = y1 * s; vr[3 * r + 2] = y2 * s;
    }
}

__global__ void k_pairs_total(int32_t n_cells, PairsView pr, int64_t* out)
{
    *out = pr.total(n_cells);
}

// Workspace of the reference path: X and two activation buffers.
static size_t ref_ws_bytes(const MlpDev& d, int64_t rows, size_t es)
{
    int wmax = 8;
    for (int l = 0; l <= d.L; ++l) wmax = wmax > d.dims[l] ? wmax : d.dims[l];
    return 256 + 3 * align_up(es * (size_t)(rows + 1) * wmax);
}

template <typename T>
static int ref_forward(const MlpDev& d, const T* X, int64_t B, const int64_t* nrows_dev, T* buf0,
                       T* buf1, T* zsave, T* Yout, hipStream_t s)
{
    const T* hin = X;
    T* bufs[2] = {buf0, buf1};
    int64_t zoff = 0;
    for (int l = 0; l < d.L; ++l) {
        const bool hidden = l < d.L - 1;
        T* hout = hidden ? bufs[l & 1] : Yout;
        T* z = (hidden && zsave) ? zsave + zoff : nullptr;
        const int64_t n_el = B * d.dims[l + 1];
        int blocks = (int)((n_el + 255) / 256);
        const int pb = persistent_blocks(256);
        if (blocks > pb) blocks = pb;
        if (blocks < 1) blocks = 1;
        k_layer<T, T><<<blocks, 256, 0, s>>>(hin, B, nrows_dev, d.dims[l], d.dims[l + 1],
                                             static_cast<const T*>(d.W[l]),
                                             static_cast<const T*>(d.b[l]), d.act, hidden, z, hout);
        DSMC_LAUNCH_CHECK("mlp_ref:layer");
        if (hidden) zoff += B * d.dims[l + 1];
        hin = hout;
    }
    return DSMC_OK;
}

// ------------------------------------------------------------------------
// Backward (reference arithmetic in T; for the BF16 network T = float and
// the activations are rounded to bf16 exactly as the forward used them)
// ------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_project_backward(int64_t B, const T* __restrict__ Y, int dout, const T* __restrict__ g,
                   const T* __restrict__ G, T* __restrict__ dY)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < B;
         r += (int64_t)gridDim.x * blockDim.x) {
        const T y0 = Y[r * dout], y1 = Y[r * dout + 1], y2 = Y[r * dout + 2];
        const T n = dev_sqrt<T>(y0 * y0 + y1 * y1 + y2 * y2);
        T* o = dY + r * dout;
        for (int q = 0; q < dout; ++q) o[q] = T(0);
        if (!(n > T(1e-30))) continue;
        const T u0 = y0 / n, u1 = y1 / n, u2 = y2 / n;
        const T G0 = G[3 * r], G1 = G[3 * r + 1], G2 = G[3 * r + 2];
        const T Gu = G0 * u0 + G1 * u1 + G2 * u2;
        const T f = g[r] / n;
        o[0] = f * (G0 - Gu * u0);
        o[1] = f * (G1 - Gu * u1);
        o[2] = f * (G2 - Gu * u2);
    }
}

// h_{l-1} for layer l's weight gradient: x for l == 0, act(z) otherwise
// (rounded to bf16 when the network is bf16, as the forward used it).
template <typename T>
__global__ void __launch_bounds__(256)
k_hprev(int64_t n_el, const T* __restrict__ X, const T* __restrict__ Zp, int l, int act, int bf16,
        T* __restrict__ H)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n_el;
         q += (int64_t)gridDim.x * blockDim.x) {
        const T a = (l == 0) ? X[q] : act_t<T>(Zp[q], act);
        H[q] = bf16 ? (T)(float)(__bf16)(float)a : a;
    }
}

// Partial sums over row chunks: part[c][n][k] = sum_{r in chunk c} dY[r][n] H[r][k],
// partb[c][n] = sum dY[r][n].  One thread per (n, k) of one chunk; threads of
// a block share n and read consecutive k (coalesced H, broadcast dY).
template <typename T>
__global__ void __launch_bounds__(256)
k_dw_partial(int64_t B, int64_t chunk, const T* __restrict__ dY, int out, const T* __restrict__ H,
             int in, T* __restrict__ part, T* __restrict__ partb)
{
    const int64_t c = blockIdx.y;
    const int64_t r0 = c * chunk, r1 = (r0 + chunk < B) ? r0 + chunk : B;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < out * (in + 1);
         q += gridDim.x * blockDim.x) {
        const int n = q / (in + 1), k = q % (in + 1);
        T acc = T(0);
        if (k < in) {
            for (int64_t r = r0; r < r1; ++r) acc += dY[r * out + n] * H[r * in + k];
            part[(c * out + n) * (size_t)in + k] = acc;
        } else {
            for (int64_t r = r0; r < r1; ++r) acc += dY[r * out + n];
            partb[c * out + n] = acc;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_dw_reduce(int64_t n_chunks, const T* __restrict__ part, const T* __restrict__ partb, int out,
            int in, T* __restrict__ dW, T* __restrict__ db, int accumulate)
{
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < out * (in + 1);
         q += gridDim.x * blockDim.x) {
        const int n = q / (in + 1), k = q % (in + 1);
        T acc = T(0);
        if (k < in) {
            for (int64_t c = 0; c < n_chunks; ++c) acc += part[(c * out + n) * (size_t)in + k];
            const size_t o = (size_t)n * in + k;
            dW[o] = accumulate ? dW[o] + acc : acc;
        } else {
            for (int64_t c = 0; c < n_chunks; ++c) acc += partb[c * out + n];
            db[n] = accumulate ? db[n] + acc : acc;
        }
    }
}

// dH[r][k] = sum_n dY[r][n] W[n][k] (times act'(z) for hidden layers).
template <typename T, typename WT>
__global__ void __launch_bounds__(256)
k_delta_prev(int64_t B, const T* __restrict__ dY, int out, const WT* __restrict__ W, int in,
             const T* __restrict__ Zp, int act, int apply_act, T* __restrict__ dH)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < B * in;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / in;
        const int k = (int)(q % in);
        T acc = T(0);
        for (int n = 0; n < out; ++n) acc += dY[r * out + n] * (T)W[(size_t)n * in + k];
        if (apply_act) acc *= act_grad_t<T>(Zp[q], act);
        dH[q] = acc;
    }
}

template <typename T, typename WT>
static int backward_impl(const MlpDev& d, int64_t B, const T* X, const T* Z, const T* Y,
                         const T* g, const T* G, T* const* dW, T* const* db, T* dx, int accumulate,
                         bool bf16, void* ws, hipStream_t s)
{
    int wmax = 8;
    for (int l = 0; l <= d.L; ++l) wmax = wmax > d.dims[l] ? wmax : d.dims[l];
    const int64_t chunk = 2048;
    const int64_t n_chunks = (B + chunk - 1) / chunk;
    uint8_t* w = static_cast<uint8_t*>(ws);
    T* dA = reinterpret_cast<T*>(w);
    w += align_up(sizeof(T) * (size_t)B * wmax);
    T* dB = reinterpret_cast<T*>(w);
    w += align_up(sizeof(T) * (size_t)B * wmax);
    T* part = reinterpret_cast<T*>(w);
    w += align_up(sizeof(T) * (size_t)n_chunks * wmax * wmax);
    T* partb = reinterpret_cast<T*>(w);
    w += align_up(sizeof(T) * (size_t)n_chunks * wmax);
    T* H = reinterpret_cast<T*>(w);
    const int pb = persistent_blocks(256);
    auto grid1 = [&](int64_t n) {
        int64_t b = (n + 255) / 256;
        return (int)(b < 1 ? 1 : (b > pb ? pb : b));
    };
    const int dout = d.dims[d.L];
    k_project_backward<T><<<grid1(B), 256, 0, s>>>(B, Y, dout, g, G, dA);
    DSMC_LAUNCH_CHECK("mlp_bwd:project");
    // z offsets of hidden layers
    int64_t zoff[MLP_MAX_LAYERS] = {0};
    for (int l = 1; l < d.L; ++l) zoff[l] = zoff[l - 1] + B * d.dims[l];
    T* cur = dA;
    T* nxt = dB;
    for (int l = d.L - 1; l >= 0; --l) {
        const int out = d.dims[l + 1], in = d.dims[l];
        const T* Zp = (l > 0) ? Z + zoff[l - 1] : nullptr;
        k_hprev<T><<<grid1(B * in), 256, 0, s>>>(B * in, X, Zp, l, d.act, bf16, H);
        DSMC_LAUNCH_CHECK("mlp_bwd:hprev");
        dim3 gp((unsigned)((out * (in + 1) + 255) / 256), (unsigned)n_chunks);
        k_dw_partial<T><<<gp, 256, 0, s>>>(B, chunk, cur, out, H, in, part, partb);
        DSMC_LAUNCH_CHECK("mlp_bwd:dw_partial");
        k_dw_reduce<T><<<grid1(out * (in + 1)), 256, 0, s>>>(n_chunks, part, partb, out, in, dW[l],
                                                             db[l], accumulate);
        DSMC_LAUNCH_CHECK("mlp_bwd:dw_reduce");
        if (l > 0 || dx) {
            T* target = (l > 0) ? nxt : dx;
            k_delta_prev<T, WT><<<grid1(B * in), 256, 0, s>>>(
                B, cur, out, static_cast<const WT*>(d.W[l]), in, Zp, d.act, l > 0, target);
            DSMC_LAUNCH_CHECK("mlp_bwd:delta");
            if (l > 0) {
                T* t = cur;
                cur = nxt;
                nxt = t;
            }
        }
    }
    return DSMC_OK;
}

// BF16 network: the weight and input gradients on the matrix cores.
// dW_l = delta_l^T h_{l-1} (K = B split over workgroups, fixed-order sum),
// delta_{l-1} = (delta_l W_l) * act'(z_{l-1}) with the derivative fused in the
// GEMM epilogue; db_l by a fixed-order column sum.  delta is kept in FP32 (for
// db) and bf16 (the GEMM operand); h_{l-1} is the bf16 activation the forward
// used.
struct Bf16BwdWs {
    __bf16* dt[2];  // delta^T, row-blocked (ping-pong): k-contiguous A of the weight-gradient GEMM
    float* part;
    float* apart;   // per-split row sums of delta^T (bias gradient)
    size_t bytes;
};

constexpr int BWD_SPLITS_MAX = 256;

static Bf16BwdWs bf16_bwd_layout(void* base, const MlpDev& d, int64_t B)
{
    int wmax = 8;
    for (int l = 0; l <= d.L; ++l) wmax = wmax > d.dims[l] ? wmax : d.dims[l];
    Bf16BwdWs w{};
    uint8_t* p = static_cast<uint8_t*>(base);
    size_t o = 0;
    auto take = [&](size_t b) { uint8_t* r = p ? p + o : nullptr; o += align_up(b); return r; };
    const size_t Bp = (size_t)(row_blocks(B) * GEMM_RB);
    for (int q = 0; q < 2; ++q)
        w.dt[q] = reinterpret_cast<__bf16*>(take(sizeof(__bf16) * Bp * wmax));
    w.part = reinterpret_cast<float*>(take(sizeof(float) * BWD_SPLITS_MAX * (size_t)wmax * wmax));
    w.apart = reinterpret_cast<float*>(take(sizeof(float) * BWD_SPLITS_MAX * (size_t)wmax));
    w.bytes = o;
    return w;
}

// Projection backward of the bf16 rows form, written as delta^T of the output
// layer in bf16 (row-blocked, three units): the same arithmetic as
// k_project_backward.
__global__ void __launch_bounds__(256)
k_project_backward_t16(int64_t B, const float* __restrict__ Y, const float* __restrict__ g,
                       const float* __restrict__ G, __bf16* __restrict__ dt)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < B;
         r += (int64_t)gridDim.x * blockDim.x) {
        const float y0 = Y[r * 3], y1 = Y[r * 3 + 1], y2 = Y[r * 3 + 2];
        const float n = dev_sqrt<float>(y0 * y0 + y1 * y1 + y2 * y2);
        float o[3] = {0.f, 0.f, 0.f};
        if (n > 1e-30f) {
            const float u0 = y0 / n, u1 = y1 / n, u2 = y2 / n;
            const float G0 = G[3 * r], G1 = G[3 * r + 1], G2 = G[3 * r + 2];
            const float Gu = G0 * u0 + G1 * u1 + G2 * u2;
            const float f = g[r] / n;
            o[0] = f * (G0 - Gu * u0);
            o[1] = f * (G1 - Gu * u1);
            o[2] = f * (G2 - Gu * u2);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) dt[gemm_off(c, r, 0, 3 * GEMM_RB)] = (__bf16)o[c];
    }
}

// Backward of the bf16 rows form.  Everything runs on transposed ([unit][row])
// bf16 matrices, row-blocked as the forward saves them (blocks of GEMM_RB
// rows, so a tile's rows sit in one contiguous block), so that both factors
// of each weight gradient (K = batch) are k-contiguous and no transpose pass
// is needed:
//   dW_l = delta_l^T h_{l-1}     (h^T and x^T from the forward's act_save)
//   db_l = row sums of delta_l^T (summed by the same GEMM from its A tiles)
//   delta_{l-1}^T = (W_l^T delta_l^T) * act'(z_{l-1}^T)   (a GEMM with
//   M = units, N = batch, whose epilogue reads z^T and writes delta^T)
static int backward_bf16(const MlpDev& d, int64_t B, const float* X, const float* Z,
                         const float* Y, const float* g, const float* G, float* const* dW,
                         float* const* db, float* dx, int accumulate, void* ws, hipStream_t s)
{
    const Bf16BwdWs w = bf16_bwd_layout(ws, d, B);
    const int pb = persistent_blocks(256);
    auto grid1 = [&](int64_t n) {
        int64_t b = (n + 255) / 256;
        return (int)(b < 1 ? 1 : (b > pb ? pb : b));
    };
    int splits = (int)(B / 256);
    splits = splits < 1 ? 1 : (splits > BWD_SPLITS_MAX ? BWD_SPLITS_MAX : splits);
    const int64_t Bp = row_blocks(B) * GEMM_RB;
    int64_t zoff[MLP_MAX_LAYERS] = {0};
    for (int l = 1; l < d.L; ++l) zoff[l] = zoff[l - 1] + Bp * d.dims[l];
    const uint8_t* zb = reinterpret_cast<const uint8_t*>(Z);
    const size_t hoff = align_up(sizeof(float) * (size_t)zoff[d.L - 1]);
    const __bf16* Hs = reinterpret_cast<const __bf16*>(zb + hoff);
    const __bf16* Xs = reinterpret_cast<const __bf16*>(
        zb + hoff + align_up(sizeof(__bf16) * (size_t)zoff[d.L - 1]));
    int cur = 0;
    k_project_backward_t16<<<grid1(B), 256, 0, s>>>(B, Y, g, G, w.dt[cur]);
    DSMC_LAUNCH_CHECK("mlp_bwd16:project");
    const int gact = d.act == DSMC_ACT_RELU ? GEMM_ACT_RELU : GEMM_ACT_SILU;
    for (int l = d.L - 1; l >= 0; --l) {
        const int out = d.dims[l + 1], in = d.dims[l];
        const __bf16* hT = (l > 0) ? Hs + zoff[l - 1] : Xs;   // saved by the forward
        GemmArgs gw{};
        gw.a = w.dt[cur];
        gw.lda = GEMM_RB;
        gw.bsa = (int64_t)out * GEMM_RB;
        gw.ta = 0;
        gw.b = hT;
        gw.ldb = GEMM_RB;
        gw.bsb = (int64_t)in * GEMM_RB;
        gw.tb = 1;
        gw.M = out;
        gw.N = in;
        gw.K = B;
        gw.act = GEMM_ACT_NONE;
        gw.accumulate = accumulate;
        gw.out_f32 = dW[l];
        gw.ldo = in;
        gw.partial = w.part;
        gw.asum_out = db[l];       // db_l = row sums of delta_l^T, the A operand
        gw.asum_part = w.apart;
        int rc = gemm_bf16(gw, splits, s);
        if (rc) return rc;
        if (l > 0) {
            GemmArgs gd{};
            gd.a = static_cast<const __bf16*>(d.W[l]);   // A(m = unit of l-1, k) = W[k][m]
            gd.lda = in;
            gd.ta = 1;
            gd.b = w.dt[cur];                             // B(k, n = row) = delta^T[k][n]
            gd.ldb = GEMM_RB;
            gd.bsb = (int64_t)out * GEMM_RB;
            gd.tb = 0;
            gd.M = in;
            gd.N = B;
            gd.K = out;
            gd.dact_z = Z + zoff[l - 1];                  // z^T, row-blocked
            gd.ldz = GEMM_RB;
            gd.bsz = (int64_t)in * GEMM_RB;
            gd.act = gact;
            gd.out_bf16 = w.dt[1 - cur];
            gd.ldo = GEMM_RB;
            gd.bso = (int64_t)in * GEMM_RB;
            rc = gemm_bf16(gd, 1, s);
            if (rc) return rc;
            cur = 1 - cur;
        } else if (dx) {
            GemmArgs gd{};
            gd.a = w.dt[cur];                             // A(m = row, k) = delta^T[k][m]
            gd.lda = GEMM_RB;
            gd.bsa = (int64_t)out * GEMM_RB;
            gd.ta = 1;
            gd.b = static_cast<const __bf16*>(d.W[0]);   // B(k, n) = W[k][n]
            gd.ldb = in;
            gd.tb = 0;
            gd.M = B;
            gd.N = in;
            gd.K = out;
            gd.act = GEMM_ACT_NONE;
            gd.out_f32 = dx;
            gd.ldo = in;
            rc = gemm_bf16(gd, 1, s);
            if (rc) return rc;
        }
    }
    return DSMC_OK;
}

static size_t backward_ws_bytes(const MlpDev& d, int64_t B, size_t es)
{
    const size_t b16 = bf16_bwd_layout(nullptr, d, B).bytes + 256;
    int wmax = 8;
    for (int l = 0; l <= d.L; ++l) wmax = wmax > d.dims[l] ? wmax : d.dims[l];
    const int64_t n_chunks = (B + 2047) / 2048;
    const size_t gen = 256 + 3 * align_up(es * (size_t)B * wmax) +
                       align_up(es * (size_t)n_chunks * wmax * wmax) +
                       align_up(es * (size_t)n_chunks * wmax);
    return gen > b16 ? gen : b16;
}

// ------------------------------------------------------------------------
// Training helpers
// ------------------------------------------------------------------------
// Loss kernels: a grid of workgroups, each summing its rows in a fixed order
// and adding its share to *loss with one FP64 atomic (the order of those few
// hundred additions varies between runs; the gradient does not).
__device__ __forceinline__ void block_add_loss(double acc, double scale, double* loss)
{
    __shared__ double red[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w];
        if (sum != 0.0) atomicAdd(loss, sum * scale);
    }
}

__global__ void __launch_bounds__(256)
k_mse(int64_t B, const float* __restrict__ a, const float* __restrict__ t, double scale,
      float* __restrict__ grad, double* loss)
{
    double acc = 0.0;
    const int64_t n3 = 3 * B;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n3;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double dd = (double)a[q] - (double)t[q];
        acc += dd * dd;
        grad[q] = (float)(2.0 * scale * dd);
    }
    block_add_loss(acc, scale, loss);
}

// MSE on the scattering directions: each pair's term and gradient are
// normalised by its own g^2 = |v_r'*|^2.
__global__ void __launch_bounds__(256)
k_dir_loss(int64_t B, const float* __restrict__ a, const float* __restrict__ t,
           float* __restrict__ grad, double* loss)
{
    double acc = 0.0;
    const double invB = 1.0 / (double)B;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < B;
         r += (int64_t)gridDim.x * blockDim.x) {
        double d[3], g2 = 0.0, dd = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double tv = (double)t[3 * r + c];
            d[c] = (double)a[3 * r + c] - tv;
            g2 += tv * tv;
            dd += d[c] * d[c];
        }
        const double w = g2 > 0.0 ? 1.0 / g2 : 0.0;
        acc += 0.25 * dd * w;
#pragma unroll
        for (int c = 0; c < 3; ++c) grad[3 * r + c] = (float)(0.5 * d[c] * w * invB);
    }
    block_add_loss(acc, invB, loss);
}

__global__ void __launch_bounds__(256)
k_adam(int64_t n, float* __restrict__ p, __bf16* __restrict__ pb, const float* __restrict__ g,
       float* __restrict__ m, float* __restrict__ v, float b1, float b2, float lr_c, float eps_c,
       float bc2_sqrt)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float gg = g[q];
        const float mm = b1 * m[q] + (1.0f - b1) * gg;
        const float vv = b2 * v[q] + (1.0f - b2) * gg * gg;
        m[q] = mm;
        v[q] = vv;
        // bias-corrected step: lr m_hat / (sqrt(v_hat) + eps), folded as
        // (lr / (1-b1^t)) m / (sqrt(v) / sqrt(1-b2^t) + eps)
        const float np = p[q] - lr_c * mm / (sqrtf(vv) / bc2_sqrt + eps_c);
        p[q] = np;
        if (pb) pb[q] = (__bf16)np;
    }
}

}  // namespace dsmc

using namespace dsmc;

// ------------------------------------------------------------------------
// C-ABI
// ------------------------------------------------------------------------
static size_t neural_ws_extra(const MlpDev& d, int64_t cap, int dtype)
{
    return 256 + ref_ws_bytes(d, cap, dtype == DSMC_F64 ? 8 : 4);
}

extern "C" int dsmc_neural_collide(const dsmc_mlp* net, int32_t n_cells, int32_t dtype,
                                   dsmc_vec3 v, dsmc_pairs pairs, dsmc_rng rng, int32_t schedule,
                                   void* ws, size_t ws_bytes, dsmc_status* st,
                                   dsmc_stream_t stream)
{
    (void)st;
    MlpDev d;
    int rc = check_mlp(net, &d);
    if (rc) return rc;
    rc = check_pairs("dsmc_neural_collide", n_cells, v, pairs, dtype, ws, ws_bytes);
    if (rc) return rc;
    if (d.dims[0] != 8 || d.dims[d.L] != 3)
        return arg_error("dsmc_neural_collide: network must map 8 inputs to 3 outputs");
    if (schedule < DSMC_SCHED_AUTO || schedule > DSMC_SCHED_WAVE)
        return arg_error("dsmc_neural_collide: schedule %d", schedule);
    hipStream_t s = as_stream(stream);
    const PairsView pr = PairsView::of(pairs);
    const size_t dir_bytes = dsmc_collide_ws(pairs.cap, dtype);
    if (net->wdtype == DSMC_BF16) {
        int H;
        if (!mfma_shape_ok(d, &H))
            return DSMC_E_UNSUPPORTED + 0 * arg_error("dsmc_neural_collide: bf16 shape unsupported");
        const FragLayout f = frag_layout(d);
        if (f.bytes > MLP_LDS_BYTES)
            return DSMC_E_UNSUPPORTED + 0 * arg_error("dsmc_neural_collide: the bf16 weights need "
                                                      "%zu bytes of LDS, more than %zu",
                                                      f.bytes, MLP_LDS_BYTES);
        RowsIO rio{};
        if (dtype == DSMC_F64) {
            PairsIO<double> pio{pr, n_cells, v3<const double>(v), rng, PairBuf<double>::of(ws, pairs.cap)};
            if (H == 128) rc = launch_mlp_bf16<128, true, double>(d, f, rio, pio, pairs.cap, s);
            else if (H == 64) rc = launch_mlp_bf16<64, true, double>(d, f, rio, pio, pairs.cap, s);
            else rc = launch_mlp_bf16<256, true, double>(d, f, rio, pio, pairs.cap, s);
        } else {
            PairsIO<float> pio{pr, n_cells, v3<const float>(v), rng, PairBuf<float>::of(ws, pairs.cap)};
            if (H == 128) rc = launch_mlp_bf16<128, true, float>(d, f, rio, pio, pairs.cap, s);
            else if (H == 64) rc = launch_mlp_bf16<64, true, float>(d, f, rio, pio, pairs.cap, s);
            else rc = launch_mlp_bf16<256, true, float>(d, f, rio, pio, pairs.cap, s);
        }
        if (rc) return rc;
    } else {
        // reference path in the velocity dtype (weights must match it)
        if ((dtype == DSMC_F64) != (net->wdtype == DSMC_F64))
            return arg_error("dsmc_neural_collide: reference path needs wdtype == dtype");
        if (ws_bytes < dir_bytes + neural_ws_extra(d, pairs.cap, dtype))
            return arg_error("dsmc_neural_collide: workspace too small for the reference path "
                             "(need dsmc_collide_ws + dsmc_neural_act_bytes(net, cap))");
        uint8_t* w = static_cast<uint8_t*>(ws) + dir_bytes;
        int wmax = 8;
        for (int l = 0; l <= d.L; ++l) wmax = wmax > d.dims[l] ? wmax : d.dims[l];
        const size_t es = dtype == DSMC_F64 ? 8 : 4;
        int64_t* nrows = reinterpret_cast<int64_t*>(w);
        w += 256;
        void* X = w;
        w += align_up(es * (size_t)(pairs.cap + 1) * wmax);
        void* b0 = w;
        w += align_up(es * (size_t)(pairs.cap + 1) * wmax);
        void* b1 = w;
        const int pb = persistent_blocks(256);
        k_pairs_total<<<1, 1, 0, s>>>(n_cells, pr, nrows);
        DSMC_LAUNCH_CHECK("neural:total");
        if (dtype == DSMC_F64) {
            k_x_from_pairs<double><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const double>(v),
                                                      d.inv_sigma_v, (double*)X);
            DSMC_LAUNCH_CHECK("neural:x");
            rc = ref_forward<double>(d, (double*)X, pairs.cap, nrows, (double*)b0, (double*)b1,
                                     nullptr, (double*)X, s);
            if (rc) return rc;
            k_project_pairs<double><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const double>(v),
                                                       (double*)X, 3,
                                                       PairBuf<double>::of(ws, pairs.cap));
        } else {
            k_x_from_pairs<float><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const float>(v),
                                                     (float)d.inv_sigma_v, (float*)X);
            DSMC_LAUNCH_CHECK("neural:x");
            rc = ref_forward<float>(d, (float*)X, pairs.cap, nrows, (float*)b0, (float*)b1, nullptr,
                                    (float*)X, s);
            if (rc) return rc;
            k_project_pairs<float><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const float>(v),
                                                      (float*)X, 3, PairBuf<float>::of(ws, pairs.cap));
        }
        DSMC_LAUNCH_CHECK("neural:project");
    }
    if (schedule == DSMC_SCHED_DEFER) return DSMC_OK;
    return phase_b(RULE_DIR, dtype, n_cells, nullptr, v, pairs, ws, pairs.cap, schedule, s);
}

extern "C" size_t dsmc_neural_act_bytes(const dsmc_mlp* net, int64_t B)
{
    MlpDev d;
    if (check_mlp(net, &d) != DSMC_OK || B < 0) return 0;
    // bf16: row-blocked, rows padded to whole blocks
    const int64_t Bz = net->wdtype == DSMC_BF16 ? row_blocks(B) * GEMM_RB : B;
    size_t n = 0;
    for (int l = 1; l < d.L; ++l) n += (size_t)Bz * d.dims[l];
    const size_t es = net->wdtype == DSMC_F64 ? 8 : 4;
    // hidden pre-activations, plus (bf16) their bf16 activations, plus
    // (reference path) X copy and two buffers
    const size_t h16 = net->wdtype == DSMC_BF16
                           ? align_up(sizeof(__bf16) * n) +
                                 align_up(sizeof(__bf16) * (size_t)Bz * d.dims[0])
                           : 0;
    return 256 + align_up(es * n) + h16 + ref_ws_bytes(d, B, es);
}

extern "C" int dsmc_neural_forward_rows(const dsmc_mlp* net, int64_t B, const void* x,
                                        const void* g, void* y_raw, void* vr_out, void* act_save,
                                        size_t act_bytes, dsmc_stream_t stream)
{
    MlpDev d;
    int rc = check_mlp(net, &d);
    if (rc) return rc;
    if (B < 0 || (B > 0 && (!x || !g || !y_raw)))
        return arg_error("dsmc_neural_forward_rows: bad arguments");
    if (B == 0) return DSMC_OK;
    hipStream_t s = as_stream(stream);
    size_t nz = 0;
    for (int l = 1; l < d.L; ++l) nz += (size_t)B * d.dims[l];
    if (net->wdtype == DSMC_BF16) {
        int H;
        if (!mfma_shape_ok(d, &H)) return DSMC_E_UNSUPPORTED + 0 * arg_error("bf16 shape unsupported");
        if (act_save && act_bytes < dsmc_neural_act_bytes(net, B))
            return arg_error("dsmc_neural_forward_rows: act_save too small");
        const FragLayout f = frag_layout(d);
        if (f.bytes > MLP_LDS_BYTES)
            return DSMC_E_UNSUPPORTED + 0 * arg_error("dsmc_neural_forward_rows: the bf16 weights "
                                                      "need %zu bytes of LDS, more than %zu",
                                                      f.bytes, MLP_LDS_BYTES);
        // act_save: pre-activations z^T (FP32), activations h^T (bf16), then
        // the inputs x^T (bf16), each layer row-blocked over row_blocks(B)
        // blocks
        const size_t nzp = nz / (size_t)B * (size_t)(row_blocks(B) * GEMM_RB);
        uint8_t* as = static_cast<uint8_t*>(act_save);
        const size_t hoff = align_up(sizeof(float) * nzp);
        const size_t xoff = hoff + align_up(sizeof(__bf16) * nzp);
        RowsIO rio{(const float*)x, (const float*)g, (float*)y_raw, (float*)vr_out,
                   act_save ? (float*)act_save : nullptr,
                   act_save ? reinterpret_cast<__bf16*>(as + hoff) : nullptr,
                   act_save ? reinterpret_cast<__bf16*>(as + xoff) : nullptr,
                   B};
        PairsIO<float> pio{};
        if (H == 128) rc = launch_mlp_bf16<128, false, float>(d, f, rio, pio, B, s);
        else if (H == 64) rc = launch_mlp_bf16<64, false, float>(d, f, rio, pio, B, s);
        else rc = launch_mlp_bf16<256, false, float>(d, f, rio, pio, B, s);
        return rc;
    }
    // reference path: needs act_save as scratch
    if (!act_save || act_bytes < dsmc_neural_act_bytes(net, B))
        return arg_error("dsmc_neural_forward_rows: reference path needs act_save of "
                         "dsmc_neural_act_bytes(net, B)");
    const size_t es = net->wdtype == DSMC_F64 ? 8 : 4;
    uint8_t* w = static_cast<uint8_t*>(act_save);
    void* Z = w;
    w += align_up(es * nz) + 256;
    int wmax = 8;
    for (int l = 0; l <= d.L; ++l) wmax = wmax > d.dims[l] ? wmax : d.dims[l];
    void* b0 = w + 256;
    void* b1 = (uint8_t*)b0 + align_up(es * (size_t)(B + 1) * wmax);
    const int pb = persistent_blocks(256);
    int blocks = (int)((B + 255) / 256);
    blocks = blocks > pb ? pb : blocks;
    if (net->wdtype == DSMC_F64) {
        rc = ref_forward<double>(d, (const double*)x, B, nullptr, (double*)b0, (double*)b1,
                                 (double*)Z, (double*)y_raw, s);
        if (rc) return rc;
        if (vr_out && d.dims[d.L] == 3) {
            k_project_rows<double><<<blocks, 256, 0, s>>>(B, (const double*)y_raw, 3,
                                                          (const double*)g, (double*)vr_out);
            DSMC_LAUNCH_CHECK("forward_rows:project");
        }
    } else {
        rc = ref_forward<float>(d, (const float*)x, B, nullptr, (float*)b0, (float*)b1, (float*)Z,
                                (float*)y_raw, s);
        if (rc) return rc;
        if (vr_out && d.dims[d.L] == 3) {
            k_project_rows<float><<<blocks, 256, 0, s>>>(B, (const float*)y_raw, 3,
                                                         (const float*)g, (float*)vr_out);
            DSMC_LAUNCH_CHECK("forward_rows:project");
        }
    }
    return DSMC_OK;
}

extern "C" size_t dsmc_neural_backward_ws(const dsmc_mlp* net, int64_t B)
{
    MlpDev d;
    if (check_mlp(net, &d) != DSMC_OK || B < 0) return 0;
    return backward_ws_bytes(d, B, net->wdtype == DSMC_F64 ? 8 : 4);
}

extern "C" int dsmc_neural_backward(const dsmc_mlp* net, int64_t B, const void* x,
                                    const void* act_save, const void* y_raw, const void* g,
                                    const void* dL_dvr, void* const* dW, void* const* db, void* dx,
                                    int32_t accumulate, void* ws, size_t ws_bytes,
                                    dsmc_stream_t stream)
{
    MlpDev d;
    int rc = check_mlp(net, &d);
    if (rc) return rc;
    if (B < 1 || !x || !act_save || !y_raw || !g || !dL_dvr || !dW || !db || !ws)
        return arg_error("dsmc_neural_backward: bad arguments");
    if (d.dims[d.L] != 3) return arg_error("dsmc_neural_backward: network must have 3 outputs");
    for (int l = 0; l < d.L; ++l)
        if (!dW[l] || !db[l]) return arg_error("dsmc_neural_backward: null dW/db %d", l);
    if (ws_bytes < dsmc_neural_backward_ws(net, B))
        return arg_error("dsmc_neural_backward: workspace too small");
    hipStream_t s = as_stream(stream);
    if (net->wdtype == DSMC_F64) {
        return backward_impl<double, double>(d, B, (const double*)x, (const double*)act_save,
                                             (const double*)y_raw, (const double*)g,
                                             (const double*)dL_dvr, (double* const*)dW,
                                             (double* const*)db, (double*)dx, accumulate, false, ws,
                                             s);
    }
    if (net->wdtype == DSMC_BF16) {
        return backward_bf16(d, B, (const float*)x, (const float*)act_save, (const float*)y_raw,
                             (const float*)g, (const float*)dL_dvr, (float* const*)dW,
                             (float* const*)db, (float*)dx, accumulate, ws, s);
    }
    return backward_impl<float, float>(d, B, (const float*)x, (const float*)act_save,
                                       (const float*)y_raw, (const float*)g, (const float*)dL_dvr,
                                       (float* const*)dW, (float* const*)db, (float*)dx, accumulate,
                                       false, ws, s);
}

constexpr int LOSS_BLOCKS = 128;

extern "C" int dsmc_mse_loss(int64_t B, const float* vr_new, const float* vr_target,
                             double sigma_v, float* dL_dvr, double* loss, dsmc_stream_t stream)
{
    if (B < 1 || !vr_new || !vr_target || !dL_dvr || !loss || !(sigma_v > 0))
        return arg_error("dsmc_mse_loss: bad arguments");
    const double scale = 1.0 / (4.0 * sigma_v * sigma_v * (double)B);
    // few workgroups: each adds its share with one FP64 atomic on the same
    // address, and those serialise
    int blocks = (int)((3 * B + 255) / 256);
    if (blocks > LOSS_BLOCKS) blocks = LOSS_BLOCKS;
    k_mse<<<blocks, 256, 0, as_stream(stream)>>>(B, vr_new, vr_target, scale, dL_dvr, loss);
    DSMC_LAUNCH_CHECK("mse");
    return DSMC_OK;
}

extern "C" int dsmc_direction_loss(int64_t B, const float* vr_new, const float* vr_target,
                                   float* dL_dvr, double* loss, dsmc_stream_t stream)
{
    if (B < 1 || !vr_new || !vr_target || !dL_dvr || !loss)
        return arg_error("dsmc_direction_loss: bad arguments");
    int blocks = (int)((B + 255) / 256);
    if (blocks > LOSS_BLOCKS) blocks = LOSS_BLOCKS;
    k_dir_loss<<<blocks, 256, 0, as_stream(stream)>>>(B, vr_new, vr_target, dL_dvr, loss);
    DSMC_LAUNCH_CHECK("direction_loss");
    return DSMC_OK;
}

extern "C" double dsmc_cosine_lr(int64_t t, int64_t T, double lr_max, double lr_min)
{
    if (T < 1) return lr_max;
    const double f = (double)(t < T ? (t > 0 ? t : 0) : T) / (double)T;
    return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + cos(M_PI * f));
}

extern "C" int dsmc_adam_step(int64_t n, float* param, void* param_bf16, const float* grad,
                              float* m, float* v, int64_t t, double lr, double beta1, double beta2,
                              double eps, dsmc_stream_t stream)
{
    if (n < 0 || (n > 0 && (!param || !grad || !m || !v)) || t < 1)
        return arg_error("dsmc_adam_step: bad arguments");
    if (n == 0) return DSMC_OK;
    const double bc1 = 1.0 - pow(beta1, (double)t);
    const double bc2 = 1.0 - pow(beta2, (double)t);
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    k_adam<<<blocks, 256, 0, as_stream(stream)>>>(n, param, (__bf16*)param_bf16, grad, m, v,
                                                  (float)beta1, (float)beta2, (float)(lr / bc1),
                                                  (float)eps, (float)sqrt(bc2));
    DSMC_LAUNCH_CHECK("adam");
    return DSMC_OK;
}
