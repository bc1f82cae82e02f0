// Angle network, its training pieces, the deflection-angle table it
// synthesises and the table collision rule (sections "Neural Network
// Architecture", "Neural Surrogate Training" and "Runtime Acceleration via
// Neural Table Look-up").
//
// Layer 0 (2 inputs) runs on the VALU in FP32 so the normalised ln E input is
// not rounded to bf16 (its 8-bit mantissa would move a grid row by ~4 % in
// E); layers 1.. run on the tiled BF16 MFMA GEMM with fused bias + SiLU (or
// Softplus on the output) epilogues.  The backward chains the same GEMMs: dW
// as dZ^T H with K split over workgroups (fixed-order sum), dH = dZ W with the
// SiLU derivative fused into the epilogue, db and the layer-0 weights by
// fixed-order column reductions.
#include <math.h>

#include "collide.hpp"
#include "gemm.hpp"

namespace dsmc {

constexpr double KB_SI = 1.380649e-23;
constexpr int ANET_SPLITS = 16;        // K split of the dW GEMMs
constexpr int64_t TABLE_CHUNK = 65536; // rows per table-synthesis pass

struct AnetDims {
    int L;
    int d[DSMC_ANET_MAX_LAYERS + 1];
    int dmax;   // widest layer output among layers 0..L-2
};

static int check_anet(const dsmc_anet* net, AnetDims* a)
{
    if (!net) return arg_error("dsmc_anet: null");
    if (net->n_layers < 2 || net->n_layers > DSMC_ANET_MAX_LAYERS)
        return arg_error("dsmc_anet: n_layers %d not in [2, %d]", net->n_layers,
                         DSMC_ANET_MAX_LAYERS);
    a->L = net->n_layers;
    a->dmax = 1;
    for (int l = 0; l <= a->L; ++l) {
        const int d = net->dims[l];
        if (d < 1 || d > 1024) return arg_error("dsmc_anet: dims[%d] = %d not in [1, 1024]", l, d);
        a->d[l] = d;
    }
    if (a->d[0] != 2 || a->d[a->L] != 1)
        return arg_error("dsmc_anet: dims[0] must be 2 and dims[n_layers] 1");
    for (int l = 0; l < a->L; ++l) {
        if (!net->W[l] || !net->b[l]) return arg_error("dsmc_anet: null W/b of layer %d", l);
        if (l < a->L - 1 && a->d[l + 1] > a->dmax) a->dmax = a->d[l + 1];
    }
    return DSMC_OK;
}

// Workspace of forward + backward on R rows.
struct AnetWs {
    float* x;                            // inputs [R][2] (for the layer-0 gradient)
    float* z[DSMC_ANET_MAX_LAYERS];      // pre-activations [R][d_{l+1}]
    __bf16* h[DSMC_ANET_MAX_LAYERS];     // activations of hidden layers [R][d_{l+1}]
    float* dz32[2];                      // [R][dmax]
    __bf16* dz16[2];                     // [R][dmax]
    float* partial;                      // [ANET_SPLITS][dmax][dmax]
    float* red;                          // [chunks][dmax][3]
    size_t bytes;
};

static AnetWs anet_layout(void* base, const AnetDims& a, int64_t R)
{
    AnetWs w{};
    uint8_t* p = static_cast<uint8_t*>(base);
    size_t o = 0;
    auto take = [&](size_t b) { uint8_t* r = p ? p + o : nullptr; o += align_up(b); return r; };
    w.x = reinterpret_cast<float*>(take(sizeof(float) * 2 * (size_t)R));
    for (int l = 0; l < a.L; ++l) {
        w.z[l] = reinterpret_cast<float*>(take(sizeof(float) * (size_t)R * a.d[l + 1]));
        if (l < a.L - 1)
            w.h[l] = reinterpret_cast<__bf16*>(take(sizeof(__bf16) * (size_t)R * a.d[l + 1]));
    }
    for (int q = 0; q < 2; ++q) {
        w.dz32[q] = reinterpret_cast<float*>(take(sizeof(float) * (size_t)R * a.dmax));
        w.dz16[q] = reinterpret_cast<__bf16*>(take(sizeof(__bf16) * (size_t)R * a.dmax));
    }
    size_t dd = 1;
    for (int l = 0; l < a.L; ++l) {
        const size_t x = (size_t)a.d[l] * a.d[l + 1];
        if (x > dd) dd = x;
    }
    w.partial = reinterpret_cast<float*>(take(sizeof(float) * ANET_SPLITS * dd));
    w.red = reinterpret_cast<float*>(take(sizeof(float) * colsum_ws_floats(R, a.dmax)));
    w.bytes = o;
    return w;
}

__device__ __forceinline__ float silu_f(float z)
{
    return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// Layer 0 on the VALU: z0 = W0 x + b0 (FP32), h0 = bf16(SiLU(z0)).  With
// grid != nullptr, x is the table grid node of row row0 + r.
struct TableGrid {
    int32_t n_e, n_b;
    double lne_lo, lne_hi;
};

// One wave per row at a time: the row's two inputs are formed once (table
// grid node or x), lane l computes outputs l, l + 64, ... with the layer-0
// weights of those columns held in registers across rows (n <= 1024).
constexpr int FIRST_COLS = 16;

__global__ void __launch_bounds__(256)
k_anet_first(int64_t R, int n, const float* __restrict__ x, const __bf16* __restrict__ W0,
             const float* __restrict__ b0, float* __restrict__ z0, __bf16* __restrict__ h0,
             float* __restrict__ xkeep, int64_t row0, TableGrid tg, int use_grid)
{
    const int lane = threadIdx.x & 63;
    float wa[FIRST_COLS], wb[FIRST_COLS], bb[FIRST_COLS];
#pragma unroll
    for (int e = 0; e < FIRST_COLS; ++e) {
        const int c = lane + 64 * e;
        wa[e] = c < n ? (float)W0[2 * c] : 0.0f;
        wb[e] = c < n ? (float)W0[2 * c + 1] : 0.0f;
        bb[e] = c < n ? b0[c] : 0.0f;
    }
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = wave; r < R; r += nwaves) {
        float x0, x1;
        if (use_grid) {
            const int64_t g = row0 + r;
            const int64_t i = g / tg.n_b, j = g - i * tg.n_b;
            // normalised ln E of node i: 2 i / (n_e - 1) - 1; b / b_max = j / (n_b - 1)
            x0 = (float)(2.0 * (double)i / (double)(tg.n_e - 1) - 1.0);
            x1 = (float)((double)j / (double)(tg.n_b - 1));
        } else {
            x0 = x[2 * r];
            x1 = x[2 * r + 1];
        }
        if (xkeep && lane == 0) {
            xkeep[2 * r] = x0;
            xkeep[2 * r + 1] = x1;
        }
#pragma unroll
        for (int e = 0; e < FIRST_COLS; ++e) {
            const int c = lane + 64 * e;
            if (c >= n) break;
            const float zz = wa[e] * x0 + wb[e] * x1 + bb[e];
            if (z0) z0[r * n + c] = zz;
            h0[r * n + c] = (__bf16)silu_f(zz);
        }
    }
}

// dz of the Softplus output: dy * sigmoid(z).
__global__ void __launch_bounds__(256)
k_out_delta(int64_t R, const float* __restrict__ dy, const float* __restrict__ z,
            float* __restrict__ d32, __bf16* __restrict__ d16)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < R;
         r += (int64_t)gridDim.x * blockDim.x) {
        const float d = dy[r] / (1.0f + expf(-z[r]));
        d32[r] = d;
        d16[r] = (__bf16)d;
    }
}

static int grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    const int pb = persistent_blocks(256);
    if (b > pb) b = pb;
    return (int)(b < 1 ? 1 : b);
}

// Forward of rows [0, R): layer 0 from x (or the table grid), then the GEMMs.
// z_keep: keep every layer's pre-activation (training); else only the last.
static int anet_forward_impl(const dsmc_anet* net, const AnetDims& a, int64_t R, const float* x,
                             float* y, const AnetWs& w, bool keep, int64_t row0,
                             const TableGrid* tg, hipStream_t s)
{
    const int n1 = a.d[1];
    k_anet_first<<<grid_for(R * n1), 256, 0, s>>>(
        R, n1, x, static_cast<const __bf16*>(net->W[0]), net->b[0], keep ? w.z[0] : nullptr,
        w.h[0], keep ? w.x : nullptr, row0, tg ? *tg : TableGrid{2, 2, 0.0, 1.0}, tg ? 1 : 0);
    DSMC_LAUNCH_CHECK("anet:first");
    for (int l = 1; l < a.L; ++l) {
        const bool last = l == a.L - 1;
        GemmArgs g{};
        g.a = w.h[l - 1];
        g.lda = a.d[l];
        g.ta = 0;
        g.b = static_cast<const __bf16*>(net->W[l]);
        g.ldb = a.d[l];
        g.tb = 1;
        g.M = R;
        g.N = a.d[l + 1];
        g.K = a.d[l];
        g.bias = net->b[l];
        g.z_out = (keep || last) ? w.z[l] : nullptr;
        g.ldz = a.d[l + 1];
        g.act = last ? GEMM_ACT_SOFTPLUS : GEMM_ACT_SILU;
        if (last) {
            g.out_f32 = y;
            g.ldo = 1;
        } else {
            g.out_bf16 = w.h[l];
            g.ldo = a.d[l + 1];
        }
        int rc = gemm_bf16(g, 1, s);
        if (rc) return rc;
    }
    return DSMC_OK;
}

// theta = clip(exp(y) - 1, 0, pi), in place.
__global__ void __launch_bounds__(256)
k_theta_from_y(int64_t n, float* __restrict__ t)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        float th = expm1f(t[q]);
        th = th < 0.f ? 0.f : (th > 3.14159265358979f ? 3.14159265358979f : th);
        t[q] = th;
    }
}

__global__ void __launch_bounds__(256)
k_anet_rows(int64_t n, const double* __restrict__ b, const double* __restrict__ g,
            const double* __restrict__ chi, double hmk, double lne_lo, double lne_hi,
            double inv_bmax, float* __restrict__ x, float* __restrict__ y)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        const double E = hmk * g[r] * g[r];
        x[2 * r] = (float)(2.0 * (log(E) - lne_lo) / (lne_hi - lne_lo) - 1.0);
        x[2 * r + 1] = (float)(b[r] * inv_bmax);
        const double th = acos(fmin(1.0, fmax(-1.0, cos(chi[r]))));
        y[r] = (float)log1p(th);
    }
}

// Huber loss: per-block partial sums, then one fixed-order final sum.
__global__ void __launch_bounds__(256)
k_huber(int64_t n, const float* __restrict__ yh, const float* __restrict__ y,
        float* __restrict__ dy, double* __restrict__ part)
{
    __shared__ double sh[256];
    double s = 0.0;
    const double inv_n = 1.0 / (double)n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)yh[q] - (double)y[q];
        const double ad = fabs(d);
        s += ad < 1.0 ? 0.5 * d * d : ad - 0.5;
        dy[q] = (float)(fmin(1.0, fmax(-1.0, d)) * inv_n);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_huber_final(const double* __restrict__ part, int nb, int64_t n, double* loss)
{
    double s = 0.0;
    for (int q = 0; q < nb; ++q) s += part[q];
    *loss = s / (double)n;
}

// Phase A of the table rule (RULE_CHI results: cos, sin, xi).
struct TableView {
    const float* theta;
    int32_t n_e, n_b;
    double lne_lo, lne_hi;
};

template <typename T>
__global__ void __launch_bounds__(256)
k_phaseA_table(int32_t n_cells, PairsView pr, dsmc_rng rng, V3<const T> v, T hmk, TableView tv,
               PairBuf<T> out)
{
    const int64_t np = pr.total(n_cells);
    const T span = T(tv.lne_hi - tv.lne_lo);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // two pairs per thread and iteration: the dependent loads of both (pair
    // record, velocities, table corners) are in flight together
    constexpr int U = 2;
    for (int64_t p0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p0 < np; p0 += U * stride) {
        int64_t pp[U];
        bool ok[U];
        int32_t kk[U], ii[U], jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            pp[u] = p0 + u * stride;
            ok[u] = pp[u] < np;
            const int64_t q = ok[u] ? pp[u] : p0;
            kk[u] = pr.cell[q];
            ii[u] = pr.i[q];
            jj[u] = pr.j[q];
        }
        T rx[U], ry[U], rz[U];
        uint32_t aa[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = ok[u] ? pp[u] : p0;
            aa[u] = (uint32_t)(q - pr.off[kk[u]]);
            rx[u] = v.x[ii[u]] - v.x[jj[u]];
            ry[u] = v.y[ii[u]] - v.y[jj[u]];
            rz[u] = v.z[ii[u]] - v.z[jj[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            T xi[3], z[2], u4;
            pair_latents(rng, aa[u], (uint32_t)kk[u], xi, z, u4);
            const T E = hmk * (rx[u] * rx[u] + ry[u] * ry[u] + rz[u] * rz[u]);
            T fe = (log(E) - T(tv.lne_lo)) / span * T(tv.n_e - 1);
            T fb = sqrt(u4) * T(tv.n_b - 1);
            fe = fe > T(0) ? (fe < T(tv.n_e - 1) ? fe : T(tv.n_e - 1)) : T(0);
            fb = fb > T(0) ? (fb < T(tv.n_b - 1) ? fb : T(tv.n_b - 1)) : T(0);
            int32_t i0 = (int32_t)floor(fe), j0 = (int32_t)floor(fb);
            if (i0 > tv.n_e - 2) i0 = tv.n_e - 2;
            if (j0 > tv.n_b - 2) j0 = tv.n_b - 2;
            const T te = fe - T(i0), tb = fb - T(j0);
            const float* row0 = tv.theta + (int64_t)i0 * tv.n_b + j0;
            const float* row1 = row0 + tv.n_b;
            const T t00 = row0[0], t01 = row0[1], t10 = row1[0], t11 = row1[1];
            const T th = (T(1) - te) * ((T(1) - tb) * t00 + tb * t01) +
                         te * ((T(1) - tb) * t10 + tb * t11);
            if (ok[u]) {
                const int64_t p = pp[u];
                out.a[p] = cos(th);
                out.b[p] = sin(th);
                out.c[p] = xi[0];
                out.d[p] = xi[1];
                out.e[p] = xi[2];
            }
        }
    }
}

static int check_table(const dsmc_chi_table* tab)
{
    if (!tab || !tab->theta) return arg_error("dsmc_chi_table: null");
    if (tab->n_e < 2 || tab->n_b < 2) return arg_error("dsmc_chi_table: n_e, n_b must be >= 2");
    if ((int64_t)tab->n_e * tab->n_b > ((int64_t)1 << 31))
        return arg_error("dsmc_chi_table: too many nodes");
    if (!(tab->lne_lo < tab->lne_hi)) return arg_error("dsmc_chi_table: lne_lo < lne_hi required");
    return DSMC_OK;
}

}  // namespace dsmc

using namespace dsmc;

extern "C" size_t dsmc_anet_ws(const dsmc_anet* net, int64_t rows)
{
    AnetDims a;
    if (check_anet(net, &a) || rows < 0) return 0;
    return anet_layout(nullptr, a, rows).bytes + 256;
}

extern "C" int dsmc_anet_forward(const dsmc_anet* net, int64_t rows, const float* x, float* y,
                                 void* ws, size_t ws_bytes, dsmc_stream_t stream)
{
    AnetDims a;
    int rc = check_anet(net, &a);
    if (rc) return rc;
    if (rows < 0) return arg_error("dsmc_anet_forward: rows < 0");
    if (rows == 0) return DSMC_OK;
    if (!x || !y || !ws) return arg_error("dsmc_anet_forward: null pointer");
    if (ws_bytes < dsmc_anet_ws(net, rows))
        return arg_error("dsmc_anet_forward: workspace %zu < %zu", ws_bytes, dsmc_anet_ws(net, rows));
    const AnetWs w = anet_layout(ws, a, rows);
    return anet_forward_impl(net, a, rows, x, y, w, true, 0, nullptr, as_stream(stream));
}

extern "C" int dsmc_anet_backward(const dsmc_anet* net, int64_t rows, const float* dy,
                                  float* const* dW, float* const* db, void* ws, size_t ws_bytes,
                                  dsmc_stream_t stream)
{
    AnetDims a;
    int rc = check_anet(net, &a);
    if (rc) return rc;
    if (rows <= 0) return arg_error("dsmc_anet_backward: rows must be > 0");
    if (!dy || !dW || !db || !ws) return arg_error("dsmc_anet_backward: null pointer");
    for (int l = 0; l < a.L; ++l)
        if (!dW[l] || !db[l]) return arg_error("dsmc_anet_backward: null dW/db of layer %d", l);
    if (ws_bytes < dsmc_anet_ws(net, rows))
        return arg_error("dsmc_anet_backward: workspace %zu < %zu", ws_bytes,
                         dsmc_anet_ws(net, rows));
    hipStream_t s = as_stream(stream);
    const AnetWs w = anet_layout(ws, a, rows);
    int cur = 0;
    const int L = a.L;
    k_out_delta<<<grid_for(rows), 256, 0, s>>>(rows, dy, w.z[L - 1], w.dz32[cur], w.dz16[cur]);
    DSMC_LAUNCH_CHECK("anet:out_delta");
    for (int l = L - 1; l >= 1; --l) {
        const int n_out = a.d[l + 1], n_in = a.d[l];
        // dW_l = dz_l^T h_{l-1}
        GemmArgs g{};
        g.a = w.dz16[cur];
        g.lda = n_out;
        g.ta = 1;
        g.b = w.h[l - 1];
        g.ldb = n_in;
        g.tb = 0;
        g.M = n_out;
        g.N = n_in;
        g.K = rows;
        g.act = GEMM_ACT_NONE;
        g.out_f32 = dW[l];
        g.ldo = n_in;
        g.partial = w.partial;
        rc = gemm_bf16(g, ANET_SPLITS, s);
        if (rc) return rc;
        // db_l
        rc = colsum_f32(w.dz32[cur], rows, n_out, nullptr, w.red, db[l], nullptr, 0, s);
        if (rc) return rc;
        // dz_{l-1} = (dz_l W_l) * SiLU'(z_{l-1})
        GemmArgs d{};
        d.a = w.dz16[cur];
        d.lda = n_out;
        d.ta = 0;
        d.b = static_cast<const __bf16*>(net->W[l]);
        d.ldb = n_in;
        d.tb = 0;
        d.M = rows;
        d.N = n_in;
        d.K = n_out;
        d.dact_z = w.z[l - 1];
        d.ldz = n_in;
        d.act = GEMM_ACT_SILU;
        d.out_f32 = w.dz32[1 - cur];
        d.out_bf16 = w.dz16[1 - cur];
        d.ldo = n_in;
        rc = gemm_bf16(d, 1, s);
        if (rc) return rc;
        cur = 1 - cur;
    }
    // layer 0: db_0 = sum dz_0, dW_0 = dz_0^T x
    return colsum_f32(w.dz32[cur], rows, a.d[1], w.x, w.red, db[0], dW[0], 0, s);
}

extern "C" int dsmc_huber_loss(int64_t n, const float* yhat, const float* y, float* dy,
                               double* loss, dsmc_stream_t stream)
{
    if (n <= 0) return arg_error("dsmc_huber_loss: n must be > 0");
    if (!yhat || !y || !dy || !loss) return arg_error("dsmc_huber_loss: null pointer");
    hipStream_t s = as_stream(stream);
    // one workgroup: its partial sum is the loss word itself, then divided by n
    k_huber<<<1, 256, 0, s>>>(n, yhat, y, dy, loss);
    DSMC_LAUNCH_CHECK("huber");
    k_huber_final<<<1, 1, 0, s>>>(loss, 1, n, loss);
    DSMC_LAUNCH_CHECK("huber_final");
    return DSMC_OK;
}

extern "C" int dsmc_anet_rows(int64_t n, const double* b, const double* g, const double* chi,
                              double m_red, double lne_lo, double lne_hi, double b_max, float* x,
                              float* y, dsmc_stream_t stream)
{
    if (n < 0) return arg_error("dsmc_anet_rows: n < 0");
    if (n == 0) return DSMC_OK;
    if (!b || !g || !chi || !x || !y) return arg_error("dsmc_anet_rows: null pointer");
    if (!(m_red > 0) || !(b_max > 0) || !(lne_lo < lne_hi))
        return arg_error("dsmc_anet_rows: m_red, b_max > 0 and lne_lo < lne_hi required");
    hipStream_t s = as_stream(stream);
    k_anet_rows<<<grid_for(n), 256, 0, s>>>(n, b, g, chi, 0.5 * m_red / KB_SI, lne_lo, lne_hi,
                                            1.0 / b_max, x, y);
    DSMC_LAUNCH_CHECK("anet_rows");
    return DSMC_OK;
}

static int64_t table_rows(const dsmc_chi_table* tab)
{
    const int64_t n = (int64_t)tab->n_e * tab->n_b;
    return n < TABLE_CHUNK ? n : TABLE_CHUNK;
}

extern "C" size_t dsmc_chi_table_ws(const dsmc_anet* net, const dsmc_chi_table* tab)
{
    AnetDims a;
    if (check_anet(net, &a) || check_table(tab)) return 0;
    return anet_layout(nullptr, a, table_rows(tab)).bytes + 256;
}

extern "C" int dsmc_chi_table_build(const dsmc_anet* net, const dsmc_chi_table* tab, void* ws,
                                    size_t ws_bytes, dsmc_stream_t stream)
{
    AnetDims a;
    int rc = check_anet(net, &a);
    if (rc) return rc;
    rc = check_table(tab);
    if (rc) return rc;
    if (!ws) return arg_error("dsmc_chi_table_build: null workspace");
    if (ws_bytes < dsmc_chi_table_ws(net, tab))
        return arg_error("dsmc_chi_table_build: workspace %zu < %zu", ws_bytes,
                         dsmc_chi_table_ws(net, tab));
    hipStream_t s = as_stream(stream);
    const int64_t total = (int64_t)tab->n_e * tab->n_b;
    const int64_t RC = table_rows(tab);
    const AnetWs w = anet_layout(ws, a, RC);
    const TableGrid tg{tab->n_e, tab->n_b, tab->lne_lo, tab->lne_hi};
    for (int64_t r0 = 0; r0 < total; r0 += RC) {
        const int64_t R = total - r0 < RC ? total - r0 : RC;
        rc = anet_forward_impl(net, a, R, nullptr, tab->theta + r0, w, false, r0, &tg, s);
        if (rc) return rc;
    }
    k_theta_from_y<<<grid_for(total), 256, 0, s>>>(total, tab->theta);
    DSMC_LAUNCH_CHECK("chi_table:theta");
    return DSMC_OK;
}

extern "C" int dsmc_collide_table(const dsmc_chi_table* tab, int32_t n_cells, int32_t dtype,
                                  dsmc_vec3 v, dsmc_pairs pairs, dsmc_rng rng, double m_red,
                                  int32_t schedule, void* ws, size_t ws_bytes,
                                  dsmc_stream_t stream)
{
    int rc = check_table(tab);
    if (rc) return rc;
    rc = check_pairs("dsmc_collide_table", n_cells, v, pairs, dtype, ws, ws_bytes);
    if (rc) return rc;
    if (!(m_red > 0)) return arg_error("dsmc_collide_table: m_red must be > 0");
    if (schedule < DSMC_SCHED_AUTO || schedule > DSMC_SCHED_WAVE)
        return arg_error("dsmc_collide_table: schedule %d", schedule);
    hipStream_t s = as_stream(stream);
    const PairsView pr = PairsView::of(pairs);
    const int pb = persistent_blocks(256);
    const TableView tv{tab->theta, tab->n_e, tab->n_b, tab->lne_lo, tab->lne_hi};
    const double hmk = 0.5 * m_red / KB_SI;
    if (dtype == DSMC_F64)
        k_phaseA_table<double><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const double>(v), hmk, tv,
                                                 PairBuf<double>::of(ws, pairs.cap));
    else
        k_phaseA_table<float><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const float>(v), (float)hmk,
                                                tv, PairBuf<float>::of(ws, pairs.cap));
    DSMC_LAUNCH_CHECK("collide_table:phaseA");
    if (schedule == DSMC_SCHED_DEFER) return DSMC_OK;
    return phase_b(RULE_CHI, dtype, n_cells, nullptr, v, pairs, ws, pairs.cap, schedule, s);
}
