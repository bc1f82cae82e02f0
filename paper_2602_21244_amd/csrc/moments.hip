// Cell moments and cell-wise moment matching (section "Optional Cell-Wise
// Energy Drift Correction", eq. cell_energy_clamp).  One wavefront per cell;
// lanes stride over the cell's contiguous particles with coalesced SoA loads,
// sums are kept in FP64 and combined with cross-lane shuffles in a fixed
// order (deterministic).
#include "common.hpp"

namespace dsmc {

struct CellSums {
    double ux, uy, uz, S, cmax, E;
};

// Two passes over the cell: mean, then centred sums.
template <typename T>
__device__ __forceinline__ CellSums cell_sums(V3<T> v, int32_t s0, int32_t N, int lane)
{
    CellSums r{0, 0, 0, 0, 0, 0};
    if (N <= 0) return r;
    // each lane adds its slots lane, lane + 64, ... in order; the loads of
    // SUM_BATCH consecutive terms are issued together
    constexpr int SUM_BATCH = 4;
    double sx = 0, sy = 0, sz = 0;
    for (int32_t q0 = lane; q0 < N; q0 += 64 * SUM_BATCH) {
        T x[SUM_BATCH], y[SUM_BATCH], z[SUM_BATCH];
#pragma unroll
        for (int b = 0; b < SUM_BATCH; ++b) {
            const int32_t q = q0 + 64 * b;
            if (q < N) { x[b] = v.x[s0 + q]; y[b] = v.y[s0 + q]; z[b] = v.z[s0 + q]; }
        }
#pragma unroll
        for (int b = 0; b < SUM_BATCH; ++b)
            if (q0 + 64 * b < N) {
                sx += (double)x[b];
                sy += (double)y[b];
                sz += (double)z[b];
            }
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    sz = wave_sum(sz);
    r.ux = sx / N; r.uy = sy / N; r.uz = sz / N;
    double S = 0, c2max = 0, E = 0;
    for (int32_t q0 = lane; q0 < N; q0 += 64 * SUM_BATCH) {
        T xb[SUM_BATCH], yb[SUM_BATCH], zb[SUM_BATCH];
#pragma unroll
        for (int b = 0; b < SUM_BATCH; ++b) {
            const int32_t q = q0 + 64 * b;
            if (q < N) { xb[b] = v.x[s0 + q]; yb[b] = v.y[s0 + q]; zb[b] = v.z[s0 + q]; }
        }
#pragma unroll
        for (int b = 0; b < SUM_BATCH; ++b) {
            if (q0 + 64 * b >= N) continue;
            const double x = xb[b], y = yb[b], z = zb[b];
            const double dx = x - r.ux, dy = y - r.uy, dz = z - r.uz;
            const double c2 = dx * dx + dy * dy + dz * dz;
            S += c2;
            c2max = fmax(c2max, c2);
            E += x * x + y * y + z * z;
        }
    }
    r.S = wave_sum(S);
    r.cmax = sqrt(wave_max(c2max));
    r.E = wave_sum(E);
    return r;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_capture(const int32_t* __restrict__ cell_start, int32_t n_cells, V3<T> v, double* mom)
{
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int64_t kstep = (int64_t)gridDim.x * wpb;
    int64_t k = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
    // the next cell's bounds are loaded while the current cell is summed
    int32_t a0 = k < n_cells ? cell_start[k] : 0, a1 = k < n_cells ? cell_start[k + 1] : 0;
    for (; k < n_cells; k += kstep) {
        const int32_t s0 = a0, N = a1 - a0;
        const int64_t kn = k + kstep;
        a0 = kn < n_cells ? cell_start[kn] : 0;
        a1 = kn < n_cells ? cell_start[kn + 1] : 0;
        const CellSums c = cell_sums(v, s0, N, lane);
        if (lane == 0) {
            double* m = mom + 6 * (size_t)k;
            m[0] = c.ux; m[1] = c.uy; m[2] = c.uz; m[3] = c.S; m[4] = c.cmax; m[5] = c.E;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_apply(const int32_t* __restrict__ cell_start, int32_t n_cells, V3<T> v,
        const double* __restrict__ mom, const int32_t* __restrict__ pair_cnt, int literal,
        dsmc_status* st)
{
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    for (int32_t k = blockIdx.x * wpb + (threadIdx.x >> 6); k < n_cells; k += gridDim.x * wpb) {
        const int32_t s0 = cell_start[k], N = cell_start[k + 1] - s0;
        if (N < 2) continue;
        if (pair_cnt && pair_cnt[k] == 0) continue;
        const CellSums c = cell_sums(v, s0, N, lane);
        const double* m = mom + 6 * (size_t)k;
        const double post = literal ? c.E : c.S;
        if (!(post > 0.0) || !isfinite(post)) {
            if (lane == 0 && st) atomicAdd(&st->mm_skipped, 1);
            continue;
        }
        const double alpha = sqrt((literal ? m[5] : m[3]) / post);
        for (int32_t q = lane; q < N; q += 64) {
            const int32_t s = s0 + q;
            if (literal) {
                v.x[s] = (T)(alpha * (double)v.x[s]);
                v.y[s] = (T)(alpha * (double)v.y[s]);
                v.z[s] = (T)(alpha * (double)v.z[s]);
            } else {
                v.x[s] = (T)(m[0] + alpha * ((double)v.x[s] - c.ux));
                v.y[s] = (T)(m[1] + alpha * ((double)v.y[s] - c.uy));
                v.z[s] = (T)(m[2] + alpha * ((double)v.z[s] - c.uz));
            }
        }
    }
}

// Adjoint of the centred matching of one cell (for training on cell groups).
__global__ void __launch_bounds__(256)
k_match_backward(const int32_t* __restrict__ cell_start, int32_t n_cells,
                 const double* __restrict__ mom, V3<const double> vp, V3<const double> G,
                 V3<double> out)
{
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    for (int32_t k = blockIdx.x * wpb + (threadIdx.x >> 6); k < n_cells; k += gridDim.x * wpb) {
        const int32_t s0 = cell_start[k], N = cell_start[k + 1] - s0;
        if (N <= 0) continue;
        const CellSums c = cell_sums(V3<double>{const_cast<double*>(vp.x), const_cast<double*>(vp.y),
                                                const_cast<double*>(vp.z)},
                                     s0, N, lane);
        const bool pass = (N < 2) || !(c.S > 0.0);
        double gx = 0, gy = 0, gz = 0, gc = 0;
        for (int32_t q = lane; q < N; q += 64) {
            const int32_t s = s0 + q;
            gx += G.x[s]; gy += G.y[s]; gz += G.z[s];
            gc += G.x[s] * (vp.x[s] - c.ux) + G.y[s] * (vp.y[s] - c.uy) + G.z[s] * (vp.z[s] - c.uz);
        }
        gx = wave_sum(gx) / N; gy = wave_sum(gy) / N; gz = wave_sum(gz) / N;
        gc = wave_sum(gc);
        const double alpha = pass ? 1.0 : sqrt(mom[6 * (size_t)k + 3] / c.S);
        for (int32_t q = lane; q < N; q += 64) {
            const int32_t s = s0 + q;
            if (pass) {
                out.x[s] = G.x[s]; out.y[s] = G.y[s]; out.z[s] = G.z[s];
            } else {
                const double f = alpha / c.S * gc;
                out.x[s] = alpha * (G.x[s] - gx) - f * (vp.x[s] - c.ux);
                out.y[s] = alpha * (G.y[s] - gy) - f * (vp.y[s] - c.uy);
                out.z[s] = alpha * (G.z[s] - gz) - f * (vp.z[s] - c.uz);
            }
        }
    }
}

static int cell_blocks(int32_t n_cells)
{
    const int pb = persistent_blocks(256);
    int b = (n_cells + 3) / 4;
    return b < 1 ? 1 : (b > pb ? pb : b);
}

template <typename T>
static int mm_impl(int32_t n_cells, const int32_t* cell_start, dsmc_vec3 v, double* mom,
                   int32_t mode, const int32_t* pair_cnt, dsmc_status* st, hipStream_t s)
{
    const int blocks = cell_blocks(n_cells);
    if (mode == DSMC_MM_CAPTURE) {
        k_capture<T><<<blocks, 256, 0, s>>>(cell_start, n_cells, v3<T>(v), mom);
        DSMC_LAUNCH_CHECK("moment_match:capture");
    } else {
        k_apply<T><<<blocks, 256, 0, s>>>(cell_start, n_cells, v3<T>(v), mom, pair_cnt,
                                          mode == DSMC_MM_APPLY_LITERAL, st);
        DSMC_LAUNCH_CHECK("moment_match:apply");
    }
    return DSMC_OK;
}

}  // namespace dsmc

using namespace dsmc;

extern "C" int dsmc_moment_match(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                                 dsmc_vec3 v, double* mom, int32_t mode, const int32_t* pair_cnt,
                                 dsmc_status* st, dsmc_stream_t stream)
{
    if (n_cells < 1) return arg_error("dsmc_moment_match: n_cells=%d", n_cells);
    if (!cell_start || !mom || !v.x || !v.y || !v.z)
        return arg_error("dsmc_moment_match: null pointer");
    if (mode != DSMC_MM_CAPTURE && mode != DSMC_MM_APPLY && mode != DSMC_MM_APPLY_LITERAL)
        return arg_error("dsmc_moment_match: mode %d", mode);
    hipStream_t s = as_stream(stream);
    if (dtype == DSMC_F64) return mm_impl<double>(n_cells, cell_start, v, mom, mode, pair_cnt, st, s);
    if (dtype == DSMC_F32) return mm_impl<float>(n_cells, cell_start, v, mom, mode, pair_cnt, st, s);
    return arg_error("dsmc_moment_match: dtype %d", dtype);
}

extern "C" int dsmc_moment_match_backward(int32_t n_cells, const int32_t* cell_start,
                                          const double* mom_pre, const double* vx,
                                          const double* vy, const double* vz,
                                          const double* gx, const double* gy, const double* gz,
                                          double* ox, double* oy, double* oz,
                                          dsmc_stream_t stream)
{
    if (n_cells < 1) return arg_error("dsmc_moment_match_backward: n_cells=%d", n_cells);
    if (!cell_start || !mom_pre || !vx || !vy || !vz || !gx || !gy || !gz || !ox || !oy || !oz)
        return arg_error("dsmc_moment_match_backward: null pointer");
    k_match_backward<<<cell_blocks(n_cells), 256, 0, as_stream(stream)>>>(
        cell_start, n_cells, mom_pre, V3<const double>{vx, vy, vz}, V3<const double>{gx, gy, gz},
        V3<double>{ox, oy, oz});
    DSMC_LAUNCH_CHECK("moment_match_backward");
    return DSMC_OK;
}
