// Collision application.
//
// Phase A (one lane per accepted pair, on the pre-collision velocities) turns
// the pair's latents into a post-collision direction (isotropic rule) or, for
// the other rules, is done by their own kernels.  Phase B applies the pairs of
// each cell in candidate order on the current velocities with the
// centre-of-mass update of eq. v_update_pair.  Two Phase-B schedules:
//   LANE  -- one lane walks one cell's pairs sequentially;
//   WAVE  -- one 64-lane workgroup per cell, the cell's velocities staged in
//            LDS, applying in parallel, round by round, every pending pair
//            that is the earliest pending pair of both of its particles;
//   BLOCK -- the same dependency rounds by a 256-lane workgroup on
//            velocities in global memory (cells too big for WAVE).
// A pair's update depends only on the current velocities of its two particles,
// and BLOCK applies each pair after every earlier pair that shares a particle,
// so both schedules produce bit-identical velocities.
#include "collide.hpp"

#include <limits.h>

namespace dsmc {

// ------------------------------------------------------------------------
// Phase A of the isotropic rule: cos chi = 2 U4 - 1 (uniform on [-1, 1]),
// azimuth from xi; u = cos chi vhat + sin chi e_perp.
// ------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_phaseA_vhs(int32_t n_cells, PairsView pr, dsmc_rng rng, V3<const T> v, PairBuf<T> out)
{
    const int64_t np = pr.total(n_cells);
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = pr.cell[p];
        const uint32_t a = (uint32_t)(p - pr.off[k]);
        T xi[3], z[2], u4;
        pair_latents(rng, a, (uint32_t)k, xi, z, u4);
        const int32_t i = pr.i[p], j = pr.j[p];
        T vh[3], e[3];
        unit3<T>(v.x[i] - v.x[j], v.y[i] - v.y[j], v.z[i] - v.z[j], vh);
        // cos chi = 2 U4 - 1; sin chi = sqrt((1 - cos)(1 + cos)) = 2 sqrt(U4 (1 - U4))
        const T cc = T(2) * u4 - T(1);
        const T sc = T(2) * dev_sqrt<T>(u4 * (T(1) - u4));
        perp_dir<T>(xi, vh, e);
        out.a[p] = cc * vh[0] + sc * e[0];
        out.b[p] = cc * vh[1] + sc * e[1];
        out.c[p] = cc * vh[2] + sc * e[2];
    }
}

// ------------------------------------------------------------------------
// One pair update on the current velocities (FP64 arithmetic, stored in T).
// RULE_DIR: v_r' = |v_r| u.  RULE_CHI: v_r' = |v_r| (cos chi vhat + sin chi
// e_perp(xi, vhat)) with vhat of the current v_r.
// ------------------------------------------------------------------------
template <typename T, int RULE>
__device__ __forceinline__ void apply_pair(V3<T> v, int32_t a, int32_t b, const PairBuf<T>& d,
                                           int64_t p)
{
    const double xa = v.x[a], ya = v.y[a], za = v.z[a];
    const double xb = v.x[b], yb = v.y[b], zb = v.z[b];
    const double rx = xa - xb, ry = ya - yb, rz = za - zb;
    double u[3];
    double g;
    if (RULE == RULE_DIR) {
        g = sqrt(rx * rx + ry * ry + rz * rz);
        // renormalised in FP64 so |v_r'| = |v_r| holds to rounding even when
        // the direction came from a lower-precision rule
        const double a0 = d.a[p], a1 = d.b[p], a2 = d.c[p];
        const double inv = 1.0 / sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        u[0] = a0 * inv; u[1] = a1 * inv; u[2] = a2 * inv;
    } else {
        double vh[3], e[3];
        g = unit3<double>(rx, ry, rz, vh);
        const double xi[3] = {(double)d.c[p], (double)d.d[p], (double)d.e[p]};
        perp_dir<double>(xi, vh, e);
        const double cc = d.a[p], sc = d.b[p];
        u[0] = cc * vh[0] + sc * e[0];
        u[1] = cc * vh[1] + sc * e[1];
        u[2] = cc * vh[2] + sc * e[2];
    }
    const double cx = 0.5 * (xa + xb), cy = 0.5 * (ya + yb), cz = 0.5 * (za + zb);
    const double px = 0.5 * g * u[0], py = 0.5 * g * u[1], pz = 0.5 * g * u[2];
    v.x[a] = (T)(cx + px); v.y[a] = (T)(cy + py); v.z[a] = (T)(cz + pz);
    v.x[b] = (T)(cx - px); v.y[b] = (T)(cy - py); v.z[b] = (T)(cz - pz);
}

template <typename T, int RULE>
__global__ void __launch_bounds__(256)
k_phaseB_lane(int32_t n_cells, PairsView pr, V3<T> v, PairBuf<T> d, int32_t max_pairs)
{
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_cells;
         k += gridDim.x * blockDim.x) {
        const int32_t c = pr.cnt[k];
        if (c == 0 || c > max_pairs) continue;
        const int64_t o = pr.off[k];
        for (int32_t q = 0; q < c; ++q)
            apply_pair<T, RULE>(v, pr.i[o + q], pr.j[o + q], d, o + q);
    }
}

constexpr int WV_NMAX = 1024;
constexpr int WV_PPL = 4;

__device__ __forceinline__ bool wave_fits(int32_t c, int32_t span)
{
    return c <= 64 * WV_PPL && span <= WV_NMAX;
}

constexpr int BLK_THREADS = 256;
constexpr int BLK_NMAX = 8192;   // particles of a cell tracked in LDS
constexpr int BLK_MMAX = 8192;   // pairs of a cell tracked in LDS

template <typename T, int RULE>
__global__ void __launch_bounds__(BLK_THREADS)
k_phaseB_block(int32_t n_cells, PairsView pr, V3<T> v, PairBuf<T> d, int32_t min_pairs,
               int32_t skip_wave_cells)
{
    __shared__ int32_t first[BLK_NMAX];     // earliest pending pair of each particle
    __shared__ uint32_t pij[BLK_MMAX];      // local (i | j << 16) of each pair, ~0 once applied
    __shared__ int32_t red[2][BLK_THREADS / 64];
    __shared__ int32_t remaining;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int32_t k = blockIdx.x; k < n_cells; k += gridDim.x) {
        const int32_t c = pr.cnt[k];
        if (c == 0 || c < min_pairs) continue;
        const int64_t o = pr.off[k];
        // local frame: the span of sorted slots the cell's pairs touch
        int32_t lo = INT32_MAX, hi = -1;
        for (int32_t q = threadIdx.x; q < c; q += BLK_THREADS) {
            const int32_t a = pr.i[o + q], b = pr.j[o + q];
            lo = min(lo, min(a, b));
            hi = max(hi, max(a, b));
        }
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) {
            lo = min(lo, __shfl_xor(lo, s, 64));
            hi = max(hi, __shfl_xor(hi, s, 64));
        }
        if (lane == 0) { red[0][wid] = lo; red[1][wid] = hi; }
        __syncthreads();
        lo = red[0][0]; hi = red[1][0];
        for (int w = 1; w < BLK_THREADS / 64; ++w) { lo = min(lo, red[0][w]); hi = max(hi, red[1][w]); }
        const int32_t span = hi - lo + 1;
        if (skip_wave_cells && wave_fits(c, span)) continue;  // uniform: done by the WAVE kernel
        if (span > BLK_NMAX || c > BLK_MMAX || span > 65535) {
            // beyond the LDS tables: sequential, still in candidate order
            if (threadIdx.x == 0)
                for (int32_t q = 0; q < c; ++q)
                    apply_pair<T, RULE>(v, pr.i[o + q], pr.j[o + q], d, o + q);
            __syncthreads();
            continue;
        }
        for (int32_t q = threadIdx.x; q < c; q += BLK_THREADS)
            pij[q] = (uint32_t)(pr.i[o + q] - lo) | ((uint32_t)(pr.j[o + q] - lo) << 16);
        if (threadIdx.x == 0) remaining = c;
        __syncthreads();
        while (remaining > 0) {
            for (int32_t q = threadIdx.x; q < span; q += BLK_THREADS) first[q] = INT32_MAX;
            __syncthreads();
            for (int32_t q = threadIdx.x; q < c; q += BLK_THREADS) {
                const uint32_t w = pij[q];
                if (w != 0xffffffffu) {
                    atomicMin(&first[w & 0xffff], q);
                    atomicMin(&first[w >> 16], q);
                }
            }
            __syncthreads();
            int done_here = 0;
            for (int32_t q = threadIdx.x; q < c; q += BLK_THREADS) {
                const uint32_t w = pij[q];
                if (w == 0xffffffffu) continue;
                const int32_t li = w & 0xffff, lj = w >> 16;
                if (first[li] == q && first[lj] == q) {
                    apply_pair<T, RULE>(v, lo + li, lo + lj, d, o + q);
                    pij[q] = 0xffffffffu;
                    ++done_here;
                }
            }
            __syncthreads();
            if (done_here) atomicSub(&remaining, done_here);
            __syncthreads();
        }
    }
}

// WAVE schedule: one 64-lane workgroup per cell with the cell's velocities
// staged in LDS; each lane owns up to WV_PPL pairs; dependency rounds as in
// the BLOCK schedule but entirely in LDS.  Cells with more pairs, or whose
// pairs span more than WV_NMAX slots, are left to the BLOCK kernel.

template <typename T, int RULE>
__device__ __forceinline__ void apply_pair_lds(T* lx, T* ly, T* lz, int32_t a, int32_t b,
                                               const PairBuf<T>& d, int64_t p)
{
    const double xa = lx[a], ya = ly[a], za = lz[a];
    const double xb = lx[b], yb = ly[b], zb = lz[b];
    const double rx = xa - xb, ry = ya - yb, rz = za - zb;
    double u[3];
    double g;
    if (RULE == RULE_DIR) {
        g = sqrt(rx * rx + ry * ry + rz * rz);
        const double a0 = d.a[p], a1 = d.b[p], a2 = d.c[p];
        const double inv = 1.0 / sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        u[0] = a0 * inv; u[1] = a1 * inv; u[2] = a2 * inv;
    } else {
        double vh[3], e[3];
        g = unit3<double>(rx, ry, rz, vh);
        const double xi[3] = {(double)d.c[p], (double)d.d[p], (double)d.e[p]};
        perp_dir<double>(xi, vh, e);
        const double cc = d.a[p], sc = d.b[p];
        u[0] = cc * vh[0] + sc * e[0];
        u[1] = cc * vh[1] + sc * e[1];
        u[2] = cc * vh[2] + sc * e[2];
    }
    const double cx = 0.5 * (xa + xb), cy = 0.5 * (ya + yb), cz = 0.5 * (za + zb);
    const double px = 0.5 * g * u[0], py = 0.5 * g * u[1], pz = 0.5 * g * u[2];
    lx[a] = (T)(cx + px); ly[a] = (T)(cy + py); lz[a] = (T)(cz + pz);
    lx[b] = (T)(cx - px); ly[b] = (T)(cy - py); lz[b] = (T)(cz - pz);
}

template <typename T, int RULE>
__global__ void __launch_bounds__(64)
k_phaseB_wave(int32_t n_cells, PairsView pr, V3<T> v, PairBuf<T> d, int32_t min_pairs)
{
    __shared__ T lx[WV_NMAX], ly[WV_NMAX], lz[WV_NMAX];
    __shared__ int32_t first[WV_NMAX];
    const int lane = threadIdx.x;
    for (int32_t k = blockIdx.x; k < n_cells; k += gridDim.x) {
        const int32_t c = pr.cnt[k];
        if (c == 0 || c < min_pairs || c > 64 * WV_PPL) continue;
        const int64_t o = pr.off[k];
        int32_t pa[WV_PPL], pb[WV_PPL];
        int32_t lo = INT32_MAX, hi = -1;
        uint32_t pend = 0;
#pragma unroll
        for (int m = 0; m < WV_PPL; ++m) {
            const int32_t q = lane + 64 * m;
            pa[m] = 0;
            pb[m] = 0;
            if (q < c) {
                pa[m] = pr.i[o + q];
                pb[m] = pr.j[o + q];
                lo = min(lo, min(pa[m], pb[m]));
                hi = max(hi, max(pa[m], pb[m]));
                pend |= 1u << m;
            }
        }
#pragma unroll
        for (int sft = 32; sft > 0; sft >>= 1) {
            lo = min(lo, __shfl_xor(lo, sft, 64));
            hi = max(hi, __shfl_xor(hi, sft, 64));
        }
        const int32_t span = hi - lo + 1;
        if (!wave_fits(c, span)) continue;
        for (int32_t q = lane; q < span; q += 64) {
            lx[q] = v.x[lo + q];
            ly[q] = v.y[lo + q];
            lz[q] = v.z[lo + q];
        }
#pragma unroll
        for (int m = 0; m < WV_PPL; ++m) { pa[m] -= lo; pb[m] -= lo; }
        __syncthreads();
        while (__ballot(pend != 0)) {
            for (int32_t q = lane; q < span; q += 64) first[q] = INT32_MAX;
            __syncthreads();
#pragma unroll
            for (int m = 0; m < WV_PPL; ++m)
                if (pend & (1u << m)) {
                    atomicMin(&first[pa[m]], lane + 64 * m);
                    atomicMin(&first[pb[m]], lane + 64 * m);
                }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < WV_PPL; ++m) {
                const int32_t q = lane + 64 * m;
                if ((pend & (1u << m)) && first[pa[m]] == q && first[pb[m]] == q) {
                    apply_pair_lds<T, RULE>(lx, ly, lz, pa[m], pb[m], d, o + q);
                    pend &= ~(1u << m);
                }
            }
            __syncthreads();
        }
        for (int32_t q = lane; q < span; q += 64) {
            v.x[lo + q] = lx[q];
            v.y[lo + q] = ly[q];
            v.z[lo + q] = lz[q];
        }
        __syncthreads();
    }
}

int phase_b(int rule, int dtype, int32_t n_cells, const int32_t* cell_start, dsmc_vec3 v,
            const dsmc_pairs& pairs, void* dirs, int64_t cap, int32_t schedule, hipStream_t s)
{
    (void)cell_start;
    const PairsView pr = PairsView::of(pairs);
    const int pb = persistent_blocks(256);
    int lb = (n_cells + 255) / 256;
    lb = lb < 1 ? 1 : (lb > pb ? pb : lb);
    // cells with at most `thr` pairs: LANE; larger: WAVE if they fit its LDS
    // tables (AUTO, WAVE), else BLOCK
    int32_t thr = block_threshold();
    bool use_wave = true;
    if (schedule == DSMC_SCHED_LANE) thr = INT32_MAX;
    if (schedule == DSMC_SCHED_BLOCK) { thr = 0; use_wave = false; }
    if (schedule == DSMC_SCHED_WAVE) thr = 0;
    const bool need_lane = thr > 0;
    const bool need_rest = thr < INT32_MAX;
    int bb = n_cells < pb ? n_cells : pb;
    bb = bb < 1 ? 1 : bb;
    int wb = n_cells < pb * 8 ? n_cells : pb * 8;
    wb = wb < 1 ? 1 : wb;
#define DSMC_PHASEB(T, R)                                                                   \
    do {                                                                                    \
        PairBuf<T> d = PairBuf<T>::of(dirs, cap);                                           \
        if (need_lane) {                                                                    \
            k_phaseB_lane<T, R><<<lb, 256, 0, s>>>(n_cells, pr, v3<T>(v), d, thr);          \
            DSMC_LAUNCH_CHECK("phaseB:lane");                                               \
        }                                                                                   \
        if (need_rest && use_wave) {                                                        \
            k_phaseB_wave<T, R><<<wb, 64, 0, s>>>(n_cells, pr, v3<T>(v), d, thr + 1);       \
            DSMC_LAUNCH_CHECK("phaseB:wave");                                               \
        }                                                                                   \
        if (need_rest) {                                                                    \
            k_phaseB_block<T, R><<<bb, BLK_THREADS, 0, s>>>(n_cells, pr, v3<T>(v), d,       \
                                                            thr + 1, use_wave ? 1 : 0);     \
            DSMC_LAUNCH_CHECK("phaseB:block");                                              \
        }                                                                                   \
    } while (0)
    if (dtype == DSMC_F64) {
        if (rule == RULE_DIR) DSMC_PHASEB(double, RULE_DIR); else DSMC_PHASEB(double, RULE_CHI);
    } else {
        if (rule == RULE_DIR) DSMC_PHASEB(float, RULE_DIR); else DSMC_PHASEB(float, RULE_CHI);
    }
#undef DSMC_PHASEB
    return DSMC_OK;
}

int check_pairs(const char* who, int32_t n_cells, dsmc_vec3 v, const dsmc_pairs& pairs,
                int32_t dtype, void* ws, size_t ws_bytes)
{
    if (n_cells < 1) return arg_error("%s: n_cells=%d", who, n_cells);
    if (!v.x || !v.y || !v.z || !pairs.off || !pairs.cnt || !ws ||
        (pairs.cap > 0 && (!pairs.i || !pairs.j || !pairs.cell)))
        return arg_error("%s: null pointer", who);
    if (dtype != DSMC_F32 && dtype != DSMC_F64) return arg_error("%s: dtype %d", who, dtype);
    if (pairs.cap < 0) return arg_error("%s: cap < 0", who);
    if (ws_bytes < dsmc_collide_ws(pairs.cap, dtype))
        return arg_error("%s: workspace %zu < %zu", who, ws_bytes, dsmc_collide_ws(pairs.cap, dtype));
    return DSMC_OK;
}

}  // namespace dsmc

using namespace dsmc;

extern "C" size_t dsmc_collide_ws(int64_t cap, int32_t dtype)
{
    const size_t es = dtype == DSMC_F64 ? 8 : 4;
    return align_up(PairBuf<double>::kFields * es * (size_t)(cap + 1)) + 256;
}

extern "C" int dsmc_collide_vhs(int32_t n_cells, int32_t dtype, dsmc_vec3 v, dsmc_pairs pairs,
                                dsmc_rng rng, int32_t schedule, void* ws, size_t ws_bytes,
                                dsmc_stream_t stream)
{
    int rc = check_pairs("dsmc_collide_vhs", n_cells, v, pairs, dtype, ws, ws_bytes);
    if (rc) return rc;
    if (schedule < DSMC_SCHED_AUTO || schedule > DSMC_SCHED_WAVE)
        return arg_error("dsmc_collide_vhs: schedule %d", schedule);
    hipStream_t s = as_stream(stream);
    const PairsView pr = PairsView::of(pairs);
    const int pb = persistent_blocks(256);
    if (dtype == DSMC_F64) {
        k_phaseA_vhs<double><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const double>(v),
                                               PairBuf<double>::of(ws, pairs.cap));
    } else {
        k_phaseA_vhs<float><<<pb, 256, 0, s>>>(n_cells, pr, rng, v3<const float>(v),
                                              PairBuf<float>::of(ws, pairs.cap));
    }
    DSMC_LAUNCH_CHECK("collide_vhs:phaseA");
    if (schedule == DSMC_SCHED_DEFER) return DSMC_OK;
    return phase_b(RULE_DIR, dtype, n_cells, nullptr, v, pairs, ws, pairs.cap, schedule, s);
}

extern "C" int dsmc_apply_pairs(int32_t n_cells, int32_t dtype, dsmc_vec3 v, dsmc_pairs pairs,
                                int32_t kind, int32_t schedule, void* ws, size_t ws_bytes,
                                dsmc_stream_t stream)
{
    int rc = check_pairs("dsmc_apply_pairs", n_cells, v, pairs, dtype, ws, ws_bytes);
    if (rc) return rc;
    if (kind != DSMC_APPLY_DIRECTIONS && kind != DSMC_APPLY_ANGLES)
        return arg_error("dsmc_apply_pairs: kind %d", kind);
    if (schedule < DSMC_SCHED_AUTO || schedule > DSMC_SCHED_WAVE || schedule == DSMC_SCHED_DEFER)
        return arg_error("dsmc_apply_pairs: schedule %d", schedule);
    return phase_b(kind == DSMC_APPLY_ANGLES ? RULE_CHI : RULE_DIR, dtype, n_cells, nullptr, v, pairs,
                   ws, pairs.cap, schedule, as_stream(stream));
}
