// One persistent launch per collision step for the isotropic rule: each
// workgroup takes cells from a work queue (an atomic counter, so cells of any
// population balance across the grid), stages the cell's velocities in LDS
// and runs moments, NTC selection, Phase A, Phase B (dependency rounds) and
// moment matching without touching HBM again.  The launch runs with one wave
// per workgroup and small LDS tables, so many cells of a few hundred
// particles are in flight on every CU; cells larger than those tables are
// listed and taken by a second, block-wide launch with tables for up to 3072
// particles.  HBM traffic is one read and one
// write of the velocities per step.  The arithmetic (including the order of
// every reduction) is that of the separate entry points, so the results are
// bit-identical to dsmc_moment_match(CAPTURE) -> dsmc_select_pairs_ntc ->
// dsmc_collide_vhs -> dsmc_moment_match(APPLY).  A cell with more accepted
// pairs than LDS holds is applied in batches, in candidate order: the pairs
// gathered so far get Phase A and Phase B before the next candidates are
// decided, which then read the pre-step velocities from global memory (not
// written until the cell's write-back).
#include <limits.h>
#include <math.h>

#include "collide.hpp"

namespace dsmc {

int xs_law_public(const dsmc_xs& xs, double* C, double* e);

// Wave form: particles of a cell staged in LDS, accepted pairs of one LDS
// batch.  Block form: the same for the listed (larger) cells.
constexpr int FW_THREADS = 64, FW_NMAX = 320, FW_MMAX = 256;
constexpr int FS_THREADS = 256, FS_NMAX = 3072, FS_MMAX = 2048;

struct FusedArgs {
    int32_t n_cells;
    const int32_t* cell_start;
    const double* lambda;
    double C, e;
    dsmc_rng rng;
    int32_t match;
    int32_t* pair_cnt;
    int32_t* queue;     // [0]: wave-form queue, [1]: block-form queue, [2]: listed cells
    int32_t* big;       // cells listed for the block form
    dsmc_status* st;
};

// Same reduction order as the wave-per-cell moments kernel: lane-strided
// partial sums, then a butterfly over the 64 lanes (wave 0 only).
__device__ __forceinline__ void wave0_sums(const double* vx, const double* vy, const double* vz,
                                           int32_t N, int lane, double* out6)
{
    double sx = 0, sy = 0, sz = 0;
    for (int32_t q = lane; q < N; q += 64) { sx += vx[q]; sy += vy[q]; sz += vz[q]; }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    sz = wave_sum(sz);
    const double ux = sx / N, uy = sy / N, uz = sz / N;
    double S = 0, c2max = 0, E = 0;
    for (int32_t q = lane; q < N; q += 64) {
        const double x = vx[q], y = vy[q], z = vz[q];
        const double dx = x - ux, dy = y - uy, dz = z - uz;
        const double c2 = dx * dx + dy * dy + dz * dz;
        S += c2;
        c2max = fmax(c2max, c2);
        E += x * x + y * y + z * z;
    }
    out6[0] = ux; out6[1] = uy; out6[2] = uz;
    out6[3] = wave_sum(S);
    out6[4] = sqrt(wave_max(c2max));
    out6[5] = wave_sum(E);
}

// LISTED = false: every cell from the queue, cells above NMAX particles go to
// the list; LISTED = true: the listed cells, those above NMAX are left alone.
template <typename T, int NT, int NMAX, int MMAX, bool LISTED>
__global__ void __launch_bounds__(NT)
k_step_vhs_fused(FusedArgs A, V3<T> v)
{
    __shared__ double lvx[NMAX], lvy[NMAX], lvz[NMAX];
    __shared__ uint32_t lpair[MMAX];
    __shared__ T ldir[3][MMAX];
    __shared__ int32_t first[NMAX];
    __shared__ double mom[6], post[6];
    __shared__ int32_t s_cell, s_M, s_acc, s_remaining, s_base;
    __shared__ int32_t wtot[NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

    for (;;) {
        if (tid == 0) {
            if (LISTED) {
                const int32_t idx = atomicAdd(&A.queue[1], 1);
                s_cell = idx < A.queue[2] ? A.big[idx] : INT32_MAX;
            } else {
                s_cell = atomicAdd(&A.queue[0], 1);
            }
        }
        __syncthreads();
        const int32_t k = s_cell;
        if (k >= A.n_cells) break;
        const int32_t s0 = A.cell_start[k], N = A.cell_start[k + 1] - s0;
        if (N < 2 || N > NMAX) {
            if (tid == 0) {
                if (N < 2) {
                    A.pair_cnt[k] = 0;
                } else if (!LISTED) {
                    A.big[atomicAdd(&A.queue[2], 1)] = k;
                } else {
                    A.pair_cnt[k] = -1;
                    if (A.st) atomicOr(&A.st->flags, (uint32_t)DSMC_ST_PAIR_OVERFLOW);
                }
            }
            __syncthreads();
            continue;
        }
        for (int32_t q = tid; q < N; q += NT) {
            lvx[q] = (double)v.x[s0 + q];
            lvy[q] = (double)v.y[s0 + q];
            lvz[q] = (double)v.z[s0 + q];
        }
        __syncthreads();
        if (wid == 0) {
            double m6[6];
            wave0_sums(lvx, lvy, lvz, N, lane, m6);
            if (lane == 0) {
                for (int q = 0; q < 6; ++q) mom[q] = m6[q];
                // candidate count: same arithmetic as the selection kernel
                const double ghat = 2.0 * m6[4];
                const double sgmax = A.C * pow(ghat, A.e);
                const U4 r = draw(A.rng, 0u, (uint32_t)k, SLOT_COUNT);
                const double U = unif53(r.a, r.b);
                double x = __dmul_rn(0.5, (double)N);
                x = __dmul_rn(x, (double)(N - 1));
                x = __dmul_rn(x, A.lambda[k]);
                x = __dmul_rn(x, sgmax);
                x = __dadd_rn(x, U);
                s_M = (!(x >= 0.0) || !(x < 2147483647.0)) ? 0 : (int32_t)floor(x);
                s_acc = 0;
            }
        }
        __syncthreads();
        const int32_t M = s_M;
        const double ghat = 2.0 * mom[4];
        if (tid == 0) s_base = 0;
        __syncthreads();
        // Pre-step velocity of slot i: LDS until the first batch of pairs has
        // been applied there, then global memory, which keeps the pre-step
        // values until the write-back (the same numbers either way).
        auto pre = [&](int32_t i, double& x, double& y, double& z) {
            if (s_base == 0) {
                x = lvx[i]; y = lvy[i]; z = lvz[i];
            } else {
                x = (double)v.x[s0 + i]; y = (double)v.y[s0 + i]; z = (double)v.z[s0 + i];
            }
        };
        // Phase A and Phase B of the s_acc pairs gathered in lpair (accepted
        // pairs s_base .. s_base + s_acc - 1 of the cell, in candidate order)
        auto flush = [&]() {
            const int32_t nb = s_acc, b0 = s_base;
            // Phase A on the pre-collision velocities (arithmetic in T, as
            // the separate isotropic kernel)
            for (int32_t q = tid; q < nb; q += NT) {
                T xi[3], z[2], u4;
                pair_latents(A.rng, (uint32_t)(b0 + q), (uint32_t)k, xi, z, u4);
                const int32_t i = lpair[q] & 0xffff, j = lpair[q] >> 16;
                double xa, ya, za, xb, yb, zb;
                pre(i, xa, ya, za);
                pre(j, xb, yb, zb);
                T vh[3], e[3];
                unit3<T>((T)xa - (T)xb, (T)ya - (T)yb, (T)za - (T)zb, vh);
                const T cc = T(2) * u4 - T(1);
                const T sc = T(2) * dev_sqrt<T>(u4 * (T(1) - u4));
                perp_dir<T>(xi, vh, e);
                ldir[0][q] = cc * vh[0] + sc * e[0];
                ldir[1][q] = cc * vh[1] + sc * e[1];
                ldir[2][q] = cc * vh[2] + sc * e[2];
            }
            if (tid == 0) s_remaining = nb;
            __syncthreads();
            // Phase B: dependency rounds, every value rounded to T as stored
            while (s_remaining > 0) {
                for (int32_t q = tid; q < N; q += NT) first[q] = INT32_MAX;
                __syncthreads();
                for (int32_t q = tid; q < nb; q += NT) {
                    const uint32_t w = lpair[q];
                    if (w != 0xffffffffu) {
                        atomicMin(&first[w & 0xffff], q);
                        atomicMin(&first[w >> 16], q);
                    }
                }
                __syncthreads();
                int done_here = 0;
                for (int32_t q = tid; q < nb; q += NT) {
                    const uint32_t w = lpair[q];
                    if (w == 0xffffffffu) continue;
                    const int32_t a = w & 0xffff, b = w >> 16;
                    if (first[a] != q || first[b] != q) continue;
                    const double xa = lvx[a], ya = lvy[a], za = lvz[a];
                    const double xb = lvx[b], yb = lvy[b], zb = lvz[b];
                    const double rx = xa - xb, ry = ya - yb, rz = za - zb;
                    const double g = sqrt(rx * rx + ry * ry + rz * rz);
                    const double a0 = ldir[0][q], a1 = ldir[1][q], a2 = ldir[2][q];
                    const double inv = 1.0 / sqrt(a0 * a0 + a1 * a1 + a2 * a2);
                    const double u0 = a0 * inv, u1 = a1 * inv, u2 = a2 * inv;
                    const double cx = 0.5 * (xa + xb), cy = 0.5 * (ya + yb), cz = 0.5 * (za + zb);
                    const double px = 0.5 * g * u0, py = 0.5 * g * u1, pz = 0.5 * g * u2;
                    lvx[a] = (double)(T)(cx + px); lvy[a] = (double)(T)(cy + py); lvz[a] = (double)(T)(cz + pz);
                    lvx[b] = (double)(T)(cx - px); lvy[b] = (double)(T)(cy - py); lvz[b] = (double)(T)(cz - pz);
                    lpair[q] = 0xffffffffu;
                    ++done_here;
                }
                __syncthreads();
                if (done_here) atomicSub(&s_remaining, done_here);
                __syncthreads();
            }
            if (tid == 0) {
                s_base = b0 + nb;
                s_acc = 0;
            }
            __syncthreads();
        };
        // candidates in blocks of NT; ordered compaction of the
        // accepted ones into lpair, flushed before a block could overflow it
        for (int32_t base = 0; base < M; base += NT) {
            if (s_acc + NT > MMAX) flush();
            const int32_t t = base + tid;
            bool acc = false;
            uint32_t packed = 0;
            if (t < M) {
                const U4 r = draw(A.rng, (uint32_t)t, (uint32_t)k, SLOT_CAND);
                int32_t i = (int32_t)(((uint64_t)r.a * (uint64_t)N) >> 32);
                int32_t j = (int32_t)(((uint64_t)r.b * (uint64_t)(N - 1)) >> 32);
                if (j >= i) j += 1;
                const double U = unif53(r.c, r.d);
                double xa, ya, za, xb, yb, zb;
                pre(i, xa, ya, za);
                pre(j, xb, yb, zb);
                const double dx = xa - xb, dy = ya - yb, dz = za - zb;
                const double g2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                            __dmul_rn(dz, dz));
                const double ratio = sqrt(g2) / ghat;
                const double p = (A.e == 1.0) ? ratio : pow(ratio, A.e);
                acc = U < p;
                packed = (uint32_t)i | ((uint32_t)j << 16);
            }
            const uint64_t bal = __ballot(acc);
            const int before = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) wtot[wid] = __popcll(bal);
            __syncthreads();
            int off = s_acc;
            for (int w = 0; w < wid; ++w) off += wtot[w];
            if (acc) lpair[off + before] = packed;
            __syncthreads();
            if (tid == 0) {
                int tot = 0;
                for (int w = 0; w < NT / 64; ++w) tot += wtot[w];
                s_acc += tot;
            }
            __syncthreads();
        }
        if (s_acc > 0) flush();
        const int32_t na = s_base;
        // moment matching (centred), same arithmetic as the separate kernel
        bool write_raw = true;
        if (A.match && na > 0) {
            if (wid == 0) {
                double m6[6];
                wave0_sums(lvx, lvy, lvz, N, lane, m6);
                if (lane == 0)
                    for (int q = 0; q < 6; ++q) post[q] = m6[q];
            }
            __syncthreads();
            const double Sp = post[3];
            if (!(Sp > 0.0) || !isfinite(Sp)) {
                if (tid == 0 && A.st) atomicAdd(&A.st->mm_skipped, 1);
            } else {
                const double alpha = sqrt(mom[3] / Sp);
                for (int32_t q = tid; q < N; q += NT) {
                    v.x[s0 + q] = (T)(mom[0] + alpha * (lvx[q] - post[0]));
                    v.y[s0 + q] = (T)(mom[1] + alpha * (lvy[q] - post[1]));
                    v.z[s0 + q] = (T)(mom[2] + alpha * (lvz[q] - post[2]));
                }
                write_raw = false;
            }
        }
        if (write_raw) {
            for (int32_t q = tid; q < N; q += NT) {
                v.x[s0 + q] = (T)lvx[q];
                v.y[s0 + q] = (T)lvy[q];
                v.z[s0 + q] = (T)lvz[q];
            }
        }
        if (tid == 0) A.pair_cnt[k] = na;
        __syncthreads();
    }
}

}  // namespace dsmc

using namespace dsmc;

extern "C" size_t dsmc_step_vhs_ws(int32_t n_cells, int64_t cap)
{
    (void)cap;
    if (n_cells < 1) return 0;
    return 256 + align_up(sizeof(int32_t) * (size_t)n_cells);
}

extern "C" int dsmc_step_vhs_fused(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                                   dsmc_vec3 v, dsmc_xs xs, const double* lambda, dsmc_rng rng,
                                   int32_t match, int32_t* pair_cnt, void* ws, size_t ws_bytes,
                                   dsmc_status* st, dsmc_stream_t stream)
{
    if (n_cells < 1) return arg_error("dsmc_step_vhs_fused: n_cells=%d", n_cells);
    if (!cell_start || !lambda || !pair_cnt || !ws || !v.x || !v.y || !v.z)
        return arg_error("dsmc_step_vhs_fused: null pointer");
    if (ws_bytes < dsmc_step_vhs_ws(n_cells, 0))
        return arg_error("dsmc_step_vhs_fused: workspace too small");
    FusedArgs A;
    int rc = xs_law_public(xs, &A.C, &A.e);
    if (rc) return rc;
    A.n_cells = n_cells;
    A.cell_start = cell_start;
    A.lambda = lambda;
    A.rng = rng;
    A.match = match;
    A.pair_cnt = pair_cnt;
    A.queue = static_cast<int32_t*>(ws);
    A.big = reinterpret_cast<int32_t*>(static_cast<uint8_t*>(ws) + 256);
    A.st = st;
    if (dtype != DSMC_F64 && dtype != DSMC_F32)
        return arg_error("dsmc_step_vhs_fused: dtype %d", dtype);
    hipStream_t s = as_stream(stream);
    rc = fill_i32(A.queue, 0, 3, s);
    if (rc) return rc;
    // wave form: as many one-wave workgroups as the LDS tables let stay
    // resident (a dozen per CU); block form: one workgroup per CU
    const int cus = device_cus();
    int wb = cus * 12, bb = cus;
    if (wb > n_cells) wb = n_cells;
    if (bb > n_cells) bb = n_cells;
    if (dtype == DSMC_F64) {
        k_step_vhs_fused<double, FW_THREADS, FW_NMAX, FW_MMAX, false>
            <<<wb, FW_THREADS, 0, s>>>(A, v3<double>(v));
        DSMC_LAUNCH_CHECK("step_vhs_fused:wave");
        k_step_vhs_fused<double, FS_THREADS, FS_NMAX, FS_MMAX, true>
            <<<bb, FS_THREADS, 0, s>>>(A, v3<double>(v));
    } else {
        k_step_vhs_fused<float, FW_THREADS, FW_NMAX, FW_MMAX, false>
            <<<wb, FW_THREADS, 0, s>>>(A, v3<float>(v));
        DSMC_LAUNCH_CHECK("step_vhs_fused:wave");
        k_step_vhs_fused<float, FS_THREADS, FS_NMAX, FS_MMAX, true>
            <<<bb, FS_THREADS, 0, s>>>(A, v3<float>(v));
    }
    DSMC_LAUNCH_CHECK("step_vhs_fused:block");
    return DSMC_OK;
}
