// Particle-to-cell binning: stable counting sort by cell id with an SoA
// velocity gather (section "Computational Framework", item 1: particles sorted
// by cell index so that each cell is contiguous in memory).
//
// Pipeline: count (atomics, one per distinct cell per wave) -> exclusive scan
// -> scatter into cell segments (atomic cursors, order within a segment not
// yet fixed) -> per-cell LDS bitonic sort of the original indices, which makes
// the order the stable one regardless of atomic timing -> coalesced gather of
// vx, vy, vz into sorted order.
#include "common.hpp"

namespace dsmc {

constexpr int SMALL_MAX = 1024;   // cells up to this size: one wave, LDS bitonic
constexpr int BIG_MAX = 16384;    // up to this size: one 256-thread block

// Distinct-value aggregation inside a wave: lanes holding the same cell id
// issue a single atomic; returns this lane's rank among equal lanes (in lane
// order) and the old counter value of the group.
__device__ __forceinline__ int wave_aggregated_add(int32_t* counters, int32_t c, bool valid,
                                                   int* rank)
{
    const int lane = threadIdx.x & 63;
    uint64_t pending = __ballot(valid);
    int my_old = 0;
    *rank = 0;
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int32_t lc = __shfl(c, leader, 64);
        const uint64_t same = __ballot(valid && c == lc) & pending;
        int old = 0;
        if (lane == leader) old = atomicAdd(&counters[lc], __popcll(same));
        old = __shfl(old, leader, 64);
        if (valid && c == lc) {
            my_old = old;
            *rank = __popcll(same & ((1ull << lane) - 1ull));
        }
        pending &= ~same;
    }
    return my_old;
}

__global__ void __launch_bounds__(256)
k_count(const int32_t* __restrict__ cell_of, int32_t n, int32_t n_cells, int32_t* counts,
        dsmc_status* st)
{
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = base + threadIdx.x;
        int32_t c = (p < n) ? cell_of[p] : -1;
        const bool bad = (p < n) && (c < 0 || c >= n_cells);
        const bool valid = (p < n) && !bad;
        if (bad && st) {
            atomicAdd(&st->bad_cell, 1);
            atomicOr(&st->flags, (uint32_t)DSMC_ST_BAD_CELL);
        }
        int rank;
        wave_aggregated_add(counts, c, valid, &rank);
    }
}

__global__ void __launch_bounds__(256)
k_scatter(const int32_t* __restrict__ cell_of, int32_t n, int32_t n_cells, int32_t* cursor,
          int32_t* __restrict__ tmp)
{
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = base + threadIdx.x;
        const int32_t c = (p < n) ? cell_of[p] : -1;
        const bool valid = (p < n) && c >= 0 && c < n_cells;
        int rank;
        const int old = wave_aggregated_add(cursor, c, valid, &rank);
        if (valid) tmp[old + rank] = (int32_t)p;
    }
}

__global__ void k_copy_i32(const int32_t* a, int32_t* b, int32_t n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        b[i] = a[i];
}

// Bitonic sort of P (power of two) ints in LDS by `nthreads` threads.
__device__ __forceinline__ void lds_bitonic(int32_t* a, int P, int tid, int nthreads)
{
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int e = tid; e < P; e += nthreads) {
                const int q = e ^ j;
                if (q > e) {
                    const int32_t x = a[e], y = a[q];
                    const bool up = (e & k) == 0;
                    if ((x > y) == up) { a[e] = y; a[q] = x; }
                }
            }
            __syncthreads();
        }
    }
}

template <typename T>
__device__ __forceinline__ void gather_seg(const int32_t* perm, int32_t s0, int32_t s1,
                                           V3<const T> vin, V3<T> vout, int tid, int nthreads)
{
    for (int32_t s = s0 + tid; s < s1; s += nthreads) {
        const int32_t p = perm[s];
        vout.x[s] = vin.x[p];
        vout.y[s] = vin.y[p];
        vout.z[s] = vin.z[p];
    }
}

// One 64-thread block per cell (grid-stride) for cells up to SMALL_MAX.
template <typename T>
__global__ void __launch_bounds__(64)
k_fix_small(const int32_t* __restrict__ cell_start, int32_t n_cells,
            const int32_t* __restrict__ tmp, int32_t* __restrict__ perm, V3<const T> vin,
            V3<T> vout)
{
    __shared__ int32_t a[SMALL_MAX];
    for (int32_t k = blockIdx.x; k < n_cells; k += gridDim.x) {
        const int32_t s0 = cell_start[k], s1 = cell_start[k + 1], N = s1 - s0;
        if (N == 0 || N > SMALL_MAX) continue;
        int P = 1;
        while (P < N) P <<= 1;
        for (int e = threadIdx.x; e < P; e += 64) a[e] = (e < N) ? tmp[s0 + e] : INT32_MAX;
        __syncthreads();
        if (N > 1) lds_bitonic(a, P, threadIdx.x, 64);
        for (int e = threadIdx.x; e < N; e += 64) perm[s0 + e] = a[e];
        __syncthreads();
        gather_seg<T>(perm, s0, s1, vin, vout, threadIdx.x, 64);
    }
}

// One 256-thread block per big cell; cells beyond BIG_MAX use rank counting
// in global memory (correct for any size, quadratic cost).
template <typename T>
__global__ void __launch_bounds__(256)
k_fix_big(const int32_t* __restrict__ cell_start, int32_t n_cells,
          const int32_t* __restrict__ tmp, int32_t* __restrict__ perm, V3<const T> vin,
          V3<T> vout)
{
    __shared__ int32_t a[BIG_MAX];
    for (int32_t k = blockIdx.x; k < n_cells; k += gridDim.x) {
        const int32_t s0 = cell_start[k], s1 = cell_start[k + 1], N = s1 - s0;
        if (N <= SMALL_MAX) continue;
        if (N <= BIG_MAX) {
            int P = 1;
            while (P < N) P <<= 1;
            for (int e = threadIdx.x; e < P; e += 256) a[e] = (e < N) ? tmp[s0 + e] : INT32_MAX;
            __syncthreads();
            lds_bitonic(a, P, threadIdx.x, 256);
            for (int e = threadIdx.x; e < N; e += 256) perm[s0 + e] = a[e];
        } else {
            for (int e = threadIdx.x; e < N; e += 256) {
                const int32_t x = tmp[s0 + e];
                int32_t r = 0;
                for (int32_t f = 0; f < N; ++f) r += (tmp[s0 + f] < x);
                perm[s0 + r] = x;
            }
        }
        __syncthreads();
        gather_seg<T>(perm, s0, s1, vin, vout, threadIdx.x, 256);
        __syncthreads();
    }
}

template <typename T>
static int sort_impl(int32_t n, int32_t n_cells, const int32_t* cell_of, dsmc_vec3 vin,
                     dsmc_vec3 vout, int32_t* cell_start, int32_t* perm, void* ws,
                     dsmc_status* st, hipStream_t s)
{
    uint8_t* w = static_cast<uint8_t*>(ws);
    int32_t* counts = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * ((size_t)n_cells + 1));
    int32_t* cursor = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * ((size_t)n_cells + 1));
    int32_t* tmp = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * ((size_t)n + 1));
    void* scan_ws = w;

    int rc = fill_i32(counts, 0, n_cells, s);
    if (rc) return rc;
    const int pblocks = persistent_blocks(256);
    int blocks = (int)((n + 255) / 256);
    if (blocks > pblocks) blocks = pblocks;
    if (blocks < 1) blocks = 1;
    if (n > 0) {
        k_count<<<blocks, 256, 0, s>>>(cell_of, n, n_cells, counts, st);
        DSMC_LAUNCH_CHECK("sort:count");
    }
    rc = exclusive_scan_i32(counts, cell_start, n_cells, nullptr, scan_ws, s);
    if (rc) return rc;
    if (n == 0) return DSMC_OK;
    k_copy_i32<<<(n_cells + 255) / 256, 256, 0, s>>>(cell_start, cursor, n_cells);
    DSMC_LAUNCH_CHECK("sort:cursor");
    k_scatter<<<blocks, 256, 0, s>>>(cell_of, n, n_cells, cursor, tmp);
    DSMC_LAUNCH_CHECK("sort:scatter");
    const int cb = n_cells < pblocks * 4 ? n_cells : pblocks * 4;
    k_fix_small<T><<<cb > 0 ? cb : 1, 64, 0, s>>>(cell_start, n_cells, tmp, perm,
                                                 v3<const T>(vin), v3<T>(vout));
    DSMC_LAUNCH_CHECK("sort:fix_small");
    k_fix_big<T><<<cb > 1024 ? 1024 : (cb > 0 ? cb : 1), 256, 0, s>>>(
        cell_start, n_cells, tmp, perm, v3<const T>(vin), v3<T>(vout));
    DSMC_LAUNCH_CHECK("sort:fix_big");
    return DSMC_OK;
}

}  // namespace dsmc

using namespace dsmc;

extern "C" size_t dsmc_sort_cells_ws(int32_t n, int32_t n_cells)
{
    if (n < 0 || n_cells < 0) return 0;
    return 2 * align_up(sizeof(int32_t) * ((size_t)n_cells + 1)) +
           align_up(sizeof(int32_t) * ((size_t)n + 1)) + scan_ws_bytes(n_cells) + 256;
}

extern "C" int dsmc_sort_cells(int32_t n, int32_t n_cells, const int32_t* cell_of, int32_t dtype,
                               dsmc_vec3 v_in, dsmc_vec3 v_out, int32_t* cell_start,
                               int32_t* perm, void* ws, size_t ws_bytes, dsmc_status* st,
                               dsmc_stream_t stream)
{
    if (n < 0 || n_cells < 1) return arg_error("dsmc_sort_cells: n=%d n_cells=%d", n, n_cells);
    if (!cell_start || !ws || (n > 0 && (!cell_of || !perm || !v_in.x || !v_in.y || !v_in.z ||
                                         !v_out.x || !v_out.y || !v_out.z)))
        return arg_error("dsmc_sort_cells: null pointer");
    if (v_in.x == v_out.x || v_in.y == v_out.y || v_in.z == v_out.z)
        return arg_error("dsmc_sort_cells: v_in and v_out must be distinct buffers");
    if (ws_bytes < dsmc_sort_cells_ws(n, n_cells))
        return arg_error("dsmc_sort_cells: workspace %zu < %zu", ws_bytes,
                         dsmc_sort_cells_ws(n, n_cells));
    hipStream_t s = as_stream(stream);
    if (dtype == DSMC_F64)
        return sort_impl<double>(n, n_cells, cell_of, v_in, v_out, cell_start, perm, ws, st, s);
    if (dtype == DSMC_F32)
        return sort_impl<float>(n, n_cells, cell_of, v_in, v_out, cell_start, perm, ws, st, s);
    return arg_error("dsmc_sort_cells: dtype %d", dtype);
}
