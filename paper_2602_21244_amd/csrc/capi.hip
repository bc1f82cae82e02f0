// Host plumbing of the library: errors, device selection, status word,
// device-wide scans and fills used by several entry points.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "common.hpp"

namespace dsmc {

static thread_local char g_err[512] = "";
static int32_t g_block_threshold = 48;
static dsmc_match_schedule g_match_schedule = {40, 2, 1, 0};

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int arg_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return DSMC_E_ARG;
}

int hip_check(hipError_t e, const char* what)
{
    if (e == hipSuccess) return DSMC_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return DSMC_E_HIP;
}

// Compute units of the current device (queried once per device).
int device_cus()
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

int persistent_blocks(int threads_per_block)
{
    const int cus = device_cus();
    const int waves_per_block = (threads_per_block + 63) / 64;
    return cus * (32 / waves_per_block > 0 ? 32 / waves_per_block : 1);
}

int32_t block_threshold() { return g_block_threshold; }
dsmc_match_schedule match_schedule() { return g_match_schedule; }

// --------------------------------------------------------------------------
// Fills
// --------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_bytes(uint8_t* p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

int fill_i32(int32_t* p, int32_t value, int64_t n, hipStream_t s)
{
    if (n <= 0) return DSMC_OK;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    k_fill_i32<<<blocks, 256, 0, s>>>(p, value, n);
    DSMC_LAUNCH_CHECK("fill_i32");
    return DSMC_OK;
}

int fill_bytes_zero(void* p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return DSMC_OK;
    int blocks = (int)((bytes + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    k_zero_bytes<<<blocks, 256, 0, s>>>(static_cast<uint8_t*>(p), bytes);
    DSMC_LAUNCH_CHECK("fill_bytes_zero");
    return DSMC_OK;
}

// --------------------------------------------------------------------------
// Device-wide exclusive scan (reduce tiles, scan tile sums, scan tiles).
// --------------------------------------------------------------------------
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Exclusive scan of one int per thread over a 256-thread block; returns the
// exclusive prefix, *total gets the block sum.
__device__ __forceinline__ int block_excl_scan(int x, int* total)
{
    __shared__ int wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / 64; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + inc - x;
}

__device__ __forceinline__ int64_t scan_n(int64_t n, const int64_t* n_dev, int64_t n_max)
{
    if (n_dev) {
        int64_t v = *n_dev;
        return v < 0 ? 0 : (v > n_max ? n_max : v);
    }
    return n;
}

__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_reduce(const int32_t* in, int64_t n, const int64_t* n_dev, int32_t* tile_sums)
{
    n = scan_n(n, n_dev, n);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int s = 0;
    if (base < n) {
        for (int q = 0; q < SCAN_ITEMS; ++q) {
            const int64_t i = base + (int64_t)q * SCAN_THREADS + threadIdx.x;
            if (i < n) s += in[i];
        }
    }
    int tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_tiles(int32_t* tile_sums, int64_t n_tiles)
{
    int carry = 0;
    for (int64_t b = 0; b < n_tiles; b += SCAN_THREADS) {
        const int64_t i = b + threadIdx.x;
        const int x = (i < n_tiles) ? tile_sums[i] : 0;
        int tot;
        const int ex = block_excl_scan(x, &tot);
        if (i < n_tiles) tile_sums[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sums[n_tiles] = carry;
}

__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_down(const int32_t* in, int32_t* out, int64_t n, const int64_t* n_dev, int64_t n_max,
            const int32_t* tile_off, int64_t n_tiles, int64_t* total64)
{
    n = scan_n(n, n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        out[n] = tile_off[n_tiles];
        if (total64) *total64 = tile_off[n_tiles];
    }
    if (base >= n) return;
    // blocked arrangement: thread t owns items [t*ITEMS, (t+1)*ITEMS)
    int v[SCAN_ITEMS];
    int s = 0;
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + q;
        v[q] = (i < n) ? in[i] : 0;
        s += v[q];
    }
    int tot;
    int run = block_excl_scan(s, &tot) + tile_off[blockIdx.x];
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + q;
        if (i < n) out[i] = run;
        run += v[q];
    }
}

size_t scan_ws_bytes(int64_t n)
{
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    return align_up(sizeof(int32_t) * (size_t)(tiles + 1));
}

static int scan_impl(const int32_t* in, int32_t* out, int64_t n, const int64_t* n_dev,
                     int64_t n_max, int64_t* total64, void* ws, hipStream_t s)
{
    const int64_t n_cap = n_dev ? n_max : n;
    const int64_t tiles = (n_cap + SCAN_TILE - 1) / SCAN_TILE;
    int32_t* tile = static_cast<int32_t*>(ws);
    const int grid = (int)(tiles > 0 ? tiles : 1);
    // reduce: tiles beyond the device count contribute 0
    k_scan_reduce<<<grid, SCAN_THREADS, 0, s>>>(in, n_cap, n_dev, tile);
    DSMC_LAUNCH_CHECK("scan_reduce");
    k_scan_tiles<<<1, SCAN_THREADS, 0, s>>>(tile, grid);
    DSMC_LAUNCH_CHECK("scan_tiles");
    k_scan_down<<<grid, SCAN_THREADS, 0, s>>>(in, out, n_cap, n_dev, n_max, tile, grid,
                                              total64);
    DSMC_LAUNCH_CHECK("scan_down");
    return DSMC_OK;
}

int exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int64_t* total64, void* ws,
                       hipStream_t s)
{
    return scan_impl(in, out, n, nullptr, n, total64, ws, s);
}

int exclusive_scan_i32_dev(const int32_t* in, int32_t* out, const int64_t* n_dev, int64_t n_max,
                           void* ws, hipStream_t s)
{
    return scan_impl(in, out, n_max, n_dev, n_max, nullptr, ws, s);
}

}  // namespace dsmc

using namespace dsmc;

extern "C" {

int dsmc_init(int device)
{
    if (device < 0) return arg_error("dsmc_init: device %d < 0", device);
    return hip_check(hipSetDevice(device), "hipSetDevice");
}

const char* dsmc_last_error(void) { return g_err; }

const char* dsmc_version(void) { return "dsmc-gfx950 0.1"; }

int dsmc_status_clear(dsmc_status* st, dsmc_stream_t stream)
{
    if (!st) return arg_error("dsmc_status_clear: null status");
    return fill_bytes_zero(st, sizeof(dsmc_status), as_stream(stream));
}

int dsmc_set_block_threshold(int32_t pairs)
{
    if (pairs < 1) return arg_error("dsmc_set_block_threshold: %d < 1", pairs);
    g_block_threshold = pairs;
    return DSMC_OK;
}

int32_t dsmc_get_block_threshold(void) { return g_block_threshold; }

int dsmc_set_match_schedule(const dsmc_match_schedule* ms)
{
    if (!ms) return arg_error("dsmc_set_match_schedule: null");
    if (ms->wave_per_cu < 1 || ms->wave_per_cu > 256 || ms->medium_per_cu < 1 ||
        ms->medium_per_cu > 64 || ms->big_per_cu < 1 || ms->big_per_cu > 64)
        return arg_error("dsmc_set_match_schedule: %d/%d/%d workgroups per CU out of range",
                         ms->wave_per_cu, ms->medium_per_cu, ms->big_per_cu);
    g_match_schedule = *ms;
    g_match_schedule.reserved = 0;
    return DSMC_OK;
}

int dsmc_get_match_schedule(dsmc_match_schedule* ms)
{
    if (!ms) return arg_error("dsmc_get_match_schedule: null");
    *ms = g_match_schedule;
    return DSMC_OK;
}

}  // extern "C"
