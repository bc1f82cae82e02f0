// Particle-to-cell binning: stable sort by cell id with an SoA velocity
// gather (section "Computational Framework", item 1: particles sorted by cell
// index so that each cell is contiguous in memory).
//
// Least-significant-digit radix sort of the cell ids, 9 bits per pass (two
// passes for up to 2^18 - 1 cells).  Every pass is stable, so the result is
// the stable order (original order inside a cell) whatever the input order
// and without atomics on the particle data:
//   up    : per 4096-particle tile, a 512-bucket digit histogram (LDS
//           atomics), stored tile-major so every store is a row segment
//   scan  : offsets of the (tile, digit) table in digit-major order by three
//           small kernels over chunks of tiles (column sums, a scan of those
//           per digit, expansion of the chunk rows)
//   down  : 512 threads per tile; each wave ranks its 512 particles in index
//           order (digit groups split off by ballots, per-wave digit
//           counters in LDS), the tile is reordered by digit through one LDS
//           array (keys, then values) and written out as contiguous digit
//           runs
// The last down pass also gathers vx, vy, vz into sorted order and adds the
// cell counts (its tiles are sorted by the whole key, so a few integer
// atomics per tile); an in-place exclusive scan of the counts gives
// cell_start.
// Ids outside [0, n_cells) are mapped to the key n_cells, so they sort after
// every kept particle.
#include <mutex>

#include "common.hpp"

namespace dsmc {

constexpr int RADIX_BITS = 9;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;   // 4096
// down kernel: same tile, DN_THREADS threads of DN_ITEMS particles
constexpr int DN_THREADS = 512;
constexpr int DN_ITEMS = SORT_TILE / DN_THREADS;
constexpr int DN_WAVES = DN_THREADS / 64;
constexpr int DN_DPT = RADIX / DN_THREADS;               // digits owned per thread
constexpr int WAVE_SPAN = 64 * DN_ITEMS;                // particles per wave

__device__ __forceinline__ int32_t sort_key(const int32_t* cell_of, int64_t p, int32_t n_cells)
{
    const int32_t c = cell_of[p];
    return (c < 0 || c >= n_cells) ? n_cells : c;
}

// Digit histogram of one tile: each thread counts 16 consecutive keys
// (16-byte loads) and adds runs of equal digits with one LDS atomic each, so
// the cell-sorted-with-movers order typical after streaming costs a few
// atomics per thread.  The first pass reads cell_of, maps bad ids and counts
// them in the status word.
template <bool FIRST>
__global__ void __launch_bounds__(SORT_THREADS)
k_radix_up(const int32_t* __restrict__ keys_in, int32_t n, int32_t n_cells, int shift,
           int32_t mask, int32_t* __restrict__ ghist, dsmc_status* st)
{
    __shared__ int32_t h[RADIX];
    for (int i = threadIdx.x; i <= mask; i += SORT_THREADS) h[i] = 0;
    __syncthreads();
    const int64_t p0 = (int64_t)blockIdx.x * SORT_TILE + (int64_t)threadIdx.x * SORT_ITEMS;
    int32_t key[SORT_ITEMS];
    const bool full = p0 + SORT_ITEMS <= n;
    if (full && ((reinterpret_cast<uintptr_t>(keys_in + p0) & 15) == 0)) {
        const int4* src = reinterpret_cast<const int4*>(keys_in + p0);
#pragma unroll
        for (int q = 0; q < SORT_ITEMS / 4; ++q) {
            const int4 x = src[q];
            key[4 * q] = x.x; key[4 * q + 1] = x.y; key[4 * q + 2] = x.z; key[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < SORT_ITEMS; ++q) key[q] = (p0 + q < n) ? keys_in[p0 + q] : -1;
    }
    int bad = 0;
    int32_t run_d = -1, run_n = 0;
#pragma unroll
    for (int q = 0; q < SORT_ITEMS; ++q) {
        if (p0 + q >= n) break;
        int32_t kk = key[q];
        if (FIRST && (kk < 0 || kk >= n_cells)) {
            kk = n_cells;
            ++bad;
        }
        const int32_t d = (kk >> shift) & mask;
        if (d == run_d) {
            ++run_n;
        } else {
            if (run_n) atomicAdd(&h[run_d], run_n);
            run_d = d;
            run_n = 1;
        }
    }
    if (run_n) atomicAdd(&h[run_d], run_n);
    if (FIRST && st) {
        const int wbad = wave_sum_i(bad);
        if ((threadIdx.x & 63) == 0 && wbad > 0) {
            atomicAdd(&st->bad_cell, wbad);
            atomicOr(&st->flags, (uint32_t)DSMC_ST_BAD_CELL);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= mask; i += SORT_THREADS)
        ghist[(int64_t)blockIdx.x * (mask + 1) + i] = h[i];
}

// Exclusive scan of RADIX values in LDS by the 256 threads (two per thread).
__device__ __forceinline__ void block_scan_radix(const int32_t* tot, int32_t* ex)
{
    __shared__ int32_t wsum[SORT_THREADS / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int32_t a = tot[2 * t], b = tot[2 * t + 1];
    int32_t x = a + b;
    // inclusive wave scan
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int32_t before = 0;
    for (int q = 0; q < w; ++q) before += wsum[q];
    const int32_t excl = before + x - (a + b);
    ex[2 * t] = excl;
    ex[2 * t + 1] = excl + a;
}

// Offsets of the tile-major (tile, digit) count table H[nblk][R]:
//   O[b][d] = sum_{d' < d} T[d'] + sum_{b' < b} H[b'][d],  T[d] = sum_b H[b][d]
// in three small kernels over chunks of HCHUNK tiles (rows), every access a
// coalesced row segment: chunk column sums, an exclusive scan of those over
// the chunks per digit (with the digit totals), and the expansion of each
// chunk's rows.
constexpr int HCHUNK = 32;
constexpr int HSEG = 16;        // chunk segments per digit in the chunk scan
constexpr int HDIG = 256 / HSEG;

__global__ void __launch_bounds__(256)
k_hist_chunk_sum(const int32_t* __restrict__ h, int32_t nblk, int32_t R, int32_t* __restrict__ csum)
{
    const int64_t b0 = (int64_t)blockIdx.x * HCHUNK;
    const int nb = (int)((nblk - b0) < HCHUNK ? (nblk - b0) : HCHUNK);
    for (int d = threadIdx.x; d < R; d += 256) {
        int32_t v[HCHUNK];
#pragma unroll
        for (int r = 0; r < HCHUNK; ++r) v[r] = r < nb ? h[(b0 + r) * R + d] : 0;
        int32_t s = 0;
#pragma unroll
        for (int r = 0; r < HCHUNK; ++r) s += v[r];
        csum[(int64_t)blockIdx.x * R + d] = s;
    }
}

// One workgroup per HDIG digits; HSEG threads per digit split the chunks.
__global__ void __launch_bounds__(256)
k_hist_chunk_scan(const int32_t* __restrict__ csum, int32_t nch, int32_t R,
                  int32_t* __restrict__ cpre, int32_t* __restrict__ tot)
{
    __shared__ int32_t seg[HSEG][HDIG];
    const int dl = threadIdx.x % HDIG, g = threadIdx.x / HDIG;
    const int d = blockIdx.x * HDIG + dl;
    const int per = (nch + HSEG - 1) / HSEG;
    const int c0 = g * per, c1 = (c0 + per) < nch ? (c0 + per) : nch;
    int32_t s = 0;
    if (d < R) {
#pragma unroll 8
        for (int c = c0; c < c1; ++c) s += csum[(int64_t)c * R + d];
    }
    seg[g][dl] = s;
    __syncthreads();
    int32_t run = 0, all = 0;
#pragma unroll
    for (int q = 0; q < HSEG; ++q) {
        const int32_t x = seg[q][dl];
        run += q < g ? x : 0;
        all += x;
    }
    if (d < R) {
#pragma unroll 8
        for (int c = c0; c < c1; ++c) {
            const int32_t x = csum[(int64_t)c * R + d];
            cpre[(int64_t)c * R + d] = run;
            run += x;
        }
        if (g == 0) tot[d] = all;
    }
}

__global__ void __launch_bounds__(256)
k_hist_expand(const int32_t* __restrict__ h, const int32_t* __restrict__ cpre,
              const int32_t* __restrict__ tot, int32_t nblk, int32_t R, int32_t* __restrict__ goff)
{
    __shared__ int32_t t_s[RADIX];
    __shared__ int32_t e_s[RADIX];
    for (int d = threadIdx.x; d < RADIX; d += 256) t_s[d] = d < R ? tot[d] : 0;
    __syncthreads();
    block_scan_radix(t_s, e_s);
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * HCHUNK;
    const int nb = (int)((nblk - b0) < HCHUNK ? (nblk - b0) : HCHUNK);
    for (int d = threadIdx.x; d < R; d += 256) {
        int32_t v[HCHUNK];
#pragma unroll
        for (int r = 0; r < HCHUNK; ++r) v[r] = r < nb ? h[(b0 + r) * R + d] : 0;
        int32_t run = e_s[d] + cpre[(int64_t)blockIdx.x * R + d];
#pragma unroll
        for (int r = 0; r < HCHUNK; ++r) {
            if (r < nb) goff[(b0 + r) * R + d] = run;
            run += v[r];
        }
    }
}

constexpr int PEEL = 4;   // digit groups split off one at a time before the bit match

// Rank of this lane's item among the wave's valid items with the same digit
// (lanes in index order), and the size of that group.  Groups are split off
// by the digit of their lowest lane, at most PEEL times (input close to
// sorted has few distinct digits per wave); lanes left after that are
// matched bit by bit among themselves.
__device__ __forceinline__ void wave_rank(int32_t d, bool valid, int dbits, int lane,
                                          int32_t& before, int32_t& count)
{
    uint64_t todo = __ballot(valid);
    before = 0;
    count = 0;
    for (int it = 0; it < PEEL && todo; ++it) {
        const int leader = __builtin_ctzll(todo);
        const int32_t dl = __builtin_amdgcn_readlane(d, leader);
        const uint64_t grp = __ballot(d == dl) & todo;
        if ((grp >> lane) & 1) {
            before = (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(grp >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)grp, 0u));
            count = __popcll(grp);
        }
        todo &= ~grp;
    }
    if (todo) {
        uint64_t same = todo;
        for (int b = 0; b < dbits; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t ones = __ballot(bit);
            same &= bit ? ones : ~ones;
        }
        if ((todo >> lane) & 1) {
            before = (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0u));
            count = __popcll(same);
        }
    }
}

// Cell counts from the last pass: its tile is sorted by the whole key, so a
// wave's 64 consecutive slots hold a few runs of equal ids; the first lane of
// each run adds the run length (integer atomics: the counts do not depend on
// their order).  Dropped particles (key n_cells) are not counted.
__device__ __forceinline__ void count_runs(int32_t k, bool ok, int s, int32_t tn, int lane,
                                           int32_t* counts, int32_t n_cells)
{
    const int32_t kp = __shfl_up(k, 1, 64);
    const bool start = ok && (lane == 0 || kp != k);
    const uint64_t starts = __ballot(start);
    if (start && k < n_cells) {
        const uint64_t after = starts & ~((2ull << lane) - 1ull);
        int end = after ? __builtin_ctzll(after) : 64;
        const int nvalid = tn - (s - lane);
        if (end > nvalid) end = nvalid;
        atomicAdd(&counts[k], end - lane);
    }
}

// LAST: the final pass also gathers the velocities into sorted order
// (vals are then the original indices, i.e. perm).
template <bool FIRST, bool LAST, typename T>
__global__ void __launch_bounds__(DN_THREADS, 8)
k_radix_down(const int32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in, int32_t n,
             int32_t n_cells, int shift, int32_t mask, int dbits,
             const int32_t* __restrict__ goff, int32_t* __restrict__ keys_out,
             int32_t* __restrict__ vals_out, V3<const T> vin, V3<T> vout,
             int32_t* __restrict__ counts)
{
    __shared__ int32_t cnt[DN_WAVES][RADIX];   // per wave and digit
    __shared__ int32_t gb[RADIX];                       // global slot of tile slot 0, per digit
    __shared__ int32_t wsum[DN_WAVES];
    __shared__ int32_t stage[SORT_TILE];               // keys, then values, in tile order

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < DN_WAVES * RADIX; i += DN_THREADS)
        (&cnt[0][0])[i] = 0;
    // this tile's global digit offsets (digits 2t, 2t+1), loaded early
    int32_t g[DN_DPT];
#pragma unroll
    for (int e = 0; e < DN_DPT; ++e) {
        const int d = DN_DPT * threadIdx.x + e;
        g[e] = d <= mask ? goff[(int64_t)blockIdx.x * (mask + 1) + d] : 0;
    }
    __syncthreads();

    const int64_t tbase = (int64_t)blockIdx.x * SORT_TILE;
    const int32_t tn = (int32_t)(((int64_t)n - tbase) < SORT_TILE ? ((int64_t)n - tbase) : SORT_TILE);
    const int32_t* kt = keys_in + tbase;
    const int32_t* vt = FIRST ? nullptr : vals_in + tbase;
    const int woff = w * WAVE_SPAN;
    int32_t key[DN_ITEMS], val[DN_ITEMS], rank[DN_ITEMS];
    // all loads of the wave's 1024 items first (independent, coalesced)
#pragma unroll
    for (int it = 0; it < DN_ITEMS; ++it) {
        const int q = woff + it * 64 + lane;
        key[it] = 0;
        val[it] = 0;
        if (q < tn) {
            if (FIRST) {
                const int32_t c = kt[q];
                key[it] = (c < 0 || c >= n_cells) ? n_cells : c;
                val[it] = (int32_t)(tbase + q);
            } else {
                key[it] = kt[q];
                val[it] = vt[q];
            }
        }
    }
#pragma unroll
    for (int it = 0; it < DN_ITEMS; ++it) {
        const bool valid = woff + it * 64 + lane < tn;
        const int32_t d = (key[it] >> shift) & mask;
        int32_t before, count;
        wave_rank(d, valid, dbits, lane, before, count);
        const int32_t old = cnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid && before == 0) cnt[w][d] = old + count;
        __builtin_amdgcn_wave_barrier();
        rank[it] = valid ? old + before : -1;
    }
    __syncthreads();
    // thread t owns digits DN_DPT t .. DN_DPT t + DN_DPT - 1: exclusive over
    // the waves, then the tile's exclusive scan over digits; cnt[w][d]
    // becomes the tile slot of wave w's first item of digit d, gb[d] the
    // global slot of tile slot 0
    {
        const int t = threadIdx.x;
        int32_t c[DN_DPT][DN_WAVES], tsum[DN_DPT];
        int32_t x = 0;
#pragma unroll
        for (int e = 0; e < DN_DPT; ++e) {
            const int d = DN_DPT * t + e;
            int32_t acc = 0;
#pragma unroll
            for (int q = 0; q < DN_WAVES; ++q) {
                c[e][q] = acc;
                acc += cnt[q][d];
            }
            tsum[e] = acc;
            x += acc;
        }
        const int32_t own = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        int32_t be = x - own;
        for (int q = 0; q < w; ++q) be += wsum[q];
#pragma unroll
        for (int e = 0; e < DN_DPT; ++e) {
            const int d = DN_DPT * t + e;
#pragma unroll
            for (int q = 0; q < DN_WAVES; ++q) cnt[q][d] = c[e][q] + be;
            gb[d] = g[e] - be;
            be += tsum[e];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < DN_ITEMS; ++it) {
        if (rank[it] < 0) continue;
        const int32_t d = (key[it] >> shift) & mask;
        rank[it] += cnt[w][d];                          // tile slot
        stage[rank[it]] = key[it];
    }
    __syncthreads();
    int32_t oo[DN_ITEMS], vv[DN_ITEMS];
#pragma unroll
    for (int it = 0; it < DN_ITEMS; ++it) {
        const int s = threadIdx.x + it * DN_THREADS;
        const bool ok = s < tn;
        const int32_t k = ok ? stage[s] : -1;
        oo[it] = -1;
        if (ok) {
            const int32_t o = gb[(k >> shift) & mask] + s;
            if (!LAST) keys_out[o] = k;
            oo[it] = o;
        }
        if (LAST) count_runs(k, ok, s, tn, lane, counts, n_cells);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < DN_ITEMS; ++it)
        if (rank[it] >= 0) stage[rank[it]] = val[it];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < DN_ITEMS; ++it) {
        const int s = threadIdx.x + it * DN_THREADS;
        vv[it] = 0;
        if (oo[it] >= 0) {
            vv[it] = stage[s];
            vals_out[oo[it]] = vv[it];
        }
    }
    if (LAST) {
        // all gathers first, then all stores, so the loads overlap
        T gx[DN_ITEMS], gy[DN_ITEMS], gz[DN_ITEMS];
#pragma unroll
        for (int it = 0; it < DN_ITEMS; ++it) {
            if (oo[it] < 0) continue;
            gx[it] = vin.x[vv[it]];
            gy[it] = vin.y[vv[it]];
            gz[it] = vin.z[vv[it]];
        }
#pragma unroll
        for (int it = 0; it < DN_ITEMS; ++it) {
            if (oo[it] < 0) continue;
            vout.x[oo[it]] = gx[it];
            vout.y[oo[it]] = gy[it];
            vout.z[oo[it]] = gz[it];
        }
    }
}

static int sort_passes(int32_t n_cells, int* bits_total)
{
    const int nbits = 32 - __builtin_clz((unsigned)n_cells);   // keys go up to n_cells
    *bits_total = nbits;
    return (nbits + RADIX_BITS - 1) / RADIX_BITS;
}

static int64_t sort_tiles(int32_t n) { return ((int64_t)n + SORT_TILE - 1) / SORT_TILE; }

template <typename T>
static int sort_impl(int32_t n, int32_t n_cells, const int32_t* cell_of, dsmc_vec3 vin,
                     dsmc_vec3 vout, int32_t* cell_start, int32_t* perm, void* ws,
                     dsmc_status* st, hipStream_t s)
{
    if (n == 0) return fill_i32(cell_start, 0, (int64_t)n_cells + 1, s);
    const int64_t nblk = sort_tiles(n);
    uint8_t* w = static_cast<uint8_t*>(ws);
    int32_t* keys_a = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * (size_t)n);
    int32_t* keys_b = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * (size_t)n);
    int32_t* vals_a = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * (size_t)n);
    int32_t* ghist = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * (size_t)(RADIX * nblk));
    int32_t* goff = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * (size_t)(RADIX * nblk));
    const int64_t nch = (nblk + HCHUNK - 1) / HCHUNK;
    int32_t* csum = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * (size_t)(RADIX * nch));
    int32_t* cpre = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * (size_t)(RADIX * nch));
    int32_t* dtot = reinterpret_cast<int32_t*>(w);
    w += align_up(sizeof(int32_t) * (size_t)RADIX);
    void* scan_ws = w;
    {
        const int rc = fill_i32(cell_start, 0, (int64_t)n_cells + 1, s);
        if (rc) return rc;
    }

    int nbits = 0;
    const int passes = sort_passes(n_cells, &nbits);
    const int32_t* kin = cell_of;
    const int32_t* vin_idx = nullptr;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * RADIX_BITS;
        const int dbits = (nbits - shift) < RADIX_BITS ? (nbits - shift) : RADIX_BITS;
        const int32_t mask = (1 << dbits) - 1;
        const bool to_final = ((passes - 1 - pass) % 2) == 0;
        int32_t* kout = to_final ? keys_b : keys_a;
        int32_t* vout_idx = to_final ? perm : vals_a;
        if (pass == 0)
            k_radix_up<true><<<(int)nblk, SORT_THREADS, 0, s>>>(kin, n, n_cells, shift, mask, ghist,
                                                                st);
        else
            k_radix_up<false><<<(int)nblk, SORT_THREADS, 0, s>>>(kin, n, n_cells, shift, mask, ghist,
                                                                 st);
        DSMC_LAUNCH_CHECK("sort:up");
        const int32_t R = mask + 1;
        k_hist_chunk_sum<<<(int)nch, 256, 0, s>>>(ghist, (int32_t)nblk, R, csum);
        k_hist_chunk_scan<<<(R + HDIG - 1) / HDIG, 256, 0, s>>>(csum, (int32_t)nch, R, cpre, dtot);
        k_hist_expand<<<(int)nch, 256, 0, s>>>(ghist, cpre, dtot, (int32_t)nblk, R, goff);
        DSMC_LAUNCH_CHECK("sort:scan");
        const bool last = pass == passes - 1;
        const V3<const T> vi = v3<const T>(vin);
        const V3<T> vo = v3<T>(vout);
        if (pass == 0 && last)
            k_radix_down<true, true, T><<<(int)nblk, DN_THREADS, 0, s>>>(
                kin, vin_idx, n, n_cells, shift, mask, dbits, goff, kout, vout_idx,
                vi, vo, cell_start);
        else if (pass == 0)
            k_radix_down<true, false, T><<<(int)nblk, DN_THREADS, 0, s>>>(
                kin, vin_idx, n, n_cells, shift, mask, dbits, goff, kout, vout_idx,
                vi, vo, cell_start);
        else if (last)
            k_radix_down<false, true, T><<<(int)nblk, DN_THREADS, 0, s>>>(
                kin, vin_idx, n, n_cells, shift, mask, dbits, goff, kout, vout_idx,
                vi, vo, cell_start);
        else
            k_radix_down<false, false, T><<<(int)nblk, DN_THREADS, 0, s>>>(
                kin, vin_idx, n, n_cells, shift, mask, dbits, goff, kout, vout_idx,
                vi, vo, cell_start);
        DSMC_LAUNCH_CHECK("sort:down");
        kin = kout;
        vin_idx = vout_idx;
    }
    // cell_start: exclusive scan, in place, of the counts the last pass added
    int rc = exclusive_scan_i32(cell_start, cell_start, n_cells, nullptr, scan_ws, s);
    if (rc) return rc;
    return DSMC_OK;
}

}  // namespace dsmc

using namespace dsmc;

// ------------------------------------------------------------------------
// Allocation-free variant: the scratch lives in a file-scope device array,
// one copy per GPU, held until the process ends.  Sized for the limits
// below with a margin (the scan's tile table of the cell counts needs far
// less than one int per cell).
// ------------------------------------------------------------------------
namespace dsmc {

constexpr int32_t NOALLOC_MAX_N = 1 << 20;
constexpr int32_t NOALLOC_MAX_CELLS = 1 << 20;
constexpr size_t noalloc_round(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t NOALLOC_TILES = ((size_t)NOALLOC_MAX_N + SORT_TILE - 1) / SORT_TILE;
constexpr size_t NOALLOC_CHUNKS = (NOALLOC_TILES + HCHUNK - 1) / HCHUNK;
constexpr size_t NOALLOC_SCRATCH_BYTES =
    3 * noalloc_round(sizeof(int32_t) * (size_t)NOALLOC_MAX_N) +
    2 * noalloc_round(sizeof(int32_t) * RADIX * NOALLOC_TILES) +
    2 * noalloc_round(sizeof(int32_t) * RADIX * NOALLOC_CHUNKS) +
    noalloc_round(sizeof(int32_t) * RADIX) +
    noalloc_round(sizeof(int32_t) * ((size_t)NOALLOC_MAX_CELLS + 2)) + 256;

static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on each GPU, taken once per device with that
// device current (the host-side name of the array is not a device address).
constexpr int NOALLOC_MAX_DEVICES = 64;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

static int scratch_ptr(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(e, "dsmc_sort_cells_noalloc: hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return arg_error("dsmc_sort_cells_noalloc: device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_check(e, "dsmc_sort_cells_noalloc: hipGetSymbolAddress");
        if (!p) return arg_error("dsmc_sort_cells_noalloc: null scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DSMC_OK;
}

}  // namespace dsmc

extern "C" int dsmc_sort_cells_noalloc(int32_t n, int32_t n_cells, const int32_t* cell_of,
                                       int32_t dtype, dsmc_vec3 v_in, dsmc_vec3 v_out,
                                       int32_t* cell_start, int32_t* perm, dsmc_status* st,
                                       dsmc_stream_t stream)
{
    if (n < 0 || n_cells < 1) return arg_error("dsmc_sort_cells_noalloc: n=%d n_cells=%d", n, n_cells);
    if (n > NOALLOC_MAX_N || n_cells > NOALLOC_MAX_CELLS)
        return arg_error("dsmc_sort_cells_noalloc: n=%d, n_cells=%d beyond the static scratch "
                         "limits (%d particles, %d cells); use dsmc_sort_cells with a workspace",
                         n, n_cells, NOALLOC_MAX_N, NOALLOC_MAX_CELLS);
    if (!cell_start || (n > 0 && (!cell_of || !perm || !v_in.x || !v_in.y || !v_in.z ||
                                  !v_out.x || !v_out.y || !v_out.z)))
        return arg_error("dsmc_sort_cells_noalloc: null pointer");
    if (dtype != DSMC_F64 && dtype != DSMC_F32)
        return arg_error("dsmc_sort_cells_noalloc: dtype %d", dtype);
    if (dsmc_sort_cells_ws(n, n_cells) > NOALLOC_SCRATCH_BYTES)
        return arg_error("dsmc_sort_cells_noalloc: scratch %zu < %zu", NOALLOC_SCRATCH_BYTES,
                         dsmc_sort_cells_ws(n, n_cells));
    void* ws = nullptr;
    int rc = scratch_ptr(&ws);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    if (dtype == DSMC_F64)
        return sort_impl<double>(n, n_cells, cell_of, v_in, v_out, cell_start, perm, ws, st, s);
    return sort_impl<float>(n, n_cells, cell_of, v_in, v_out, cell_start, perm, ws, st, s);
}

extern "C" size_t dsmc_sort_cells_ws(int32_t n, int32_t n_cells)
{
    if (n < 0 || n_cells < 0) return 0;
    const int64_t nblk = sort_tiles(n);
    const int64_t nch = (nblk + HCHUNK - 1) / HCHUNK;
    return 3 * align_up(sizeof(int32_t) * (size_t)n) +
           2 * align_up(sizeof(int32_t) * (size_t)(RADIX * nblk)) +
           2 * align_up(sizeof(int32_t) * (size_t)(RADIX * nch)) +
           align_up(sizeof(int32_t) * (size_t)RADIX) + scan_ws_bytes(n_cells) + 256;
}

extern "C" int dsmc_sort_cells(int32_t n, int32_t n_cells, const int32_t* cell_of, int32_t dtype,
                               dsmc_vec3 v_in, dsmc_vec3 v_out, int32_t* cell_start,
                               int32_t* perm, void* ws, size_t ws_bytes, dsmc_status* st,
                               dsmc_stream_t stream)
{
    if (n < 0 || n_cells < 1) return arg_error("dsmc_sort_cells: n=%d n_cells=%d", n, n_cells);
    if (n_cells == INT32_MAX) return arg_error("dsmc_sort_cells: n_cells must be < 2^31 - 1");
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
