// No-Time-Counter pair selection (section "Cell partition and collision-pair
// selection").  Candidates are generated for all cells at once, one lane per
// candidate, so the work is balanced however uneven the cell populations are:
//   count M_k per cell -> scan (candidate offsets) -> accept pass: each wave
//   takes a chunk of 1024 consecutive candidates (one binary search for the
//   chunk's first cell, then a forward walk), draws and decides them and
//   counts the accepted ones -> scan of the chunk counts -> emit pass: the
//   same decisions again, accepted pairs written densely (cell-major,
//   candidate order) at the chunk's offset, with each cell's pair offset ->
//   per-cell counts.
// Deciding twice costs arithmetic and L2-resident velocity reads, and saves
// writing and re-reading every candidate.  The decision arithmetic (g, the
// candidate count) uses explicitly rounded FP64 operations so it is the same
// on every launch shape and in both passes.
#include <math.h>

#include "common.hpp"

namespace dsmc {

struct XsLaw {
    double C, e;  // sigma(g) g = C g^e
};

static int xs_law(const dsmc_xs& xs, XsLaw* out)
{
    constexpr double KB = 1.380649e-23;
    constexpr double PI = 3.14159265358979323846;
    if (xs.kind == DSMC_XS_VHS) {
        if (!(xs.m > 0) || !(xs.d_ref > 0) || !(xs.T_ref > 0) || !(xs.omega > 0.5) ||
            !(xs.omega < 1.0))
            return arg_error("dsmc_xs: bad VHS parameters");
        const double mr = xs.m / 2.0;
        out->C = PI * xs.d_ref * xs.d_ref * pow(2.0 * KB * xs.T_ref / mr, xs.omega - 0.5) /
                 tgamma(2.5 - xs.omega);
        out->e = 2.0 - 2.0 * xs.omega;
        return DSMC_OK;
    }
    if (xs.kind == DSMC_XS_CONST) {
        if (!(xs.sigma > 0)) return arg_error("dsmc_xs: sigma must be > 0");
        out->C = xs.sigma;
        out->e = 1.0;
        return DSMC_OK;
    }
    return arg_error("dsmc_xs: kind %d", xs.kind);
}

__device__ __forceinline__ int32_t cand_count(int32_t N, double lam, XsLaw law, double cmax,
                                              const dsmc_rng& rng, int32_t k)
{
    if (N < 2) return 0;
    const double ghat = 2.0 * cmax;
    const double sgmax = law.C * pow(ghat, law.e);
    const U4 r = draw(rng, 0u, (uint32_t)k, SLOT_COUNT);
    const double U = unif53(r.a, r.b);
    double x = __dmul_rn(0.5, (double)N);
    x = __dmul_rn(x, (double)(N - 1));
    x = __dmul_rn(x, lam);
    x = __dmul_rn(x, sgmax);
    x = __dadd_rn(x, U);
    if (!(x >= 0.0) || !(x < 2147483647.0)) return 0;
    return (int32_t)floor(x);
}

__global__ void __launch_bounds__(256)
k_cand_count(const int32_t* __restrict__ cell_start, int32_t n_cells,
             const double* __restrict__ lambda, const double* __restrict__ mom, XsLaw law,
             dsmc_rng rng, int32_t* __restrict__ cnt)
{
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_cells;
         k += gridDim.x * blockDim.x) {
        const int32_t N = cell_start[k + 1] - cell_start[k];
        cnt[k] = cand_count(N, lambda[k], law, mom[6 * (size_t)k + 4], rng, k);
    }
}

constexpr int CAND_ROUNDS = 16;
constexpr int CAND_CHUNK = 64 * CAND_ROUNDS;

// Overflow decision: total candidates vs capacity; number of chunks.
__global__ void k_cand_check(const int64_t* total, int64_t cap, int32_t* ok, int64_t* n_use,
                             int64_t* n_chunks, dsmc_status* st)
{
    const int64_t t = *total;
    const bool fits = t <= cap;
    *ok = fits ? 1 : 0;
    *n_use = fits ? t : 0;
    *n_chunks = fits ? (t + CAND_CHUNK - 1) / CAND_CHUNK : 0;
    if (st) {
        st->n_cand = t;
        if (!fits) atomicOr(&st->flags, (uint32_t)DSMC_ST_PAIR_OVERFLOW);
    }
}

// Largest k with off[k] <= c (off non-decreasing, off[0] = 0).
__device__ __forceinline__ int32_t find_cell(const int32_t* __restrict__ off, int32_t n_cells,
                                             int32_t c)
{
    int32_t lo = 0, hi = n_cells;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// Candidate t of cell k: indices (Lemire multiply-shift, j != i) and the
// acceptance test U < (g / g_hat)^e.
template <typename T>
__device__ __forceinline__ bool cand_decide(const int32_t* __restrict__ cell_start, int32_t k,
                                            int32_t t, const double* __restrict__ mom, double e,
                                            const dsmc_rng& rng, const V3<const T>& v,
                                            int32_t& pi, int32_t& pj)
{
    const int32_t s0 = cell_start[k], N = cell_start[k + 1] - s0;
    const U4 r = draw(rng, (uint32_t)t, (uint32_t)k, SLOT_CAND);
    int32_t i = (int32_t)(((uint64_t)r.a * (uint64_t)N) >> 32);
    int32_t j = (int32_t)(((uint64_t)r.b * (uint64_t)(N - 1)) >> 32);
    if (j >= i) j += 1;
    const double U = unif53(r.c, r.d);
    const double dx = (double)v.x[s0 + i] - (double)v.x[s0 + j];
    const double dy = (double)v.y[s0 + i] - (double)v.y[s0 + j];
    const double dz = (double)v.z[s0 + i] - (double)v.z[s0 + j];
    const double g2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                __dmul_rn(dz, dz));
    const double g = sqrt(g2);
    const double ghat = 2.0 * mom[6 * (size_t)k + 4];
    const double ratio = g / ghat;
    const double p = (e == 1.0) ? ratio : pow(ratio, e);
    pi = s0 + i;
    pj = s0 + j;
    return U < p;
}

// EMIT = false: accepted candidates per chunk.  EMIT = true: write the
// accepted pairs from the chunk offsets, and pair_off[k] for every cell whose
// candidates start inside the chunk (empty cells get the offset of the next
// candidate).
template <typename T, bool EMIT>
__global__ void __launch_bounds__(256)
k_cand_chunks(const int32_t* __restrict__ cell_start, int32_t n_cells,
              const int32_t* __restrict__ cand_off, const int64_t* __restrict__ n_use,
              const double* __restrict__ mom, double e, dsmc_rng rng, V3<const T> v,
              int32_t* __restrict__ chunk_cnt, const int32_t* __restrict__ chunk_off,
              int32_t* __restrict__ pi, int32_t* __restrict__ pj, int32_t* __restrict__ pc,
              int32_t* __restrict__ pair_off)
{
    const int64_t total = *n_use;
    const int64_t nch = (total + CAND_CHUNK - 1) / CAND_CHUNK;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t ch = wave; ch < nch; ch += nwaves) {
        const int64_t cbase = ch * CAND_CHUNK;
        int32_t kw = find_cell(cand_off, n_cells, (int32_t)cbase);
        int32_t pos = EMIT ? chunk_off[ch] : 0;
        int32_t acc = 0;
        for (int r = 0; r < CAND_ROUNDS; ++r) {
            const int64_t base = cbase + r * 64;
            if (base >= total) break;
            const int64_t c = base + lane;
            const bool valid = c < total;
            int32_t k = kw, i = 0, j = 0;
            bool take = false;
            if (valid) {
                while (k + 1 < n_cells && cand_off[k + 1] <= c) ++k;
                take = cand_decide<T>(cell_start, k, (int32_t)(c - cand_off[k]), mom, e, rng, v,
                                      i, j);
            }
            const uint64_t ab = __ballot(take);
            if (EMIT) {
                const int32_t p = pos + (int32_t)__popcll(ab & lt);
                if (take) {
                    pi[p] = i;
                    pj[p] = j;
                    pc[p] = k;
                }
                if (valid && c == cand_off[k]) {
                    pair_off[k] = p;
                    for (int32_t q = k - 1; q >= 0 && cand_off[q] == c; --q) pair_off[q] = p;
                }
                pos += (int32_t)__popcll(ab);
            } else {
                acc += (int32_t)__popcll(ab);
            }
            kw = __shfl(k, 63, 64);
        }
        if (!EMIT && lane == 0) chunk_cnt[ch] = acc;
    }
}

// Pair counts per cell; cells whose candidates would start at or after the
// last candidate (none left) get the total as offset.
__global__ void __launch_bounds__(256)
k_pair_counts(int32_t n_cells, const int32_t* __restrict__ cand_off,
              const int32_t* __restrict__ ok, const int64_t* __restrict__ n_use,
              const int64_t* __restrict__ n_chunks, const int32_t* __restrict__ chunk_off,
              int32_t* __restrict__ off, int32_t* __restrict__ cnt, dsmc_status* st)
{
    const bool fits = *ok != 0;
    const int64_t total = *n_use;
    const int32_t npairs = fits ? chunk_off[*n_chunks] : 0;
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_cells;
         k += gridDim.x * blockDim.x) {
        if (!fits) {
            off[k] = 0;
            cnt[k] = 0;
            continue;
        }
        const bool tail = cand_off[k] >= total;
        const int32_t a = tail ? npairs : off[k];
        const int32_t b = (k + 1 == n_cells || cand_off[k + 1] >= total) ? npairs : off[k + 1];
        if (tail) off[k] = a;
        cnt[k] = b - a;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && st) st->n_pairs = npairs;
}

struct SelectWs {
    int32_t* cand_cnt;   // [n_cells]
    int32_t* cand_off;   // [n_cells + 1]
    int64_t* total;      // candidates
    int64_t* n_use;      // candidates processed (0 on overflow)
    int64_t* n_chunks;
    int32_t* ok;
    int32_t* chunk_cnt;  // [max chunks]
    int32_t* chunk_off;  // [max chunks + 1]
    void* scan;
    size_t bytes;
};

static int64_t max_chunks(int64_t cap) { return (cap + CAND_CHUNK - 1) / CAND_CHUNK + 1; }

static SelectWs select_ws_layout(void* base, int32_t n_cells, int64_t cap)
{
    SelectWs w{};
    uint8_t* p = static_cast<uint8_t*>(base);
    size_t o = 0;
    auto take = [&](size_t b) { uint8_t* r = p ? p + o : nullptr; o += align_up(b); return r; };
    const int64_t mc = max_chunks(cap);
    w.cand_cnt = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)n_cells + 1)));
    w.cand_off = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)n_cells + 2)));
    w.total = reinterpret_cast<int64_t*>(take(sizeof(int64_t)));
    w.n_use = reinterpret_cast<int64_t*>(take(sizeof(int64_t)));
    w.n_chunks = reinterpret_cast<int64_t*>(take(sizeof(int64_t)));
    w.ok = reinterpret_cast<int32_t*>(take(sizeof(int32_t)));
    w.chunk_cnt = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)mc));
    w.chunk_off = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)mc + 1)));
    const size_t sb = scan_ws_bytes((int64_t)(mc > n_cells ? mc : n_cells) + 1);
    w.scan = take(sb);
    w.bytes = o;
    return w;
}

template <typename T>
static int select_impl(int32_t n_cells, const int32_t* cell_start, dsmc_vec3 v, XsLaw law,
                       const double* lambda, const double* mom, dsmc_rng rng,
                       dsmc_pairs pairs, void* ws, dsmc_status* st, hipStream_t s)
{
    SelectWs w = select_ws_layout(ws, n_cells, pairs.cap);
    const int pb = persistent_blocks(256);
    int cb = (n_cells + 255) / 256;
    cb = cb < 1 ? 1 : (cb > pb ? pb : cb);
    k_cand_count<<<cb, 256, 0, s>>>(cell_start, n_cells, lambda, mom, law, rng, w.cand_cnt);
    DSMC_LAUNCH_CHECK("select:count");
    int rc = exclusive_scan_i32(w.cand_cnt, w.cand_off, n_cells, w.total, w.scan, s);
    if (rc) return rc;
    k_cand_check<<<1, 1, 0, s>>>(w.total, pairs.cap, w.ok, w.n_use, w.n_chunks, st);
    DSMC_LAUNCH_CHECK("select:check");
    const V3<const T> vv = v3<const T>(v);
    k_cand_chunks<T, false><<<pb, 256, 0, s>>>(cell_start, n_cells, w.cand_off, w.n_use, mom,
                                               law.e, rng, vv, w.chunk_cnt, nullptr, nullptr,
                                               nullptr, nullptr, nullptr);
    DSMC_LAUNCH_CHECK("select:accept");
    rc = exclusive_scan_i32_dev(w.chunk_cnt, w.chunk_off, w.n_chunks, max_chunks(pairs.cap),
                                w.scan, s);
    if (rc) return rc;
    k_cand_chunks<T, true><<<pb, 256, 0, s>>>(cell_start, n_cells, w.cand_off, w.n_use, mom,
                                              law.e, rng, vv, nullptr, w.chunk_off, pairs.i,
                                              pairs.j, pairs.cell, pairs.off);
    DSMC_LAUNCH_CHECK("select:emit");
    k_pair_counts<<<cb, 256, 0, s>>>(n_cells, w.cand_off, w.ok, w.n_use, w.n_chunks, w.chunk_off,
                                     pairs.off, pairs.cnt, st);
    DSMC_LAUNCH_CHECK("select:counts");
    return DSMC_OK;
}

}  // namespace dsmc

using namespace dsmc;

extern "C" size_t dsmc_select_pairs_ntc_ws(int32_t n_cells, int64_t cap)
{
    if (n_cells < 1 || cap < 0) return 0;
    return select_ws_layout(nullptr, n_cells, cap).bytes + 256;
}

extern "C" int dsmc_select_pairs_ntc(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                                     dsmc_vec3 v, dsmc_xs xs, const double* lambda,
                                     const double* mom, dsmc_rng rng, dsmc_pairs pairs,
                                     void* ws, size_t ws_bytes, dsmc_status* st,
                                     dsmc_stream_t stream)
{
    if (n_cells < 1) return arg_error("dsmc_select_pairs_ntc: n_cells=%d", n_cells);
    if (!cell_start || !lambda || !mom || !ws || !v.x || !v.y || !v.z || !pairs.off ||
        !pairs.cnt || (pairs.cap > 0 && (!pairs.i || !pairs.j || !pairs.cell)))
        return arg_error("dsmc_select_pairs_ntc: null pointer");
    if (pairs.cap < 0 || pairs.cap >= (int64_t)INT32_MAX - 2)
        return arg_error("dsmc_select_pairs_ntc: cap %lld out of range", (long long)pairs.cap);
    if (ws_bytes < dsmc_select_pairs_ntc_ws(n_cells, pairs.cap))
        return arg_error("dsmc_select_pairs_ntc: workspace %zu < %zu", ws_bytes,
                         dsmc_select_pairs_ntc_ws(n_cells, pairs.cap));
    XsLaw law;
    int rc = xs_law(xs, &law);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    if (dtype == DSMC_F64)
        return select_impl<double>(n_cells, cell_start, v, law, lambda, mom, rng, pairs, ws, st, s);
    if (dtype == DSMC_F32)
        return select_impl<float>(n_cells, cell_start, v, law, lambda, mom, rng, pairs, ws, st, s);
    return arg_error("dsmc_select_pairs_ntc: dtype %d", dtype);
}

namespace dsmc {
// Shared with the fused step kernel.
int xs_law_public(const dsmc_xs& xs, double* C, double* e)
{
    XsLaw l;
    int rc = xs_law(xs, &l);
    *C = l.C;
    *e = l.e;
    return rc;
}
}  // namespace dsmc
