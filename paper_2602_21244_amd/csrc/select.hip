// No-Time-Counter pair selection (section "Cell partition and collision-pair
// selection").  Candidates are generated for all cells at once, one lane per
// candidate, so the work is balanced however uneven the cell populations are:
//   count M_k per cell -> scan (candidate offsets) -> draw + accept per
//   candidate -> scan of the accept flags -> scatter accepted pairs densely
//   (cell-major, candidate order) -> per-cell offsets and counts.
// The decision arithmetic (g, the candidate count) uses explicitly rounded
// FP64 operations so it is the same on every launch shape.
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

// Overflow decision: total candidates vs capacity.
__global__ void k_cand_check(const int64_t* total, int64_t cap, int32_t* ok, int64_t* n_use,
                             dsmc_status* st)
{
    const int64_t t = *total;
    const bool fits = t <= cap;
    *ok = fits ? 1 : 0;
    *n_use = fits ? t : 0;
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

template <typename T>
__global__ void __launch_bounds__(256)
k_candidates(const int32_t* __restrict__ cell_start, int32_t n_cells,
             const int32_t* __restrict__ cand_off, const int64_t* __restrict__ n_use,
             const double* __restrict__ mom, double e, dsmc_rng rng, V3<const T> v,
             int32_t* __restrict__ flag, int32_t* __restrict__ ci, int32_t* __restrict__ cj,
             int32_t* __restrict__ ck)
{
    const int64_t total = *n_use;
    const int lane = threadIdx.x & 63;
    // one binary search per wavefront (for its first candidate); lanes then
    // step forward over the few cells the wave's 64 candidates span
    for (int64_t base = (blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63)); base < total;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = base + lane;
        int32_t k = find_cell(cand_off, n_cells, (int32_t)base);
        if (c >= total) continue;
        while (k + 1 < n_cells && cand_off[k + 1] <= c) ++k;
        const int32_t t = (int32_t)c - cand_off[k];
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
        flag[c] = (U < p) ? 1 : 0;
        ci[c] = s0 + i;
        cj[c] = s0 + j;
        ck[c] = k;
    }
}

__global__ void __launch_bounds__(256)
k_pairs_scatter(const int64_t* __restrict__ n_use, const int32_t* __restrict__ flag,
                const int32_t* __restrict__ pos, const int32_t* __restrict__ ci,
                const int32_t* __restrict__ cj, const int32_t* __restrict__ ck,
                int32_t* __restrict__ pi, int32_t* __restrict__ pj, int32_t* __restrict__ pc)
{
    const int64_t total = *n_use;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < total;
         c += (int64_t)gridDim.x * blockDim.x) {
        if (flag[c]) {
            const int32_t p = pos[c];
            pi[p] = ci[c];
            pj[p] = cj[c];
            pc[p] = ck[c];
        }
    }
}

__global__ void __launch_bounds__(256)
k_pair_offsets(int32_t n_cells, const int32_t* __restrict__ cand_off,
               const int32_t* __restrict__ pos, const int32_t* __restrict__ ok,
               const int64_t* __restrict__ n_use, int32_t* __restrict__ off,
               int32_t* __restrict__ cnt, dsmc_status* st)
{
    const bool fits = *ok != 0;
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_cells;
         k += gridDim.x * blockDim.x) {
        if (fits) {
            const int32_t a = pos[cand_off[k]], b = pos[cand_off[k + 1]];
            off[k] = a;
            cnt[k] = b - a;
        } else {
            off[k] = 0;
            cnt[k] = 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && st) {
        st->n_pairs = fits ? (int64_t)pos[*n_use] : 0;
    }
}

struct SelectWs {
    int32_t* cand_cnt;  // [n_cells]
    int32_t* cand_off;  // [n_cells + 1]
    int64_t* total;     // candidates
    int64_t* n_use;     // candidates processed (0 on overflow)
    int32_t* ok;
    int32_t* flag;      // [cap]
    int32_t* pos;       // [cap + 1]
    int32_t* ci;        // [cap]
    int32_t* cj;        // [cap]
    int32_t* ck;        // [cap]
    void* scan;
    size_t bytes;
};

static SelectWs select_ws_layout(void* base, int32_t n_cells, int64_t cap)
{
    SelectWs w{};
    uint8_t* p = static_cast<uint8_t*>(base);
    size_t o = 0;
    auto take = [&](size_t b) { uint8_t* r = p ? p + o : nullptr; o += align_up(b); return r; };
    w.cand_cnt = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)n_cells + 1)));
    w.cand_off = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)n_cells + 2)));
    w.total = reinterpret_cast<int64_t*>(take(sizeof(int64_t)));
    w.n_use = reinterpret_cast<int64_t*>(take(sizeof(int64_t)));
    w.ok = reinterpret_cast<int32_t*>(take(sizeof(int32_t)));
    w.flag = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)cap + 1)));
    w.pos = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)cap + 2)));
    w.ci = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)cap + 1)));
    w.cj = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)cap + 1)));
    w.ck = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)cap + 1)));
    const size_t sb = scan_ws_bytes((int64_t)(cap > n_cells ? cap : n_cells) + 1);
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
    k_cand_check<<<1, 1, 0, s>>>(w.total, pairs.cap, w.ok, w.n_use, st);
    DSMC_LAUNCH_CHECK("select:check");
    k_candidates<T><<<pb, 256, 0, s>>>(cell_start, n_cells, w.cand_off, w.n_use, mom, law.e, rng,
                                       v3<const T>(v), w.flag, w.ci, w.cj, w.ck);
    DSMC_LAUNCH_CHECK("select:candidates");
    rc = exclusive_scan_i32_dev(w.flag, w.pos, w.n_use, pairs.cap, w.scan, s);
    if (rc) return rc;
    k_pairs_scatter<<<pb, 256, 0, s>>>(w.n_use, w.flag, w.pos, w.ci, w.cj, w.ck, pairs.i,
                                       pairs.j, pairs.cell);
    DSMC_LAUNCH_CHECK("select:scatter");
    k_pair_offsets<<<cb, 256, 0, s>>>(n_cells, w.cand_off, w.pos, w.ok, w.n_use, pairs.off,
                                      pairs.cnt, st);
    DSMC_LAUNCH_CHECK("select:offsets");
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
