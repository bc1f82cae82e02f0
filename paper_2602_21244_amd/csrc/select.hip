// No-Time-Counter pair selection (section "Cell partition and collision-pair
// selection").  Candidates are generated for all cells at once, one lane per
// candidate, so the work is balanced however uneven the cell populations are:
//   count M_k per cell -> scan (candidate offsets) -> the cell of each
//   1024-candidate chunk's first candidate -> decide pass: each wave takes a
//   chunk, walks its cells forward, draws and decides the candidates and
//   stages the accepted pairs compactly in the chunk's own slots, with each
//   cell's offset inside the chunk -> scan of the chunk counts -> copy pass:
//   the staged pairs of every chunk to their dense, cell-major place -> per
//   cell offsets and counts.
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

constexpr int CAND_ROUNDS = 16;
constexpr int CAND_CHUNK = 64 * CAND_ROUNDS;
constexpr int CAND_GROUP = 4;
constexpr int CAND_WIN = 4;      // scalar cell window of a group (see k_cand_decide)

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

// Candidate t of cell k: indices (Lemire multiply-shift, j != i) and the
// acceptance uniform.
struct CandDraw {
    int32_t i, j;   // sorted slots
    double U;
};

__device__ __forceinline__ CandDraw cand_draw_sn(int32_t s0, int32_t N, int32_t k, int32_t t,
                                                 const dsmc_rng& rng)
{
    const U4 r = draw(rng, (uint32_t)t, (uint32_t)k, SLOT_CAND);
    int32_t i = (int32_t)(((uint64_t)r.a * (uint64_t)N) >> 32);
    int32_t j = (int32_t)(((uint64_t)r.b * (uint64_t)(N - 1)) >> 32);
    if (j >= i) j += 1;
    return CandDraw{s0 + i, s0 + j, unif53(r.c, r.d)};
}

__device__ __forceinline__ CandDraw cand_draw(const int32_t* __restrict__ cell_start, int32_t k,
                                              int32_t t, const dsmc_rng& rng)
{
    const int32_t s0 = cell_start[k], N = cell_start[k + 1] - s0;
    const U4 r = draw(rng, (uint32_t)t, (uint32_t)k, SLOT_CAND);
    int32_t i = (int32_t)(((uint64_t)r.a * (uint64_t)N) >> 32);
    int32_t j = (int32_t)(((uint64_t)r.b * (uint64_t)(N - 1)) >> 32);
    if (j >= i) j += 1;
    return CandDraw{s0 + i, s0 + j, unif53(r.c, r.d)};
}

// Acceptance test U < (g / g_hat)^e on the pre-step velocities.
template <typename T>
__device__ __forceinline__ bool cand_accept(const CandDraw& d, const V3<const T>& v, double ghat,
                                            double e)
{
    const double dx = (double)v.x[d.i] - (double)v.x[d.j];
    const double dy = (double)v.y[d.i] - (double)v.y[d.j];
    const double dz = (double)v.z[d.i] - (double)v.z[d.j];
    const double g2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                __dmul_rn(dz, dz));
    const double g = sqrt(g2);
    const double ratio = g / ghat;
    const double p = (e == 1.0) ? ratio : pow(ratio, e);
    return d.U < p;
}

// Simplified Bernoulli Trials (Stefanov 2011): trial t of cell k is the
// particle in slot t; its partner is drawn uniformly among the m = N-1-t
// later slots and the pair collides with probability P = m lambda_k sigma(g) g
// (values above 1 act as 1 and are counted).
__device__ __forceinline__ CandDraw sbt_draw_sn(int32_t s0, int32_t N, int32_t k, int32_t t,
                                                const dsmc_rng& rng, int32_t& m)
{
    m = N - 1 - t;
    const U4 r = draw(rng, (uint32_t)t, (uint32_t)k, SLOT_SBT);
    const int32_t j = t + 1 + (int32_t)(((uint64_t)r.a * (uint64_t)m) >> 32);
    return CandDraw{s0 + t, s0 + j, unif53(r.c, r.d)};
}

__device__ __forceinline__ CandDraw sbt_draw(const int32_t* __restrict__ cell_start, int32_t k,
                                             int32_t t, const dsmc_rng& rng, int32_t& m)
{
    const int32_t s0 = cell_start[k], N = cell_start[k + 1] - s0;
    m = N - 1 - t;
    const U4 r = draw(rng, (uint32_t)t, (uint32_t)k, SLOT_SBT);
    const int32_t j = t + 1 + (int32_t)(((uint64_t)r.a * (uint64_t)m) >> 32);
    return CandDraw{s0 + t, s0 + j, unif53(r.c, r.d)};
}

template <typename T>
__device__ __forceinline__ bool sbt_accept(const CandDraw& d, int32_t m, const V3<const T>& v,
                                           double lam, double C, double e, bool& clamped)
{
    const double dx = (double)v.x[d.i] - (double)v.x[d.j];
    const double dy = (double)v.y[d.i] - (double)v.y[d.j];
    const double dz = (double)v.z[d.i] - (double)v.z[d.j];
    const double g2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                __dmul_rn(dz, dz));
    const double g = sqrt(g2);
    const double sg = __dmul_rn(C, (e == 1.0) ? g : pow(g, e));
    const double P = __dmul_rn(__dmul_rn((double)m, lam), sg);
    clamped = P > 1.0;
    return d.U < P;
}

// Trials per cell of the SBT scheme: N - 1.
__global__ void __launch_bounds__(256)
k_trial_count(const int32_t* __restrict__ cell_start, int32_t n_cells, int32_t* __restrict__ cnt)
{
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_cells;
         k += gridDim.x * blockDim.x) {
        const int32_t N = cell_start[k + 1] - cell_start[k];
        cnt[k] = N >= 2 ? N - 1 : 0;
    }
}

enum { SEL_NTC = 0, SEL_SBT = 1 };

// Cell owning the first candidate of each 64-candidate round (one thread per
// cell writes the rounds that start inside its candidate range).
__global__ void __launch_bounds__(256)
k_round_cells(int32_t n_cells, const int32_t* __restrict__ cand_off,
              const int64_t* __restrict__ n_use, int32_t* __restrict__ round_cell)
{
    const int64_t total = *n_use;
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n_cells;
         k += gridDim.x * blockDim.x) {
        const int64_t a = cand_off[k];
        const int64_t nxt = k + 1 < n_cells ? (int64_t)cand_off[k + 1] : total;
        const int64_t b = nxt < total ? nxt : total;
        for (int64_t r = (a + 63) / 64; r * 64 < b; ++r) round_cell[r] = k;
    }
}

// Decide every candidate of a chunk; accepted pairs go to the chunk's slots
// [ch * 1024, ...) of the staging arrays in candidate order; loc[k] = number
// of accepted pairs of the chunk before cell k's first candidate (for every
// cell whose candidates start inside the chunk; empty cells take the value of
// the next candidate).
template <typename T, int SEL>
__global__ void __launch_bounds__(256)
k_cand_decide(const int32_t* __restrict__ cell_start, int32_t n_cells,
              const int32_t* __restrict__ cand_off, const int64_t* __restrict__ n_use,
              const int32_t* __restrict__ round_cell, const double* __restrict__ mom,
              const double* __restrict__ lambda, double C, double e, dsmc_rng rng,
              V3<const T> v, int32_t* __restrict__ chunk_cnt, int32_t* __restrict__ si,
              int32_t* __restrict__ sj, int32_t* __restrict__ sc, int32_t* __restrict__ loc,
              dsmc_status* st)
{
    int clamped_n = 0;
    const int64_t total = *n_use;
    const int64_t nch = (total + CAND_CHUNK - 1) / CAND_CHUNK;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t ch = wave; ch < nch; ch += nwaves) {
        const int64_t cbase = ch * CAND_CHUNK;
        int32_t acc = 0;
        // CAND_GROUP rounds at a time.  Cells are looked up in two ways:
        //  - when the group's candidates lie in the CAND_WIN cells from the
        //    cell of its first candidate (cells of many candidates), those
        //    cells are read once by scalar loads and a lane's cell is the
        //    number of their starts at or below its candidate;
        //  - otherwise each round of 64 candidates reads a window of 64 cells
        //    from the cell of its first candidate (one coalesced load per
        //    lane and field), a lane finds its cell by a binary search over
        //    the window's candidate offsets with lane shuffles, and a round
        //    that crosses more than 63 cell starts (runs of cells without
        //    candidates) walks on from the window's last cell.
        for (int r0 = 0; r0 < CAND_ROUNDS; r0 += CAND_GROUP) {
            const int64_t gfirst = cbase + r0 * 64;
            if (gfirst >= total) break;
            int32_t kk[CAND_GROUP], s0u[CAND_GROUP], nu[CAND_GROUP], au[CAND_GROUP];
            double gu[CAND_GROUP];
            bool val[CAND_GROUP];
            int64_t cc[CAND_GROUP];
            const int32_t kw = __builtin_amdgcn_readfirstlane(round_cell[gfirst >> 6]);
            const int64_t glast = (gfirst + CAND_GROUP * 64 < total ? gfirst + CAND_GROUP * 64
                                                                      : total) - 1;
            int32_t wb[CAND_WIN];
#pragma unroll
            for (int q = 0; q < CAND_WIN; ++q)
                wb[q] = kw + 1 + q < n_cells ? cand_off[kw + 1 + q] : INT32_MAX;
            if (glast < (int64_t)wb[CAND_WIN - 1]) {
                int32_t ws0[CAND_WIN + 1];
                double wg[CAND_WIN];
#pragma unroll
                for (int q = 0; q <= CAND_WIN; ++q)
                    ws0[q] = cell_start[kw + q <= n_cells ? kw + q : n_cells];
#pragma unroll
                for (int q = 0; q < CAND_WIN; ++q) {
                    const int32_t kq = kw + q < n_cells ? kw + q : n_cells - 1;
                    wg[q] = SEL == SEL_NTC ? 2.0 * mom[6 * (size_t)kq + 4] : lambda[kq];
                }
                const int32_t wa0 = cand_off[kw];
#pragma unroll
                for (int u = 0; u < CAND_GROUP; ++u) {
                    cc[u] = gfirst + u * 64 + lane;
                    val[u] = cc[u] < total;
                    int32_t w = 0;
#pragma unroll
                    for (int q = 0; q < CAND_WIN - 1; ++q) w += cc[u] >= wb[q] ? 1 : 0;
                    int32_t s0 = ws0[0], s1 = ws0[1], a = wa0;
                    double g = wg[0];
#pragma unroll
                    for (int q = 1; q < CAND_WIN; ++q)
                        if (w == q) { s0 = ws0[q]; s1 = ws0[q + 1]; g = wg[q]; a = wb[q - 1]; }
                    kk[u] = kw + w;
                    au[u] = a;
                    s0u[u] = s0;
                    nu[u] = s1 - s0;
                    gu[u] = g;
                }
            } else {
#pragma unroll
                for (int u = 0; u < CAND_GROUP; ++u) {
                    cc[u] = gfirst + u * 64 + lane;
                    val[u] = cc[u] < total;
                    const int64_t rfirst = gfirst + u * 64;
                    const int32_t kr =
                        rfirst < total ? __builtin_amdgcn_readfirstlane(round_cell[rfirst >> 6])
                                       : 0;
                    const int32_t kl = kr + lane;
                    const int32_t A = kl < n_cells ? cand_off[kl] : INT32_MAX;
                    const int32_t An = kl + 1 < n_cells ? cand_off[kl + 1] : INT32_MAX;
                    const int32_t S = cell_start[kl < n_cells ? kl : n_cells];
                    const int32_t Sn = cell_start[kl < n_cells ? kl + 1 : n_cells];
                    const int32_t kq = kl < n_cells ? kl : n_cells - 1;
                    const double G = SEL == SEL_NTC ? 2.0 * mom[6 * (size_t)kq + 4] : lambda[kq];
                    // largest window index l with A[l] <= cc (A[0] <= cc holds)
                    int32_t l = 0;
#pragma unroll
                    for (int stp = 32; stp > 0; stp >>= 1) {
                        const int32_t c = l + stp;
                        const int32_t Ac = __shfl(A, c < 64 ? c : 63, 64);
                        if (c < 64 && (int64_t)Ac <= cc[u]) l = c;
                    }
                    int32_t k = kr + l;
                    int32_t a = __shfl(A, l, 64);
                    int32_t s0 = __shfl(S, l, 64), s1 = __shfl(Sn, l, 64);
                    double g = __shfl(G, l, 64);
                    const int32_t an = __shfl(An, l, 64);
                    if (val[u] && (int64_t)an <= cc[u]) {
                        // beyond the window
                        while (k + 1 < n_cells && cand_off[k + 1] <= cc[u]) ++k;
                        a = cand_off[k];
                        s0 = cell_start[k];
                        s1 = cell_start[k + 1];
                        g = SEL == SEL_NTC ? 2.0 * mom[6 * (size_t)k + 4] : lambda[k];
                    }
                    kk[u] = k;
                    au[u] = a;
                    s0u[u] = s0;
                    nu[u] = s1 - s0;
                    gu[u] = g;
                }
            }
            CandDraw dr[CAND_GROUP];
            int32_t mm[CAND_GROUP];
#pragma unroll
            for (int u = 0; u < CAND_GROUP; ++u) {
                const int32_t t = (int32_t)(cc[u] - au[u]);
                mm[u] = 0;
                if (!val[u]) dr[u] = CandDraw{0, 0, 1.0};
                else if (SEL == SEL_NTC) dr[u] = cand_draw_sn(s0u[u], nu[u], kk[u], t, rng);
                else dr[u] = sbt_draw_sn(s0u[u], nu[u], kk[u], t, rng, mm[u]);
            }
            bool take[CAND_GROUP];
#pragma unroll
            for (int u = 0; u < CAND_GROUP; ++u) {
                if (SEL == SEL_NTC) {
                    take[u] = val[u] && cand_accept<T>(dr[u], v, gu[u], e);
                } else {
                    bool cl = false;
                    take[u] = val[u] && sbt_accept<T>(dr[u], mm[u], v, gu[u], C, e, cl);
                    clamped_n += (val[u] && cl) ? 1 : 0;
                }
            }
#pragma unroll
            for (int u = 0; u < CAND_GROUP; ++u) {
                const uint64_t ab = __ballot(take[u]);
                const int32_t p = acc + (int32_t)__popcll(ab & lt);
                if (take[u]) {
                    si[cbase + p] = dr[u].i;
                    sj[cbase + p] = dr[u].j;
                    sc[cbase + p] = kk[u];
                }
                if (val[u] && cc[u] == au[u]) {
                    loc[kk[u]] = p;
                    for (int32_t q = kk[u] - 1; q >= 0 && cand_off[q] == cc[u]; --q) loc[q] = p;
                }
                acc += (int32_t)__popcll(ab);
            }
        }
        if (lane == 0) chunk_cnt[ch] = acc;
    }
    if (SEL == SEL_SBT && st) {
        const int w = wave_sum_i(clamped_n);
        if (lane == 0 && w > 0) {
            atomicAdd(&st->prob_clamped, w);
            atomicOr(&st->flags, (uint32_t)DSMC_ST_PROB_CLAMP);
        }
    }
}

// Staged pairs of each chunk to their dense place (one wave per chunk).
__global__ void __launch_bounds__(256)
k_stage_copy(const int64_t* __restrict__ n_chunks, const int32_t* __restrict__ chunk_cnt,
             const int32_t* __restrict__ chunk_off, const int32_t* __restrict__ si,
             const int32_t* __restrict__ sj, const int32_t* __restrict__ sc,
             int32_t* __restrict__ pi, int32_t* __restrict__ pj, int32_t* __restrict__ pc)
{
    const int64_t nch = *n_chunks;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t ch = wave; ch < nch; ch += nwaves) {
        const int32_t n = chunk_cnt[ch], o = chunk_off[ch];
        const int64_t src = ch * CAND_CHUNK;
        for (int32_t q = lane; q < n; q += 64) {
            pi[o + q] = si[src + q];
            pj[o + q] = sj[src + q];
            pc[o + q] = sc[src + q];
        }
    }
}

// Pair offsets and counts per cell; cells whose candidates would start at or
// after the last candidate (none left) get the total as offset.
__global__ void __launch_bounds__(256)
k_pair_counts(int32_t n_cells, const int32_t* __restrict__ cand_off,
              const int32_t* __restrict__ ok, const int64_t* __restrict__ n_use,
              const int64_t* __restrict__ n_chunks, const int32_t* __restrict__ chunk_off,
              const int32_t* __restrict__ loc, int32_t* __restrict__ off,
              int32_t* __restrict__ cnt, dsmc_status* st)
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
        const int64_t ca = cand_off[k];
        const int32_t a = ca >= total ? npairs : chunk_off[ca / CAND_CHUNK] + loc[k];
        int32_t b = npairs;
        if (k + 1 < n_cells) {
            const int64_t cb = cand_off[k + 1];
            b = cb >= total ? npairs : chunk_off[cb / CAND_CHUNK] + loc[k + 1];
        }
        off[k] = a;
        cnt[k] = b - a;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && st) st->n_pairs = npairs;
}

struct SelectWs {
    int32_t* cand_cnt;    // [n_cells]
    int32_t* cand_off;    // [n_cells + 1]
    int32_t* loc;         // [n_cells]
    int64_t* total;       // candidates
    int64_t* n_use;       // candidates processed (0 on overflow)
    int64_t* n_chunks;
    int32_t* ok;
    int32_t* round_cell;  // [max chunks * 16]
    int32_t* chunk_cnt;   // [max chunks]
    int32_t* chunk_off;   // [max chunks + 1]
    int32_t* si;          // staging [max chunks * 1024]
    int32_t* sj;
    int32_t* sc;
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
    w.loc = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)n_cells + 1)));
    w.total = reinterpret_cast<int64_t*>(take(sizeof(int64_t)));
    w.n_use = reinterpret_cast<int64_t*>(take(sizeof(int64_t)));
    w.n_chunks = reinterpret_cast<int64_t*>(take(sizeof(int64_t)));
    w.ok = reinterpret_cast<int32_t*>(take(sizeof(int32_t)));
    w.round_cell = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)mc * CAND_ROUNDS));
    w.chunk_cnt = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)mc));
    w.chunk_off = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * ((size_t)mc + 1)));
    const size_t stage = sizeof(int32_t) * (size_t)mc * CAND_CHUNK;
    w.si = reinterpret_cast<int32_t*>(take(stage));
    w.sj = reinterpret_cast<int32_t*>(take(stage));
    w.sc = reinterpret_cast<int32_t*>(take(stage));
    const size_t sb = scan_ws_bytes((int64_t)(mc > n_cells ? mc : n_cells) + 1);
    w.scan = take(sb);
    w.bytes = o;
    return w;
}

template <typename T, int SEL>
static int select_impl(int32_t n_cells, const int32_t* cell_start, dsmc_vec3 v, XsLaw law,
                       const double* lambda, const double* mom, dsmc_rng rng,
                       dsmc_pairs pairs, void* ws, dsmc_status* st, hipStream_t s)
{
    SelectWs w = select_ws_layout(ws, n_cells, pairs.cap);
    const int pb = persistent_blocks(256);
    int cb = (n_cells + 255) / 256;
    cb = cb < 1 ? 1 : (cb > pb ? pb : cb);
    if (SEL == SEL_NTC)
        k_cand_count<<<cb, 256, 0, s>>>(cell_start, n_cells, lambda, mom, law, rng, w.cand_cnt);
    else
        k_trial_count<<<cb, 256, 0, s>>>(cell_start, n_cells, w.cand_cnt);
    DSMC_LAUNCH_CHECK("select:count");
    int rc = exclusive_scan_i32(w.cand_cnt, w.cand_off, n_cells, w.total, w.scan, s);
    if (rc) return rc;
    k_cand_check<<<1, 1, 0, s>>>(w.total, pairs.cap, w.ok, w.n_use, w.n_chunks, st);
    DSMC_LAUNCH_CHECK("select:check");
    k_round_cells<<<cb, 256, 0, s>>>(n_cells, w.cand_off, w.n_use, w.round_cell);
    DSMC_LAUNCH_CHECK("select:round_cells");
    k_cand_decide<T, SEL><<<pb, 256, 0, s>>>(cell_start, n_cells, w.cand_off, w.n_use,
                                             w.round_cell, mom, lambda, law.C, law.e, rng,
                                             v3<const T>(v), w.chunk_cnt, w.si, w.sj, w.sc,
                                             w.loc, st);
    DSMC_LAUNCH_CHECK("select:decide");
    rc = exclusive_scan_i32_dev(w.chunk_cnt, w.chunk_off, w.n_chunks, max_chunks(pairs.cap),
                                w.scan, s);
    if (rc) return rc;
    k_stage_copy<<<pb, 256, 0, s>>>(w.n_chunks, w.chunk_cnt, w.chunk_off, w.si, w.sj, w.sc,
                                    pairs.i, pairs.j, pairs.cell);
    DSMC_LAUNCH_CHECK("select:copy");
    k_pair_counts<<<cb, 256, 0, s>>>(n_cells, w.cand_off, w.ok, w.n_use, w.n_chunks, w.chunk_off,
                                     w.loc, pairs.off, pairs.cnt, st);
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
        return select_impl<double, SEL_NTC>(n_cells, cell_start, v, law, lambda, mom, rng, pairs,
                                            ws, st, s);
    if (dtype == DSMC_F32)
        return select_impl<float, SEL_NTC>(n_cells, cell_start, v, law, lambda, mom, rng, pairs,
                                           ws, st, s);
    return arg_error("dsmc_select_pairs_ntc: dtype %d", dtype);
}

extern "C" size_t dsmc_select_pairs_sbt_ws(int32_t n_cells, int64_t cap)
{
    return dsmc_select_pairs_ntc_ws(n_cells, cap);
}

extern "C" int dsmc_select_pairs_sbt(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                                     dsmc_vec3 v, dsmc_xs xs, const double* lambda,
                                     dsmc_rng rng, dsmc_pairs pairs, void* ws, size_t ws_bytes,
                                     dsmc_status* st, dsmc_stream_t stream)
{
    if (n_cells < 1) return arg_error("dsmc_select_pairs_sbt: n_cells=%d", n_cells);
    if (!cell_start || !lambda || !ws || !v.x || !v.y || !v.z || !pairs.off || !pairs.cnt ||
        (pairs.cap > 0 && (!pairs.i || !pairs.j || !pairs.cell)))
        return arg_error("dsmc_select_pairs_sbt: null pointer");
    if (pairs.cap < 0 || pairs.cap >= (int64_t)INT32_MAX - 2)
        return arg_error("dsmc_select_pairs_sbt: cap %lld out of range", (long long)pairs.cap);
    if (ws_bytes < dsmc_select_pairs_sbt_ws(n_cells, pairs.cap))
        return arg_error("dsmc_select_pairs_sbt: workspace %zu < %zu", ws_bytes,
                         dsmc_select_pairs_sbt_ws(n_cells, pairs.cap));
    XsLaw law;
    int rc = xs_law(xs, &law);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    if (dtype == DSMC_F64)
        return select_impl<double, SEL_SBT>(n_cells, cell_start, v, law, lambda, nullptr, rng,
                                            pairs, ws, st, s);
    if (dtype == DSMC_F32)
        return select_impl<float, SEL_SBT>(n_cells, cell_start, v, law, lambda, nullptr, rng,
                                           pairs, ws, st, s);
    return arg_error("dsmc_select_pairs_sbt: dtype %d", dtype);
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
