// Collision application.
//
// Phase A (one lane per accepted pair, on the pre-collision velocities) turns
// the pair's latents into a post-collision direction (isotropic rule) or, for
// the other rules, is done by their own kernels.  Phase B applies the pairs of
// each cell in candidate order on the current velocities with the
// centre-of-mass update of eq. v_update_pair.  Schedules:
//   LANE  -- one lane walks one cell's pairs sequentially;
//   WAVE  -- one 64-lane workgroup per cell (up to 256 pairs), the cell's
//            velocities staged in LDS, applying in parallel, round by round,
//            every pending pair that is the earliest pending pair of both of
//            its particles;
//   BLOCK -- the same dependency rounds by a 256-lane workgroup (up to 2048
//            pairs in LDS, larger cells on velocities in global memory).
// A pair's update depends only on the current velocities of its two
// particles, and every schedule applies each pair after every earlier pair
// that shares a particle, so all schedules produce bit-identical velocities.
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

// ------------------------------------------------------------------------
// Dependency rounds with the cell's velocities staged in LDS.  Each thread
// owns up to PPL pairs (pair q = thread + NT m) with their Phase-A results
// prefetched into registers.  Round search: in round r every pending pair
// offers the key ((R - r) << 16 | q) to both of its particles (LDS
// atomicMin; keys of later rounds are smaller, so the table never needs
// clearing); a pair whose key wins at both particles is the earliest pending
// pair of both and belongs to round r.  Pairs of one round share no particle,
// so they commute.  The pairs are then bucketed by round in LDS (record and
// Phase-A result at a compact position) and applied round by round, each
// round's pairs spread over all lanes: every pair costs one pass of the
// update, however many rounds the cell needs.  The result is the sequential
// application in candidate order, bit for bit.
// ------------------------------------------------------------------------
constexpr int32_t ROUND_MAX = 32767;

template <typename T, int RULE>
struct Payload {
    static constexpr int W = RULE == RULE_CHI ? 5 : 3;
    T a, b, c, d, e;
    __device__ __forceinline__ void load(const PairBuf<T>& buf, int64_t p)
    {
        a = buf.a[p]; b = buf.b[p]; c = buf.c[p];
        if (RULE == RULE_CHI) { d = buf.d[p]; e = buf.e[p]; }
    }
    __device__ __forceinline__ void put(T* s) const
    {
        s[0] = a; s[1] = b; s[2] = c;
        if (RULE == RULE_CHI) { s[3] = d; s[4] = e; }
    }
    __device__ __forceinline__ void get(const T* s)
    {
        a = s[0]; b = s[1]; c = s[2];
        if (RULE == RULE_CHI) { d = s[3]; e = s[4]; }
    }
};

template <typename T, int RULE>
__device__ __forceinline__ void apply_pair_lds(T* lx, T* ly, T* lz, int32_t a, int32_t b,
                                               const Payload<T, RULE>& pl)
{
    const double xa = lx[a], ya = ly[a], za = lz[a];
    const double xb = lx[b], yb = ly[b], zb = lz[b];
    const double rx = xa - xb, ry = ya - yb, rz = za - zb;
    double u[3];
    double g;
    if (RULE == RULE_DIR) {
        g = sqrt(rx * rx + ry * ry + rz * rz);
        const double a0 = pl.a, a1 = pl.b, a2 = pl.c;
        const double inv = 1.0 / sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        u[0] = a0 * inv; u[1] = a1 * inv; u[2] = a2 * inv;
    } else {
        double vh[3], e[3];
        g = unit3<double>(rx, ry, rz, vh);
        const double xi[3] = {(double)pl.c, (double)pl.d, (double)pl.e};
        perp_dir<double>(xi, vh, e);
        const double cc = pl.a, sc = pl.b;
        u[0] = cc * vh[0] + sc * e[0];
        u[1] = cc * vh[1] + sc * e[1];
        u[2] = cc * vh[2] + sc * e[2];
    }
    const double cx = 0.5 * (xa + xb), cy = 0.5 * (ya + yb), cz = 0.5 * (za + zb);
    const double px = 0.5 * g * u[0], py = 0.5 * g * u[1], pz = 0.5 * g * u[2];
    lx[a] = (T)(cx + px); ly[a] = (T)(cy + py); lz[a] = (T)(cz + pz);
    lx[b] = (T)(cx - px); ly[b] = (T)(cy - py); lz[b] = (T)(cz - pz);
}

// Any thread of the workgroup with a pending pair (also a barrier).
template <int NT>
__device__ __forceinline__ bool any_pending(uint32_t pend)
{
    if (NT == 64) {
        __syncthreads();
        return __ballot(pend != 0) != 0;
    }
    return __syncthreads_or(pend != 0) != 0;
}

// LDS of one staged cell: velocities [3][NMAX]; a union of the round-search
// tables first[TABLES][NMAX] (two for multi-wave workgroups, see pair_batch)
// and the bucketed Phase-A results pay[PMAX][W]; the
// bucketed pair records rab[PMAX] (slot a | slot b << 16); the round table
// rc[RMAX + 1] (counts, then starts).
template <typename T, int RULE, int NT, int PPL, int NMAX, int RMAX>
struct CellLds {
    static constexpr int PMAX = NT * PPL;
    static constexpr int TABLES = NT > 64 ? 2 : 1;
    static constexpr size_t v_bytes = (size_t)3 * NMAX * sizeof(T);
    static constexpr size_t f_bytes = (size_t)TABLES * NMAX * sizeof(int32_t);
    static constexpr size_t p_bytes = (size_t)PMAX * Payload<T, RULE>::W * sizeof(T);
    static constexpr size_t u_bytes = f_bytes > p_bytes ? f_bytes : p_bytes;
    static constexpr size_t bytes = v_bytes + u_bytes + (size_t)PMAX * 4 + (size_t)(RMAX + 1) * 4;
    T *lx, *ly, *lz, *pay;
    int32_t *first, *rab, *rc;
    __device__ __forceinline__ explicit CellLds(char* smem)
    {
        lx = reinterpret_cast<T*>(smem);
        ly = lx + NMAX;
        lz = ly + NMAX;
        first = reinterpret_cast<int32_t*>(smem + v_bytes);
        pay = reinterpret_cast<T*>(smem + v_bytes);
        rab = reinterpret_cast<int32_t*>(smem + v_bytes + u_bytes);
        rc = rab + PMAX;
    }
};

// Exclusive scan of rc[0..R) in place by the first wave; rc[R] = total.
__device__ __forceinline__ void round_scan(int32_t* rc, int32_t R)
{
    const int t = threadIdx.x;
    if (t < 64) {
        int32_t carry = 0;
        for (int32_t base = 0; base < R; base += 64) {
            const int32_t x = base + t < R ? rc[base + t] : 0;
            int32_t y = x;
#pragma unroll
            for (int s = 1; s < 64; s <<= 1) {
                const int32_t u = __shfl_up(y, s, 64);
                if (t >= s) y += u;
            }
            if (base + t < R) rc[base + t] = carry + y - x;
            carry += __shfl(y, 63, 64);
        }
        if (t == 0) rc[R] = carry;
    }
}

// One batch of c <= NT * PPL pairs (from offset o) of a cell whose
// velocities (slots [lo, lo + span), span <= NMAX) are staged in L; pa_g /
// pb_g are this thread's pairs (global slots, padded with lo).  Applies the
// batch in candidate order and ends with a barrier.  A cell with more pairs
// than one batch holds runs its batches one after another in candidate order.
template <typename T, int RULE, int NT, int PPL, int NMAX, int RMAX>
__device__ __forceinline__ void pair_batch(const PairBuf<T>& d, int32_t c, int64_t o, int32_t lo,
                                           int32_t span, const int32_t (&pa_g)[PPL],
                                           const int32_t (&pb_g)[PPL],
                                           const CellLds<T, RULE, NT, PPL, NMAX, RMAX>& L)
{
    constexpr int W = Payload<T, RULE>::W;
    constexpr bool DUAL = CellLds<T, RULE, NT, PPL, NMAX, RMAX>::TABLES == 2;
    const int t = threadIdx.x;
    int32_t pa[PPL], pb[PPL], rnd[PPL];
    Payload<T, RULE> pl[PPL];
    uint32_t pend = 0;
#pragma unroll
    for (int m = 0; m < PPL; ++m) {
        const int32_t q = t + NT * m;
        pa[m] = pa_g[m] - lo;
        pb[m] = pb_g[m] - lo;
        rnd[m] = -1;
        if (q < c) {
            pl[m].load(d, o + q);
            pend |= 1u << m;
        }
    }
    for (int32_t q = t; q < span; q += NT) {
        L.first[q] = INT32_MAX;
        if (DUAL) L.first[NMAX + q] = INT32_MAX;
    }
    int32_t r = 0;
    if (DUAL) {
        // Rounds alternate between two tables, so one barrier per round
        // suffices: a wave may offer round r + 1's keys while others still
        // read round r's table, and a table is written again only after every
        // wave has passed the barrier that follows the reads of it.
        __syncthreads();
        for (;;) {
            int32_t* tb = L.first + (r & 1) * NMAX;
            const int32_t kb = (ROUND_MAX - r) << 16;
#pragma unroll
            for (int m = 0; m < PPL; ++m)
                if (pend & (1u << m)) {
                    const int32_t key = kb | (t + NT * m);
                    atomicMin(&tb[pa[m]], key);
                    atomicMin(&tb[pb[m]], key);
                }
            if (!any_pending<NT>(pend)) break;
#pragma unroll
            for (int m = 0; m < PPL; ++m) {
                const int32_t key = kb | (t + NT * m);
                if ((pend & (1u << m)) && tb[pa[m]] == key && tb[pb[m]] == key) {
                    rnd[m] = r;
                    pend &= ~(1u << m);
                }
            }
            ++r;
        }
    } else {
        while (any_pending<NT>(pend)) {
            const int32_t kb = (ROUND_MAX - r) << 16;
#pragma unroll
            for (int m = 0; m < PPL; ++m)
                if (pend & (1u << m)) {
                    const int32_t key = kb | (t + NT * m);
                    atomicMin(&L.first[pa[m]], key);
                    atomicMin(&L.first[pb[m]], key);
                }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < PPL; ++m) {
                const int32_t key = kb | (t + NT * m);
                if ((pend & (1u << m)) && L.first[pa[m]] == key && L.first[pb[m]] == key) {
                    rnd[m] = r;
                    pend &= ~(1u << m);
                }
            }
            ++r;
        }
    }
    const int32_t R = r;
    if (R <= RMAX) {
        // bucket by round: position inside the round, round starts, records
        for (int32_t q = t; q < R; q += NT) L.rc[q] = 0;
        __syncthreads();
        int32_t pos[PPL];
#pragma unroll
        for (int m = 0; m < PPL; ++m) pos[m] = rnd[m] >= 0 ? atomicAdd(&L.rc[rnd[m]], 1) : 0;
        __syncthreads();
        round_scan(L.rc, R);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PPL; ++m)
            if (rnd[m] >= 0) {
                const int32_t s = L.rc[rnd[m]] + pos[m];
                L.rab[s] = pa[m] | (pb[m] << 16);
                pl[m].put(L.pay + (size_t)s * W);
            }
        __syncthreads();
        for (int32_t rr = 0; rr < R; ++rr) {
            const int32_t s1 = L.rc[rr + 1];
            for (int32_t s = L.rc[rr] + t; s < s1; s += NT) {
                const int32_t ab = L.rab[s];
                Payload<T, RULE> p;
                p.get(L.pay + (size_t)s * W);
                apply_pair_lds<T, RULE>(L.lx, L.ly, L.lz, ab & 0xffff, ab >> 16, p);
            }
            __syncthreads();
        }
    } else {
        // more rounds than the round table holds: apply from the registers
        for (int32_t rr = 0; rr < R; ++rr) {
#pragma unroll
            for (int m = 0; m < PPL; ++m)
                if (rnd[m] == rr) apply_pair_lds<T, RULE>(L.lx, L.ly, L.lz, pa[m], pb[m], pl[m]);
            __syncthreads();
        }
    }
}

template <typename T, int RULE, int NT, int PPL, int NMAX, int RMAX>
__device__ __forceinline__ void stage_cell(V3<T> v, int32_t lo, int32_t span,
                                           const CellLds<T, RULE, NT, PPL, NMAX, RMAX>& L)
{
    // STAGE_BATCH slots per thread in flight: their loads are issued before
    // any LDS store waits on them
    constexpr int STAGE_BATCH = 4;
    for (int32_t q0 = threadIdx.x; q0 < span; q0 += NT * STAGE_BATCH) {
        T x[STAGE_BATCH], y[STAGE_BATCH], z[STAGE_BATCH];
#pragma unroll
        for (int b = 0; b < STAGE_BATCH; ++b) {
            const int32_t q = q0 + NT * b;
            if (q < span) {
                x[b] = v.x[lo + q];
                y[b] = v.y[lo + q];
                z[b] = v.z[lo + q];
            }
        }
#pragma unroll
        for (int b = 0; b < STAGE_BATCH; ++b) {
            const int32_t q = q0 + NT * b;
            if (q < span) {
                L.lx[q] = x[b];
                L.ly[q] = y[b];
                L.lz[q] = z[b];
            }
        }
    }
}

template <typename T, int RULE, int NT, int PPL, int NMAX, int RMAX>
__device__ __forceinline__ void unstage_cell(V3<T> v, int32_t lo, int32_t span,
                                             const CellLds<T, RULE, NT, PPL, NMAX, RMAX>& L)
{
    for (int32_t q = threadIdx.x; q < span; q += NT) {
        v.x[lo + q] = L.lx[q];
        v.y[lo + q] = L.ly[q];
        v.z[lo + q] = L.lz[q];
    }
    __syncthreads();
}

// One cell of at most NT * PPL pairs: stage, apply, and (WB) write back.
template <typename T, int RULE, int NT, int PPL, int NMAX, int RMAX, bool WB>
__device__ __forceinline__ void cell_rounds(const PairsView& pr, V3<T> v, const PairBuf<T>& d,
                                            int32_t c, int64_t o, int32_t lo, int32_t span,
                                            const int32_t (&pa_g)[PPL],
                                            const int32_t (&pb_g)[PPL],
                                            const CellLds<T, RULE, NT, PPL, NMAX, RMAX>& L)
{
    (void)pr;
    stage_cell(v, lo, span, L);
    pair_batch(d, c, o, lo, span, pa_g, pb_g, L);
    if (WB) unstage_cell(v, lo, span, L);
}

// Min / max of the cell's pair slots over the workgroup.
template <int NT>
__device__ __forceinline__ void group_minmax(int32_t& lo, int32_t& hi, int32_t* red)
{
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
        lo = min(lo, __shfl_xor(lo, s, 64));
        hi = max(hi, __shfl_xor(hi, s, 64));
    }
    if (NT == 64) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { red[wid] = lo; red[NT / 64 + wid] = hi; }
    __syncthreads();
    lo = red[0];
    hi = red[NT / 64];
    for (int w = 1; w < NT / 64; ++w) { lo = min(lo, red[w]); hi = max(hi, red[NT / 64 + w]); }
    __syncthreads();
}

// BLOCK schedule, in two size classes so that the common large cells keep two
// workgroups per CU:
//   medium: 256 threads, cells whose pairs span up to 2496 slots (1280 for
//           FP64 velocities), LDS rounds on batches of 2048 pairs (1024);
//   big:    512 threads, spans up to 4096 slots (2048) in LDS, batches of
//           4096 pairs (2048); larger cells (up to 8192 pairs and slots) run
//           the rounds on velocities in global memory with the tables in LDS;
//           beyond that one thread applies the pairs in order.
// The WAVE kernel lists the cells it cannot hold (list[0] = length, then k
// for a medium cell or -1 - k for a big one); each class kernel works through
// the list and takes its own entries.  Without a list every cell with at
// least min_pairs pairs is classified in the kernel.
constexpr int BLK_GMAX = 8192;      // global-memory rounds
template <typename T, bool BIG> struct BlkShape;
template <> struct BlkShape<float, false> {
    static constexpr int NT = 256, PPL = 8, NMAX = 2496, RMAX = 512;
};
template <> struct BlkShape<float, true> {
    static constexpr int NT = 512, PPL = 8, NMAX = 4096, RMAX = 1024;
};
template <> struct BlkShape<double, false> {
    static constexpr int NT = 256, PPL = 4, NMAX = 1280, RMAX = 512;
};
template <> struct BlkShape<double, true> {
    static constexpr int NT = 512, PPL = 4, NMAX = 2048, RMAX = 1024;
};
template <typename T, int RULE, bool BIG>
using BlockLds = CellLds<T, RULE, BlkShape<T, BIG>::NT, BlkShape<T, BIG>::PPL,
                         BlkShape<T, BIG>::NMAX, BlkShape<T, BIG>::RMAX>;

template <typename T, int RULE, bool BIG>
struct BlkSmem {
    static constexpr size_t glb = BIG ? (size_t)BLK_GMAX * 2 * sizeof(int32_t) : 0;
    static constexpr size_t bytes =
        BlockLds<T, RULE, BIG>::bytes > glb ? BlockLds<T, RULE, BIG>::bytes : glb;
};

// Size class of a cell whose pairs span `span` slots (any pair count: the
// pairs run in batches of NT * PPL).
template <typename T>
__host__ __device__ __forceinline__ bool is_big_cell(int32_t c, int32_t span)
{
    (void)c;
    return span > BlkShape<T, false>::NMAX;
}

// Work list of the cells the WAVE kernel cannot hold, in the sixth Phase-A
// field: p[0] = number of heavy cells (more pairs than one medium batch),
// stored from p[2] upward; p[1] = number of the others, stored from p[top]
// downward, top = the first int32 past the field (inside the workspace's
// 256-byte tail).  Heavy cells are handed out first, which balances the block
// kernels' long cells.  An entry is k (medium class) or -1 - k (big class).
// Every listed cell holds a pair, so the entries number at most cap < top - 1
// and the two ends never meet or reach the counters.
struct CellList {
    int32_t* p;
    int64_t top;
};

template <typename T>
__device__ __forceinline__ void list_cell(const CellList& L, int32_t k, int32_t c, int32_t span)
{
    using M = BlkShape<T, false>;
    const int32_t e = is_big_cell<T>(c, span) ? -1 - k : k;
    if (c > M::NT * M::PPL) {
        const int32_t at = atomicAdd(&L.p[0], 1);
        L.p[2 + at] = e;
    } else {
        const int32_t at = atomicAdd(&L.p[1], 1);
        L.p[L.top - at] = e;
    }
}

__device__ __forceinline__ int64_t list_items(const CellList& L) { return (int64_t)L.p[0] + L.p[1]; }

// WAVE schedule: one 64-lane workgroup per cell with at most 256 pairs whose
// slots span at most 320 (free-stream cells of a few hundred particles; small
// LDS tables, so many workgroups stay resident to hide the cell loads); every other cell goes to the list the BLOCK kernel
// works through (list[0] = length, list[1..] = cells).  The next cell's count
// and offset are loaded while the current cell runs.
constexpr int WV_NMAX = 320;
constexpr int WV_PPL = 4;
constexpr int WV_RMAX = 64 * WV_PPL;
template <typename T, int RULE>
using WaveLds = CellLds<T, RULE, 64, WV_PPL, WV_NMAX, WV_RMAX>;

template <typename T, int RULE>
__global__ void __launch_bounds__(64)
k_phaseB_wave(int32_t n_cells, PairsView pr, V3<T> v, PairBuf<T> d, int32_t min_pairs,
              CellList list)
{
    __shared__ __attribute__((aligned(16))) char smem[WaveLds<T, RULE>::bytes];
    const WaveLds<T, RULE> L(smem);
    const int lane = threadIdx.x;
    int64_t k = blockIdx.x;
    int32_t c = k < n_cells ? pr.cnt[k] : 0;
    int32_t o32 = k < n_cells ? pr.off[k] : 0;
    for (; k < n_cells; k += gridDim.x) {
        const int64_t kn = k + gridDim.x;
        const int32_t c_next = kn < n_cells ? pr.cnt[kn] : 0;
        const int32_t o_next = kn < n_cells ? pr.off[kn] : 0;
        const int64_t o = o32;
        const int32_t cc = c;
        c = c_next;
        o32 = o_next;
        if (cc == 0 || cc < min_pairs) continue;
        if (cc > 64 * WV_PPL) {
            int32_t lo = INT32_MAX, hi = -1;
            for (int32_t q = lane; q < cc; q += 64) {
                lo = min(lo, min(pr.i[o + q], pr.j[o + q]));
                hi = max(hi, max(pr.i[o + q], pr.j[o + q]));
            }
            group_minmax<64>(lo, hi, nullptr);
            if (lane == 0) list_cell<T>(list, (int32_t)k, cc, hi - lo + 1);
            continue;
        }
        int32_t pa[WV_PPL], pb[WV_PPL];
        int32_t lo = INT32_MAX, hi = -1;
#pragma unroll
        for (int m = 0; m < WV_PPL; ++m) {
            const int32_t q = lane + 64 * m;
            pa[m] = 0;
            pb[m] = 0;
            if (q < cc) {
                pa[m] = pr.i[o + q];
                pb[m] = pr.j[o + q];
                lo = min(lo, min(pa[m], pb[m]));
                hi = max(hi, max(pa[m], pb[m]));
            }
        }
        group_minmax<64>(lo, hi, nullptr);
        const int32_t span = hi - lo + 1;
        if (span > WV_NMAX) {
            if (lane == 0) list_cell<T>(list, (int32_t)k, cc, span);
            continue;
        }
#pragma unroll
        for (int m = 0; m < WV_PPL; ++m)
            if (lane + 64 * m >= cc) { pa[m] = lo; pb[m] = lo; }
        cell_rounds<T, RULE, 64, WV_PPL, WV_NMAX, WV_RMAX, true>(pr, v, d, cc, o, lo, span, pa, pb,
                                                                 L);
    }
}

template <typename T, int RULE, int NT>
__device__ void cell_rounds_global(V3<T> v, const PairBuf<T>& d, const PairsView& pr, int32_t c,
                                   int64_t o, int32_t lo, int32_t span, int32_t* first,
                                   uint32_t* pij)
{
    __shared__ int32_t remaining;
    for (int32_t q = threadIdx.x; q < c; q += NT)
        pij[q] = (uint32_t)(pr.i[o + q] - lo) | ((uint32_t)(pr.j[o + q] - lo) << 16);
    if (threadIdx.x == 0) remaining = c;
    __syncthreads();
    while (remaining > 0) {
        for (int32_t q = threadIdx.x; q < span; q += NT) first[q] = INT32_MAX;
        __syncthreads();
        for (int32_t q = threadIdx.x; q < c; q += NT) {
            const uint32_t w = pij[q];
            if (w != 0xffffffffu) {
                atomicMin(&first[w & 0xffff], q);
                atomicMin(&first[w >> 16], q);
            }
        }
        __syncthreads();
        int done_here = 0;
        for (int32_t q = threadIdx.x; q < c; q += NT) {
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

// One BLOCK cell (pairs [o, o + c), slots [lo, lo + span)); the updated
// velocities are left in LDS when the LDS rounds ran (returns true), else in
// v.  The medium class is only given cells that fit its LDS tables.
template <typename T, int RULE, bool BIG, bool WB>
__device__ __forceinline__ bool block_cell(const PairsView& pr, V3<T> v, const PairBuf<T>& d,
                                           int32_t c, int64_t o, int32_t lo, int32_t span,
                                           char* smem)
{
    using S = BlkShape<T, BIG>;
    if (span <= S::NMAX) {
        const BlockLds<T, RULE, BIG> L(smem);
        stage_cell(v, lo, span, L);
        for (int32_t b = 0; b < c; b += S::NT * S::PPL) {
            const int32_t cb = c - b < S::NT * S::PPL ? c - b : S::NT * S::PPL;
            int32_t pa[S::PPL], pb[S::PPL];
#pragma unroll
            for (int m = 0; m < S::PPL; ++m) {
                const int32_t q = threadIdx.x + S::NT * m;
                pa[m] = lo;
                pb[m] = lo;
                if (q < cb) {
                    pa[m] = pr.i[o + b + q];
                    pb[m] = pr.j[o + b + q];
                }
            }
            pair_batch(d, cb, o + b, lo, span, pa, pb, L);
        }
        if (WB) unstage_cell(v, lo, span, L);
        return true;
    }
    if (BIG && c <= BLK_GMAX && span <= BLK_GMAX) {
        int32_t* gfirst = reinterpret_cast<int32_t*>(smem);
        uint32_t* pij = reinterpret_cast<uint32_t*>(gfirst + BLK_GMAX);
        cell_rounds_global<T, RULE, S::NT>(v, d, pr, c, o, lo, span, gfirst, pij);
    } else {
        // beyond the LDS tables: sequential, still in candidate order
        if (threadIdx.x == 0)
            for (int32_t q = 0; q < c; ++q)
                apply_pair<T, RULE>(v, pr.i[o + q], pr.j[o + q], d, o + q);
        __syncthreads();
    }
    return false;
}

// Entry idx of the work list, or -1 when it belongs to the other class.
template <bool BIG>
__device__ __forceinline__ int32_t class_cell(const CellList& L, int64_t idx)
{
    const int32_t a = L.p[0];
    const int32_t e = idx < a ? L.p[2 + idx] : L.p[L.top - (idx - a)];
    if (BIG) return e < 0 ? -1 - e : -1;
    return e >= 0 ? e : -1;
}

template <typename T, int RULE, bool BIG>
__global__ void __launch_bounds__((BlkShape<T, BIG>::NT))
k_phaseB_block(int32_t n_cells, PairsView pr, V3<T> v, PairBuf<T> d, int32_t min_pairs,
               CellList list, bool use_list)
{
    constexpr int NT = BlkShape<T, BIG>::NT;
    __shared__ __attribute__((aligned(16))) char smem[BlkSmem<T, RULE, BIG>::bytes];
    __shared__ int32_t red[2 * (NT / 64)];
    const int64_t n_items = use_list ? list_items(list) : (int64_t)n_cells;
    for (int64_t idx = blockIdx.x; idx < n_items; idx += gridDim.x) {
        int32_t k;
        if (use_list) {
            k = class_cell<BIG>(list, idx);
            if (k < 0) continue;
        } else {
            k = (int32_t)idx;
            const int32_t c = pr.cnt[k];
            if (c == 0 || c < min_pairs) continue;
        }
        const int32_t c = pr.cnt[k];
        const int64_t o = pr.off[k];
        int32_t lo = INT32_MAX, hi = -1;
        for (int32_t q = threadIdx.x; q < c; q += NT) {
            lo = min(lo, min(pr.i[o + q], pr.j[o + q]));
            hi = max(hi, max(pr.i[o + q], pr.j[o + q]));
        }
        group_minmax<NT>(lo, hi, red);
        const int32_t span = hi - lo + 1;
        if (!use_list && is_big_cell<T>(c, span) != BIG) continue;
        block_cell<T, RULE, BIG, true>(pr, v, d, c, o, lo, span, smem);
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// Phase B fused with the cell-wise moment matching (eq. cell_energy_clamp):
// the whole cell [s0, s0 + N) is staged in LDS, its pairs applied in
// dependency rounds, then the first wave forms the cell's post-collision sums
// with the same lane assignment, loop order and butterfly as the separate
// matching kernel (so the result is bit-identical to Phase B followed by
// dsmc_moment_match(APPLY)) and writes the matched velocities once.
// ------------------------------------------------------------------------
struct MatchArgs {
    const int32_t* cell_start;
    const double* mom;
    int literal;
    dsmc_status* st;
};

template <typename T, typename LD>
__device__ __forceinline__ void match_cell(LD ld, int32_t N, const double* m, int literal,
                                           V3<T> v, int32_t s0, dsmc_status* st)
{
    const int lane = threadIdx.x & 63;
    // the cell's captured moments are loaded first, their latency overlaps
    // the sums
    const double m0 = m[0], m1 = m[1], m2 = m[2], mt = literal ? m[5] : m[3];
    double sx = 0, sy = 0, sz = 0;
    for (int32_t q = lane; q < N; q += 64) {
        sx += (double)ld.x(q);
        sy += (double)ld.y(q);
        sz += (double)ld.z(q);
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    sz = wave_sum(sz);
    const double ux = sx / N, uy = sy / N, uz = sz / N;
    double S = 0, E = 0;
    for (int32_t q = lane; q < N; q += 64) {
        const double x = ld.x(q), y = ld.y(q), z = ld.z(q);
        const double dx = x - ux, dy = y - uy, dz = z - uz;
        S += dx * dx + dy * dy + dz * dz;
        E += x * x + y * y + z * z;
    }
    S = wave_sum(S);
    E = wave_sum(E);
    const double post = literal ? E : S;
    if (!(post > 0.0) || !isfinite(post)) {
        if (lane == 0 && st) atomicAdd(&st->mm_skipped, 1);
        for (int32_t q = lane; q < N; q += 64) {
            v.x[s0 + q] = ld.x(q);
            v.y[s0 + q] = ld.y(q);
            v.z[s0 + q] = ld.z(q);
        }
        return;
    }
    const double alpha = sqrt(mt / post);
    for (int32_t q = lane; q < N; q += 64) {
        const int32_t s = s0 + q;
        if (literal) {
            v.x[s] = (T)(alpha * (double)ld.x(q));
            v.y[s] = (T)(alpha * (double)ld.y(q));
            v.z[s] = (T)(alpha * (double)ld.z(q));
        } else {
            v.x[s] = (T)(m0 + alpha * ((double)ld.x(q) - ux));
            v.y[s] = (T)(m1 + alpha * ((double)ld.y(q) - uy));
            v.z[s] = (T)(m2 + alpha * ((double)ld.z(q) - uz));
        }
    }
}

template <typename T> struct CellView {
    const T *px, *py, *pz;
    __device__ T x(int32_t q) const { return px[q]; }
    __device__ T y(int32_t q) const { return py[q]; }
    __device__ T z(int32_t q) const { return pz[q]; }
};

// WAVE form: cells with <= 256 pairs and <= WV_NMAX particles; others go to the list.
// At most four waves per SIMD: with the 320-slot LDS that is 14 cells per CU.
template <typename T, int RULE>
__global__ void __launch_bounds__(64, 4)
k_phaseB_match_wave(int32_t n_cells, PairsView pr, V3<T> v, PairBuf<T> d, MatchArgs ma,
                    CellList list)
{
    __shared__ __attribute__((aligned(16))) char smem[WaveLds<T, RULE>::bytes];
    const WaveLds<T, RULE> L(smem);
    const int lane = threadIdx.x;
    int64_t k = blockIdx.x;
    int32_t c = k < n_cells ? pr.cnt[k] : 0;
    int32_t o32 = k < n_cells ? pr.off[k] : 0;
    int32_t s0 = k < n_cells ? ma.cell_start[k] : 0;
    int32_t s1 = k < n_cells ? ma.cell_start[k + 1] : 0;
    for (; k < n_cells; k += gridDim.x) {
        const int64_t kn = k + gridDim.x;
        const int32_t c_next = kn < n_cells ? pr.cnt[kn] : 0;
        const int32_t o_next = kn < n_cells ? pr.off[kn] : 0;
        const int32_t s0_next = kn < n_cells ? ma.cell_start[kn] : 0;
        const int32_t s1_next = kn < n_cells ? ma.cell_start[kn + 1] : 0;
        const int32_t cc = c, N = s1 - s0, b0 = s0;
        const int64_t o = o32;
        c = c_next;
        o32 = o_next;
        s0 = s0_next;
        s1 = s1_next;
        if (cc == 0 || N < 2) continue;
        if (cc > 64 * WV_PPL || N > WV_NMAX) {
            if (lane == 0) list_cell<T>(list, (int32_t)k, cc, N);
            continue;
        }
        int32_t pa[WV_PPL], pb[WV_PPL];
#pragma unroll
        for (int m = 0; m < WV_PPL; ++m) {
            const int32_t q = lane + 64 * m;
            pa[m] = b0;
            pb[m] = b0;
            if (q < cc) {
                pa[m] = pr.i[o + q];
                pb[m] = pr.j[o + q];
            }
        }
        cell_rounds<T, RULE, 64, WV_PPL, WV_NMAX, WV_RMAX, false>(pr, v, d, cc, o, b0, N, pa, pb,
                                                                  L);
        match_cell<T>(CellView<T>{L.lx, L.ly, L.lz}, N, ma.mom + 6 * (size_t)k, ma.literal, v, b0,
                      ma.st);
        __syncthreads();
    }
}

// BLOCK forms (medium, big) for the listed cells; the first wave matches.
template <typename T, int RULE, bool BIG>
__global__ void __launch_bounds__((BlkShape<T, BIG>::NT))
k_phaseB_match_block(int32_t n_cells, PairsView pr, V3<T> v, PairBuf<T> d, MatchArgs ma,
                     CellList list)
{
    __shared__ __attribute__((aligned(16))) char smem[BlkSmem<T, RULE, BIG>::bytes];
    const int64_t n_items = list_items(list);
    for (int64_t idx = blockIdx.x; idx < n_items; idx += gridDim.x) {
        const int32_t k = class_cell<BIG>(list, idx);
        if (k < 0) continue;
        const int32_t c = pr.cnt[k];
        const int64_t o = pr.off[k];
        const int32_t b0 = ma.cell_start[k], N = ma.cell_start[k + 1] - b0;
        const bool in_lds = block_cell<T, RULE, BIG, false>(pr, v, d, c, o, b0, N, smem);
        if (threadIdx.x < 64) {
            const double* m = ma.mom + 6 * (size_t)k;
            if (in_lds) {
                const BlockLds<T, RULE, BIG> L(smem);
                match_cell<T>(CellView<T>{L.lx, L.ly, L.lz}, N, m, ma.literal, v, b0, ma.st);
            } else {
                match_cell<T>(CellView<T>{v.x + b0, v.y + b0, v.z + b0}, N, m, ma.literal, v, b0,
                              ma.st);
            }
        }
        __syncthreads();
    }
}

__global__ void k_zero_list(int32_t* p) { p[0] = 0; p[1] = 0; }

int phase_b(int rule, int dtype, int32_t n_cells, const int32_t* cell_start, dsmc_vec3 v,
            const dsmc_pairs& pairs, void* dirs, int64_t cap, int32_t schedule, hipStream_t s)
{
    (void)cell_start;
    const PairsView pr = PairsView::of(pairs);
    const int pb = persistent_blocks(256);
    int lb = (n_cells + 255) / 256;
    lb = lb < 1 ? 1 : (lb > pb ? pb : lb);
    // cells with at most `thr` pairs: LANE; larger: WAVE when they fit its
    // LDS tables (AUTO, WAVE), else BLOCK
    int32_t thr = block_threshold();
    bool use_wave = true;
    if (schedule == DSMC_SCHED_LANE) thr = INT32_MAX;
    if (schedule == DSMC_SCHED_BLOCK) { thr = 0; use_wave = false; }
    if (schedule == DSMC_SCHED_WAVE) thr = 0;
    const bool need_lane = thr > 0;
    const bool need_rest = thr < INT32_MAX;
    const int cus = device_cus();
    const dsmc_match_schedule ms = match_schedule();
    auto grid = [&](int per_cu) {
        const int64_t g = (int64_t)cus * per_cu;
        return (int)(g < n_cells ? (g < 1 ? 1 : g) : n_cells);
    };
    const int wb = grid(ms.wave_per_cu), bb = grid(ms.medium_per_cu), bg = grid(ms.big_per_cu);
#define DSMC_PHASEB(T, R)                                                                   \
    do {                                                                                    \
        PairBuf<T> d = PairBuf<T>::of(dirs, cap);                                           \
        const CellList list{reinterpret_cast<int32_t*>(d.f),                                \
                            (cap + 1) * (int64_t)sizeof(T) / 4};                            \
        if (need_lane) {                                                                    \
            k_phaseB_lane<T, R><<<lb, 256, 0, s>>>(n_cells, pr, v3<T>(v), d, thr);          \
            DSMC_LAUNCH_CHECK("phaseB:lane");                                               \
        }                                                                                   \
        if (need_rest && use_wave) {                                                        \
            k_zero_list<<<1, 1, 0, s>>>(list.p);                                            \
            DSMC_LAUNCH_CHECK("phaseB:list");                                               \
            k_phaseB_wave<T, R><<<wb, 64, 0, s>>>(n_cells, pr, v3<T>(v), d, thr + 1, list); \
            DSMC_LAUNCH_CHECK("phaseB:wave");                                               \
        }                                                                                   \
        if (need_rest) {                                                                    \
            k_phaseB_block<T, R, false><<<bb, BlkShape<T, false>::NT, 0, s>>>(              \
                n_cells, pr, v3<T>(v), d, thr + 1, list, use_wave);                         \
            DSMC_LAUNCH_CHECK("phaseB:block");                                              \
            k_phaseB_block<T, R, true><<<bg, BlkShape<T, true>::NT, 0, s>>>(                \
                n_cells, pr, v3<T>(v), d, thr + 1, list, use_wave);                         \
            DSMC_LAUNCH_CHECK("phaseB:block_big");                                          \
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

extern "C" int dsmc_apply_pairs_match(int32_t n_cells, const int32_t* cell_start, int32_t dtype,
                                      dsmc_vec3 v, dsmc_pairs pairs, int32_t kind,
                                      const double* mom, int32_t mode, void* ws,
                                      size_t ws_bytes, dsmc_status* st, dsmc_stream_t stream)
{
    int rc = check_pairs("dsmc_apply_pairs_match", n_cells, v, pairs, dtype, ws, ws_bytes);
    if (rc) return rc;
    if (!cell_start || !mom) return arg_error("dsmc_apply_pairs_match: null pointer");
    if (kind != DSMC_APPLY_DIRECTIONS && kind != DSMC_APPLY_ANGLES)
        return arg_error("dsmc_apply_pairs_match: kind %d", kind);
    if (mode != DSMC_MM_APPLY && mode != DSMC_MM_APPLY_LITERAL)
        return arg_error("dsmc_apply_pairs_match: mode %d", mode);
    hipStream_t s = as_stream(stream);
    const PairsView pr = PairsView::of(pairs);
    const MatchArgs ma{cell_start, mom, mode == DSMC_MM_APPLY_LITERAL ? 1 : 0, st};
    const int cus = device_cus();
    const dsmc_match_schedule ms = match_schedule();
    auto grid = [&](int per_cu) {
        const int64_t g = (int64_t)cus * per_cu;
        return (int)(g < n_cells ? (g < 1 ? 1 : g) : n_cells);
    };
    const int wb = grid(ms.wave_per_cu), bb = grid(ms.medium_per_cu), bg = grid(ms.big_per_cu);
#define DSMC_PHASEB_MATCH(T, R)                                                              \
    do {                                                                                     \
        PairBuf<T> d = PairBuf<T>::of(ws, pairs.cap);                                        \
        const CellList list{reinterpret_cast<int32_t*>(d.f),                                 \
                            (pairs.cap + 1) * (int64_t)sizeof(T) / 4};                       \
        k_zero_list<<<1, 1, 0, s>>>(list.p);                                                 \
        DSMC_LAUNCH_CHECK("phaseB_match:list");                                              \
        k_phaseB_match_wave<T, R><<<wb, 64, 0, s>>>(n_cells, pr, v3<T>(v), d, ma, list);     \
        DSMC_LAUNCH_CHECK("phaseB_match:wave");                                              \
        k_phaseB_match_block<T, R, false><<<bb, BlkShape<T, false>::NT, 0, s>>>(              \
            n_cells, pr, v3<T>(v), d, ma, list);                                             \
        DSMC_LAUNCH_CHECK("phaseB_match:block");                                             \
        k_phaseB_match_block<T, R, true><<<bg, BlkShape<T, true>::NT, 0, s>>>(               \
            n_cells, pr, v3<T>(v), d, ma, list);                                             \
        DSMC_LAUNCH_CHECK("phaseB_match:block");                                             \
    } while (0)
    const int rule = kind == DSMC_APPLY_ANGLES ? RULE_CHI : RULE_DIR;
    if (dtype == DSMC_F64) {
        if (rule == RULE_DIR) DSMC_PHASEB_MATCH(double, RULE_DIR); else DSMC_PHASEB_MATCH(double, RULE_CHI);
    } else {
        if (rule == RULE_DIR) DSMC_PHASEB_MATCH(float, RULE_DIR); else DSMC_PHASEB_MATCH(float, RULE_CHI);
    }
#undef DSMC_PHASEB_MATCH
    return DSMC_OK;
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
